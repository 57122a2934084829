"""Operation counts of the oracle's formulas (test and measurement
infrastructure; writes the per-operation counts that the benchmark's
roofline uses as algorithmic work).

Each formula of oracle.physics is evaluated on one state (or one pair) under a
torch function mode that counts elementwise operations per output element:
additions and subtractions, multiplications, divisions, square roots,
logarithms and exponentials; comparisons, selections, abs and data movement
count nothing, a sum over k terms counts k - 1 additions.  The counts are
those of the formulas as the paper states them (Sec. 7.1-7.2), with the
primitive variables of a node formed once per node (a pair's flux takes the
two nodes' rho, v, p and their logarithms as given), and both logarithmic
means on the branch the given pair takes.

    python -m oracle.opcount [out.json]

writes the counts (default: paper_2312_07874_amd/flopmodel.json, merged with
the instruction weights already there)."""
from __future__ import annotations

import json
import os
import sys
from collections import Counter

import torch
from torch.overrides import TorchFunctionMode

from . import physics as ph

DT = torch.float64

_ADD = {"__add__", "__radd__", "add", "__sub__", "__rsub__", "sub", "__neg__", "neg", "__iadd__", "__isub__"}
_MUL = {"__mul__", "__rmul__", "mul", "__imul__"}
_DIV = {"__truediv__", "__rtruediv__", "div", "__itruediv__"}
_FUN = {"log": "log", "exp": "exp", "sqrt": "sqrt"}


class _Count(TorchFunctionMode):
    def __init__(self):
        super().__init__()
        self.c = Counter()

    def __torch_function__(self, func, types, args=(), kwargs=None):
        kwargs = kwargs or {}
        out = func(*args, **kwargs)
        name = getattr(func, "__name__", "")
        n = out.numel() if torch.is_tensor(out) else 0
        if name in _ADD:
            self.c["add"] += n
        elif name in _MUL:
            self.c["mul"] += n
        elif name in _DIV:
            # a division by a constant is a multiplication by its reciprocal
            const = any(isinstance(a, (int, float)) for a in args[:2])
            self.c["mul" if const else "div"] += n
        elif name in _FUN:
            self.c[_FUN[name]] += n
        elif name == "sum" and torch.is_tensor(args[0]):
            self.c["add"] += args[0].numel() - max(n, 1)
        return out


def count(fn, *args):
    with _Count() as m:
        fn(*args)
    return dict(m.c)


def _state(dim, rho, v, p, gamma=1.4):
    v = torch.tensor(v, dtype=DT)[:dim]
    E = p / (gamma - 1.0) + 0.5 * rho * float((v * v).sum())
    return torch.cat([torch.tensor([rho], dtype=DT), rho * v, torch.tensor([E], dtype=DT)])[None]


def _minus(a, b):
    return {k: a.get(k, 0) - b.get(k, 0) for k in set(a) | set(b) if a.get(k, 0) - b.get(k, 0)}


def counts(dim: int) -> dict:
    g = 1.4
    n = torch.tensor([[0.3, -0.2, 0.5][:dim]], dtype=DT)
    um = _state(dim, 1.0, [0.1, 0.2, -0.1], 1.0)
    near = _state(dim, 1.0 + 1e-4, [0.12, 0.18, -0.1], 1.0 - 1e-4)     # series branch of both means
    far = _state(dim, 1.3, [0.12, 0.18, -0.1], 0.7)                    # log branch of both means
    prim = count(ph.prim, um, g)
    out = {"per_node": {"prim": prim,
                        "entropy_vars": count(ph.entropy_vars, um, g),
                        "cons_from_entropy": count(ph.cons_from_entropy, ph.entropy_vars(um, g), g)}}
    pair = {}
    orig = (ph.log_mean, ph.inv_log_mean)
    for fname, f in (("ranocha", ph.ranocha_flux), ("chandrashekar", ph.chandrashekar_flux)):
        for branch, up in (("series", near), ("log", far)):
            # the branch the pair takes, alone
            ph.log_mean, ph.inv_log_mean = ((ph.log_mean_series, ph.inv_log_mean_series) if branch == "series"
                                            else (ph.log_mean_log, ph.inv_log_mean_log))
            try:
                c = count(f, um, up, n, g)
            finally:
                ph.log_mean, ph.inv_log_mean = orig
            # the primitive variables of both nodes are formed once per node,
            # and so are rho/p of each node for the mean of rho/p (Ranocha) or
            # beta = rho/(2p) (Chandrashekar)
            c = _minus(c, {k: 2 * v for k, v in prim.items()})
            c = _minus(c, {"div": 2})
            # the logarithms of the node values are formed once per node: a
            # log-branch mean takes the difference of two cached logarithms
            c.pop("log", None)
            pair[f"{fname}_{branch}"] = c
    out["per_pair_flux"] = pair
    # the dissipation term of eq. (num_flux) beyond the entropy-conservative flux
    with_d = count(ph.interface_flux, um, near, n, g, 0, 1)
    no_d = count(ph.interface_flux, um, near, n, g, 0, 0)
    out["per_interface_node_dissipation"] = _minus(_minus(with_d, no_d), {k: 2 * v for k, v in prim.items()})
    return out


def main(argv):
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = argv[0] if argv else os.path.join(here, "paper_2312_07874_amd", "flopmodel.json")
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        data = {}
    data["oracle_op_counts"] = {"2": counts(2), "3": counts(3),
                                "source": "python -m oracle.opcount (oracle.physics formulas, one state or pair)"}
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(json.dumps(data["oracle_op_counts"], indent=1, sort_keys=True))


if __name__ == "__main__":
    main(sys.argv[1:])
