"""Algorithmic work and minimum HBM traffic of one residual evaluation, per
element, for the roofline.

Flops.  Every pointwise formula is counted from the oracle's formulas
(flopmodel.json "oracle_op_counts", written by ``python -m oracle.opcount``:
additions, multiplications, divisions, square roots, logarithms, exponentials
of the paper's expressions, Sec. 7.1-7.2), with each division, square root,
logarithm and exponential weighted by the FP64 flop-equivalent of the code
gfx950 executes for it (flopmodel.json "fp64_weights", written by
``python -m paper_2312_07874_amd.flopweights``: FP64 instructions of the
compiled sequence, a fused multiply-add counting two).  Structure counts are
those of the method as the paper organises it: node states once per node
(their logarithms included), one directional two-point flux per distinct pair
of a collapsed-coordinate line with the direction sum_l S^l_ab (g_l(a) + g_l(b))
over the S^l the pair belongs to, the facet-correction pairs of the nonzeros
of R^T B, the interface flux per facet node, and the sum-factorised PKD
transforms of Sec. 5.2 (multiply-adds = 2 flops).  The log means are counted
on the series branch, which the smooth workloads take at almost every pair.

Bytes.  min_bytes is the single-pass minimum: modal state in and out, own and
neighbour facet states, G and J at the volume nodes, G^T nhat at the facet
nodes, 8 [N_c (2 N_p + 2 N_f N_qf) + (d^2 + 1) N_q + d N_f N_qf].  The
library's layout moves more (pre-scaled line metrics, facet Jacobians,
connectivity; see k2_bytes); layout_bytes reports it for the ratio.
"""
from __future__ import annotations

import json
import os

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 vector
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E

_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "flopmodel.json")
_cache = {}


def _model():
    if "m" not in _cache:
        with open(_MODEL) as fh:
            _cache["m"] = json.load(fh)
    return _cache["m"]


def weights():
    w = _model()["fp64_weights"]
    return {k: w[k]["flops"] for k in ("div", "sqrt", "log", "exp")}


def weighted(c: dict) -> int:
    w = weights()
    return int(c.get("add", 0) + c.get("mul", 0) + sum(c.get(k, 0) * w[k] for k in w))


def _sizes(dim: int, p: int):
    Q = p + 1
    NC = dim + 2
    NQ = Q ** dim
    NP = (p + 1) * (p + 2) // 2 if dim == 2 else (p + 1) * (p + 2) * (p + 3) // 6
    NQF = Q if dim == 2 else Q * Q
    NFQ = (dim + 1) * NQF
    return Q, NC, NQ, NP, NQF, NFQ


def transform_macs(dim: int, p: int) -> int:
    """Multiply-adds of one sum-factorised application of V (or V^T) to one variable."""
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    if dim == 2:
        return NP * Q + (p + 1) * Q * Q
    npair = (p + 1) * (p + 2) // 2
    return NP * Q + npair * Q * Q + (p + 1) * Q ** 3


def extrapolation_macs(dim: int, p: int) -> int:
    """Multiply-adds of R (facet extrapolation) or R^T for one variable: faces
    along a line take Q per facet node, tetrahedral face 4 Q^2."""
    Q = p + 1
    return 3 * Q * Q if dim == 2 else 3 * Q ** 3 + Q ** 4


def pair_counts(dim: int, p: int):
    """Per element: [(distinct volume pairs, number of S^l they belong to)],
    facet-correction pairs, facet nodes."""
    Q = p + 1
    per_line = Q * (Q - 1) // 2
    lines = Q ** (dim - 1)
    if dim == 2:
        vol = [(lines * per_line, 2), (lines * per_line, 1)]
        return vol, 3 * Q * Q, 3 * Q
    vol = [(lines * per_line, 3), (lines * per_line, 2), (lines * per_line, 1)]
    return vol, 3 * Q ** 3 + Q ** 4, 4 * Q * Q


def residual_flops(dim: int, p: int, ecflux: int = 0, dissipation: int = 1) -> dict:
    """Algorithmic FP64 flops of one residual evaluation of one element, split
    into the entropy projection (K1's work) and the right-hand side (K2's)."""
    m = _model()["oracle_op_counts"][str(dim)]
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    node = m["per_node"]
    prim = weighted(node["prim"])
    flux = weighted(m["per_pair_flux"][("ranocha" if ecflux == 0 else "chandrashekar") + "_series"])
    w = weights()
    xf = 2 * NC * transform_macs(dim, p)                 # one transform of all variables
    ext = 2 * NC * extrapolation_macs(dim, p)
    # K1: u = V u~; W(u) (primitive variables inside) times w J; V^T, w/J, V, V^T;
    # w = V w~ and its facet values R w
    k1 = xf + NQ * (weighted(node["entropy_vars"]) + NC) + 3 * xf + NC * NQ + xf + ext
    # K2: w = V w~; node states U(w) with rho, p and their logarithms, b = rho/p
    states = NQ * (weighted(node["cons_from_entropy"]) + prim + 2 * w["log"] + w["div"])
    vol_pairs, fac_pairs, fnodes = pair_counts(dim, p)
    vol = sum(n * (flux + 3 * dim * terms - dim + 2 * NC) for n, terms in vol_pairs)
    fac = fac_pairs * (flux + 2 * dim + 3 * NC)
    diss = weighted(m["per_interface_node_dissipation"]) if dissipation else 0
    iface = fnodes * (2 * (weighted(node["cons_from_entropy"]) + prim) + flux + diss + NC + 1 + NC)
    k2 = xf + states + vol + fac + iface + ext + 3 * xf + NC * NQ + xf
    return {"k1": k1, "k2": k2, "total": k1 + k2, "volume_pairs": vol, "facet_pairs": fac, "interface": iface,
            "node_states": states, "flux_per_pair": flux}


def min_bytes(dim: int, p: int) -> int:
    """Single-pass minimum HBM bytes of one residual of one element."""
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    return 8 * (NC * (2 * NP + 2 * NFQ) + (dim * dim + 1) * NQ + dim * NFQ)


def k2_bytes(dim: int, p: int) -> int:
    """The right-hand-side kernel in this library's layout: w~ and the own and
    neighbour facet values in, du~/dt out, pre-scaled line metrics and w/J,
    facet G^T nhat and J_f, the int32 facet connectivity."""
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    ngv = 8 if dim == 2 else 17
    return 8 * (NC * NP + 2 * NC * NFQ + (ngv - 1) * NQ + (dim + 1) * NFQ + NC * NP) + 4 * NFQ


def k1_bytes(dim: int, p: int) -> int:
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    return 8 * (NC * NP + 2 * NQ + NC * NP + NC * NFQ)


def layout_bytes(dim: int, p: int) -> int:
    """K1 + K2 of one residual in the library's layout (w~ and facet values
    written by K1 and read back by K2)."""
    return k1_bytes(dim, p) + k2_bytes(dim, p)


def k2_rk_bytes(dim: int, p: int) -> int:
    """K2 inside an RK4 step with the stage combination formed by its output:
    instead of writing du~/dt it reads u and acc and writes acc and U (stage 1
    skips the acc read, stage 4 reads acc and writes u), 3.25 state arrays on
    average over the four stages in place of one."""
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    return k2_bytes(dim, p) + (8 * NC * NP * 9) // 4


def k2_next_bytes(dim: int, p: int) -> int:
    """The fused RK4 stage kernel: K2 forming the stage combination and
    projecting the next stage input (2.5 state arrays on average over the four
    stages instead of du~/dt, plus the projection's w J read and w~ and facet
    values written)."""
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    return k2_bytes(dim, p) + (8 * NC * NP * 3) // 2 + 8 * (NC * NP + NC * NFQ + NQ)
