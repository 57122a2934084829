"""FP64 cost of one log, exp, sqrt and division on gfx950, measured from the
code the compiler emits (same flags as the library), for the roofline's
algorithmic flop count.

    python -m paper_2312_07874_amd.flopweights

compiles measure/probe_fp64_ops.hip for gfx950, reads the kernel bodies of its
assembly and counts, beyond the baseline kernel's, the FP64 VALU instructions
(v_*_f64) with fused multiply-adds counted twice: the flop-equivalent of the
sequence at the FP64 peak, where one FMA is two flops.  Writes "fp64_weights"
into flopmodel.json (next to this file)."""
from __future__ import annotations

import json
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
PROBE = os.path.join(HERE, "measure", "probe_fp64_ops.hip")
MODEL = os.path.join(HERE, "flopmodel.json")


def _bodies(asm: str):
    out = {}
    for k in ("k_base", "k_log", "k_exp", "k_sqrt", "k_div"):
        m = re.search(r"^%s:[^\n]*\n(.*?)s_endpgm" % k, asm, re.S | re.M)
        ins = []
        for line in m.group(1).split("\n"):
            t = line.strip()
            if not t or t.startswith((";", ".")) or t.endswith(":"):
                continue
            ins.append(t.split()[0])
        out[k] = ins
    return out


def _flops(ins):
    f64 = [i for i in ins if i.startswith("v_") and "f64" in i]
    return len(f64) + sum(1 for i in f64 if "fma" in i), len(f64)


def measure():
    from .build import HIP_FLAGS, HIPCC
    with tempfile.TemporaryDirectory() as d:
        asm = os.path.join(d, "probe.s")
        subprocess.run([HIPCC, *HIP_FLAGS, "--cuda-device-only", "-S", PROBE, "-o", asm], check=True,
                       capture_output=True)
        with open(asm) as fh:
            b = _bodies(fh.read())
    base_fl, base_n = _flops(b["k_base"])
    w = {}
    for k, name in (("k_log", "log"), ("k_exp", "exp"), ("k_sqrt", "sqrt"), ("k_div", "div")):
        fl, n = _flops(b[k])
        # the baseline's one multiply stands for the operation itself
        w[name] = {"flops": fl - base_fl + 1, "fp64_instructions": n - base_n + 1}
    return w


def main():
    w = measure()
    try:
        with open(MODEL) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        data = {}
    data["fp64_weights"] = dict(w, source="python -m paper_2312_07874_amd.flopweights (gfx950 code of "
                                          "measure/probe_fp64_ops.hip, FMA = 2 flops)")
    with open(MODEL, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(json.dumps(w, indent=1))


if __name__ == "__main__":
    main()
