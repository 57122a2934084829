"""Long-time robustness runs (Sec. 7.5 of the paper): under-resolved
Kelvin-Helmholtz instability on triangles and Taylor-Green vortex on
tetrahedra, entropy-conservative (no interface dissipation) against entropy-
stable (Lax-Friedrichs interface flux), with the entropy integral monitored.
Every step runs on the GPU path (esd_rk4, esd_diagnostics); the paper used an
eighth-order Dormand-Prince integrator, this driver the classical RK4 with a
fixed step from an initial wave-speed estimate.

    python -m paper_2312_07874_amd.robustness [--problems khi,tgv0.1,tgv0.7] [--degrees 4,5,6,7,8]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import EsdError, Plan


def stable_dt(wk, plan, cfl: float) -> float:
    """cfl * h / ((p+1)^2 * max(|v| + c)) from the initial state at the volume nodes."""
    x = plan.node_coords().cpu().numpy()
    u = wk.state(x)
    d = wk.dim
    rho = u[..., 0]
    v = u[..., 1:1 + d] / rho[..., None]
    p = (wk.gamma - 1.0) * (u[..., d + 1] - 0.5 * rho * (v * v).sum(-1))
    lam = float((np.sqrt((v * v).sum(-1)) + np.sqrt(wk.gamma * p / rho)).max())
    h = wk.L / wk.M
    return cfl * h / ((wk.degree + 1) ** 2 * lam)


def run(wk, T: float, cfl: float = 0.5, snapshots: int = 100, log=None) -> dict:
    """Integrates wk to time T.  Returns whether it completed, the time reached,
    and (time, entropy, entropy rate) at about `snapshots` instants."""
    import torch

    plan = Plan.from_workload(wk)
    x = plan.node_coords().cpu().numpy()
    u = plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
    plan.sync_status()
    dt = stable_dt(wk, plan, cfl)
    nsteps = int(math.ceil(T / dt))
    dt = T / nsteps
    chunk = max(1, nsteps // snapshots)
    hist = []
    t, done, ok = 0.0, 0, True
    t0 = time.perf_counter()
    d = plan.diagnostics(u)
    hist.append((t, d["entropy"], d["entropy_rate"]))
    while done < nsteps:
        n = min(chunk, nsteps - done)
        plan.rk4(u, dt, n)
        try:
            plan.sync_status()
            d = plan.diagnostics(u)
        except EsdError:
            ok = False
            break
        if not (math.isfinite(d["entropy"]) and math.isfinite(d["entropy_rate"])):
            ok = False
            break
        done += n
        t = done * dt
        hist.append((t, d["entropy"], d["entropy_rate"]))
    wall = time.perf_counter() - t0
    res = {"workload": wk.name, "dissipation": wk.dissipation, "completed": ok, "t_end": t if ok else done * dt,
           "T": T, "dt": dt, "steps": done, "wall_s": wall,
           "entropy_change": hist[-1][1] - hist[0][1],
           "max_entropy_rate": max(h[2] for h in hist),
           "entropy_nonincreasing": all(hist[i + 1][1] <= hist[i][1] + 1e-12 * abs(hist[0][1])
                                        for i in range(len(hist) - 1)),
           "history": hist}
    if log:
        log(f"{wk.name} {'ES' if wk.dissipation else 'EC'}: {'completed' if ok else 'failed'} at t = "
            f"{res['t_end']:.3f} / {T} ({done} steps of {dt:.2e}, {wall:.1f} s), entropy change "
            f"{res['entropy_change']:.3e}, max entropy rate {res['max_entropy_rate']:.3e}")
    return res


def main():
    import workloads as wl

    ap = argparse.ArgumentParser()
    ap.add_argument("--problems", default="khi,tgv0.1,tgv0.7")
    ap.add_argument("--degrees", default="4,5,6,7,8")
    ap.add_argument("--cfl", type=float, default=0.5)
    ap.add_argument("--out", default=None, help="write the results (without histories) as JSON")
    args = ap.parse_args()
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    results = []
    for prob in args.problems.split(","):
        for p in [int(s) for s in args.degrees.split(",")]:
            for diss in (0, 1):
                if prob == "khi":
                    wk, T = wl.khi_tri(16, p, diss), 15.0
                else:
                    wk, T = wl.tgv_tet_mach(4, p, float(prob[3:]), diss), 14.0
                results.append(run(wk, T, args.cfl, log=log))
    slim = [{k: v for k, v in r.items() if k != "history"} for r in results]
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(slim, fh, indent=1)
    print(json.dumps(slim))


if __name__ == "__main__":
    main()
