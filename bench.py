#!/usr/bin/env python3
"""Benchmark of the entropy-stable modal DSEM residual on one MI355X.

A step is one classical RK4 step of the workload (4 residual evaluations, each
the whole path: entropy projection, flux differencing, facet correction,
interface flux, weight-adjusted inverse; the stage combinations are formed by
the right-hand-side kernel), with the state resident in HBM, replayed from the
plan's captured HIP graph.  The headline workload is the largest single-GPU
configuration: four periodic meshes of curved tetrahedra (6 M^3 elements,
M = 8, 10, 12, 14; 35,904 elements) with per-element degrees uniform on
2..10 in one batched plan.  Prints one JSON line:

  value     FP64 residual evaluations x DOF per second (DOF = elements x (d+2) x modes)
  roofline  the right-hand-side kernel K2 (all degree buckets of the residual):
            algorithmic FP64 flops per launch (perfmodel: the oracle's formulas,
            transcendentals and divisions weighted by their gfx950 instruction
            cost) / its average duration from HIP events recorded around every
            launch on its stream; "residual" gives the same for K1 + K2 (+ the
            mixed-degree interface kernel)
  cpu_baseline  the dense FP64 oracle on a bounded element sample, all
            physical host cores; cpu_baseline_protocol adds the 1-core run and
            the median of 5 on a cheap workload
  extra     Taylor-Green tetrahedra at p = 4..10, the vortex triangles at p = 4
            and 8, and the 20-step gradient workload

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402

METRIC = "FP64 residual evals × DOF/s and flux-pairs/s vs FP64 roofline; VJP/forward cost"
HEADLINE = "batched_tets_M8-10-12-14_p2-10"

# Taylor-Green tetrahedra at p = 4..10 (at p = 9, 10 a smaller mesh keeps the
# plan's geometry and workspaces near 1 GB), the vortex triangles at p = 4, 8
WORKLOADS = {n: (lambda n=n: wl.named(n)) for n in
             [f"tgv_tet_M16_p{p}" for p in range(4, 9)] + ["tgv_tet_M12_p9", "tgv_tet_M12_p10",
                                                           "vortex_tri_M64_p4", "vortex_tri_M64_p8"]}
DEFAULT_EXTRA = ",".join(WORKLOADS)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(name: str):
    from paper_2312_07874_amd import profiling
    return profiling.measured_traffic(name)


# ---------------------------------------------------------------- roofline
def _roof(flops: float, bytes_: float, seconds: float, kernel: str, traffic=None):
    from paper_2312_07874_amd import perfmodel as pm
    t_fl = flops / (pm.PEAK_FP64_TFLOPS * 1e12)
    t_by = bytes_ / (pm.PEAK_HBM_GBS * 1e9)
    if t_fl >= t_by:
        r = {"bound": "alu", "achieved": flops / seconds / 1e12, "peak": pm.PEAK_FP64_TFLOPS, "unit": "TFLOP/s"}
    else:
        r = {"bound": "hbm", "achieved": bytes_ / seconds / 1e9, "peak": pm.PEAK_HBM_GBS, "unit": "GB/s"}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = traffic
    r["kernel"] = kernel
    r["algorithmic_flops_per_launch"] = flops
    r["algorithmic_bytes_per_launch"] = bytes_
    r["avg_launch_ms"] = seconds * 1e3
    return r


def _work(buckets, ecflux, dissipation, dim):
    """Algorithmic flops (K1, K2) and minimum / layout bytes per residual over
    the buckets [(degree, elements)]."""
    from paper_2312_07874_amd import perfmodel as pm
    k1 = k2 = mb = lb = 0
    for p, n in buckets:
        f = pm.residual_flops(dim, p, ecflux, dissipation)
        k1 += n * f["k1"]
        k2 += n * f["k2"]
        mb += n * pm.min_bytes(dim, p)
        lb += n * pm.layout_bytes(dim, p)
    return k1, k2, mb, lb


# ---------------------------------------------------------------- timing helpers
def time_residual_kernels(plan, u, reps: int = 5):
    """K1 (with the mixed-degree interface kernel of batched plans) and K2 of
    the plain residual (esd_residual), from HIP events around each launch on
    its stream: (K1 ms, K2 ms) averages per residual."""
    import torch

    out = torch.empty_like(u)
    plan.residual(u, out)
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.get_timing()
    for _ in range(reps):
        plan.residual(u, out)
    k1, k2, n = plan.get_timing()
    plan.set_timing(False)
    plan.sync_status()
    return k1 / n, k2 / n


def time_rk4_steps(plan, u, dt, steps, warmup):
    """RK4 steps replayed from the plan's captured graph: ms per step."""
    import torch

    plan.rk4(u, dt, max(1, warmup))   # captures the graph
    torch.cuda.synchronize()
    plan.sync_status()
    t0 = time.perf_counter()
    plan.rk4(u, dt, steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plan.sync_status()
    return elapsed


def time_vjp(plan, u, reps: int = 5):
    """One residual VJP (forward projection + the two adjoint kernels) against
    one residual evaluation, both timed with events on the stream the library
    launches on (torch's current stream)."""
    import torch

    g = torch.Generator(device="cuda").manual_seed(0)
    vbar = torch.randn(tuple(u.shape), generator=g, dtype=torch.float64, device="cuda")
    out = torch.empty_like(u)
    plan.vjp(u, vbar, out)
    plan.residual(u, out)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(reps):
        plan.residual(u, out)
    ev[1].record()
    ev[2].record()
    for _ in range(reps):
        plan.vjp(u, vbar, out)
    ev[3].record()
    torch.cuda.synchronize()
    plan.sync_status()
    f = ev[0].elapsed_time(ev[1]) / reps
    b = ev[2].elapsed_time(ev[3]) / reps
    return {"residual_ms": f, "vjp_ms": b, "vjp_over_forward": b / f}


# ---------------------------------------------------------------- workloads
def _measure(plan, u, name, buckets, dim, ecflux, dissipation, steps, warmup, vjp):
    info = plan.info
    dt = 1e-4
    elapsed = time_rk4_steps(plan, u, dt, steps, warmup)
    n_res = 4 * steps
    k1_ms, k2_ms = time_residual_kernels(plan, u)
    k1f, k2f, mb, lb = _work(buckets, ecflux, dissipation, dim)
    roof = _roof(k2f, mb, k2_ms * 1e-3, "k_rhs (right-hand side; every degree bucket of one residual)",
                 measured_traffic(name))
    roof_res = _roof(k1f + k2f, mb, (k1_ms + k2_ms) * 1e-3,
                     "whole residual: k_entropy_projection (+ k_mixed_exterior) + k_rhs")
    out = {
        "workload": name,
        "elements": int(info.n_elements),
        "dof": int(info.n_dof),
        "value": n_res * info.n_dof / elapsed,
        "ms_per_step": elapsed / steps * 1e3,
        "steps": steps,
        "ms_per_residual_k1_k2": k1_ms + k2_ms,
        "k1_avg_ms": k1_ms,
        "k2_avg_ms": k2_ms,
        "flux_pairs_per_s": n_res * info.flux_pairs_paper / elapsed,
        "flux_pairs_distinct_per_s": n_res * info.flux_pairs_distinct / elapsed,
        "roofline": roof,
        "roofline_residual": roof_res,
        "algorithmic_flops_per_residual": k1f + k2f,
        "min_bytes_per_residual": mb,
        "layout_bytes_over_min_bytes": lb / mb,
        "rk4_stages_fused": plan.tuning_fused(),
    }
    if vjp:
        out["vjp"] = time_vjp(plan, u)
        out["vjp_over_forward"] = out["vjp"]["vjp_over_forward"]
    return out


def run_single(name: str, steps: int, warmup: int, autotune: bool = True):
    import torch

    import paper_2312_07874_amd as esd

    wk = WORKLOADS[name]()
    t0 = time.perf_counter()
    plan = esd.Plan.from_workload(wk)
    log(f"[bench] {name}: plan {plan.info.n_elements} elements, p={wk.degree}, "
        f"{plan.info.n_dof} DOF, setup {time.perf_counter() - t0:.1f}s")
    x = plan.node_coords().cpu().numpy()
    u = plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
    plan.sync_status()
    if autotune:
        plan.autotune(u)
        log(f"[bench] {name}: autotuned at {time.perf_counter() - t0:.1f}s")
    r = _measure(plan, u, name, [(wk.degree, plan.info.n_elements)], wk.dim, wk.ecflux, wk.dissipation, steps,
                 warmup, True)
    log(f"[bench] {name}: measured at {time.perf_counter() - t0:.1f}s")
    r["degree"] = wk.degree
    r["k2_block_autotuned"] = plan.tuning()[0]
    r["k1_block_autotuned"] = plan.tuning_k1()[0]
    return r


def run_batched(steps: int, warmup: int, autotune: bool = True):
    """Four periodic tetrahedral meshes (6 M^3 elements, M = 8, 10, 12, 14) with
    per-element degrees uniform on 2..10 in one batched plan."""
    import torch

    import paper_2312_07874_amd as esd

    bt = wl.batched_tets()
    t0 = time.perf_counter()
    plan = esd.BatchedPlan(3, [(m.elem_vertex_ids, m.elem_vertex_coords, d) for m, d in zip(bt.meshes, bt.degrees)],
                           bt.warp, bt.gamma, bt.ecflux, bt.dissipation)
    log(f"[bench] {bt.name}: plan {plan.info.n_elements} elements in {len(plan.buckets)} buckets, "
        f"{plan.info.n_dof} DOF, setup {time.perf_counter() - t0:.1f}s")
    x = plan.node_coords().cpu().numpy()
    u = plan.project(torch.tensor(bt.state(x), device="cuda").reshape(plan.nodal_shape).contiguous())
    plan.sync_status()
    blocks = plan.autotune(u) if autotune else plan.tuning()
    buckets = [(int(b["degree"]), int(b["n_elements"])) for b in plan.buckets]
    r = _measure(plan, u, bt.name, buckets, 3, bt.ecflux, bt.dissipation, steps, warmup, True)
    r["buckets"] = [list(b) for b in buckets]
    r["k2_blocks_autotuned"] = list(blocks)
    return r, plan, u


def run_adjoint(nsteps: int = 20):
    """The gradient workload: tgv tet M12 p6 (10,368 curved tetrahedra), nsteps
    RK4 steps (dt = 5e-4) forward with the stage inputs checkpointed, then the
    discrete adjoint of those steps for a seeded random cotangent of the final
    state; times against the same steps without checkpoints, and the
    checkpoint memory."""
    import torch

    import paper_2312_07874_amd as esd

    wk = wl.tgv_tet(M=12, degree=6)
    plan = esd.Plan.from_workload(wk)
    x = plan.node_coords().cpu().numpy()
    u0 = plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
    plan.autotune(u0)
    dt = 5e-4
    ckpt = torch.empty((4 * nsteps,) + tuple(u0.shape), dtype=torch.float64, device="cuda")
    g = torch.Generator(device="cuda").manual_seed(1)
    ubar0 = torch.randn(tuple(u0.shape), generator=g, dtype=torch.float64, device="cuda")
    # warm-up of every path
    plan.rk4(u0.clone(), dt, 1)
    plan.rk4(u0.clone(), dt, 1, ckpt=ckpt[:4])
    plan.rk4_vjp(ckpt[:4], dt, 1, ubar0.clone())
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    u = u0.clone()
    ev[0].record()
    plan.rk4(u, dt, nsteps)
    ev[1].record()
    u = u0.clone()
    ev[2].record()
    plan.rk4(u, dt, nsteps, ckpt=ckpt)
    ev[3].record()
    ubar = ubar0.clone()
    ev[4].record()
    plan.rk4_vjp(ckpt, dt, nsteps, ubar)
    ev[5].record()
    torch.cuda.synchronize()
    plan.sync_status()
    fwd = ev[0].elapsed_time(ev[1])
    fwd_ck = ev[2].elapsed_time(ev[3])
    adj = ev[4].elapsed_time(ev[5])
    return {
        "workload": f"{wk.name} gradient over {nsteps} RK4 steps (dt 5e-4)",
        "elements": plan.info.n_elements,
        "dof": plan.info.n_dof,
        "forward_ms": fwd,
        "forward_checkpointed_ms": fwd_ck,
        "adjoint_ms": adj,
        "gradient_over_forward": (fwd_ck + adj) / fwd,
        "adjoint_over_forward": adj / fwd,
        "checkpoint_bytes": ckpt.numel() * 8,
        "peak_memory_bytes": torch.cuda.max_memory_allocated(),
        "rk4_stages_fused": plan.tuning_fused(),
    }


def run_dense_vs_lines():
    """The all-pairs (dense-operator) residual against the line-based one on
    the same nodes (esd_residual_dense vs esd_residual), K1 and K2 timed with
    HIP events, at p = 2, 5, 10 on triangles (2 x 24^2 curved) and tetrahedra
    (6 x 5^3 curved), next to the two-point flux counts: the line-based
    kernel's distinct pairs, the all-pairs count of the dense loops, and the
    paper's reduction factors (tensor-product vs multidimensional operators on
    their own node sets, Sec. 5.3), which it counts on symmetric quadrature
    rules this library does not have."""
    import torch

    import paper_2312_07874_amd as esd

    paper = {(2, 2): 1.56, (2, 5): 2.78, (2, 10): 4.57, (3, 2): 1.88, (3, 5): 3.44, (3, 10): 10.99}
    out = []
    for (dim, p), fac in paper.items():
        wk = wl.random_tri(M=24, degree=p, seed=5) if dim == 2 else wl.random_tet(M=5, degree=p, seed=5)
        plan = esd.Plan.from_workload(wk)
        x = plan.node_coords().cpu().numpy()
        u = plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
        o = torch.empty_like(u)
        res = {}
        for kind, fn in (("lines", plan.residual), ("dense", plan.residual_dense)):
            fn(u, o)
            torch.cuda.synchronize()
            plan.set_timing(True)
            plan.get_timing()
            for _ in range(3):
                fn(u, o)
            k1, k2, n = plan.get_timing()
            plan.set_timing(False)
            res[kind] = (k1 / n, k2 / n)
        plan.sync_status()
        Q, nq = p + 1, (p + 1) ** dim
        nfq = (dim + 1) * (Q if dim == 2 else Q * Q)
        lines = plan.info.flux_pairs_distinct // plan.info.n_elements
        out.append({"dim": dim, "degree": p, "elements": int(plan.info.n_elements),
                    "k2_ms_lines": res["lines"][1], "k2_ms_dense": res["dense"][1],
                    "residual_ms_lines": sum(res["lines"]), "residual_ms_dense": sum(res["dense"]),
                    "time_ratio_k2": res["dense"][1] / res["lines"][1],
                    "time_ratio_residual": sum(res["dense"]) / sum(res["lines"]),
                    "flux_evaluations_per_element_lines": int(lines),
                    "flux_evaluations_per_element_dense": nq * nq + nq * nfq,
                    "paper_reduction_factor": fac})
        log(f"[bench] dense vs lines dim {dim} p {p}: K2 {res['dense'][1]:.3f} / {res['lines'][1]:.3f} ms")
    return out


# ---------------------------------------------------------------- CPU baseline (the oracle)
def host_cpu():
    """(physical cores, model name) from lscpu."""
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, check=True).stdout
    except (OSError, subprocess.CalledProcessError):
        return os.cpu_count() or 1, "unknown"
    kv = {}
    for line in txt.splitlines():
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        cores = int(kv.get("Core(s) per socket", "0")) * int(kv.get("Socket(s)", "1"))
    except ValueError:
        cores = 0
    return (cores or os.cpu_count() or 1), kv.get("Model name", "unknown")


def cpu_baseline_batched(buckets, per_degree=6, reps=3):
    """The oracle's residual timed on per_degree elements of every degree of the
    headline batch (on a 162-tetrahedron mesh of the same warped kind, all
    physical host cores, median of reps after one warm-up), scaled by the
    bucket sizes to one residual of the batch."""
    import torch

    from oracle import residual as R

    cores, model = host_cpu()
    torch.set_num_threads(cores)
    bt = wl.batched_tets()
    per = {}
    for p, _ in buckets:
        wk = wl.Workload(f"sample_p{p}", 3, 3, bt.L, p, bt.warp, bt.state, bt.ecflux, bt.dissipation)
        prob = R.setup(wk.mesh(), p, wk.warp, wk.gamma, wk.ecflux, wk.dissipation)
        ut = R.project(prob, torch.tensor(wk.state(prob.geo.x_vol.numpy())))
        el = list(range(7, 7 + 25 * per_degree, 25))
        R.residual(prob, ut, el)               # warm-up
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            R.residual(prob, ut, el)
            ts.append(time.perf_counter() - t)
        per[p] = statistics.median(ts) / len(el)
        log(f"[bench] oracle, {len(el)} tetrahedra at p = {p}: {per[p] * len(el):.2f}s")
    t_res = sum(n * per[p] for p, n in buckets)
    ndof = sum(n * 5 * (p + 1) * (p + 2) * (p + 3) // 6 for p, n in buckets)
    spent = sum(per.values()) * per_degree * (reps + 1)
    return {"value": ndof / t_res, "unit": "DOF*residual-evals/s", "cores": cores, "kind": "oracle",
            "cpu_model": model,
            "sample": (f"dense oracle residual of {per_degree} curved tetrahedra of each degree 2..10 (each with its "
                       f"neighbours' entropy projection; median of {reps} after one warm-up; {spent:.1f}s of CPU "
                       f"work), per-element times scaled by the bucket sizes to one residual of the "
                       f"35,904-element batch")}


def cpu_baseline_protocol(name="vortex_tri_M64_p4", nel=64, reps=5):
    """1-core and all-core median of 5 (after one warm-up) of the oracle's
    residual on a fixed element sample."""
    import torch

    from oracle import residual as R

    cores, model = host_cpu()
    wk = WORKLOADS[name]()
    prob = R.setup(wk.mesh(), wk.degree, wk.warp, wk.gamma, wk.ecflux, wk.dissipation)
    ut = R.project(prob, torch.tensor(wk.state(prob.geo.x_vol.numpy())))
    el = np.random.default_rng(0).permutation(prob.ne)[:nel]
    ndof = nel * prob.nc * prob.ref.Np
    res = {}
    for threads in (1, cores):
        torch.set_num_threads(threads)
        R.residual(prob, ut, el)
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            R.residual(prob, ut, el)
            ts.append(time.perf_counter() - t)
        res[threads] = statistics.median(ts)
    torch.set_num_threads(cores)
    return {"workload": name, "unit": "DOF*residual-evals/s", "cpu_model": model,
            "value_1_core": ndof / res[1], "value_all_cores": ndof / res[cores], "cores": cores,
            "sample": f"{nel} elements, median of {reps} after one warm-up"}


# ---------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=HEADLINE, choices=[HEADLINE] + sorted(WORKLOADS))
    ap.add_argument("--extra", default=DEFAULT_EXTRA,
                    help="comma-separated additional workloads reported under 'extra' ('' for none)")
    ap.add_argument("--extra-steps", type=int, default=4)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the 20-step gradient workload")
    ap.add_argument("--no-dense", action="store_true", help="skip the all-pairs vs line-based comparison")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default block sizes")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="finish with a plain 1 GiB device-to-device copy (counter calibration for profiles)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path (the sharding design is "
              "in the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == HEADLINE:
        main_res, _, _ = run_batched(args.steps, args.warmup, not args.no_autotune)
        config = {"workload": HEADLINE, "elements": main_res["elements"], "degrees": "2..10 (per element)",
                  "buckets": main_res["buckets"], "dof": main_res["dof"],
                  "step": "one classical RK4 step (4 residual evaluations + stage combinations), graph-replayed"}
    else:
        main_res = run_single(args.workload, args.steps, args.warmup, not args.no_autotune)
        config = {"workload": args.workload, "elements": main_res["elements"], "degree": main_res["degree"],
                  "dof": main_res["dof"],
                  "step": "one classical RK4 step (4 residual evaluations + stage combinations), graph-replayed"}
    extra = []
    for name in [s for s in args.extra.split(",") if s]:
        if name != args.workload:
            extra.append(run_single(name, args.extra_steps, 1, not args.no_autotune))
    if not args.no_adjoint:
        extra.append(run_adjoint())
    dense = None if args.no_dense else run_dense_vs_lines()
    cpu = proto = None
    if not args.no_cpu_baseline:
        if args.workload == HEADLINE:
            cpu = cpu_baseline_batched([tuple(b) for b in main_res["buckets"]])
        proto = cpu_baseline_protocol()
    out = {
        "metric": METRIC,
        "value": main_res["value"],
        "unit": "DOF*residual-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": config,
        "flux_pairs_per_s": main_res["flux_pairs_per_s"],
        "flux_pairs_distinct_per_s": main_res["flux_pairs_distinct_per_s"],
        "ms_per_residual_k1_k2": main_res["ms_per_residual_k1_k2"],
        "k1_avg_ms": main_res["k1_avg_ms"],
        "k2_avg_ms": main_res["k2_avg_ms"],
        "roofline": main_res["roofline"],
        "roofline_residual": main_res["roofline_residual"],
        "layout_bytes_over_min_bytes": main_res["layout_bytes_over_min_bytes"],
        "rk4_stages_fused": main_res["rk4_stages_fused"],
        "cpu_baseline": cpu,
        "cpu_baseline_protocol": proto,
        "extra": extra,
        "dense_vs_lines": dense,
    }
    for k in ("vjp_over_forward", "vjp", "k2_blocks_autotuned", "k2_block_autotuned", "k1_block_autotuned"):
        if k in main_res:
            out[k] = main_res[k]
    print(json.dumps(out), flush=True)
    if args.calibrate_copy:
        import torch

        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 1 GiB read + 1 GiB written")


if __name__ == "__main__":
    main()
