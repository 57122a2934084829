#!/usr/bin/env python3
"""Benchmark of the entropy-stable modal DSEM residual on one MI355X.

A step is one classical RK4 step on the workload (4 residual evaluations, each
the whole path: entropy projection, flux differencing, facet correction,
interface flux, weight-adjusted inverse; the stage combinations are fused into
the right-hand-side kernel's output), with the state resident in HBM.  Prints
one JSON line:

  value     FP64 residual evaluations x DOF per second (DOF = elements x (d+2) x modes)
  roofline  for the dominant kernel (the right-hand-side kernel K2, with its
            fused stage combination): algorithmic flops or bytes per launch,
            whichever bound is binding, / its average duration, from HIP events
            recorded around every launch on its stream during the timed steps
  cpu_baseline  the dense FP64 oracle on a bounded sample of the same workload

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402

METRIC = "FP64 residual evals × DOF/s and flux-pairs/s vs FP64 roofline; VJP/forward cost"

WORKLOADS = {
    "vortex_tri_M64_p4": lambda: wl.vortex_tri(M=64, degree=4),
    "vortex_tri_M64_p8": lambda: wl.vortex_tri(M=64, degree=8),
    "tgv_tet_M16_p4": lambda: wl.tgv_tet(M=16, degree=4),
    "tgv_tet_M16_p6": lambda: wl.tgv_tet(M=16, degree=6),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ("device.hpp", "physics.hpp", "kernels.hip", "plan.hpp")


def kernel_source_hash() -> str:
    """sha256 over the sources the right-hand-side kernel is built from."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2312_07874_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(name: str):
    """HBM bytes per K2 launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs
    recorded in profiles/traffic.json, if they were taken on these kernel
    sources (else None)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    w = t.get("workloads", {}).get(name)
    return None if w is None else w["read_bytes_per_launch"] + w["write_bytes_per_launch"]


def run_gpu(name: str, steps: int, warmup: int, autotune: bool = True):
    import torch

    import paper_2312_07874_amd as esd
    from paper_2312_07874_amd import perfmodel as pm

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
    blocks = plan.tuning()
    blocks_k1 = plan.tuning_k1()
    dt = 1e-4
    if warmup:
        plan.rk4(u, dt, warmup)
    torch.cuda.synchronize()
    plan.sync_status()
    plan.set_timing(True)
    plan.get_timing()
    torch.cuda.synchronize()
    # the timed steps: one call (one projection of u, then per stage one kernel
    # that forms the stage combination and projects the next stage input)
    t0 = time.perf_counter()
    plan.rk4(u, dt, steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plan.set_timing(False)
    k1_ms, k2_ms, nlaunch = plan.get_timing()
    plan.sync_status()
    fused = plan.tuning_fused()
    info = plan.info
    n_res = 4 * steps
    d, p = wk.dim, wk.degree
    k2_avg_s = k2_ms / nlaunch * 1e-3
    res_k1_ms, res_k2_ms = time_residual_kernels(plan, u)
    # the dominant kernel of a stage: K2 forming the stage combination, and,
    # with fused stages, projecting the next stage input
    fl = pm.k2_flops(d, p, wk.ecflux, wk.dissipation) * info.n_elements
    if fused:
        fl += pm.k1_flops(d, p) * info.n_elements
    by = (pm.k2_next_bytes(d, p) if fused else pm.k2_rk_bytes(d, p)) * info.n_elements
    t_fl = fl / (pm.PEAK_FP64_TFLOPS * 1e12)
    t_by = by / (pm.PEAK_HBM_GBS * 1e9)
    if t_fl >= t_by:
        roof = {"bound": "alu", "achieved": fl / k2_avg_s / 1e12, "peak": pm.PEAK_FP64_TFLOPS, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": by / k2_avg_s / 1e9, "peak": pm.PEAK_HBM_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(name)
    roof["kernel"] = ("k_rhs<..., true> (RK4 stage: right-hand side, stage combination, next projection)" if fused
                      else "k_rhs<..., false> (RK4 stage: right-hand side and stage combination; K1 separate)")
    roof["algorithmic_flops_per_launch"] = fl
    roof["algorithmic_bytes_per_launch"] = by
    roof["avg_launch_ms"] = k2_avg_s * 1e3
    vjp = time_vjp(plan, u)
    graph_ms = time_graph_steps(plan, u, dt, steps)
    return {
        "workload": name,
        "elements": info.n_elements,
        "degree": p,
        "dof": info.n_dof,
        "value": n_res * info.n_dof / elapsed,
        "ms_per_step": elapsed / steps * 1e3,
        "rk4_stages_fused": fused,
        "ms_per_stage_kernel": k2_avg_s * 1e3,
        "ms_per_stage_k1": k1_ms / nlaunch,
        "ms_per_residual_k1_k2": res_k1_ms + res_k2_ms,
        "k1_avg_ms": res_k1_ms,
        "k2_avg_ms": res_k2_ms,
        "flux_pairs_per_s": n_res * info.flux_pairs_paper / elapsed,
        "flux_pairs_distinct_per_s": n_res * info.flux_pairs_distinct / elapsed,
        "roofline": roof,
        "k1_flop_rate_tflops": pm.k1_flops(d, p) * info.n_elements / res_k1_ms / 1e9,
        "vjp": vjp,
        "k2_block_autotuned": blocks[0],
        "k1_block_autotuned": blocks_k1[0],
        "ms_per_step_graph": graph_ms,
    }


def time_residual_kernels(plan, u, reps: int = 5):
    """K1 and K2 of the plain residual (esd_residual), from HIP events around
    each launch: (K1 ms, K2 ms) averages."""
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
    return k1 / n, k2 / n


def time_graph_steps(plan, u, dt, steps):
    """The same RK4 steps replayed from the captured graph (no per-kernel events)."""
    import torch

    plan.rk4(u, dt, 1)            # capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.rk4(u, dt, steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    plan.sync_status()
    return ms


def time_vjp(plan, u, reps: int = 5):
    """Cost of one residual VJP (forward projection + the two adjoint kernels)
    against one residual evaluation, both timed with events on the stream the
    library launches on (torch's current stream)."""
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


def run_batched(steps: int, warmup: int):
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
    blocks = plan.autotune(u)
    dt = 1e-4
    if warmup:
        plan.rk4(u, dt, warmup)
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.get_timing()
    t0 = time.perf_counter()
    plan.rk4(u, dt, steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plan.set_timing(False)
    stage_k1_ms, stage_ms, nstage = plan.get_timing()
    plan.sync_status()
    res_k1_ms, res_k2_ms = time_residual_kernels(plan, u)
    graph_ms = time_graph_steps(plan, u, dt, steps)
    n_res = 4 * steps
    return {
        "workload": bt.name,
        "elements": int(plan.info.n_elements),
        "dof": int(plan.info.n_dof),
        "buckets": [[b["degree"], int(b["n_elements"])] for b in plan.buckets],
        "value": n_res * plan.info.n_dof / elapsed,
        "ms_per_step": elapsed / steps * 1e3,
        "rk4_stages_fused": plan.tuning_fused(),
        "ms_per_stage_all_buckets": (stage_k1_ms + stage_ms) / nstage,
        "ms_per_residual_k1_k2": res_k1_ms + res_k2_ms,
        "k1_and_interfaces_avg_ms": res_k1_ms,
        "k2_all_buckets_avg_ms": res_k2_ms,
        "flux_pairs_per_s": n_res * plan.info.flux_pairs_paper / elapsed,
        "k2_blocks_autotuned": blocks,
        "ms_per_step_graph": graph_ms,
    }


def run_adjoint(nsteps: int = 20):
    """The gradient workload: tgv tet M12 p6 (10,368 curved tetrahedra), nsteps
    RK4 steps forward with the stage inputs checkpointed, then the discrete
    adjoint of those steps for a seeded random cotangent of the final state;
    times against the same steps without checkpoints, and the checkpoint memory."""
    import torch

    import paper_2312_07874_amd as esd

    wk = wl.tgv_tet(M=12, degree=6)
    plan = esd.Plan.from_workload(wk)
    x = plan.node_coords().cpu().numpy()
    u0 = plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
    plan.autotune(u0)
    dt = 1e-3
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
        "workload": f"{wk.name} gradient over {nsteps} RK4 steps",
        "elements": plan.info.n_elements,
        "dof": plan.info.n_dof,
        "forward_ms": fwd,
        "forward_checkpointed_ms": fwd_ck,
        "adjoint_ms": adj,
        "gradient_over_forward": (fwd_ck + adj) / fwd,
        "adjoint_over_forward": adj / fwd,
        "checkpoint_bytes": ckpt.numel() * 8,
        "rk4_stages_fused": plan.tuning_fused(),
    }


def cpu_baseline(name: str, budget_s: float):
    """The oracle (dense FP64, PyTorch CPU) timed on a bounded element sample."""
    import torch

    from oracle import residual as R

    wk = WORKLOADS[name]()
    t0 = time.perf_counter()
    prob = R.setup(wk.mesh(), wk.degree, wk.warp, wk.gamma, wk.ecflux, wk.dissipation)
    ut = R.project(prob, torch.tensor(wk.state(prob.geo.x_vol.numpy())))
    log(f"[bench] oracle setup {time.perf_counter() - t0:.1f}s")
    rng = np.random.default_rng(0)
    order = rng.permutation(prob.ne)
    chunk = 8
    done, spent = 0, 0.0
    while spent < budget_s and done < prob.ne:
        el = order[done:done + chunk]
        t = time.perf_counter()
        R.residual(prob, ut, el)
        spent += time.perf_counter() - t
        done += len(el)
    ndof = done * prob.nc * prob.ref.Np
    return {"value": ndof / spent, "unit": "DOF*residual-evals/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"dense oracle residual of {done} of {prob.ne} elements of {name} "
                      f"(each with its neighbours' entropy projection), {spent:.1f}s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="vortex_tri_M64_p4", choices=sorted(WORKLOADS))
    ap.add_argument("--extra", default="vortex_tri_M64_p8,tgv_tet_M16_p4,tgv_tet_M16_p6",
                    help="comma-separated additional workloads reported under 'extra' ('' for none)")
    ap.add_argument("--extra-steps", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched mixed-degree workload")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the 20-step gradient workload")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default block sizes")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="finish with a plain 1 GiB device-to-device copy (counter calibration for profiles)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see the sharding "
              "design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    main_res = run_gpu(args.workload, args.steps, args.warmup, not args.no_autotune)
    extra = []
    for name in [s for s in args.extra.split(",") if s]:
        if name != args.workload:
            extra.append(run_gpu(name, args.extra_steps, 1, not args.no_autotune))
    if not args.no_batched:
        extra.append(run_batched(args.extra_steps, 1))
    if not args.no_adjoint:
        extra.append(run_adjoint())
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.workload, args.cpu_seconds)
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
        "config": {"workload": args.workload, "elements": main_res["elements"], "degree": main_res["degree"],
                   "dof": main_res["dof"],
                   "step": "one classical RK4 step (4 residual evaluations + stage combinations)"},
        "flux_pairs_per_s": main_res["flux_pairs_per_s"],
        "flux_pairs_distinct_per_s": main_res["flux_pairs_distinct_per_s"],
        "rk4_stages_fused": main_res["rk4_stages_fused"],
        "ms_per_stage_kernel": main_res["ms_per_stage_kernel"],
        "ms_per_residual_k1_k2": main_res["ms_per_residual_k1_k2"],
        "ms_per_step_graph": main_res["ms_per_step_graph"],
        "k1_avg_ms": main_res["k1_avg_ms"],
        "k2_block_autotuned": main_res["k2_block_autotuned"],
        "k1_block_autotuned": main_res["k1_block_autotuned"],
        "roofline": main_res["roofline"],
        "vjp_over_forward": main_res["vjp"]["vjp_over_forward"],
        "vjp": main_res["vjp"],
        "cpu_baseline": cpu,
        "extra": extra,
    }
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
