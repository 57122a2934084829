"""Graph-replayed RK4 steps and the right-hand-side autotuner.

Every replay is compared with the same step launched kernel by kernel, with
the program's own eager work and synchronisations between replays; equality
is up to the order of the LDS atomic sums (1e-13 of the state per variable)."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from tests.parity_util import gpu_plan, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def _close(a, b, what):
    a, b = a.detach().cpu(), b.detach().cpu()
    err = float((a - b).abs().max())
    scale = float(b.abs().max())
    log(f"{what}: max |graph - eager| / max |eager| = {err / scale:.2e}")
    assert err <= 1e-13 * scale, what


def _replays_match_eager(plan, u0, dt, nrep):
    ug = u0.clone()
    ue = u0.clone()
    scratch = torch.empty_like(u0)
    for r in range(nrep):
        plan.set_graphs(True)
        plan.rk4(ug, dt, 1)                      # replay (captured at r = 0)
        plan.residual(ue, scratch)               # unrelated eager work between replays
        torch.cuda.synchronize()
        plan.set_graphs(False)
        plan.rk4(ue, dt, 1)
        torch.cuda.synchronize()
        plan.sync_status()
        _close(ug, ue, f"replay {r}")
    # several replays in one call
    plan.set_graphs(True)
    plan.rk4(ug, dt, 3)
    plan.set_graphs(False)
    plan.rk4(ue, dt, 3)
    torch.cuda.synchronize()
    _close(ug, ue, "3 replays in one call")


def test_graph_rk4_single_plan():
    wk = wl.random_tet(M=3, degree=3, seed=7)
    plan = gpu_plan(wk)
    x = plan.node_coords().cpu().numpy()
    u0 = plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
    _replays_match_eager(plan, u0, 1e-3, 4)


def test_graph_rk4_batched_plan():
    import paper_2312_07874_amd as esd
    L = 2 * math.pi
    m = wl.split_box_mesh(3, 3, L)
    deg = wl.mixed_degrees(m.n_elements, 3, 2, 5)
    plan = esd.BatchedPlan(3, [(m.elem_vertex_ids, m.elem_vertex_coords, deg)], wl.make_warp_sinprod(L, 0.05))
    x = plan.node_coords().cpu().numpy()
    u0 = plan.project(torch.tensor(wl.RandomSmooth(3, L, 2)(x), device="cuda").reshape(plan.nodal_shape).contiguous())
    _replays_match_eager(plan, u0, 1e-3, 3)


def test_autotune_keeps_the_residual():
    wk = wl.random_tet(M=3, degree=6, seed=9)
    plan = gpu_plan(wk)
    x = plan.node_coords().cpu().numpy()
    u = plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
    before = plan.residual(u).clone()
    blocks = plan.autotune(u)
    after = plan.residual(u)
    plan.sync_status()
    log(f"autotuned right-hand-side block: {blocks}, fused RK4 stages: {plan.tuning_fused()}")
    assert blocks[0] % 64 == 0 and 64 <= blocks[0] <= 512
    _close(after, before, "residual after autotune")


def _fused_matches_stage_by_stage(plan, u0, dt):
    """esd_rk4 without checkpoints, with fused stages (one projection per call,
    then per stage one kernel forming the stage combination and projecting the
    next stage input, alternating two workspaces) and without, against esd_rk4
    with stage checkpoints (stages unfused), eager and graph, over several
    steps and across calls."""
    n = u0.numel()
    ref = u0.clone()
    ckpt = torch.empty((4 * 4, n), dtype=torch.float64, device="cuda")
    plan.rk4(ref, dt, 4, ckpt=ckpt)
    for fused in (True, False):
        plan.set_fused(fused)
        assert plan.tuning_fused() == fused
        for graphs in (False, True):
            plan.set_graphs(graphs)
            one = u0.clone()
            plan.rk4(one, dt, 4)
            two = u0.clone()
            plan.rk4(two, dt, 1)
            plan.rk4(two, dt, 3)
            torch.cuda.synchronize()
            plan.sync_status()
            _close(one, ref, f"4 steps (fused {fused}, graphs {graphs}) vs checkpointed")
            _close(two, ref, f"1 + 3 steps (fused {fused}, graphs {graphs}) vs checkpointed")
        # the checkpointed stage inputs agree with the first step
        u1 = u0.clone()
        plan.set_graphs(False)
        plan.rk4(u1, dt, 1)
        _close(ckpt[4].reshape(u0.shape), u1, f"stage-1 input of step 2 (fused {fused})")


def test_fused_rk4_single_plans():
    for wk in (wl.random_tri(M=4, degree=5, seed=3), wl.random_tet(M=3, degree=4, seed=5)):
        plan = gpu_plan(wk)
        x = plan.node_coords().cpu().numpy()
        u0 = plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
        log(f"{wk.name}")
        _fused_matches_stage_by_stage(plan, u0, 2e-3)


@pytest.mark.parametrize("dim,p", [(2, 9), (2, 10), (3, 9), (3, 10)])
def test_fused_rk4_high_degree(dim, p):
    """The fused stage kernel where K2 keeps its tables in the facet-record
    buffer's tail (tet p = 9), keeps its facet records in the workspace
    (tet p = 10) or runs three triangles per workgroup (tri p >= 8)."""
    wk = wl.random_tri(M=3, degree=p, seed=11) if dim == 2 else wl.random_tet(M=3, degree=p, seed=13)
    plan = gpu_plan(wk)
    x = plan.node_coords().cpu().numpy()
    u0 = plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
    log(f"{wk.name}")
    _fused_matches_stage_by_stage(plan, u0, 1e-3)


def test_fused_rk4_batched_plan():
    import paper_2312_07874_amd as esd
    L = 2 * math.pi
    m = wl.split_box_mesh(3, 3, L)
    deg = wl.mixed_degrees(m.n_elements, 11, 1, 6)
    plan = esd.BatchedPlan(3, [(m.elem_vertex_ids, m.elem_vertex_coords, deg)], wl.make_warp_sinprod(L, 0.05))
    x = plan.node_coords().cpu().numpy()
    u0 = plan.project(torch.tensor(wl.RandomSmooth(3, L, 4)(x), device="cuda").reshape(plan.nodal_shape).contiguous())
    _fused_matches_stage_by_stage(plan, u0, 2e-3)


def test_plan_memory_from_torch_allocator():
    """esd_plan_create_ex with a torch-backed allocator: the plan's own arrays
    are torch blocks (counted by torch, released at destroy) and the residual
    is the same as with the library's own allocation."""
    import gc

    import paper_2312_07874_amd as esd
    wk = wl.random_tet(M=3, degree=4, seed=61)
    mesh = wk.mesh()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    alloc = esd.TorchAllocator()
    plan = esd.Plan(3, 4, mesh.elem_vertex_ids, mesh.elem_vertex_coords, wk.warp, wk.gamma, wk.ecflux,
                    wk.dissipation, allocator=alloc)
    held = alloc.bytes
    assert held > 0 and torch.cuda.memory_allocated() - before >= held
    ref_plan = esd.Plan.from_workload(wk)
    x = ref_plan.node_coords().cpu().numpy()
    u = ref_plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
    a, b = plan.residual(u), ref_plan.residual(u)
    plan.sync_status()
    ref_plan.sync_status()
    for c in range(a.shape[1]):
        assert float((a[:, c] - b[:, c]).abs().max()) <= 1e-13 * float(b[:, c].abs().max())
    del plan
    gc.collect()
    assert alloc.bytes == 0


def test_batched_plan_memory_from_torch_allocator():
    import gc

    import paper_2312_07874_amd as esd
    L = 2.0
    mesh = wl.split_box_mesh(2, 3, L)
    deg = wl.mixed_degrees(mesh.n_elements, 62, 1, 4)
    alloc = esd.TorchAllocator()
    plan = esd.BatchedPlan(2, [(mesh.elem_vertex_ids, mesh.elem_vertex_coords, deg)], wl.make_warp_sinprod(L, 0.05),
                           1.4, 0, 1, allocator=alloc)
    ref = esd.BatchedPlan(2, [(mesh.elem_vertex_ids, mesh.elem_vertex_coords, deg)], wl.make_warp_sinprod(L, 0.05),
                          1.4, 0, 1)
    assert alloc.bytes > 0
    x = ref.node_coords().cpu().numpy()
    u = ref.project(torch.tensor(wl.RandomSmooth(2, L, 3)(x), device="cuda").reshape(ref.nodal_shape).contiguous())
    a, b = plan.residual(u), ref.residual(u)
    plan.sync_status()
    assert float((a - b).abs().max()) <= 1e-13 * float(b.abs().max())
    del plan
    gc.collect()
    assert alloc.bytes == 0
