"""esd_residual_noalloc (library scratch, no allocation) against esd_residual
(caller workspace): bitwise-level agreement is not expected (LDS accumulation
order varies between runs), so both are held to the oracle-free bar of 1e-13
relative per conserved variable against each other, on two calls in a row, the
second with a smaller mesh (its scratch keeps the first call's contents)."""
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


def _state(plan, wk):
    x = plan.node_coords().cpu().numpy()
    f = wk.state if hasattr(wk, "state") else wk
    return plan.project(torch.tensor(f(x), device="cuda").reshape(plan.nodal_shape).contiguous())


def _compare(plan, u, what):
    ref = plan.residual(u)
    out = torch.full_like(u, float("nan"))
    plan.residual_noalloc(u, out)
    plan.sync_status()
    torch.cuda.synchronize()
    ref, out = ref.cpu(), out.cpu()
    assert bool(torch.isfinite(out).all()), what
    buckets = range(len(plan.buckets)) if hasattr(plan, "buckets") else [None]
    for b in buckets:
        rb = ref if b is None else plan.bucket_view(ref, b)
        ob = out if b is None else plan.bucket_view(out, b)
        for c in range(rb.shape[1]):
            err = float((ob[:, c] - rb[:, c]).abs().max())
            scale = float(rb[:, c].abs().max())
            log(f"noalloc {what} bucket {b} variable {c}: max |noalloc - residual| / ||r||_inf = {err / scale:.2e}")
            assert err <= 1e-13 * scale, what


def test_noalloc_matches_residual_two_calls_second_smaller():
    big = wl.random_tet(M=4, degree=5, seed=31)        # 384 tets
    small = wl.random_tet(M=3, degree=3, seed=32)      # 162 tets
    pb = gpu_plan(big)
    _compare(pb, _state(pb, big), "tet M4 p5")
    ps = gpu_plan(small)
    _compare(ps, _state(ps, small), "tet M3 p3 after M4 p5")


def test_noalloc_batched_and_triangles():
    import paper_2312_07874_amd as esd
    L = 2.0
    warp = wl.make_warp_sinprod(L, 0.05)
    mesh = wl.split_box_mesh(2, 4, L)
    deg = wl.mixed_degrees(mesh.n_elements, 5, 2, 6)
    plan = esd.BatchedPlan(2, [(mesh.elem_vertex_ids, mesh.elem_vertex_coords, deg)], warp, 1.4, 0, 1)
    _compare(plan, _state(plan, wl.RandomSmooth(2, L, 4)), "batched tri p2..6")
    tri = wl.random_tri(M=3, degree=8, seed=33)
    pt = gpu_plan(tri)
    _compare(pt, _state(pt, tri), "tri M3 p8")


def test_noalloc_rejects_oversized_workspace():
    import paper_2312_07874_amd as esd
    wk = wl.tgv_tet(M=16, degree=6)                    # 275 MB workspace
    plan = gpu_plan(wk)
    assert plan.info.workspace_bytes > 64 << 20
    u = torch.zeros(plan.state_shape, dtype=torch.float64, device="cuda")
    with pytest.raises(esd.EsdError) as e:
        plan.residual_noalloc(u, torch.empty_like(u))
    assert e.value.status == -1
