"""GPU checks of the deterministic right-hand side (esd_plan_set_deterministic):
the fixed-order sums give the oracle's residual (same bar as the default
mode), and residuals and RK4 steps repeat bit for bit, on single-degree and
batched plans."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from tests.parity_util import assert_parity, gpu_plan, log, oracle_problem, oracle_state, oracle_with_spread

pytestmark = pytest.mark.gpu

CASES = [
    ("tri_p3_random_lf", wl.random_tri(M=3, degree=3, seed=61)),
    ("tri_p8_random_ec", wl.random_tri(M=3, degree=8, seed=62, dissipation=0)),
    ("tet_p2_random_lf", wl.random_tet(M=3, degree=2, seed=63)),
    ("tet_p4_tgv_ec", wl.tgv_tet(M=3, degree=4)),
    ("tet_p7_random_lf", wl.random_tet(M=3, degree=7, seed=64)),
]


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


@pytest.mark.parametrize("name,wk", CASES, ids=[c[0] for c in CASES])
def test_deterministic_residual_parity(name, wk):
    from oracle import residual as R
    log(f"case {name}: dim={wk.dim} M={wk.M} p={wk.degree}")
    prob = oracle_problem(wk)
    ut = oracle_state(prob, wk)
    plan = gpu_plan(wk)
    plan.set_deterministic(True)
    out = plan.residual(ut.cuda().contiguous())
    plan.sync_status()
    if wk.degree <= 4:
        ref, spread = oracle_with_spread(lambda pr: R.residual_chunked(pr, ut), prob, lambda: oracle_problem(wk))
        assert_parity(out, ref, what=f"deterministic {name}", spread=spread)
    else:
        el = np.random.default_rng(9).choice(prob.ne, 3, replace=False)
        ref, spread = oracle_with_spread(lambda pr: R.residual_chunked(pr, ut, el, chunk=4), prob,
                                         lambda: oracle_problem(wk))
        assert_parity(out.cpu()[el], ref, what=f"deterministic {name} (sampled)", spread=spread)
    # against the default (atomic) mode: the same sums in another order
    plan.set_deterministic(False)
    fast = plan.residual(ut.cuda().contiguous())
    d = float((out - fast).abs().max() / fast.abs().max())
    log(f"deterministic vs default: max diff / ||r||_inf = {d:.2e}")
    assert d <= 1e-11


def _repeat(fn, n=4):
    outs = [fn().clone() for _ in range(n)]
    torch.cuda.synchronize()
    return outs


def test_deterministic_residual_and_rk4_repeat_bitwise():
    """3,072 curved tetrahedra at p = 6 (Taylor-Green, EC): five residuals and
    two 3-step RK4 runs (graph replay) from the same state are identical bit for
    bit; the default mode is reported for comparison."""
    wk = wl.tgv_tet(M=8, degree=6)
    plan = gpu_plan(wk)
    x = plan.node_coords().cpu().numpy()
    u = plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
    plan.set_deterministic(False)
    fast = _repeat(lambda: plan.residual(u))
    nd = sum(not torch.equal(fast[0], f) for f in fast[1:])
    log(f"default mode: {nd} of {len(fast) - 1} repeats differ from the first "
        f"(max {max(float((fast[0] - f).abs().max()) for f in fast[1:]):.2e})")
    plan.set_deterministic(True)
    det = _repeat(lambda: plan.residual(u), 5)
    for k, r in enumerate(det[1:]):
        assert torch.equal(det[0], r), f"repeat {k + 1} differs"
    runs = []
    for _ in range(2):
        v = u.clone()
        plan.rk4(v, 1e-3, 3)
        runs.append(v)
    plan.sync_status()
    assert torch.equal(runs[0], runs[1])
    d = plan.diagnostics(runs[0])
    d2 = plan.diagnostics(runs[1])
    assert d["entropy"] == d2["entropy"] and np.array_equal(d["conserved"], d2["conserved"])
    log("deterministic: 5 residuals, two RK4 runs and their diagnostics identical")


def test_deterministic_batched_plan_repeats_bitwise():
    """A mixed-degree batch (p = 2..6, two tetrahedral meshes): residuals in
    the deterministic mode repeat bit for bit and agree with the default mode
    to rounding."""
    import paper_2312_07874_amd as esd
    L = 2 * math.pi
    warp = wl.make_warp_sinprod(L, 0.05)
    m1, m2 = wl.split_box_mesh(3, 4, L), wl.split_box_mesh(3, 5, L)
    d1, d2 = wl.mixed_degrees(m1.n_elements, 71, 2, 6), wl.mixed_degrees(m2.n_elements, 72, 2, 6)
    plan = esd.BatchedPlan(3, [(m.elem_vertex_ids, m.elem_vertex_coords, d) for m, d in ((m1, d1), (m2, d2))],
                           warp, 1.4, 0, 1)
    st = wl.RandomSmooth(3, L, 5)
    x = plan.node_coords().cpu().numpy()
    u = plan.project(torch.tensor(st(x), device="cuda").reshape(plan.nodal_shape).contiguous())
    fast = plan.residual(u)
    plan.set_deterministic(True)
    det = _repeat(lambda: plan.residual(u))
    plan.sync_status()
    for r in det[1:]:
        assert torch.equal(det[0], r)
    diff = float((det[0] - fast).abs().max() / fast.abs().max())
    log(f"batched deterministic vs default: {diff:.2e}")
    assert diff <= 1e-11
