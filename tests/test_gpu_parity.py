"""GPU parity: the HIP library against the oracle, element by element.

Every case builds the same mesh on both sides (each side computes its own
operators and geometry), feeds the same modal state (the oracle's projection of
a seeded smooth workload state), and compares du~/dt per conserved variable:
max |gpu - oracle| <= max(1e-12 ||oracle^(e)||_inf, 4 d_e), d_e the oracle's own
rounding spread (tests/parity_util.py).  Small meshes are compared in full
(several workgroups and a ragged last block); the benchmark-size meshes and the
high degrees are compared on sampled elements that the oracle evaluates one by
one."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from tests.parity_util import assert_parity, gpu_plan, log, oracle_problem, oracle_state, oracle_with_spread

pytestmark = pytest.mark.gpu

SMALL = [
    # name, workload
    ("tri_p2_affine_chandrashekar_ec", wl.density_wave_tri(M=3, degree=2, ecflux=1, dissipation=0)),
    ("tri_p1_random_lf", wl.random_tri(M=3, degree=1, seed=1)),
    ("tri_p3_random_lf", wl.random_tri(M=3, degree=3, seed=2)),
    ("tri_p5_random_ec", wl.random_tri(M=3, degree=5, seed=3, dissipation=0)),
    ("tri_p8_random_lf", wl.random_tri(M=2 + 1, degree=8, seed=4)),
    ("tri_p10_random_ec", wl.random_tri(M=3, degree=10, seed=10, dissipation=0)),
    ("tet_p1_random_lf", wl.random_tet(M=3, degree=1, seed=5)),
    ("tet_p2_random_ec", wl.random_tet(M=3, degree=2, seed=6, dissipation=0)),
    ("tet_p3_random_lf", wl.random_tet(M=3, degree=3, seed=7)),
    ("tet_p4_tgv_ec", wl.tgv_tet(M=3, degree=4)),
    # the entropy-variable dissipation variants (scalar on the jump, matrix)
    ("tri_p4_random_entropy_jump", wl.random_tri(M=3, degree=4, seed=51, dissipation=2)),
    ("tri_p3_random_matrix", wl.random_tri(M=3, degree=3, seed=52, dissipation=3)),
    ("tet_p3_random_entropy_jump", wl.random_tet(M=3, degree=3, seed=53, dissipation=2)),
    ("tet_p4_random_matrix", wl.random_tet(M=3, degree=4, seed=54, dissipation=3)),
]


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


@pytest.mark.parametrize("name,wk", SMALL, ids=[s[0] for s in SMALL])
def test_residual_parity_small(name, wk):
    from oracle import residual as R
    log(f"case {name}: dim={wk.dim} M={wk.M} p={wk.degree}")
    prob = oracle_problem(wk)
    ut = oracle_state(prob, wk)
    ref, spread = oracle_with_spread(lambda pr: R.residual_chunked(pr, ut), prob, lambda: oracle_problem(wk))
    plan = gpu_plan(wk)
    u = ut.cuda().contiguous()
    out = plan.residual(u)
    plan.sync_status()
    torch.cuda.synchronize()
    assert_parity(out, ref, what=name, spread=spread)


PROJ = [c for c in SMALL if c[0] in ("tri_p2_affine_chandrashekar_ec", "tri_p1_random_lf", "tet_p1_random_lf",
                                     "tet_p2_random_ec")]


@pytest.mark.parametrize("name,wk", PROJ, ids=[s[0] for s in PROJ])
def test_projection_parity(name, wk):
    from oracle import residual as R
    prob = oracle_problem(wk)
    un = torch.tensor(wk.state(prob.geo.x_vol.numpy()))
    ref = R.project(prob, un)
    plan = gpu_plan(wk)
    out = plan.project(un.cuda().contiguous())
    torch.cuda.synchronize()
    assert_parity(out, ref, what=f"project {name}")
    x = plan.node_coords().cpu()
    assert float((x - prob.geo.x_vol).abs().max()) < 1e-12


def test_rk4_density_wave_parity():
    """1 residual + 10 RK4 steps, dt = 1e-3, p = 2, 128 affine triangles on
    [0,2]^2, Chandrashekar flux with entropy-conservative interface flux."""
    from oracle import residual as R
    wk = wl.density_wave_tri(M=8, degree=2, ecflux=1, dissipation=0)
    prob = oracle_problem(wk)
    ut = oracle_state(prob, wk)
    plan = gpu_plan(wk)
    u = ut.cuda().contiguous()
    assert_parity(plan.residual(u), R.residual_chunked(prob, ut), what="density wave residual")
    ref = R.rk4(prob, ut, 1e-3, 10)
    ckpt = torch.empty((40,) + tuple(u.shape), dtype=torch.float64, device="cuda")
    plan.rk4(u, 1e-3, 10, ckpt)
    plan.sync_status()
    assert_parity(u, ref, what="density wave 10 RK4 steps")
    assert float((ckpt[0].cpu() - ut).abs().max()) == 0.0
    # entropy conservation of the EC scheme at the final state (Theorem entropy stability)
    du = plan.residual(u)
    er = float(R.entropy_rate(prob, u.cpu(), du.cpu()))
    assert abs(er) < 1e-12 * float(du.abs().max()) * prob.ne


def test_vjp_of_the_entropy_variable_dissipations_is_rejected():
    import paper_2312_07874_amd as esd
    wk = wl.random_tri(M=3, degree=2, seed=55, dissipation=3)
    plan = gpu_plan(wk)
    u = torch.zeros(plan.state_shape, dtype=torch.float64, device="cuda")
    with pytest.raises(esd.EsdError) as e:
        plan.vjp(u, u.clone())
    assert e.value.status == -4


def test_inadmissible_state_sets_flag():
    import paper_2312_07874_amd as esd
    wk = wl.random_tri(M=3, degree=2, seed=9)
    prob = oracle_problem(wk)
    ut = oracle_state(prob, wk)
    ut[4, -1, :] = -5.0          # negative energy in one element -> negative pressure
    plan = gpu_plan(wk)
    plan.residual(ut.cuda().contiguous())
    with pytest.raises(esd.EsdError) as e:
        plan.sync_status()
    assert e.value.status == -3
    plan.sync_status()           # the flag is cleared after being reported


FULL = [
    ("vortex_tri_M64_p4", wl.vortex_tri(M=64, degree=4), 24),
    ("vortex_tri_M64_p8", wl.vortex_tri(M=64, degree=8), 12),
    ("tgv_tet_M16_p4", wl.tgv_tet(M=16, degree=4), 8),
    ("tgv_tet_M16_p6", wl.tgv_tet(M=16, degree=6), 4),
    # every single-degree kernel from p = 5 up, both interface fluxes, on a
    # small mesh: the dense oracle is O(N_q^2) per element
    ("tet_p5_random_lf_M3", wl.random_tet(M=3, degree=5, seed=21), 4),
    ("tet_p5_random_ec_M3", wl.random_tet(M=3, degree=5, seed=22, dissipation=0), 4),
    ("tet_p6_random_lf_M3", wl.random_tet(M=3, degree=6, seed=23), 3),
    ("tet_p6_tgv_ec_M3", wl.tgv_tet(M=3, degree=6), 3),
    ("tet_p7_random_lf_M3", wl.random_tet(M=3, degree=7, seed=24), 2),
    ("tet_p7_random_ec_M3", wl.random_tet(M=3, degree=7, seed=25, dissipation=0), 2),
    ("tet_p8_random_lf_M3", wl.random_tet(M=3, degree=8, seed=26), 2),
    ("tet_p8_random_ec_M3", wl.random_tet(M=3, degree=8, seed=27, dissipation=0), 2),
    ("tet_p9_random_lf_M3", wl.random_tet(M=3, degree=9, seed=8), 2),
    ("tet_p10_random_ec_M3", wl.random_tet(M=3, degree=10, seed=9, dissipation=0), 2),
    ("tri_p9_random_lf_M4", wl.random_tri(M=4, degree=9, seed=28), 6),
]


@pytest.mark.parametrize("name,wk,nsample", FULL, ids=[f[0] for f in FULL])
def test_residual_parity_full_size_sampled(name, wk, nsample):
    from oracle import residual as R
    log(f"full-size case {name}: building oracle geometry")
    prob = oracle_problem(wk)
    ut = oracle_state(prob, wk)
    plan = gpu_plan(wk)
    out = plan.residual(ut.cuda().contiguous())
    plan.sync_status()
    out = out.cpu()
    rng = np.random.default_rng(1234)
    el = np.unique(np.concatenate([[0, prob.ne - 1], rng.choice(prob.ne, nsample, replace=False)]))
    log(f"  oracle on {len(el)} sampled elements")
    ref, spread = oracle_with_spread(lambda pr: R.residual_chunked(pr, ut, el, chunk=4), prob,
                                     lambda: oracle_problem(wk))
    assert_parity(out[el], ref, what=name, spread=spread)


DIAG = [c for c in SMALL if c[0] in ("tri_p2_affine_chandrashekar_ec", "tri_p3_random_lf", "tet_p2_random_ec",
                                     "tet_p3_random_lf", "tet_p4_tgv_ec")]


@pytest.mark.parametrize("name,wk", DIAG, ids=[s[0] for s in DIAG])
def test_diagnostics_parity(name, wk):
    """esd_diagnostics against the oracle's conserved integrals, entropy
    integral and entropy rate; the rate vanishes to rounding with the
    entropy-conservative interface flux and is negative with dissipation."""
    from oracle import physics as PH
    from oracle import residual as R
    prob = oracle_problem(wk)
    ut = oracle_state(prob, wk)
    plan = gpu_plan(wk)
    d = plan.diagnostics(ut.cuda().contiguous())
    ref_c = R.conserved_integrals(prob, ut).numpy()
    u = torch.einsum("ki,eci->ekc", prob.ref.V, ut)
    wJ = prob.ref.w[None, :] * prob.geo.J
    S = PH.entropy(u, prob.gamma)
    ref_s = float((wJ * S).sum())
    dudt = R.residual_chunked(prob, ut)
    ref_r = float(R.entropy_rate(prob, ut, dudt))
    # magnitude of the rate's terms, for its rounding bound
    Wu = PH.entropy_vars(u, prob.gamma)
    du = torch.einsum("ki,eci->ekc", prob.ref.V, dudt)
    mag_r = float((wJ[..., None] * (Wu * du).abs()).sum())
    log(f"diagnostics {name}: conserved {d['conserved']}, entropy {d['entropy']:.15e}, "
        f"rate {d['entropy_rate']:.3e} (oracle {ref_r:.3e}, terms {mag_r:.3e})")
    scale_c = float((wJ[..., None] * u.abs()).sum((0, 1)).max())
    assert np.abs(d["conserved"] - ref_c).max() <= 1e-13 * scale_c
    assert abs(d["entropy"] - ref_s) <= 1e-13 * float((wJ * S.abs()).sum())
    assert abs(d["entropy_rate"] - ref_r) <= 1e-12 * mag_r
    if wk.dissipation:
        assert d["entropy_rate"] < 0
    else:
        assert abs(d["entropy_rate"]) <= 1e-12 * mag_r
