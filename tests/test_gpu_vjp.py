"""GPU parity of the hand-written adjoint (esd_residual_vjp, esd_rk4_vjp).

The oracle's vector-Jacobian product is reverse-mode autodiff of its dense
residual (pinned by finite differences and the dot-product identity in
test_oracle_vjp).  Small meshes are compared in full with the same seeded
state and cotangent; benchmark-size meshes on sampled elements (the oracle
differentiates their 1-ring); the library's own VJP is also checked against
central differences of its own residual at full size and at tet p = 6-8
(entropy-conservative flux, where the residual is smooth), and the discrete RK4
adjoint against the oracle's autograd through its RK4 and against central
differences of a kinetic-energy objective after 20 steps on 10,368 curved
tetrahedra at p = 6."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from tests.parity_util import gpu_plan, log, oracle_problem, oracle_state

pytestmark = pytest.mark.gpu

TOL = 1e-12

SMALL = [
    ("tri_p2_affine_chandrashekar_ec", wl.density_wave_tri(M=3, degree=2, ecflux=1, dissipation=0)),
    ("tri_p1_random_lf", wl.random_tri(M=3, degree=1, seed=1)),
    ("tri_p3_random_lf", wl.random_tri(M=3, degree=3, seed=2)),
    ("tri_p5_random_ec", wl.random_tri(M=3, degree=5, seed=3, dissipation=0)),
    ("tet_p1_random_lf", wl.random_tet(M=3, degree=1, seed=5)),
    ("tet_p2_random_ec", wl.random_tet(M=3, degree=2, seed=6, dissipation=0)),
    ("tet_p3_random_lf", wl.random_tet(M=3, degree=3, seed=7)),
    ("tet_p2_chandrashekar_lf", wl.Workload("random_tet_chandrashekar", 3, 3, 2 * math.pi, 2,
                                           wl.make_warp_sinprod(2 * math.pi, 0.05),
                                           wl.RandomSmooth(3, 2 * math.pi, 12), 1, 1)),
]


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def cotangent(shape, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.randn(shape, generator=g, dtype=torch.float64)


def assert_close(gpu, ora, what, tol=TOL):
    """Per conserved variable: max |gpu - oracle| <= tol ||oracle_e||_inf."""
    gpu = gpu.detach().cpu().double()
    ora = ora.detach().cpu().double()
    ratios = []
    for c in range(ora.shape[1]):
        err = float((gpu[:, c] - ora[:, c]).abs().max())
        scale = float(ora[:, c].abs().max())
        ratios.append(err / scale)
    log(f"vjp parity {what}: max err / ||g_e||_inf per var {['%.2e' % r for r in ratios]}")
    assert max(ratios) <= tol, f"{what}: {ratios}"


def oracle_vjp_pair(prob, ut, vbar, elems=None):
    """The oracle's VJP (mean of the one-sided derivatives at near-ties of the
    wave speed, the library's convention) and, with dissipation, the spread
    between the two one-sided choices, reported for information."""
    from oracle import physics as PH
    from oracle import residual as R
    ref = R.vjp(prob, ut, vbar, elems)
    if prob.dissipation:
        with PH.tie_derivative("-"):
            a = R.vjp(prob, ut, vbar, elems)
        with PH.tie_derivative("+"):
            b = R.vjp(prob, ut, vbar, elems)
        log(f"one-sided tie spread: max |g- - g+| = {float((a - b).abs().max()):.2e}")
    return ref


@pytest.mark.parametrize("name,wk", SMALL, ids=[s[0] for s in SMALL])
def test_vjp_parity_small(name, wk):
    from oracle import residual as R
    log(f"case {name}: dim={wk.dim} M={wk.M} p={wk.degree}")
    prob = oracle_problem(wk)
    ut = oracle_state(prob, wk)
    vbar = cotangent(ut.shape, 17)
    ref = oracle_vjp_pair(prob, ut, vbar)
    plan = gpu_plan(wk)
    out = plan.vjp(ut.cuda().contiguous(), vbar.cuda().contiguous())
    plan.sync_status()
    torch.cuda.synchronize()
    assert_close(out, ref, name)


def test_vjp_parity_high_degree_sampled():
    """Tet p = 5 and tri p = 8 on small meshes, 8 sampled elements each (the
    oracle differentiates their 1-ring densely)."""
    from oracle import residual as R
    for wk in (wl.random_tet(M=3, degree=5, seed=13), wl.random_tri(M=3, degree=8, seed=14)):
        prob = oracle_problem(wk)
        ut = oracle_state(prob, wk)
        vbar = cotangent(ut.shape, 29)
        plan = gpu_plan(wk)
        out = plan.vjp(ut.cuda().contiguous(), vbar.cuda().contiguous()).cpu()
        plan.sync_status()
        el = np.random.default_rng(5).choice(prob.ne, 8, replace=False)
        ref = oracle_vjp_pair(prob, ut, vbar, el)
        assert_close(out[el], ref, wk.name)


FULL = [("vortex_tri_M64_p4", lambda: wl.vortex_tri(M=64, degree=4)),
        ("tgv_tet_M16_p4", lambda: wl.tgv_tet(M=16, degree=4))]


@pytest.mark.parametrize("name,make", FULL, ids=[f[0] for f in FULL])
def test_vjp_parity_full_sampled(name, make):
    """Benchmark-size meshes in the benchmark's launch configuration; the
    oracle differentiates the 1-ring of 24 sampled elements."""
    from oracle import residual as R
    wk = make()
    log(f"case {name}: full size, sampled")
    plan = gpu_plan(wk)
    x = plan.node_coords().cpu().numpy()
    un = torch.tensor(wk.state(x), device="cuda").contiguous()
    u = plan.project(un)
    vbar = cotangent(tuple(u.shape), 23).cuda()
    out = plan.vjp(u, vbar).cpu()
    plan.sync_status()
    prob = oracle_problem(wk)
    el = np.random.default_rng(3).choice(prob.ne, 24, replace=False)
    ref = oracle_vjp_pair(prob, u.cpu(), vbar.cpu(), el)
    assert_close(out[el], ref, name)


def test_vjp_matches_central_differences_full_size():
    """<vbar, R(u + h d) - R(u - h d)>/(2h) = <VJP(vbar), d> on 10,368 curved
    tetrahedra at p = 6, library only (no oracle)."""
    wk = wl.tgv_tet(M=12, degree=6)
    plan = gpu_plan(wk)
    x = plan.node_coords().cpu().numpy()
    u = plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
    vbar = cotangent(tuple(u.shape), 31).cuda()
    g = plan.vjp(u, vbar)
    h = 1e-6
    for k in range(4):
        d = cotangent(tuple(u.shape), 100 + k).cuda()
        fp = (plan.residual((u + h * d).contiguous()) * vbar).sum()
        fm = (plan.residual((u - h * d).contiguous()) * vbar).sum()
        fd = float((fp - fm) / (2 * h))
        ad = float((g * d).sum())
        log(f"direction {k}: fd {fd:.12e} adjoint {ad:.12e} rel {abs(fd - ad) / abs(ad):.2e}")
        assert abs(fd - ad) <= 1e-6 * abs(ad)
    plan.sync_status()


@pytest.mark.parametrize("p", [6, 7, 8, 9, 10])
def test_vjp_matches_central_differences_high_degree(p):
    """The same identity on a small curved tetrahedral mesh at p = 6-10 (the
    adjoint kernels' LDS-table and composed-transform variants there, and at
    p = 9, 10 their per-element slices of the global workspace), library
    only.  The interface flux is the entropy-conservative one: with the Davis
    wave speed (a maximum of two states that nearly agree on a smooth field)
    the residual has kinks, and central differences there stall near 1e-5
    relative at any h, while the smooth residual converges as h^2 (about 1e-9
    relative at h = 1e-6).  The dissipative branch is checked against the
    oracle below."""
    wk = wl.random_tet(M=3, degree=p, seed=40 + p, dissipation=0)
    plan = gpu_plan(wk)
    x = plan.node_coords().cpu().numpy()
    u = plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
    vbar = cotangent(tuple(u.shape), 41).cuda()
    g = plan.vjp(u, vbar)
    h = 1e-6
    for k in range(3):
        d = cotangent(tuple(u.shape), 200 + k).cuda()
        fp = (plan.residual((u + h * d).contiguous()) * vbar).sum()
        fm = (plan.residual((u - h * d).contiguous()) * vbar).sum()
        fd = float((fp - fm) / (2 * h))
        ad = float((g * d).sum())
        log(f"p {p} direction {k}: fd {fd:.12e} adjoint {ad:.12e} rel {abs(fd - ad) / abs(ad):.2e}")
        assert abs(fd - ad) <= 1e-6 * abs(ad)
    plan.sync_status()


def test_vjp_parity_tet_p7_lax_friedrichs_sampled():
    """Tet p = 7 with the Davis dissipation against the oracle on 4 sampled
    elements (above the degrees the full-mesh comparisons reach)."""
    wk = wl.random_tet(M=3, degree=7, seed=13)
    prob = oracle_problem(wk)
    ut = oracle_state(prob, wk)
    vbar = cotangent(ut.shape, 29)
    plan = gpu_plan(wk)
    out = plan.vjp(ut.cuda().contiguous(), vbar.cuda().contiguous()).cpu()
    plan.sync_status()
    el = np.random.default_rng(5).choice(prob.ne, 4, replace=False)
    ref = oracle_vjp_pair(prob, ut, vbar, el)
    assert_close(out[el], ref, wk.name)


@pytest.mark.parametrize("p", [9, 10])
def test_vjp_parity_tet_top_degrees_sampled(p):
    """Tet p = 9 and 10 with the Davis dissipation against the oracle on 2
    sampled elements: the adjoint kernels keep part of their per-element
    arrays in a global workspace slice at these degrees."""
    wk = wl.random_tet(M=3, degree=p, seed=50 + p)
    log(f"case tet p{p}: M=3, dissipation {wk.dissipation}")
    prob = oracle_problem(wk)
    ut = oracle_state(prob, wk)
    vbar = cotangent(ut.shape, 37)
    plan = gpu_plan(wk)
    out = plan.vjp(ut.cuda().contiguous(), vbar.cuda().contiguous()).cpu()
    plan.sync_status()
    el = np.random.default_rng(7).choice(prob.ne, 2, replace=False)
    ref = oracle_vjp_pair(prob, ut, vbar, el)
    assert_close(out[el], ref, wk.name)


def test_residual_autograd_function():
    import paper_2312_07874_amd as esd
    from oracle import residual as R
    wk = wl.random_tri(M=3, degree=3, seed=2)
    prob = oracle_problem(wk)
    ut = oracle_state(prob, wk)
    vbar = cotangent(ut.shape, 5)
    plan = gpu_plan(wk)
    x = ut.cuda().contiguous().requires_grad_(True)
    (esd.residual(x, plan) * vbar.cuda()).sum().backward()
    assert_close(x.grad, R.vjp(prob, ut, vbar), "autograd residual")


def test_rk4_adjoint_matches_oracle_autograd():
    """Discrete adjoint of 3 RK4 steps against reverse-mode autodiff through the
    oracle's RK4."""
    from oracle import residual as R
    wk = wl.random_tri(M=3, degree=3, seed=2)
    prob = oracle_problem(wk)
    ut = oracle_state(prob, wk)
    dt, n = 2e-3, 3
    ubar = cotangent(ut.shape, 9)
    x = ut.detach().clone().requires_grad_(True)
    uT = R.rk4(prob, x, dt, n)
    (ref,) = torch.autograd.grad((uT * ubar).sum(), x)
    plan = gpu_plan(wk)
    u = ut.cuda().contiguous()
    ckpt = torch.empty((4 * n,) + tuple(u.shape), dtype=torch.float64, device="cuda")
    uT_gpu = plan.rk4(u.clone(), dt, n, ckpt)
    g = plan.rk4_vjp(ckpt, dt, n, ubar.cuda().contiguous())
    plan.sync_status()
    assert_close(uT_gpu, uT.detach(), "rk4 forward")
    assert_close(g, ref, "rk4 adjoint")


def _kinetic_energy_fn(plan, degree):
    """KE(u~) = sum_e sum_k w_k J_k |rho v|^2 / (2 rho) at the volume nodes."""
    from oracle import refelem
    ref = refelem.ref_element(3, degree)
    V = ref.V.cuda()
    wJ = (ref.w[None, :] * torch.tensor(plan.host_array("J"))).cuda()

    def ke(u):
        un = torch.einsum("ki,eci->eck", V, u)
        return 0.5 * (wJ * (un[:, 1:4] ** 2).sum(1) / un[:, 0]).sum()

    return ke


def test_rk4_adjoint_kinetic_energy_central_differences():
    """d KE(u(T)) / d u(0) after 20 RK4 steps on 10,368 curved tetrahedra at
    p = 6 (Taylor-Green vortex, entropy-conservative): the discrete adjoint
    against central differences along 32 random directions, h = 1e-6, each
    direction at 1e-6 relative to its own directional derivative, or to the
    root mean square over the directions where that is larger (a direction
    whose derivative nearly vanishes is judged against the typical size, as
    the difference quotient's rounding does not shrink with it); dt = 5e-4."""
    import paper_2312_07874_amd as esd
    wk = wl.tgv_tet(M=12, degree=6)
    plan = gpu_plan(wk)
    x = plan.node_coords().cpu().numpy()
    u0 = plan.project(torch.tensor(wk.state(x), device="cuda").contiguous())
    ke = _kinetic_energy_fn(plan, 6)
    dt, n = 5e-4, 20
    x0 = u0.clone().requires_grad_(True)
    J = ke(esd.rk4(x0, plan, dt, n))
    (grad,) = torch.autograd.grad(J, x0)
    plan.sync_status()
    h = 1e-6
    fds, ads = [], []
    for k in range(32):
        d = cotangent(tuple(u0.shape), 1000 + k).cuda()
        d /= d.abs().max()
        up = plan.rk4((u0 + h * d).contiguous(), dt, n)
        um = plan.rk4((u0 - h * d).contiguous(), dt, n)
        fds.append(float((ke(up) - ke(um)) / (2 * h)))
        ads.append(float((grad * d).sum()))
        log(f"direction {k}: fd {fds[-1]:.12e} adjoint {ads[-1]:.12e}")
    plan.sync_status()
    fd, ad = np.array(fds), np.array(ads)
    per = np.abs(fd - ad) / np.maximum(np.abs(ad), np.sqrt(np.mean(ad ** 2)))
    rel = float(np.linalg.norm(fd - ad) / np.linalg.norm(ad))
    log(f"32 directions: per-direction |fd - adjoint| / |adjoint| max {per.max():.2e} median {np.median(per):.2e}; "
        f"||fd - adjoint|| / ||adjoint|| = {rel:.2e}")
    assert per.max() <= 1e-6, per
