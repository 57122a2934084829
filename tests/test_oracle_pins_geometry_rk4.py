"""Further pins of the oracle against what the mathematics fixes, independent of
the oracle's own routes:

  * curved geometry against the analytic warp x~ = x + a prod_k sin(2 pi x_k/L)
    (Sec. 4.1, 4.2): the discrete mesh tiles the periodic box, so the quadrature
    of det(grad x_h) over all elements is L^d (exact for d (p-1) <= 2q: every p
    in 2D, p <= 3 in 3D); the interpolated map at the volume nodes converges to
    the warp of the affine image as p grows; the metric terms G (exact adjugate
    in 2D, the conservative curl form in 3D) converge to the adjugate of the
    analytic Jacobian of the warped map;
  * the classical four-stage RK4 on a linear ODE, where one step is the degree-4
    Taylor polynomial of the exponential;
  * the derivative of Davis' wave speed away from the near-tie window is the
    derivative of a plain max;
  * order p+1 convergence of the scheme on curved triangles (isentropic vortex
    on a coarse mesh, Sec. 7.4's convergence statement) and on curved
    tetrahedra (three-dimensional density wave)."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import geometry as geom
from oracle import physics as ph
from oracle import residual as R


def _warped(dim, M, p, L, amp=0.05):
    mesh = wl.split_box_mesh(dim, M, L)
    return R.setup(mesh, p, wl.make_warp_sinprod(L, amp), 1.4, 0, 1), mesh


def _affine_points(prob, xi):
    """affine images of reference points xi [n, d] in every element [Ne, n, d]"""
    vx = torch.tensor(prob.geo.vx)                       # oriented vertices [Ne, d+1, d]
    lam = geom._barycentric(prob.ref.dim, torch.as_tensor(xi))
    return torch.einsum("kv,evd->ekd", lam, vx)


def _warp_jacobian(x, L, amp):
    """analytic d x~ / d x of x~_i = x_i + amp prod_k sin(2 pi x_k / L)"""
    d = x.shape[-1]
    s = torch.sin(2 * math.pi * x / L)
    c = torch.cos(2 * math.pi * x / L)
    grad = []
    for k in range(d):
        g = amp * 2 * math.pi / L * c[..., k]
        for j in range(d):
            if j != k:
                g = g * s[..., j]
        grad.append(g)
    grad = torch.stack(grad, -1)                          # d(prod)/dx_k
    return torch.eye(d, dtype=x.dtype) + grad[..., None, :].expand(*x.shape, d)


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 5), (2, 8), (3, 2), (3, 3)])
def test_curved_mesh_volume_is_the_box(dim, p):
    L = 2.0 if dim == 2 else 2 * math.pi
    prob, _ = _warped(dim, 3, p, L, amp=0.08)
    vol = float(torch.einsum("k,ek->", prob.ref.w, prob.geo.J_exact))
    assert abs(vol - L ** dim) < 1e-12 * L ** dim, vol


@pytest.mark.parametrize("dim", [2, 3])
def test_curved_map_and_metrics_converge_to_the_analytic_warp(dim):
    L = 2.0 if dim == 2 else 2 * math.pi
    amp = 0.05
    errs_x, errs_G = [], []
    degrees = (2, 4, 6)
    for p in degrees:
        prob, _ = _warped(dim, 3, p, L, amp)
        xa = _affine_points(prob, prob.ref.xi)                         # [Ne, Nq, d]
        xw = torch.tensor(wl.make_warp_sinprod(L, amp)(xa.numpy()))
        errs_x.append(float((prob.geo.x_vol - xw).abs().max()))
        # adjugate of the analytic Jacobian of the warped map w.r.t. xi:
        # d x~/d xi = (d x~/d x)(d x/d xi), d x/d xi the affine part
        vx = torch.tensor(prob.geo.vx)
        A = 0.5 * (vx[:, 1:, :] - vx[:, :1, :]).transpose(1, 2)          # [Ne, c, m]
        Jw = _warp_jacobian(xa, L, amp) @ A[:, None]                     # [Ne, Nq, c, m]
        adj = torch.linalg.det(Jw)[..., None, None] * torch.linalg.inv(Jw)
        errs_G.append(float((prob.geo.G - adj).abs().max() / adj.abs().max()))
    # spectral convergence of the interpolated map and of the metric terms:
    # every degree step cuts both errors (the map by 3 at least, the metric
    # terms, one derivative lower, by 1.5), p = 2 -> 6 by 5 at least
    assert all(errs_x[i + 1] < errs_x[i] / 3 for i in range(2)), errs_x
    assert all(errs_G[i + 1] < errs_G[i] / 1.5 for i in range(2)) and errs_G[0] > 5 * errs_G[2], errs_G
    # and a transposed or sign-flipped G would sit at O(1) from the adjugate
    prob, _ = _warped(dim, 3, degrees[-1], L, amp)
    assert float((prob.geo.G.transpose(-1, -2) - prob.geo.G).abs().max()) > 1e-2 * float(prob.geo.G.abs().max())


def test_rk4_one_step_is_the_taylor_polynomial(monkeypatch):
    """u' = A u with A diagonal: one classical RK4 step multiplies each mode by
    1 + z + z^2/2 + z^3/6 + z^4/24, z = lambda dt."""
    lam = torch.tensor([-3.0, -0.5, 0.25, 1.5], dtype=torch.float64)
    monkeypatch.setattr(R, "residual_chunked", lambda prob, u, chunk=64: lam[None, None, :] * u)
    u0 = torch.ones((2, 3, 4), dtype=torch.float64)
    dt = 0.1
    u1 = R.rk4(None, u0, dt, 1)
    z = lam * dt
    expect = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    assert torch.allclose(u1, expect.expand_as(u1), rtol=0, atol=1e-15)
    u3 = R.rk4(None, u0, dt, 3)
    assert torch.allclose(u3, (expect ** 3).expand_as(u3), rtol=0, atol=1e-14)


def test_wave_speed_derivative_away_from_ties_is_that_of_max():
    """Outside the 1e-10 near-tie window the oracle's derivative of eq.
    (wave_speed) equals autograd of torch.maximum."""
    g = 1.4
    rng = np.random.default_rng(5)
    n_st = 200
    rho = rng.uniform(0.5, 1.5, (2, n_st))
    v = rng.uniform(-0.5, 0.5, (2, n_st, 3))
    p = rng.uniform(0.5, 1.5, (2, n_st))
    um = torch.tensor(wl.prim_to_cons(rho[0], v[0], p[0], g)).requires_grad_(True)
    up = torch.tensor(wl.prim_to_cons(rho[1], v[1], p[1], g)).requires_grad_(True)
    n = torch.tensor(rng.standard_normal((n_st, 3)))
    lam = ph.davis_speed(um, up, n, g)
    ga, gb = torch.autograd.grad(lam.sum(), (um, up))
    a2 = um.detach().clone().requires_grad_(True)
    b2 = up.detach().clone().requires_grad_(True)
    rm, vm, pm = ph.prim(a2, g)
    rp, vp, pp = ph.prim(b2, g)
    am, ap = (vm * n).sum(-1).abs(), (vp * n).sum(-1).abs()
    cm, cp = torch.sqrt(g * pm / rm), torch.sqrt(g * pp / rp)
    # the random states have no near-ties
    assert float(((am - ap).abs() / torch.maximum(am, ap)).min()) > 1e-8
    assert float(((cm - cp).abs() / torch.maximum(cm, cp)).min()) > 1e-8
    lam2 = torch.maximum(am, ap) + torch.maximum(cm, cp)
    gc, gd = torch.autograd.grad(lam2.sum(), (a2, b2))
    assert torch.equal(lam.detach(), lam2.detach())
    assert torch.allclose(ga, gc, rtol=1e-14, atol=1e-15) and torch.allclose(gb, gd, rtol=1e-14, atol=1e-15)


def _l2_error(prob, ut, exact):
    u = torch.einsum("ki,eci->ekc", prob.ref.V, ut)
    ex = torch.tensor(exact(prob.geo.x_vol.numpy()))
    return float(torch.einsum("k,ek,ek->", prob.ref.w, prob.geo.J, (u[..., 0] - ex[..., 0]) ** 2).sqrt())


@pytest.mark.slow
def test_vortex_convergence_curved_triangles():
    """Isentropic vortex on the warped [0,10]^2 mesh at p = 2, M = 8 -> 16,
    Lax-Friedrichs interface flux: the density error after t = 0.5 converges
    at about h^(p+1) (measured 2.68 on these coarse meshes; the vortex's
    periodicity defect, 2.4e-5 at the box edges, is far below these errors)."""
    p, T = 2, 0.5
    errs = []
    for M in (8, 16):
        mesh = wl.split_box_mesh(2, M, 10.0)
        prob = R.setup(mesh, p, wl.make_warp_sinprod(10.0, 0.05), 1.4, 0, 1)
        ut = R.project(prob, torch.tensor(wl.isentropic_vortex(prob.geo.x_vol.numpy())))
        n = 4 * M
        ut = R.rk4(prob, ut, T / n, n, chunk=512)
        errs.append(_l2_error(prob, ut, lambda x: wl.isentropic_vortex(x, t=T)))
    rate = math.log(errs[0] / errs[1], 2)
    assert rate > p + 0.5, (errs, rate)


@pytest.mark.slow
def test_density_wave_convergence_curved_tetrahedra():
    """Three-dimensional density wave (rho = 1 + 0.2 sin(2 pi (x+y+z)/L), v = 1,
    p = 1) on warped tetrahedra of [0,2]^3 at p = 1, M = 3 -> 6, Lax-Friedrichs:
    the density error after t = 0.02 falls faster than h^(p+1/2) (measured
    1.57 on these coarse meshes, where the wave spans under four elements)."""
    p, T, L = 1, 0.02, 2.0
    errs = []
    for M in (3, 6):
        mesh = wl.split_box_mesh(3, M, L)
        prob = R.setup(mesh, p, wl.make_warp_sinprod(L, 0.05), 1.4, 0, 1)
        ut = R.project(prob, torch.tensor(wl.density_wave(prob.geo.x_vol.numpy(), L)))
        n = max(1, M // 2)
        ut = R.rk4(prob, ut, T / n, n, chunk=512)
        errs.append(_l2_error(prob, ut, lambda x: wl.density_wave(np.asarray(x) - T, L)))
    rate = math.log(errs[0] / errs[1], 2)
    assert rate > p + 0.5, (errs, rate)
