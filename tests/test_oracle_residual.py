"""Pins for the oracle's geometry and residual (Sec. 4, 6, 7).

Conformity of the mesh (Assumption conformal), metric terms (adjugate on affine
elements, discrete metric identities), and the analysis theorems of Sec. 6:
equivalence with the hybridized formulation, conservation, free-stream
preservation, entropy conservation / stability; plus a brute-force check that
the line-by-line pair loop (each unordered pair of a collapsed-coordinate line
once, summed direction) equals the dense Hadamard-product volume term, the
affine special case of the weight-adjusted inverse, and the p+1 convergence
rate on the density wave of Sec. 7.4."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import physics as ph
from oracle import residual as R
from oracle.geometry import equispaced

CASES = [
    # dim, M, p, warp amplitude, ecflux, dissipation
    (2, 3, 2, 0.05, 0, 1),
    (2, 3, 4, 0.05, 1, 0),
    (3, 3, 2, 0.05, 0, 0),
    (3, 3, 3, 0.08, 0, 1),
]


def _prob(dim, M, p, amp, ecflux, diss, L=None):
    L = L or (2.0 if dim == 2 else 2 * math.pi)
    mesh = wl.split_box_mesh(dim, M, L)
    warp = wl.make_warp_sinprod(L, amp) if amp else wl.warp_none
    return R.setup(mesh, p, warp, 1.4, ecflux, diss), L


_cache = {}


def prob_for(case):
    if case not in _cache:
        _cache[case] = _prob(*case)
    return _cache[case]


def smooth_state(prob, L, seed=3):
    st = wl.RandomSmooth(prob.ref.dim, L, seed)
    return R.project(prob, torch.tensor(st(prob.geo.x_vol.numpy())))


@pytest.mark.parametrize("case", CASES)
def test_conforming_facets(case):
    prob, L = prob_for(case)
    geo, con = prob.geo, prob.con
    for z in range(prob.ref.Nf):
        nb, nz = con.nbr_elem[:, z], con.nbr_face[:, z]
        for e in range(prob.ne):
            m = con.node_map[e, z]
            dx = (geo.x_f[z][e] - geo.x_f[nz[e]][nb[e]][m]).numpy()
            dx -= L * np.round(dx / L)
            assert np.abs(dx).max() < 1e-12
            assert float((geo.n[z][e] + geo.n[nz[e]][nb[e]][m]).abs().max()) < 1e-12
            wa = prob.ref.w_f[z] * geo.Jf[z][e]
            wb = prob.ref.w_f[nz[e]][m] * geo.Jf[nz[e]][nb[e]][m]
            assert float((wa - wb).abs().max()) < 1e-12
    assert float(prob.geo.J.min()) > 0


@pytest.mark.parametrize("dim", [2, 3])
def test_affine_metrics_are_adjugate(dim):
    prob, L = _prob(dim, 3, 3, 0.0, 0, 1)
    for e in range(0, prob.ne, 7):
        X = torch.tensor(prob.geo.vx[e])
        A = 0.5 * (X[1:] - X[0]).T                     # d x / d xi
        adj = torch.linalg.det(A) * torch.linalg.inv(A)
        np.testing.assert_allclose(prob.geo.G[e].numpy(), adj.expand_as(prob.geo.G[e]).numpy(), atol=1e-12)
        np.testing.assert_allclose(prob.geo.J[e].numpy(), float(torch.linalg.det(A)), rtol=1e-12)
    vol = float(torch.einsum("k,ek->", prob.ref.w, prob.geo.J))
    assert abs(vol - L ** dim) < 1e-11 * L ** dim


@pytest.mark.parametrize("case", CASES)
def test_discrete_metric_identities(case):
    """sum_l D^l G_lm = 0 at volume nodes (metric identities, eq. metric_identities,
    with G in P_q and D exact on P_q)."""
    prob, _ = prob_for(case)
    G = prob.geo.G
    for m in range(prob.ref.dim):
        div = sum(torch.einsum("ij,ej->ei", prob.ref.D[l], G[:, :, l, m]) for l in range(prob.ref.dim))
        scale = float(G.abs().max()) * max(float(Dl.abs().sum(1).max()) for Dl in prob.ref.D)
        assert float(div.abs().max()) < 1e-13 * scale


@pytest.mark.parametrize("case", CASES)
def test_hybridized_equivalence(case):
    """Theorem (equivalence): eq. (entropy_stable) + eq. (dudt_modal) equals eq. (skew_hybridized)."""
    prob, L = prob_for(case)
    ut = smooth_state(prob, L)
    el = np.arange(0, prob.ne, max(1, prob.ne // 6))
    a = R.residual(prob, ut, el)
    b = R.residual_hybridized(prob, ut, el)
    assert float((a - b).abs().max()) < 1e-12 * float(a.abs().max())


@pytest.mark.parametrize("case", CASES)
def test_conservation_free_stream_entropy(case):
    prob, L = prob_for(case)
    d = prob.ref.dim
    ut = smooth_state(prob, L)
    du = R.residual_chunked(prob, ut)
    scale = float(du.abs().max())
    # Theorem (conservation), periodic: d/dt sum 1^T W J u = 0
    V = prob.ref.V
    rate = torch.einsum("k,ek,ekc->c", prob.ref.w, prob.geo.J, torch.einsum("ki,eci->ekc", V, du))
    assert float(rate.abs().max()) < 1e-12 * scale * prob.ne
    # Theorem (entropy stability): rate 0 for EC interface flux, <= 0 with LF
    er = float(R.entropy_rate(prob, ut, du))
    if prob.dissipation:
        assert er < 0
    else:
        assert abs(er) < 1e-12 * scale * prob.ne
    # Theorem (free stream)
    u0 = torch.tensor(wl.prim_to_cons(np.array(1.1), np.array([0.4, -0.3, 0.2][:d]), np.array(0.8)))
    uf = R.project(prob, u0.expand(prob.ne, prob.ref.Nq, d + 2))
    assert float(R.residual_chunked(prob, uf).abs().max()) < 1e-12


@pytest.mark.parametrize("case", CASES[:3])
def test_line_pair_loop_equals_dense_volume_term(case):
    """Brute force: summing each unordered pair (a<b) with S^l_ab != 0 once, with
    the summed direction n_ab = sum_l S^l_ab (g_l(a) + g_l(b)) and r_a -= F,
    r_b += F, reproduces the dense volume term of eq. (entropy_stable)."""
    prob, L = prob_for(case)
    ref = prob.ref
    d = ref.dim
    ut = smooth_state(prob, L)
    e = 1
    wt = R.entropy_projection(prob, ut, torch.tensor([e]))[0]
    ub = ph.cons_from_entropy((ref.V @ wt.T), prob.gamma)      # [Nq, Nc]
    G = prob.geo.G[e]
    # dense
    dense = torch.zeros_like(ub)
    for l in range(d):
        for i in range(ref.Nq):
            for j in range(ref.Nq):
                n = G[i, l] + G[j, l]
                dense[i] -= ref.S[l][i, j] * ph.EC_FLUXES[prob.ecflux](ub[i], ub[j], n, prob.gamma)
    # line-based
    line = torch.zeros_like(ub)
    npairs = 0
    for a in range(ref.Nq):
        for b in range(a + 1, ref.Nq):
            coeff = [float(ref.S[l][a, b]) for l in range(d)]
            if all(abs(c) < 1e-13 for c in coeff):
                continue
            npairs += 1
            n = sum(coeff[l] * (G[a, l] + G[b, l]) for l in range(d))
            F = ph.EC_FLUXES[prob.ecflux](ub[a], ub[b], n, prob.gamma)
            line[a] -= F
            line[b] += F
    Q = prob.ref.q + 1
    expected_pairs = Q ** (d - 1) * Q * (Q - 1) // 2 * d
    assert npairs == expected_pairs
    assert float((dense - line).abs().max()) < 1e-12 * float(dense.abs().max())


@pytest.mark.parametrize("dim", [2, 3])
def test_weight_adjusted_inverse_affine_is_exact(dim):
    prob, L = _prob(dim, 3, 3, 0.0, 0, 1)
    A = R.wadj_inverse(prob, torch.arange(4))
    V, w = prob.ref.V, prob.ref.w
    for k in range(4):
        Mk = V.T @ torch.diag(w * prob.geo.J[k]) @ V
        np.testing.assert_allclose((A[k] @ Mk).numpy(), np.eye(prob.ref.Np), atol=1e-12)


@pytest.mark.slow
@pytest.mark.parametrize("p", [2, 3])
def test_density_wave_convergence_order(p):
    """Sec. 7.4: with interface dissipation the density error converges at O(h^{p+1})."""
    errs = []
    T, L = 0.25, 2.0
    for M in (4, 8):
        mesh = wl.split_box_mesh(2, M, L)
        prob = R.setup(mesh, p, wl.warp_none, 1.4, 0, 1)
        u0 = torch.tensor(wl.density_wave(prob.geo.x_vol.numpy(), L))
        ut = R.project(prob, u0)
        dt = 0.0125 / M
        n = int(round(T / dt))
        ut = R.rk4(prob, ut, dt, n, chunk=256)
        u = torch.einsum("ki,eci->ekc", prob.ref.V, ut)
        x = prob.geo.x_vol.numpy() - T
        ex = torch.tensor(wl.density_wave(x, L))
        err = torch.einsum("k,ek,ek->", prob.ref.w, prob.geo.J, (u[..., 0] - ex[..., 0]) ** 2).sqrt()
        errs.append(float(err))
    rate = math.log(errs[0] / errs[1], 2)
    assert rate > p + 1 - 0.35, (errs, rate)
