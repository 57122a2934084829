"""Pins for the oracle's reference-element operators (Sec. 2.2-3.2, 4.3, 5.1, 5.3).

SBP property, accuracy of D and R, quadrature exactness against closed-form
simplex integrals, orthonormality of the PKD basis under an independent (scipy)
quadrature, and the flux-evaluation counts against the ratios printed in the
paper (tests/golden/flux_count_ratios.txt)."""
import math
import os
from itertools import product

import numpy as np
import pytest
import scipy.special as sp
import torch

from oracle.refelem import num_flux_evals, pkd, pkd_grad, ref_element

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "flux_count_ratios.txt")


def simplex_monomial_integral(dim, powers):
    """Exact integral of prod (1+xi_k)^{a_k} over the reference simplex
    {xi >= -1, sum xi <= 2-dim... } via the Dirichlet formula: with
    lambda_k = (1+xi_k)/2 the simplex is the unit simplex scaled by 2."""
    a = list(powers)
    num = np.prod([math.factorial(k) for k in a])
    den = math.factorial(sum(a) + dim)
    return 2 ** (dim + sum(a)) * num / den


@pytest.mark.parametrize("dim,q", [(2, 1), (2, 2), (2, 4), (2, 7), (3, 1), (3, 2), (3, 4)])
def test_volume_quadrature_exact_degree_2q(dim, q):
    r = ref_element(dim, q)
    x1 = 1 + r.xi
    for pw in product(range(2 * q + 1), repeat=dim):
        if sum(pw) > 2 * q:
            continue
        f = torch.ones(r.Nq, dtype=torch.float64)
        for k in range(dim):
            f = f * x1[:, k] ** pw[k]
        exact = simplex_monomial_integral(dim, pw)
        assert abs(float((r.w * f).sum()) - exact) < 1e-12 * max(1, exact)


@pytest.mark.parametrize("dim,q", [(2, 2), (2, 5), (3, 2), (3, 4)])
def test_facet_weights_sum_to_facet_measure(dim, q):
    r = ref_element(dim, q)
    meas = [2.0, 2.0 * math.sqrt(2.0), 2.0] if dim == 2 else [2.0, 2.0 * math.sqrt(3.0), 2.0, 2.0]
    for z in range(r.Nf):
        assert abs(float(r.w_f[z].sum()) - meas[z]) < 1e-13


@pytest.mark.parametrize("dim,q", [(2, 1), (2, 3), (2, 6), (3, 1), (3, 3), (3, 5)])
def test_sbp_property_and_accuracy(dim, q):
    """Definition (sbp): Q + Q^T = E, D exact on P_q, R exact on P_q (eq. extrap_acc)."""
    r = ref_element(dim, q)
    for m in range(dim):
        assert float((r.Q[m] + r.Q[m].T - r.E[m]).abs().max()) < 1e-13
        assert float((r.S[m] + r.S[m].T).abs().max()) < 1e-13
    x = r.xi
    for pw in product(range(q + 1), repeat=dim):
        if sum(pw) > q:
            continue
        f = torch.ones(r.Nq, dtype=torch.float64)
        for k in range(dim):
            f = f * x[:, k] ** pw[k]
        for m in range(dim):
            g = torch.ones(r.Nq, dtype=torch.float64) * pw[m]
            for k in range(dim):
                e = pw[k] - (1 if k == m else 0)
                g = g * (x[:, k] ** e if e >= 0 else 0.0)
            assert float((r.D[m] @ f - g).abs().max()) < 1e-10
        for z in range(r.Nf):
            xf = r.xi_f[z]
            ff = torch.ones(xf.shape[0], dtype=torch.float64)
            for k in range(dim):
                ff = ff * xf[:, k] ** pw[k]
            assert float((r.R[z] @ f - ff).abs().max()) < 1e-12


@pytest.mark.parametrize("dim,q", [(2, 3), (3, 3)])
def test_e_integrates_boundary_products(dim, q):
    """eq. (facet_accuracy): u^T E^m v = boundary integral of u v n_m, for u, v in P_q;
    checked with u = 1 (E^m 1 sums to zero: the boundary normal integrates to zero)
    and with u = xi_m, v = 1 (equals the volume of the reference element)."""
    r = ref_element(dim, q)
    one = torch.ones(r.Nq, dtype=torch.float64)
    vol = 2.0 if dim == 2 else 4.0 / 3.0
    for m in range(dim):
        assert abs(float(one @ r.E[m] @ one)) < 1e-13
        assert abs(float(r.xi[:, m] @ r.E[m] @ one) - vol) < 1e-13


def _scipy_collapsed_rule(dim, n):
    """Independent conical-product rule from scipy's Gauss-Jacobi roots."""
    x0, w0 = sp.roots_jacobi(n, 0, 0)
    x1, w1 = sp.roots_jacobi(n, 1, 0)
    if dim == 2:
        pts, wts = [], []
        for i in range(n):
            for j in range(n):
                a, b = x0[i], x1[j]
                pts.append(((1 + a) * (1 - b) / 2 - 1, b))
                wts.append(w0[i] * w1[j] / 2)
        return torch.tensor(pts), torch.tensor(wts)
    x2, w2 = sp.roots_jacobi(n, 2, 0)
    pts, wts = [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                a, b, c = x0[i], x1[j], x2[k]
                pts.append(((1 + a) * (1 - b) * (1 - c) / 4 - 1, (1 + b) * (1 - c) / 2 - 1, c))
                wts.append(w0[i] * w1[j] * w2[k] / 8)
    return torch.tensor(pts), torch.tensor(wts)


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 4), (2, 8), (3, 1), (3, 3), (3, 6)])
def test_pkd_orthonormal_under_independent_rule(dim, p):
    X, wq = _scipy_collapsed_rule(dim, p + 2)
    Phi = pkd(dim, p, X)
    M = Phi.T @ torch.diag(wq) @ Phi
    np.testing.assert_allclose(M.numpy(), np.eye(M.shape[0]), atol=1e-12)


@pytest.mark.parametrize("dim,q", [(2, 2), (2, 5), (3, 2), (3, 5)])
def test_mass_matrix_identity(dim, q):
    """V^T W V = I for tau >= 2p (Sec. 4.3)."""
    r = ref_element(dim, q)
    M = r.V.T @ torch.diag(r.w) @ r.V
    np.testing.assert_allclose(M.numpy(), np.eye(r.Np), atol=1e-13)


def test_pkd_constant_mode_is_inverse_sqrt_volume():
    X = torch.tensor([[-0.3, -0.2]], dtype=torch.float64)
    assert abs(float(pkd(2, 0, X)[0, 0]) - 1 / math.sqrt(2.0)) < 1e-15
    X = torch.tensor([[-0.3, -0.2, -0.4]], dtype=torch.float64)
    assert abs(float(pkd(3, 0, X)[0, 0]) - math.sqrt(3.0 / 4.0)) < 1e-15


@pytest.mark.parametrize("dim,p", [(2, 5), (3, 4)])
def test_pkd_gradient(dim, p):
    """Finite differences at interior points; exact derivatives of interpolated
    monomials at the collapsed vertices (where the chain rule is singular)."""
    rng = np.random.default_rng(0)
    lam = rng.dirichlet(np.ones(dim + 1), size=9)
    verts = np.array([[-1, -1], [1, -1], [-1, 1]]) if dim == 2 else \
        np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]])
    X = torch.tensor(lam @ verts, dtype=torch.float64)
    G = pkd_grad(dim, p, X)
    h = 1e-6
    for m in range(dim):
        e = torch.zeros(dim, dtype=torch.float64)
        e[m] = h
        fd = (pkd(dim, p, X + e) - pkd(dim, p, X - e)) / (2 * h)
        np.testing.assert_allclose(G[m].numpy(), fd.numpy(), atol=2e-7)
    # vertices: gradient of p-th power monomials through the basis expansion
    V = torch.tensor(verts, dtype=torch.float64)
    Xq, wq = _scipy_collapsed_rule(dim, p + 2)
    Phi = pkd(dim, p, Xq)
    for pw in product(range(p + 1), repeat=dim):
        if sum(pw) > p:
            continue
        f = torch.ones(Xq.shape[0], dtype=torch.float64)
        for k in range(dim):
            f = f * Xq[:, k] ** pw[k]
        coef = Phi.T @ (wq * f)                       # exact L2 projection (orthonormal)
        Gv = pkd_grad(dim, p, V)
        for m in range(dim):
            g = torch.ones(V.shape[0], dtype=torch.float64) * pw[m]
            for k in range(dim):
                ex = pw[k] - (1 if k == m else 0)
                g = g * (V[:, k] ** ex if ex >= 0 else 0.0)
            assert float((Gv[m] @ coef - g).abs().max()) < 1e-11


@pytest.mark.parametrize("q", [1, 2, 3, 4, 6])
def test_flux_counts_closed_forms(q):
    """Structural count of eq. (num_fluxes): tri 1.5(q+1)^2(q+2), tet 4(q+1)^4."""
    assert num_flux_evals(ref_element(2, q)) == int(1.5 * (q + 1) ** 2 * (q + 2))
    if q <= 4:
        assert num_flux_evals(ref_element(3, q)) == 4 * (q + 1) ** 4


def _read_golden():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                s, q, r = line.split()
                rows.append((s, int(q), float(r)))
    return rows


def test_printed_flux_reduction_ratios():
    """The six printed reduction factors are reproduced by the oracle's counts:
    for each triangle case a unique symmetric-rule size N matches the printed
    ratio; each tetrahedron case then matches with its facets integrated by the
    triangle rule of the same q (the paper's construction), again uniquely."""
    rows = _read_golden()
    tri_N = {}
    for shape, q, ratio in rows:
        if shape != "tri":
            continue
        n_t = num_flux_evals(ref_element(2, q))
        hits = [N for N in range(1, 3000)
                if round((N * (N - 1) + 3 * N * (q + 1)) / n_t, 2) == ratio]
        assert len(hits) == 1, (q, hits)
        tri_N[q] = hits[0]
    for shape, q, ratio in rows:
        if shape != "tet":
            continue
        n_t = 4 * (q + 1) ** 4 if q > 5 else num_flux_evals(ref_element(3, q))
        Nf = tri_N[q]
        hits = [N for N in range(1, 5000)
                if round((3 * N * (N - 1) // 2 + 4 * N * Nf) / n_t, 2) == ratio]
        assert len(hits) == 1, (q, hits)


@pytest.mark.slow
def test_flux_count_tet_q10_from_operators():
    assert num_flux_evals(ref_element(3, 10)) == 4 * 11 ** 4
