"""Pins for the oracle's 1D building blocks (Sec. 2.4) against scipy and closed forms."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.special as sp
import torch

from oracle.poly1d import gauss_jacobi, jacobi, jacobi_deriv, lagrange, lagrange_deriv


def _norm_const(n, a, b):
    # squared L2 norm of the classical (scipy) Jacobi polynomial P_n^{(a,b)}
    return (2 ** (a + b + 1) / (2 * n + a + b + 1) * math.gamma(n + a + 1) * math.gamma(n + b + 1)
            / (math.gamma(n + a + b + 1) * math.factorial(n)))


@pytest.mark.parametrize("a,b", [(0, 0), (1, 0), (3, 0), (7, 0), (2, 0)])
def test_jacobi_matches_scipy_normalized(a, b):
    x = np.linspace(-1, 1, 37)
    P = jacobi(9, a, b, x).numpy()
    for n in range(10):
        ref = sp.eval_jacobi(n, a, b, x) / math.sqrt(_norm_const(n, a, b))
        np.testing.assert_allclose(P[n], ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("a,b", [(0, 0), (1, 0), (5, 0)])
def test_jacobi_derivative_finite_difference(a, b):
    x = np.linspace(-0.9, 0.9, 11)
    h = 1e-6
    dP = jacobi_deriv(8, a, b, x).numpy()
    fd = (jacobi(8, a, b, x + h).numpy() - jacobi(8, a, b, x - h).numpy()) / (2 * h)
    np.testing.assert_allclose(dP, fd, rtol=1e-7, atol=1e-6)


@pytest.mark.parametrize("q", [0, 1, 2, 5, 10, 15])
@pytest.mark.parametrize("a", [0, 1])
def test_gauss_jacobi_matches_scipy(q, a):
    x, w = gauss_jacobi(q, a, 0)
    xs, ws = sp.roots_jacobi(q + 1, a, 0)
    np.testing.assert_allclose(x.numpy(), xs, atol=1e-14)
    np.testing.assert_allclose(w.numpy(), ws, rtol=1e-12)


@pytest.mark.parametrize("q", [1, 3, 6, 10])
@pytest.mark.parametrize("a", [0, 1])
def test_gauss_exactness_degree_2q_plus_1(q, a):
    """eq. (quad_1d): exact for degree 2q+1 against the Beta-function integral."""
    x, w = gauss_jacobi(q, a, 0)
    for k in range(2 * q + 2):
        # int (1-x)^a x^k dx over [-1,1] in exact rational arithmetic
        exact = float(sum(Fraction(math.comb(a, i) * (-1) ** i) * Fraction(1 - (-1) ** (k + i + 1), k + i + 1)
                          for i in range(a + 1)))
        approx = float((w * x ** k).sum())
        assert abs(approx - exact) < 1e-12 * max(1.0, abs(exact))


def test_lagrange_kronecker_and_polynomial_exactness():
    nodes, _ = gauss_jacobi(6, 0, 0)
    L = lagrange(nodes, nodes)
    np.testing.assert_allclose(L.numpy(), np.eye(7), atol=1e-14)
    x = torch.linspace(-1, 1, 23, dtype=torch.float64)
    L = lagrange(nodes, x)
    dL = lagrange_deriv(nodes, x)
    for k in range(7):
        np.testing.assert_allclose((L @ nodes ** k).numpy(), (x ** k).numpy(), atol=1e-13)
        ref = k * x ** (k - 1) if k > 0 else torch.zeros_like(x)
        np.testing.assert_allclose((dL @ nodes ** k).numpy(), ref.numpy(), atol=1e-12)
