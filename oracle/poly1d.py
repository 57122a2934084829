"""One-dimensional orthogonal polynomials, Gauss quadrature and Lagrange bases.

Test infrastructure (see the package docstring).  Follows Sec. 2.4 of the paper:
normalized Jacobi polynomials orthonormal w.r.t. (1-x)^a (1+x)^b, Gauss rules
whose q+1 nodes are the zeros of P_{q+1}^{(a,b)} (exact to degree 2q+1), the
Lagrange polynomials of eq. (lagrange) and their derivatives.
"""
from __future__ import annotations

import math

import numpy as np
import torch

DT = torch.float64


def _gamma0(a: float, b: float) -> float:
    # integral of (1-x)^a (1+x)^b over [-1,1]
    return 2.0 ** (a + b + 1) * math.gamma(a + 1) * math.gamma(b + 1) / math.gamma(a + b + 2)


def _rec_coeffs(n_max: int, a: float, b: float):
    """Three-term recurrence x P_n = A_{n+1} P_{n+1} + B_n P_n + A_n P_{n-1}
    of the orthonormal Jacobi polynomials."""
    A = np.zeros(n_max + 2)
    B = np.zeros(n_max + 2)
    for n in range(0, n_max + 2):
        s = 2 * n + a + b
        if n == 0:
            B[0] = (b - a) / (a + b + 2)
        else:
            B[n] = (b * b - a * a) / (s * (s + 2)) if s * (s + 2) != 0 else 0.0
        if n >= 1:
            num = 4.0 * n * (n + a + b) * (n + a) * (n + b)
            den = s * s * (s - 1) * (s + 1)
            A[n] = math.sqrt(num / den)
    return A, B


def jacobi(n_max: int, a: float, b: float, x) -> torch.Tensor:
    """Orthonormal Jacobi polynomials P_0..P_{n_max} at x -> [n_max+1, len(x)]."""
    x = torch.as_tensor(x, dtype=DT)
    A, B = _rec_coeffs(n_max, a, b)
    P = torch.zeros((n_max + 1,) + tuple(x.shape), dtype=DT)
    P[0] = 1.0 / math.sqrt(_gamma0(a, b))
    if n_max >= 1:
        P[1] = (x - B[0]) * P[0] / A[1]
    for n in range(1, n_max):
        P[n + 1] = ((x - B[n]) * P[n] - A[n] * P[n - 1]) / A[n + 1]
    return P


def jacobi_deriv(n_max: int, a: float, b: float, x) -> torch.Tensor:
    """d/dx of the orthonormal Jacobi polynomials: sqrt(n(n+a+b+1)) P_{n-1}^{(a+1,b+1)}."""
    x = torch.as_tensor(x, dtype=DT)
    dP = torch.zeros((n_max + 1,) + tuple(x.shape), dtype=DT)
    if n_max >= 1:
        Q = jacobi(n_max - 1, a + 1, b + 1, x)
        for n in range(1, n_max + 1):
            dP[n] = math.sqrt(n * (n + a + b + 1)) * Q[n - 1]
    return dP


def gauss_jacobi(q: int, a: float, b: float):
    """q+1 Gauss nodes (zeros of P_{q+1}^{(a,b)}) and weights for (1-x)^a(1+x)^b.

    Golub-Welsch: eigenvalues of the symmetric tridiagonal recurrence matrix are
    the nodes; weights are gamma0 times squared first eigenvector components."""
    n = q + 1
    A, B = _rec_coeffs(n, a, b)
    T = np.diag(B[:n]) + np.diag(A[1:n], 1) + np.diag(A[1:n], -1)
    lam, vec = np.linalg.eigh(T)
    w = _gamma0(a, b) * vec[0, :] ** 2
    order = np.argsort(lam)
    return torch.tensor(lam[order], dtype=DT), torch.tensor(w[order], dtype=DT)


def lagrange(nodes, x) -> torch.Tensor:
    """Lagrange basis of eq. (lagrange): L[k, j] = l_j(x_k) (product formula)."""
    nodes = torch.as_tensor(nodes, dtype=DT)
    x = torch.as_tensor(x, dtype=DT).reshape(-1)
    n = nodes.shape[0]
    L = torch.ones((x.shape[0], n), dtype=DT)
    for j in range(n):
        for m in range(n):
            if m != j:
                L[:, j] = L[:, j] * (x - nodes[m]) / (nodes[j] - nodes[m])
    return L


def lagrange_deriv(nodes, x) -> torch.Tensor:
    """dL[k, j] = l_j'(x_k): derivative of the product formula, term by term."""
    nodes = torch.as_tensor(nodes, dtype=DT)
    x = torch.as_tensor(x, dtype=DT).reshape(-1)
    n = nodes.shape[0]
    dL = torch.zeros((x.shape[0], n), dtype=DT)
    for j in range(n):
        for m in range(n):
            if m == j:
                continue
            term = torch.full_like(x, 1.0 / float(nodes[j] - nodes[m]))
            for k in range(n):
                if k != j and k != m:
                    term = term * (x - nodes[k]) / (nodes[j] - nodes[k])
            dL[:, j] += term
    return dL
