"""Rounding-noise mode of the oracle (test infrastructure).

Inside rounding_noise(seed) every quantity the residual forms or reads --
input coefficients; every intermediate of the physics formulas (primitive
variables, entropy and its variables, the inverse map U(w), the logarithmic
means and the averages, every component of the two-point and interface
fluxes); nodal entropy variables, their projection and facet values; the
nodal right-hand side and the output; and the operator and geometry tables it
applies (V, R, R^T B, S^l, the weight-adjusted inverse, w J, G, J_f n, n,
w J_f), and, when the geometry is built inside the context, every
intermediate of the geometry (warp displacement at the mapping nodes, Lagrange
interpolation and derivative matrices, mapping gradients, the Jacobian at the
mapping nodes and its interpolant, the curl-form products and curls, G, J_f n,
J_f, n) -- is multiplied by (1 + u z) with u = 2^-53 (the FP64 unit roundoff)
and z uniform on [-1, 1], independently per entry (symmetric in (i, j) for
S^l, which stays skew): one rounding of every intermediate.  The change of the
result under it is the rounding spread that any correct FP64 evaluation of the
same definition (in another order, with other groupings) carries, including
the amplification by cancellation inside the formulas (e.g. ln rho as the
difference of two numbers near ln p at a large uniform pressure).  The GPU
parity tests bound the library's difference from the oracle by a small
multiple of it.  Outside the context every function is the identity.
"""
from __future__ import annotations

import contextlib

import torch

_NOISE = {"gen": None, "scale": 0.0}


@contextlib.contextmanager
def rounding_noise(seed: int, scale: float = 2.0 ** -53):
    old = dict(_NOISE)
    _NOISE.update(gen=torch.Generator().manual_seed(int(seed)), scale=float(scale))
    try:
        yield
    finally:
        _NOISE.update(old)


def active() -> bool:
    return _NOISE["gen"] is not None


def rn(x):
    """x (1 + u z) per entry, or x itself outside the context."""
    g = _NOISE["gen"]
    if g is None:
        return x
    if not torch.is_tensor(x):
        x = torch.as_tensor(x, dtype=torch.float64)
    z = torch.rand(x.shape, generator=g, dtype=x.dtype) * 2.0 - 1.0
    return x * (1.0 + _NOISE["scale"] * z)


def rn_skew(S):
    """As rn for a skew matrix, with z symmetric so that the result stays skew."""
    g = _NOISE["gen"]
    if g is None:
        return S
    z = torch.rand(S.shape, generator=g, dtype=S.dtype) * 2.0 - 1.0
    z = torch.triu(z, 1) + torch.triu(z, 1).T + torch.diag(torch.diagonal(z))
    return S * (1.0 + _NOISE["scale"] * z)


def rsum(t, dim: int):
    """t.sum(dim); inside the context every partial sum of the sequential sum
    along dim (in index order) carries one rounding: the exact sum plus
    sum_k delta_k s_k, s_k the k-th partial sum, delta_k = u z_k for the terms
    that are not zero (adding an exact zero does not round)."""
    s = t.sum(dim)
    g = _NOISE["gen"]
    if g is None:
        return s
    c = torch.cumsum(t, dim)
    z = torch.rand(c.shape, generator=g, dtype=c.dtype) * 2.0 - 1.0
    return s + (_NOISE["scale"] * z * (t != 0) * c).sum(dim)


def esum(eq: str, *ops):
    """torch.einsum(eq, *ops) for an equation that contracts index letters;
    inside the context the products are formed explicitly and each contraction
    is a sequential sum whose partial sums carry one rounding (rsum)."""
    if _NOISE["gen"] is None:
        return torch.einsum(eq, *ops)
    lhs, out = eq.split("->")
    letters = [c for c in dict.fromkeys(lhs.replace(",", "")) if c not in out]
    prod = torch.einsum(f"{lhs}->{out}{''.join(letters)}", *ops)
    for _ in letters:
        prod = rsum(prod, -1)
    return prod
