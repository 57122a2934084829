"""Pins for the oracle's Euler physics (Sec. 2.2, 4.6, 7.1-7.2).

Entropy variables against finite differences of the entropy, the inverse map,
the log mean against 50-digit arithmetic across its series threshold, and the
defining properties of the EC two-point fluxes (consistency, symmetry, Tadmor's
condition) and of the interface flux (conservation, consistency, entropy
stability)."""
import contextlib

import mpmath
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import physics as ph

G = 1.4


def random_states(n, d, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, n)
    v = rng.uniform(-1, 1, (n, d))
    p = rng.uniform(0.5, 3.0, n)
    return torch.tensor(wl.prim_to_cons(rho, v, p, G))


@pytest.mark.parametrize("d", [2, 3])
def test_entropy_variables_are_gradient_of_entropy(d):
    u = random_states(20, d, 1)
    W = ph.entropy_vars(u, G)
    h = 1e-6
    for k in range(d + 2):
        e = torch.zeros(d + 2, dtype=torch.float64)
        e[k] = h
        fd = (ph.entropy(u + e, G) - ph.entropy(u - e, G)) / (2 * h)
        np.testing.assert_allclose(W[:, k].numpy(), fd.numpy(), rtol=1e-7, atol=1e-7)


@pytest.mark.parametrize("d", [2, 3])
def test_entropy_variable_inverse(d):
    u = random_states(50, d, 2)
    np.testing.assert_allclose(ph.cons_from_entropy(ph.entropy_vars(u, G), G).numpy(), u.numpy(), rtol=1e-13)


def test_log_mean_against_high_precision():
    mpmath.mp.dps = 50
    rng = np.random.default_rng(3)
    a = rng.uniform(0.1, 10, 400)
    # ratios straddling the series threshold f^2 = 1e-4 (|f| = 0.01)
    f = np.concatenate([rng.uniform(-0.03, 0.03, 300), rng.uniform(-0.9, 0.9, 100)])
    b = a * (1 + f) / (1 - f)
    lm = ph.log_mean(torch.tensor(a), torch.tensor(b)).numpy()
    ilm = ph.inv_log_mean(torch.tensor(a), torch.tensor(b)).numpy()
    for i in range(len(a)):
        A, B = mpmath.mpf(a[i]), mpmath.mpf(b[i])
        ex = A if A == B else (B - A) / (mpmath.log(B) - mpmath.log(A))
        assert abs(lm[i] - float(ex)) <= 2e-14 * float(ex)
        assert abs(ilm[i] - float(1 / ex)) <= 2e-14 * float(1 / ex)


@pytest.mark.parametrize("flux", [0, 1])
@pytest.mark.parametrize("d", [2, 3])
def test_ec_flux_consistency_symmetry_tadmor(flux, d):
    um = random_states(200, d, 4)
    up = random_states(200, d, 5)
    rng = np.random.default_rng(6)
    n = torch.tensor(rng.standard_normal((200, d)))
    F = ph.EC_FLUXES[flux]
    # consistency: f#(U,U,n) = f(U,n)
    np.testing.assert_allclose(F(um, um, n, G).numpy(), ph.euler_flux(um, n, G).numpy(), rtol=1e-13, atol=1e-13)
    # symmetry
    np.testing.assert_allclose(F(um, up, n, G).numpy(), F(up, um, n, G).numpy(), rtol=1e-13, atol=1e-13)
    # Tadmor: (W+ - W-)^T f# = (psi+ - psi-) . n
    lhs = ((ph.entropy_vars(up, G) - ph.entropy_vars(um, G)) * F(um, up, n, G)).sum(-1)
    rhs = ((ph.flux_potential(up, G) - ph.flux_potential(um, G)) * n).sum(-1)
    np.testing.assert_allclose(lhs.numpy(), rhs.numpy(), atol=1e-12)


def test_printed_energy_grouping_is_inconsistent():
    """The reading of eq. (ranocha_flux): with 1/2 multiplying the whole bracket
    the energy flux is not consistent, with 1/2 on v-.v+ only it is."""
    u = random_states(10, 3, 7)
    n = torch.tensor([[0.3, -0.4, 0.8]] * 10, dtype=torch.float64)
    rho, v, p = ph.prim(u, G)
    vn = (v * n).sum(-1)
    printed = 0.5 * rho * vn * ((v * v).sum(-1) + p / rho / (G - 1)) + p * vn
    exact = ph.euler_flux(u, n, G)[:, -1]
    assert float((printed - exact).abs().max()) > 1e-2
    np.testing.assert_allclose(ph.ranocha_flux(u, u, n, G)[:, -1].numpy(), exact.numpy(), rtol=1e-13)


@pytest.mark.parametrize("diss", [0, 1])
def test_interface_flux_properties(diss):
    d = 3
    um = random_states(100, d, 8)
    up = random_states(100, d, 9)
    rng = np.random.default_rng(10)
    n = torch.tensor(rng.standard_normal((100, d)))
    n = n / n.norm(dim=-1, keepdim=True)
    f = ph.interface_flux(um, up, n, G, 0, diss)
    np.testing.assert_allclose(f.numpy(), -ph.interface_flux(up, um, -n, G, 0, diss).numpy(), atol=1e-13)
    np.testing.assert_allclose(ph.interface_flux(um, um, n, G, 0, diss).numpy(),
                               ph.euler_flux(um, n, G).numpy(), rtol=1e-13, atol=1e-13)
    lhs = ((ph.entropy_vars(up, G) - ph.entropy_vars(um, G)) * f).sum(-1)
    rhs = ((ph.flux_potential(up, G) - ph.flux_potential(um, G)) * n).sum(-1)
    if diss:
        assert bool((lhs <= rhs + 1e-12).all())
    else:
        np.testing.assert_allclose(lhs.numpy(), rhs.numpy(), atol=1e-12)


def test_tie_derivative_changes_only_the_derivative():
    """At equal sound speeds the wave speed max(c-, c+) is not differentiable:
    the one-sided derivatives differ by J (grad c+ - grad c-) x [u].  The
    default derivative there is the mean of the one-sided ones; under
    tie_derivative it moves entirely to the chosen side; the value is
    bit-identical in every mode, and away from ties nothing changes."""
    g = 1.4
    # same p/rho (same c), different velocity and density
    f64 = dict(dtype=torch.float64)
    um = torch.tensor([[1.0, 0.3, -0.2, 1.0 / 0.4 + 0.5 * 1.0 * (0.3 ** 2 + 0.2 ** 2)]], **f64)
    rp, vp = 2.0, torch.tensor([-0.1, 0.4], **f64)
    pp = 2.0   # p/rho = 1 on both sides
    up = torch.cat([torch.tensor([rp], **f64), rp * vp,
                    torch.tensor([pp / 0.4 + 0.5 * rp * float((vp * vp).sum())], **f64)])[None]
    n = torch.tensor([[0.6, 0.8]], dtype=torch.float64)
    vals, grads = [], []
    for side in (None, "-", "+"):
        a = um.clone().requires_grad_(True)
        b = up.clone().requires_grad_(True)
        ctx = contextlib.nullcontext() if side is None else ph.tie_derivative(side)
        with ctx:
            lam = ph.davis_speed(a, b, n, g)
        lam.sum().backward()
        vals.append(lam.detach())
        grads.append((a.grad.clone(), b.grad.clone()))
    assert torch.equal(vals[0], vals[1]) and torch.equal(vals[0], vals[2])
    # the default is the mean of the two one-sided derivatives
    for k in (0, 1):
        assert torch.allclose(grads[0][k], 0.5 * (grads[1][k] + grads[2][k]), rtol=0, atol=1e-15)
    dc_p = grads[2][1] - grads[1][1]
    dc_m = grads[1][0] - grads[2][0]
    assert float(dc_p.abs().max()) > 0.1 and float(dc_m.abs().max()) > 0.1
    # away from a tie the context manager changes nothing
    up2 = up.clone()
    up2[0, 3] += 1.0
    res = []
    for side in (None, "+"):
        b = up2.clone().requires_grad_(True)
        ctx = contextlib.nullcontext() if side is None else ph.tie_derivative(side)
        with ctx:
            ph.davis_speed(um, b, n, g).sum().backward()
        res.append(b.grad.clone())
    assert torch.equal(res[0], res[1])
