"""Pins of the interface dissipation variants the paper names after eq.
(num_flux): scalar dissipation on the jump of the entropy variables and
matrix dissipation.  The closed-form dU/dW against automatic differentiation
of U(W); the basis-free |A_n| against an eigendecomposition of the flux
Jacobian; conservation, consistency and entropy stability of both fluxes;
the residual's entropy rate is negative on a periodic curved mesh."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import physics as ph
from oracle import residual as R

G = 1.4


def _states(d, n, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 1.5, n)
    v = rng.uniform(-0.6, 0.6, (n, d))
    p = rng.uniform(0.5, 1.5, n)
    return torch.tensor(wl.prim_to_cons(rho, v, p, G))


@pytest.mark.parametrize("d", [2, 3])
def test_entropy_jacobian_is_du_dw(d):
    u = _states(d, 7, 1)
    rho, v, p = ph.prim(u, G)
    A = ph.entropy_jacobian(rho, v, p, G)
    for k in range(u.shape[0]):
        w = ph.entropy_vars(u[k], G)
        J = torch.autograd.functional.jacobian(lambda x: ph.cons_from_entropy(x, G), w)
        np.testing.assert_allclose(A[k].numpy(), J.numpy(), rtol=1e-12, atol=1e-12)
        assert float(torch.linalg.eigvalsh(A[k]).min()) > 0


@pytest.mark.parametrize("d", [2, 3])
def test_abs_flux_jacobian_against_eigendecomposition(d):
    u = _states(d, 5, 2)
    rng = np.random.default_rng(3)
    for k in range(u.shape[0]):
        n = torch.tensor(rng.standard_normal(d))
        n = n / n.norm()
        A = torch.autograd.functional.jacobian(lambda x: ph.euler_flux(x, n, G), u[k])
        lam, X = np.linalg.eig(A.numpy())
        absA = (X @ np.diag(np.abs(lam)) @ np.linalg.inv(X)).real
        dU = torch.tensor(rng.standard_normal(d + 2))
        rho, v, p = ph.prim(u[k], G)
        got = ph.abs_flux_jacobian_apply(rho, v, p, n, G, dU)
        np.testing.assert_allclose(got.numpy(), absA @ dU.numpy(), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("diss", [2, 3])
@pytest.mark.parametrize("d", [2, 3])
def test_dissipative_fluxes_conservative_consistent_entropy_stable(diss, d):
    um, up = _states(d, 200, 4), _states(d, 200, 5)
    rng = np.random.default_rng(6)
    n = torch.tensor(rng.standard_normal((200, d)))
    n = n / n.norm(dim=-1, keepdim=True)
    f = ph.interface_flux(um, up, n, G, 0, diss)
    np.testing.assert_allclose(f.numpy(), -ph.interface_flux(up, um, -n, G, 0, diss).numpy(), atol=1e-13)
    np.testing.assert_allclose(ph.interface_flux(um, um, n, G, 0, diss).numpy(), ph.euler_flux(um, n, G).numpy(),
                               rtol=1e-13, atol=1e-13)
    dw = ph.entropy_vars(up, G) - ph.entropy_vars(um, G)
    lhs = (dw * f).sum(-1)
    rhs = ((ph.flux_potential(up, G) - ph.flux_potential(um, G)) * n).sum(-1)
    # strictly dissipative where the states differ
    assert bool((lhs < rhs).all())


@pytest.mark.parametrize("diss", [2, 3])
def test_residual_entropy_rate_negative(diss):
    L = 2.0
    mesh = wl.split_box_mesh(2, 3, L)
    prob = R.setup(mesh, 3, wl.make_warp_sinprod(L, 0.05), G, 0, diss)
    st = wl.RandomSmooth(2, L, 9)
    ut = R.project(prob, torch.tensor(st(prob.geo.x_vol.numpy())))
    du = R.residual_chunked(prob, ut)
    V = prob.ref.V
    rate = torch.einsum("k,ek,ekc->c", prob.ref.w, prob.geo.J, torch.einsum("ki,eci->ekc", V, du))
    assert float(rate.abs().max()) < 1e-12 * float(du.abs().max()) * prob.ne
    assert float(R.entropy_rate(prob, ut, du)) < 0
