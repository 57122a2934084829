"""Pins of the conservative and skew-symmetric weak forms, eqs. (rhs_cons) and
(rhs_skew), without entropy projection: on affine meshes the two are equal
(SBP property and Nanson's formula make their difference vanish); both
conserve the conserved integrals on periodic meshes (the weight-adjusted
inverse reproduces constants) and preserve a free stream on curved elements
(discrete metric identities); on curved elements the two differ (the
skew-symmetric form's metric terms are not those of the conservative one)."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import residual as R


def _prob(dim, amp, diss=1):
    L = 2.0 if dim == 2 else 2 * math.pi
    mesh = wl.split_box_mesh(dim, 3, L)
    warp = wl.make_warp_sinprod(L, amp) if amp else wl.warp_none
    prob = R.setup(mesh, 3, warp, 1.4, 0, diss)
    ut = R.project(prob, torch.tensor(wl.RandomSmooth(dim, L, 4)(prob.geo.x_vol.numpy())))
    return prob, ut


@pytest.mark.parametrize("dim", [2, 3])
def test_forms_agree_on_affine_meshes(dim):
    prob, ut = _prob(dim, 0.0)
    el = np.arange(0, prob.ne, 5)
    c, s = R.residual_conservative(prob, ut, el), R.residual_skew(prob, ut, el)
    assert float((c - s).abs().max()) < 1e-12 * float(c.abs().max())


@pytest.mark.parametrize("dim", [2, 3])
def test_forms_conservative_free_stream_and_distinct_on_curved_meshes(dim):
    prob, ut = _prob(dim, 0.05)
    V = prob.ref.V
    outs = {}
    for name, fn in (("cons", R.residual_conservative), ("skew", R.residual_skew)):
        du = fn(prob, ut)
        rate = torch.einsum("k,ek,ekc->c", prob.ref.w, prob.geo.J, torch.einsum("ki,eci->ekc", V, du))
        assert float(rate.abs().max()) < 1e-12 * float(du.abs().max()) * prob.ne, name
        u0 = torch.tensor(wl.prim_to_cons(np.array(1.1), np.array([0.4, -0.3, 0.2][:dim]), np.array(0.8)))
        uf = R.project(prob, u0.expand(prob.ne, prob.ref.Nq, dim + 2))
        assert float(fn(prob, uf).abs().max()) < 1e-12, name
        outs[name] = du
    assert float((outs["cons"] - outs["skew"]).abs().max()) > 1e-4 * float(outs["cons"].abs().max())
