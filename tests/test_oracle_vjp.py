"""Pins for the oracle's vector-Jacobian product of the residual.

The VJP is reverse-mode autodiff of the dense residual.  It is pinned by
central finite differences (h = 1e-6), by the dot-product identity against a
forward-mode directional derivative, and by the 1-ring restriction used for
sampled checks on large meshes."""
import math

import numpy as np
import pytest
import torch
from torch.func import jvp

import workloads as wl
from oracle import residual as R


def _setup(dim, M, p, diss):
    L = 2.0 if dim == 2 else 2 * math.pi
    prob = R.setup(wl.split_box_mesh(dim, M, L), p, wl.make_warp_sinprod(L, 0.05), 1.4, 0, diss)
    st = wl.RandomSmooth(dim, L, 11)
    ut = R.project(prob, torch.tensor(st(prob.geo.x_vol.numpy())))
    return prob, ut


@pytest.mark.parametrize("dim,M,p,diss", [(2, 3, 2, 0), (2, 3, 3, 1), (3, 3, 2, 0)])
def test_vjp_finite_difference_and_dot(dim, M, p, diss):
    prob, ut = _setup(dim, M, p, diss)
    g = torch.Generator().manual_seed(1)
    vbar = torch.randn(ut.shape, generator=g, dtype=torch.float64)
    grad = R.vjp(prob, ut, vbar)
    h = 1e-6
    for k in range(3):
        delta = torch.randn(ut.shape, generator=g, dtype=torch.float64)
        fp = (R.residual_chunked(prob, ut + h * delta) * vbar).sum()
        fm = (R.residual_chunked(prob, ut - h * delta) * vbar).sum()
        fd = float((fp - fm) / (2 * h))
        ad = float((grad * delta).sum())
        assert abs(fd - ad) < 1e-6 * max(1.0, abs(ad)), (fd, ad)
        _, jd = jvp(lambda x: R.residual_chunked(prob, x), (ut,), (delta,))
        lhs = float((vbar * jd).sum())
        assert abs(lhs - ad) < 1e-11 * max(1.0, abs(ad))


def test_vjp_subset_rows_equal_full():
    prob, ut = _setup(3, 3, 2, 1)
    vbar = torch.randn(ut.shape, generator=torch.Generator().manual_seed(2), dtype=torch.float64)
    full = R.vjp(prob, ut, vbar)
    el = np.array([0, 17, 100])
    sub = R.vjp(prob, ut, vbar, el)
    assert float((sub - full[el]).abs().max()) < 1e-12 * float(full.abs().max())
