"""The oracle's rounding-noise mode (the spread the parity bars use):
identity outside its context, reproducible per seed inside it, and a change
of the residual at the size of FP64 rounding (not zero, not more than a
rounding amplified by the residual's own cancellation)."""
import math

import torch

import workloads as wl
from oracle import residual as R
from oracle.noise import active, rounding_noise


def _case():
    L = 2.0
    mesh = wl.split_box_mesh(2, 3, L)
    warp = wl.make_warp_sinprod(L, 0.05)
    setup = lambda: R.setup(mesh, 3, warp, 1.4, 0, 1)
    prob = setup()
    ut = R.project(prob, torch.tensor(wl.RandomSmooth(2, L, 4)(prob.geo.x_vol.numpy())))
    return setup, prob, ut


def test_noise_mode_is_identity_outside_and_reproducible_inside():
    setup, prob, ut = _case()
    ref = R.residual(prob, ut)
    assert not active()
    assert torch.equal(R.residual(prob, ut), ref)
    with rounding_noise(7):
        assert active()
        a = R.residual(setup(), ut)
    with rounding_noise(7):
        b = R.residual(setup(), ut)
    with rounding_noise(8):
        c = R.residual(setup(), ut)
    assert not active()
    assert torch.equal(a, b)
    assert not torch.equal(a, c)
    assert torch.equal(R.residual(prob, ut), ref)


def test_noise_spread_is_rounding_sized():
    setup, prob, ut = _case()
    ref = R.residual(prob, ut)
    with rounding_noise(11):
        a = R.residual(setup(), ut)
    rel = float((a - ref).abs().max() / ref.abs().max())
    # one rounding per intermediate: well above zero, far below any modelling error
    assert 1e-16 < rel < 1e-12, rel
    # the noise scale argument scales the spread
    with rounding_noise(11, scale=2.0 ** -40):
        big = R.residual(setup(), ut)
    rel_big = float((big - ref).abs().max() / ref.abs().max())
    assert rel_big > 100 * rel
