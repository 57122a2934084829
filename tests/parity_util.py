"""Shared helpers for the GPU parity tests (oracle vs HIP library)."""
import math
import sys

import numpy as np
import torch

import workloads as wl

TOL = 1e-12


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_problem(wk, degree=None):
    from oracle import residual as R
    mesh = wk.mesh()
    return R.setup(mesh, degree or wk.degree, wk.warp, wk.gamma, wk.ecflux, wk.dissipation)


def gpu_plan(wk, degree=None, **kw):
    import paper_2312_07874_amd as esd
    return esd.Plan.from_workload(wk, degree, **kw)


def oracle_state(prob, wk):
    """u~ from the oracle's weight-adjusted projection of the workload state."""
    from oracle import residual as R
    un = torch.tensor(wk.state(prob.geo.x_vol.numpy()))
    return R.project(prob, un)


def parity_report(gpu: torch.Tensor, ora: torch.Tensor, mag: torch.Tensor = None):
    """max |gpu - ora| / ||s^(e)||_inf per conserved variable e (state layout
    [element][variable][mode]) with s = ora, or with s = mag (the residual
    evaluated with absolute values of all terms) when given; also the entrywise
    relative error over entries with |ora| >= 1e-3 ||ora^(e)||_inf."""
    gpu = gpu.detach().cpu().double()
    ora = ora.detach().cpu().double()
    ref = ora if mag is None else mag.detach().cpu().double()
    rel, ent = [], []
    for c in range(ora.shape[1]):
        scale = float(ref[:, c].abs().max())
        err = float((gpu[:, c] - ora[:, c]).abs().max())
        rel.append(err / scale if scale > 0 else err)
        oscale = float(ora[:, c].abs().max())
        big = ora[:, c].abs() >= 1e-3 * oscale
        if oscale > 0 and bool(big.any()):
            ent.append(float(((gpu[:, c] - ora[:, c]).abs()[big] / ora[:, c].abs()[big]).max()))
    return max(rel), (max(ent) if ent else 0.0), rel


# The bar for the residual (and every state derived from it) per conserved
# variable e:  max |gpu - oracle| <= max(1e-12 ||r_e||_inf, NOISE_FACTOR * d_e),
# where d_e is the oracle's own rounding spread: the largest change of its
# result over NOISE_SEEDS when every intermediate it forms carries one rounding
# (oracle.residual.rounding_noise).  Where the residual does not cancel, the
# first term binds; where it cancels a large background (a uniform pressure of
# 1/(gamma Ma^2) at Ma 0.1 against a divergence-free velocity) the second does,
# and then only by the oracle's own measured rounding, never by anything the
# library computes.
NOISE_FACTOR = 4.0
NOISE_SEEDS = (101, 202)


def oracle_with_spread(fn, prob, setup=None, seeds=NOISE_SEEDS):
    """(fn(prob), spread): spread is the entrywise maximum over the seeds of
    |fn(prob) - fn(prob_s)|, fn(prob_s) evaluated inside
    oracle.noise.rounding_noise(seed) with prob_s = setup() built inside the
    same context (geometry included), or prob itself when setup is None."""
    from oracle.noise import rounding_noise
    ref = fn(prob)
    spread = None
    for s in seeds:
        with rounding_noise(s):
            d = (fn(setup() if setup is not None else prob) - ref).abs()
        spread = d if spread is None else torch.maximum(spread, d)
    return ref, spread


def assert_parity(gpu, ora, tol=TOL, what="", spread=None, factor=NOISE_FACTOR):
    """Per conserved variable e:  max |gpu - ora| <= max(tol ||ora_e||_inf,
    factor * max spread_e) (the second term only when the oracle's rounding
    spread is given).  Logs the error, the spread and err / bound per variable."""
    gpu = gpu.detach().cpu().double()
    ora = ora.detach().cpu().double()
    worst, entry, per = parity_report(gpu, ora)
    msg = (f"parity {what}: max err / ||r_e||_inf = {worst:.3e} (per var {['%.1e' % x for x in per]}), "
           f"entrywise rel (|r|>=1e-3 max) = {entry:.3e}")
    ok = True
    ratios, spreads = [], []
    for c in range(ora.shape[1]):
        err = float((gpu[:, c] - ora[:, c]).abs().max())
        scale = float(ora[:, c].abs().max())
        bound = tol * scale
        if spread is not None:
            d = float(spread[:, c].abs().max())
            spreads.append(d / scale if scale > 0 else d)
            bound = max(bound, factor * d)
        ratios.append(err / bound if bound > 0 else err)
        ok &= err <= bound
    if spread is not None:
        msg += f"; oracle spread / ||r_e||_inf per var {['%.1e' % x for x in spreads]}"
    msg += f"; err / bound per var {['%.2f' % x for x in ratios]}"
    cw = int(np.argmax(ratios))
    flat = int((gpu[:, cw] - ora[:, cw]).abs().argmax())
    msg += f"; worst at (element, mode) {divmod(flat, ora.shape[2]) if ora.dim() == 3 else flat} of var {cw}"
    log(msg)
    assert ok, f"{what}: exceeds bound, ratios {ratios}"
