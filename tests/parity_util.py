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


ROUNDING = 2.0 ** -46      # 64 units in the last place of the summands' magnitude


def assert_parity(gpu, ora, tol=TOL, what="", mag=None):
    """Per conserved variable e:  max |gpu - ora| <= max(tol ||r_e||_inf,
    2^-46 || |r|_e ||_inf), where |r| (if given) is the residual evaluated with
    the absolute value of every term.  The second bound is the rounding error a
    correct FP64 evaluation may carry when the residual cancels a large
    background (a uniform pressure of 1/(gamma Ma^2) at Ma 0.1); elsewhere the
    first bound is the binding one."""
    gpu = gpu.detach().cpu().double()
    ora = ora.detach().cpu().double()
    worst, entry, per = parity_report(gpu, ora)
    msg = (f"parity {what}: max err / ||r_e||_inf = {worst:.3e} (per var {['%.1e' % x for x in per]}), "
           f"entrywise rel (|r|>=1e-3 max) = {entry:.3e}")
    ok = True
    ratios = []
    for c in range(ora.shape[1]):
        err = float((gpu[:, c] - ora[:, c]).abs().max())
        bound = tol * float(ora[:, c].abs().max())
        if mag is not None:
            bound = max(bound, ROUNDING * float(mag[:, c].abs().max()))
        ratios.append(err / bound if bound > 0 else err)
        ok &= err <= bound
    msg += f"; err / bound per var {['%.2f' % x for x in ratios]}"
    log(msg)
    assert ok, f"{what}: exceeds bound, ratios {ratios}"
