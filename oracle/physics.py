"""Compressible Euler physics for the entropy-stable scheme.

Test infrastructure (see the package docstring).  Written from Sec. 7.1-7.2:
  * eq. (euler): conservative variables (rho, rho v, E), fluxes, ideal gas;
  * eq. (euler_entropy): S = -rho s/(gamma-1) with s = ln p - gamma ln rho; the
    entropy variables are W = dS/dU (Sec. 2.2) and U(W) is their inverse;
  * arithmetic and logarithmic means, the latter (a+ - a-)/(ln a+ - ln a-) with a
    series for nearly equal arguments (ln(a+/a-) = 2 atanh f, f = (a+-a-)/(a++a-),
    truncated after f^6/7 when f^2 < 1e-4);
  * eq. (ranocha_flux): Ranocha's entropy-conservative, kinetic-energy
    preserving flux.  Reading: the factor 1/2 in the energy component multiplies
    v- . v+ only (the printed grouping is not consistent with f_m(U));
  * Chandrashekar's entropy-conservative flux (cited for dissipation in Sec. 4.6),
    used by the small 2D density-wave workload;
  * eqs. (num_flux, wave_speed): f* = f# - lambda/2 (u+ - u-) with Davis' wave
    speed; the entropy-conservative variant drops the dissipation.
States are tensors [..., d+2]; directions n are [..., d].
"""
from __future__ import annotations

import contextlib

import torch

from .noise import rn

LOG_SERIES_THRESHOLD = 1.0e-4


def prim(u: torch.Tensor, gamma: float):
    d = u.shape[-1] - 2
    rho = u[..., 0]
    v = rn(u[..., 1:1 + d] / rho[..., None])
    p = rn((gamma - 1.0) * rn(u[..., d + 1] - rn(0.5 * rho * (v * v).sum(-1))))
    return rho, v, p


def euler_flux(u: torch.Tensor, n: torch.Tensor, gamma: float) -> torch.Tensor:
    """f(U, n) = sum_m n_m f_m(U)."""
    d = u.shape[-1] - 2
    rho, v, p = prim(u, gamma)
    vn = (v * n).sum(-1)
    out = [rho * vn]
    for i in range(d):
        out.append(rho * v[..., i] * vn + p * n[..., i])
    out.append(vn * (u[..., d + 1] + p))
    return torch.stack(out, -1)


def entropy(u: torch.Tensor, gamma: float) -> torch.Tensor:
    rho, v, p = prim(u, gamma)
    s = torch.log(p) - gamma * torch.log(rho)
    return -rho * s / (gamma - 1.0)


def entropy_vars(u: torch.Tensor, gamma: float) -> torch.Tensor:
    """W(U) = dS/dU."""
    d = u.shape[-1] - 2
    rho, v, p = prim(u, gamma)
    s = rn(rn(torch.log(p)) - rn(gamma * rn(torch.log(rho))))
    w1 = rn(rn((gamma - s) / (gamma - 1.0)) - rn(0.5 * rho * (v * v).sum(-1) / p))
    out = [w1]
    for i in range(d):
        out.append(rn(rho * v[..., i] / p))
    out.append(rn(-rho / p))
    return torch.stack(out, -1)


def cons_from_entropy(w: torch.Tensor, gamma: float) -> torch.Tensor:
    """U(W), the inverse of entropy_vars."""
    d = w.shape[-1] - 2
    b = -w[..., d + 1]                       # rho / p
    v = rn(w[..., 1:1 + d] / b[..., None])
    s = rn(gamma - rn((gamma - 1.0) * rn(w[..., 0] + rn(0.5 * b * (v * v).sum(-1)))))
    rho = rn(torch.exp(rn(-rn(s + rn(torch.log(b))) / (gamma - 1.0))))
    p = rn(rho / b)
    E = rn(rn(p / (gamma - 1.0)) + rn(0.5 * rho * (v * v).sum(-1)))
    return torch.cat([rho[..., None], rn(rho[..., None] * v), E[..., None]], -1)


def flux_potential(u: torch.Tensor, gamma: float) -> torch.Tensor:
    """psi_m = W^T f_m - F_m = rho v_m for this entropy pair."""
    d = u.shape[-1] - 2
    rho, v, p = prim(u, gamma)
    return rho[..., None] * v


def _series(f2):
    return rn(1.0 + f2 / 3.0 + f2 * f2 / 5.0 + f2 * f2 * f2 / 7.0)


def _f2(am, ap):
    f = (ap - am) / (ap + am)
    return f * f


def log_mean_series(am, ap):
    """(a- + a+) / (2 (1 + f^2/3 + f^4/5 + f^6/7)): the log mean for f^2 < 1e-4."""
    return rn(rn(am + ap) / (2.0 * _series(rn(_f2(am, ap)))))


def log_mean_log(am, ap):
    """(a+ - a-) / (ln a+ - ln a-)."""
    return rn(rn(ap - am) / rn(rn(torch.log(ap)) - rn(torch.log(am))))


def inv_log_mean_series(am, ap):
    return rn(2.0 * _series(rn(_f2(am, ap))) / rn(am + ap))


def inv_log_mean_log(am, ap):
    return rn(rn(rn(torch.log(ap)) - rn(torch.log(am))) / rn(ap - am))


def log_mean(am: torch.Tensor, ap: torch.Tensor) -> torch.Tensor:
    """{a}_ln = (a+ - a-)/(ln a+ - ln a-); series branch for nearly equal args.
    The log branch is evaluated on safe arguments where the series is used, so
    that autograd never sees 0/0."""
    small = _f2(am, ap) < LOG_SERIES_THRESHOLD
    one = torch.ones_like(am)
    big = log_mean_log(torch.where(small, one, am), torch.where(small, 2.0 * one, ap))
    return torch.where(small, log_mean_series(am, ap), big)


def inv_log_mean(am: torch.Tensor, ap: torch.Tensor) -> torch.Tensor:
    """1/{a}_ln."""
    small = _f2(am, ap) < LOG_SERIES_THRESHOLD
    one = torch.ones_like(am)
    big = inv_log_mean_log(torch.where(small, one, am), torch.where(small, 2.0 * one, ap))
    return torch.where(small, inv_log_mean_series(am, ap), big)


def ranocha_flux(um: torch.Tensor, up: torch.Tensor, n: torch.Tensor, gamma: float) -> torch.Tensor:
    """Directional EC flux f#(U-, U+, n) = sum_m n_m f#_m (eq. ranocha_flux)."""
    d = um.shape[-1] - 2
    rm, vm, pm = prim(um, gamma)
    rp, vp, pp = prim(up, gamma)
    rho_ln = log_mean(rm, rp)
    inv_rp_ln = inv_log_mean(rn(rm / pm), rn(rp / pp))       # 1 / {rho/p}_ln
    vavg = rn(0.5 * (vm + vp))
    pavg = rn(0.5 * (pm + pp))
    vn = rn((vavg * n).sum(-1))
    f_rho = rn(rho_ln * vn)
    out = [f_rho]
    for i in range(d):
        out.append(rn(rn(f_rho * vavg[..., i]) + rn(pavg * n[..., i])))
    vmvp = rn((vm * vp).sum(-1))
    fE = rn(rn(f_rho * rn(rn(0.5 * vmvp) + rn(inv_rp_ln / (gamma - 1.0))))
            + rn(0.5 * rn(rn(pm * (vp * n).sum(-1)) + rn(pp * (vm * n).sum(-1)))))
    out.append(fE)
    return torch.stack(out, -1)


def chandrashekar_flux(um: torch.Tensor, up: torch.Tensor, n: torch.Tensor, gamma: float) -> torch.Tensor:
    """Chandrashekar's EC flux with beta = rho/(2p): f_rho = {rho}_ln {v}.n,
    f_rhov = f_rho {v} + {rho}/(2{beta}) n, energy closing Tadmor's condition."""
    d = um.shape[-1] - 2
    rm, vm, pm = prim(um, gamma)
    rp, vp, pp = prim(up, gamma)
    bm = rn(rm / (2.0 * pm))
    bp = rn(rp / (2.0 * pp))
    rho_ln = log_mean(rm, rp)
    inv_b_ln = inv_log_mean(bm, bp)
    vavg = rn(0.5 * (vm + vp))
    phat = rn(rn(0.5 * (rm + rp)) / rn(bm + bp))              # {rho} / (2 {beta})
    vn = rn((vavg * n).sum(-1))
    f_rho = rn(rho_ln * vn)
    out = [f_rho]
    for i in range(d):
        out.append(rn(rn(f_rho * vavg[..., i]) + rn(phat * n[..., i])))
    vmvp = rn((vm * vp).sum(-1))
    fE = rn(rn(f_rho * rn(rn(0.5 * vmvp) + rn(0.5 * inv_b_ln / (gamma - 1.0)))) + rn(phat * vn))
    out.append(fE)
    return torch.stack(out, -1)


EC_FLUXES = {0: ranocha_flux, 1: chandrashekar_flux}


# Reverse-mode derivative of max(a-, a+) at ties.  max is not differentiable
# where its arguments agree, and a tie up to rounding makes the one-sided
# choice depend on rounding.  Convention: where |a- - a+| <= TIE_REL max(|a-|,
# |a+|) the derivative is the mean of the two one-sided derivatives (the value
# is max either way).  Inside tie_derivative(side) the derivative at such
# near-ties is instead taken from one side ("-" interior, "+" exterior), to
# measure the spread of the valid one-sided derivatives.
TIE_REL = 1.0e-10
_TIE = {"side": None}


@contextlib.contextmanager
def tie_derivative(side: str):
    assert side in ("-", "+")
    old = dict(_TIE)
    _TIE.update(side=side)
    try:
        yield
    finally:
        _TIE.update(old)


def _max(a, b):
    val = torch.where(a >= b, a, b)
    near = (a - b).abs() <= TIE_REL * torch.maximum(a.abs(), b.abs())
    side = _TIE["side"]
    tie = 0.5 * (a + b) if side is None else (a if side == "-" else b)
    src = torch.where(near, tie, val)
    return val.detach() + (src - src.detach())


def davis_speed(um, up, n, gamma):
    """lambda of eq. (wave_speed); its derivative at near-ties as in _max."""
    rm, vm, pm = prim(um, gamma)
    rp, vp, pp = prim(up, gamma)
    a = (vm * n).sum(-1).abs()
    b = (vp * n).sum(-1).abs()
    cm = torch.sqrt(gamma * pm / rm)
    cp = torch.sqrt(gamma * pp / rp)
    return _max(a, b) + _max(cm, cp)


def entropy_jacobian(rho, v, p, gamma):
    """A0 = dU/dW, the (symmetric positive definite) Jacobian of the
    conservative variables with respect to the entropy variables of
    eq. (euler_entropy), at the primitive state (rho, v, p):
        [[rho,   rho v^T,              E],
         [rho v, rho v v^T + p I,      rho H v],
         [E,     rho H v^T,            rho H^2 - a^2 p/(gamma-1)]]
    with a^2 = gamma p/rho, H = a^2/(gamma-1) + |v|^2/2, E = p/(gamma-1) + rho |v|^2/2."""
    d = v.shape[-1]
    v2 = (v * v).sum(-1)
    a2 = gamma * p / rho
    H = a2 / (gamma - 1.0) + 0.5 * v2
    E = p / (gamma - 1.0) + 0.5 * rho * v2
    n = d + 2
    A = torch.zeros(rho.shape + (n, n), dtype=rho.dtype)
    A[..., 0, 0] = rho
    A[..., 0, 1:1 + d] = rho[..., None] * v
    A[..., 1:1 + d, 0] = rho[..., None] * v
    A[..., 0, d + 1] = E
    A[..., d + 1, 0] = E
    A[..., 1:1 + d, 1:1 + d] = rho[..., None, None] * v[..., :, None] * v[..., None, :] \
        + p[..., None, None] * torch.eye(d, dtype=rho.dtype)
    A[..., 1:1 + d, d + 1] = (rho * H)[..., None] * v
    A[..., d + 1, 1:1 + d] = (rho * H)[..., None] * v
    A[..., d + 1, d + 1] = rho * H * H - a2 * p / (gamma - 1.0)
    return A


def abs_flux_jacobian_apply(rho, v, p, n, gamma, dU):
    """|A_n| dU for the Euler flux Jacobian A_n = d(F . n)/dU (n a unit vector)
    at the primitive state (rho, v, p): the acoustic waves of speeds
    v.n -+ a with strengths alpha_-+ = (dp -+ rho a dv_n)/(2 a^2) along
    r_-+ = (1, v -+ a n, H -+ a v.n), and the rest of dU (entropy and shear
    waves) at speed v.n; dp and dv are the primitive jumps that dU stands for
    at the state."""
    d = v.shape[-1]
    v2 = (v * v).sum(-1)
    a = torch.sqrt(gamma * p / rho)
    H = a * a / (gamma - 1.0) + 0.5 * v2
    vn = (v * n).sum(-1)
    drho = dU[..., 0]
    dm = dU[..., 1:1 + d]
    dE = dU[..., d + 1]
    dv = (dm - v * drho[..., None]) / rho[..., None]
    dp = (gamma - 1.0) * (dE - (v * dm).sum(-1) + 0.5 * v2 * drho)
    dvn = (dv * n).sum(-1)
    am = (dp - rho * a * dvn) / (2.0 * a * a)
    ap = (dp + rho * a * dvn) / (2.0 * a * a)

    def r(sign):
        return torch.cat([torch.ones_like(rho)[..., None], v + sign * a[..., None] * n,
                          (H + sign * a * vn)[..., None]], -1)

    rm_, rp_ = r(-1.0), r(1.0)
    rest = dU - am[..., None] * rm_ - ap[..., None] * rp_
    return (vn.abs()[..., None] * rest + (vn - a).abs()[..., None] * am[..., None] * rm_
            + (vn + a).abs()[..., None] * ap[..., None] * rp_)


def _mean_state(um, up, gamma):
    rm, vm, pm = prim(um, gamma)
    rp, vp, pp = prim(up, gamma)
    return 0.5 * (rm + rp), 0.5 * (vm + vp), 0.5 * (pm + pp)


def interface_flux(um, up, n, gamma, ecflux: int, dissipation: int):
    """f*(U-, U+, n) of eq. (num_flux) with unit normal n.  dissipation:
      0  none (entropy-conservative interface flux);
      1  local Lax-Friedrichs with Davis' wave speed, - lambda/2 (u+ - u-);
      2  scalar dissipation on the jump of the entropy variables,
         - lambda/2 A0(u_mean) (w+ - w-), lambda Davis' wave speed;
      3  matrix dissipation, - 1/2 |A_n(u_mean)| A0(u_mean) (w+ - w-).
    The last two are the alternatives the paper names after eq. (num_flux);
    A0 = dU/dW and |A_n| are symmetric positive semidefinite in product, so
    both are entropy stable.  u_mean: arithmetic means of rho, v, p."""
    f = EC_FLUXES[ecflux](um, up, n, gamma)
    if dissipation == 1:
        lam = rn(davis_speed(um, up, n, gamma))
        f = rn(f - rn(0.5 * lam[..., None] * rn(up - um)))
    elif dissipation in (2, 3):
        dw = entropy_vars(up, gamma) - entropy_vars(um, gamma)
        rho, v, p = _mean_state(um, up, gamma)
        dU = (entropy_jacobian(rho, v, p, gamma) @ dw[..., None])[..., 0]
        if dissipation == 2:
            lam = davis_speed(um, up, n, gamma)
            f = f - 0.5 * lam[..., None] * dU
        else:
            f = f - 0.5 * abs_flux_jacobian_apply(rho, v, p, n, gamma, dU)
    return f
