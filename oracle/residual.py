"""Dense reference residual of the entropy-stable weight-adjusted modal DSEM.

Test infrastructure (see the package docstring).  Each function follows the
paper's equations literally, with dense matrices and all-pairs Hadamard sums:

  u = V u~                                               eq. (modal_to_nodal)
  w~ = Mt^{-1} V^T W J W(u),  Mt^{-1} = M^{-1}V^T W J^{-1} V M^{-1}
                                                         eqs. (entropy_expansion, weight_adjusted_inverse)
  w = V w~,  w^z = R^z w,  u_bar = U(w)                  eqs. (entropy_variables, two_point_flux_*)
  r = - sum_l (2 S^l o sum_m {G_lm} o F^m) 1
      - sum_z ( C^z 1 + R^zT (B^z J^z f*^z - C^zT 1) )   eqs. (entropy_stable, facet_correction)
  du~/dt = Mt^{-1} V^T r                                 eq. (dudt_modal)

and the hybridized form of Theorem (equivalence), eq. (skew_hybridized), as an
independent second formula.  M = V^T W V is formed explicitly.  The state
layout is [element][variable][mode]; a residual can be evaluated for any subset
of elements (their neighbours' entropy projections are computed as needed).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import physics as ph
from .noise import esum, rsum as _rsum, rn as _rn, rn_skew as _rn_skew, rounding_noise  # noqa: F401
from .geometry import Connectivity, Geometry, build_geometry, connectivity
from .poly1d import DT
from .refelem import RefElement, ref_element


@dataclass
class Problem:
    ref: RefElement
    geo: Geometry
    con: Connectivity
    gamma: float
    ecflux: int
    dissipation: int
    Minv: torch.Tensor

    @property
    def ne(self):
        return self.geo.J.shape[0]

    @property
    def nc(self):
        return self.ref.dim + 2


def setup(mesh, degree: int, warp, gamma: float = 1.4, ecflux: int = 0, dissipation: int = 1) -> Problem:
    ref = ref_element(mesh.dim, degree, degree)
    geo = build_geometry(ref, mesh.elem_vertex_ids, mesh.elem_vertex_coords, warp)
    con = connectivity(geo.vids, degree)
    M = ref.V.T @ torch.diag(ref.w) @ ref.V
    return Problem(ref, geo, con, gamma, ecflux, dissipation, torch.linalg.inv(M))


def wadj_inverse(prob: Problem, elems) -> torch.Tensor:
    """Mt^{-1} = M^{-1} V^T W J^{-1} V M^{-1} for the given elements -> [nE, Np, Np]."""
    V, w, Mi = prob.ref.V, prob.ref.w, prob.Minv
    J = prob.geo.J[elems]
    inner = torch.einsum("ki,ek,kj->eij", V, w[None, :] / J, V)
    return Mi[None] @ inner @ Mi[None]


def project(prob: Problem, u_nodal: torch.Tensor, elems=None) -> torch.Tensor:
    """Weight-adjusted L2 projection of nodal values at the volume quadrature
    nodes: u~ = Mt^{-1} V^T W J u -> [nE, Nc, Np]."""
    if elems is None:
        elems = torch.arange(prob.ne)
    elems = torch.as_tensor(elems)
    V, w = prob.ref.V, prob.ref.w
    out = []
    for i in range(0, len(elems), 2048):
        el = elems[i:i + 2048]
        J = prob.geo.J[el]
        b = torch.einsum("ki,ek,ekc->eci", V, w[None, :] * J, u_nodal[i:i + 2048])
        A = wadj_inverse(prob, el)
        out.append(torch.einsum("eij,ecj->eci", A, b))
    return torch.cat(out, 0)


def entropy_projection(prob: Problem, ut: torch.Tensor, elems) -> torch.Tensor:
    """w~ of eq. (entropy_expansion) for the given elements -> [nE, Nc, Np]."""
    V, w = prob.ref.V, prob.ref.w
    u = _rn(esum("ki,eci->ekc", _rn(V), _rn(ut[elems])))
    W = _rn(ph.entropy_vars(u, prob.gamma))
    J = prob.geo.J[elems]
    b = _rn(esum("ki,ekc->eci", _rn(V), _rn(w[None, :, None] * J[..., None]) * W))
    A = _rn(wadj_inverse(prob, elems))
    return _rn(esum("eij,ecj->eci", A, b))


def _pair_fluxes(prob: Problem, ua: torch.Tensor, ub: torch.Tensor) -> torch.Tensor:
    """F^m_ij = f#_m(ua_i, ub_j) for every pair -> [nE, Na, Nb, Nc, d]."""
    d = prob.ref.dim
    flux = ph.EC_FLUXES[prob.ecflux]
    A = ua[:, :, None, :].expand(-1, -1, ub.shape[1], -1)
    B = ub[:, None, :, :].expand(-1, ua.shape[1], -1, -1)
    out = []
    for m in range(d):
        n = torch.zeros(A.shape[:-1] + (d,), dtype=DT)
        n[..., m] = 1.0
        out.append(_rn(flux(A, B, n, prob.gamma)))
    return torch.stack(out, -1)


def _facet_states(prob: Problem, wt_all: torch.Tensor, idx_of: dict, elems, exterior=None):
    """Own facet entropy-projected states and exterior states for each facet.
    exterior(elems, z, ext_z) may replace the exterior states of facet z (used
    for neighbours of another degree)."""
    ref, con = prob.ref, prob.con
    own, ext = [], []
    for z in range(ref.Nf):
        wv = _rn(esum("ki,eci->ekc", _rn(ref.V), wt_all[[idx_of[int(e)] for e in elems]]))
        wz = _rn(esum("jk,ekc->ejc", _rn(ref.R[z]), wv))
        own.append(_rn(ph.cons_from_entropy(wz, prob.gamma)))
        nb = con.nbr_elem[elems, z]
        nz = con.nbr_face[elems, z]
        wt_nb = wt_all[[idx_of[int(e)] for e in nb]]
        wv_nb = _rn(esum("ki,eci->ekc", _rn(ref.V), wt_nb))
        wp = torch.stack([esum("jk,kc->jc", _rn(ref.R[int(nz[i])]), wv_nb[i]) for i in range(len(elems))])  # [nE, Nqf, Nc]
        perm = torch.as_tensor(con.node_map[elems, z])
        wp = _rn(torch.gather(wp, 1, perm[:, :, None].expand(-1, -1, wp.shape[-1])))
        ext_z = _rn(ph.cons_from_entropy(wp, prob.gamma))
        ext.append(ext_z if exterior is None else exterior(elems, z, ext_z))
    return own, ext


def _neighbourhood(prob: Problem, elems):
    elems = np.asarray(elems, dtype=np.int64).reshape(-1)
    need = np.unique(np.concatenate([elems, prob.con.nbr_elem[elems].reshape(-1)]))
    return elems, need


def residual_nodal(prob: Problem, ut: torch.Tensor, elems=None, exterior=None):
    """Nodal right-hand side r of eq. (entropy_stable) for the given elements.
    Returns (r [nE, Nq, Nc], w [nE, Nq, Nc]).  exterior: see _facet_states."""
    ref, geo = prob.ref, prob.geo
    d, g = ref.dim, prob.gamma
    if elems is None:
        elems = np.arange(prob.ne)
    elems, need = _neighbourhood(prob, elems)
    wt_need = entropy_projection(prob, ut, torch.as_tensor(need))
    idx_of = {int(e): i for i, e in enumerate(need)}
    wt = wt_need[[idx_of[int(e)] for e in elems]]
    w = _rn(esum("ki,eci->ekc", _rn(ref.V), wt))
    ubar = _rn(ph.cons_from_entropy(w, g))
    G = _rn(geo.G[elems])                              # [nE, Nq, l, m]
    # volume term: - sum_l (2 S^l o sum_m {G_lm} o F^m) 1
    F = _pair_fluxes(prob, ubar, ubar)                 # [nE, Nq, Nq, Nc, m]
    r = torch.zeros_like(ubar)
    for l in range(d):
        Gavg = 0.5 * (G[:, :, None, l, :] + G[:, None, :, l, :])     # [nE, i, j, m]
        H = _rn(esum("eijm,eijcm->eijc", Gavg, F))
        r = _rn(r - esum("ij,eijc->eic", 2.0 * _rn_skew(ref.S[l]), H))
    del F
    own, ext = _facet_states(prob, wt_need, idx_of, elems, exterior)
    for z in range(ref.Nf):
        uf = own[z]
        # facet correction C^z = R^T B o sum_m {J n_m} o F^{z,m}
        Fz = _pair_fluxes(prob, ubar, uf)              # [nE, Nq, Nqf, Nc, m]
        nh = ref.nhat[z]
        GnV = torch.einsum("l,eilm->eim", nh, G)                  # G(xi_i)^T nhat
        GnF = _rn(geo.nJ[z][elems])                               # G(xi_j^z)^T nhat
        avg = 0.5 * (GnV[:, :, None, :] + GnF[:, None, :, :])     # [nE, i, j, m]
        RtB = _rn(ref.R[z].T @ torch.diag(ref.w_f[z]))            # [Nq, Nqf]
        C = _rn(RtB[None, :, :, None] * esum("eijm,eijcm->eijc", avg, Fz))
        C1 = _rsum(C, 2)
        Ct1 = _rsum(C, 1)
        fstar = _rn(ph.interface_flux(uf, ext[z], _rn(geo.n[z][elems]), g, prob.ecflux, prob.dissipation))
        s = _rn(_rn(ref.w_f[z][None, :, None] * geo.Jf[z][elems][..., None]) * fstar - Ct1)
        r = _rn(_rn(r - C1) - esum("ji,ejc->eic", _rn(ref.R[z]), s))
    return _rn(r), w


def residual(prob: Problem, ut: torch.Tensor, elems=None, exterior=None) -> torch.Tensor:
    """du~/dt = Mt^{-1} V^T r for the given elements -> [nE, Nc, Np]."""
    if elems is None:
        elems = np.arange(prob.ne)
    elems = np.asarray(elems, dtype=np.int64).reshape(-1)
    r, _ = residual_nodal(prob, ut, elems, exterior)
    A = _rn(wadj_inverse(prob, torch.as_tensor(elems)))
    b = _rn(esum("ki,ekc->eci", _rn(prob.ref.V), r))
    return _rn(esum("eij,ecj->eci", A, b))


def residual_chunked(prob: Problem, ut: torch.Tensor, elems=None, chunk: int = 64) -> torch.Tensor:
    if elems is None:
        elems = np.arange(prob.ne)
    elems = np.asarray(elems, dtype=np.int64).reshape(-1)
    outs = [residual(prob, ut, elems[i:i + chunk]) for i in range(0, len(elems), chunk)]
    return torch.cat(outs, 0)


def residual_hybridized(prob: Problem, ut: torch.Tensor, elems=None) -> torch.Tensor:
    """du~/dt from eq. (skew_hybridized): hybridized SBP operators Qbar^l
    (eq. q_hybridized), split-form physical operators (eq. phys_hybridized),
    block two-point flux matrices over volume and facet nodes (eq. flux_hybridized)."""
    ref, geo = prob.ref, prob.geo
    d, g = ref.dim, prob.gamma
    if elems is None:
        elems = np.arange(prob.ne)
    elems, need = _neighbourhood(prob, elems)
    wt_need = entropy_projection(prob, ut, torch.as_tensor(need))
    idx_of = {int(e): i for i, e in enumerate(need)}
    wt = wt_need[[idx_of[int(e)] for e in elems]]
    w = torch.einsum("ki,eci->ekc", ref.V, wt)
    ubar = ph.cons_from_entropy(w, g)
    own, ext = _facet_states(prob, wt_need, idx_of, elems)
    Nq, Nf = ref.Nq, ref.Nf
    sizes = [Nq] + [ref.R[z].shape[0] for z in range(Nf)]
    off = np.cumsum([0] + sizes)
    Nb = int(off[-1])
    Qbar = []
    for l in range(d):
        Qb = torch.zeros((Nb, Nb), dtype=DT)
        Qb[:Nq, :Nq] = ref.S[l]
        for z in range(Nf):
            a, b = int(off[z + 1]), int(off[z + 2])
            B = torch.diag(ref.w_f[z])
            nl = ref.nhat[z, l]
            Qb[:Nq, a:b] = 0.5 * nl * ref.R[z].T @ B
            Qb[a:b, :Nq] = -0.5 * nl * B @ ref.R[z]
            Qb[a:b, a:b] = 0.5 * nl * B
        Qbar.append(Qb)
    Gbar = torch.cat([geo.G[elems]] + [geo.Gf[z][elems] for z in range(Nf)], 1)   # [nE, Nb, l, m]
    ub = torch.cat([ubar] + own, 1)                                                # [nE, Nb, Nc]
    F = _pair_fluxes(prob, ub, ub)                                                 # [nE, Nb, Nb, Nc, m]
    Vbig = torch.cat([ref.V] + [ref.R[z] @ ref.V for z in range(Nf)], 0)           # [Nb, Np]
    rhs = torch.zeros((len(elems), ref.Np, d + 2), dtype=DT)
    for m in range(d):
        Qkm = torch.zeros((len(elems), Nb, Nb), dtype=DT)
        for l in range(d):
            Gavg = 0.5 * (Gbar[:, :, None, l, m] + Gbar[:, None, :, l, m])
            Qkm = Qkm + Qbar[l][None] * Gavg
        vol = torch.einsum("eij,eijc->eic", 2.0 * Qkm, F[..., m])
        rhs = rhs - torch.einsum("ik,eic->ekc", Vbig, vol)
    for z in range(Nf):
        fstar = ph.interface_flux(own[z], ext[z], geo.n[z][elems], g, prob.ecflux, prob.dissipation)
        fm = sum(geo.n[z][elems][..., m:m + 1] * _cart_flux(own[z], m, g) for m in range(d))
        s = (ref.w_f[z][None, :, None] * geo.Jf[z][elems][..., None]) * (fstar - fm)
        rhs = rhs - torch.einsum("jk,ejc->ekc", ref.R[z] @ ref.V, s)
    A = wadj_inverse(prob, torch.as_tensor(elems))
    return torch.einsum("eij,ejc->eci", A, rhs)


def _cart_flux(u, m, g):
    d = u.shape[-1] - 2
    n = torch.zeros(u.shape[:-1] + (d,), dtype=DT)
    n[..., m] = 1.0
    return ph.euler_flux(u, n, g)


def rk4(prob: Problem, ut: torch.Tensor, dt: float, nsteps: int, chunk: int = 64) -> torch.Tensor:
    """Classical four-stage Runge-Kutta."""
    u = ut.clone()
    for _ in range(nsteps):
        k1 = residual_chunked(prob, u, chunk=chunk)
        k2 = residual_chunked(prob, u + 0.5 * dt * k1, chunk=chunk)
        k3 = residual_chunked(prob, u + 0.5 * dt * k2, chunk=chunk)
        k4 = residual_chunked(prob, u + dt * k3, chunk=chunk)
        u = u + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return u


def vjp(prob: Problem, ut: torch.Tensor, vbar: torch.Tensor, elems=None) -> torch.Tensor:
    """(dR/du~)^T vbar by reverse-mode autodiff of the dense residual.  If elems
    is given, only those rows of the gradient are returned (the residual is
    evaluated on their 1-ring, which holds every dependence)."""
    if elems is None:
        x = ut.detach().clone().requires_grad_(True)
        R = residual_chunked(prob, x)
        (gr,) = torch.autograd.grad((R * vbar).sum(), x)
        return gr
    elems = np.asarray(elems, dtype=np.int64).reshape(-1)
    ring = np.unique(np.concatenate([elems, prob.con.nbr_elem[elems].reshape(-1)]))
    x = ut.detach().clone().requires_grad_(True)
    R = residual(prob, x, ring)
    (gr,) = torch.autograd.grad((R * vbar[ring]).sum(), x)
    return gr[elems]


# ---------------------------------------------------------------- diagnostics
def conserved_integrals(prob: Problem, ut: torch.Tensor) -> torch.Tensor:
    """sum_k 1^T W J u per variable (Theorem conservation)."""
    u = torch.einsum("ki,eci->ekc", prob.ref.V, ut)
    return torch.einsum("k,ek,ekc->c", prob.ref.w, prob.geo.J, u)


def entropy_rate(prob: Problem, ut: torch.Tensor, dudt: torch.Tensor) -> torch.Tensor:
    """d/dt sum_k 1^T W J S(u) = sum_k (W J W(u))^T V du~/dt."""
    V, w = prob.ref.V, prob.ref.w
    u = torch.einsum("ki,eci->ekc", V, ut)
    Wu = ph.entropy_vars(u, prob.gamma)
    du = torch.einsum("ki,eci->ekc", V, dudt)
    return torch.einsum("k,ek,ekc,ekc->", w, prob.geo.J, Wu, du)


# ---------------------------------------------------------------- alternative forms
def _nodal_states(prob: Problem, ut: torch.Tensor, elems):
    """u = V u~ at the volume nodes of elems, u^z = R^z u at their facet nodes
    and the exterior states (the neighbours' facet values at the matched
    nodes), without any entropy projection."""
    ref, con = prob.ref, prob.con
    elems, need = _neighbourhood(prob, elems)
    idx_of = {int(e): i for i, e in enumerate(need)}
    u_need = torch.einsum("ki,eci->ekc", ref.V, ut[torch.as_tensor(need)])
    u = u_need[[idx_of[int(e)] for e in elems]]
    own, ext = [], []
    for z in range(ref.Nf):
        own.append(torch.einsum("jk,ekc->ejc", ref.R[z], u))
        nb, nz = con.nbr_elem[elems, z], con.nbr_face[elems, z]
        wp = torch.stack([ref.R[int(nz[i])] @ u_need[idx_of[int(nb[i])]] for i in range(len(elems))])
        perm = torch.as_tensor(con.node_map[elems, z])
        ext.append(torch.gather(wp, 1, perm[:, :, None].expand(-1, -1, wp.shape[-1])))
    return elems, u, own, ext


def _cart_fluxes(u, g):
    """[..., Nc, d]: the Cartesian Euler fluxes f_m(u)."""
    d = u.shape[-1] - 2
    return torch.stack([_cart_flux(u, m, g) for m in range(d)], -1)


def residual_conservative(prob: Problem, ut: torch.Tensor, elems=None) -> torch.Tensor:
    """du~/dt of the standard (conservative) weak form eq. (rhs_cons):
    r = sum_l Q^lT sum_m G^(l,m) f^m - sum_z R^zT B^z J^z f*^z, with u = V u~
    at the volume nodes and u^z = R^z u at the facet nodes (no entropy
    projection), then the weight-adjusted inverse."""
    ref, geo = prob.ref, prob.geo
    d, g = ref.dim, prob.gamma
    if elems is None:
        elems = np.arange(prob.ne)
    elems, u, own, ext = _nodal_states(prob, ut, elems)
    f = _cart_fluxes(u, g)                                      # [nE, Nq, Nc, m]
    G = geo.G[elems]                                            # [nE, Nq, l, m]
    r = torch.zeros_like(u)
    for l in range(d):
        Gf = torch.einsum("eim,eicm->eic", G[:, :, l, :], f)
        r = r + torch.einsum("ji,ejc->eic", ref.Q[l], Gf)
    for z in range(ref.Nf):
        fstar = ph.interface_flux(own[z], ext[z], geo.n[z][elems], g, prob.ecflux, prob.dissipation)
        s = (ref.w_f[z][None, :, None] * geo.Jf[z][elems][..., None]) * fstar
        r = r - torch.einsum("ji,ejc->eic", ref.R[z], s)
    A = wadj_inverse(prob, torch.as_tensor(elems))
    return torch.einsum("eij,ecj->eci", A, torch.einsum("ki,ekc->eci", ref.V, r))


def residual_skew(prob: Problem, ut: torch.Tensor, elems=None) -> torch.Tensor:
    """du~/dt of the skew-symmetric weak form eq. (rhs_skew):
    r = 1/2 sum_l (Q^lT sum_m G^(l,m) f^m - sum_m G^(l,m) Q^l f^m)
        - sum_z R^zT B^z J^z (f*^z - 1/2 sum_m N^(z,m) R^z f^m),
    u = V u~ at the volume nodes, u^z = R^z u (no entropy projection)."""
    ref, geo = prob.ref, prob.geo
    d, g = ref.dim, prob.gamma
    if elems is None:
        elems = np.arange(prob.ne)
    elems, u, own, ext = _nodal_states(prob, ut, elems)
    f = _cart_fluxes(u, g)                                      # [nE, Nq, Nc, m]
    G = geo.G[elems]
    r = torch.zeros_like(u)
    for l in range(d):
        Gf = torch.einsum("eim,eicm->eic", G[:, :, l, :], f)
        Qf = torch.einsum("ij,ejcm->eicm", ref.Q[l], f)
        r = r + 0.5 * (torch.einsum("ji,ejc->eic", ref.Q[l], Gf) - torch.einsum("eim,eicm->eic", G[:, :, l, :], Qf))
    for z in range(ref.Nf):
        fstar = ph.interface_flux(own[z], ext[z], geo.n[z][elems], g, prob.ecflux, prob.dissipation)
        Rf = torch.einsum("jk,ekcm->ejcm", ref.R[z], f)
        Nf = torch.einsum("ejm,ejcm->ejc", geo.n[z][elems], Rf)
        s = (ref.w_f[z][None, :, None] * geo.Jf[z][elems][..., None]) * (fstar - 0.5 * Nf)
        r = r - torch.einsum("ji,ejc->eic", ref.R[z], s)
    A = wadj_inverse(prob, torch.as_tensor(elems))
    return torch.einsum("eij,ecj->eci", A, torch.einsum("ki,ekc->eci", ref.V, r))
