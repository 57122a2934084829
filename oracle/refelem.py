"""Tensor-product SBP operators in collapsed coordinates and the PKD basis.

Test infrastructure (see the package docstring).  Dense matrices written from:
  * Sec. 3.1, eqs. (tri_mapping, tri_quadrature, tri_facet_quadrature_nodes,
    d_2d, r_2d): reference triangle, LG x LG volume rule, LG facets;
  * Sec. 3.2, eqs. (tet_mapping, tet_quadrature, tet facet nodes/weights,
    d_3d, r_3d): reference tetrahedron, LG x LG x GJ(1,0) volume rule,
    LG x GJ(1,0) facets;
  * Sec. 2.2-2.3: W = diag(w), Q = W D, E = sum_z n_z R^T B R (eq. e_decomp),
    S = Q - E/2;
  * Sec. 4.3, eqs. (principal_functions, modal_basis_2d/3d): orthonormal PKD
    basis and the generalized Vandermonde matrix V (eq. modal_to_nodal).

Readings of the printed text (listed with reasons in the design notes):
  - the first component of the tet collapsed map is taken as
    (1+e1)(1-e2)(1-e3)/4 - 1 (the printed (1-e2)(1-e2) maps outside the tet);
  - the Kronecker factor printed as delta_{a3 a3} in D^(2), D^(3) is delta_{a3 b3}.

Orderings (the paper leaves them free): volume node sigma(a) = a1 + Q a2 + Q^2 a3
(a1 fastest, Q = q+1); facet node a1 + Q a2; modes pi ordered with a1 outermost,
then a2, then a3 innermost.  Facets are numbered as in the paper, 0-based here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from functools import lru_cache

import torch

from .poly1d import DT, gauss_jacobi, jacobi, jacobi_deriv, lagrange, lagrange_deriv


def mode_list(dim: int, p: int):
    out = []
    if dim == 2:
        for a1 in range(p + 1):
            for a2 in range(p + 1 - a1):
                out.append((a1, a2))
    else:
        for a1 in range(p + 1):
            for a2 in range(p + 1 - a1):
                for a3 in range(p + 1 - a1 - a2):
                    out.append((a1, a2, a3))
    return out


# ---------------------------------------------------------------- collapsed maps
def chi(eta: torch.Tensor) -> torch.Tensor:
    """Collapsed map from the square/cube to the reference simplex."""
    if eta.shape[-1] == 2:
        e1, e2 = eta[..., 0], eta[..., 1]
        return torch.stack([0.5 * (1 + e1) * (1 - e2) - 1, e2], -1)
    e1, e2, e3 = eta[..., 0], eta[..., 1], eta[..., 2]
    return torch.stack([0.25 * (1 + e1) * (1 - e2) * (1 - e3) - 1,
                        0.5 * (1 + e2) * (1 - e3) - 1, e3], -1)


def chi_inverse(xi: torch.Tensor) -> torch.Tensor:
    """Inverse collapsed map; at collapsed points the free coordinate is set to -1."""
    xi = torch.as_tensor(xi, dtype=DT)
    if xi.shape[-1] == 2:
        x1, x2 = xi[..., 0], xi[..., 1]
        den = 1 - x2
        ok = den.abs() > 1e-14
        e1 = torch.where(ok, 2 * (1 + x1) / torch.where(ok, den, torch.ones_like(den)) - 1, -torch.ones_like(x1))
        return torch.stack([e1, x2], -1)
    x1, x2, x3 = xi[..., 0], xi[..., 1], xi[..., 2]
    den3 = 1 - x3
    ok3 = den3.abs() > 1e-14
    e2 = torch.where(ok3, 2 * (1 + x2) / torch.where(ok3, den3, torch.ones_like(den3)) - 1, -torch.ones_like(x2))
    den12 = -x2 - x3
    ok12 = den12.abs() > 1e-14
    e1 = torch.where(ok12, 2 * (1 + x1) / torch.where(ok12, den12, torch.ones_like(den12)) - 1, -torch.ones_like(x1))
    return torch.stack([e1, e2, x3], -1)


# ---------------------------------------------------------------- PKD basis
def pkd(dim: int, p: int, xi) -> torch.Tensor:
    """Orthonormal PKD basis phi_j(xi_i) -> [n_points, N_p] (eqs. principal_functions,
    modal_basis_2d/3d), evaluated through the collapsed coordinates."""
    eta = chi_inverse(torch.as_tensor(xi, dtype=DT))
    cols = []
    if dim == 2:
        a, b = eta[..., 0], eta[..., 1]
        for (i, j) in mode_list(2, p):
            psi1 = math.sqrt(2.0) * jacobi(i, 0, 0, a)[i]
            psi2 = (1 - b) ** i * jacobi(j, 2 * i + 1, 0, b)[j]
            cols.append(psi1 * psi2)
    else:
        a, b, c = eta[..., 0], eta[..., 1], eta[..., 2]
        for (i, j, k) in mode_list(3, p):
            psi1 = math.sqrt(2.0) * jacobi(i, 0, 0, a)[i]
            psi2 = (1 - b) ** i * jacobi(j, 2 * i + 1, 0, b)[j]
            psi3 = 2.0 * (1 - c) ** (i + j) * jacobi(k, 2 * i + 2 * j + 2, 0, c)[k]
            cols.append(psi1 * psi2 * psi3)
    return torch.stack(cols, -1)


def _pow(x, n):
    # (x)^n with 0^0 = 1; only non-negative n reach here
    return x ** n if n > 0 else torch.ones_like(x)


def pkd_grad(dim: int, p: int, xi) -> torch.Tensor:
    """Gradient of the PKD basis with respect to xi -> [dim, n_points, N_p].

    Chain rule through the collapsed coordinates, with the factors 1/(1-e2),
    1/(1-e3) absorbed into the polynomial prefactors so that the expression is
    finite (and exact) at the collapsed vertices and edges."""
    eta = chi_inverse(torch.as_tensor(xi, dtype=DT))
    out = []
    if dim == 2:
        a, b = eta[..., 0], eta[..., 1]
        g1, g2 = [], []
        for (i, j) in mode_list(2, p):
            f1 = math.sqrt(2.0) * jacobi(i, 0, 0, a)[i]
            df1 = math.sqrt(2.0) * jacobi_deriv(i, 0, 0, a)[i]
            P = jacobi(j, 2 * i + 1, 0, b)[j]
            dP = jacobi_deriv(j, 2 * i + 1, 0, b)[j]
            if i >= 1:
                bm = _pow(1 - b, i - 1)  # (1-b)^(i-1)
                d_xi1 = 2.0 * df1 * bm * P
                # d/db[(1-b)^i P] = (1-b)^(i-1) [ -i P + (1-b) P' ]
                d_xi2 = df1 * (1 + a) * bm * P + f1 * bm * (-i * P + (1 - b) * dP)
            else:
                d_xi1 = torch.zeros_like(a)
                d_xi2 = f1 * dP
            g1.append(d_xi1)
            g2.append(d_xi2)
        return torch.stack([torch.stack(g1, -1), torch.stack(g2, -1)], 0)
    a, b, c = eta[..., 0], eta[..., 1], eta[..., 2]
    g1, g2, g3 = [], [], []
    for (i, j, k) in mode_list(3, p):
        f1 = math.sqrt(2.0) * jacobi(i, 0, 0, a)[i]
        df1 = math.sqrt(2.0) * jacobi_deriv(i, 0, 0, a)[i]
        P2 = jacobi(j, 2 * i + 1, 0, b)[j]
        dP2 = jacobi_deriv(j, 2 * i + 1, 0, b)[j]
        P3 = jacobi(k, 2 * i + 2 * j + 2, 0, c)[k]
        dP3 = jacobi_deriv(k, 2 * i + 2 * j + 2, 0, c)[k]
        s = i + j
        # psi2 = (1-b)^i P2 ; psi3 = 2 (1-c)^s P3
        psi2 = _pow(1 - b, i) * P2
        psi3 = 2.0 * _pow(1 - c, s) * P3
        # derivative of psi3 w.r.t. c: 2 (1-c)^(s-1) [ -s P3 + (1-c) dP3 ]  (s>=1), 2 dP3 (s=0)
        if s >= 1:
            cm = 2.0 * _pow(1 - c, s - 1) * P3      # psi3 / (1-c)
            dpsi3 = 2.0 * _pow(1 - c, s - 1) * (-s * P3 + (1 - c) * dP3)
        else:
            cm = torch.zeros_like(c)
            dpsi3 = 2.0 * dP3
        if i >= 1:
            bm = _pow(1 - b, i - 1) * P2            # psi2 / (1-b)
            dpsi2 = _pow(1 - b, i - 1) * (-i * P2 + (1 - b) * dP2)
        else:
            bm = torch.zeros_like(b)
            dpsi2 = dP2
        # phi_a/((1-b)(1-c)) = df1 * bm * cm ; phi_b/(1-c) = f1 * dpsi2 * cm
        A = df1 * bm * cm
        Bt = f1 * dpsi2 * cm
        d1 = 4.0 * A
        d2 = 2.0 * (1 + a) * A + 2.0 * Bt
        d3 = 2.0 * (1 + a) * A + (1 + b) * Bt + f1 * psi2 * dpsi3
        g1.append(d1)
        g2.append(d2)
        g3.append(d3)
    return torch.stack([torch.stack(g1, -1), torch.stack(g2, -1), torch.stack(g3, -1)], 0)


# ---------------------------------------------------------------- SBP operators
@dataclass
class RefElement:
    dim: int
    q: int
    p: int
    xi: torch.Tensor          # [Nq, d] volume nodes
    w: torch.Tensor           # [Nq] volume weights
    xi_f: list                # per facet [Nqf, d]
    w_f: list                 # per facet [Nqf]
    nhat: torch.Tensor        # [Nf, d] reference outward normals
    D: list                   # [d] dense [Nq, Nq]
    R: list                   # [Nf] dense [Nqf, Nq]
    Q: list
    E: list
    S: list
    V: torch.Tensor           # [Nq, Np]
    eta1: torch.Tensor        # LG nodes
    eta_gj: torch.Tensor      # GJ(1,0) nodes (tet only)

    @property
    def Nq(self):
        return self.xi.shape[0]

    @property
    def Np(self):
        return self.V.shape[1]

    @property
    def Nf(self):
        return len(self.R)

    @property
    def Nqf(self):
        return self.R[0].shape[0]


@lru_cache(maxsize=None)
def ref_element(dim: int, q: int, p: int | None = None) -> RefElement:
    if p is None:
        p = q
    Qn = q + 1
    x_lg, w_lg = gauss_jacobi(q, 0.0, 0.0)
    x_gj, w_gj = gauss_jacobi(q, 1.0, 0.0)
    I = torch.eye(Qn, dtype=DT)
    dl_lg = lagrange_deriv(x_lg, x_lg)       # [k, j] = l_j'(eta_k)
    dl_gj = lagrange_deriv(x_gj, x_gj)
    lg_m1 = lagrange(x_lg, torch.tensor([-1.0], dtype=DT))[0]
    lg_p1 = lagrange(x_lg, torch.tensor([1.0], dtype=DT))[0]
    gj_m1 = lagrange(x_gj, torch.tensor([-1.0], dtype=DT))[0]
    if dim == 2:
        # node sigma(a) = a1 + Q a2
        A1, A2 = torch.meshgrid(torch.arange(Qn), torch.arange(Qn), indexing="xy")
        a1 = A1.reshape(-1)
        a2 = A2.reshape(-1)
        eta = torch.stack([x_lg[a1], x_lg[a2]], -1)
        xi = chi(eta)
        w = 0.5 * (1 - x_lg[a2]) * w_lg[a1] * w_lg[a2]
        Nq = Qn * Qn
        # dense D^(1), D^(2) of eq. (d_2d), entry (alpha, beta) by broadcasting
        e1 = x_lg[a1][:, None]
        e2 = x_lg[a2][:, None]
        d11 = (a1[:, None] == a1[None, :]).to(DT)
        d22 = (a2[:, None] == a2[None, :]).to(DT)
        dl1 = dl_lg[a1[:, None], a1[None, :]]
        dl2 = dl_lg[a2[:, None], a2[None, :]]
        D1 = 2.0 / (1 - e2) * dl1 * d22
        D2 = (1 + e1) / (1 - e2) * dl1 * d22 + d11 * dl2
        D = [D1, D2]
        # facets (eq. tri_facet_quadrature_nodes, r_2d)
        xi_f = [chi(torch.stack([x_lg, -torch.ones(Qn, dtype=DT)], -1)),
                chi(torch.stack([torch.ones(Qn, dtype=DT), x_lg], -1)),
                chi(torch.stack([-torch.ones(Qn, dtype=DT), x_lg], -1))]
        w_f = [w_lg.clone(), math.sqrt(2.0) * w_lg, w_lg.clone()]
        F = torch.arange(Qn)[:, None]
        B1 = a1[None, :]
        B2 = a2[None, :]
        R1 = I[F, B1] * lg_m1[B2]          # l_b1(eta_f,i) l_b2(-1)
        R2 = lg_p1[B1] * I[F, B2]          # l_b1(1) l_b2(eta_f,i)
        R3 = lg_m1[B1] * I[F, B2]          # l_b1(-1) l_b2(eta_f,i)
        R = [R1, R2, R3]
        nhat = torch.tensor([[0.0, -1.0], [1 / math.sqrt(2.0), 1 / math.sqrt(2.0)], [-1.0, 0.0]], dtype=DT)
    else:
        Nq = Qn ** 3
        idx = torch.arange(Nq)
        a1 = idx % Qn
        a2 = (idx // Qn) % Qn
        a3 = idx // (Qn * Qn)
        eta = torch.stack([x_lg[a1], x_lg[a2], x_gj[a3]], -1)
        xi = chi(eta)
        w = (1 - x_lg[a2]) * (1 - x_gj[a3]) / 8.0 * w_lg[a1] * w_lg[a2] * w_gj[a3]
        # dense D^(1..3) of eq. (d_3d), entry (alpha, beta) by broadcasting
        e1 = x_lg[a1][:, None]
        e2 = x_lg[a2][:, None]
        e3 = x_gj[a3][:, None]
        d1 = (a1[:, None] == a1[None, :]).to(DT)
        d2 = (a2[:, None] == a2[None, :]).to(DT)
        d3 = (a3[:, None] == a3[None, :]).to(DT)
        t1 = dl_lg[a1[:, None], a1[None, :]] * d2 * d3
        t2 = d1 * dl_lg[a2[:, None], a2[None, :]] * d3
        t3 = d1 * d2 * dl_gj[a3[:, None], a3[None, :]]
        D1 = 4.0 / ((1 - e2) * (1 - e3)) * t1
        D2 = 2.0 * (1 + e1) / ((1 - e2) * (1 - e3)) * t1 + 2.0 / (1 - e3) * t2
        D3 = 2.0 * (1 + e1) / ((1 - e2) * (1 - e3)) * t1 + (1 + e2) / (1 - e3) * t2 + t3
        D = [D1, D2, D3]
        Nqf = Qn * Qn
        fidx = torch.arange(Nqf)
        f1 = fidx % Qn
        f2 = fidx // Qn
        ones = torch.ones(Nqf, dtype=DT)
        ef1 = x_lg[f1]
        ef2 = x_gj[f2]
        xi_f = [chi(torch.stack([ef1, -ones, ef2], -1)),
                chi(torch.stack([ones, ef1, ef2], -1)),
                chi(torch.stack([-ones, ef1, ef2], -1)),
                chi(torch.stack([ef1, ef2, -ones], -1))]
        wf = w_lg[f1] * w_gj[f2]
        w_f = [0.5 * wf, math.sqrt(3.0) / 2.0 * wf, 0.5 * wf, 0.5 * wf]
        # eq. r_3d
        l_lg_at_gj = lagrange(x_lg, x_gj)   # [k, j] = l^LG_j(eta^GJ_k)
        F1 = f1[:, None]
        F2 = f2[:, None]
        B1 = a1[None, :]
        B2 = a2[None, :]
        B3 = a3[None, :]
        R = [I[F1, B1] * lg_m1[B2] * I[F2, B3],
             lg_p1[B1] * I[F1, B2] * I[F2, B3],
             lg_m1[B1] * I[F1, B2] * I[F2, B3],
             I[F1, B1] * l_lg_at_gj[F2, B2] * gj_m1[B3]]
        s3 = 1 / math.sqrt(3.0)
        nhat = torch.tensor([[0.0, -1.0, 0.0], [s3, s3, s3], [-1.0, 0.0, 0.0], [0.0, 0.0, -1.0]], dtype=DT)
    W = torch.diag(w)
    Qm = [W @ Dm for Dm in D]
    E = []
    for m in range(dim):
        Em = torch.zeros((xi.shape[0], xi.shape[0]), dtype=DT)
        for z in range(len(R)):
            Em = Em + nhat[z, m] * R[z].T @ torch.diag(w_f[z]) @ R[z]
        E.append(Em)
    S = [Qm[m] - 0.5 * E[m] for m in range(dim)]
    V = pkd(dim, p, xi)
    return RefElement(dim, q, p, xi, w, xi_f, w_f, nhat, D, R, Qm, E, S, V,
                      x_lg, x_gj if dim == 3 else None)


def num_flux_evals(ref: RefElement, tol: float = 1e-13) -> int:
    """Structural count of eq. (num_fluxes): sum_l nnz(S^l)/2 + sum_z nnz(R_z^T B_z),
    counting entries above tol in magnitude."""
    n = 0
    for Sm in ref.S:
        n += int((Sm.abs() > tol).sum().item()) // 2
    for z in range(ref.Nf):
        RtB = ref.R[z].T @ torch.diag(ref.w_f[z])
        n += int((RtB.abs() > tol).sum().item())
    return n
