"""Mesh orientation, isoparametric mapping, metric terms and connectivity.

Test infrastructure (see the package docstring).  Written from:
  * Sec. 4.1, eq. (poly_mapping): x(xi) = sum_i x_i l_i(xi) of degree p_g = p,
    J = det(grad x) > 0 (eq. jacobian_positive), G = J (grad x)^{-1};
  * Sec. 4.2: exact metrics in 2D; in 3D the conservative curl form
    (eqs. metric_interpolants, conservative_curl) with degree q+1 interpolants;
    Nanson normals and facet Jacobians (eq. nanson);
  * Sec. 4.5, eq. (jacobian_approx): J interpolated with degree p_g at the
    mapping nodes, used in the mass matrix and entropy projection;
  * Sec. 7.3 and Remark (connectivity): split-Cartesian meshes with local
    orientation chosen so that facet quadrature nodes of neighbours coincide;
  * Assumption (conformal): matching facet nodes across every interface.

Readings (listed in the design notes): mapping and curl-interpolation nodes are
equispaced simplex nodes, whose Lagrange basis has a closed product form in
barycentric coordinates; the curl-form columns give G_{l m} for m = 1, 2, 3
(so that G equals the adjugate for affine maps); element-local coordinates
(physical minus the element's first vertex) are used and only the warp
displacement is interpolated (interpolation reproduces the affine part), which
leaves G and J unchanged; orientation puts the largest global vertex id at local vertex d+1
and (in 3D) the second largest at local vertex 3, the other two in increasing
id order, swapped if the affine Jacobian is negative.
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import numpy as np
import torch

from .noise import rn
from .poly1d import DT
from .refelem import RefElement, pkd, pkd_grad


# ------------------------------------------------------------------ nodes
@lru_cache(maxsize=None)
def equispaced(dim: int, N: int) -> torch.Tensor:
    pts = []
    if dim == 2:
        for j in range(N + 1):
            for i in range(N + 1 - j):
                pts.append((-1 + 2 * i / N, -1 + 2 * j / N))
    else:
        for k in range(N + 1):
            for j in range(N + 1 - k):
                for i in range(N + 1 - j - k):
                    pts.append((-1 + 2 * i / N, -1 + 2 * j / N, -1 + 2 * k / N))
    return torch.tensor(pts, dtype=DT)


def lattice_multi_indices(dim: int, N: int) -> torch.Tensor:
    """Barycentric integer coordinates alpha (sum N) of the equispaced nodes, in
    the order of equispaced(): alpha_k = N lambda_k, lambda_{k>=1} = (1+xi_k)/2."""
    X = equispaced(dim, N)
    lam = 0.5 * (1 + X)
    lam0 = 1 - lam.sum(-1, keepdim=True)
    return torch.round(N * torch.cat([lam0, lam], -1)).to(torch.int64)


def lagrange_matrices(dim: int, N: int, X: torch.Tensor):
    """Interpolation matrix L[k, i] = l_i(X_k) and gradients dL[m][k, i] for the
    degree-N Lagrange basis on equispaced nodes, from the closed-form product
    formula l_a(lambda) = prod_k prod_{j<a_k} (N lambda_k - j)/(a_k - j)
    (barycentric coordinates; no linear solve)."""
    X = torch.as_tensor(X, dtype=DT)
    A = lattice_multi_indices(dim, N)                       # [Nn, d+1]
    lam = 0.5 * (1 + X)
    lam = torch.cat([1 - lam.sum(-1, keepdim=True), lam], -1)   # [npts, d+1]
    npts, nn = X.shape[0], A.shape[0]
    fac = torch.ones((dim + 1, npts, nn), dtype=DT)          # per barycentric coordinate factor
    dfac = torch.zeros((dim + 1, npts, nn), dtype=DT)        # its derivative w.r.t. lambda_k
    for k in range(dim + 1):
        ak = A[:, k]
        t = N * lam[:, k:k + 1]                               # [npts, 1]
        for j in range(N):
            on = (ak > j)[None, :]                            # factor present for this node
            f = torch.where(on, (t - j) / torch.where(on, (ak - j).to(DT), torch.ones(1, dtype=DT)), torch.ones(1, dtype=DT))
            df = torch.where(on, N / torch.where(on, (ak - j).to(DT), torch.ones(1, dtype=DT)), torch.zeros(1, dtype=DT))
            dfac[k] = dfac[k] * f + fac[k] * df
            fac[k] = fac[k] * f
    L = torch.prod(fac, 0)
    dl = []                                                  # d l / d lambda_k
    for k in range(dim + 1):
        others = torch.ones((npts, nn), dtype=DT)
        for kk in range(dim + 1):
            if kk != k:
                others = others * fac[kk]
        dl.append(dfac[k] * others)
    # lambda_0 = 1 - sum lambda_m, lambda_m = (1+xi_m)/2  ->  d/dxi_m = (dl_m - dl_0)/2
    dL = [0.5 * (dl[m + 1] - dl[0]) for m in range(dim)]
    return L, dL


# ------------------------------------------------------------------ orientation
def reference_vertices(dim: int) -> torch.Tensor:
    if dim == 2:
        return torch.tensor([[-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]], dtype=DT)
    return torch.tensor([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]], dtype=DT)


def orient(elem_ids: np.ndarray, elem_x: np.ndarray):
    """Local vertex order: last vertex = largest global id; in 3D local vertex 3 =
    second largest; the remaining two by increasing id, swapped if det < 0."""
    ne, nv = elem_ids.shape
    dim = nv - 1
    ids_out = np.empty_like(elem_ids)
    x_out = np.empty_like(elem_x)
    for e in range(ne):
        order = list(np.argsort(elem_ids[e], kind="stable"))  # increasing id
        # increasing: [o0, o1, (o2), top]
        loc = order  # v1, v2, (v3), v_{d+1} in increasing order already puts max last
        X = elem_x[e][loc]
        A = (X[1:] - X[0]).T
        if np.linalg.det(A) < 0:
            loc = [loc[1], loc[0]] + loc[2:]
        ids_out[e] = elem_ids[e][loc]
        x_out[e] = elem_x[e][loc]
    return ids_out, x_out


# ------------------------------------------------------------------ geometry
@dataclass
class Geometry:
    dim: int
    p: int
    q: int
    vids: np.ndarray          # oriented global vertex ids [Ne, d+1]
    vx: np.ndarray            # oriented vertex coords [Ne, d+1, d]
    x_vol: torch.Tensor       # physical coords of volume nodes [Ne, Nq, d]
    J: torch.Tensor           # interpolated Jacobian at volume nodes [Ne, Nq]
    G: torch.Tensor           # metric terms at volume nodes [Ne, Nq, d(l), d(m)]
    Gf: list                  # per facet: metric terms at facet nodes [Ne, Nqf, d, d]
    nJ: list                  # per facet: G^T nhat at facet nodes [Ne, Nqf, d]
    Jf: list                  # per facet: |G^T nhat| [Ne, Nqf]
    n: list                   # per facet: unit normal [Ne, Nqf, d]
    x_f: list                 # per facet: physical coords [Ne, Nqf, d]
    J_exact: torch.Tensor     # det(grad x) at volume nodes (diagnostics only)


def build_geometry(ref: RefElement, elem_ids: np.ndarray, elem_x: np.ndarray, warp) -> Geometry:
    dim, p, q = ref.dim, ref.p, ref.q
    vids, vx = orient(np.asarray(elem_ids), np.asarray(elem_x, dtype=np.float64))
    ne = vids.shape[0]
    # affine image of the mapping nodes and the warp displacement delta there.
    # x_h = X_aff + I[delta]: interpolation reproduces the affine part exactly,
    # so only the displacement is interpolated; coordinates are element-local
    # (relative to the first vertex), which leaves G and J unchanged.
    Xm = equispaced(dim, p)                             # mapping nodes (degree p_g = p)
    lam = _barycentric(dim, Xm)                         # [Ng, d+1]
    x_aff = np.einsum("gk,ekd->egd", lam.numpy(), vx)   # [Ne, Ng, d]
    x_map = warp(x_aff.reshape(-1, dim)).reshape(ne, -1, dim)
    dlt = rn(torch.tensor(x_map - x_aff, dtype=DT))     # [Ne, Ng, d]
    origin = vx[:, 0, :]
    org = torch.tensor(origin, dtype=DT)
    Aff = torch.tensor(0.5 * (vx[:, 1:, :] - vx[:, :1, :]).transpose(0, 2, 1), dtype=DT)   # [Ne, c, m] = dX_c/dxi_m

    def X_aff(X):                                       # local affine coordinates at reference points
        return torch.einsum("ecm,km->ekc", Aff, 1 + X)

    def grad_x(X):
        L, dL = lagrange_matrices(dim, p, X)
        xv = X_aff(X) + torch.einsum("ki,eid->ekd", L, dlt)
        gd = rn(torch.stack([torch.einsum("ki,eic->ekc", rn(dL[m]), dlt) for m in range(dim)], -1))  # [Ne,k,c,m]
        return xv, gd                                   # gradient of the displacement only

    # interpolated Jacobian (eq. jacobian_approx)
    _, gd_map = grad_x(Xm)
    Jmap = rn(torch.linalg.det(rn(Aff[:, None] + gd_map)))
    Lvol, _ = lagrange_matrices(dim, p, ref.xi)
    J = rn(torch.einsum("ki,ei->ek", rn(Lvol), Jmap))

    def cross(a, b):
        return torch.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                            a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                            a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], -1)

    def metrics(X):
        xv, gd = grad_x(X)
        gx = rn(Aff[:, None] + gd)
        if dim == 2:
            G = torch.empty(gx.shape, dtype=DT)
            G[..., 0, 0] = gx[..., 1, 1]
            G[..., 0, 1] = -gx[..., 0, 1]
            G[..., 1, 0] = -gx[..., 1, 0]
            G[..., 1, 1] = gx[..., 0, 0]
            return xv, G
        # conservative curl form with degree q+1 interpolants, x = X + delta:
        # x3 grad x2 = X3 grad X2 + (X3 grad d2 + d3 grad X2 + d3 grad d2); the
        # first term is linear (interpolated exactly) with curl grad X3 x grad X2
        Xc = equispaced(3, q + 1)
        Lc, dLc_ = lagrange_matrices(3, p, Xc)
        Xa = X_aff(Xc)                                                    # [Ne, Nc, 3]
        dc = rn(torch.einsum("ki,eid->ekd", rn(Lc), dlt))                 # delta at curl nodes
        gdc = rn(torch.stack([torch.einsum("ki,eic->ekc", rn(dLc_[m]), dlt) for m in range(3)], -1))  # [Ne,Nc,c,m]
        a = [Aff[:, None, c, :] for c in range(3)]                        # grad X_c (constant rows)

        def rvec(c1, c2):     # x_c1 grad x_c2 minus its affine-affine part
            return rn(Xa[..., c1:c1 + 1] * gdc[..., c2, :] + dc[..., c1:c1 + 1] * a[c2] + dc[..., c1:c1 + 1] * gdc[..., c2, :])

        r1, r2, r3 = rvec(2, 1), rvec(2, 0), rvec(0, 1)
        _, dLc = lagrange_matrices(3, q + 1, X)

        def curl(r):
            dr = [rn(torch.einsum("ki,eic->ekc", rn(dLc[m]), r)) for m in range(3)]  # dr[m][..., c] = d r_c / d xi_m
            return torch.stack([dr[1][..., 2] - dr[2][..., 1],
                                dr[2][..., 0] - dr[0][..., 2],
                                dr[0][..., 1] - dr[1][..., 0]], -1)

        npt = X.shape[0]
        c1 = -(cross(a[2], a[1]).expand(-1, npt, -1) + curl(r1))
        c2 = cross(a[2], a[0]).expand(-1, npt, -1) + curl(r2)
        c3 = cross(a[0], a[1]).expand(-1, npt, -1) + curl(r3)
        G = rn(torch.stack([c1, c2, c3], -1))    # G[..., l, m]: column m from the m-th curl
        return xv, G

    xv, G = metrics(ref.xi)
    x_vol = xv + org[:, None, :]
    _, gd_vol = grad_x(ref.xi)
    J_exact = torch.linalg.det(Aff[:, None] + gd_vol)
    Gf, nJ, Jf, nn, xf = [], [], [], [], []
    for z in range(ref.Nf):
        xfz, Gz = metrics(ref.xi_f[z])
        v = rn(torch.einsum("l,ekl m->ekm".replace(" ", ""), ref.nhat[z], Gz))
        jf = rn(torch.linalg.norm(v, dim=-1))
        Gf.append(Gz)
        nJ.append(v)
        Jf.append(jf)
        nn.append(rn(v / jf[..., None]))
        xf.append(xfz + org[:, None, :])
    return Geometry(dim, p, q, vids, vx, x_vol, J, G, Gf, nJ, Jf, nn, xf, J_exact)


def _barycentric(dim: int, xi: torch.Tensor) -> torch.Tensor:
    if dim == 2:
        l2 = 0.5 * (1 + xi[:, 0])
        l3 = 0.5 * (1 + xi[:, 1])
        return torch.stack([1 - l2 - l3, l2, l3], -1)
    l2 = 0.5 * (1 + xi[:, 0])
    l3 = 0.5 * (1 + xi[:, 1])
    l4 = 0.5 * (1 + xi[:, 2])
    return torch.stack([1 - l2 - l3 - l4, l2, l3, l4], -1)


# ------------------------------------------------------------------ connectivity
# local facets: (vertex tuple, base start vertex); vertex indices are local 0-based
FACETS = {
    2: [((0, 1), 0), ((1, 2), 1), ((0, 2), 0)],
    3: [((0, 1, 3), 0), ((1, 2, 3), 1), ((0, 2, 3), 0), ((0, 1, 2), 0)],
}


@dataclass
class Connectivity:
    nbr_elem: np.ndarray   # [Ne, Nf]
    nbr_face: np.ndarray   # [Ne, Nf]
    flip: np.ndarray       # [Ne, Nf] bool: LG facet coordinate reversed on the neighbour
    node_map: np.ndarray   # [Ne, Nf, Nqf] index of the matching node on the neighbour facet


def connectivity(vids: np.ndarray, q: int) -> Connectivity:
    ne, nv = vids.shape
    dim = nv - 1
    faces = FACETS[dim]
    nf = len(faces)
    Qn = q + 1
    table = {}
    for e in range(ne):
        for z, (verts, _) in enumerate(faces):
            key = tuple(sorted(int(vids[e, v]) for v in verts))
            table.setdefault(key, []).append((e, z))
    nbr_elem = np.full((ne, nf), -1, dtype=np.int64)
    nbr_face = np.full((ne, nf), -1, dtype=np.int64)
    flip = np.zeros((ne, nf), dtype=bool)
    nqf = Qn if dim == 2 else Qn * Qn
    node_map = np.zeros((ne, nf, nqf), dtype=np.int64)
    for key, lst in table.items():
        if len(lst) != 2:
            raise ValueError(f"non-conforming facet {key}: {lst}")
        (e0, z0), (e1, z1) = lst
        for (ea, za), (eb, zb) in (((e0, z0), (e1, z1)), ((e1, z1), (e0, z0))):
            nbr_elem[ea, za] = eb
            nbr_face[ea, za] = zb
            sa = int(vids[ea, faces[za][1]])
            sb = int(vids[eb, faces[zb][1]])
            if dim == 3:
                apex_a = int(vids[ea, faces[za][0][2]])
                apex_b = int(vids[eb, faces[zb][0][2]])
                if apex_a != apex_b:
                    raise ValueError("facet collapse vertices differ; orientation failed")
            fl = sa != sb
            flip[ea, za] = fl
            for j in range(nqf):
                a1, a2 = j % Qn, j // Qn
                b1 = (Qn - 1 - a1) if fl else a1
                node_map[ea, za, j] = b1 + Qn * a2
    return Connectivity(nbr_elem, nbr_face, flip, node_map)
