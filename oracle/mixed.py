"""Residual on meshes whose elements carry different polynomial degrees.

Test infrastructure (see the package docstring).  The paper assumes conforming
facets of equal degree (Assumption conformal).  Reading for elements of
different degree: every element uses the operators and geometry of its own
degree (p = q = p_g); the exterior state at a facet node j of element e is the
neighbour's modal entropy expansion evaluated at the neighbour's reference
point of j,

    w+_j = sum_k w~^(nu)_k phi_k(xi^(nu)_j),

where xi^(nu)_j is obtained by carrying j's reference point through e's affine
(vertex) map and back through the neighbour's affine map (with the periodic
shift of the shared face).  For equal degrees this is exactly the conforming
rule (R V w~ is exact on P_p, and the facet nodes coincide).  The rule is not
conservative or entropy-stable across a change of degree.

Elements are held per degree: ut[p] is a [Ne, Nc, Np(p)] tensor over the whole
mesh of which only the rows of elements of degree p are used.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import physics as ph
from . import residual as R
from .poly1d import DT
from .refelem import pkd


@dataclass
class MixedProblem:
    dim: int
    degrees: np.ndarray           # [Ne]
    probs: dict                   # degree -> residual.Problem on the whole mesh
    gamma: float
    L: float                      # periodic box length

    @property
    def ne(self):
        return int(self.degrees.shape[0])


def setup(mesh, degrees, warp, gamma: float = 1.4, ecflux: int = 0, dissipation: int = 1) -> MixedProblem:
    degrees = np.asarray(degrees, dtype=np.int64)
    probs = {int(p): R.setup(mesh, int(p), warp, gamma, ecflux, dissipation) for p in np.unique(degrees)}
    return MixedProblem(mesh.dim, degrees, probs, gamma, float(mesh.box[0]))


def project(mp: MixedProblem, state) -> dict:
    """Weight-adjusted projection of state(x) for every degree -> {p: ut}."""
    return {p: R.project(pr, torch.tensor(state(pr.geo.x_vol.numpy()))) for p, pr in mp.probs.items()}


def _neighbour_points(mp: MixedProblem, e: int, z: int) -> tuple:
    """(nu, xi^(nu)_j for the facet nodes j of facet z of element e)."""
    p = int(mp.degrees[e])
    pr = mp.probs[p]
    nu = int(pr.con.nbr_elem[e, z])
    pn = int(mp.degrees[nu])
    geo_e, geo_n = pr.geo, mp.probs[pn].geo
    vx_e, vx_n = geo_e.vx[e], geo_n.vx[nu]
    ids_e, ids_n = geo_e.vids[e], geo_n.vids[nu]
    # periodic shift: a vertex shared by the face, in both elements' coordinates
    shared = [int(g) for g in ids_e if int(g) in set(int(h) for h in ids_n)]
    ke = int(np.where(ids_e == shared[0])[0][0])
    kn = int(np.where(ids_n == shared[0])[0][0])
    shift = vx_e[ke] - vx_n[kn]
    xi = pr.ref.xi_f[z].numpy()                                     # [Nqf, d]
    A_e = 0.5 * (vx_e[1:] - vx_e[:1]).T                             # dX/dxi
    y = vx_e[0][None, :] + (1.0 + xi) @ A_e.T - shift[None, :]      # affine image in nu's frame
    A_n = 0.5 * (vx_n[1:] - vx_n[:1]).T
    xin = np.linalg.solve(A_n, (y - vx_n[0][None, :]).T).T - 1.0
    return nu, pn, torch.tensor(xin, dtype=DT)


def residual(mp: MixedProblem, uts: dict, elems, force_eval: bool = False) -> list:
    """du~/dt for the given elements (list of [Nc, Np(p_e)] tensors, in order).
    force_eval evaluates the exterior states by the modal rule on every facet,
    also between equal degrees (used to pin the rule)."""
    elems = np.asarray(elems, dtype=np.int64).reshape(-1)
    out = {}
    for p in np.unique(mp.degrees[elems]):
        p = int(p)
        pr = mp.probs[p]
        sel = elems[mp.degrees[elems] == p]

        def exterior(es, z, ext_z, p=p, pr=pr):
            rows = []
            for i, e in enumerate(np.asarray(es)):
                nu = int(pr.con.nbr_elem[e, z])
                pn = int(mp.degrees[nu])
                if pn == p and not force_eval:
                    rows.append(ext_z[i])
                    continue
                _, _, xin = _neighbour_points(mp, int(e), z)
                prn = mp.probs[pn]
                wt_nu = R.entropy_projection(prn, uts[pn], torch.as_tensor([nu]))[0]     # [Nc, Np(pn)]
                phi = pkd(mp.dim, pn, xin)                                           # [Nqf, Np(pn)]
                wp = R._rn(R.esum("jk,ck->jc", phi, wt_nu))                          # [Nqf, Nc]
                rows.append(R._rn(ph.cons_from_entropy(wp, mp.gamma)))
            return torch.stack(rows)

        res = R.residual(pr, uts[p], sel, exterior)
        for i, e in enumerate(sel):
            out[int(e)] = res[i]
    return [out[int(e)] for e in elems]
