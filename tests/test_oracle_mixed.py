"""Pins for the oracle's mixed-degree residual (reading of the paper's
conforming-interface assumption for elements of different degree).

  * with one degree everywhere, evaluating the exterior states by the modal
    rule (neighbour expansion at the carried reference points) reproduces the
    conforming residual: pins the reference-point construction, including
    periodic shifts and reversed facet orientation;
  * free-stream preservation on a curved mesh of mixed degree: a constant state
    is exactly representable on every element, so the residual vanishes to
    rounding;
  * elements whose neighbours all share their degree give the equal-degree
    residual;
  * the carried reference points, mapped by the neighbour's vertices, are the
    facet nodes' physical positions (modulo the period) and lie on the
    neighbour's reference boundary."""
import math

import numpy as np
import torch

import workloads as wl
from oracle import mixed as MX
from oracle import residual as R


def _mesh(dim, M):
    L = 2.0 if dim == 2 else 2 * math.pi
    return wl.split_box_mesh(dim, M, L), L


def test_modal_exterior_rule_reproduces_conforming_residual():
    for dim, p in ((2, 3), (3, 2)):
        mesh, L = _mesh(dim, 3)
        warp = wl.make_warp_sinprod(L, 0.05)
        deg = np.full(mesh.n_elements, p)
        mp = MX.setup(mesh, deg, warp, 1.4, 0, 1)
        uts = MX.project(mp, wl.RandomSmooth(dim, L, 4))
        el = np.arange(0, mesh.n_elements, max(1, mesh.n_elements // 9))
        got = torch.stack(MX.residual(mp, uts, el, force_eval=True))
        ref = R.residual(mp.probs[p], uts[p], el)
        assert float((got - ref).abs().max()) <= 1e-12 * float(ref.abs().max())


def test_free_stream_on_mixed_degree_curved_mesh():
    for dim in (2, 3):
        mesh, L = _mesh(dim, 3)
        warp = wl.make_warp_sinprod(L, 0.05)
        deg = wl.mixed_degrees(mesh.n_elements, 7, 1, 3)
        mp = MX.setup(mesh, deg, warp, 1.4, 0, 1)
        const = lambda x: wl.prim_to_cons(np.full(x.shape[:-1], 1.3), np.tile([0.4, -0.2, 0.3][:dim], x.shape[:-1] + (1,)),
                                          np.full(x.shape[:-1], 0.8), 1.4)
        uts = MX.project(mp, const)
        el = np.arange(mesh.n_elements)
        res = MX.residual(mp, uts, el)
        worst = max(float(r.abs().max()) for r in res)
        assert worst <= 1e-12, worst
        # and the neighbours really have other degrees somewhere
        pr = mp.probs[int(deg[0])]
        assert np.any(deg[mp.probs[int(deg[0])].con.nbr_elem[deg == deg[0]]] != deg[0])


def test_elements_with_equal_degree_neighbours_match_the_conforming_residual():
    mesh, L = _mesh(2, 4)
    warp = wl.make_warp_sinprod(L, 0.05)
    deg = np.full(mesh.n_elements, 2)
    deg[:5] = 3       # a few elements of another degree
    mp = MX.setup(mesh, deg, warp, 1.4, 0, 1)
    uts = MX.project(mp, wl.RandomSmooth(2, L, 5))
    nb = mp.probs[2].con.nbr_elem
    far = [e for e in range(mesh.n_elements) if deg[e] == 2 and np.all(deg[nb[e]] == 2)][:6]
    got = torch.stack(MX.residual(mp, uts, far))
    ref = R.residual(mp.probs[2], uts[2], far)
    assert torch.equal(got, ref)


def _barycentric(dim, xi):
    """Barycentric coordinates on the reference simplex with vertices
    (-1, ..., -1) and -1 + 2 e_k: lambda_k = (1 + xi_k)/2 for k >= 1 and
    lambda_0 = 1 - sum_k lambda_k."""
    xi = np.asarray(xi, dtype=np.float64)
    lam_k = 0.5 * (1.0 + xi)
    lam_0 = 1.0 - lam_k.sum(-1, keepdims=True)
    return np.concatenate([lam_0, lam_k], axis=-1)


def test_carried_reference_points_land_on_the_facet_nodes():
    """The neighbour reference point of every facet node, mapped by the
    neighbour's own vertices (barycentric combination), is the node's physical
    position from the geometry module, up to a whole number of periods, and it
    lies on the boundary of the neighbour's reference simplex (one barycentric
    coordinate zero, none negative).  Affine meshes of mixed degree, both
    dimensions, every facet (equal and unequal neighbour degrees)."""
    for dim, M, lo, hi in ((2, 3, 1, 5), (3, 3, 1, 4)):
        mesh, L = _mesh(dim, M)
        deg = wl.mixed_degrees(mesh.n_elements, 30 + dim, lo, hi)
        mp = MX.setup(mesh, deg, wl.warp_none, 1.4, 0, 1)
        n_unequal = 0
        for e in range(mesh.n_elements):
            pr = mp.probs[int(deg[e])]
            for z in range(dim + 1):
                nu, pn, xin = MX._neighbour_points(mp, e, z)
                n_unequal += int(pn != deg[e])
                lam = _barycentric(dim, xin.numpy())
                assert lam.min() >= -1e-13
                assert np.abs(lam.min(axis=1)).max() <= 1e-13
                vx_nu = mp.probs[pn].geo.vx[nu]                         # [d+1, d]
                x = lam @ vx_nu
                xf = pr.geo.x_f[z][e].numpy()
                k = np.round((x - xf) / L)
                assert np.abs(x - xf - k * L).max() <= 1e-12 * L
        assert n_unequal > 0
