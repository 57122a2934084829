"""CPU tests of the C-ABI library: it loads, exports every symbol the header
declares, and its host-side setup (geometry and connectivity, built in C++
independently of the oracle) agrees with the oracle's.  No device calls."""
import math
import os
import re
import subprocess

import numpy as np
import pytest
import torch

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "esdsem.h")


def _lib():
    import paper_2312_07874_amd as esd
    return esd


def test_library_exports_every_header_symbol():
    esd = _lib()
    decl = set(re.findall(r"\b(esd_[a-z_0-9]+)\s*\(", open(HEADER).read()))
    decl.discard("esd_warp_fn")
    out = subprocess.run(["nm", "-D", "--defined-only", esd.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (esd_[a-z_0-9]+)$", out, re.M))
    assert decl, "no declarations parsed"
    assert decl <= exported, decl - exported
    assert decl == set(esd.EXPORTS), decl ^ set(esd.EXPORTS)


def test_plan_create_rejects_bad_arguments():
    esd = _lib()
    mesh = wl.split_box_mesh(2, 3, 2.0)
    with pytest.raises(esd.EsdError) as e:
        esd.Plan(2, 42, mesh.elem_vertex_ids, mesh.elem_vertex_coords, host_only=True)
    assert e.value.status == -4
    with pytest.raises(esd.EsdError) as e:
        esd.Plan(2, 2, mesh.elem_vertex_ids, mesh.elem_vertex_coords, gamma=0.9, host_only=True)
    assert e.value.status == -1
    # an over-warped mesh folds: the mapping Jacobian becomes negative
    with pytest.raises(esd.EsdError) as e:
        esd.Plan(2, 3, mesh.elem_vertex_ids, mesh.elem_vertex_coords, wl.make_warp_sinprod(2.0, 0.6), host_only=True)
    assert e.value.status == -2


CASES = [(2, 3, 2, 0.05), (2, 3, 5, 0.05), (3, 3, 2, 0.05), (3, 3, 4, 0.08)]


@pytest.mark.parametrize("dim,M,p,amp", CASES)
def test_host_geometry_matches_oracle(dim, M, p, amp):
    esd = _lib()
    from oracle import residual as R
    L = 2.0 if dim == 2 else 2 * math.pi
    mesh = wl.split_box_mesh(dim, M, L)
    warp = wl.make_warp_sinprod(L, amp)
    plan = esd.Plan(dim, p, mesh.elem_vertex_ids, mesh.elem_vertex_coords, warp, host_only=True)
    prob = R.setup(mesh, p, warp)
    geo = prob.geo
    np.testing.assert_allclose(plan.host_array("x_vol"), geo.x_vol.numpy(), atol=1e-12)
    np.testing.assert_allclose(plan.host_array("J"), geo.J.numpy(), rtol=1e-11)
    Gs = float(geo.G.abs().max())
    np.testing.assert_allclose(plan.host_array("G"), geo.G.numpy(), atol=1e-12 * Gs)
    nJ = plan.host_array("nJ").reshape(prob.ne, prob.ref.Nf, -1, dim)
    Jf = plan.host_array("Jf").reshape(prob.ne, prob.ref.Nf, -1)
    for z in range(prob.ref.Nf):
        np.testing.assert_allclose(nJ[:, z], geo.nJ[z].numpy(), atol=1e-12 * Gs)
        np.testing.assert_allclose(Jf[:, z], geo.Jf[z].numpy(), rtol=1e-11)
    # connectivity: neighbour (element, facet, node) identical to the oracle's
    nbr = plan.host_array("nbr").astype(np.int64).reshape(prob.ne, prob.ref.Nf, -1)
    nqf = nbr.shape[-1]
    con = prob.con
    for z in range(prob.ref.Nf):
        e_n = nbr[:, z] // (prob.ref.Nf * nqf)
        f_n = (nbr[:, z] // nqf) % prob.ref.Nf
        j_n = nbr[:, z] % nqf
        assert (e_n == con.nbr_elem[:, z, None]).all()
        assert (f_n == con.nbr_face[:, z, None]).all()
        assert (j_n == con.node_map[:, z]).all()


def test_plan_info_counts():
    esd = _lib()
    mesh = wl.split_box_mesh(3, 3, 2 * math.pi)
    plan = esd.Plan(3, 4, mesh.elem_vertex_ids, mesh.elem_vertex_coords, host_only=True)
    i = plan.info
    assert i.n_modes == 35 and i.n_vol_nodes == 125 and i.n_facets == 4 and i.n_facet_nodes == 25
    assert i.flux_pairs_paper == 4 * 5 ** 4 * mesh.n_elements
    assert i.flux_pairs_distinct == 5 ** 3 * (2.5 * 4 + 4) * mesh.n_elements
    assert i.n_dof == mesh.n_elements * 5 * 35


def test_workspace_sizes_and_host_only_rejection():
    """Workspace sizes follow the documented layout; compute entry points refuse
    a host-only plan with ESD_EINVAL before touching any device."""
    esd = _lib()
    mesh = wl.split_box_mesh(3, 3, 2 * math.pi)
    plan = esd.Plan(3, 3, mesh.elem_vertex_ids, mesh.elem_vertex_coords, host_only=True)
    i = plan.info
    a256 = lambda n: (n + 255) // 256 * 256
    ndof_b = a256(i.n_dof * 8)
    fac_b = a256(i.n_elements * i.n_vars * i.n_facets * i.n_facet_nodes * 8)
    assert i.workspace_bytes == ndof_b + fac_b
    assert i.rk4_workspace_bytes == 2 * i.workspace_bytes + 3 * ndof_b
    assert i.vjp_workspace_bytes == i.workspace_bytes + fac_b
    assert i.rk4_vjp_workspace_bytes == i.vjp_workspace_bytes + 3 * ndof_b
    L = esd._lib
    fake = 256
    assert L.esd_residual(plan._h, fake, 2 * fake, 3 * fake, None) == -1
    assert L.esd_residual_vjp(plan._h, fake, 2 * fake, 3 * fake, 4 * fake, None) == -1
    assert L.esd_rk4(plan._h, fake, 1e-3, 1, 2 * fake, None, None) == -1
    assert L.esd_rk4_vjp(plan._h, fake, 1e-3, 1, 2 * fake, 3 * fake, None) == -1
    assert b"host-only" in L.esd_last_error()


def test_batched_plan_buckets_and_element_map():
    """Host-only batched plan: buckets by ascending degree over all meshes,
    slots in mesh order, offsets consistent with the per-degree sizes."""
    esd = _lib()
    L = 2 * math.pi
    m1, m2 = wl.split_box_mesh(3, 3, L), wl.split_box_mesh(3, 4, L)
    d1, d2 = wl.mixed_degrees(m1.n_elements, 1, 2, 5), wl.mixed_degrees(m2.n_elements, 2, 3, 6)
    plan = esd.BatchedPlan(3, [(m1.elem_vertex_ids, m1.elem_vertex_coords, d1),
                               (m2.elem_vertex_ids, m2.elem_vertex_coords, d2)], host_only=True)
    degs = np.concatenate([d1, d2])
    assert [b["degree"] for b in plan.buckets] == sorted(set(degs.tolist()))
    for bi, b in enumerate(plan.buckets):
        members = np.where(degs == b["degree"])[0]
        assert b["n_elements"] == len(members)
        assert np.array_equal(plan.elem_bucket[members], np.full(len(members), bi))
        assert np.array_equal(plan.elem_slot[members], np.arange(len(members)))
        np_ = (b["degree"] + 1) * (b["degree"] + 2) * (b["degree"] + 3) // 6
        assert b["dof"][1] - b["dof"][0] == len(members) * 5 * np_
        assert b["nodes"][1] - b["nodes"][0] == len(members) * (b["degree"] + 1) ** 3
    assert plan.info.n_dof == plan.buckets[-1]["dof"][1]
    assert plan.info.n_elements == len(degs)


def test_batched_vjp_workspace_layout():
    """The batched VJP workspace: the residual workspace, then per bucket
    n_elements N_c N_fq doubles of exterior cotangents (256-byte aligned), then
    the adjoint kernels' per-element slices (tetrahedra at p = 9, 10 only);
    the RK4 adjoint adds three state arrays.  Host-only: the entry points
    refuse with ESD_EINVAL."""
    esd = _lib()
    L = 2 * math.pi
    m1 = wl.split_box_mesh(3, 3, L)
    d1 = wl.mixed_degrees(m1.n_elements, 1, 2, 5)
    plan = esd.BatchedPlan(3, [(m1.elem_vertex_ids, m1.elem_vertex_coords, d1)], host_only=True)
    a256 = lambda n: (n + 255) // 256 * 256
    xbar = sum(a256(b["n_elements"] * 5 * 4 * (b["degree"] + 1) ** 2 * 8) for b in plan.buckets)
    i = plan.info
    assert i.vjp_workspace_bytes == i.workspace_bytes + xbar
    assert i.rk4_vjp_workspace_bytes == i.vjp_workspace_bytes + 3 * a256(i.n_dof * 8)
    fake = 256
    assert esd._lib.esd_residual_vjp(plan._h, fake, 2 * fake, 3 * fake, 4 * fake, None) == -1
