"""GPU checks of batched plans (several meshes, per-element degrees).

  * a batch whose buckets each cover a whole mesh of one degree runs the same
    kernels on the same elements as the single-degree plans: equal up to the
    order of the LDS atomic sums (which varies from run to run);
  * mixed degrees on small curved meshes, and two meshes in one batch, against
    the oracle's mixed-degree residual element by element (1e-12 per
    variable, or the oracle's own rounding spread where that is larger);
  * the benchmark-size batch (4 meshes, 35,904 tetrahedra, p = 2..10)
    preserves a constant state to rounding, a property that holds at any size;
  * RK4 and diagnostics run on batched plans."""
import math

import numpy as np
import pytest
import torch

import workloads as wl
from tests.parity_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def batched(dim, meshes, degrees, warp, ecflux=0, dissipation=1):
    import paper_2312_07874_amd as esd
    return esd.BatchedPlan(dim, [(m.elem_vertex_ids, m.elem_vertex_coords, d) for m, d in zip(meshes, degrees)],
                           warp, 1.4, ecflux, dissipation)


def project_state(plan, state):
    x = plan.node_coords().cpu().numpy()
    return plan.project(torch.tensor(state(x), device="cuda").reshape(plan.nodal_shape).contiguous())


def test_equal_degree_batch_equals_the_single_plan():
    import paper_2312_07874_amd as esd
    L = 2 * math.pi
    warp = wl.make_warp_sinprod(L, 0.05)
    st = wl.RandomSmooth(3, L, 3)
    m1, m2 = wl.split_box_mesh(3, 3, L), wl.split_box_mesh(3, 4, L)
    plan = batched(3, [m1, m2], [np.full(m1.n_elements, 3), np.full(m2.n_elements, 5)], warp)
    assert [b["degree"] for b in plan.buckets] == [3, 5]
    u = project_state(plan, st)
    out = plan.residual(u)
    plan.sync_status()
    for b, (m, p) in enumerate(((m1, 3), (m2, 5))):
        single = esd.Plan(3, p, m.elem_vertex_ids, m.elem_vertex_coords, warp, 1.4, 0, 1)
        us = plan.bucket_view(u, b).contiguous()
        ref = single.residual(us)
        single.sync_status()
        got = plan.bucket_view(out, b)
        for c in range(ref.shape[1]):
            err = float((got[:, c] - ref[:, c]).abs().max())
            scale = float(ref[:, c].abs().max())
            log(f"bucket {b} variable {c}: max |batched - single| / ||r||_inf = {err / scale:.2e}")
            assert err <= 1e-13 * scale, f"bucket {b}"


def _oracle_compare(plan, meshes, degrees, warp, state, ecflux, dissipation, what, sample=None):
    """Batched residual against the oracle's mixed-degree residual, per
    conserved variable: max |r_gpu - r_oracle| <= max(1e-12 ||r_oracle||_inf,
    4 d), d the oracle's own rounding spread on the same elements (every
    intermediate of the oracle carrying one rounding, tests/parity_util.py);
    nothing the library computes enters the bar."""
    from oracle import mixed as MX
    from tests.parity_util import NOISE_FACTOR, oracle_with_spread
    worst = 0.0
    base = 0
    # one flat state from the oracle's per-degree projections
    u = torch.zeros(plan.state_shape, dtype=torch.float64)
    mps, utss = [], []
    for m, deg in zip(meshes, degrees):
        mp = MX.setup(m, deg, warp, 1.4, ecflux, dissipation)
        uts = MX.project(mp, state)
        mps.append(mp)
        utss.append(uts)
    nc = plan.info.n_vars
    for k, (m, deg) in enumerate(zip(meshes, degrees)):
        for e in range(m.n_elements):
            g = base + e
            b, s = int(plan.elem_bucket[g]), int(plan.elem_slot[g])
            plan.bucket_view(u, b)[s] = utss[k][int(deg[e])][e]
        base += m.n_elements
    out = plan.residual(u.cuda().contiguous())
    plan.sync_status()
    out = out.cpu()
    base = 0
    for k, (m, deg) in enumerate(zip(meshes, degrees)):
        el = np.arange(m.n_elements) if sample is None else sample
        # ragged per-element results stacked along the mode axis for the spread
        flat = lambda mp: torch.cat([x for x in MX.residual(mp, utss[k], el)], 1)
        ref_flat, spread_flat = oracle_with_spread(flat, mps[k],
                                                   lambda: MX.setup(meshes[k], degrees[k], warp, 1.4, ecflux, dissipation))
        scale, err, spr = np.zeros(nc), np.zeros(nc), np.zeros(nc)
        off = 0
        for i, e in enumerate(el):
            g = base + int(e)
            b, s = int(plan.elem_bucket[g]), int(plan.elem_slot[g])
            got = plan.bucket_view(out, b)[s]
            n = got.shape[1]
            ref = ref_flat[:, off:off + n]
            scale = np.maximum(scale, ref.abs().amax(1).numpy())
            err = np.maximum(err, (got - ref).abs().amax(1).numpy())
            spr = np.maximum(spr, spread_flat[:, off:off + n].abs().amax(1).numpy())
            off += n
        bound = np.maximum(1e-12 * scale, NOISE_FACTOR * spr)
        log(f"batched parity {what} mesh {k}: max err / ||r_e||_inf per var {['%.1e' % x for x in err / scale]}, "
            f"oracle spread / ||r_e||_inf {['%.1e' % x for x in spr / scale]}, "
            f"err / bound {['%.2f' % x for x in err / bound]}")
        worst = max(worst, float((err / bound).max()))
        base += m.n_elements
    assert worst <= 1.0, worst


@pytest.mark.parametrize("dim,M,lo,hi,ecflux,diss", [(2, 3, 1, 5, 0, 1), (3, 3, 1, 4, 0, 1), (3, 3, 2, 4, 1, 0)])
def test_mixed_degree_parity_with_oracle(dim, M, lo, hi, ecflux, diss):
    L = 2.0 if dim == 2 else 2 * math.pi
    warp = wl.make_warp_sinprod(L, 0.05)
    mesh = wl.split_box_mesh(dim, M, L)
    deg = wl.mixed_degrees(mesh.n_elements, 11 + dim, lo, hi)
    plan = batched(dim, [mesh], [deg], warp, ecflux, diss)
    log(f"case dim={dim} M={M} degrees {lo}..{hi}: buckets {[(b['degree'], b['n_elements']) for b in plan.buckets]}")
    _oracle_compare(plan, [mesh], [deg], warp, wl.RandomSmooth(dim, L, 6), ecflux, diss, f"dim{dim}_p{lo}-{hi}")


def test_mixed_degree_parity_high_degrees_sampled():
    """Degrees 5..10 on 162 curved tetrahedra (facets of 36 to 121 nodes: the
    mixed-interface contraction split over lane slices at p = 5, one lane per
    node above), 12 sampled elements against the oracle."""
    L = 2 * math.pi
    warp = wl.make_warp_sinprod(L, 0.05)
    mesh = wl.split_box_mesh(3, 3, L)
    deg = wl.mixed_degrees(mesh.n_elements, 14, 5, 10)
    plan = batched(3, [mesh], [deg], warp, 0, 1)
    el = np.random.default_rng(3).choice(mesh.n_elements, 12, replace=False)
    log(f"case degrees 5..10: buckets {[(b['degree'], b['n_elements']) for b in plan.buckets]}, sampled {deg[el].tolist()}")
    _oracle_compare(plan, [mesh], [deg], warp, wl.RandomSmooth(3, L, 6), 0, 1, "dim3_p5-10", sample=el)


def test_two_meshes_in_one_batch():
    L = 2.0
    warp = wl.make_warp_sinprod(L, 0.05)
    m1, m2 = wl.split_box_mesh(2, 3, L), wl.split_box_mesh(2, 4, L)
    d1, d2 = wl.mixed_degrees(m1.n_elements, 1, 1, 4), wl.mixed_degrees(m2.n_elements, 2, 2, 6)
    plan = batched(2, [m1, m2], [d1, d2], warp)
    _oracle_compare(plan, [m1, m2], [d1, d2], warp, wl.RandomSmooth(2, L, 9), 0, 1, "two meshes")


def test_benchmark_batch_free_stream_and_rk4():
    """Constant state on the 4-mesh batch (p = 2..10): the residual vanishes to
    rounding relative to the flux magnitude; a few RK4 steps of a smooth state
    stay admissible and conserve the conserved integrals."""
    bt = wl.batched_tets()
    plan = batched(3, bt.meshes, bt.degrees, bt.warp)
    log(f"benchmark batch: {plan.info.n_elements} elements, {plan.info.n_dof} DOF, buckets "
        f"{[(b['degree'], b['n_elements']) for b in plan.buckets]}")
    const = lambda x: wl.prim_to_cons(np.full(x.shape[:-1], 1.1), np.tile([0.2, -0.1, 0.15], x.shape[:-1] + (1,)),
                                      np.full(x.shape[:-1], 0.9), 1.4)
    u = project_state(plan, const)
    r = plan.residual(u)
    plan.sync_status()
    # flux magnitude scale: rho v^2 + p ~ 1; residual entries are O(p^2 / h) times that
    worst = float(r.abs().max())
    log(f"free stream: max |du~/dt| = {worst:.3e}")
    assert worst <= 1e-9
    u = project_state(plan, bt.state)
    d0 = plan.diagnostics(u)
    plan.rk4(u, 1e-4, 3)
    plan.sync_status()
    d1 = plan.diagnostics(u)
    log(f"conserved before {d0['conserved']}, after {d1['conserved']}; entropy rate {d1['entropy_rate']:.3e}")
    # conservation holds within each conforming equal-degree region only; across
    # a change of degree the interface terms do not cancel exactly: report, and
    # check that mass changes far less than the state
    assert np.all(np.isfinite(d1["conserved"]))
    assert abs(d1["conserved"][0] - d0["conserved"][0]) <= 1e-6 * abs(d0["conserved"][0])


def test_batched_rk4_step_matches_oracle():
    """One classical RK4 step on a mixed-degree mesh: the library's RK4 on the
    batched plan against RK4 written out with the oracle's mixed residual."""
    from oracle import mixed as MX
    L = 2.0
    warp = wl.make_warp_sinprod(L, 0.05)
    mesh = wl.split_box_mesh(2, 3, L)
    deg = wl.mixed_degrees(mesh.n_elements, 21, 1, 4)
    plan = batched(2, [mesh], [deg], warp)
    mp = MX.setup(mesh, deg, warp, 1.4, 0, 1)
    uts = MX.project(mp, wl.RandomSmooth(2, L, 8))
    ne = mesh.n_elements
    cur = [uts[int(deg[e])][e].clone() for e in range(ne)]

    def rhs(state):
        full = {p: uts[p].clone() for p in uts}
        for e in range(ne):
            full[int(deg[e])][e] = state[e]
        return MX.residual(mp, full, np.arange(ne))

    dt = 2e-3
    k1 = rhs(cur)
    k2 = rhs([cur[e] + 0.5 * dt * k1[e] for e in range(ne)])
    k3 = rhs([cur[e] + 0.5 * dt * k2[e] for e in range(ne)])
    k4 = rhs([cur[e] + dt * k3[e] for e in range(ne)])
    ref = [cur[e] + dt / 6 * (k1[e] + 2 * k2[e] + 2 * k3[e] + k4[e]) for e in range(ne)]
    u = torch.zeros(plan.state_shape, dtype=torch.float64)
    for e in range(ne):
        plan.bucket_view(u, int(plan.elem_bucket[e]))[int(plan.elem_slot[e])] = cur[e]
    ug = u.cuda().contiguous()
    plan.rk4(ug, dt, 1)
    plan.sync_status()
    ug = ug.cpu()
    nc = plan.info.n_vars
    err, scale = np.zeros(nc), np.zeros(nc)
    for e in range(ne):
        got = plan.bucket_view(ug, int(plan.elem_bucket[e]))[int(plan.elem_slot[e])]
        err = np.maximum(err, (got - ref[e]).abs().amax(1).numpy())
        scale = np.maximum(scale, ref[e].abs().amax(1).numpy())
    log(f"batched RK4 step: max err / ||u_e||_inf per var {['%.1e' % x for x in err / scale]}")
    assert float((err / scale).max()) <= 1e-12


# ---------------------------------------------------------------- VJP of batched plans
def _flat_state(plan, meshes, degrees, utss):
    """One flat batched state from the oracle's per-degree tensors."""
    u = torch.zeros(plan.state_shape, dtype=torch.float64)
    base = 0
    for k, (m, deg) in enumerate(zip(meshes, degrees)):
        for e in range(m.n_elements):
            g = base + e
            b, s = int(plan.elem_bucket[g]), int(plan.elem_slot[g])
            plan.bucket_view(u, b)[s] = utss[k][int(deg[e])][e]
        base += m.n_elements
    return u


def _mixed_oracle_vjp(mp, uts, vbar_of, elems):
    """Rows elems of (dR/du~)^T vbar for the oracle's mixed-degree residual, by
    reverse-mode autodiff: the residual is evaluated on the 1-ring of elems
    (every element whose residual reads their w~: face neighbours, across a
    change of degree too), vbar_of(e) the cotangent of element e."""
    con = next(iter(mp.probs.values())).con
    elems = np.asarray(elems, dtype=np.int64)
    ring = np.unique(np.concatenate([elems, con.nbr_elem[elems].reshape(-1)]))
    leaves = {p: t.detach().clone().requires_grad_(True) for p, t in uts.items()}
    from oracle import mixed as MX
    res = MX.residual(mp, leaves, ring)
    obj = sum((r * vbar_of(int(e))).sum() for r, e in zip(res, ring))
    grads = torch.autograd.grad(obj, list(leaves.values()), allow_unused=True)
    gd = {p: (g if g is not None else torch.zeros_like(leaves[p])) for p, g in zip(leaves, grads)}
    return [gd[int(mp.degrees[e])][e] for e in elems]


def _vjp_compare(dim, meshes, degrees, warp, state, ecflux, diss, what, sample=None, seed=71):
    from oracle import mixed as MX
    plan = batched(dim, meshes, degrees, warp, ecflux, diss)
    log(f"batched VJP {what}: buckets {[(b['degree'], b['n_elements']) for b in plan.buckets]}")
    mps = [MX.setup(m, d, warp, 1.4, ecflux, diss) for m, d in zip(meshes, degrees)]
    utss = [MX.project(mp, state) for mp in mps]
    u = _flat_state(plan, meshes, degrees, utss)
    vbar = torch.randn(plan.state_shape, generator=torch.Generator().manual_seed(seed), dtype=torch.float64)
    g = plan.vjp(u.cuda().contiguous(), vbar.cuda().contiguous())
    plan.sync_status()
    g = g.cpu()
    nc = plan.info.n_vars
    worst = 0.0
    base = 0
    for k, (m, deg) in enumerate(zip(meshes, degrees)):
        def vbar_of(e, base=base):
            b, s = int(plan.elem_bucket[base + e]), int(plan.elem_slot[base + e])
            return plan.bucket_view(vbar, b)[s]
        el = np.arange(m.n_elements) if sample is None else np.asarray(sample)
        ref = _mixed_oracle_vjp(mps[k], utss[k], vbar_of, el)
        err, scale = np.zeros(nc), np.zeros(nc)
        for i, e in enumerate(el):
            b, s = int(plan.elem_bucket[base + e]), int(plan.elem_slot[base + e])
            got = plan.bucket_view(g, b)[s]
            scale = np.maximum(scale, ref[i].abs().amax(1).numpy())
            err = np.maximum(err, (got - ref[i]).abs().amax(1).numpy())
        log(f"batched VJP {what} mesh {k}: max err / ||g_e||_inf per var {['%.2e' % x for x in err / scale]}")
        worst = max(worst, float((err / scale).max()))
        base += m.n_elements
    assert worst <= 1e-12, worst
    return plan


@pytest.mark.parametrize("dim,M,lo,hi,ecflux,diss", [(2, 3, 1, 5, 0, 1), (3, 3, 1, 4, 0, 1), (3, 3, 2, 4, 1, 0)])
def test_batched_vjp_parity_with_oracle(dim, M, lo, hi, ecflux, diss):
    """The batched VJP (with the adjoint of the mixed-degree exterior values)
    against reverse-mode autodiff of the oracle's mixed-degree residual, every
    element, 1e-12 per variable relative to ||g_e||_inf."""
    L = 2.0 if dim == 2 else 2 * math.pi
    warp = wl.make_warp_sinprod(L, 0.05)
    mesh = wl.split_box_mesh(dim, M, L)
    deg = wl.mixed_degrees(mesh.n_elements, 31 + dim, lo, hi)
    _vjp_compare(dim, [mesh], [deg], warp, wl.RandomSmooth(dim, L, 6), ecflux, diss, f"dim{dim}_p{lo}-{hi}")


def test_batched_vjp_two_meshes_and_high_degrees_sampled():
    """Two triangle meshes in one batch in full; tetrahedra at degrees 5..10 on
    6 sampled elements (the oracle differentiates their 1-ring)."""
    L = 2.0
    warp = wl.make_warp_sinprod(L, 0.05)
    m1, m2 = wl.split_box_mesh(2, 3, L), wl.split_box_mesh(2, 4, L)
    d1, d2 = wl.mixed_degrees(m1.n_elements, 41, 1, 4), wl.mixed_degrees(m2.n_elements, 42, 2, 6)
    _vjp_compare(2, [m1, m2], [d1, d2], warp, wl.RandomSmooth(2, L, 9), 0, 1, "two meshes")
    L = 2 * math.pi
    warp = wl.make_warp_sinprod(L, 0.05)
    mesh = wl.split_box_mesh(3, 3, L)
    deg = wl.mixed_degrees(mesh.n_elements, 43, 5, 10)
    el = np.random.default_rng(4).choice(mesh.n_elements, 6, replace=False)
    _vjp_compare(3, [mesh], [deg], warp, wl.RandomSmooth(3, L, 6), 0, 1, "dim3_p5-10", sample=el)


def test_batched_vjp_equal_degree_buckets_equal_the_single_plans():
    """Buckets that each cover a whole mesh of one degree: the batched VJP is
    the single-degree plans' VJP (no mixed-degree facet), up to the order of
    the LDS atomic sums."""
    import paper_2312_07874_amd as esd
    L = 2 * math.pi
    warp = wl.make_warp_sinprod(L, 0.05)
    st = wl.RandomSmooth(3, L, 3)
    m1, m2 = wl.split_box_mesh(3, 3, L), wl.split_box_mesh(3, 4, L)
    plan = batched(3, [m1, m2], [np.full(m1.n_elements, 3), np.full(m2.n_elements, 9)], warp)
    u = project_state(plan, st)
    vbar = torch.randn(plan.state_shape, generator=torch.Generator().manual_seed(5), dtype=torch.float64).cuda()
    g = plan.vjp(u, vbar)
    plan.sync_status()
    for b, (m, p) in enumerate(((m1, 3), (m2, 9))):
        single = esd.Plan(3, p, m.elem_vertex_ids, m.elem_vertex_coords, warp, 1.4, 0, 1)
        ref = single.vjp(plan.bucket_view(u, b).contiguous(), plan.bucket_view(vbar, b).contiguous())
        single.sync_status()
        got = plan.bucket_view(g, b)
        for c in range(ref.shape[1]):
            err = float((got[:, c] - ref[:, c]).abs().max())
            scale = float(ref[:, c].abs().max())
            log(f"VJP bucket {b} (p {p}) variable {c}: max |batched - single| / ||g||_inf = {err / scale:.2e}")
            assert err <= 1e-13 * scale, f"bucket {b}"


def test_batched_vjp_central_differences_benchmark_batch():
    """<vbar, R(u + h d) - R(u - h d)> / (2h) = <VJP(vbar), d> on the 4-mesh
    batch (35,904 curved tetrahedra, p = 2..10) with the entropy-conservative
    interface flux (smooth residual), and the discrete RK4 adjoint of one step
    against the same identity; library only."""
    bt = wl.batched_tets()
    plan = batched(3, bt.meshes, bt.degrees, bt.warp, 0, 0)
    u = project_state(plan, bt.state)
    vbar = torch.randn(plan.state_shape, generator=torch.Generator().manual_seed(8), dtype=torch.float64).cuda()
    g = plan.vjp(u, vbar)
    h = 1e-6
    for k in range(3):
        d = torch.randn(plan.state_shape, generator=torch.Generator().manual_seed(300 + k), dtype=torch.float64).cuda()
        fp = (plan.residual((u + h * d).contiguous()) * vbar).sum()
        fm = (plan.residual((u - h * d).contiguous()) * vbar).sum()
        fd = float((fp - fm) / (2 * h))
        ad = float((g * d).sum())
        log(f"batch direction {k}: fd {fd:.12e} adjoint {ad:.12e} rel {abs(fd - ad) / abs(ad):.2e}")
        assert abs(fd - ad) <= 1e-6 * abs(ad)
    # one RK4 step: d/du0 <vbar, u1(u0)>
    dt = 1e-4
    ckpt = torch.empty((4,) + plan.state_shape, dtype=torch.float64, device="cuda")
    u1 = u.clone()
    plan.rk4(u1, dt, 1, ckpt)
    ubar = vbar.clone()
    plan.rk4_vjp(ckpt, dt, 1, ubar)
    d = torch.randn(plan.state_shape, generator=torch.Generator().manual_seed(400), dtype=torch.float64).cuda()
    up, um = (u + h * d).contiguous(), (u - h * d).contiguous()
    plan.rk4(up, dt, 1)
    plan.rk4(um, dt, 1)
    fd = float(((up - um) * vbar).sum() / (2 * h))
    ad = float((ubar * d).sum())
    log(f"batch RK4 step: fd {fd:.12e} adjoint {ad:.12e} rel {abs(fd - ad) / abs(ad):.2e}")
    assert abs(fd - ad) <= 1e-6 * abs(ad)
    plan.sync_status()
