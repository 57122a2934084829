// C ABI of the library (declared in include/esdsem.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <exception>
#include <algorithm>
#include <array>
#include <limits>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "scratch.hpp"

#include "esdsem.h"
#include "plan.hpp"

namespace {
thread_local std::string g_err;

esd_status fail(esd_status s, const std::string& m) {
  g_err = m;
  return s;
}

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

#define HIP_TRY(x)                                                                   \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) return fail(ESD_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// the allocator of the plan being created (set by the creating entry point
// for the duration of the call; copied into every plan it creates)
thread_local const esd_allocator* g_alloc = nullptr;

void adopt_allocator(esd_plan* p) {
  if (g_alloc && g_alloc->alloc && g_alloc->free) {
    p->dev_alloc = g_alloc->alloc;
    p->dev_free = g_alloc->free;
    p->alloc_ctx = g_alloc->ctx;
  }
}

void* dev_alloc(const esd_plan* p, size_t bytes) {
  if (p->dev_alloc) return p->dev_alloc(bytes, p->alloc_ctx);
  void* ptr = nullptr;
  return hipMalloc(&ptr, bytes) == hipSuccess ? ptr : nullptr;
}

void dev_free(const esd_plan* p, void* ptr) {
  if (!ptr) return;
  if (p->dev_free) p->dev_free(ptr, p->alloc_ctx);
  else (void)hipFree(ptr);
}

template <typename T>
esd_status upload(const esd_plan* p, T** dst, const std::vector<T>& src) {
  *dst = (T*)dev_alloc(p, std::max<size_t>(1, src.size()) * sizeof(T));
  if (!*dst) return fail(ESD_ENOMEM, "device allocation failed");
  if (((uintptr_t)*dst) % 256 != 0) return fail(ESD_EINVAL, "the device allocator returned memory not 256-byte aligned");
  HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return ESD_OK;
}

void free_device(esd_plan* p) {
  dev_free(p, p->d_tables);
  dev_free(p, p->d_gvol);
  dev_free(p, p->d_gfac);
  dev_free(p, p->d_conn);
  dev_free(p, p->d_xvol);
  if (p->flag_owned) dev_free(p, p->d_flag);
  dev_free(p, p->d_wext_off);
  dev_free(p, p->d_mats);
  dev_free(p, p->d_mat_off);
  dev_free(p, p->d_wt_off);
  dev_free(p, p->d_arecs);
  dev_free(p, p->d_asegs);
  dev_free(p, p->d_xbar_off);
  p->d_tables = p->d_gvol = p->d_gfac = p->d_xvol = p->d_mats = nullptr;
  p->d_conn = p->d_arecs = p->d_asegs = nullptr;
  p->d_mat_off = p->d_wt_off = p->d_wext_off = p->d_xbar_off = nullptr;
  p->d_flag = nullptr;
}

// Scaled metric rows for the line families (see plan.hpp), w J and w / J.
std::vector<double> pack_gvol(const esd_plan& P) {
  const esd::RefTables& R = P.ref;
  const int dim = P.dim, NQ = R.NQ, Q = R.Q, NGV = esd::ngv(dim);
  std::vector<double> g((size_t)P.ne * NGV * NQ);
  for (int64_t e = 0; e < P.ne; ++e)
    for (int k = 0; k < NQ; ++k) {
      const double* G = &P.geo.G[((size_t)e * NQ + k) * dim * dim];   // G[l*dim + m]
      double* o = &g[(size_t)e * NGV * NQ];
      const double J = P.geo.J[(size_t)e * NQ + k];
      if (dim == 2) {
        const int a1 = k % Q, a2 = k / Q;
        const double w1 = R.wl[a1], w2 = R.wl[a2];
        for (int m = 0; m < 2; ++m) {
          o[(0 + m) * NQ + k] = w2 * G[0 * 2 + m];
          o[(2 + m) * NQ + k] = 0.5 * w2 * G[1 * 2 + m];
          o[(4 + m) * NQ + k] = 0.5 * w1 * G[1 * 2 + m];
        }
      } else {
        const int a1 = k % Q, a2 = (k / Q) % Q, a3 = k / (Q * Q);
        const double w1 = R.wl[a1], w2 = R.wl[a2], w3 = R.wj[a3], e2 = R.xl[a2];
        for (int m = 0; m < 3; ++m) {
          o[(0 + m) * NQ + k] = 0.5 * w2 * w3 * G[0 * 3 + m];
          o[(3 + m) * NQ + k] = 0.25 * w2 * w3 * (G[1 * 3 + m] + G[2 * 3 + m]);
          o[(6 + m) * NQ + k] = 0.25 * w1 * w3 * G[1 * 3 + m];
          o[(9 + m) * NQ + k] = 0.125 * w1 * w3 * G[2 * 3 + m];
          o[(12 + m) * NQ + k] = 0.125 * w1 * w2 * (1.0 - e2) * G[2 * 3 + m];
        }
      }
      o[(NGV - 2) * NQ + k] = R.w[k] * J;
      o[(NGV - 1) * NQ + k] = R.w[k] / J;
    }
  return g;
}
}  // namespace

extern "C" {

const char* esd_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {
// One plan for elements of one degree.  connect = false leaves the facet
// permutation to the caller (elements of one degree out of a mixed mesh, whose
// facet-state region then holds 2 ne slots: own values and exterior values).
esd_status create_single(const esd_mesh_desc* mesh, const esd_scheme_desc* scheme, uint32_t flags, bool connect,
                         esd_plan** out) {
  *out = nullptr;
  if (mesh->dim != 2 && mesh->dim != 3) return fail(ESD_EUNSUPPORTED, "dim must be 2 or 3");
  if (!esd::degree_supported(mesh->dim, mesh->degree))
    return fail(ESD_EUNSUPPORTED, "degree " + std::to_string(mesh->degree) + " not built for dim " +
                                      std::to_string(mesh->dim));
  if (mesh->n_elements <= 0 || !mesh->elem_vertex_ids || !mesh->elem_vertex_coords)
    return fail(ESD_EINVAL, "empty mesh");
  if (!(scheme->gamma > 1.0) || scheme->ecflux < 0 || scheme->ecflux > 1 || scheme->dissipation < 0 ||
      scheme->dissipation > 3)
    return fail(ESD_EINVAL, "bad scheme parameters");
  esd_plan* P = new (std::nothrow) esd_plan();
  if (!P) return fail(ESD_ENOMEM, "host allocation failed");
  adopt_allocator(P);
  try {
    P->dim = mesh->dim;
    P->p = mesh->degree;
    P->nc = mesh->dim + 2;
    P->ne = mesh->n_elements;
    P->scheme.gamma = scheme->gamma;
    P->scheme.gm1_inv = 1.0 / (scheme->gamma - 1.0);
    P->scheme.ecflux = scheme->ecflux;
    P->scheme.dissipation = scheme->dissipation;
    P->host_only = (flags & 1u) != 0;
    P->ref = esd::build_ref_tables(P->dim, P->p);
    std::string msg;
    const int rc = esd::build_geometry(P->ref, P->ne, mesh->elem_vertex_ids, mesh->elem_vertex_coords,
                                       (esd::warp_fn)mesh->warp, mesh->warp_ctx, P->geo, msg, connect);
    P->wext = !connect;
    if (rc != 0) {
      delete P;
      return fail((esd_status)rc, msg);
    }
    const esd::RefTables& R = P->ref;
    const size_t ndof = (size_t)P->ne * P->nc * R.NP;
    const size_t fbytes = align256((size_t)P->ne * P->nc * R.NFQ * sizeof(double) * (P->wext ? 2 : 1));
    P->frec_bytes = esd::needs_facet_records(P->dim, P->p)
                        ? align256((size_t)P->ne * 8 * R.NFQ * sizeof(double)) : 0;
    P->ws_bytes = align256(ndof * sizeof(double)) + fbytes + P->frec_bytes;
    P->rk_ws_bytes = 2 * P->ws_bytes + 3 * align256(ndof * sizeof(double));
    P->fuse_next = P->dim == 2;
    P->vscr_bytes = align256((size_t)P->ne * esd::vjp_scratch_doubles(P->dim, P->p) * sizeof(double));
    P->vjp_ws_bytes = P->ws_bytes + fbytes + P->vscr_bytes;
    P->rk_vjp_ws_bytes = P->vjp_ws_bytes + 3 * align256(ndof * sizeof(double));
    if (P->host_only) {
      *out = P;
      return ESD_OK;
    }
    if (hipGetDevice(&P->device) != hipSuccess) {
      delete P;
      return fail(ESD_EHIP, "no HIP device");
    }
    // reference tables, packed
    std::vector<double> tb;
    std::vector<size_t> off;
    auto add = [&](const std::vector<double>& v) {
      off.push_back(tb.size());
      tb.insert(tb.end(), v.begin(), v.end());
    };
    add(R.psi1);
    add(R.psi2);
    add(R.psi3);
    add(R.lgm1);
    add(R.lgp1);
    add(R.gjm1);
    add(R.I42);
    add(R.A);
    add(R.wf);
    add(R.wl);
    add(R.wj);
    add(R.xl);
    add(R.psiM);
    esd_status st = upload(P, &P->d_tables, tb);
    if (st != ESD_OK) {
      free_device(P);
      delete P;
      return st;
    }
    const double* b = P->d_tables;
    P->tab = {b + off[0], b + off[1], b + off[2], b + off[3], b + off[4],  b + off[5],
              b + off[6], b + off[7], b + off[8], b + off[9], b + off[10], b + off[11], b + off[12]};
    // geometry
    st = upload(P, &P->d_gvol, pack_gvol(*P));
    const int NFQ = R.NFQ, NQF = R.NQF, dim = P->dim, NF = R.NF;
    std::vector<double> gf((size_t)P->ne * (dim + 1) * NFQ);
    std::vector<int32_t> conn((size_t)P->ne * NFQ);
    const int64_t stride = (int64_t)P->nc * NFQ;
    if ((int64_t)P->ne * stride >= std::numeric_limits<int32_t>::max()) {
      free_device(P);
      delete P;
      return fail(ESD_EUNSUPPORTED, "mesh too large for 32-bit facet addressing");
    }
    for (int64_t e = 0; e < P->ne; ++e)
      for (int j = 0; j < NFQ; ++j) {
        for (int m = 0; m < dim; ++m) gf[((size_t)e * (dim + 1) + m) * NFQ + j] = P->geo.nJ[((size_t)e * NFQ + j) * dim + m];
        gf[((size_t)e * (dim + 1) + dim) * NFQ + j] = P->geo.Jf[(size_t)e * NFQ + j];
        if (!connect) continue;
        const int64_t nb = P->geo.nbr[(size_t)e * NFQ + j];
        const int64_t ne_ = nb / NFQ, rem = nb % NFQ;
        const int64_t nf = rem / NQF, nn = rem % NQF;
        (void)NF;
        conn[(size_t)e * NFQ + j] = (int32_t)(ne_ * stride + nf * NQF + nn);
      }
    // the VJP gathers exterior cotangents through the same permutation, which
    // needs it to pair facet nodes both ways
    P->conn_involutive = connect;
    for (int64_t e = 0; e < P->ne && P->conn_involutive; ++e)
      for (int j = 0; j < NFQ; ++j) {
        const int64_t a = conn[(size_t)e * NFQ + j];
        const int64_t e2 = a / stride, j2 = a % stride;
        if (j2 >= NFQ || conn[(size_t)e2 * NFQ + j2] != (int32_t)(e * stride + j)) {
          P->conn_involutive = false;
          break;
        }
      }
    if (st == ESD_OK) st = upload(P, &P->d_gfac, gf);
    if (st == ESD_OK && connect) st = upload(P, &P->d_conn, conn);
    if (st == ESD_OK) st = upload(P, &P->d_xvol, P->geo.x_vol);
    if (st == ESD_OK) st = upload(P, &P->d_flag, std::vector<int>(1, 0));
    if (st != ESD_OK) {
      free_device(P);
      delete P;
      return st;
    }
  } catch (const std::exception& ex) {
    free_device(P);
    delete P;
    return fail(ESD_ENOMEM, std::string("setup failed: ") + ex.what());
  }
  *out = P;
  return ESD_OK;
}
}  // namespace

extern "C" {

esd_status esd_plan_create(const esd_mesh_desc* mesh, const esd_scheme_desc* scheme, uint32_t flags,
                           esd_plan** out) {
  if (!out) return fail(ESD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!mesh || !scheme) return fail(ESD_EINVAL, "mesh or scheme is NULL");
  return create_single(mesh, scheme, flags, true, out);
}

esd_status esd_plan_create_ex(const esd_mesh_desc* mesh, const esd_scheme_desc* scheme, uint32_t flags,
                              const esd_allocator* alloc, esd_plan** out) {
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(ESD_EINVAL, "allocator needs both functions");
  g_alloc = alloc;
  const esd_status st = esd_plan_create(mesh, scheme, flags, out);
  g_alloc = nullptr;
  return st;
}

esd_status esd_plan_create_batched_ex(const esd_batch_desc* batch, const esd_scheme_desc* scheme, uint32_t flags,
                                      const esd_allocator* alloc, esd_plan** out) {
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(ESD_EINVAL, "allocator needs both functions");
  g_alloc = alloc;
  const esd_status st = esd_plan_create_batched(batch, scheme, flags, out);
  g_alloc = nullptr;
  return st;
}

esd_status esd_plan_create_batched(const esd_batch_desc* d, const esd_scheme_desc* scheme, uint32_t flags,
                                   esd_plan** out) {
  if (!out) return fail(ESD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d || !scheme || d->n_meshes <= 0 || !d->n_elements || !d->elem_vertex_ids || !d->elem_vertex_coords ||
      !d->elem_degree)
    return fail(ESD_EINVAL, "bad batch description");
  if (d->dim != 2 && d->dim != 3) return fail(ESD_EUNSUPPORTED, "dim must be 2 or 3");
  if (!(scheme->gamma > 1.0) || scheme->ecflux < 0 || scheme->ecflux > 1 || scheme->dissipation < 0 ||
      scheme->dissipation > 3)
    return fail(ESD_EINVAL, "bad scheme parameters");
  const int dim = d->dim, nv = dim + 1, NF = dim + 1, nc = dim + 2;
  const bool host_only = (flags & 1u) != 0;
  esd_plan* P = new (std::nothrow) esd_plan();
  if (!P) return fail(ESD_ENOMEM, "host allocation failed");
  adopt_allocator(P);
  auto bail = [&](esd_status st, const std::string& m) {
    esd_plan_destroy(P);
    return fail(st, m);
  };
  try {
    P->batched = true;
    P->dim = dim;
    P->nc = nc;
    P->p = 0;
    P->host_only = host_only;
    P->scheme.gamma = scheme->gamma;
    P->scheme.gm1_inv = 1.0 / (scheme->gamma - 1.0);
    P->scheme.ecflux = scheme->ecflux;
    P->scheme.dissipation = scheme->dissipation;
    // ---- face adjacency and orientation of every mesh, from a degree-1 pass
    //      (orientation depends only on vertex ids and coordinates)
    const esd::RefTables r1 = esd::build_ref_tables(dim, 1);
    const int nqf1 = r1.NQF;
    std::vector<std::vector<int64_t>> nbr_e(d->n_meshes);
    std::vector<std::vector<int8_t>> nbr_f(d->n_meshes), flip(d->n_meshes);
    std::vector<int64_t> first(d->n_meshes + 1, 0);
    std::vector<int> present(esd::MAX_DEGREE + 1, 0);
    for (int m = 0; m < d->n_meshes; ++m) {
      const int64_t ne = d->n_elements[m];
      if (ne <= 0 || !d->elem_vertex_ids[m] || !d->elem_vertex_coords[m] || !d->elem_degree[m])
        return bail(ESD_EINVAL, "mesh " + std::to_string(m) + ": empty or NULL arrays");
      for (int64_t e = 0; e < ne; ++e) {
        const int p = d->elem_degree[m][e];
        if (!esd::degree_supported(dim, p))
          return bail(ESD_EUNSUPPORTED, "degree " + std::to_string(p) + " not built");
        present[p] = 1;
      }
      esd::HostGeometry g;
      std::string msg;
      const int rc = esd::build_geometry(r1, ne, d->elem_vertex_ids[m], d->elem_vertex_coords[m],
                                         (esd::warp_fn)d->warp, d->warp_ctx, g, msg, true);
      if (rc != 0) return bail((esd_status)rc, "mesh " + std::to_string(m) + ": " + msg);
      nbr_e[m].resize(ne * NF);
      nbr_f[m].resize(ne * NF);
      flip[m].resize(ne * NF);
      for (int64_t e = 0; e < ne; ++e)
        for (int f = 0; f < NF; ++f) {
          const int64_t nb = g.nbr[((size_t)e * NF + f) * nqf1];   // facet node 0 (a1 = a2 = 0)
          nbr_e[m][e * NF + f] = nb / (NF * nqf1);
          nbr_f[m][e * NF + f] = (int8_t)((nb / nqf1) % NF);
          flip[m][e * NF + f] = (int8_t)((nb % nqf1) % 2 == 1);    // its partner has a1 = Q - 1 = 1
        }
      first[m + 1] = first[m] + ne;
    }
    // ---- buckets by degree, slots in mesh order
    std::vector<int> degs;
    for (int p = 0; p <= esd::MAX_DEGREE; ++p)
      if (present[p]) degs.push_back(p);
    std::vector<int> bidx(esd::MAX_DEGREE + 1, -1);
    for (size_t b = 0; b < degs.size(); ++b) bidx[degs[b]] = (int)b;
    const int nb_ = (int)degs.size();
    P->elem_bucket.resize(first.back());
    P->elem_slot.resize(first.back());
    std::vector<std::vector<std::pair<int, int64_t>>> members(nb_);
    for (int m = 0; m < d->n_meshes; ++m)
      for (int64_t e = 0; e < d->n_elements[m]; ++e) {
        const int b = bidx[d->elem_degree[m][e]];
        P->elem_bucket[first[m] + e] = b;
        P->elem_slot[first[m] + e] = (int64_t)members[b].size();
        members[b].push_back({m, e});
      }
    // ---- one single-degree plan per bucket (geometry without connectivity)
    for (int b = 0; b < nb_; ++b) {
      const int64_t ne_b = (int64_t)members[b].size();
      std::vector<int64_t> ids(ne_b * nv);
      std::vector<double> xy(ne_b * nv * dim);
      for (int64_t i = 0; i < ne_b; ++i) {
        const int m = members[b][i].first;
        const int64_t e = members[b][i].second;
        for (int k = 0; k < nv; ++k) ids[i * nv + k] = d->elem_vertex_ids[m][e * nv + k];
        for (int k = 0; k < nv * dim; ++k) xy[i * nv * dim + k] = d->elem_vertex_coords[m][e * nv * dim + k];
      }
      esd_mesh_desc md{dim, degs[b], ne_b, ids.data(), xy.data(), d->warp, d->warp_ctx};
      esd_plan* sp = nullptr;
      const esd_status st = create_single(&md, scheme, flags, false, &sp);
      if (st != ESD_OK) {
        const std::string m = g_err;
        return bail(st, "bucket p=" + std::to_string(degs[b]) + ": " + m);
      }
      P->sub.push_back(sp);
    }
    // ---- facet permutation tables, mixed-interface tasks and matrices; the
    //      adjoint records of each task, keyed by the element whose w~ it reads
    std::vector<std::map<int64_t, std::vector<std::array<int32_t, 8>>>> arec(nb_);
    std::map<std::array<int, 4>, int> matid;
    std::vector<double> mats;
    std::vector<int64_t> mat_off;
    for (int b = 0; b < nb_; ++b) {
      esd_plan* sp = P->sub[b];
      const esd::RefTables& R = sp->ref;
      const int NFQ = R.NFQ, NQF = R.NQF, Q = R.Q;
      const int64_t ne_b = sp->ne, stride = (int64_t)nc * NFQ;
      if (2 * ne_b * stride >= std::numeric_limits<int32_t>::max())
        return bail(ESD_EUNSUPPORTED, "bucket too large for 32-bit facet addressing");
      std::vector<int32_t> conn(ne_b * NFQ);
      for (int64_t i = 0; i < ne_b; ++i) {
        const int m = members[b][i].first;
        const int64_t e = members[b][i].second;
        for (int f = 0; f < NF; ++f) {
          const int64_t en = nbr_e[m][e * NF + f];
          const int fn = nbr_f[m][e * NF + f];
          const bool fl = flip[m][e * NF + f] != 0;
          const int bn = P->elem_bucket[first[m] + en];
          const int64_t in = P->elem_slot[first[m] + en];
          if (bn == b) {
            for (int j = 0; j < NQF; ++j) {
              const int a1 = j % Q, a2 = j / Q;
              const int b1 = fl ? Q - 1 - a1 : a1;
              const int jb = dim == 2 ? b1 : b1 + Q * a2;
              conn[i * NFQ + f * NQF + j] = (int32_t)(in * stride + fn * NQF + jb);
            }
            continue;
          }
          for (int j = 0; j < NQF; ++j)
            conn[i * NFQ + f * NQF + j] = (int32_t)(ne_b * stride + i * stride + f * NQF + j);
          const int pn = degs[bn];
          const std::array<int, 4> key = {degs[b], pn, fn, fl ? 1 : 0};
          auto it = matid.find(key);
          if (it == matid.end()) {
            // the neighbour's PKD basis at the reference points of this degree's
            // facet nodes, carried across the shared facet (reversed Legendre
            // coordinate when the orientations differ)
            // stored transposed, [k][j]
            const int npn = esd::n_modes(dim, pn);
            const size_t base = mats.size();
            mat_off.push_back((int64_t)base);
            mats.resize(base + (size_t)npn * NQF);
            std::vector<double> row(npn);
            for (int j = 0; j < NQF; ++j) {
              const int a1 = j % Q, a2 = j / Q;
              const double sc = fl ? -R.xl[a1] : R.xl[a1];
              const double tc = dim == 3 ? R.xj[a2] : 0.0;
              double xi[3];
              esd::facet_point(dim, fn, sc, tc, xi);
              esd::pkd_eval(dim, pn, xi, 1, row.data());
              for (int k = 0; k < npn; ++k) mats[base + (size_t)k * NQF + j] = row[k];
            }
            it = matid.emplace(key, (int)mat_off.size() - 1).first;
          }
          arec[bn][in].push_back({b, (int32_t)i, f, it->second, (int32_t)in, NQF, NFQ, 0});
        }
      }
      // the VJP gathers exterior cotangents through the same permutation on
      // facets between equal degrees: it must pair those nodes both ways
      sp->conn_involutive = true;
      for (int64_t i = 0; i < ne_b && sp->conn_involutive; ++i)
        for (int j = 0; j < NFQ; ++j) {
          const int64_t a = conn[i * NFQ + j];
          if (a >= ne_b * stride) continue;   // exterior slot of a mixed-degree facet
          const int64_t i2 = a / stride, j2 = a % stride;
          if (j2 >= NFQ || conn[i2 * NFQ + j2] != (int32_t)(i * stride + j)) {
            sp->conn_involutive = false;
            break;
          }
        }
      if (!host_only) {
        esd_status st = upload(sp, &sp->d_conn, conn);
        if (st != ESD_OK) return bail(st, "upload failed");
      }
    }
    for (int b = 0; b < nb_; ++b) {
      esd_plan* sp = P->sub[b];
      std::vector<int32_t> recs, segs;
      for (const auto& kv : arec[b]) {   // target slots in increasing order
        segs.push_back((int32_t)(recs.size() / 8));
        segs.push_back((int32_t)kv.second.size());
        for (const auto& r : kv.second) recs.insert(recs.end(), r.begin(), r.end());
      }
      sp->n_asegs = (int64_t)segs.size() / 2;
      if (!host_only && sp->n_asegs > 0) {
        esd_status st = upload(sp, &sp->d_arecs, recs);
        if (st == ESD_OK) st = upload(sp, &sp->d_asegs, segs);
        if (st != ESD_OK) return bail(st, "upload failed");
      }
    }
    // ---- offsets and workspace
    P->dof_off.assign(nb_ + 1, 0);
    P->node_off.assign(nb_ + 1, 0);
    P->ws_off.assign(nb_, 0);
    size_t ws = 0;
    std::vector<int64_t> wt_off(nb_), wext_off(nb_);
    for (int b = 0; b < nb_; ++b) {
      esd_plan* sp = P->sub[b];
      P->dof_off[b + 1] = P->dof_off[b] + sp->ne * nc * sp->ref.NP;
      P->node_off[b + 1] = P->node_off[b] + sp->ne * sp->ref.NQ;
      P->ws_off[b] = ws;
      wt_off[b] = (int64_t)(ws / sizeof(double));
      // the exterior slots follow the own facet values (split_ws)
      wext_off[b] = (int64_t)((ws + align256((size_t)sp->ne * nc * sp->ref.NP * sizeof(double))) / sizeof(double)) +
                    sp->ne * nc * sp->ref.NFQ;
      ws += align256(sp->ws_bytes);
    }
    P->ne = first.back();
    const size_t ndof = (size_t)P->dof_off.back();
    P->ws_bytes = ws;
    P->rk_ws_bytes = 2 * ws + 3 * align256(ndof * sizeof(double));
    P->fuse_next = dim == 2;
    // VJP: the residual workspace, every bucket's x_bar, every bucket's slices
    P->xbar_off.assign(nb_, 0);
    P->vscr_off.assign(nb_, 0);
    std::vector<int64_t> xbar_off(nb_);
    size_t vws = ws;
    for (int b = 0; b < nb_; ++b) {
      const esd_plan* sp = P->sub[b];
      P->xbar_off[b] = vws;
      xbar_off[b] = (int64_t)(vws / sizeof(double));
      vws += align256((size_t)sp->ne * nc * sp->ref.NFQ * sizeof(double));
    }
    for (int b = 0; b < nb_; ++b) {
      P->vscr_off[b] = vws;
      vws += align256(P->sub[b]->vscr_bytes);
    }
    P->vjp_ws_bytes = vws;
    P->rk_vjp_ws_bytes = vws + 3 * align256(ndof * sizeof(double));
    if (!host_only) {
      if (hipGetDevice(&P->device) != hipSuccess) return bail(ESD_EHIP, "no HIP device");
      esd_status st = upload(P, &P->d_flag, std::vector<int>(1, 0));
      if (st == ESD_OK && !mats.empty()) st = upload(P, &P->d_mats, mats);
      if (st == ESD_OK && !mat_off.empty()) st = upload(P, &P->d_mat_off, mat_off);
      if (st == ESD_OK) st = upload(P, &P->d_wt_off, wt_off);
      if (st == ESD_OK) st = upload(P, &P->d_wext_off, wext_off);
      if (st == ESD_OK) st = upload(P, &P->d_xbar_off, xbar_off);
      if (st != ESD_OK) return bail(st, "upload failed");
      for (esd_plan* sp : P->sub) {
        dev_free(sp, sp->d_flag);
        sp->d_flag = P->d_flag;
        sp->flag_owned = false;
      }
    }
  } catch (const std::exception& ex) {
    return bail(ESD_ENOMEM, std::string("setup failed: ") + ex.what());
  }
  *out = P;
  return ESD_OK;
}

esd_status esd_plan_buckets(const esd_plan* P, int32_t* n_buckets, int32_t* degree, int64_t* n_elements,
                            int64_t* dof_offset, int64_t* node_offset) {
  if (!P || !n_buckets || !degree || !n_elements || !dof_offset || !node_offset)
    return fail(ESD_EINVAL, "NULL argument");
  if (!P->batched) {
    *n_buckets = 1;
    degree[0] = P->p;
    n_elements[0] = P->ne;
    dof_offset[0] = node_offset[0] = 0;
    dof_offset[1] = P->ne * P->nc * P->ref.NP;
    node_offset[1] = P->ne * P->ref.NQ;
    return ESD_OK;
  }
  const int nb = (int)P->sub.size();
  *n_buckets = nb;
  for (int b = 0; b < nb; ++b) {
    degree[b] = P->sub[b]->p;
    n_elements[b] = P->sub[b]->ne;
  }
  for (int b = 0; b <= nb; ++b) {
    dof_offset[b] = P->dof_off[b];
    node_offset[b] = P->node_off[b];
  }
  return ESD_OK;
}

esd_status esd_plan_element_map(const esd_plan* P, int32_t* bucket, int64_t* slot, int64_t count) {
  if (!P || !bucket || !slot) return fail(ESD_EINVAL, "NULL argument");
  if (count != P->ne) return fail(ESD_EINVAL, "count must equal the number of elements");
  for (int64_t i = 0; i < count; ++i) {
    bucket[i] = P->batched ? P->elem_bucket[i] : 0;
    slot[i] = P->batched ? P->elem_slot[i] : i;
  }
  return ESD_OK;
}

void esd_plan_destroy(esd_plan* plan) {
  if (!plan) return;
  for (esd_plan* b : plan->sub) esd_plan_destroy(b);
  for (auto& g : plan->graphs) (void)hipGraphExecDestroy(g.exec);
  if (plan->gev[0]) (void)hipEventDestroy(plan->gev[0]);
  if (plan->gev[1]) (void)hipEventDestroy(plan->gev[1]);
  if (plan->gstream) (void)hipStreamDestroy(plan->gstream);
  for (hipEvent_t e : plan->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : plan->ev_pool) (void)hipEventDestroy(e);
  free_device(plan);
  delete plan;
}

esd_status esd_plan_set_timing(esd_plan* P, int32_t enable) {
  if (!P) return fail(ESD_EINVAL, "plan is NULL");
  P->timing = enable != 0;
  return ESD_OK;
}

esd_status esd_plan_get_timing(esd_plan* P, double* k1_ms, double* k2_ms, int64_t* launches) {
  if (!P || !k1_ms || !k2_ms || !launches) return fail(ESD_EINVAL, "NULL argument");
  *k1_ms = *k2_ms = 0.0;
  *launches = 0;
  if (P->ev.size() % 3 != 0) return fail(ESD_EHIP, "incomplete timing record");
  for (size_t i = 0; i < P->ev.size(); i += 3) {
    HIP_TRY(hipEventSynchronize(P->ev[i + 2]));
    float a = 0.f, b = 0.f;
    HIP_TRY(hipEventElapsedTime(&a, P->ev[i], P->ev[i + 1]));
    HIP_TRY(hipEventElapsedTime(&b, P->ev[i + 1], P->ev[i + 2]));
    *k1_ms += a;
    *k2_ms += b;
    *launches += 1;
  }
  P->ev_pool.insert(P->ev_pool.end(), P->ev.begin(), P->ev.end());
  P->ev.clear();
  return ESD_OK;
}

esd_status esd_plan_query(const esd_plan* P, esd_plan_info* out) {
  if (!P || !out) return fail(ESD_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  if (P->batched) {
    out->dim = P->dim;
    out->n_vars = P->nc;
    out->n_facets = P->dim + 1;
    out->n_elements = P->ne;
    out->n_dof = P->dof_off.back();
    for (const esd_plan* b : P->sub) {
      esd_plan_info bi;
      esd_plan_query(b, &bi);
      out->flux_pairs_paper += bi.flux_pairs_paper;
      out->flux_pairs_distinct += bi.flux_pairs_distinct;
    }
    out->workspace_bytes = P->ws_bytes;
    out->rk4_workspace_bytes = P->rk_ws_bytes;
    out->vjp_workspace_bytes = P->vjp_ws_bytes;
    out->rk4_vjp_workspace_bytes = P->rk_vjp_ws_bytes;
    return ESD_OK;
  }
  const esd::RefTables& R = P->ref;
  out->dim = P->dim;
  out->degree = P->p;
  out->n_vars = P->nc;
  out->n_modes = R.NP;
  out->n_vol_nodes = R.NQ;
  out->n_facets = R.NF;
  out->n_facet_nodes = R.NQF;
  out->n_elements = P->ne;
  out->n_dof = P->ne * P->nc * R.NP;
  const int64_t Q = R.Q;
  int64_t paper, distinct;
  if (P->dim == 2) {
    paper = 3 * Q * Q * (Q + 1) / 2;          // 1.5 (q+1)^2 (q+2)
    distinct = Q * Q * (Q + 2);
  } else {
    paper = 4 * Q * Q * Q * Q;
    distinct = Q * Q * Q * (5 * Q + 3) / 2;   // (q+1)^3 (2.5 q + 4)
  }
  out->flux_pairs_paper = paper * P->ne;
  out->flux_pairs_distinct = distinct * P->ne;
  out->workspace_bytes = P->ws_bytes;
  out->rk4_workspace_bytes = P->rk_ws_bytes;
  out->vjp_workspace_bytes = P->vjp_ws_bytes;
  out->rk4_vjp_workspace_bytes = P->rk_vjp_ws_bytes;
  return ESD_OK;
}

esd_status esd_plan_host_array(const esd_plan* P, const char* name, double* out, int64_t count) {
  if (!P || !name || !out) return fail(ESD_EINVAL, "NULL argument");
  if (P->batched) return fail(ESD_EINVAL, "setup arrays of a batched plan are per bucket; not exposed");
  const std::string n(name);
  if (n == "nbr") {
    if ((int64_t)P->geo.nbr.size() != count) return fail(ESD_EINVAL, "count mismatch for nbr");
    for (int64_t i = 0; i < count; ++i) out[i] = (double)P->geo.nbr[i];
    return ESD_OK;
  }
  const std::vector<double>* v = nullptr;
  if (n == "x_vol") v = &P->geo.x_vol;
  else if (n == "J") v = &P->geo.J;
  else if (n == "G") v = &P->geo.G;
  else if (n == "nJ") v = &P->geo.nJ;
  else if (n == "Jf") v = &P->geo.Jf;
  else if (n == "x_fac") v = &P->geo.x_fac;
  if (!v) return fail(ESD_EINVAL, "unknown array " + n);
  if ((int64_t)v->size() != count) return fail(ESD_EINVAL, "count mismatch for " + n);
  std::memcpy(out, v->data(), v->size() * sizeof(double));
  return ESD_OK;
}

static esd_status check_device(const esd_plan* P) {
  if (!P) return fail(ESD_EINVAL, "plan is NULL");
  if (P->host_only) return fail(ESD_EINVAL, "host-only plan");
  return ESD_OK;
}

esd_status esd_node_coords(const esd_plan* P, double* x_dev, void* stream) {
  esd_status st = check_device(P);
  if (st != ESD_OK) return st;
  if (!x_dev) return fail(ESD_EINVAL, "x_dev is NULL");
  if (P->batched) {
    for (size_t b = 0; b < P->sub.size(); ++b)
      HIP_TRY(hipMemcpyAsync(x_dev + P->node_off[b] * P->dim, P->sub[b]->d_xvol,
                             P->sub[b]->geo.x_vol.size() * sizeof(double), hipMemcpyDeviceToDevice,
                             (hipStream_t)stream));
    return ESD_OK;
  }
  HIP_TRY(hipMemcpyAsync(x_dev, P->d_xvol, P->geo.x_vol.size() * sizeof(double), hipMemcpyDeviceToDevice,
                         (hipStream_t)stream));
  return ESD_OK;
}

esd_status esd_project(const esd_plan* P, const double* u_nodal_dev, double* u_dev, void* stream) {
  esd_status st = check_device(P);
  if (st != ESD_OK) return st;
  if (!u_nodal_dev || !u_dev) return fail(ESD_EINVAL, "NULL buffer");
  if (P->batched) {
    for (size_t b = 0; b < P->sub.size(); ++b) {
      const int rc = esd::launch_project(P->sub[b], u_nodal_dev + P->node_off[b] * P->nc, u_dev + P->dof_off[b],
                                         (hipStream_t)stream);
      if (rc != 0) return fail(ESD_EHIP, std::string("launch failed: ") + hipGetErrorString((hipError_t)rc));
    }
    return ESD_OK;
  }
  const int rc = esd::launch_project(P, u_nodal_dev, u_dev, (hipStream_t)stream);
  if (rc < 0) return fail(ESD_EUNSUPPORTED, "degree not built");
  if (rc != 0) return fail(ESD_EHIP, std::string("launch failed: ") + hipGetErrorString((hipError_t)rc));
  return ESD_OK;
}

static esd::Workspace split_ws(const esd_plan* P, void* ws) {
  const size_t ndof = (size_t)P->ne * P->nc * P->ref.NP;
  esd::Workspace w;
  w.wt = (double*)ws;
  w.wf = (double*)((char*)ws + align256(ndof * sizeof(double)));
  w.frec = P->frec_bytes ? (double*)((char*)ws + P->ws_bytes - P->frec_bytes) : nullptr;
  w.xbar = (double*)((char*)ws + P->ws_bytes);   // inside the workspace only for the VJP entry points
  w.vscr = (double*)((char*)ws + P->vjp_ws_bytes - P->vscr_bytes);
  return w;
}

static int64_t total_dof(const esd_plan* P) {
  return P->batched ? P->dof_off.back() : P->ne * P->nc * P->ref.NP;
}

// one residual evaluation; for a batched plan: K1 of every bucket, the
// mixed-interface exterior values, then K2 of every bucket
static esd::RkEpilogue shift(const esd::RkEpilogue& e, int64_t off) {
  esd::RkEpilogue r = e;
  if (r.acc) {
    r.u += off;
    r.acc += off;
    r.U += off;
  }
  return r;
}

static int residual_any(const esd_plan* P, const double* u, double* dudt, void* ws, hipStream_t s,
                        const esd::RkEpilogue& epi = esd::RkEpilogue()) {
  if (!P->batched) return esd::launch_residual(P, u, dudt, split_ws(P, ws), s, epi);
  const int nb = (int)P->sub.size();
  if (P->timing) esd::timing_event(P, s);
  for (int b = 0; b < nb; ++b) {
    const int rc = esd::launch_entropy_projection(P->sub[b], u + P->dof_off[b],
                                                  split_ws(P->sub[b], (char*)ws + P->ws_off[b]), s);
    if (rc != 0) return rc;
  }
  for (int b = 0; b < nb; ++b) {
    const int rc = esd::launch_mixed_exterior(P->sub[b], b, P, (const double*)ws, s);
    if (rc != 0) return rc;
  }
  if (P->timing) esd::timing_event(P, s);
  for (int b = 0; b < nb; ++b) {
    const int rc = esd::launch_rhs(P->sub[b], dudt + P->dof_off[b], split_ws(P->sub[b], (char*)ws + P->ws_off[b]), s,
                                   shift(epi, P->dof_off[b]));
    if (rc != 0) return rc;
  }
  if (P->timing) esd::timing_event(P, s);
  return 0;
}

esd_status esd_residual(const esd_plan* P, const double* u_dev, double* dudt_dev, void* ws_dev, void* stream) {
  esd_status st = check_device(P);
  if (st != ESD_OK) return st;
  if (!u_dev || !dudt_dev || !ws_dev) return fail(ESD_EINVAL, "NULL buffer");
  if ((const void*)u_dev == (const void*)dudt_dev) return fail(ESD_EINVAL, "u and dudt overlap");
  if (((uintptr_t)ws_dev) % 256 != 0) return fail(ESD_EINVAL, "workspace not 256-byte aligned");
  const int rc = residual_any(P, u_dev, dudt_dev, ws_dev, (hipStream_t)stream);
  if (rc < 0) return fail(ESD_EUNSUPPORTED, "degree not built");
  if (rc != 0) return fail(ESD_EHIP, std::string("launch failed: ") + hipGetErrorString((hipError_t)rc));
  return ESD_OK;
}

esd_status esd_residual_dense(const esd_plan* P, const double* u_dev, double* dudt_dev, void* ws_dev, void* stream) {
  esd_status st = check_device(P);
  if (st != ESD_OK) return st;
  if (P->batched) return fail(ESD_EUNSUPPORTED, "the all-pairs residual takes single-degree plans");
  if (!u_dev || !dudt_dev || !ws_dev) return fail(ESD_EINVAL, "NULL buffer");
  if ((const void*)u_dev == (const void*)dudt_dev) return fail(ESD_EINVAL, "u and dudt overlap");
  if (((uintptr_t)ws_dev) % 256 != 0) return fail(ESD_EINVAL, "workspace not 256-byte aligned");
  const int rc = esd::launch_residual_dense(P, u_dev, dudt_dev, split_ws(P, ws_dev), (hipStream_t)stream);
  if (rc < 0) return fail(ESD_EUNSUPPORTED, "degree not built");
  if (rc != 0) return fail(ESD_EHIP, std::string("launch failed: ") + hipGetErrorString((hipError_t)rc));
  return ESD_OK;
}

esd_status esd_residual_noalloc(const esd_plan* P, const double* u_dev, double* dudt_dev, void* stream) {
  esd_status st = check_device(P);
  if (st != ESD_OK) return st;
  if (!u_dev || !dudt_dev) return fail(ESD_EINVAL, "NULL buffer");
  if ((const void*)u_dev == (const void*)dudt_dev) return fail(ESD_EINVAL, "u and dudt overlap");
  if (P->timing) return fail(ESD_EINVAL, "kernel timing is enabled on this plan (it records events)");
  if (P->ws_bytes > esd::SCRATCH_BYTES)
    return fail(ESD_EINVAL, "residual workspace of " + std::to_string(P->ws_bytes) + " bytes exceeds the " +
                                std::to_string(esd::SCRATCH_BYTES) + "-byte library scratch");
  void* ws = nullptr;
  const int e = esd::scratch_address(&ws, nullptr);
  if (e != 0) return fail(ESD_EHIP, std::string("scratch address: ") + hipGetErrorString((hipError_t)e));
  const int rc = residual_any(P, u_dev, dudt_dev, ws, (hipStream_t)stream);
  if (rc < 0) return fail(ESD_EUNSUPPORTED, "degree not built");
  if (rc != 0) return fail(ESD_EHIP, std::string("launch failed: ") + hipGetErrorString((hipError_t)rc));
  return ESD_OK;
}

// one RK4 step: four residual evaluations, each right-hand-side kernel
// combining its stage into the accumulator and the next stage's input
// (classical RK4: u + dt/6 (k1 + 2 k2 + 2 k3 + k4))
static int rk4_step(const esd_plan* P, double* u_dev, double dt, void* ws_dev, double* ckpt, hipStream_t s) {
  const int64_t n = total_dof(P);
  const size_t nb = align256((size_t)n * sizeof(double));
  double* U = (double*)((char*)ws_dev + P->ws_bytes + nb);
  double* acc = (double*)((char*)ws_dev + P->ws_bytes + 2 * nb);
  const double ca[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};
  const double cu[4] = {0.5 * dt, 0.5 * dt, dt, 0.0};
  for (int stg = 0; stg < 4; ++stg) {
    const double* in = (stg == 0) ? u_dev : U;
    if (ckpt) {
      const hipError_t e = hipMemcpyAsync(ckpt + (int64_t)stg * n, in, n * sizeof(double), hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return (int)e;
    }
    esd::RkEpilogue epi;
    epi.u = u_dev;
    epi.acc = acc;
    epi.U = U;
    epi.ca = ca[stg];
    epi.cu = cu[stg];
    epi.first = stg == 0;
    epi.last = stg == 3;
    const int rc = residual_any(P, in, nullptr, ws_dev, s, epi);
    if (rc != 0) return rc;
  }
  return 0;
}

// entropy projection of u into the residual workspace ws (K1 of every bucket
// and, for a batched plan, the mixed-interface exterior values)
static int project_all(const esd_plan* P, const double* u, void* ws, hipStream_t s) {
  if (!P->batched) return esd::launch_entropy_projection(P, u, split_ws(P, ws), s);
  const int nb = (int)P->sub.size();
  for (int b = 0; b < nb; ++b) {
    const int rc = esd::launch_entropy_projection(P->sub[b], u + P->dof_off[b],
                                                  split_ws(P->sub[b], (char*)ws + P->ws_off[b]), s);
    if (rc != 0) return rc;
  }
  for (int b = 0; b < nb; ++b) {
    const int rc = esd::launch_mixed_exterior(P->sub[b], b, P, (const double*)ws, s);
    if (rc != 0) return rc;
  }
  return 0;
}

// one RK4 stage as right-hand-side kernels that also project the next stage
// input: reads the projection in cur, writes the next one to nxt
static int fused_stage(const esd_plan* P, void* cur, void* nxt, const esd::RkEpilogue& epi, hipStream_t s) {
  if (P->timing) {
    esd::timing_event(P, s);
    esd::timing_event(P, s);
  }
  if (!P->batched) {
    esd::RkEpilogue e = epi;
    const esd::Workspace wn = split_ws(P, nxt);
    e.wt_next = wn.wt;
    e.wf_next = wn.wf;
    const int rc = esd::launch_rhs(P, nullptr, split_ws(P, cur), s, e);
    if (rc != 0) return rc;
  } else {
    const int nb = (int)P->sub.size();
    for (int b = 0; b < nb; ++b) {
      esd::RkEpilogue e = shift(epi, P->dof_off[b]);
      const esd::Workspace wn = split_ws(P->sub[b], (char*)nxt + P->ws_off[b]);
      e.wt_next = wn.wt;
      e.wf_next = wn.wf;
      const int rc = esd::launch_rhs(P->sub[b], nullptr, split_ws(P->sub[b], (char*)cur + P->ws_off[b]), s, e);
      if (rc != 0) return rc;
    }
    for (int b = 0; b < nb; ++b) {
      const int rc = esd::launch_mixed_exterior(P->sub[b], b, P, (const double*)nxt, s);
      if (rc != 0) return rc;
    }
  }
  if (P->timing) esd::timing_event(P, s);
  return 0;
}

// one RK4 step from the projection of u held in the first residual workspace
// (A); the stages alternate between A and a second one (B) at the end of the
// RK workspace, and the last stage leaves the projection of the new u in A
static int rk4_step_fused(const esd_plan* P, double* u_dev, double dt, void* ws_dev, hipStream_t s) {
  const int64_t n = total_dof(P);
  const size_t nb = align256((size_t)n * sizeof(double));
  double* acc = (double*)((char*)ws_dev + P->ws_bytes + 2 * nb);
  void* A = ws_dev;
  void* B = (char*)ws_dev + P->ws_bytes + 3 * nb;
  const double ca[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};
  const double cu[4] = {0.5 * dt, 0.5 * dt, dt, 0.0};
  for (int stg = 0; stg < 4; ++stg) {
    esd::RkEpilogue epi;
    epi.u = u_dev;
    epi.acc = acc;
    epi.ca = ca[stg];
    epi.cu = cu[stg];
    epi.first = stg == 0;
    epi.last = stg == 3;
    const int rc = fused_stage(P, stg % 2 == 0 ? A : B, stg % 2 == 0 ? B : A, epi, s);
    if (rc != 0) return rc;
  }
  return 0;
}

// whether RK4 stages run fused (deterministic plans run them unfused)
static bool fused(const esd_plan* P) { return P->fuse_next && !P->deterministic; }

// nsteps RK4 steps launched kernel by kernel, fused or not as the plan says
static int rk4_eager(const esd_plan* P, double* u_dev, double dt, int nsteps, void* ws_dev, hipStream_t s) {
  if (fused(P)) {
    int rc = project_all(P, u_dev, ws_dev, s);
    for (int step = 0; step < nsteps && rc == 0; ++step) rc = rk4_step_fused(P, u_dev, dt, ws_dev, s);
    return rc;
  }
  int rc = 0;
  for (int step = 0; step < nsteps && rc == 0; ++step) rc = rk4_step(P, u_dev, dt, ws_dev, nullptr, s);
  return rc;
}

// the instantiated graph of one RK4 step for (u, ws, dt), captured on the
// plan's own stream at first use
static esd_status step_graph(const esd_plan* P, double* u_dev, double dt, void* ws_dev, hipGraphExec_t* exec) {
  for (const auto& g : P->graphs)
    if (g.u == u_dev && g.ws == ws_dev && g.dt == dt && g.fused == fused(P)) {
      *exec = g.exec;
      return ESD_OK;
    }
  if (!P->gstream) {
    HIP_TRY(hipStreamCreateWithFlags(&P->gstream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&P->gev[0], hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&P->gev[1], hipEventDisableTiming));
  }
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(P->gstream, hipStreamCaptureModeThreadLocal));
  const int rc = fused(P) ? rk4_step_fused(P, u_dev, dt, ws_dev, P->gstream)
                              : rk4_step(P, u_dev, dt, ws_dev, nullptr, P->gstream);
  const hipError_t ec = hipStreamEndCapture(P->gstream, &graph);
  if (rc != 0 || ec != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(ESD_EHIP, "graph capture failed");
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return fail(ESD_EHIP, std::string("graph instantiation: ") + hipGetErrorString(ei));
  if (P->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(P->graphs.front().exec);
    P->graphs.erase(P->graphs.begin());
  }
  P->graphs.push_back({u_dev, ws_dev, dt, fused(P), ex});
  *exec = ex;
  return ESD_OK;
}

esd_status esd_rk4(const esd_plan* P, double* u_dev, double dt, int32_t nsteps, void* ws_dev,
                   double* stage_ckpt_dev, void* stream) {
  esd_status st = check_device(P);
  if (st != ESD_OK) return st;
  if (!u_dev || !ws_dev || nsteps < 0 || !std::isfinite(dt)) return fail(ESD_EINVAL, "bad argument");
  if (((uintptr_t)ws_dev) % 256 != 0) return fail(ESD_EINVAL, "workspace not 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = total_dof(P);
  auto launch_rc = [](int rc) {
    if (rc < 0) return fail(ESD_EUNSUPPORTED, "degree not built");
    return fail(ESD_EHIP, std::string("RK4 launch failed: ") + hipGetErrorString((hipError_t)rc));
  };
  if (stage_ckpt_dev) {
    // stage inputs checkpointed for the adjoint: residual and stage kernels one by one
    for (int step = 0; step < nsteps; ++step) {
      const int rc = rk4_step(P, u_dev, dt, ws_dev, stage_ckpt_dev + (int64_t)4 * step * n, s);
      if (rc != 0) return launch_rc(rc);
    }
    return ESD_OK;
  }
  if (nsteps == 0) return ESD_OK;
  if (!P->timing && P->use_graphs) {
    // with fused stages the step starts from the projection of u in the first
    // residual workspace: project once, then replay
    if (fused(P)) {
      const int rc = project_all(P, u_dev, ws_dev, s);
      if (rc != 0) return launch_rc(rc);
    }
    hipGraphExec_t ex = nullptr;
    st = step_graph(P, u_dev, dt, ws_dev, &ex);
    if (st != ESD_OK) return st;
    // order the replays after the caller's stream and the caller's later work after them
    HIP_TRY(hipEventRecord(P->gev[0], s));
    HIP_TRY(hipStreamWaitEvent(P->gstream, P->gev[0], 0));
    for (int step = 0; step < nsteps; ++step) HIP_TRY(hipGraphLaunch(ex, P->gstream));
    HIP_TRY(hipEventRecord(P->gev[1], P->gstream));
    HIP_TRY(hipStreamWaitEvent(s, P->gev[1], 0));
    return ESD_OK;
  }
  const int rc = rk4_eager(P, u_dev, dt, nsteps, ws_dev, s);
  return rc == 0 ? ESD_OK : launch_rc(rc);
}

esd_status esd_plan_set_fused(esd_plan* P, int32_t enable) {
  if (!P) return fail(ESD_EINVAL, "plan is NULL");
  P->fuse_next = enable != 0;
  return ESD_OK;
}

esd_status esd_plan_set_deterministic(esd_plan* P, int32_t enable) {
  if (!P) return fail(ESD_EINVAL, "plan is NULL");
  P->deterministic = enable != 0;
  for (esd_plan* b : P->sub) b->deterministic = P->deterministic;
  // graphs captured before the change launch the other right-hand side
  if (P->gstream) (void)hipStreamSynchronize(P->gstream);
  for (auto& g : P->graphs) (void)hipGraphExecDestroy(g.exec);
  P->graphs.clear();
  return ESD_OK;
}

esd_status esd_plan_set_graphs(esd_plan* P, int32_t enable) {
  if (!P) return fail(ESD_EINVAL, "plan is NULL");
  P->use_graphs = enable != 0;
  return ESD_OK;
}

// K2 block size per bucket, timed on the given state: the full residual once
// (facet values of every bucket), then each candidate launch of each bucket's
// right-hand side three times after one warm-up; the fastest is kept.
esd_status esd_plan_autotune(esd_plan* P, const double* u_dev, void* ws_dev, void* stream) {
  esd_status st = check_device(P);
  if (st != ESD_OK) return st;
  if (!u_dev || !ws_dev) return fail(ESD_EINVAL, "NULL buffer");
  if (((uintptr_t)ws_dev) % 256 != 0) return fail(ESD_EINVAL, "workspace not 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  double* dudt = (double*)((char*)ws_dev + P->ws_bytes);   // inside the RK4 workspace
  const bool timing = P->timing;
  P->timing = false;
  int rc = residual_any(P, u_dev, dudt, ws_dev, s);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int nbk = P->batched ? (int)P->sub.size() : 1;
  for (int b = 0; b < nbk && rc == 0; ++b) {
    esd_plan* B = P->batched ? P->sub[b] : P;
    void* wsb = P->batched ? (char*)ws_dev + P->ws_off[b] : ws_dev;
    double* out = dudt + (P->batched ? P->dof_off[b] : 0);
    // K2 first (its inputs stay valid), then K1, which rewrites the facet values
    // with the same data
    for (int which = 2; which >= 1 && rc == 0; --which) {
      float best = 1e30f;
      int best_bs = 0;
      for (int bs : which == 2 ? esd::rhs_block_candidates(B->dim, B->p) : esd::k1_block_candidates(B->dim, B->p)) {
        (which == 2 ? B->k2_block : B->k1_block) = bs;
        auto launch = [&]() {
          return which == 2 ? esd::launch_rhs(B, out, split_ws(B, wsb), s)
                            : esd::launch_entropy_projection(B, u_dev + (P->batched ? P->dof_off[b] : 0),
                                                             split_ws(B, wsb), s);
        };
        rc = launch();
        if (rc != 0) break;
        HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < 3 && rc == 0; ++r) rc = launch();
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          best_bs = bs;
        }
      }
      (which == 2 ? B->k2_block : B->k1_block) = best_bs;
    }
  }
  // RK4 stages fused or not: four steps of each in one call (the fused call's
  // one projection of u then weighs a quarter step) after one untimed, with
  // dt = 0 (the same work) on a copy of u in the first state-sized buffer, run
  // as esd_rk4 runs them (graph replays unless graphs are off)
  esd_status trial = ESD_OK;
  if (rc == 0) {
    const int64_t n = total_dof(P);
    float best = 1e30f;
    bool best_f = P->fuse_next;
    for (int f = P->deterministic ? 0 : 1; f >= 0 && trial == ESD_OK; --f) {
      P->fuse_next = f != 0;
      HIP_TRY(hipMemcpyAsync(dudt, u_dev, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
      trial = esd_rk4(P, dudt, 0.0, 1, ws_dev, nullptr, stream);
      if (trial != ESD_OK) break;
      HIP_TRY(hipEventRecord(e0, s));
      trial = esd_rk4(P, dudt, 0.0, 4, ws_dev, nullptr, stream);
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_f = f != 0;
      }
    }
    P->fuse_next = best_f;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->timing = timing;
  // graphs captured before the change keep the old launch shape
  for (auto& g : P->graphs) (void)hipGraphExecDestroy(g.exec);
  P->graphs.clear();
  if (trial != ESD_OK) return trial;   // its message is already set
  if (rc < 0) return fail(ESD_EUNSUPPORTED, "degree not built");
  if (rc != 0) return fail(ESD_EHIP, std::string("autotune launch failed: ") + hipGetErrorString((hipError_t)rc));
  return ESD_OK;
}

esd_status esd_plan_get_tuning(const esd_plan* P, int32_t* k2_block, int32_t capacity) {
  if (!P || !k2_block) return fail(ESD_EINVAL, "NULL argument");
  const int nbk = P->batched ? (int)P->sub.size() : 1;
  if (capacity < nbk) return fail(ESD_EINVAL, "capacity below the number of buckets");
  for (int b = 0; b < nbk; ++b) {
    const esd_plan* B = P->batched ? P->sub[b] : P;
    k2_block[b] = B->k2_block > 0 ? B->k2_block : esd::rhs_block_candidates(B->dim, B->p)[0];
    if (capacity >= 2 * nbk) k2_block[nbk + b] = B->k1_block > 0 ? B->k1_block : esd::rhs_block_candidates(B->dim, B->p)[0];
  }
  if (capacity > 2 * nbk) k2_block[2 * nbk] = fused(P) ? 1 : 0;
  return ESD_OK;
}

// what the VJP entry points need of a plan (every bucket of a batch)
static esd_status vjp_check(const esd_plan* P) {
  if (P->scheme.dissipation > 1)
    return fail(ESD_EUNSUPPORTED, "VJP built for the entropy-conservative and Lax-Friedrichs interface fluxes");
  const int nbk = P->batched ? (int)P->sub.size() : 1;
  for (int b = 0; b < nbk; ++b) {
    const esd_plan* B = P->batched ? P->sub[b] : P;
    if (!B->conn_involutive) return fail(ESD_EUNSUPPORTED, "facet permutation is not an involution");
    if (!esd::vjp_degree_supported(B->dim, B->p)) return fail(ESD_EUNSUPPORTED, "VJP not built for this degree");
  }
  return ESD_OK;
}

// the VJP workspace slices of bucket b of a batch
static esd::Workspace vjp_ws_bucket(const esd_plan* P, int b, void* ws) {
  esd::Workspace w = split_ws(P->sub[b], (char*)ws + P->ws_off[b]);
  w.xbar = (double*)((char*)ws + P->xbar_off[b]);
  w.vscr = (double*)((char*)ws + P->vscr_off[b]);
  return w;
}

// one VJP; for a batch: K1 of every bucket, the mixed-interface exterior
// values, VK2 of every bucket, the mixed-interface adjoint (into the w~_bar
// of the elements the exterior values were read from), VK1 of every bucket
static int vjp_any(const esd_plan* P, const double* u, const double* vbar, double* grad, void* ws, hipStream_t s) {
  if (!P->batched) return esd::launch_vjp(P, u, vbar, grad, split_ws(P, ws), s);
  const int nb = (int)P->sub.size();
  int rc = 0;
  for (int b = 0; b < nb && rc == 0; ++b)
    rc = esd::launch_entropy_projection(P->sub[b], u + P->dof_off[b], vjp_ws_bucket(P, b, ws), s);
  for (int b = 0; b < nb && rc == 0; ++b)
    rc = esd::launch_mixed_exterior(P->sub[b], b, P, (const double*)ws, s);
  for (int b = 0; b < nb && rc == 0; ++b)
    rc = esd::launch_vjp_part(P->sub[b], 0, u + P->dof_off[b], vbar + P->dof_off[b], grad + P->dof_off[b],
                              vjp_ws_bucket(P, b, ws), s);
  for (int b = 0; b < nb && rc == 0; ++b)
    rc = esd::launch_mixed_exterior_vjp(P->sub[b], P, (const double*)ws, grad + P->dof_off[b], s);
  for (int b = 0; b < nb && rc == 0; ++b)
    rc = esd::launch_vjp_part(P->sub[b], 1, u + P->dof_off[b], vbar + P->dof_off[b], grad + P->dof_off[b],
                              vjp_ws_bucket(P, b, ws), s);
  return rc;
}

esd_status esd_residual_vjp(const esd_plan* P, const double* u_dev, const double* vbar_dev, double* grad_dev,
                            void* ws_dev, void* stream) {
  esd_status st = check_device(P);
  if (st != ESD_OK) return st;
  if (!u_dev || !vbar_dev || !grad_dev || !ws_dev) return fail(ESD_EINVAL, "NULL buffer");
  if ((const void*)grad_dev == (const void*)u_dev || (const void*)grad_dev == (const void*)vbar_dev)
    return fail(ESD_EINVAL, "grad overlaps u or vbar");
  if (((uintptr_t)ws_dev) % 256 != 0) return fail(ESD_EINVAL, "workspace not 256-byte aligned");
  st = vjp_check(P);
  if (st != ESD_OK) return st;
  const int rc = vjp_any(P, u_dev, vbar_dev, grad_dev, ws_dev, (hipStream_t)stream);
  if (rc < 0) return fail(ESD_EUNSUPPORTED, "degree not built");
  if (rc != 0) return fail(ESD_EHIP, std::string("VJP launch failed: ") + hipGetErrorString((hipError_t)rc));
  return ESD_OK;
}

esd_status esd_rk4_vjp(const esd_plan* P, const double* stage_ckpt_dev, double dt, int32_t nsteps, double* ubar_dev,
                       void* ws_dev, void* stream) {
  esd_status st = check_device(P);
  if (st != ESD_OK) return st;
  if (!stage_ckpt_dev || !ubar_dev || !ws_dev || nsteps < 0 || !std::isfinite(dt))
    return fail(ESD_EINVAL, "bad argument");
  if (((uintptr_t)ws_dev) % 256 != 0) return fail(ESD_EINVAL, "workspace not 256-byte aligned");
  st = vjp_check(P);
  if (st != ESD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = total_dof(P);
  const size_t nb = align256((size_t)n * sizeof(double));
  double* kb = (double*)((char*)ws_dev + P->vjp_ws_bytes);
  double* G = (double*)((char*)ws_dev + P->vjp_ws_bytes + nb);
  double* acc = (double*)((char*)ws_dev + P->vjp_ws_bytes + 2 * nb);
  // reverse of U_k = u + c_k dt k_{k-1}, u+ = u + dt/6 (k1 + 2 k2 + 2 k3 + k4)
  const double cu[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};   // weight of stage k in u+
  const double cs[4] = {0.5 * dt, 0.5 * dt, dt, 0.0};               // weight of k_k in U_{k+1}
  for (int step = nsteps - 1; step >= 0; --step) {
    int rc = esd::launch_scale(kb, ubar_dev, cu[3], n, s);
    for (int stg = 3; stg >= 0 && rc == 0; --stg) {
      const double* U = stage_ckpt_dev + ((int64_t)4 * step + stg) * n;
      rc = vjp_any(P, U, kb, G, ws_dev, s);
      if (rc != 0) break;
      if (stg > 0)
        rc = esd::launch_adj_stage(acc, kb, ubar_dev, G, cu[stg - 1], cs[stg - 1], stg == 3, n, s);
      else
        rc = esd::launch_axpy(ubar_dev, acc, 1.0, G, n, s);
    }
    if (rc < 0) return fail(ESD_EUNSUPPORTED, "degree not built");
    if (rc != 0) return fail(ESD_EHIP, std::string("adjoint launch failed: ") + hipGetErrorString((hipError_t)rc));
  }
  return ESD_OK;
}

esd_status esd_diagnostics(const esd_plan* P, const double* u_dev, double* out_host, void* ws_dev, void* stream) {
  esd_status st = check_device(P);
  if (st != ESD_OK) return st;
  if (!u_dev || !out_host || !ws_dev) return fail(ESD_EINVAL, "NULL buffer");
  if (((uintptr_t)ws_dev) % 256 != 0) return fail(ESD_EINVAL, "workspace not 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = total_dof(P);
  const size_t nb = align256((size_t)n * sizeof(double));
  const int no = P->nc + 2;
  // residual workspace, then du~/dt, then the partial sums and the results
  double* dudt = (double*)((char*)ws_dev + P->ws_bytes);
  double* part = (double*)((char*)ws_dev + P->ws_bytes + nb);
  double* res = part + P->ne * no;
  int rc = residual_any(P, u_dev, dudt, ws_dev, s);
  const int nbk = P->batched ? (int)P->sub.size() : 1;
  int64_t eoff = 0;
  for (int b = 0; b < nbk && rc == 0; ++b) {
    const esd_plan* B = P->batched ? P->sub[b] : P;
    const int64_t doff = P->batched ? P->dof_off[b] : 0;
    rc = esd::launch_diagnostics(B, u_dev + doff, dudt + doff, part + eoff * no, res + b * no, s);
    eoff += B->ne;
  }
  if (rc < 0) return fail(ESD_EUNSUPPORTED, "degree not built");
  if (rc != 0) return fail(ESD_EHIP, std::string("diagnostics launch failed: ") + hipGetErrorString((hipError_t)rc));
  std::vector<double> h((size_t)nbk * no);
  HIP_TRY(hipMemcpyAsync(h.data(), res, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int c = 0; c < no; ++c) {
    double acc = 0.0;
    for (int b = 0; b < nbk; ++b) acc += h[(size_t)b * no + c];
    out_host[c] = acc;
  }
  return ESD_OK;
}

esd_status esd_sync_status(const esd_plan* P, void* stream) {
  esd_status st = check_device(P);
  if (st != ESD_OK) return st;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  int flag = 0;
  HIP_TRY(hipMemcpy(&flag, P->d_flag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) {
    const int zero = 0;
    HIP_TRY(hipMemcpy(P->d_flag, &zero, sizeof(int), hipMemcpyHostToDevice));
    if (flag & 2) return fail(ESD_EINVAL, "entropy projection launched with fewer threads than its in-place stages need");
    return fail(ESD_EADMISSIBLE, "inadmissible state (rho <= 0, p <= 0 or non-finite) seen by a kernel");
  }
  return ESD_OK;
}

}  // extern "C"
