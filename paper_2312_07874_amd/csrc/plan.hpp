// Plan object shared by the C ABI (api.cpp) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "host_setup.hpp"
#include "physics.hpp"

namespace esd {

// Device pointers to the per-degree reference tables (all FP64, see RefTables).
struct DevTables {
  const double* psi1;   // [P+1][Q]
  const double* psi2;   // [P+1][P+1][Q]
  const double* psi3;   // [P+1][P+1][Q]
  const double* lgm1;   // [Q]
  const double* lgp1;   // [Q]
  const double* gjm1;   // [Q]
  const double* I42;    // [Q][Q]
  const double* A;      // [5][Q][Q]
  const double* wf;     // [NF][NQF]
  const double* wl;     // [Q]
  const double* wj;     // [Q]
  const double* xl;     // [Q]
  const double* psiM;   // [P+1][Q][Q] line compositions of V V^T
};

// Classical RK4 stage combination fused into the right-hand-side kernel's
// output (acc == nullptr: plain du~/dt output).  With k = du~/dt of the stage:
//   stages 1-3:  acc = (first ? u : acc) + ca k,  U = u + cu k
//   stage 4:     u = acc + ca k   (in place on the state)
// All pointers address the same state layout as du~/dt.
// With wt_next set, the kernel also projects the next stage input (U, or the
// new u at stage 4) of its elements, kept in LDS instead of U, into wt_next and
// wf_next (the other of two residual workspaces).
struct RkEpilogue {
  double* u = nullptr;
  double* acc = nullptr;
  double* U = nullptr;
  double* wt_next = nullptr;
  double* wf_next = nullptr;
  double ca = 0.0, cu = 0.0;
  int first = 0, last = 0;
};

// Scheme constants passed to kernels.
struct Scheme {
  double gamma;
  double gm1_inv;       // 1/(gamma-1)
  int ecflux;
  int dissipation;
};

// Per-element geometric data on the device (element-major):
//   gvol [e][NGV][NQ]  scaled metric rows for the line families, then w*J, w/J
//     tri : h1(2) = w2 g1, h2(2) = (w2/2) g2, h2'(2) = (w1/2) g2           NGV = 8
//     tet : h1(3) = (w2 w3/2) g1, h23(3) = (w2 w3/4)(g2+g3),
//           h2(3) = (w1 w3/4) g2, h3(3) = (w1 w3/8) g3,
//           hz(3) = (w1 w2 (1-eta2)/8) g3                                    NGV = 17
//   gfac [e][dim+1][NFQ]  G^T nhat (dim rows), J_f
//   conn [e][NFQ]         neighbour address in the facet-state buffer:
//                          nbr_e*NC*NFQ + nbr_facet*NQF + nbr_node
inline int ngv(int dim) { return dim == 2 ? 8 : 17; }

struct Workspace {
  double* wt;     // [ne][NC][NP]  projected entropy variables (modal)
  double* wf;     // [ne][NC][NFQ] projected entropy variables at facet nodes
  double* xbar;   // [ne][NC][NFQ] VJP only: cotangent of the neighbour's facet value seen at each own facet node
  double* vscr;   // VJP only: per-element slices for the adjoint arrays that do not fit LDS (high degree)
  double* frec;   // [ne][8][NFQ] own facet node records, only for degrees whose right-hand side
                  // does not fit them in LDS (else nullptr)
};

}  // namespace esd

struct esd_plan {
  int dim = 0, p = 0, nc = 0;
  int64_t ne = 0;
  esd::Scheme scheme{};
  esd::RefTables ref;
  esd::HostGeometry geo;
  bool host_only = false;
  int device = 0;
  double* d_tables = nullptr;
  esd::DevTables tab{};
  double* d_gvol = nullptr;
  double* d_gfac = nullptr;
  int32_t* d_conn = nullptr;
  double* d_xvol = nullptr;
  int* d_flag = nullptr;
  bool flag_owned = true;         // false for buckets sharing the batched plan's flag
  // device allocator of the plan's own arrays (null members: hipMalloc / hipFree)
  void* (*dev_alloc)(size_t, void*) = nullptr;
  void (*dev_free)(void*, void*) = nullptr;
  void* alloc_ctx = nullptr;
  size_t ws_bytes = 0;
  size_t frec_bytes = 0;          // tail of the residual workspace holding Workspace::frec
  size_t rk_ws_bytes = 0;
  size_t vjp_ws_bytes = 0;
  size_t vscr_bytes = 0;          // tail of the VJP workspace holding Workspace::vscr
  size_t rk_vjp_ws_bytes = 0;
  bool conn_involutive = false;   // facet permutation pairs nodes both ways (needed by the VJP gather)
  // measurement: events bracketing each K1 / K2 launch (mutable: recorded by const calls)
  // mixed-degree batches: elements of this degree out of several meshes; the
  // facet-state region of the workspace holds 2 ne slots (own values, then the
  // exterior values of facets whose neighbour has another degree)
  bool wext = false;
  // the facets of other buckets whose exterior values read the w~ of this
  // bucket's elements, grouped by that element (see batch.hip): records
  // [n_arecs][8], segments [n_asegs][2] (first, count); used by the
  // mixed-interface kernel and its adjoint
  int32_t* d_arecs = nullptr;
  int32_t* d_asegs = nullptr;
  int64_t n_asegs = 0;
  // batched plan: container of one single-degree plan per bucket
  bool batched = false;
  std::vector<esd_plan*> sub;
  std::vector<int64_t> dof_off;   // [nb+1] offsets of the buckets in the state (doubles)
  std::vector<int64_t> node_off;  // [nb+1] offsets in volume nodes
  std::vector<size_t> ws_off;     // [nb] residual workspace slice of each bucket (bytes)
  std::vector<int32_t> elem_bucket;   // per input element (meshes concatenated)
  std::vector<int64_t> elem_slot;
  double* d_mats = nullptr;       // mixed-interface evaluation matrices
  int64_t* d_mat_off = nullptr;   // [n_mats] offsets into d_mats
  int64_t* d_wt_off = nullptr;    // [nb] offsets (doubles) of each bucket's w~ in the workspace
  int64_t* d_wext_off = nullptr;  // [nb] offsets (doubles) of each bucket's exterior facet values
  // VJP workspace of a batch: the residual workspace, then per bucket its
  // x_bar (ne NC NFQ doubles) and its adjoint scratch slices
  std::vector<size_t> xbar_off, vscr_off;   // [nb] bytes from the workspace start
  int64_t* d_xbar_off = nullptr;  // [nb] the x_bar offsets in doubles
  int k2_block = 0;               // right-hand-side block size chosen by esd_plan_autotune (0: default)
  int k1_block = 0;               // entropy-projection block size chosen likewise
  // RK4 steps replayed from a captured graph (no checkpoints, no timing)
  // (the cache below is filled by const compute calls, hence mutable)
  bool use_graphs = true;
  // RK4 stages as right-hand-side kernels that also project the next stage
  // input (else K1 and K2 per stage); set at creation (triangles), by
  // esd_plan_autotune (the faster on the device) or esd_plan_set_fused
  bool fuse_next = false;
  // right-hand side with fixed-order sums instead of LDS atomics (bitwise
  // repeatable); set by esd_plan_set_deterministic; RK4 stages then unfused
  bool deterministic = false;
  mutable hipStream_t gstream = nullptr;
  mutable hipEvent_t gev[2] = {nullptr, nullptr};
  struct GraphEntry {
    const void* u;
    const void* ws;
    double dt;
    bool fused;
    hipGraphExec_t exec;
  };
  mutable std::vector<GraphEntry> graphs;
  bool timing = false;
  mutable std::vector<hipEvent_t> ev;       // triples: before K1, between, after K2
  mutable std::vector<hipEvent_t> ev_pool;
};

namespace esd {
// kernel launchers (kernels.hip); return hipError_t as int, or -1 for an
// unsupported degree
int launch_residual(const esd_plan* P, const double* u, double* dudt, Workspace ws, hipStream_t s,
                    const RkEpilogue& epi = RkEpilogue());
int launch_project(const esd_plan* P, const double* u_nodal, double* u, hipStream_t s);
// the residual with all-pairs (dense-operator) volume and facet loops
int launch_residual_dense(const esd_plan* P, const double* u, double* dudt, Workspace ws, hipStream_t s);
int launch_axpy(double* y, const double* x, double a, const double* z, int64_t n, hipStream_t s);
int launch_entropy_projection(const esd_plan* P, const double* u, Workspace ws, hipStream_t s);
// adjoint.hip
int launch_vjp(const esd_plan* P, const double* u, const double* vbar, double* grad, Workspace ws,
               hipStream_t s);
// VK2 (which = 0: partial w~_bar into grad, x_bar) or VK1 (which = 1) alone
int launch_vjp_part(const esd_plan* P, int which, const double* u, const double* vbar, double* grad, Workspace ws,
                    hipStream_t s);
int launch_adj_stage(double* acc, double* kb, const double* ubar, const double* G, double cu, double cg, int first,
                     int64_t n, hipStream_t s);
int launch_scale(double* y, const double* x, double a, int64_t n, hipStream_t s);
// K2 alone (K1 must have run for every element whose facet values it reads)
int launch_rhs(const esd_plan* P, double* dudt, Workspace ws, hipStream_t s, const RkEpilogue& epi = RkEpilogue());
// batch.hip: exterior facet values of mixed-degree interfaces of one bucket
// (bucket bi of top: the facets that read the w~ of its elements)
int launch_mixed_exterior(const esd_plan* bucket, int bi, const esd_plan* top, const double* ws_base, hipStream_t s);
// and its adjoint: w~_bar of this bucket's elements (grad, the bucket's slice)
// += I^T x_bar of the facets that read them (VJP workspace at ws_base)
int launch_mixed_exterior_vjp(const esd_plan* bucket, const esd_plan* top, const double* ws_base, double* grad,
                              hipStream_t s);
hipEvent_t timing_event(const esd_plan* pl, hipStream_t s);
// diagnostics.hip: part [ne][dim+4] partial sums, out [dim+4] (device)
int launch_diagnostics(const esd_plan* P, const double* u, const double* dudt, double* part, double* out,
                       hipStream_t s);
bool degree_supported(int dim, int p);
bool vjp_degree_supported(int dim, int p);
bool needs_facet_records(int dim, int p);   // the residual workspace holds Workspace::frec
int vjp_scratch_doubles(int dim, int p);    // per element, of Workspace::vscr (0 if none)
std::vector<int> rhs_block_candidates(int dim, int p);
std::vector<int> k1_block_candidates(int dim, int p);
}  // namespace esd
