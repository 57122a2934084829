/*
 * esdsem.h -- C ABI of the MI355X (gfx950) library for the entropy-stable
 * modal discontinuous spectral-element method on curved triangles and
 * tetrahedra with tensor-product SBP operators in collapsed coordinates
 * (Montoya & Zingg, "Efficient entropy-stable discontinuous spectral-element
 * methods using tensor-product summation-by-parts operators on triangles and
 * tetrahedra").
 *
 * Conventions for every call
 *   - All floating point is IEEE binary64.
 *   - Pointers named *_dev are device (HBM) pointers on the plan's device;
 *     all other pointers are host pointers.
 *   - The caller owns every state, output, workspace and checkpoint buffer;
 *     the plan owns operator tables, geometry, connectivity and a status flag.
 *   - Compute calls are asynchronous on the given HIP stream (pass 0 for the
 *     null stream).  esd_plan_create, esd_plan_query, esd_plan_host_array and
 *     esd_sync_status synchronise with the host.
 *   - A non-zero status comes with a message from esd_last_error(); output
 *     buffers are then unspecified.  No C++ exception crosses the ABI.
 *
 * Data layout (element-major, SoA inside an element)
 *   modal state u~ : [element][variable][mode], N_c = dim+2 variables ordered
 *                    (rho, rho v_1..rho v_dim, E); modes of the orthonormal PKD
 *                    basis (Sec. 4.3) ordered by multi-index (a1, a2[, a3]) with
 *                    a1 outermost and the last index innermost.
 *   volume nodes   : tensor-product collapsed-coordinate nodes (Sec. 3),
 *                    index a1 + Q a2 [+ Q^2 a3], Q = p+1.
 *   Elements keep the order of the mesh description.  Each element's local
 *   vertex order is normalised by the library: the largest global vertex id
 *   becomes local vertex dim+1, in 3D the second largest becomes local vertex 3,
 *   the other two follow in increasing id order, swapped if the affine map
 *   would be orientation-reversing (Remark on connectivity, Sec. 6).
 */
#ifndef ESDSEM_H
#define ESDSEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct esd_plan esd_plan;          /* opaque, owned by the library */

typedef enum {
  ESD_OK = 0,
  ESD_EINVAL = -1,          /* bad argument (null pointer, size, enum)          */
  ESD_EJACOBIAN = -2,       /* mapping Jacobian <= 0 at a node (eq. jacobian_positive) */
  ESD_EADMISSIBLE = -3,     /* rho <= 0, p <= 0 or non-finite state seen by a kernel (sticky) */
  ESD_EUNSUPPORTED = -4,    /* degree or dimension not built into the library   */
  ESD_ENONCONFORMING = -5,  /* facet nodes of neighbours do not coincide (Assumption conformal) */
  ESD_EHIP = -6,            /* a HIP runtime call failed                        */
  ESD_ENOMEM = -7           /* device allocation failed                         */
} esd_status;

/* Entropy-conservative two-point flux used in the volume and facet terms. */
typedef enum {
  ESD_FLUX_RANOCHA = 0,       /* eq. (ranocha_flux), Sec. 7.2                    */
  ESD_FLUX_CHANDRASHEKAR = 1  /* Chandrashekar's EC flux (cited in Sec. 4.6)     */
} esd_ecflux;

/* Interface dissipation of eq. (num_flux). */
typedef enum {
  ESD_DISS_NONE = 0,          /* entropy-conservative interface flux (Sec. 7.2)  */
  ESD_DISS_LLF_DAVIS = 1,     /* local Lax-Friedrichs with eq. (wave_speed)      */
  /* the entropy-stable alternatives named after eq. (num_flux), both on the
   * jump of the entropy variables, A0 = dU/dW at the arithmetic-mean state
   * (rho, v, p); forward only (the VJP entry points return ESD_EUNSUPPORTED): */
  ESD_DISS_ENTROPY_JUMP = 2,  /* scalar: lambda/2 A0 (w+ - w-), lambda of eq. (wave_speed) */
  ESD_DISS_MATRIX = 3         /* matrix: 1/2 |A_n| A0 (w+ - w-), |A_n| the absolute Euler flux Jacobian */
} esd_dissipation;

/* Maps n points x_in [n][dim] (physical, unwarped) to x_out [n][dim].  Called
 * on the host during esd_plan_create with the affine images of the mapping
 * nodes of eq. (poly_mapping); NULL means no warp (affine elements). */
typedef void (*esd_warp_fn)(int64_t n, const double* x_in, double* x_out, void* ctx);

typedef struct {
  int32_t dim;                         /* 2 (triangles) or 3 (tetrahedra)          */
  int32_t degree;                      /* p = q = p_g for every element (Sec. 7.3); built:
                                          1..10 (triangles and tetrahedra), the VJP
                                          entry points included                     */
  int64_t n_elements;
  const int64_t* elem_vertex_ids;      /* host [n_elements][dim+1] global ids; periodic
                                          images of a vertex share one id           */
  const double* elem_vertex_coords;    /* host [n_elements][dim+1][dim] physical coords */
  esd_warp_fn warp;                    /* may be NULL                               */
  void* warp_ctx;
} esd_mesh_desc;

typedef struct {
  double gamma;                        /* ratio of specific heats, > 1 (Sec. 7.1)  */
  int32_t ecflux;                      /* esd_ecflux                               */
  int32_t dissipation;                 /* esd_dissipation                          */
} esd_scheme_desc;

typedef struct {
  int32_t dim, degree, n_vars, n_modes;   /* N_c, N_p* per element                  */
  int32_t n_vol_nodes, n_facets, n_facet_nodes;   /* per element; n_facet_nodes per facet */
  int64_t n_elements;
  int64_t n_dof;                          /* n_elements * n_vars * n_modes          */
  int64_t flux_pairs_paper;               /* per residual, count of eq. (num_fluxes) */
  int64_t flux_pairs_distinct;            /* per residual, pairs evaluated by the line loops */
  size_t workspace_bytes;                 /* esd_residual workspace                 */
  size_t rk4_workspace_bytes;             /* esd_rk4 workspace                      */
  size_t vjp_workspace_bytes;             /* esd_residual_vjp workspace             */
  size_t rk4_vjp_workspace_bytes;         /* esd_rk4_vjp workspace                  */
} esd_plan_info;

/* Builds operators (Sec. 3, 4.3), geometry (Sec. 4.1-4.2, 4.5) and facet
 * connectivity (Assumption conformal) on the host and uploads them to the
 * current HIP device.  Synchronous.  Errors: ESD_EINVAL, ESD_EUNSUPPORTED,
 * ESD_EJACOBIAN, ESD_ENONCONFORMING, ESD_ENOMEM, ESD_EHIP.  flags: bit 0 set =
 * host-only plan (no device allocation; only esd_plan_query and
 * esd_plan_host_array may be used with it). */
esd_status esd_plan_create(const esd_mesh_desc* mesh, const esd_scheme_desc* scheme,
                           uint32_t flags, esd_plan** out);

/* Device allocator for the plan's own arrays (operator tables, geometry,
 * connectivity, status flag), so that a caller such as PyTorch owns that
 * memory too: alloc(bytes, ctx) returns a 256-byte aligned device pointer on
 * the current device, or NULL (the call then fails with ESD_ENOMEM);
 * free(ptr, ctx) releases it (called from esd_plan_destroy, and on failed
 * creation).  Both are called on the creating thread during creation. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} esd_allocator;

/* esd_plan_create / esd_plan_create_batched with a device allocator (NULL:
 * hipMalloc and hipFree, as the plain calls).  ESD_EINVAL if one of the two
 * functions is missing or a pointer is not 256-byte aligned. */
esd_status esd_plan_create_ex(const esd_mesh_desc* mesh, const esd_scheme_desc* scheme, uint32_t flags,
                              const esd_allocator* alloc, esd_plan** out);
void esd_plan_destroy(esd_plan* plan);
esd_status esd_plan_query(const esd_plan* plan, esd_plan_info* out);

/* Several independent meshes whose elements carry their own degrees, in one
 * plan.  Elements are grouped into buckets by degree (all meshes together;
 * ascending degree; within a bucket, in mesh order then element order); every
 * bucket runs its degree's kernels.  Across a facet whose two elements have
 * different degrees, the exterior state at a facet node is the neighbour's
 * modal entropy expansion at the node's reference point on the shared facet
 * (for equal degrees this is the conforming rule of Assumption conformal; with
 * a change of degree the scheme is not conservative or entropy stable there).
 * Vertex ids are per mesh; the warp applies to every mesh. */
typedef struct {
  int32_t dim;
  int32_t n_meshes;
  const int64_t* n_elements;                 /* host [n_meshes]                              */
  const int64_t* const* elem_vertex_ids;     /* host [n_meshes] -> [n_elements][dim+1]      */
  const double* const* elem_vertex_coords;   /* host [n_meshes] -> [n_elements][dim+1][dim] */
  const int32_t* const* elem_degree;         /* host [n_meshes] -> [n_elements]             */
  esd_warp_fn warp;                          /* may be NULL                                  */
  void* warp_ctx;
} esd_batch_desc;

/* Builds a batched plan (see esd_batch_desc).  Its state is
 * [bucket][element-in-bucket][variable][mode], nodal arrays (esd_project,
 * esd_node_coords) are [bucket][element-in-bucket][node][...]; offsets from
 * esd_plan_buckets.  esd_residual, esd_rk4, esd_project, esd_node_coords,
 * esd_diagnostics, esd_sync_status and the VJP entry points accept it (the
 * VJP also differentiates the exterior values of mixed-degree facets with
 * respect to the neighbour's w~); esd_plan_host_array returns ESD_EINVAL.
 * Its VJP workspace is the residual workspace followed by, per bucket, the
 * exterior cotangents (n_elements N_c N_fq doubles, 256-byte aligned) and
 * then, per bucket, the adjoint kernels' slices (tetrahedra at p = 9, 10).
 * Errors as esd_plan_create. */
esd_status esd_plan_create_batched(const esd_batch_desc* batch, const esd_scheme_desc* scheme, uint32_t flags,
                                   esd_plan** out);
esd_status esd_plan_create_batched_ex(const esd_batch_desc* batch, const esd_scheme_desc* scheme, uint32_t flags,
                                      const esd_allocator* alloc, esd_plan** out);

/* Buckets of a plan (a single-degree plan has one): count, degree[b],
 * n_elements[b], and offsets dof_offset[b] (doubles into the state) and
 * node_offset[b] (volume nodes into nodal arrays), b = 0..n (n + 1 entries).
 * The arrays hold at least 16 (17 for the offsets) entries. */
esd_status esd_plan_buckets(const esd_plan* plan, int32_t* n_buckets, int32_t* degree, int64_t* n_elements,
                            int64_t* dof_offset, int64_t* node_offset);

/* Bucket and slot of every input element (meshes concatenated in order);
 * count must equal info.n_elements. */
esd_status esd_plan_element_map(const esd_plan* plan, int32_t* bucket, int64_t* slot, int64_t count);

/* Copies a host-side setup array of the plan into out (count doubles).  Names:
 * "x_vol" [e][node][dim] physical volume-node coordinates, "J" [e][node]
 * interpolated Jacobian (eq. jacobian_approx), "G" [e][node][l][m] metric terms
 * (Sec. 4.2), "nJ" [e][facet][node][dim] = G^T nhat (eq. nanson), "Jf"
 * [e][facet][node], "x_fac" [e][facet][node][dim], "nbr" [e][facet][node]
 * neighbour element*facets*nodes + facet*nodes + node (as doubles).  Returns
 * ESD_EINVAL for an unknown name or wrong count. */
esd_status esd_plan_host_array(const esd_plan* plan, const char* name, double* out, int64_t count);

/* Physical coordinates of the volume quadrature nodes, [element][node][dim]. */
esd_status esd_node_coords(const esd_plan* plan, double* x_dev, void* stream);

/* Weight-adjusted L2 projection of nodal values given at the volume quadrature
 * nodes, u~ = Mt^{-1} V^T W J u (eqs. weight_adjusted_inverse, dudt_modal with
 * M = I): u_nodal_dev [element][node][variable] -> u_dev [element][variable][mode]. */
esd_status esd_project(const esd_plan* plan, const double* u_nodal_dev, double* u_dev, void* stream);

/* Semi-discrete right-hand side du~/dt = Mt^{-1} V^T r(u~) of eq. (dudt_modal)
 * with r of eq. (entropy_stable): entropy projection (eq. entropy_expansion),
 * line-by-line flux differencing (eq. flux_differencing, Remark on lines),
 * facet correction (eq. facet_correction), interface flux (eq. num_flux) and the
 * weight-adjusted inverse (eq. matvec_dudt).  u_dev and dudt_dev are
 * [element][variable][mode] and must not overlap; ws_dev holds
 * info.workspace_bytes (256-byte aligned).  Admissibility violations set the
 * sticky flag read by esd_sync_status. */
esd_status esd_residual(const esd_plan* plan, const double* u_dev, double* dudt_dev,
                        void* ws_dev, void* stream);

/* The same residual as esd_residual evaluated as a dense (multidimensional)
 * SBP operator would: every volume node against every volume node (N_q^2
 * two-point fluxes per element, eq. flux_differencing with dense S^l) and
 * against every facet node (N_q N_f N_qf, eq. facet_correction with dense
 * R^T B), the coefficients being those of the tensor-product operators (zero
 * off their collapsed-coordinate lines).  Measures the O(p^{2d}) formulation
 * against the O(p^{d+1}) line-based one of esd_residual on the same nodes
 * (Sec. 5.1, 5.3).  Single-degree plans only (ESD_EUNSUPPORTED otherwise);
 * arguments and errors as esd_residual. */
esd_status esd_residual_dense(const esd_plan* plan, const double* u_dev, double* dudt_dev, void* ws_dev,
                              void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * residual as esd_residual, with its workspace taken from a library-owned
 * device array of 64 MiB per GPU (allocated when the library is loaded on that
 * GPU and held until the process ends) instead of a caller buffer.  The call
 * allocates nothing.  u_dev and dudt_dev as for esd_residual.  Errors:
 * ESD_EINVAL if info.workspace_bytes exceeds 64 MiB (use esd_residual), if
 * kernel timing is enabled on the plan, or for NULL/overlapping buffers;
 * ESD_EUNSUPPORTED, ESD_EHIP as esd_residual.  All calls on one GPU share the
 * array: two calls that overlap in time on the same GPU (different streams, or
 * host threads) race and give wrong results.  Every workspace byte the call
 * reads is written earlier in the same call, so nothing needs clearing. */
esd_status esd_residual_noalloc(const esd_plan* plan, const double* u_dev, double* dudt_dev, void* stream);

/* nsteps steps of classical four-stage Runge-Kutta with step dt, in place on
 * u_dev.  ws_dev holds info.rk4_workspace_bytes (two residual workspaces and
 * three state-sized buffers).  Every stage is the residual (K1 entropy
 * projection, K2 right-hand side) with the stage combination formed by K2.
 * With fused stages (esd_plan_set_fused) and no checkpoints, the call projects
 * u once and then runs every stage as one right-hand-side launch per bucket
 * that also projects the next stage input, alternating between the two
 * residual workspaces.  If stage_ckpt_dev is not NULL it receives the four
 * stage inputs U1..U4 of every step, [4*nsteps][n_dof] (stages then unfused). */
esd_status esd_rk4(const esd_plan* plan, double* u_dev, double dt, int32_t nsteps,
                   void* ws_dev, double* stage_ckpt_dev, void* stream);

/* RK4 execution: without checkpoints and with timing off, esd_rk4 captures one
 * step (its four stage launches per bucket) into a HIP graph on the
 * plan's own stream at the first call for a given (u_dev, ws_dev, dt), and
 * replays it nsteps times, ordered after the caller's stream by events.
 * esd_plan_set_graphs(plan, 0) launches every kernel individually instead. */
esd_status esd_plan_set_graphs(esd_plan* plan, int32_t enable);

/* Whether esd_rk4 fuses each stage's right-hand side with the next stage's
 * entropy projection (one launch per stage and bucket instead of two; the
 * projection then runs at the right-hand-side kernel's occupancy).  Default:
 * fused for triangles; esd_plan_autotune keeps the faster of the two. */
esd_status esd_plan_set_fused(esd_plan* plan, int32_t enable);

/* Bitwise-repeatable right-hand side (default off).  The sums of
 * eqs. (flux_differencing) and (facet_correction) then run in a fixed order:
 * the volume pairs of one line family at a time, each node's pairs summed in
 * registers by the lane that owns it (partners' data passed between the lanes
 * of a line), and C^T 1 summed per facet node over its partners (each facet
 * pair evaluated twice, once from each side) instead of through LDS atomics,
 * whose order varies from run to run.  Results of esd_residual, esd_rk4 and
 * esd_diagnostics are then identical bit for bit across runs on the same
 * device and build; they differ from the default at rounding level.  RK4
 * stages run unfused; the VJP entry points are unaffected (their sums keep
 * LDS atomics).  Applies to every bucket of a batch; drops the plan's captured
 * RK4 graphs (after waiting for their replays).  Call while no other work of
 * the plan is in flight. */
esd_status esd_plan_set_deterministic(esd_plan* plan, int32_t enable);

/* Chooses the block sizes of the right-hand-side kernel (K2) and of the
 * entropy-projection kernel (K1) for every bucket by timing the candidates
 * (multiples of 64 up to their compiled bound) on the state u_dev, then
 * whether RK4 stages are fused (esd_plan_set_fused) by timing steps both ways
 * on a copy of u_dev; ws_dev holds info.rk4_workspace_bytes.  Synchronises.
 * The choice is kept by the plan and reported by esd_plan_get_tuning:
 * k2_block[bucket], and, when capacity allows 2 n_buckets entries, the K1 block
 * sizes in k2_block[n_buckets + bucket], and with one more entry the fusion
 * flag (1 fused) in k2_block[2 n_buckets]. */
esd_status esd_plan_autotune(esd_plan* plan, const double* u_dev, void* ws_dev, void* stream);
esd_status esd_plan_get_tuning(const esd_plan* plan, int32_t* k2_block, int32_t capacity);

/* Vector-Jacobian product of the semi-discrete right-hand side (the adjoint of
 * esd_residual, differentiating eqs. entropy_expansion, entropy_stable,
 * facet_correction, num_flux and dudt_modal exactly, including the interface
 * coupling to the neighbours):
 *   grad_dev = (d du~/dt / d u~)^T vbar_dev,  all [element][variable][mode].
 * The wave speed of eq. (wave_speed) is a max, not differentiable where its
 * arguments agree: where they agree to 1e-10 relative (a tie up to rounding)
 * the derivative is the mean of the two one-sided derivatives, elsewhere that
 * of the larger argument (|x| has derivative 0 at 0).  grad_dev must not overlap
 * u_dev or vbar_dev; ws_dev holds info.vjp_workspace_bytes (256-byte aligned;
 * for tetrahedra at p = 9, 10 it includes a slice per element for the arrays
 * of the adjoint kernels that do not fit in LDS).
 * Errors: ESD_EINVAL, ESD_EUNSUPPORTED (degree not built, or facet nodes not
 * paired both ways), ESD_EHIP; inadmissible states set the sticky flag. */
esd_status esd_residual_vjp(const esd_plan* plan, const double* u_dev, const double* vbar_dev,
                            double* grad_dev, void* ws_dev, void* stream);

/* Discrete adjoint of nsteps steps of esd_rk4 (classical four-stage
 * Runge-Kutta) with step dt.  stage_ckpt_dev holds the stage inputs written by
 * esd_rk4, [4*nsteps][n_dof].  On entry ubar_dev is the cotangent of the final
 * state, on exit that of the initial state (in place).  ws_dev holds
 * info.rk4_vjp_workspace_bytes (256-byte aligned). */
esd_status esd_rk4_vjp(const esd_plan* plan, const double* stage_ckpt_dev, double dt, int32_t nsteps,
                       double* ubar_dev, void* ws_dev, void* stream);

/* Global diagnostics of the state u_dev, written to out_host [dim + 4]:
 *   out[0..dim+1]  conserved integrals sum_k w_k J_k u_k per variable (Theorem on
 *                  conservation);
 *   out[dim+2]     entropy integral sum_k w_k J_k S(u_k), S = -rho s/(gamma-1)
 *                  (eq. euler_entropy);
 *   out[dim+3]     its semi-discrete rate sum_k w_k J_k W(u_k) . (V du~/dt)_k,
 *                  zero to rounding with the entropy-conservative interface flux,
 *                  <= 0 with dissipation (Theorems on entropy conservation and
 *                  stability);
 * with u = V u~ at the volume nodes and J the interpolated Jacobian.  Evaluates
 * the residual internally; ws_dev holds info.rk4_workspace_bytes (256-byte
 * aligned).  Synchronises the stream.  The sums are reduced in a fixed order
 * (bitwise reproducible for a given plan). */
esd_status esd_diagnostics(const esd_plan* plan, const double* u_dev, double* out_host, void* ws_dev,
                           void* stream);

/* Synchronises the stream and returns ESD_EADMISSIBLE if any kernel since the
 * last call saw an inadmissible state, ESD_EINVAL if an entropy projection
 * was launched with fewer threads than its in-place transform stages need
 * (tetrahedra at p = 10; the library's own launches never do), else ESD_OK;
 * the flag is cleared. */
esd_status esd_sync_status(const esd_plan* plan, void* stream);

/* Kernel timing for measurement: when enabled, every K1 (entropy projection)
 * and K2 (right-hand side) launch of esd_residual is bracketed by HIP events
 * on the stream it is launched on, and so is every stage of esd_rk4 (counted
 * as K2, its fused kernels including the next projection, with K1 time 0).
 * esd_plan_get_timing synchronises, returns the summed milliseconds and launch
 * counts since the last reset, and resets them.  Timing is off by default. */
esd_status esd_plan_set_timing(esd_plan* plan, int32_t enable);
esd_status esd_plan_get_timing(esd_plan* plan, double* k1_ms, double* k2_ms, int64_t* launches);

/* Thread-local message describing the last failure. */
const char* esd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ESDSEM_H */
