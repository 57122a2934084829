// HIP kernels (gfx950, FP64) for the entropy-stable modal DSEM residual.
//
// Two kernels per residual evaluation (one global dependency: neighbours'
// facet values must exist before the interface flux is formed):
//
//   K1  entropy projection, per element (eqs. entropy_expansion,
//       matvec_entropy_projection):  u = V u~;  w~ = V^T (w/J) V V^T (w J) W(u);
//       w^z = R^z V w~ written to HBM for the neighbours.
//   K2  right-hand side, per element (eqs. entropy_stable, facet_correction,
//       flux_differencing, num_flux, matvec_dudt): w = V w~, u_bar = U(w) at
//       volume and facet nodes; line-by-line flux differencing (each unordered
//       pair of a collapsed-coordinate line evaluated once, with the summed
//       direction sum_l S^l_ab (g_l(a)+g_l(b)), the line organisation the paper
//       leaves to future work); facet correction along the same lines (faces
//       1-3) and across the eta2-eta3 planes (face 4); interface flux with
//       optional Lax-Friedrichs dissipation; r -= R^T (B J_f f* - C^T 1);
//       du~/dt = V^T (w/J) V V^T r.
//
// Sum-factorised PKD transforms (Sec. 5.2) run out of LDS; one element (tet)
// or several (triangles) per workgroup; one thread per collapsed line in the
// flux phase with the line's accumulators in registers; no global atomics.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.hpp"

namespace esd {

// ------------------------------------------------------------------ K1: entropy projection
// K1 keeps every transform stage inside its nodal array (xform_V_inplace) at
// tet p = 10: the separate first-stage scratch would leave one workgroup per
// CU (115 KB of LDS); inside, 80.6 KB with both PKD tables staged, two.  Each
// thread then holds K1_MAXT middle-stage tasks, so K1 launches with at least
// k1_min_block threads there.
template <int DIM, int P>
struct K1Inplace {
  static constexpr bool ON = DIM == 3 && P == 10;
  static constexpr int MAXT = 2;
  static constexpr int TASKS = (DIM + 2) * (P + 1) * (P + 1);   // middle-stage tasks per element
  static constexpr int MIN_BLOCK = ON ? ((TASKS + MAXT - 1) / MAXT + 63) / 64 * 64 : 64;
  static constexpr int WAVES = ON ? 4 : 1;   // waves per SIMD the registers must allow
};

// w~ = V^T (w/J) V V^T b for b = (w J W) at the volume nodes in sA [nel*NC][NQ]
// (eqs. entropy_expansion, matvec_entropy_projection); result in sM; aI holds
// w/J at this thread's first nodes; VVT: V V^T as one composed transform (its
// table staged); INPLACE: every stage inside sA (xform_V_inplace, K1 only:
// sM is then sA's start and sS unused).  Ends with a barrier.
template <int DIM, int P, bool VVT, bool INPLACE = false>
__device__ __forceinline__ void weight_adjusted_projection(double* sM, double* sA, double* sS, const DevTables& T,
                                                           const double* __restrict__ gvol, int64_t e0, int nel,
                                                           const Ahead<2>& aI) {
  using Sh = Shape<DIM, P>;
  constexpr int EPB = Launch<DIM, P>::EPB;
  constexpr int NC = Sh::NC, NQ = Sh::NQ, NGV = Sh::NGV;
  const int nec = nel * NC;
  double* T1 = sS;
  double* T2 = sA;   // the tetrahedral middle layout runs in place over the nodal values
  using IP = K1Inplace<DIM, P>;
  auto ld_wi = [&](int o) { return gvol[((e0 + o / NQ) * NGV + NGV - 1) * NQ + o % NQ]; };
  if constexpr (INPLACE) {
    static_assert(!VVT && IP::ON, "in-place stages: tet p = 10, without the composed transform");
    xform_Vt_inplace<P, IP::MAXT>(sA, T, nec);
    xform_V_inplace<P, IP::MAXT>(sA, T, nec);
  } else if constexpr (VVT) {
    xform_VVt<DIM, P, MfmaEta1<P>::ON_PROJ>(sA, T1, T2, sA, T, nec);
  } else {
    xform_Vt<DIM, P, MfmaEta1<P>::ON_PROJ>(sA, T1, T2, sM, T, nec);
    xform_V<DIM, P, MfmaEta1<P>::ON_PROJ>(sM, T1, T2, sA, T, nec);
  }
  aI.each(nel * NQ, ld_wi, [&](int o, double wi) {
    const int k = o % NQ, el = o / NQ;
#pragma unroll
    for (int c = 0; c < NC; ++c) sA[(el * NC + c) * NQ + k] *= wi;
  });
  __syncthreads();
  if constexpr (INPLACE) xform_Vt_inplace<P, IP::MAXT>(sA, T, nec);
  else xform_Vt<DIM, P, MfmaEta1<P>::ON_PROJ>(sA, T1, T2, sM, T, nec);
}

// Entropy projection of a block of elements whose modal state u~ is in sM
// [nel*NC][NP] (after a barrier): u = V u~, b = w J W(u), w~ by the
// weight-adjusted projection, written to wt, and the facet values R V w~
// (eqs. r_2d, r_3d) to wf.  aJ and aI hold w J and w/J at this thread's first
// nodes.  Uses sA [nel*NC][NQ] and the transform scratch sS.
template <int DIM, int P, bool VVT, bool INPLACE = false>
__device__ __forceinline__ void project_block(double* sM, double* sA, double* sS, const DevTables& T,
                                              const double* __restrict__ gvol, const Scheme& S, int64_t e0,
                                              int nel, int* flag, double* __restrict__ wt, double* __restrict__ wf,
                                              const Ahead<2>& aJ, const Ahead<2>& aI) {
  using Sh = Shape<DIM, P>;
  constexpr int EPB = Launch<DIM, P>::EPB;
  constexpr int NC = Sh::NC, NQ = Sh::NQ, NP = Sh::NP, NFQ = Sh::NFQ, NGV = Sh::NGV;
  const int nec = nel * NC;
  const int tid = threadIdx.x, nth = blockDim.x;
  double* T1 = sS;
  double* T2 = sA;
  using IP = K1Inplace<DIM, P>;
  auto ld_wJ = [&](int o) { return gvol[((e0 + o / NQ) * NGV + NGV - 2) * NQ + o % NQ]; };
  if constexpr (INPLACE) xform_V_inplace<P, IP::MAXT>(sA, T, nec);
  else xform_V<DIM, P, MfmaEta1<P>::ON_PROJ>(sM, T1, T2, sA, T, nec);
  // entropy variables times w J at every volume node
  bool bad = false;
  aJ.each(nel * NQ, ld_wJ, [&](int o, double wJ) {
    const int k = o % NQ, el = o / NQ;
    double* a = sA + el * NC * NQ;
    const double rho = a[k];
    double v2 = 0.0, v[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      v[i] = a[(1 + i) * NQ + k] / rho;
      v2 += v[i] * v[i];
    }
    const double p = (S.gamma - 1.0) * (a[(DIM + 1) * NQ + k] - 0.5 * rho * v2);
    bad |= !(rho > 0.0) || !(p > 0.0) || !isfinite(rho) || !isfinite(p);
    const double s = log(p) - S.gamma * log(rho);
    a[k] = wJ * ((S.gamma - s) * S.gm1_inv - 0.5 * rho * v2 / p);
#pragma unroll
    for (int i = 0; i < DIM; ++i) a[(1 + i) * NQ + k] = wJ * (rho * v[i] / p);
    a[(DIM + 1) * NQ + k] = wJ * (-rho / p);
  });
  if (bad) atomicOr(flag, 1);
  __syncthreads();
  weight_adjusted_projection<DIM, P, VVT, INPLACE>(sM, sA, sS, T, gvol, e0, nel, aI);
  for (int o = tid; o < nec * NP; o += nth) wt[e0 * NC * NP + o] = sM[o];
  // facet values of the projected entropy variables, w^z = R^z V w~
  if constexpr (INPLACE) xform_V_inplace<P, IP::MAXT>(sA, T, nec);
  else xform_V<DIM, P, MfmaEta1<P>::ON_PROJ>(sM, T1, T2, sA, T, nec);
  double* wfe = wf + e0 * NC * NFQ;
  facet_values<DIM, P>(sA, sS, T, nec, [&](int o, double v) { wfe[o] = v; });
}

template <int DIM, int P, bool PROJECT_ONLY>
__global__ void __launch_bounds__((Launch<DIM, P>::BSMAX))
__attribute__((amdgpu_waves_per_eu(K1Inplace<DIM, P>::WAVES)))   // in place: two 512-thread workgroups per CU
k_entropy_projection(const double* __restrict__ u, double* __restrict__ wt, double* __restrict__ wf,
                     const double* __restrict__ gvol, DevTables T0, Scheme S, int64_t ne, int* flag) {
  using Sh = Shape<DIM, P>;
  constexpr int EPB = Launch<DIM, P>::EPB;
  constexpr int NC = Sh::NC, NQ = Sh::NQ, NP = Sh::NP, NGV = Sh::NGV;
  // the modal arrays share sA's storage: each transform reads its input in
  // its first stage and writes its output in its last, so the modal input of
  // V and the modal output of V^T never coexist with the nodal values; the
  // tetrahedral middle stage runs in place over sA too, so the transform
  // scratch is the first stage's alone (which also holds the facet scratch)
  using IP = K1Inplace<DIM, P>;
  // with in-place stages the scratch is only the facet extrapolation's
  constexpr int SS = IP::ON ? NC * Sh::Q * Sh::Q : Sh::T1;
  __shared__ double sA[EPB * NC * NQ];
  __shared__ double sS[EPB * SS];
  double* const sM = sA;
  static_assert(NP <= NQ, "modal arrays fit in the nodal array");
  static_assert(DIM == 2 || SS >= NC * Sh::Q * Sh::Q, "facet scratch fits in the transform scratch");
  static_assert(!IP::ON || EPB == 1, "in-place stages assume one element per workgroup");
  constexpr int KB = 8 * EPB * (NC * NQ + SS);
  // the composed V V^T table only where it keeps the workgroups per CU; where
  // the two PKD tables do not fit (tetrahedra at p = 10), psi2 alone
  constexpr unsigned TM0 = tab_keeps_wgs<DIM, P, TAB_PSI | TAB_FACET, TAB_PSI | TAB_FACET | TAB_PSIM>(KB, wave_cap<DIM, P>())
                               ? (TAB_PSI | TAB_FACET | TAB_PSIM)
                               : tab_mask<DIM, P, TAB_PSI | TAB_FACET>(KB);
  constexpr unsigned TM = TM0 != 0 ? TM0 : (DIM == 3 ? tab_mask<DIM, P, TAB_PSI2>(KB) : 0u);
  constexpr bool VVT = (TM & TAB_PSIM) != 0;
  __shared__ double sTab[TM ? TabLds<DIM, P, TM>::SIZE : 1];
  const DevTables T = stage_tables<DIM, P, TM>(T0, sTab);
  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const int nel = (int)((ne - e0) < EPB ? (ne - e0) : EPB);
  const int nec = nel * NC;
  const int tid = threadIdx.x, nth = blockDim.x;
  if constexpr (IP::ON) {
    // the launch keeps blockDim >= IP::MIN_BLOCK; refuse (flag bit 2) rather
    // than skip middle-stage tasks
    if (nth * IP::MAXT < IP::TASKS) {
      if (tid == 0) atomicOr(flag, 2);
      return;
    }
  }
  // w J and w/J at this thread's nodes, used after the first transforms
  auto ld_wJ = [&](int o) { return gvol[((e0 + o / NQ) * NGV + NGV - 2) * NQ + o % NQ]; };
  auto ld_wi = [&](int o) { return gvol[((e0 + o / NQ) * NGV + NGV - 1) * NQ + o % NQ]; };
  Ahead<2> aJ, aI;
  if constexpr (PROJECT_ONLY) {
    aI.load(nel * NQ, ld_wi);
    // u holds nodal values [e][node][var]; b = w J u
    for (int o = tid; o < nel * NQ * NC; o += nth) {
      const int c = o % NC, k = (o / NC) % NQ, el = o / (NC * NQ);
      const double wJ = gvol[((e0 + el) * NGV + NGV - 2) * NQ + k];
      sA[(el * NC + c) * NQ + k] = wJ * u[(e0 * NQ) * NC + o];
    }
    __syncthreads();
    weight_adjusted_projection<DIM, P, VVT, IP::ON>(sM, sA, sS, T, gvol, e0, nel, aI);
    for (int o = tid; o < nec * NP; o += nth) wt[e0 * NC * NP + o] = sM[o];
  } else {
    aJ.load(nel * NQ, ld_wJ);
    aI.load(nel * NQ, ld_wi);
    for (int o = tid; o < nec * NP; o += nth) sM[o] = u[e0 * NC * NP + o];
    __syncthreads();
    project_block<DIM, P, VVT, IP::ON>(sM, sA, sS, T, gvol, S, e0, nel, flag, wt, wf, aJ, aI);
  }
}

// ------------------------------------------------------------------ K2 helpers
// One volume task: node a of the line base + stride*k; pairs (a, b) with
// F = f#(u_a, u_b, n_ab), n_ab = A0_ab (h0_a + h0_b) [+ A1_ab (h1_a + h1_b)],
// r_a -= F, r_b += F.
template <int DIM, int P, int FLUX, int NA>
__device__ __forceinline__ void vol_task(const double* sN, const double* __restrict__ g, double* sR, int base,
                                         int stride, int a, const double* __restrict__ A0,
                                         const double* __restrict__ A1, int hc0, int hc1, const Scheme& S) {
  using Sh = Shape<DIM, P>;
  constexpr int Q = Sh::Q, NQ = Sh::NQ, NC = Sh::NC;
  const int na = base + stride * a;
  const Node<DIM> Na = load_node<DIM>(sN, NQ, na);
  double h0a[DIM], h1a[DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    h0a[i] = g[(hc0 + i) * NQ + na];
    if constexpr (NA == 2) h1a[i] = g[(hc1 + i) * NQ + na];
  }
  double racc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) racc[c] = 0.0;
  auto pair = [&](int b) {
    const int nb = base + stride * b;
    const Node<DIM> Nb = load_node<DIM>(sN, NQ, nb);
    double n[DIM];
    const double c0 = A0[a * Q + b];
#pragma unroll
    for (int i = 0; i < DIM; ++i) n[i] = c0 * (h0a[i] + g[(hc0 + i) * NQ + nb]);
    if constexpr (NA == 2) {
      const double c1 = A1[a * Q + b];
#pragma unroll
      for (int i = 0; i < DIM; ++i) n[i] += c1 * (h1a[i] + g[(hc1 + i) * NQ + nb]);
    }
    double F[NC];
    ec_flux<DIM, FLUX>(Na, Nb, n, S.gm1_inv, F);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      racc[c] -= F[c];
      atomicAdd(&sR[c * NQ + nb], F[c]);
    }
  };
#pragma unroll
  for (int k = 1; k <= (Q - 1) / 2; ++k) {
    int b = a + k;
    b = (b >= Q) ? b - Q : b;
    pair(b);
  }
  if constexpr (Q % 2 == 0) {
    if (a < Q / 2) pair(a + Q / 2);
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) atomicAdd(&sR[c * NQ + na], racc[c]);
}

// Volume pairs of one line family, deterministic form: the Q lanes of a
// line sit in one wave (64 / Q whole lines per wave), lane a owning node a of
// the line base + stride*k.  In step k = 1..(Q-1)/2 lane a evaluates the pair
// (a, a+k mod Q) exactly as vol_task does, keeps -F and passes F to the
// partner's lane (a rotation of the line's lanes, through ds_bpermute), which
// also hands it the partner's metrics; for even Q step Q/2 pairs a < Q/2 with
// a + Q/2.  r_a is summed in registers in a fixed order and added to LDS once
// (the caller runs one family at a time, so each node has one owner).  Lanes
// of no line (ok false) shadow a valid line and drop their result.
template <int DIM, int P, int FLUX, int NA>
__device__ __forceinline__ void vol_line(const double* sN, const double* __restrict__ g, double* sR, int base,
                                         int stride, int a, int lbase, bool ok, const double* __restrict__ A0,
                                         const double* __restrict__ A1, int hc0, int hc1, const Scheme& S) {
  using Sh = Shape<DIM, P>;
  constexpr int Q = Sh::Q, NQ = Sh::NQ, NC = Sh::NC;
  const int na = base + stride * a;
  const Node<DIM> Na = load_node<DIM>(sN, NQ, na);
  double h0a[DIM], h1a[DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    h0a[i] = g[(hc0 + i) * NQ + na];
    h1a[i] = NA == 2 ? g[(hc1 + i) * NQ + na] : 0.0;
  }
  double racc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) racc[c] = 0.0;
  auto step = [&](int k, bool half) {
    int b = a + k;
    b = b >= Q ? b - Q : b;
    int src = a - k;
    src = src < 0 ? src + Q : src;
    const int nb = base + stride * b;
    const Node<DIM> Nb = load_node<DIM>(sN, NQ, nb);
    double n[DIM];
    const double c0 = A0[a * Q + b];
#pragma unroll
    for (int i = 0; i < DIM; ++i) n[i] = c0 * (h0a[i] + __shfl(h0a[i], lbase + b));
    if constexpr (NA == 2) {
      const double c1 = A1[a * Q + b];
#pragma unroll
      for (int i = 0; i < DIM; ++i) n[i] += c1 * (h1a[i] + __shfl(h1a[i], lbase + b));
    }
    double F[NC];
    ec_flux<DIM, FLUX>(Na, Nb, n, S.gm1_inv, F);
    const bool keep = !half || a < Q / 2;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double f = keep ? F[c] : 0.0;
      racc[c] += __shfl(f, lbase + src) - f;
    }
  };
#pragma unroll
  for (int k = 1; k <= (Q - 1) / 2; ++k) step(k, false);
  if constexpr (Q % 2 == 0) step(Q / 2, true);
  if (ok) {
#pragma unroll
    for (int c = 0; c < NC; ++c) sR[c * NQ + na] += racc[c];
  }
}

// One facet-correction pair (eq. facet_correction): C = coef f#(u_i, u^z_j, (gn_i + nJ_j)/2);
// r_i -= C (registers), and with ATOM s_j -= C (LDS atomics; s_j starts as the
// interface term).  Without ATOM the caller sums s_j by facet node
// (facet_node_sum).
template <int DIM, int P, int FLUX, bool ATOM = true>
__device__ __forceinline__ void facet_task(const Node<DIM>& Vi, const double* gn_i, const double* sF, double* sT,
                                           const double* __restrict__ gf, int j, double coef, const Scheme& S,
                                           double* racc) {
  constexpr int NC = DIM + 2, NFQ = Shape<DIM, P>::NFQ;
  const Node<DIM> Fj = load_node<DIM>(sF, NFQ, j);
  double n[DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i) n[i] = 0.5 * (gn_i[i] + gf[i * NFQ + j]);
  double F[NC];
  ec_flux<DIM, FLUX>(Vi, Fj, n, S.gm1_inv, F);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double C = coef * F[c];
    racc[c] -= C;
    if constexpr (ATOM) atomicAdd(&sT[c * NFQ + j], -C);
  }
}

// G^T nhat at volume node i for the facets its lines reach (facet_correction's
// {J n} on the volume side), from the pre-scaled metric rows: triangles
// gA (facet 2), gB (facet 3), gC (facet 1); tetrahedra also gD (facet 4).
template <int P>
__device__ __forceinline__ void tri_volume_normals(const double* __restrict__ g, int i, int b1, int b2,
                                                   const DevTables& T0, double* gA, double* gB, double* gC) {
  constexpr int NQ = Shape<2, P>::NQ;
  const double w1 = T0.wl[b1], w2 = T0.wl[b2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const double g1 = g[(0 + m) * NQ + i] / w2;
    const double g2 = 2.0 * g[(2 + m) * NQ + i] / w2;
    gA[m] = (g1 + g2) * 0.70710678118654752440;     // facet 2: G^T nhat, nhat = (1,1)/sqrt 2
    gB[m] = -g1;                                     // facet 3: nhat = (-1, 0)
    gC[m] = -2.0 * g[(4 + m) * NQ + i] / w1;         // facet 1: nhat = (0, -1)
  }
}
template <int P>
__device__ __forceinline__ void tet_volume_normals(const double* __restrict__ g, int i, int b1, int b2, int b3,
                                                   const DevTables& T0, double* gA, double* gB, double* gC,
                                                   double* gD) {
  constexpr int NQ = Shape<3, P>::NQ;
  const double inv23 = 1.0 / (T0.wl[b2] * T0.wj[b3]);
  const double inv13 = 1.0 / (T0.wl[b1] * T0.wj[b3]);
  const double inv12 = 1.0 / (T0.wl[b1] * T0.wl[b2] * (1.0 - T0.xl[b2]));
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const double g1 = 2.0 * g[(0 + m) * NQ + i] * inv23;
    const double g23 = 4.0 * g[(3 + m) * NQ + i] * inv23;
    gA[m] = (g1 + g23) * 0.57735026918962576451;    // facet 2: nhat = (1,1,1)/sqrt 3
    gB[m] = -g1;                                     // facet 3: nhat = (-1,0,0)
    gC[m] = -4.0 * g[(6 + m) * NQ + i] * inv13;      // facet 1: nhat = (0,-1,0)
    gD[m] = -8.0 * g[(12 + m) * NQ + i] * inv12;     // facet 4: nhat = (0,0,-1)
  }
}

// C^T 1 at facet node j (face z, node jf of the face) summed by the facet
// node in a fixed order over its partners (the volume nodes whose lines reach
// it: Q along a line for faces 1-3, the Q^2 nodes of an eta2-eta3 plane for
// tet face 4), each pair re-evaluated exactly as the volume node's task
// evaluates it: s_j -= sum_i C_ij.  The deterministic form of the atomics.
template <int DIM, int P, int FLUX>
__device__ __forceinline__ void facet_node_sum(const double* sN, const double* sF, double* sT,
                                               const double* __restrict__ g, const double* __restrict__ gf, int j,
                                               const DevTables& T0, const Scheme& S) {
  using Sh = Shape<DIM, P>;
  constexpr int Q = Sh::Q, NQ = Sh::NQ, NC = Sh::NC, NQF = Sh::NQF, NFQ = Sh::NFQ;
  const int z = j / NQF, jf = j % NQF;
  const Node<DIM> Fj = load_node<DIM>(sF, NFQ, j);
  double gfj[DIM];
#pragma unroll
  for (int m = 0; m < DIM; ++m) gfj[m] = gf[m * NFQ + j];
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  auto pair = [&](int i, const double* gn, double coef) {
    const Node<DIM> Vi = load_node<DIM>(sN, NQ, i);
    double n[DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m) n[m] = 0.5 * (gn[m] + gfj[m]);
    double F[NC];
    ec_flux<DIM, FLUX>(Vi, Fj, n, S.gm1_inv, F);
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] += coef * F[c];
  };
  // loops kept rolled: one flux in flight per thread (unrolled, the compiler
  // holds several and spills)
  if constexpr (DIM == 2) {
#pragma unroll 1
    for (int k = 0; k < Q; ++k) {
      const int b1 = z == 0 ? jf : k, b2 = z == 0 ? k : jf;
      double gA[2], gB[2], gC[2];
      tri_volume_normals<P>(g, b1 + Q * b2, b1, b2, T0, gA, gB, gC);
      if (z == 1) pair(b1 + Q * b2, gA, T0.lgp1[b1] * T0.wf[j]);
      else if (z == 2) pair(b1 + Q * b2, gB, T0.lgm1[b1] * T0.wf[j]);
      else pair(b1 + Q * b2, gC, T0.lgm1[b2] * T0.wf[j]);
    }
  } else {
    if (z < 3) {
#pragma unroll 1
      for (int k = 0; k < Q; ++k) {
        // faces 1, 2: jf = b2 + Q b3, partners along b1; face 0: jf = b1 + Q b3, along b2
        const int b3 = jf / Q, b1 = z == 0 ? jf % Q : k, b2 = z == 0 ? k : jf % Q;
        double gA[3], gB[3], gC[3], gD[3];
        const int i = b1 + Q * (b2 + Q * b3);
        tet_volume_normals<P>(g, i, b1, b2, b3, T0, gA, gB, gC, gD);
        if (z == 1) pair(i, gA, T0.lgp1[b1] * T0.wf[j]);
        else if (z == 2) pair(i, gB, T0.lgm1[b1] * T0.wf[j]);
        else pair(i, gC, T0.lgm1[b2] * T0.wf[j]);
      }
    } else {
      // face 4: jf = b1 + Q a2, partners over the (b2, b3) plane
      const int b1 = jf % Q, a2 = jf / Q;
#pragma unroll 1
      for (int b3 = 0; b3 < Q; ++b3)
#pragma unroll 1
        for (int b2 = 0; b2 < Q; ++b2) {
          double gA[3], gB[3], gC[3], gD[3];
          const int i = b1 + Q * (b2 + Q * b3);
          tet_volume_normals<P>(g, i, b1, b2, b3, T0, gA, gB, gC, gD);
          pair(i, gD, T0.gjm1[b3] * T0.I42[a2 * Q + b2] * T0.wf[j]);
        }
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) sT[c * NFQ + j] -= acc[c];
}

// ------------------------------------------------------------------ K2, all-pairs variant
// The multidimensional-style evaluation of the same two terms, as an operator
// without line structure performs them: every volume node i evaluates the
// two-point flux with every volume node j (N_q^2 evaluations per element,
// eq. flux_differencing with dense S^l) and with every facet node of every
// facet (N_q N_f N_qf evaluations, eq. facet_correction with dense R^T B),
// the coefficient being zero where the tensor-product operators have no entry
// (the flux is still evaluated: a dense operator knows no zeros).  r_i is
// owned by node i's task (each ordered pair evaluated, as the dense sum runs);
// C^T 1 accumulates through LDS atomics.  Used to measure the cost of the
// dense formulation on the same nodes against the line-based one.
template <int DIM, int P, int FLUX>
__device__ __forceinline__ void dense_volume_task(const double* sN, const double* __restrict__ g, double* racc, int i,
                                                  const DevTables& T, const Scheme& S) {
  using Sh = Shape<DIM, P>;
  constexpr int Q = Sh::Q, NQ = Sh::NQ, NC = Sh::NC;
  const Node<DIM> Ni = load_node<DIM>(sN, NQ, i);
  const int i1 = i % Q, i2 = (i / Q) % Q, i3 = DIM == 3 ? i / (Q * Q) : 0;
  for (int j = 0; j < NQ; ++j) {
    const int j1 = j % Q, j2 = (j / Q) % Q, j3 = DIM == 3 ? j / (Q * Q) : 0;
    double n[DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m) n[m] = 0.0;
    // the line family the pair shares, if any (i == j shares all: coefficient 0)
    int a = 0, b = 0, t0 = -1, t1 = -1, hc0 = 0, hc1 = 0;
    if (DIM == 2) {
      if (j2 == i2) { a = i1; b = j1; t0 = 0; t1 = 1; hc0 = 0; hc1 = 2; }
      else if (j1 == i1) { a = i2; b = j2; t0 = 2; hc0 = 4; }
    } else {
      if (j2 == i2 && j3 == i3) { a = i1; b = j1; t0 = 0; t1 = 1; hc0 = 0; hc1 = 3; }
      else if (j1 == i1 && j3 == i3) { a = i2; b = j2; t0 = 2; t1 = 3; hc0 = 6; hc1 = 9; }
      else if (j1 == i1 && j2 == i2) { a = i3; b = j3; t0 = 4; hc0 = 12; }
    }
    if (t0 >= 0 && i != j) {
      const double c0 = T.A[t0 * Q * Q + a * Q + b];
#pragma unroll
      for (int m = 0; m < DIM; ++m) n[m] = c0 * (g[(hc0 + m) * NQ + i] + g[(hc0 + m) * NQ + j]);
      if (t1 >= 0) {
        const double c1 = T.A[t1 * Q * Q + a * Q + b];
#pragma unroll
        for (int m = 0; m < DIM; ++m) n[m] += c1 * (g[(hc1 + m) * NQ + i] + g[(hc1 + m) * NQ + j]);
      }
    }
    const Node<DIM> Nj = load_node<DIM>(sN, NQ, j);
    double F[NC];
    ec_flux<DIM, FLUX>(Ni, Nj, n, S.gm1_inv, F);
#pragma unroll
    for (int c = 0; c < NC; ++c) racc[c] -= F[c];
  }
}

// node i against every facet node: gn[z] is G(xi_i)^T nhat of facet z
template <int DIM, int P, int FLUX>
__device__ __forceinline__ void dense_facet_task(const Node<DIM>& Vi, const double (*gn)[DIM], const double* sF,
                                                 double* sT, const double* __restrict__ gf, int i, const DevTables& T,
                                                 const Scheme& S, double* racc) {
  using Sh = Shape<DIM, P>;
  constexpr int Q = Sh::Q, NQF = Sh::NQF, NFQ = Sh::NFQ, NC = Sh::NC;
  const int i1 = i % Q, i2 = (i / Q) % Q, i3 = DIM == 3 ? i / (Q * Q) : 0;
  for (int j = 0; j < NFQ; ++j) {
    const int z = j / NQF, jj = j % NQF;
    double coef = 0.0;
    if (DIM == 2) {
      if (z == 1 && jj == i2) coef = T.lgp1[i1] * T.wf[j];
      else if (z == 2 && jj == i2) coef = T.lgm1[i1] * T.wf[j];
      else if (z == 0 && jj == i1) coef = T.lgm1[i2] * T.wf[j];
    } else {
      if (z == 1 && jj == i2 + Q * i3) coef = T.lgp1[i1] * T.wf[j];
      else if (z == 2 && jj == i2 + Q * i3) coef = T.lgm1[i1] * T.wf[j];
      else if (z == 0 && jj == i1 + Q * i3) coef = T.lgm1[i2] * T.wf[j];
      else if (z == 3 && jj % Q == i1) coef = T.gjm1[i3] * T.I42[(jj / Q) * Q + i2] * T.wf[j];
    }
    const Node<DIM> Fj = load_node<DIM>(sF, NFQ, j);
    double n[DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m) n[m] = 0.5 * (gn[z][m] + gf[m * NFQ + j]);
    double F[NC];
    ec_flux<DIM, FLUX>(Vi, Fj, n, S.gm1_inv, F);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double C = coef * F[c];
      racc[c] -= C;
      atomicAdd(&sT[c * NFQ + j], -C);
    }
  }
}

// ------------------------------------------------------------------ K2: right-hand side
template <int DIM, int P, int FLUX, bool NEXT, bool DENSE = false, bool DET = false>
__global__ void __launch_bounds__((Launch<DIM, P>::BSMAX))
k_rhs(const double* __restrict__ wt, const double* __restrict__ wfb, double* __restrict__ dudt,
      const double* __restrict__ gvol, const double* __restrict__ gfac, const int32_t* __restrict__ conn,
      DevTables T0, Scheme S, int64_t ne, int* flag, double* frec, RkEpilogue epi) {
  using Sh = Shape<DIM, P>;
  constexpr int EPB = Launch<DIM, P>::EPB;
  constexpr int Q = Sh::Q, NC = Sh::NC, NQ = Sh::NQ, NP = Sh::NP, NQF = Sh::NQF, NFQ = Sh::NFQ, NGV = Sh::NGV;
  constexpr int LPF = Sh::LPF;
  // own facet node records live in LDS when everything fits, else in this
  // element's slice of the workspace (frec, [e][8][NFQ]; read through the caches)
  constexpr bool FLDS = Sh::K2_FACET_LDS;
  __shared__ double sN[EPB * Sh::SCR];      // node data [el][8][NQ]; transform scratch
  __shared__ double sR[EPB * NC * NQ];      // w at nodes, then r
  __shared__ double sF[FLDS ? EPB * 8 * NFQ : 1];   // own facet node records (LDS case)
  __shared__ double sT[EPB * NC * NFQ];     // C^T 1, then s = B J_f f* - C^T 1
  // operator tables in LDS: tetrahedra keep them in the tail of sN beyond the
  // first transform stage's scratch, free during both transform phases (the
  // middle stage runs in place over sR; copied again once the flux phases are
  // done), so the kernel's LDS and occupancy do not grow (measured against
  // the tail of sF, where the composed V V^T table fits only up to p = 6: K2
  // tet p7 -1%, p8 -3%, p9 -3%); triangles in an array of their own.  The
  // transforms read psi; the projection of the next stage also reads the
  // facet tables.  The interface and flux phases read theirs from T0.
  constexpr unsigned W0 = NEXT ? (TAB_PSI | TAB_FACET) : TAB_PSI;
  constexpr unsigned W1 = W0 | TAB_PSIM;   // with the composed stage of V V^T
  constexpr int ROOM = DIM != 3 ? -1 : Sh::SCR - Sh::T1;   // doubles free
  constexpr int KB = 8 * (EPB * (Sh::SCR + NC * NQ + NC * NFQ) + (FLDS ? EPB * 8 * NFQ : 1));
  constexpr unsigned TM =
      DIM == 2 ? (tab_keeps_wgs<DIM, P, W0, W1>(KB, wave_cap<DIM, P>()) ? W1 : tab_mask<DIM, P, W0>(KB))
               : (TabLds<DIM, P, W1>::SIZE <= ROOM   ? W1
                  : TabLds<DIM, P, W0>::SIZE <= ROOM ? W0
                  : TabLds<DIM, P, TAB_PSI>::SIZE <= ROOM ? TAB_PSI : 0u);
  constexpr bool TAB_SF = DIM == 3 && TM != 0;
  constexpr bool VVT = (TM & TAB_PSIM) != 0;
  static_assert(!TAB_SF || EPB == 1, "one element per workgroup when the tables share sF or sN");
  __shared__ double sTab[DIM == 2 && TM ? TabLds<DIM, P, TM>::SIZE : 1];
  double* const tab_buf = TAB_SF ? sN + Sh::T1 : sTab;
  const DevTables T = stage_tables<DIM, P, TM>(T0, tab_buf);
  static_assert(FLDS ? 8 * NFQ >= NC * NP : NFQ >= NP, "modal staging must fit the facet buffers");
  // modal w~ before the facet data exist, du~/dt after they are dead
  double* sM = FLDS ? sF : sT;
  double* lift_scratch = FLDS ? sF : sN;
  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const int nel = (int)((ne - e0) < EPB ? (ne - e0) : EPB);
  const int nec = nel * NC;
  double* fr = FLDS ? sF : frec + e0 * 8 * NFQ;
  const int tid = threadIdx.x, nth = blockDim.x;
  double* T1 = sN;
  // the middle transform stage in sN, or in place over sR where sN's tail
  // holds the tables
  double* T2 = DIM == 3 ? sR : sN + EPB * Sh::T1;

  // ---- w = V w~ at the volume nodes
  for (int o = tid; o < nec * NP; o += nth) sM[o] = wt[e0 * NC * NP + o];
  __syncthreads();
  xform_V<DIM, P>(sM, T1, T2, sR, T, nec);
  // ---- entropy-projected conservative variables at volume and own facet nodes
  bool bad = false;
  for (int o = tid; o < nel * NQ; o += nth) {
    const int k = o % NQ, el = o / NQ;
    double w[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) w[c] = sR[(el * NC + c) * NQ + k];
    Node<DIM> nd;
    bad |= !from_entropy<DIM>(w, S.gamma, S.gm1_inv, nd);
    store_node<DIM>(sN + el * Sh::SCR, NQ, k, nd);
  }
  // own facet node records, and the interface flux (eqs. num_flux,
  // entropy_stable) against the neighbour's facet state: s starts as
  // B J_f f* at the facet nodes, the facet correction subtracts C^T 1
  for (int o = tid; o < nel * NFQ; o += nth) {
    const int j = o % NFQ, el = o / NFQ;
    const int64_t e = e0 + el;
    const int32_t addr = conn[e * NFQ + j];
    double w[NC], wn[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      w[c] = wfb[(e * NC + c) * NFQ + j];
      wn[c] = wfb[addr + c * NFQ];
    }
    double nJ[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) nJ[i] = gfac[(e * (DIM + 1) + i) * NFQ + j];
    const double Jf = gfac[(e * (DIM + 1) + DIM) * NFQ + j];
    Node<DIM> Um, Up;
    bad |= !from_entropy<DIM>(w, S.gamma, S.gm1_inv, Um);
    bad |= !from_entropy<DIM>(wn, S.gamma, S.gm1_inv, Up);
    store_node<DIM>(fr + el * 8 * NFQ, NFQ, j, Um);
    double F[NC];
    interface_flux<DIM, FLUX>(Um, Up, nJ, Jf, S.gamma, S.gm1_inv, S.dissipation, F, w, wn);
    const double wj = T0.wf[j];
#pragma unroll
    for (int c = 0; c < NC; ++c) sT[(el * NC + c) * NFQ + j] = wj * F[c];
  }
  if (bad) atomicOr(flag, 1);
  __syncthreads();

  // ---- volume flux differencing: one task per (line family, line, node a);
  //      task a evaluates the pairs (a, a+k mod Q), k = 1..(Q-1)/2 (and k = Q/2
  //      for a < Q/2 when Q is even), so every unordered pair of a line is
  //      evaluated once and every task does the same work.  r_a accumulates in
  //      registers, r_b through LDS atomics.
  for (int o = tid; o < nec * NQ; o += nth) sR[o] = 0.0;
  __syncthreads();
  if constexpr (DET) {
    // one family at a time, its lines 64 / Q to a wave (blockDim is a
    // multiple of 64); every node has one owner per family
    constexpr int LPW = 64 / Q;
    static_assert(LPW >= 1, "a line fits in a wave");
    const int lane = tid & 63, wv = tid >> 6, nwv = nth >> 6;
    const int grp = lane / Q;
    const bool lane_ok = grp < LPW;
    // lanes past the last whole group pair with themselves
    const int a = lane_ok ? lane - grp * Q : 0, lbase = lane_ok ? lane - a : lane;
    const int nlines = nel * LPF;
#pragma unroll 1
    for (int fam = 0; fam < DIM; ++fam) {
      for (int wt = wv; wt * LPW < nlines; wt += nwv) {
        const int gl0 = wt * LPW + grp;
        const bool ok = lane_ok && gl0 < nlines;
        const int gl = ok ? gl0 : wt * LPW;   // groups without a line shadow the wave's first
        const int el = gl / LPF, L = gl % LPF;
        const double* sNe = sN + el * Sh::SCR;
        double* sRe = sR + el * NC * NQ;
        const double* g = gvol + (e0 + el) * NGV * NQ;
        if constexpr (DIM == 2) {
          if (fam == 0)
            vol_line<DIM, P, FLUX, 2>(sNe, g, sRe, Q * L, 1, a, lbase, ok, T.A + 0 * Q * Q, T.A + 1 * Q * Q, 0, 2, S);
          else
            vol_line<DIM, P, FLUX, 1>(sNe, g, sRe, L, Q, a, lbase, ok, T.A + 2 * Q * Q, nullptr, 4, 0, S);
        } else {
          if (fam == 0)
            vol_line<DIM, P, FLUX, 2>(sNe, g, sRe, Q * L, 1, a, lbase, ok, T.A + 0 * Q * Q, T.A + 1 * Q * Q, 0, 3,
                                      S);
          else if (fam == 1)
            vol_line<DIM, P, FLUX, 2>(sNe, g, sRe, (L % Q) + Q * Q * (L / Q), Q, a, lbase, ok, T.A + 2 * Q * Q,
                                      T.A + 3 * Q * Q, 6, 9, S);
          else
            vol_line<DIM, P, FLUX, 1>(sNe, g, sRe, L, Q * Q, a, lbase, ok, T.A + 4 * Q * Q, nullptr, 12, 0, S);
        }
      }
      __syncthreads();
    }
  } else if constexpr (DENSE) {
    for (int task = tid; task < nel * NQ; task += nth) {
      const int el = task / NQ, i = task % NQ;
      double racc[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) racc[c] = 0.0;
      dense_volume_task<DIM, P, FLUX>(sN + el * Sh::SCR, gvol + (e0 + el) * NGV * NQ, racc, i, T0, S);
#pragma unroll
      for (int c = 0; c < NC; ++c) sR[(el * NC + c) * NQ + i] += racc[c];
    }
  } else {
    constexpr int TPE = DIM * NQ;           // volume tasks per element
    for (int task = tid; task < nel * TPE; task += nth) {
      const int el = task / TPE, lt = task % TPE;
      const int fam = lt / NQ, rem = lt % NQ;
      // lanes run along a line (a fastest) for the families of stride 1 and Q,
      // across lines (L fastest) for the family of stride Q^2: consecutive
      // lanes then address distinct LDS banks (measured: across lines also for
      // the stride-Q family, tri p4 0.031 -> 0.038 ms, tet p6 2.42 -> 2.48 ms)
      const bool across = DIM == 3 && fam == 2;
      const int L = across ? rem % LPF : rem / Q, a = across ? rem / LPF : rem % Q;
      const double* sNe = sN + el * Sh::SCR;
      double* sRe = sR + el * NC * NQ;
      const double* g = gvol + (e0 + el) * NGV * NQ;
      if constexpr (DIM == 2) {
        if (fam == 0)
          vol_task<DIM, P, FLUX, 2>(sNe, g, sRe, Q * L, 1, a, T.A + 0 * Q * Q, T.A + 1 * Q * Q, 0, 2, S);
        else
          vol_task<DIM, P, FLUX, 1>(sNe, g, sRe, L, Q, a, T.A + 2 * Q * Q, nullptr, 4, 0, S);
      } else {
        if (fam == 0)
          vol_task<DIM, P, FLUX, 2>(sNe, g, sRe, Q * L, 1, a, T.A + 0 * Q * Q, T.A + 1 * Q * Q, 0, 3, S);
        else if (fam == 1)
          vol_task<DIM, P, FLUX, 2>(sNe, g, sRe, (L % Q) + Q * Q * (L / Q), Q, a, T.A + 2 * Q * Q, T.A + 3 * Q * Q,
                                    6, 9, S);
        else
          vol_task<DIM, P, FLUX, 1>(sNe, g, sRe, L, Q * Q, a, T.A + 4 * Q * Q, nullptr, 12, 0, S);
      }
    }
  }
  __syncthreads();
  // ---- facet correction (eq. facet_correction): one task per volume node i
  //      with its partners on faces 1-3 (one each, along i's lines) and, in
  //      3D, the Q face-4 nodes of its eta2-eta3 plane.  r_i is owned by the
  //      task; C^T 1 accumulates through LDS atomics.
  for (int task = tid; task < nel * NQ; task += nth) {
    const int el = task / NQ, t = task % NQ;
    const double* sNe = sN + el * Sh::SCR;
    const double* sFe = fr + el * 8 * NFQ;
    double* sTe = sT + el * NC * NFQ;
    const double* g = gvol + (e0 + el) * NGV * NQ;
    const double* gf = gfac + (e0 + el) * (DIM + 1) * NFQ;
    double racc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) racc[c] = 0.0;
    int i;
    constexpr bool ATOM = !DET;   // C^T 1 through LDS atomics, or summed by facet node below
    if constexpr (DIM == 2) {
      const int b2 = t % Q, b1 = t / Q;     // b2 fastest: neighbouring lanes hit different facet nodes
      i = b1 + Q * b2;
      const Node<DIM> Vi = load_node<DIM>(sNe, NQ, i);
      double gA[2], gB[2], gC[2];
      tri_volume_normals<P>(g, i, b1, b2, T0, gA, gB, gC);
      if constexpr (DENSE) {
        const double gn[3][2] = {{gC[0], gC[1]}, {gA[0], gA[1]}, {gB[0], gB[1]}};
        dense_facet_task<DIM, P, FLUX>(Vi, gn, sFe, sTe, gf, i, T0, S, racc);
      } else {
        facet_task<DIM, P, FLUX, ATOM>(Vi, gA, sFe, sTe, gf, 1 * NQF + b2, T0.lgp1[b1] * T0.wf[1 * NQF + b2], S,
                                       racc);
        facet_task<DIM, P, FLUX, ATOM>(Vi, gB, sFe, sTe, gf, 2 * NQF + b2, T0.lgm1[b1] * T0.wf[2 * NQF + b2], S,
                                       racc);
        facet_task<DIM, P, FLUX, ATOM>(Vi, gC, sFe, sTe, gf, 0 * NQF + b1, T0.lgm1[b2] * T0.wf[0 * NQF + b1], S,
                                       racc);
      }
    } else {
      const int b3 = t % Q, b2 = (t / Q) % Q, b1 = t / (Q * Q);
      i = b1 + Q * (b2 + Q * b3);
      const Node<DIM> Vi = load_node<DIM>(sNe, NQ, i);
      double gA[3], gB[3], gC[3], gD[3];
      tet_volume_normals<P>(g, i, b1, b2, b3, T0, gA, gB, gC, gD);
      if constexpr (DENSE) {
        const double gn[4][3] = {{gC[0], gC[1], gC[2]}, {gA[0], gA[1], gA[2]}, {gB[0], gB[1], gB[2]},
                                 {gD[0], gD[1], gD[2]}};
        dense_facet_task<DIM, P, FLUX>(Vi, gn, sFe, sTe, gf, i, T0, S, racc);
      } else {
        const int j23 = b2 + Q * b3;
        facet_task<DIM, P, FLUX, ATOM>(Vi, gA, sFe, sTe, gf, 1 * NQF + j23, T0.lgp1[b1] * T0.wf[1 * NQF + j23], S,
                                       racc);
        facet_task<DIM, P, FLUX, ATOM>(Vi, gB, sFe, sTe, gf, 2 * NQF + j23, T0.lgm1[b1] * T0.wf[2 * NQF + j23], S,
                                       racc);
        const int j13 = b1 + Q * b3;
        facet_task<DIM, P, FLUX, ATOM>(Vi, gC, sFe, sTe, gf, 0 * NQF + j13, T0.lgm1[b2] * T0.wf[0 * NQF + j13], S,
                                       racc);
        const double cz = T0.gjm1[b3];
        // without the atomics the compiler would overlap all Q pairs of an
        // unrolled loop and spill: rolled in the deterministic form
        constexpr int U4 = DET ? 1 : Q;
#pragma unroll U4
        for (int m = 0; m < Q; ++m) {
          int a2 = m + b2 + b3;                 // rotated so that neighbouring lanes hit different facet nodes
          a2 = a2 % Q;
          const int j = 3 * NQF + b1 + Q * a2;
          facet_task<DIM, P, FLUX, ATOM>(Vi, gD, sFe, sTe, gf, j, cz * T0.I42[a2 * Q + b2] * T0.wf[j], S, racc);
        }
      }
    }
    double* r = sR + el * NC * NQ;
#pragma unroll
    for (int c = 0; c < NC; ++c) r[c * NQ + i] += racc[c];
  }
  if constexpr (DET) {
    // C^T 1 by facet node (the loop above wrote r only, this one s only)
    for (int task = tid; task < nel * NFQ; task += nth) {
      const int el = task / NFQ, j = task % NFQ;
      facet_node_sum<DIM, P, FLUX>(sN + el * Sh::SCR, fr + el * 8 * NFQ, sT + el * NC * NFQ,
                                   gvol + (e0 + el) * NGV * NQ, gfac + (e0 + el) * (DIM + 1) * NFQ, j, T0, S);
    }
  }
  __syncthreads();

  if constexpr (TAB_SF) {
    (void)stage_tables<DIM, P, TM>(T0, tab_buf);   // over the dead facet (or node) records
    // the lift below reads the facet tables when they are staged
    if constexpr ((TM & TAB_FACET) != 0) __syncthreads();
  }
  auto ld_wi = [&](int o) { return gvol[((e0 + o / NQ) * NGV + NGV - 1) * NQ + o % NQ]; };
  auto ld_u = [&](int o) { return epi.u[e0 * NC * NP + o]; };
  auto ld_acc = [&](int o) { return epi.acc[e0 * NC * NP + o]; };
  Ahead<2> aI, aU, aA, aJ;
  aI.load(nel * NQ, ld_wi);
  if constexpr (NEXT) aJ.load(nel * NQ, [&](int o) { return gvol[((e0 + o / NQ) * NGV + NGV - 2) * NQ + o % NQ]; });
  if (epi.acc != nullptr && !epi.last) aU.load(nec * NP, ld_u);
  if (epi.acc != nullptr && !epi.first) aA.load(nec * NP, ld_acc);

  // ---- r -= R^T s
  facet_lift<DIM, P>(sT, lift_scratch, T, nec, [&](int o, double d) { sR[o] -= d; });
  __syncthreads();

  // ---- du~/dt = V^T (w/J) V V^T r
  if constexpr (VVT) {
    xform_VVt<DIM, P>(sR, T1, T2, sR, T, nec);
  } else {
    xform_Vt<DIM, P>(sR, T1, T2, sM, T, nec);
    xform_V<DIM, P>(sM, T1, T2, sR, T, nec);
  }
  aI.each(nel * NQ, ld_wi, [&](int o, double wi) {
    const int k = o % NQ, el = o / NQ;
#pragma unroll
    for (int c = 0; c < NC; ++c) sR[(el * NC + c) * NQ + k] *= wi;
  });
  __syncthreads();
  xform_Vt<DIM, P>(sR, T1, T2, sM, T, nec);
  // the next stage input U (or the new state at stage 4) goes to HBM, or, when
  // this kernel also projects it, stays in sM
  auto put_next = [&](int o, int64_t i, double v) {
    if constexpr (NEXT) sM[o] = v;
    else epi.U[i] = v;
  };
  if (epi.acc == nullptr) {
    for (int o = tid; o < nec * NP; o += nth) dudt[e0 * NC * NP + o] = sM[o];
  } else if (!epi.last) {
    if (epi.first) {
      aU.each(nec * NP, ld_u, [&](int o, double ui) {
        const int64_t i = e0 * NC * NP + o;
        const double k = sM[o];
        epi.acc[i] = ui + epi.ca * k;
        put_next(o, i, ui + epi.cu * k);
      });
    } else {
      // both arrays ahead: walk the iterations by hand
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const int o = tid + it * nth;
        if (o < nec * NP) {
          const int64_t i = e0 * NC * NP + o;
          const double k = sM[o];
          epi.acc[i] = aA.v[it] + epi.ca * k;
          put_next(o, i, aU.v[it] + epi.cu * k);
        }
      }
      for (int o = tid + 2 * nth; o < nec * NP; o += nth) {
        const int64_t i = e0 * NC * NP + o;
        const double k = sM[o], ui = epi.u[i];
        epi.acc[i] = epi.acc[i] + epi.ca * k;
        put_next(o, i, ui + epi.cu * k);
      }
    }
  } else {
    aA.each(nec * NP, ld_acc, [&](int o, double ai) {
      const double un = ai + epi.ca * sM[o];
      epi.u[e0 * NC * NP + o] = un;
      if constexpr (NEXT) sM[o] = un;
    });
  }
  if constexpr (NEXT) {
    // entropy projection of the next stage input, into the other workspace
    __syncthreads();
    project_block<DIM, P, VVT>(sM, sR, sN, T, gvol, S, e0, nel, flag, epi.wt_next, epi.wf_next, aJ, aI);
  }
}

// ------------------------------------------------------------------ vector helpers
__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, const double* __restrict__ z,
                       int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i] + a * z[i];
}

// ------------------------------------------------------------------ dispatch
hipEvent_t timing_event(const esd_plan* pl, hipStream_t s) {
  hipEvent_t e;
  if (!pl->ev_pool.empty()) {
    e = pl->ev_pool.back();
    pl->ev_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return nullptr;
  }
  (void)hipEventRecord(e, s);
  pl->ev.push_back(e);
  return e;
}

template <int DIM, int P>
static void launch_k2(const esd_plan* pl, double* dudt, Workspace ws, hipStream_t s, const RkEpilogue& epi, int64_t nb,
                      int bs) {
  const bool next = epi.wt_next != nullptr;
#define K2_ARGS \
  dim3(nb), dim3(bs), 0, s, ws.wt, ws.wf, dudt, pl->d_gvol, pl->d_gfac, pl->d_conn, pl->tab, pl->scheme, pl->ne, \
      pl->d_flag, ws.frec, epi
  if (pl->deterministic) {
    // fixed-order sums; the RK4 driver runs unfused stages for such plans
    if (pl->scheme.ecflux == FLUX_RANOCHA)
      hipLaunchKernelGGL((k_rhs<DIM, P, FLUX_RANOCHA, false, false, true>), K2_ARGS);
    else
      hipLaunchKernelGGL((k_rhs<DIM, P, FLUX_CHANDRASHEKAR, false, false, true>), K2_ARGS);
  } else if (pl->scheme.ecflux == FLUX_RANOCHA) {
    if (next) hipLaunchKernelGGL((k_rhs<DIM, P, FLUX_RANOCHA, true>), K2_ARGS);
    else hipLaunchKernelGGL((k_rhs<DIM, P, FLUX_RANOCHA, false>), K2_ARGS);
  } else {
    if (next) hipLaunchKernelGGL((k_rhs<DIM, P, FLUX_CHANDRASHEKAR, true>), K2_ARGS);
    else hipLaunchKernelGGL((k_rhs<DIM, P, FLUX_CHANDRASHEKAR, false>), K2_ARGS);
  }
#undef K2_ARGS
}

template <int DIM, int P>
static int run_residual(const esd_plan* pl, const double* u, double* dudt, Workspace ws, hipStream_t s,
                        const RkEpilogue& epi) {
  using L = Launch<DIM, P>;
  const int64_t nb = (pl->ne + L::EPB - 1) / L::EPB;
  if (pl->timing) timing_event(pl, s);
  const int bs1 = pl->k1_block > 0 ? pl->k1_block : L::BS;
  hipLaunchKernelGGL((k_entropy_projection<DIM, P, false>), dim3(nb), dim3(bs1), 0, s, u, ws.wt, ws.wf,
                     pl->d_gvol, pl->tab, pl->scheme, pl->ne, pl->d_flag);
  if (pl->timing) timing_event(pl, s);
  const int bs = pl->k2_block > 0 ? pl->k2_block : L::BS;
  launch_k2<DIM, P>(pl, dudt, ws, s, epi, nb, bs);
  if (pl->timing) timing_event(pl, s);
  return (int)hipGetLastError();
}

// the all-pairs variant of the residual: K1, then K2 with dense volume and facet loops
template <int DIM, int P>
static int run_residual_dense(const esd_plan* pl, const double* u, double* dudt, Workspace ws, hipStream_t s) {
  using L = Launch<DIM, P>;
  const int64_t nb = (pl->ne + L::EPB - 1) / L::EPB;
  if (pl->timing) timing_event(pl, s);
  const int bs1 = pl->k1_block > 0 ? pl->k1_block : L::BS;
  hipLaunchKernelGGL((k_entropy_projection<DIM, P, false>), dim3(nb), dim3(bs1), 0, s, u, ws.wt, ws.wf,
                     pl->d_gvol, pl->tab, pl->scheme, pl->ne, pl->d_flag);
  if (pl->timing) timing_event(pl, s);
  const int bs = pl->k2_block > 0 ? pl->k2_block : L::BS;
  const RkEpilogue epi;
#define K2D_ARGS \
  dim3(nb), dim3(bs), 0, s, ws.wt, ws.wf, dudt, pl->d_gvol, pl->d_gfac, pl->d_conn, pl->tab, pl->scheme, pl->ne, \
      pl->d_flag, ws.frec, epi
  if (pl->scheme.ecflux == FLUX_RANOCHA)
    hipLaunchKernelGGL((k_rhs<DIM, P, FLUX_RANOCHA, false, true>), K2D_ARGS);
  else
    hipLaunchKernelGGL((k_rhs<DIM, P, FLUX_CHANDRASHEKAR, false, true>), K2D_ARGS);
#undef K2D_ARGS
  if (pl->timing) timing_event(pl, s);
  return (int)hipGetLastError();
}

int launch_residual_dense(const esd_plan* pl, const double* u, double* dudt, Workspace ws, hipStream_t s) {
#define X(D, PP) \
  if (pl->dim == D && pl->p == PP) return run_residual_dense<D, PP>(pl, u, dudt, ws, s);
  ESD_TRI_DEGREES(X)
  ESD_TET_DEGREES(X)
#undef X
  return -1;
}

template <int DIM, int P>
static int run_rhs(const esd_plan* pl, double* dudt, Workspace ws, hipStream_t s, const RkEpilogue& epi) {
  using L = Launch<DIM, P>;
  const int64_t nb = (pl->ne + L::EPB - 1) / L::EPB;
  const int bs = pl->k2_block > 0 ? pl->k2_block : L::BS;
  launch_k2<DIM, P>(pl, dudt, ws, s, epi, nb, bs);
  return (int)hipGetLastError();
}

template <int DIM, int P>
static int run_project(const esd_plan* pl, const double* un, double* u, hipStream_t s) {
  using L = Launch<DIM, P>;
  const int64_t nb = (pl->ne + L::EPB - 1) / L::EPB;
  hipLaunchKernelGGL((k_entropy_projection<DIM, P, true>), dim3(nb), dim3(L::BS), 0, s, un, u, nullptr, pl->d_gvol,
                     pl->tab, pl->scheme, pl->ne, pl->d_flag);
  return (int)hipGetLastError();
}

bool degree_supported(int dim, int p) {
  if (dim == 2) return p >= 1 && p <= 10;
  if (dim == 3) return p >= 1 && p <= 10;
  return false;
}

// block sizes the right-hand-side kernel may be launched with (multiples of
// 64 up to its compiled bound), default first
std::vector<int> rhs_block_candidates(int dim, int p) {
  std::vector<int> c;
#define X(D, PP)                                                        \
  if (dim == D && p == PP) {                                            \
    c.push_back(Launch<D, PP>::BS);                                     \
    for (int b = 64; b <= Launch<D, PP>::BSMAX; b += 64)                \
      if (b != Launch<D, PP>::BS) c.push_back(b);                       \
  }
  ESD_TRI_DEGREES(X)
  ESD_TET_DEGREES(X)
#undef X
  return c;
}

// block sizes the entropy-projection kernel may be launched with (the right-
// hand side's, from the in-place stages' minimum up)
std::vector<int> k1_block_candidates(int dim, int p) {
  int lo = 64;
#define X(D, PP) \
  if (dim == D && p == PP) lo = K1Inplace<D, PP>::MIN_BLOCK;
  ESD_TRI_DEGREES(X)
  ESD_TET_DEGREES(X)
#undef X
  std::vector<int> c;
  for (int b : rhs_block_candidates(dim, p))
    if (b >= lo) c.push_back(b);
  return c;
}

bool vjp_degree_supported(int dim, int p) {
  if (dim == 2) return p >= 1 && p <= 10;
  if (dim == 3) return p >= 1 && p <= 10;
  return false;
}

bool needs_facet_records(int dim, int p) {
#define X(D, PP) \
  if (dim == D && p == PP) return !Shape<D, PP>::K2_FACET_LDS;
  ESD_TRI_DEGREES(X)
  ESD_TET_DEGREES(X)
#undef X
  return false;
}

int launch_residual(const esd_plan* pl, const double* u, double* dudt, Workspace ws, hipStream_t s,
                    const RkEpilogue& epi) {
#define X(D, PP) \
  if (pl->dim == D && pl->p == PP) return run_residual<D, PP>(pl, u, dudt, ws, s, epi);
  ESD_TRI_DEGREES(X)
  ESD_TET_DEGREES(X)
#undef X
  return -1;
}

int launch_entropy_projection(const esd_plan* pl, const double* u, Workspace ws, hipStream_t s) {
#define X(D, PP) \
  if (pl->dim == D && pl->p == PP) {                                                                          \
    using L = Launch<D, PP>;                                                                                  \
    const int64_t nb = (pl->ne + L::EPB - 1) / L::EPB;                                                        \
    hipLaunchKernelGGL((k_entropy_projection<D, PP, false>), dim3(nb),                                        \
                       dim3(pl->k1_block > 0 ? pl->k1_block : L::BS), 0, s, u, ws.wt, ws.wf,                  \
                       pl->d_gvol, pl->tab, pl->scheme, pl->ne, pl->d_flag);                                  \
    return (int)hipGetLastError();                                                                            \
  }
  ESD_TRI_DEGREES(X)
  ESD_TET_DEGREES(X)
#undef X
  return -1;
}

int launch_rhs(const esd_plan* pl, double* dudt, Workspace ws, hipStream_t s, const RkEpilogue& epi) {
#define X(D, PP) \
  if (pl->dim == D && pl->p == PP) return run_rhs<D, PP>(pl, dudt, ws, s, epi);
  ESD_TRI_DEGREES(X)
  ESD_TET_DEGREES(X)
#undef X
  return -1;
}

int launch_project(const esd_plan* pl, const double* un, double* u, hipStream_t s) {
#define X(D, PP) \
  if (pl->dim == D && pl->p == PP) return run_project<D, PP>(pl, un, u, s);
  ESD_TRI_DEGREES(X)
  ESD_TET_DEGREES(X)
#undef X
  return -1;
}

int launch_axpy(double* y, const double* x, double a, const double* z, int64_t n, hipStream_t s) {
  const int bs = 256;
  int64_t nb = (n + bs - 1) / bs;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_axpy, dim3(nb), dim3(bs), 0, s, y, x, a, z, n);
  return (int)hipGetLastError();
}


}  // namespace esd
