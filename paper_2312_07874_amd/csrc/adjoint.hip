// Adjoint (vector-Jacobian product) kernels for the entropy-stable modal DSEM
// residual, gfx950, FP64.  Reverse mode of the forward chain
//
//   u~ -> [K1] w~ = V^T (w/J) V V^T (w J) W(V u~),  w^z = R V w~
//      -> [K2] r(w~, w^z, w^z of the neighbours) -> du~/dt = V^T (w/J) V V^T r
//
// in two per-element kernels with one global dependency between them:
//
//   VK2 (reverse of K2)  r_bar = V V^T (w/J) V v_bar; the forward node states are
//        recomputed from w~ and w^z; every volume pair, facet-correction pair
//        and interface node is differentiated by hand (physics.hpp) and the
//        cotangents accumulate in LDS in the parameterisation (ln rho, ln b, v).
//        Cotangents of the neighbours' facet values are written to a buffer
//        indexed by this element's own facet node (no global atomics);
//        everything else is reduced to  V^T (w_bar + R^T w^z_bar).
//   VK1 (reverse of K1)  gathers the exterior cotangents through the facet
//        permutation (an involution), then
//        u~_bar = V^T W'(u)^T (w J) V V^T (w/J) V (w~_bar).
//
// The forward K1 runs first to provide w~ and w^z.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.hpp"

namespace esd {

// The adjoint kernels hold more live state per thread than the forward ones:
// their workgroups are capped at 256 threads so that the register file is
// not split further (same elements per workgroup as the forward launch).
template <int DIM, int P>
struct VjpLaunch {
  static constexpr int EPB = Launch<DIM, P>::EPB;
  static constexpr int BS = Launch<DIM, P>::BS > 256 ? 256 : Launch<DIM, P>::BS;
};

// Where the adjoint kernels keep their per-element arrays.  Up to tet p = 8
// everything is in LDS; above, VK2 moves its facet arrays (node records,
// t_bar, facet x_bar) and, at p = 10, r_bar to this element's slice of the
// VJP workspace, and VK1 its gathered facet cotangents at p = 10 (read
// through the caches, written and read by the element's own workgroup).
template <int DIM, int P>
struct VjpMem {
  using Sh = Shape<DIM, P>;
  static constexpr int NC = Sh::NC, NQ = Sh::NQ, NP = Sh::NP, NFQ = Sh::NFQ;
  static constexpr int NB = NQ > NFQ ? NQ : NFQ;
  static constexpr bool FG = 8 * (Sh::SCR + 2 * NC * NQ + 8 * NFQ + 2 * NC * NFQ) > LDS_BYTES;
  static constexpr bool RG = FG && 8 * (Sh::SCR + 2 * NC * NQ) > LDS_BYTES;
  static constexpr bool BG = 8 * (NC * NP + NC * NQ + NC * NB + Sh::XSCR) > LDS_BYTES;
  // doubles of the workspace slice per element (VK1 reuses VK2's slice)
  static constexpr int VK2_SLICE = (FG ? (8 + 2 * NC) * NFQ : 0) + (RG ? NC * NQ : 0);
  static constexpr int VK1_SLICE = BG ? NC * NB : 0;
  static constexpr int SLICE = VK2_SLICE > VK1_SLICE ? VK2_SLICE : VK1_SLICE;
};

// One volume adjoint task: node a of the line base + stride*k and the same
// partners as the forward task; F_bar = r_bar_b - r_bar_a.
template <int DIM, int P, int FLUX, int NA>
__device__ __forceinline__ void vol_task_vjp(const double* sN, const double* __restrict__ g, const double* sRb,
                                             double* sX, int base, int stride, int a, const double* __restrict__ A0,
                                             const double* __restrict__ A1, int hc0, int hc1, const Scheme& S) {
  using Sh = Shape<DIM, P>;
  constexpr int Q = Sh::Q, NQ = Sh::NQ, NC = Sh::NC;
  const int na = base + stride * a;
  const Node<DIM> Na = load_node<DIM>(sN, NQ, na);
  double h0a[DIM], h1a[DIM], rba[NC];
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    h0a[i] = g[(hc0 + i) * NQ + na];
    if constexpr (NA == 2) h1a[i] = g[(hc1 + i) * NQ + na];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) rba[c] = sRb[c * NQ + na];
  NodeBar<DIM> Ab;
  zero(Ab);
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
    double Fb[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) Fb[c] = sRb[c * NQ + nb] - rba[c];
    NodeBar<DIM> Bb;
    zero(Bb);
    ec_flux_vjp<DIM, FLUX>(Na, Nb, n, S.gm1_inv, Fb, Ab, Bb);
    double xb[NC];
    reduce_bar<DIM>(Nb, Bb, xb);
#pragma unroll
    for (int c = 0; c < NC; ++c) atomicAdd(&sX[c * NQ + nb], xb[c]);
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
  double xa[NC];
  reduce_bar<DIM>(Na, Ab, xa);
#pragma unroll
  for (int c = 0; c < NC; ++c) atomicAdd(&sX[c * NQ + na], xa[c]);
}

// One facet-correction adjoint pair: C = coef f#(u_i, u^z_j, n);  forward
// r_i -= C, t_j += C, so F_bar = coef (t_bar_j - r_bar_i).
template <int DIM, int P, int FLUX>
__device__ __forceinline__ void facet_task_vjp(const Node<DIM>& Vi, const double* gn_i, const double* sF,
                                               const double* sTb, double* sXF, const double* __restrict__ gf, int j,
                                               double coef, const Scheme& S, const double* rbi, NodeBar<DIM>& Vib) {
  constexpr int NC = DIM + 2, NFQ = Shape<DIM, P>::NFQ;
  const Node<DIM> Fj = load_node<DIM>(sF, NFQ, j);
  double n[DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i) n[i] = 0.5 * (gn_i[i] + gf[i * NFQ + j]);
  double Fb[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) Fb[c] = coef * (sTb[c * NFQ + j] - rbi[c]);
  NodeBar<DIM> Fjb;
  zero(Fjb);
  ec_flux_vjp<DIM, FLUX>(Vi, Fj, n, S.gm1_inv, Fb, Vib, Fjb);
  double xb[NC];
  reduce_bar<DIM>(Fj, Fjb, xb);
#pragma unroll
  for (int c = 0; c < NC; ++c) atomicAdd(&sXF[c * NFQ + j], xb[c]);
}

// ------------------------------------------------------------------ VK2: reverse of the right-hand side
template <int DIM, int P, int FLUX>
__global__ void __launch_bounds__((VjpLaunch<DIM, P>::BS))
k_rhs_vjp(const double* __restrict__ wt, const double* __restrict__ wfb, const double* __restrict__ vbar,
          double* __restrict__ gpart, double* __restrict__ xbar, const double* __restrict__ gvol,
          const double* __restrict__ gfac, const int32_t* __restrict__ conn, DevTables T0, Scheme S, int64_t ne,
          int* flag, double* gscr) {
  using Sh = Shape<DIM, P>;
  constexpr int EPB = Launch<DIM, P>::EPB;
  constexpr int Q = Sh::Q, NC = Sh::NC, NQ = Sh::NQ, NP = Sh::NP, NQF = Sh::NQF, NFQ = Sh::NFQ, NGV = Sh::NGV;
  constexpr int LPF = Sh::LPF;
  using VM = VjpMem<DIM, P>;
  static_assert(!VM::FG || EPB == 1, "workspace slices are per element");
  __shared__ double sN[EPB * Sh::SCR];      // transform scratch; node data [el][8][NQ]
  __shared__ double sX[EPB * NC * NQ];      // modal / nodal staging; x_bar, then w_bar at volume nodes
  __shared__ double sR_l[VM::RG ? 1 : EPB * NC * NQ];       // r_bar
  __shared__ double sF_l[VM::FG ? 1 : EPB * 8 * NFQ];       // own facet node data; later R^T scratch
  __shared__ double sT_l[VM::FG ? 1 : EPB * NC * NFQ];      // t_bar = R r_bar
  __shared__ double sXF_l[VM::FG ? 1 : EPB * NC * NFQ];     // x_bar, then w_bar at own facet nodes
  double* const slice = gscr + (int64_t)blockIdx.x * VM::SLICE;
  double* const sF = VM::FG ? slice : sF_l;
  double* const sT = VM::FG ? slice + 8 * NFQ : sT_l;
  double* const sXF = VM::FG ? slice + (8 + NC) * NFQ : sXF_l;
  double* const sR = VM::RG ? slice + (8 + 2 * NC) * NFQ : sR_l;
  // staged tables only where they do not lower the workgroups per CU: this
  // kernel is bound by its pair adjoints, not by the transforms, and runs at
  // about 2 waves per SIMD (about 225 VGPRs), which caps the workgroups per CU
  // at 8 waves' worth (measured at tet p = 6: VJP 8.17 -> 6.28 ms without the
  // tables, 1 -> 2 workgroups per CU; at p = 4 the tables stay)
  constexpr int VB = 8 * EPB * (Sh::SCR + NC * NQ + (VM::RG ? 0 : NC * NQ) + (VM::FG ? 0 : 8 * NFQ + 2 * NC * NFQ));
  constexpr int VT = 8 * TabLds<DIM, P, TAB_PSI | TAB_FACET>::SIZE;
  constexpr int CAP = 8 / ((VjpLaunch<DIM, P>::BS + 63) / 64);
  constexpr int WG_T = LDS_BYTES / (VB + VT) < CAP ? LDS_BYTES / (VB + VT) : CAP;
  constexpr int WG_N = LDS_BYTES / VB < CAP ? LDS_BYTES / VB : CAP;
  constexpr unsigned T0M = WG_T >= WG_N ? tab_mask<DIM, P, TAB_PSI | TAB_FACET>(VB) : 0u;
  // with the composed V V^T table where that keeps the workgroups per CU too
  constexpr unsigned TM =
      T0M != 0 && tab_keeps_wgs<DIM, P, TAB_PSI | TAB_FACET, TAB_PSI | TAB_FACET | TAB_PSIM>(VB, CAP)
          ? (TAB_PSI | TAB_FACET | TAB_PSIM)
          : T0M;
  __shared__ double sTab[TM ? TabLds<DIM, P, TM>::SIZE : 1];
  const DevTables T = stage_tables<DIM, P, TM>(T0, sTab);
  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const int nel = (int)((ne - e0) < EPB ? (ne - e0) : EPB);
  const int nec = nel * NC;
  const int tid = threadIdx.x, nth = blockDim.x;
  double* T1 = sN;
  double* T2 = sN + EPB * Sh::T1;

  // ---- r_bar = V V^T (w/J) V v_bar  (transpose of du~/dt = V^T (w/J) V V^T r)
  for (int o = tid; o < nec * NP; o += nth) sX[o] = vbar[e0 * NC * NP + o];
  __syncthreads();
  xform_V<DIM, P>(sX, T1, T2, sR, T, nec);
  for (int o = tid; o < nec * NQ; o += nth) {
    const int k = o % NQ, le = o / (NC * NQ);
    sR[o] *= gvol[((e0 + le) * NGV + NGV - 1) * NQ + k];
  }
  __syncthreads();
  if constexpr ((TM & TAB_PSIM) != 0) {
    xform_VVt<DIM, P>(sR, T1, T2, sR, T, nec);
  } else {
    xform_Vt<DIM, P>(sR, T1, T2, sX, T, nec);
    xform_V<DIM, P>(sX, T1, T2, sR, T, nec);
  }

  // ---- forward node states: w = V w~ at volume nodes, own facet values
  for (int o = tid; o < nec * NP; o += nth) sX[o] = wt[e0 * NC * NP + o];
  __syncthreads();
  xform_V<DIM, P>(sX, T1, T2, sX, T, nec);
  bool bad = false;
  for (int o = tid; o < nel * NQ; o += nth) {
    const int k = o % NQ, el = o / NQ;
    double w[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) w[c] = sX[(el * NC + c) * NQ + k];
    Node<DIM> nd;
    bad |= !from_entropy<DIM>(w, S.gamma, S.gm1_inv, nd);
    store_node<DIM>(sN + el * Sh::SCR, NQ, k, nd);
  }
  for (int o = tid; o < nel * NFQ; o += nth) {
    const int j = o % NFQ, el = o / NFQ;
    double w[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) w[c] = wfb[((e0 + el) * NC + c) * NFQ + j];
    Node<DIM> nd;
    bad |= !from_entropy<DIM>(w, S.gamma, S.gm1_inv, nd);
    store_node<DIM>(sF + el * 8 * NFQ, NFQ, j, nd);
  }
  if (bad) atomicOr(flag, 1);
  __syncthreads();
  // ---- t_bar = R r_bar (the forward subtracts R^T (B J_f f* - t))
  facet_values<DIM, P>(sR, sX, T, nec, [&](int o, double v) { sT[o] = v; });
  __syncthreads();
  for (int o = tid; o < nec * NQ; o += nth) sX[o] = 0.0;
  for (int o = tid; o < nec * NFQ; o += nth) sXF[o] = 0.0;
  // with the facet x_bar in global memory, the atomics below act in L2 and
  // the plain accesses around them go through the CU's L1: device-scope fences
  // (L1 written back and invalidated) before the barriers that order them
  if constexpr (VM::FG) __threadfence();
  __syncthreads();

  // ---- volume pairs, same task decomposition as the forward kernel
  {
    constexpr int TPE = DIM * NQ;
    for (int task = tid; task < nel * TPE; task += nth) {
      const int el = task / TPE, lt = task % TPE;
      const int fam = lt / NQ, rem = lt % NQ;
      // lanes run along a line (a fastest) for the families of stride 1 and Q,
      // across lines (L fastest) for the family of stride Q^2: consecutive
      // lanes then address distinct LDS banks
      const bool across = DIM == 3 && fam == 2;
      const int L = across ? rem % LPF : rem / Q, a = across ? rem / LPF : rem % Q;
      const double* sNe = sN + el * Sh::SCR;
      const double* sRe = sR + el * NC * NQ;
      double* sXe = sX + el * NC * NQ;
      const double* g = gvol + (e0 + el) * NGV * NQ;
      if constexpr (DIM == 2) {
        if (fam == 0)
          vol_task_vjp<DIM, P, FLUX, 2>(sNe, g, sRe, sXe, Q * L, 1, a, T.A + 0 * Q * Q, T.A + 1 * Q * Q, 0, 2, S);
        else
          vol_task_vjp<DIM, P, FLUX, 1>(sNe, g, sRe, sXe, L, Q, a, T.A + 2 * Q * Q, nullptr, 4, 0, S);
      } else {
        if (fam == 0)
          vol_task_vjp<DIM, P, FLUX, 2>(sNe, g, sRe, sXe, Q * L, 1, a, T.A + 0 * Q * Q, T.A + 1 * Q * Q, 0, 3, S);
        else if (fam == 1)
          vol_task_vjp<DIM, P, FLUX, 2>(sNe, g, sRe, sXe, (L % Q) + Q * Q * (L / Q), Q, a, T.A + 2 * Q * Q,
                                        T.A + 3 * Q * Q, 6, 9, S);
        else
          vol_task_vjp<DIM, P, FLUX, 1>(sNe, g, sRe, sXe, L, Q * Q, a, T.A + 4 * Q * Q, nullptr, 12, 0, S);
      }
    }
  }
  __syncthreads();

  // ---- facet-correction pairs: one task per volume node i (owns x_bar_i)
  for (int task = tid; task < nel * NQ; task += nth) {
    const int el = task / NQ, t = task % NQ;
    const double* sNe = sN + el * Sh::SCR;
    const double* sFe = sF + el * 8 * NFQ;
    const double* sTe = sT + el * NC * NFQ;
    double* sXFe = sXF + el * NC * NFQ;
    const double* g = gvol + (e0 + el) * NGV * NQ;
    const double* gf = gfac + (e0 + el) * (DIM + 1) * NFQ;
    NodeBar<DIM> Vib;
    zero(Vib);
    double rbi[NC];
    int i;
    if constexpr (DIM == 2) {
      const int b2 = t % Q, b1 = t / Q;
      i = b1 + Q * b2;
#pragma unroll
      for (int c = 0; c < NC; ++c) rbi[c] = sR[(el * NC + c) * NQ + i];
      const Node<DIM> Vi = load_node<DIM>(sNe, NQ, i);
      const double w1 = T.wl[b1], w2 = T.wl[b2];
      double gA[2], gB[2], gC[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const double g1 = g[(0 + m) * NQ + i] / w2;
        const double g2 = 2.0 * g[(2 + m) * NQ + i] / w2;
        gA[m] = (g1 + g2) * 0.70710678118654752440;
        gB[m] = -g1;
        gC[m] = -2.0 * g[(4 + m) * NQ + i] / w1;
      }
      facet_task_vjp<DIM, P, FLUX>(Vi, gA, sFe, sTe, sXFe, gf, 1 * NQF + b2, T.lgp1[b1] * T.wf[1 * NQF + b2], S,
                                   rbi, Vib);
      facet_task_vjp<DIM, P, FLUX>(Vi, gB, sFe, sTe, sXFe, gf, 2 * NQF + b2, T.lgm1[b1] * T.wf[2 * NQF + b2], S,
                                   rbi, Vib);
      facet_task_vjp<DIM, P, FLUX>(Vi, gC, sFe, sTe, sXFe, gf, 0 * NQF + b1, T.lgm1[b2] * T.wf[0 * NQF + b1], S,
                                   rbi, Vib);
      double xi[NC];
      reduce_bar<DIM>(Vi, Vib, xi);
#pragma unroll
      for (int c = 0; c < NC; ++c) sX[(el * NC + c) * NQ + i] += xi[c];
    } else {
      const int b3 = t % Q, b2 = (t / Q) % Q, b1 = t / (Q * Q);
      i = b1 + Q * (b2 + Q * b3);
#pragma unroll
      for (int c = 0; c < NC; ++c) rbi[c] = sR[(el * NC + c) * NQ + i];
      const Node<DIM> Vi = load_node<DIM>(sNe, NQ, i);
      const double inv23 = 1.0 / (T.wl[b2] * T.wj[b3]);
      const double inv13 = 1.0 / (T.wl[b1] * T.wj[b3]);
      const double inv12 = 1.0 / (T.wl[b1] * T.wl[b2] * (1.0 - T.xl[b2]));
      double gA[3], gB[3], gC[3], gD[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const double g1 = 2.0 * g[(0 + m) * NQ + i] * inv23;
        const double g23 = 4.0 * g[(3 + m) * NQ + i] * inv23;
        gA[m] = (g1 + g23) * 0.57735026918962576451;
        gB[m] = -g1;
        gC[m] = -4.0 * g[(6 + m) * NQ + i] * inv13;
        gD[m] = -8.0 * g[(12 + m) * NQ + i] * inv12;
      }
      const int j23 = b2 + Q * b3;
      facet_task_vjp<DIM, P, FLUX>(Vi, gA, sFe, sTe, sXFe, gf, 1 * NQF + j23, T.lgp1[b1] * T.wf[1 * NQF + j23], S,
                                   rbi, Vib);
      facet_task_vjp<DIM, P, FLUX>(Vi, gB, sFe, sTe, sXFe, gf, 2 * NQF + j23, T.lgm1[b1] * T.wf[2 * NQF + j23], S,
                                   rbi, Vib);
      const int j13 = b1 + Q * b3;
      facet_task_vjp<DIM, P, FLUX>(Vi, gC, sFe, sTe, sXFe, gf, 0 * NQF + j13, T.lgm1[b2] * T.wf[0 * NQF + j13], S,
                                   rbi, Vib);
      const double cz = T.gjm1[b3];
      // kept rolled: unrolled, the pair adjoints of all Q partners stay live
      // (tet VGPRs 388-512 with spills at p = 8; rolled about 225, which
      // doubles the waves per SIMD where LDS allows: p = 4 1.67 vs 2.27 ms)
#pragma unroll 1
      for (int m = 0; m < Q; ++m) {
        int a2 = m + b2 + b3;
        a2 = a2 % Q;
        const int j = 3 * NQF + b1 + Q * a2;
        facet_task_vjp<DIM, P, FLUX>(Vi, gD, sFe, sTe, sXFe, gf, j, cz * T.I42[a2 * Q + b2] * T.wf[j], S, rbi, Vib);
      }
      double xi[NC];
      reduce_bar<DIM>(Vi, Vib, xi);
#pragma unroll
      for (int c = 0; c < NC; ++c) sX[(el * NC + c) * NQ + i] += xi[c];
    }
  }
  if constexpr (VM::FG) __threadfence();
  __syncthreads();

  // ---- interface flux: f*_bar = -B_j t_bar_j; own side into LDS, neighbour side
  //      converted to entropy variables and written for the neighbour
  bad = false;
  for (int o = tid; o < nel * NFQ; o += nth) {
    const int j = o % NFQ, le = o / NFQ;
    const int64_t e = e0 + le;
    const Node<DIM> Um = load_node<DIM>(sF + le * 8 * NFQ, NFQ, j);
    const int32_t addr = conn[e * NFQ + j];
    double w[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) w[c] = wfb[addr + c * NFQ];
    Node<DIM> Up;
    bad |= !from_entropy<DIM>(w, S.gamma, S.gm1_inv, Up);
    double nJ[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) nJ[i] = gfac[(e * (DIM + 1) + i) * NFQ + j];
    const double Jf = gfac[(e * (DIM + 1) + DIM) * NFQ + j];
    double Fb[NC];
    const double wj = T.wf[j];
#pragma unroll
    for (int c = 0; c < NC; ++c) Fb[c] = -wj * sT[(le * NC + c) * NFQ + j];
    NodeBar<DIM> Umb, Upb;
    zero(Umb);
    zero(Upb);
    interface_flux_vjp<DIM, FLUX>(Um, Up, nJ, Jf, S.gamma, S.gm1_inv, S.dissipation, Fb, Umb, Upb);
    double xm[NC], xp[NC], wp[NC];
    reduce_bar<DIM>(Um, Umb, xm);
#pragma unroll
    for (int c = 0; c < NC; ++c) sXF[(le * NC + c) * NFQ + j] += xm[c];
    reduce_bar<DIM>(Up, Upb, xp);
    xbar_to_wbar<DIM>(Up, xp, S.gm1_inv, wp);
#pragma unroll
    for (int c = 0; c < NC; ++c) xbar[(e * NC + c) * NFQ + j] = wp[c];
  }
  if (bad) atomicOr(flag, 1);
  if constexpr (VM::FG) __threadfence();
  __syncthreads();

  // ---- x_bar -> w_bar at volume and own facet nodes
  for (int o = tid; o < nel * NQ; o += nth) {
    const int k = o % NQ, el = o / NQ;
    const Node<DIM> nd = load_node<DIM>(sN + el * Sh::SCR, NQ, k);
    double xb[NC], wb[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) xb[c] = sX[(el * NC + c) * NQ + k];
    xbar_to_wbar<DIM>(nd, xb, S.gm1_inv, wb);
#pragma unroll
    for (int c = 0; c < NC; ++c) sX[(el * NC + c) * NQ + k] = wb[c];
  }
  for (int o = tid; o < nel * NFQ; o += nth) {
    const int j = o % NFQ, el = o / NFQ;
    const Node<DIM> nd = load_node<DIM>(sF + el * 8 * NFQ, NFQ, j);
    double xb[NC], wb[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) xb[c] = sXF[(el * NC + c) * NFQ + j];
    xbar_to_wbar<DIM>(nd, xb, S.gm1_inv, wb);
#pragma unroll
    for (int c = 0; c < NC; ++c) sXF[(el * NC + c) * NFQ + j] = wb[c];
  }
  __syncthreads();
  // ---- w~_bar (partial) = V^T (w_bar + R^T w^z_bar)
  facet_lift<DIM, P>(sXF, sF, T, nec, [&](int o, double d) { sX[o] += d; });
  __syncthreads();
  xform_Vt<DIM, P>(sX, T1, T2, sX, T, nec);
  for (int o = tid; o < nec * NP; o += nth) gpart[e0 * NC * NP + o] = sX[o];
}

// ------------------------------------------------------------------ VK1: reverse of the entropy projection
// g holds the partial w~_bar on entry and u~_bar on exit (same element, read
// before it is written).
template <int DIM, int P>
__global__ void __launch_bounds__((VjpLaunch<DIM, P>::BS))
k_projection_vjp(const double* __restrict__ u, double* g, const double* __restrict__ xbar,
                 const double* __restrict__ gvol, const int32_t* __restrict__ conn, DevTables T0, Scheme S,
                 int64_t ne, double* gscr) {
  using Sh = Shape<DIM, P>;
  constexpr int EPB = Launch<DIM, P>::EPB;
  constexpr int NC = Sh::NC, NQ = Sh::NQ, NP = Sh::NP, NFQ = Sh::NFQ, NGV = Sh::NGV;
  using VM = VjpMem<DIM, P>;
  constexpr int NB = VM::NB;
  static_assert(!VM::BG || EPB == 1, "workspace slices are per element");
  __shared__ double sM[EPB * NC * NP];
  __shared__ double sA[EPB * NC * NQ];
  __shared__ double sB_l[VM::BG ? 1 : EPB * NC * NB];      // gathered facet cotangents, later u at the nodes
  __shared__ double sS[EPB * Sh::XSCR];
  double* const sB = VM::BG ? gscr + (int64_t)blockIdx.x * VM::SLICE : sB_l;
  constexpr int KB = 8 * EPB * (NC * NP + NC * NQ + (VM::BG ? 0 : NC * NB) + Sh::XSCR);
  constexpr unsigned TM =
      tab_keeps_wgs<DIM, P, TAB_PSI | TAB_FACET, TAB_PSI | TAB_FACET | TAB_PSIM>(KB, wave_cap<DIM, P>())
          ? (TAB_PSI | TAB_FACET | TAB_PSIM)
          : tab_mask<DIM, P, TAB_PSI | TAB_FACET>(KB);
  __shared__ double sTab[TM ? TabLds<DIM, P, TM>::SIZE : 1];
  const DevTables T = stage_tables<DIM, P, TM>(T0, sTab);
  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const int nel = (int)((ne - e0) < EPB ? (ne - e0) : EPB);
  const int nec = nel * NC;
  const int tid = threadIdx.x, nth = blockDim.x;
  double* T1 = sS;
  double* T2 = sS + EPB * Sh::T1;

  // ---- cotangents of this element's facet values written by its neighbours:
  //      the facet permutation is an involution, so the neighbour of node j
  //      stored them at the address conn gives for j.  In a mixed-degree
  //      batch, a facet whose neighbour has another degree points at this
  //      element's exterior slot (addresses from ne NC NFQ on): that neighbour
  //      reads this element's w~, not its facet values, so nothing is gathered
  //      there (its cotangent reaches w~_bar through the mixed-interface adjoint)
  const int64_t own_end = ne * NC * NFQ;
  for (int o = tid; o < nec * NFQ; o += nth) {
    const int j = o % NFQ, c = (o / NFQ) % NC, el = o / (NC * NFQ);
    const int32_t addr = conn[(e0 + el) * NFQ + j];
    sB[o] = addr < own_end ? xbar[addr + c * NFQ] : 0.0;
  }
  __syncthreads();
  facet_lift<DIM, P>(sB, sS, T, nec, [&](int o, double d) { sA[o] = d; });
  __syncthreads();
  xform_Vt<DIM, P>(sA, T1, T2, sM, T, nec);
  for (int o = tid; o < nec * NP; o += nth) sM[o] += g[e0 * NC * NP + o];
  __syncthreads();
  // ---- Y_bar = (w J) V V^T (w/J) V w~_bar
  xform_V<DIM, P>(sM, T1, T2, sA, T, nec);
  for (int o = tid; o < nec * NQ; o += nth) {
    const int k = o % NQ, le = o / (NC * NQ);
    sA[o] *= gvol[((e0 + le) * NGV + NGV - 1) * NQ + k];
  }
  __syncthreads();
  if constexpr ((TM & TAB_PSIM) != 0) {
    xform_VVt<DIM, P>(sA, T1, T2, sA, T, nec);
  } else {
    xform_Vt<DIM, P>(sA, T1, T2, sM, T, nec);
    xform_V<DIM, P>(sM, T1, T2, sA, T, nec);
  }
  for (int o = tid; o < nec * NQ; o += nth) {
    const int k = o % NQ, le = o / (NC * NQ);
    sA[o] *= gvol[((e0 + le) * NGV + NGV - 2) * NQ + k];
  }
  // ---- u = V u~ at the nodes, u_bar = W'(u)^T Y_bar
  for (int o = tid; o < nec * NP; o += nth) sM[o] = u[e0 * NC * NP + o];
  __syncthreads();
  xform_V<DIM, P>(sM, T1, T2, sB, T, nec);
  for (int o = tid; o < nel * NQ; o += nth) {
    const int k = o % NQ, el = o / NQ;
    double uu[NC], yb[NC], ub[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      uu[c] = sB[(el * NC + c) * NQ + k];
      yb[c] = sA[(el * NC + c) * NQ + k];
      ub[c] = 0.0;
    }
    entropy_vars_vjp<DIM>(uu, yb, S.gamma, S.gm1_inv, ub);
#pragma unroll
    for (int c = 0; c < NC; ++c) sA[(el * NC + c) * NQ + k] = ub[c];
  }
  __syncthreads();
  xform_Vt<DIM, P>(sA, T1, T2, sM, T, nec);
  for (int o = tid; o < nec * NP; o += nth) g[e0 * NC * NP + o] = sM[o];
}

// ------------------------------------------------------------------ discrete adjoint of classical RK4
// acc = (first ? ubar : acc) + G;  kb = cu ubar + cg G
__global__ void k_adj_stage(double* __restrict__ acc, double* __restrict__ kb, const double* __restrict__ ubar,
                            const double* __restrict__ G, double cu, double cg, int first, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double gi = G[i], ui = ubar[i];
    acc[i] = (first ? ui : acc[i]) + gi;
    kb[i] = cu * ui + cg * gi;
  }
}

__global__ void k_scale(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

// ------------------------------------------------------------------ dispatch
// VK2 (which = 0) or VK1 (which = 1) of one plan; K1 (and, in a batch, the
// mixed-interface exterior values) must have run before VK2
template <int DIM, int P>
static int run_vjp_part(const esd_plan* pl, int which, const double* u, const double* vbar, double* grad,
                        Workspace ws, hipStream_t s) {
  using L = VjpLaunch<DIM, P>;
  const int64_t nb = (pl->ne + L::EPB - 1) / L::EPB;
  if (which == 0) {
    if (pl->scheme.ecflux == FLUX_RANOCHA)
      hipLaunchKernelGGL((k_rhs_vjp<DIM, P, FLUX_RANOCHA>), dim3(nb), dim3(L::BS), 0, s, ws.wt, ws.wf, vbar, grad,
                         ws.xbar, pl->d_gvol, pl->d_gfac, pl->d_conn, pl->tab, pl->scheme, pl->ne, pl->d_flag,
                         ws.vscr);
    else
      hipLaunchKernelGGL((k_rhs_vjp<DIM, P, FLUX_CHANDRASHEKAR>), dim3(nb), dim3(L::BS), 0, s, ws.wt, ws.wf, vbar,
                         grad, ws.xbar, pl->d_gvol, pl->d_gfac, pl->d_conn, pl->tab, pl->scheme, pl->ne, pl->d_flag,
                         ws.vscr);
  } else {
    hipLaunchKernelGGL((k_projection_vjp<DIM, P>), dim3(nb), dim3(L::BS), 0, s, u, grad, ws.xbar, pl->d_gvol,
                       pl->d_conn, pl->tab, pl->scheme, pl->ne, ws.vscr);
  }
  return (int)hipGetLastError();
}

int vjp_scratch_doubles(int dim, int p) {
#define X(D, PP) \
  if (dim == D && p == PP) return VjpMem<D, PP>::SLICE;
  ESD_TRI_DEGREES(X)
  ESD_TET_VJP_DEGREES(X)
#undef X
  return 0;
}

int launch_vjp_part(const esd_plan* pl, int which, const double* u, const double* vbar, double* grad, Workspace ws,
                    hipStream_t s) {
#define X(D, PP) \
  if (pl->dim == D && pl->p == PP) return run_vjp_part<D, PP>(pl, which, u, vbar, grad, ws, s);
  ESD_TRI_DEGREES(X)
  ESD_TET_VJP_DEGREES(X)
#undef X
  return -1;
}

int launch_vjp(const esd_plan* pl, const double* u, const double* vbar, double* grad, Workspace ws, hipStream_t s) {
  if (!vjp_degree_supported(pl->dim, pl->p)) return -1;
  int rc = launch_entropy_projection(pl, u, ws, s);
  if (rc == 0) rc = launch_vjp_part(pl, 0, u, vbar, grad, ws, s);
  if (rc == 0) rc = launch_vjp_part(pl, 1, u, vbar, grad, ws, s);
  return rc;
}

int launch_adj_stage(double* acc, double* kb, const double* ubar, const double* G, double cu, double cg, int first,
                     int64_t n, hipStream_t s) {
  const int bs = 256;
  int64_t nb = (n + bs - 1) / bs;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_adj_stage, dim3(nb), dim3(bs), 0, s, acc, kb, ubar, G, cu, cg, first, n);
  return (int)hipGetLastError();
}

int launch_scale(double* y, const double* x, double a, int64_t n, hipStream_t s) {
  const int bs = 256;
  int64_t nb = (n + bs - 1) / bs;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_scale, dim3(nb), dim3(bs), 0, s, y, x, a, n);
  return (int)hipGetLastError();
}

}  // namespace esd
