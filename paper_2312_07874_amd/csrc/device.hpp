// Device building blocks shared by the forward and adjoint kernels (gfx950):
// element shapes and launch shapes per degree, PKD mode indexing, the
// sum-factorised transforms V and V^T (Sec. 5.2), facet extrapolation R and its
// transpose (eqs. r_2d, r_3d), and node records in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include "physics.hpp"
#include "plan.hpp"

namespace esd {

// degrees built into the library, per dimension
#define ESD_TRI_DEGREES(X) X(2, 1) X(2, 2) X(2, 3) X(2, 4) X(2, 5) X(2, 6) X(2, 7) X(2, 8) X(2, 9) X(2, 10)
#define ESD_TET_DEGREES(X) X(3, 1) X(3, 2) X(3, 3) X(3, 4) X(3, 5) X(3, 6) X(3, 7) X(3, 8) X(3, 9) X(3, 10)
// the adjoint kernels (at p = 9, 10 part of their per-element arrays in the workspace)
#define ESD_TET_VJP_DEGREES(X) X(3, 1) X(3, 2) X(3, 3) X(3, 4) X(3, 5) X(3, 6) X(3, 7) X(3, 8) X(3, 9) X(3, 10)

// ------------------------------------------------------------------ shapes
template <int DIM, int P>
struct Shape {
  static constexpr int Q = P + 1;
  static constexpr int NC = DIM + 2;
  static constexpr int NQ = DIM == 2 ? Q * Q : Q * Q * Q;
  static constexpr int NP = DIM == 2 ? (P + 1) * (P + 2) / 2 : (P + 1) * (P + 2) * (P + 3) / 6;
  static constexpr int NF = DIM + 1;
  static constexpr int NQF = DIM == 2 ? Q : Q * Q;
  static constexpr int NFQ = NF * NQF;
  static constexpr int NPAIR = (P + 1) * (P + 2) / 2;
  static constexpr int NGV = DIM == 2 ? 8 : 17;
  static constexpr int LPF = DIM == 2 ? Q : Q * Q;           // lines per family
  static constexpr int NLINES = DIM * LPF;
  static constexpr int T1 = DIM == 2 ? NC * (P + 1) * Q : NC * NPAIR * Q;
  static constexpr int T2 = DIM == 2 ? 0 : NC * (P + 1) * Q * Q;
  static constexpr int XSCR = T1 + T2;                                 // transform scratch per element
  static constexpr int SCR = (T1 + T2 > 8 * NQ) ? (T1 + T2) : 8 * NQ;   // and the right-hand side's node records
  // the right-hand-side kernel keeps the own facet node records in LDS when
  // node data, r, facet records and facet sums fit the 160 KB of a CU
  static constexpr bool K2_FACET_LDS = 8 * (SCR + NC * NQ + 8 * NFQ + NC * NFQ) <= 160 * 1024;
};

template <int DIM, int P>
struct Launch;  // block size and elements per block
template <int P>
struct Launch<3, P> {
  // one element per workgroup; small workgroups keep several elements in
  // flight per CU, which hides the latency of the barrier-separated phases
  static constexpr int EPB = 1;
  // measured on MI355X (K2 at p = 4..8): 128, 192, 256, 256, 512 threads
  static constexpr int BS = P <= 3 ? 64 : (P == 4 ? 128 : (P == 5 ? 192 : (P <= 7 ? 256 : 512)));
  // K1 and K2 are compiled for up to BSMAX threads and launched with BS or with
  // the block size the autotuner picked (their loops take any multiple of 64:
  // the matrix-core transform stages need whole waves)
  static constexpr int BSMAX = 512;
  static_assert(P <= 10, "tetrahedra up to p = 10");
  static_assert(BS % 64 == 0 && BSMAX % 64 == 0, "whole waves");
};
template <int P>
struct Launch<2, P> {
  // measured on MI355X (vortex, 8192 triangles): 8 elements per workgroup at
  // p = 4 (0.074 -> 0.063 ms per residual over 12), 3 at p = 8 (0.370 -> 0.328 ms over 6)
  static constexpr int EPB = (P <= 7) ? 8 : 3;
  static constexpr int NQ = (P + 1) * (P + 1);
  static constexpr int BS = ((EPB * NQ + 63) / 64) * 64;
  static constexpr int BSMAX = 2 * BS < 768 ? 2 * BS : (BS > 768 ? BS : 768);   // <= 3 waves per SIMD
  static_assert(BS % 64 == 0 && BSMAX % 64 == 0, "whole waves");
};

__device__ __forceinline__ int pair_index(int P, int a1, int a2) { return a1 * (P + 1) - a1 * (a1 - 1) / 2 + a2; }
__device__ __forceinline__ void decode_pair(int P, int pr, int& a1, int& a2) {
  a1 = 0;
  int cnt = P + 1;
  while (pr >= cnt) {
    pr -= cnt;
    ++a1;
    --cnt;
  }
  a2 = pr;
}
__device__ __forceinline__ int tet_mode_base(int P, int a1, int a2) {
  int b = 0;
  for (int i = 0; i < a1; ++i) b += (P + 1 - i) * (P + 2 - i) / 2;
  return b + a2 * (P + 1 - a1) - a2 * (a2 - 1) / 2;
}
__device__ __forceinline__ void decode_tet_mode(int P, int m, int& a1, int& a2, int& a3) {
  a1 = 0;
  int cnt = (P + 1) * (P + 2) / 2;
  while (m >= cnt) {
    m -= cnt;
    ++a1;
    cnt = (P + 1 - a1) * (P + 2 - a1) / 2;
  }
  a2 = 0;
  cnt = P + 1 - a1;
  while (m >= cnt) {
    m -= cnt;
    ++a2;
    --cnt;
  }
  a3 = m;
}
__device__ __forceinline__ void decode_tri_mode(int P, int m, int& a1, int& a2) {
  a1 = 0;
  int cnt = P + 1;
  while (m >= cnt) {
    m -= cnt;
    ++a1;
    --cnt;
  }
  a2 = m;
}

// ------------------------------------------------------------------ operator tables in LDS
// The transforms and the facet extrapolation index psi2, psi3, I42 and the 1D
// facet weights by a lane-dependent mode or node; as global loads each value
// costs a vector-memory instruction (a texture-addresser pass over 64 lane
// addresses), which made the transforms the largest part of both kernels.
// Kernels copy these tables into LDS at their start (before their first
// barrier) where LDS allows; psi1 stays in global memory: the transforms index
// it uniformly, through scalar loads.
constexpr int LDS_BYTES = 160 * 1024;
enum : unsigned {
  TAB_PSI = 1,     // psi2, psi3 (transforms)
  TAB_FACET = 2,   // I42, lgm1, lgp1, gjm1 (facet extrapolation and lift)
  TAB_PSIM = 4,    // psiM (the composed stage of V V^T)
  TAB_PSI2 = 8,    // psi2 alone (where both do not fit: it is read Q / (P+1-s) times as often as psi3)
};
template <int DIM, int P, unsigned M>
struct TabLds {
  static constexpr int Q = P + 1;
  static constexpr int NPSI = (P + 1) * (P + 1) * Q;
  static constexpr int SIZE = ((M & TAB_PSI) ? (DIM == 2 ? 1 : 2) * NPSI : ((M & TAB_PSI2) ? NPSI : 0)) +
                              ((M & TAB_FACET) ? Q * Q + 3 * Q : 0) + ((M & TAB_PSIM) ? (P + 1) * Q * Q : 0);
};
// the tables W if a kernel using base_bytes of LDS still fits with them, else none
template <int DIM, int P, unsigned W>
constexpr unsigned tab_mask(int base_bytes) {
  return base_bytes + 8 * TabLds<DIM, P, W>::SIZE <= LDS_BYTES ? W : 0u;
}

// whether staging the tables W1 instead of W0 keeps the number of workgroups
// per CU, for a kernel using base_bytes of LDS besides them whose waves allow
// at most cap workgroups per CU
template <int DIM, int P, unsigned W0, unsigned W1>
constexpr bool tab_keeps_wgs(int base_bytes, int cap) {
  const int b0 = base_bytes + 8 * TabLds<DIM, P, W0>::SIZE, b1 = base_bytes + 8 * TabLds<DIM, P, W1>::SIZE;
  const int g0 = LDS_BYTES / b0 < cap ? LDS_BYTES / b0 : cap, g1 = LDS_BYTES / b1 < cap ? LDS_BYTES / b1 : cap;
  return b1 <= LDS_BYTES && g1 >= g0;
}
// workgroups per CU that the waves of a default-sized block allow at 4 waves
// per SIMD (kernels at <= 128 VGPRs; an upper bound otherwise)
template <int DIM, int P>
constexpr int wave_cap() {
  return 16 / ((Launch<DIM, P>::BS + 63) / 64) > 0 ? 16 / ((Launch<DIM, P>::BS + 63) / 64) : 1;
}

// copies the tables M into buf (TabLds<DIM, P, M>::SIZE doubles of LDS) and
// returns T with those pointers redirected; no barrier
template <int DIM, int P, unsigned M>
__device__ __forceinline__ DevTables stage_tables(const DevTables& T, double* buf) {
  DevTables R = T;
  if constexpr (M != 0) {
    using L = TabLds<DIM, P, M>;
    constexpr int Q = L::Q;
    const int tid = threadIdx.x, nth = blockDim.x;
    int off = 0;
    auto copy = [&](const double* src, int n) {
      for (int o = tid; o < n; o += nth) buf[off + o] = src[o];
      const double* d = buf + off;
      off += n;
      return d;
    };
    if constexpr ((M & TAB_PSI) != 0) {
      R.psi2 = copy(T.psi2, L::NPSI);
      if constexpr (DIM == 3) R.psi3 = copy(T.psi3, L::NPSI);
    } else if constexpr ((M & TAB_PSI2) != 0) {
      R.psi2 = copy(T.psi2, L::NPSI);
    }
    if constexpr ((M & TAB_PSIM) != 0) R.psiM = copy(T.psiM, (P + 1) * Q * Q);
    if constexpr ((M & TAB_FACET) != 0) {
      R.I42 = copy(T.I42, Q * Q);
      R.lgm1 = copy(T.lgm1, Q);
      R.lgp1 = copy(T.lgp1, Q);
      R.gjm1 = copy(T.gjm1, Q);
    }
  }
  return R;
}

// ------------------------------------------------------------------ sum-factorised PKD transforms
// in/out arrays are [nel*NC][...] contiguous per (element, variable); all
// threads of the block participate.  Every thread produces a whole line of
// outputs from one set of LDS loads (register blocking along the contracted
// direction).  The stages below end without a barrier; the transforms put one
// after each.
//
// Stage layouts: triangles T1 [ec][a1][i2]; tetrahedra T1 [ec][(a1,a2)][i3],
// T2 [ec][l][a1 rotated by i2] with l = i2 + Q i3: the P + 1 = Q values of
// the eta1 line l occupy the same Q doubles as that line's nodal values, so
// the last stage of V and the first of V^T may run in place (T2 equal to the
// nodal array): each thread reads its whole line before writing it, and no
// other thread touches it.  Entry a1 of line l sits at (a1 + i2) mod Q, which
// spreads the lanes of a wave (consecutive lines) over the LDS banks.
template <int P>
struct Unroll {
  static constexpr int Q = P + 1;
  // contractions unrolled fully while the psi1 table fits scalar registers,
  // partly above (loads of the next iterations overlap the multiply-adds).
  // Measured on MI355X, K1 / K2 per residual against the rolled loop: tet p8
  // (24,576 elements) 2.15 / 6.25 -> 2.00 / 6.04 ms with 6, p9 (10,368)
  // 1.19 / 3.78 -> 1.04 / 3.51 ms with 2 (6: 1.31 / 3.54), p10 2.86 / 7.54 ->
  // 2.56 / 7.06 ms with 6; full unrolling is slower at p9 and p10
  static constexpr int XU = Q <= 7 ? Q : (Q == 10 ? 2 : 6);
};

// V, first stage: the modes of the last direction to its nodes
template <int DIM, int P>
__device__ __forceinline__ void v_first(const double* uh, double* T1, const DevTables& T, int nec) {
  using S = Shape<DIM, P>;
  constexpr int Q = S::Q, XU = Unroll<P>::XU;
  // stages whose table is indexed per lane (read from LDS) unroll one degree
  // further on tetrahedra (measured: K1 at p = 7 2.49 -> 2.19 ms; p = 8 unchanged)
  constexpr int XL = (DIM == 3 && Q <= 8) ? Q : XU;
  const int tid = threadIdx.x, nth = blockDim.x;
  if constexpr (DIM == 2) {
    // T1[ec][a1][i2] = sum_a2 psi2[a1][a2][i2] u~[ec][(a1,a2)]
    for (int o = tid; o < nec * (P + 1); o += nth) {
      const int a1 = o % (P + 1), ec = o / (P + 1);
      const int mb = a1 * (P + 1) - a1 * (a1 - 1) / 2;
      double acc[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) acc[i] = 0.0;
#pragma unroll XU
      for (int a2 = 0; a2 <= P; ++a2) {
        if (a2 <= P - a1) {
          const double x = uh[ec * S::NP + mb + a2];
          const double* ps = T.psi2 + (a1 * (P + 1) + a2) * Q;
#pragma unroll
          for (int i = 0; i < Q; ++i) acc[i] += ps[i] * x;
        }
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) T1[(ec * (P + 1) + a1) * Q + i] = acc[i];
    }
  } else {
    // T1[ec][pr][i3] = sum_a3 psi3[s][a3][i3] u~[ec][(a1,a2,a3)]
    for (int o = tid; o < nec * S::NPAIR; o += nth) {
      const int pr = o % S::NPAIR, ec = o / S::NPAIR;
      int a1, a2;
      decode_pair(P, pr, a1, a2);
      const int s = a1 + a2, mb = tet_mode_base(P, a1, a2);
      double acc[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) acc[i] = 0.0;
#pragma unroll XL
      for (int a3 = 0; a3 <= P; ++a3) {
        if (a3 <= P - s) {
          const double x = uh[ec * S::NP + mb + a3];
          const double* ps = T.psi3 + (s * (P + 1) + a3) * Q;
#pragma unroll
          for (int i = 0; i < Q; ++i) acc[i] += ps[i] * x;
        }
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) T1[(ec * S::NPAIR + pr) * Q + i] = acc[i];
    }
  }
}

// V, middle stage of tetrahedra: T2(ec, a1, i2 + Q i3) = sum_a2 psi2[a1][a2][i2] T1[ec][(a1,a2)][i3]
template <int P>
__device__ __forceinline__ void v_second(const double* T1, double* T2, const DevTables& T, int nec) {
  using S = Shape<3, P>;
  constexpr int Q = S::Q, XL = Q <= 8 ? Q : Unroll<P>::XU;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int o = tid; o < nec * (P + 1) * Q; o += nth) {
    const int i3 = o % Q, a1 = (o / Q) % (P + 1), ec = o / (Q * (P + 1));
    const int pb = pair_index(P, a1, 0);
    double acc[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) acc[i] = 0.0;
#pragma unroll XL
    for (int a2 = 0; a2 <= P; ++a2) {
      if (a2 <= P - a1) {
        const double x = T1[(ec * S::NPAIR + pb + a2) * Q + i3];
        const double* ps = T.psi2 + (a1 * (P + 1) + a2) * Q;
#pragma unroll
        for (int i = 0; i < Q; ++i) acc[i] += ps[i] * x;
      }
    }
    // line l = i + Q i3 of T2, entry a1 at (a1 + i) mod Q
    double* t2 = T2 + ((int64_t)ec * Q * Q + Q * i3) * Q;
#pragma unroll
    for (int i = 0; i < Q; ++i) t2[i * Q + (a1 + i < Q ? a1 + i : a1 + i - Q)] = acc[i];
  }
}

// ------------------------------------------------------------------ matrix-core form of the eta1 stages
// On tetrahedra the last stage of V and the first of V^T contract the Q
// values of each eta1 line with psi1, the same Q x Q matrix for all N = nec Q^2
// lines: a dense product that v_mfma_f64_16x16x4 evaluates 16 lines at a time
// (one wave per tile, ceil(Q / 4) steps of K = 4, rows and steps beyond Q
// zero).  Register layout of that instruction on gfx950 (measured with one-hot
// inputs): A[m][k] in lane m + 16 k, B[k][n] in lane n + 16 k, D[m][n] in lane
// n + 16 (m % 4), element m / 4.  Measured against the lane-per-line loop on
// the same LDS-staged stage (4,096 elements, measure/transform_mfma.hip):
// p = 6 0.031 -> 0.023 ms, p = 8 0.072 -> 0.053, p = 10 0.177 -> 0.147 ms.
// Inside the kernels (tgv on tetrahedra, K1 + K2 per call) it pays from
// p = 6 on (p = 6 3.28 -> 3.23 ms, p = 8 7.89 -> 7.48, p = 10 8.17 -> 7.40)
// and costs below (p = 4 0.79 -> 0.91, p = 5 1.50 -> 1.77: few lines per
// element, tiles half padding, and the extra registers cost occupancy).
// Each wave reads all Q values of its 16 lines before writing any, so the
// stages stay in place over a line's own slots.  The instruction reads the
// registers of all 64 lanes: the tiles go to whole waves (block sizes are
// multiples of 64), the lanes of a tile's missing lines contribute zeros.
typedef double mf_d4 __attribute__((ext_vector_type(4)));
template <int P>
struct MfmaEta1 {
  static constexpr int Q = P + 1;
  static constexpr bool ON = Q >= 7;
  // the entropy projection alone (K1) loses at p = 6, 7 (0.77 -> 0.86 ms,
  // 1.55 -> 1.70 ms on 24,576 elements) and gains from p = 8 on
  static constexpr bool ON_PROJ = Q >= 9;
  static constexpr int KS = (Q + 3) / 4;
};

// V, last stage: sum over a1 with psi1 into the nodes (Tin is T1 on
// triangles, T2 on tetrahedra)
template <int DIM, int P, bool MF = MfmaEta1<P>::ON>
__device__ __forceinline__ void v_last(const double* Tin, double* out, const DevTables& T, int nec) {
  using S = Shape<DIM, P>;
  constexpr int Q = S::Q, XU = Unroll<P>::XU;
  constexpr int L = DIM == 2 ? Q : Q * Q;   // lines of the last stage per (element, variable)
  const int tid = threadIdx.x, nth = blockDim.x;
  // out[ec][i1 + Q l] = sum_a1 psi1[a1][i1] Tin(ec, a1, l); on tetrahedra Tin
  // may equal out (the line is read whole before it is written)
  if constexpr (DIM == 3 && MF) {
    constexpr int KS = MfmaEta1<P>::KS;
    const int lane = tid & 63, n = lane % 16, kq = lane / 16;
    double a[KS];
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      const int k = 4 * st + kq;
      a[st] = (n < Q && k < Q) ? T.psi1[k * Q + n] : 0.0;   // A[m = n][k] = psi1[k][m]
    }
    const int ncol = nec * L, tiles = (ncol + 15) / 16;
    for (int t = tid >> 6; t < tiles; t += nth >> 6) {
      const int o = t * 16 + n;
      const bool valid = o < ncol;
      const double* tl = Tin + (int64_t)(valid ? o : 0) * Q;
      const int r = (o % L) % Q;
      mf_d4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < KS; ++st) {
        const int k = 4 * st + kq;
        const double b = (valid && k < Q) ? tl[k + r < Q ? k + r : k + r - Q] : 0.0;
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b, d, 0, 0, 0);
      }
      double* ol = out + (int64_t)(valid ? o : 0) * Q;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = 4 * i + kq;
        if (valid && m < Q) ol[m] = d[i];
      }
    }
    return;
  }
  for (int o = tid; o < nec * L; o += nth) {
    const int l = o % L, ec = o / L;
    double acc[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) acc[i] = 0.0;
    if constexpr (DIM == 3) {
      const double* t = Tin + (int64_t)o * Q;
      const int r = l % Q;
#pragma unroll XU
      for (int a1 = 0; a1 <= P; ++a1) {
        const double x = t[a1 + r < Q ? a1 + r : a1 + r - Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) acc[i] += T.psi1[a1 * Q + i] * x;
      }
    } else {
#pragma unroll XU
      for (int a1 = 0; a1 <= P; ++a1) {
        const double x = Tin[(ec * (P + 1) + a1) * L + l];
#pragma unroll
        for (int i = 0; i < Q; ++i) acc[i] += T.psi1[a1 * Q + i] * x;
      }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) out[ec * S::NQ + i + Q * l] = acc[i];
  }
}

// V^T, first stage: sum over i1 with psi1 (out is T1 on triangles, T2 on tetrahedra)
template <int DIM, int P, bool MF = MfmaEta1<P>::ON>
__device__ __forceinline__ void vt_first(const double* in, double* Tout, const DevTables& T, int nec) {
  using S = Shape<DIM, P>;
  constexpr int Q = S::Q, XU = Unroll<P>::XU;
  constexpr int L = DIM == 2 ? Q : Q * Q;
  const int tid = threadIdx.x, nth = blockDim.x;
  // Tout(ec, a1, l) = sum_i1 psi1[a1][i1] in[ec][i1 + Q l]; on tetrahedra Tout
  // may equal in (the line is read whole before it is written)
  if constexpr (DIM == 3 && MF) {
    constexpr int KS = MfmaEta1<P>::KS;
    const int lane = tid & 63, n = lane % 16, kq = lane / 16;
    double a[KS];
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      const int k = 4 * st + kq;
      a[st] = (n <= P && k < Q) ? T.psi1[n * Q + k] : 0.0;   // A[m = n][k] = psi1[m][k]
    }
    const int ncol = nec * L, tiles = (ncol + 15) / 16;
    for (int t = tid >> 6; t < tiles; t += nth >> 6) {
      const int o = t * 16 + n;
      const bool valid = o < ncol;
      const double* il = in + (int64_t)(valid ? o : 0) * Q;   // in[ec][i1 + Q l] = line o's slots
      const int r = (o % L) % Q;
      mf_d4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < KS; ++st) {
        const int k = 4 * st + kq;
        const double b = (valid && k < Q) ? il[k] : 0.0;
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b, d, 0, 0, 0);
      }
      double* tl = Tout + (int64_t)(valid ? o : 0) * Q;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = 4 * i + kq;
        if (valid && m <= P) tl[m + r < Q ? m + r : m + r - Q] = d[i];
      }
    }
    return;
  }
  for (int o = tid; o < nec * L; o += nth) {
    const int l = o % L, ec = o / L;
    double acc[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) acc[a] = 0.0;
#pragma unroll XU
    for (int i1 = 0; i1 < Q; ++i1) {
      const double x = in[ec * S::NQ + i1 + Q * l];
#pragma unroll
      for (int a = 0; a <= P; ++a) acc[a] += T.psi1[a * Q + i1] * x;
    }
    if constexpr (DIM == 3) {
      double* t = Tout + (int64_t)o * Q;
      const int r = l % Q;
#pragma unroll
      for (int a = 0; a <= P; ++a) t[a + r < Q ? a + r : a + r - Q] = acc[a];
    } else {
#pragma unroll
      for (int a = 0; a <= P; ++a) Tout[(ec * (P + 1) + a) * L + l] = acc[a];
    }
  }
}

// V^T, middle stage of tetrahedra: T1[ec][(a1,a2)][i3] = sum_i2 psi2[a1][a2][i2] T2(ec, a1, i2 + Q i3)
template <int P>
__device__ __forceinline__ void vt_second(const double* T2, double* T1, const DevTables& T, int nec) {
  using S = Shape<3, P>;
  constexpr int Q = S::Q, XL = Q <= 8 ? Q : Unroll<P>::XU;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int o = tid; o < nec * (P + 1) * Q; o += nth) {
    const int i3 = o % Q, a1 = (o / Q) % (P + 1), ec = o / (Q * (P + 1));
    const int pb = pair_index(P, a1, 0);
    double acc[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) acc[a] = 0.0;
    const double* t2 = T2 + ((int64_t)ec * Q * Q + Q * i3) * Q;
#pragma unroll XL
    for (int i2 = 0; i2 < Q; ++i2) {
      const double x = t2[i2 * Q + (a1 + i2 < Q ? a1 + i2 : a1 + i2 - Q)];
#pragma unroll
      for (int a = 0; a <= P; ++a) acc[a] += T.psi2[(a1 * (P + 1) + a) * Q + i2] * x;
    }
#pragma unroll
    for (int a = 0; a <= P; ++a)
      if (a <= P - a1) T1[(ec * S::NPAIR + pb + a) * Q + i3] = acc[a];
  }
}

// V^T, last stage: the nodes of the last direction to its modes
template <int DIM, int P>
__device__ __forceinline__ void vt_last(const double* T1, double* out, const DevTables& T, int nec) {
  using S = Shape<DIM, P>;
  constexpr int Q = S::Q, XU = Unroll<P>::XU;
  constexpr int XL = (DIM == 3 && Q <= 8) ? Q : XU;
  const int tid = threadIdx.x, nth = blockDim.x;
  if constexpr (DIM == 2) {
    // out[ec][(a1,a2)] = sum_i2 psi2[a1][a2][i2] T1[ec][a1][i2]
    for (int o = tid; o < nec * (P + 1); o += nth) {
      const int a1 = o % (P + 1), ec = o / (P + 1);
      const int mb = a1 * (P + 1) - a1 * (a1 - 1) / 2;
      double acc[P + 1];
#pragma unroll
      for (int a = 0; a <= P; ++a) acc[a] = 0.0;
#pragma unroll XU
      for (int i2 = 0; i2 < Q; ++i2) {
        const double x = T1[(ec * (P + 1) + a1) * Q + i2];
#pragma unroll
        for (int a = 0; a <= P; ++a) acc[a] += T.psi2[(a1 * (P + 1) + a) * Q + i2] * x;
      }
#pragma unroll
      for (int a = 0; a <= P; ++a)
        if (a <= P - a1) out[ec * S::NP + mb + a] = acc[a];
    }
  } else {
    // out[ec][(a1,a2,a3)] = sum_i3 psi3[s][a3][i3] T1[ec][(a1,a2)][i3]
    for (int o = tid; o < nec * S::NPAIR; o += nth) {
      const int pr = o % S::NPAIR, ec = o / S::NPAIR;
      int a1, a2;
      decode_pair(P, pr, a1, a2);
      const int s = a1 + a2, mb = tet_mode_base(P, a1, a2);
      double acc[P + 1];
#pragma unroll
      for (int a = 0; a <= P; ++a) acc[a] = 0.0;
#pragma unroll XL
      for (int i3 = 0; i3 < Q; ++i3) {
        const double x = T1[(ec * S::NPAIR + pr) * Q + i3];
#pragma unroll
        for (int a = 0; a <= P; ++a) acc[a] += T.psi3[(s * (P + 1) + a) * Q + i3] * x;
      }
#pragma unroll
      for (int a = 0; a <= P; ++a)
        if (a <= P - s) out[ec * S::NP + mb + a] = acc[a];
    }
  }
}

// u = V u~ at the volume nodes (eq. modal_to_nodal, Sec. 5.2); ends with a barrier
template <int DIM, int P, bool MF = MfmaEta1<P>::ON>
__device__ __forceinline__ void xform_V(const double* uh, double* T1, double* T2, double* out, const DevTables& T,
                                        int nec) {
  v_first<DIM, P>(uh, T1, T, nec);
  __syncthreads();
  if constexpr (DIM == 3) {
    v_second<P>(T1, T2, T, nec);
    __syncthreads();
    v_last<DIM, P, MF>(T2, out, T, nec);
  } else {
    v_last<DIM, P, MF>(T1, out, T, nec);
  }
  __syncthreads();
}

// V^T applied to nodal fields; ends with a barrier
template <int DIM, int P, bool MF = MfmaEta1<P>::ON>
__device__ __forceinline__ void xform_Vt(const double* in, double* T1, double* T2, double* out, const DevTables& T,
                                         int nec) {
  if constexpr (DIM == 3) {
    vt_first<DIM, P, MF>(in, T2, T, nec);
    __syncthreads();
    vt_second<P>(T2, T1, T, nec);
  } else {
    vt_first<DIM, P, MF>(in, T1, T, nec);
  }
  __syncthreads();
  vt_last<DIM, P>(T1, out, T, nec);
  __syncthreads();
}

// V V^T applied to nodal fields (in may equal out).  V^T's last stage and V's
// first contract the same direction (eta2 of triangles, eta3 of tetrahedra)
// with the same table; on each line of that direction their composition is
// the Q x Q matrix psiM[a] = sum_b psi[a][b] psi[a][b]^T (b over the line's
// modes, a = a1 on triangles, a1 + a2 on tetrahedra), applied in place by the
// thread owning the line: one stage and one barrier fewer.  Ends with a barrier.
template <int DIM, int P, bool MF = MfmaEta1<P>::ON>
__device__ __forceinline__ void xform_VVt(const double* in, double* T1, double* T2, double* out, const DevTables& T,
                                          int nec) {
  using S = Shape<DIM, P>;
  constexpr int Q = S::Q;
  constexpr int NL = DIM == 2 ? P + 1 : S::NPAIR;   // lines of the composed direction per (element, variable)
  const int tid = threadIdx.x, nth = blockDim.x;
  if constexpr (DIM == 3) {
    vt_first<DIM, P, MF>(in, T2, T, nec);
    __syncthreads();
    vt_second<P>(T2, T1, T, nec);
  } else {
    vt_first<DIM, P, MF>(in, T1, T, nec);
  }
  __syncthreads();
  for (int o = tid; o < nec * NL; o += nth) {
    const int line = o % NL;
    int a = line;
    if constexpr (DIM == 3) {
      int a1, a2;
      decode_pair(P, line, a1, a2);
      a = a1 + a2;
    }
    double* t = T1 + (int64_t)o * Q;
    double x[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) x[i] = t[i];
    const double* m = T.psiM + a * Q * Q;
    // rows rolled above Q = 7: unrolled, the compiler keeps all Q^2 table
    // values in registers
#pragma unroll Unroll<P>::XU
    for (int i = 0; i < Q; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < Q; ++k) acc += m[i * Q + k] * x[k];
      t[i] = acc;
    }
  }
  __syncthreads();
  if constexpr (DIM == 3) {
    v_second<P>(T1, T2, T, nec);
    __syncthreads();
    v_last<DIM, P, MF>(T2, out, T, nec);
  } else {
    v_last<DIM, P, MF>(T1, out, T, nec);
  }
  __syncthreads();
}

// ------------------------------------------------------------------ transforms inside the nodal array
// V and V^T on tetrahedra with every stage inside one nodal array A
// [nec][NQ]: the modal values in its first nec*NP doubles, the first stage's
// T1 right after them (NP + NPAIR Q <= Q^3 from p = 3 on), the middle stage's
// T2 over all of it.  The middle stage therefore overwrites its own input: it
// reads all of its inputs into registers (at most MAXT tasks per thread,
// MAXT * blockDim >= nec (P+1) Q, which the launch guarantees), waits at a
// barrier, then writes.  Used where the transform scratch would cost a
// workgroup per CU.
template <int P, int MAXT>
__device__ __forceinline__ void v_second_staged(const double* T1, double* T2, const DevTables& T, int nec) {
  using S = Shape<3, P>;
  constexpr int Q = S::Q;
  const int tid = threadIdx.x, nth = blockDim.x, total = nec * (P + 1) * Q;
  double xs[MAXT][P + 1];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    const int o = tid + t * nth;
    if (o < total) {
      const int i3 = o % Q, a1 = (o / Q) % (P + 1), ec = o / (Q * (P + 1));
      const int pb = pair_index(P, a1, 0);
#pragma unroll
      for (int a2 = 0; a2 <= P; ++a2) xs[t][a2] = a2 <= P - a1 ? T1[(ec * S::NPAIR + pb + a2) * Q + i3] : 0.0;
    }
  }
  __syncthreads();
  // one output at a time (a rolled loop; the register-held inputs are
  // indexed by unrolled constants only)
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    const int o = tid + t * nth;
    if (o < total) {
      const int i3 = o % Q, a1 = (o / Q) % (P + 1), ec = o / (Q * (P + 1));
      double* t2 = T2 + ((int64_t)ec * Q * Q + Q * i3) * Q;
      const double* ps = T.psi2 + a1 * (P + 1) * Q;
#pragma unroll 1
      for (int i = 0; i < Q; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int a2 = 0; a2 <= P; ++a2)
          if (a2 <= P - a1) acc += ps[a2 * Q + i] * xs[t][a2];
        t2[i * Q + (a1 + i < Q ? a1 + i : a1 + i - Q)] = acc;
      }
    }
  }
}

template <int P, int MAXT>
__device__ __forceinline__ void vt_second_staged(const double* T2, double* T1, const DevTables& T, int nec) {
  using S = Shape<3, P>;
  constexpr int Q = S::Q;
  const int tid = threadIdx.x, nth = blockDim.x, total = nec * (P + 1) * Q;
  double xs[MAXT][Q];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    const int o = tid + t * nth;
    if (o < total) {
      const int i3 = o % Q, a1 = (o / Q) % (P + 1), ec = o / (Q * (P + 1));
      const double* t2 = T2 + ((int64_t)ec * Q * Q + Q * i3) * Q;
#pragma unroll
      for (int i2 = 0; i2 < Q; ++i2) xs[t][i2] = t2[i2 * Q + (a1 + i2 < Q ? a1 + i2 : a1 + i2 - Q)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    const int o = tid + t * nth;
    if (o < total) {
      const int i3 = o % Q, a1 = (o / Q) % (P + 1), ec = o / (Q * (P + 1));
      const int pb = pair_index(P, a1, 0);
#pragma unroll 1
      for (int a = 0; a <= P - a1; ++a) {
        const double* ps = T.psi2 + (a1 * (P + 1) + a) * Q;
        double acc = 0.0;
#pragma unroll
        for (int i2 = 0; i2 < Q; ++i2) acc += ps[i2] * xs[t][i2];
        T1[(ec * S::NPAIR + pb + a) * Q + i3] = acc;
      }
    }
  }
}

// u = V u~ with A holding u~ in its first nec NP doubles on entry and u on
// exit; ends with a barrier
template <int P, int MAXT>
__device__ __forceinline__ void xform_V_inplace(double* A, const DevTables& T, int nec) {
  using S = Shape<3, P>;
  static_assert(S::NP + S::NPAIR * S::Q <= S::NQ, "first-stage scratch fits after the modal values");
  double* T1 = A + nec * S::NP;
  v_first<3, P>(A, T1, T, nec);
  __syncthreads();
  v_second_staged<P, MAXT>(T1, A, T, nec);
  __syncthreads();
  v_last<3, P>(A, A, T, nec);
  __syncthreads();
}

// V^T of the nodal fields in A, the result in A's first nec NP doubles; ends
// with a barrier
template <int P, int MAXT>
__device__ __forceinline__ void xform_Vt_inplace(double* A, const DevTables& T, int nec) {
  using S = Shape<3, P>;
  double* T1 = A + nec * S::NP;
  vt_first<3, P>(A, A, T, nec);
  __syncthreads();
  vt_second_staged<P, MAXT>(A, T1, T, nec);
  __syncthreads();
  vt_last<3, P>(T1, A, T, nec);
  __syncthreads();
}

// ------------------------------------------------------------------ loads issued ahead of their use
// Values of a block-strided loop over n items (o = tid, tid + nth, ...) for
// this thread's first PF iterations, loaded before the phases that precede
// their use so that their latency overlaps that work.
template <int PF>
struct Ahead {
  double v[PF];
  template <typename Load>
  __device__ __forceinline__ void load(int n, Load ld) {
#pragma unroll
    for (int it = 0; it < PF; ++it) {
      const int o = (int)threadIdx.x + it * (int)blockDim.x;
      v[it] = o < n ? ld(o) : 0.0;
    }
  }
  // body(o, value of o) over the whole loop; iterations past PF load directly
  template <typename Load, typename Body>
  __device__ __forceinline__ void each(int n, Load ld, Body body) const {
#pragma unroll
    for (int it = 0; it < PF; ++it) {
      const int o = (int)threadIdx.x + it * (int)blockDim.x;
      if (o < n) body(o, v[it]);
    }
    for (int o = (int)threadIdx.x + PF * (int)blockDim.x; o < n; o += blockDim.x) body(o, ld(o));
  }
};

// ------------------------------------------------------------------ node data in LDS
// node data layout in LDS: [8][stride] = rho, ln rho, b = rho/p, ln b, p, v1, v2, v3
template <int DIM>
__device__ __forceinline__ Node<DIM> load_node(const double* s, int stride, int k) {
  Node<DIM> n;
  n.rho = s[0 * stride + k];
  n.lnrho = s[1 * stride + k];
  n.b = s[2 * stride + k];
  n.lnb = s[3 * stride + k];
  n.p = s[4 * stride + k];
#pragma unroll
  for (int i = 0; i < DIM; ++i) n.v[i] = s[(5 + i) * stride + k];
  return n;
}
template <int DIM>
__device__ __forceinline__ void store_node(double* s, int stride, int k, const Node<DIM>& n) {
  s[0 * stride + k] = n.rho;
  s[1 * stride + k] = n.lnrho;
  s[2 * stride + k] = n.b;
  s[3 * stride + k] = n.lnb;
  s[4 * stride + k] = n.p;
#pragma unroll
  for (int i = 0; i < DIM; ++i) s[(5 + i) * stride + k] = n.v[i];
}

// ------------------------------------------------------------------ facet extrapolation and its transpose
// Facet values (R w)[ec][facet*NQF + node] of nodal fields w [nec][NQ] (eqs.
// r_2d, r_3d), passed to store(o, value) with o = ec*NFQ + facet*NQF + node.
// Triangles: facet 1 interpolates along eta2 to -1, facets 2 and 3 along eta1
// to +1 / -1.  Tetrahedra: faces 1-3 likewise along eta2 / eta1; face 4 first
// contracts eta3 -> -1 into scr [nec][Q*Q], then maps the eta2 line to the
// face's own Legendre nodes (I42).  No barrier at the end.
template <int DIM, int P, typename Store>
__device__ __forceinline__ void facet_values(const double* w_all, double* scr, const DevTables& T, int nec,
                                             Store store) {
  using S = Shape<DIM, P>;
  constexpr int Q = S::Q, NQ = S::NQ, NQF = S::NQF, NFQ = S::NFQ;
  const int tid = threadIdx.x, nth = blockDim.x;
  if constexpr (DIM == 3) {
    for (int o = tid; o < nec * Q * Q; o += nth) {
      const int a1 = o % Q, k2 = (o / Q) % Q, ec = o / (Q * Q);
      double acc = 0.0;
#pragma unroll
      for (int k3 = 0; k3 < Q; ++k3) acc += T.gjm1[k3] * w_all[ec * NQ + a1 + Q * k2 + Q * Q * k3];
      scr[o] = acc;
    }
    __syncthreads();
  }
  for (int o = tid; o < nec * NFQ; o += nth) {
    const int jj = o % NFQ, ec = o / NFQ, f = jj / NQF, j = jj % NQF;
    const double* w = w_all + ec * NQ;
    double acc = 0.0;
    if constexpr (DIM == 2) {
      if (f == 0) {
#pragma unroll
        for (int k = 0; k < Q; ++k) acc += T.lgm1[k] * w[j + Q * k];
      } else {
        const double* l = (f == 1) ? T.lgp1 : T.lgm1;
#pragma unroll
        for (int k = 0; k < Q; ++k) acc += l[k] * w[k + Q * j];
      }
    } else {
      const int a1 = j % Q, a2 = j / Q;
      if (f == 0) {
#pragma unroll
        for (int k = 0; k < Q; ++k) acc += T.lgm1[k] * w[a1 + Q * k + Q * Q * a2];
      } else if (f == 3) {
#pragma unroll
        for (int k = 0; k < Q; ++k) acc += T.I42[a2 * Q + k] * scr[ec * Q * Q + a1 + Q * k];
      } else {
        const double* l = (f == 1) ? T.lgp1 : T.lgm1;
#pragma unroll
        for (int k = 0; k < Q; ++k) acc += l[k] * w[k + Q * a1 + Q * Q * a2];
      }
    }
    store(o, acc);
  }
}

// Transpose of facet_values: (R^T s)[ec][k] for facet fields s [nec][NFQ],
// passed to apply(o, value) with o = ec*NQ + k.  Tet face 4 is first
// contracted back over its eta2 index into scr [nec][Q*Q].  No barrier at the end.
template <int DIM, int P, typename Apply>
__device__ __forceinline__ void facet_lift(const double* s_all, double* scr, const DevTables& T, int nec,
                                           Apply apply) {
  using S = Shape<DIM, P>;
  constexpr int Q = S::Q, NQ = S::NQ, NQF = S::NQF, NFQ = S::NFQ;
  const int tid = threadIdx.x, nth = blockDim.x;
  if constexpr (DIM == 3) {
    for (int o = tid; o < nec * Q * Q; o += nth) {
      const int b1 = o % Q, b2 = (o / Q) % Q, ec = o / (Q * Q);
      double acc4 = 0.0;
#pragma unroll
      for (int a2 = 0; a2 < Q; ++a2) acc4 += T.I42[a2 * Q + b2] * s_all[ec * NFQ + 3 * NQF + b1 + Q * a2];
      scr[o] = acc4;
    }
    __syncthreads();
  }
  for (int o = tid; o < nec * NQ; o += nth) {
    const int k = o % NQ, ec = o / NQ;
    const double* s = s_all + ec * NFQ;
    double d;
    if constexpr (DIM == 2) {
      const int b1 = k % Q, b2 = k / Q;
      d = T.lgm1[b2] * s[0 * NQF + b1] + T.lgp1[b1] * s[1 * NQF + b2] + T.lgm1[b1] * s[2 * NQF + b2];
    } else {
      const int b1 = k % Q, b2 = (k / Q) % Q, b3 = k / (Q * Q);
      d = T.lgm1[b2] * s[0 * NQF + b1 + Q * b3] + T.lgp1[b1] * s[1 * NQF + b2 + Q * b3] +
          T.lgm1[b1] * s[2 * NQF + b2 + Q * b3] + T.gjm1[b3] * scr[ec * Q * Q + b1 + Q * b2];
    }
    apply(o, d);
  }
}

}  // namespace esd
