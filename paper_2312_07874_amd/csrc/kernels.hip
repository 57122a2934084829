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

#include "plan.hpp"

namespace esd {

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
  static constexpr int SCR = (T1 + T2 > 8 * NQ) ? (T1 + T2) : 8 * NQ;   // per element
};

template <int DIM, int P>
struct Launch;  // block size and elements per block
template <int P>
struct Launch<3, P> {
  // one element per workgroup; small workgroups keep several elements in
  // flight per CU, which hides the latency of the barrier-separated phases
  static constexpr int EPB = 1;
  static constexpr int BS = P <= 3 ? 64 : (P == 4 ? 128 : (P <= 6 ? 192 : 256));
};
template <int P>
struct Launch<2, P> {
  static constexpr int EPB = (P <= 4) ? 12 : ((P <= 7) ? 8 : 6);
  static constexpr int NQ = (P + 1) * (P + 1);
  static constexpr int BS = ((EPB * NQ + 63) / 64) * 64;
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

// ------------------------------------------------------------------ sum-factorised PKD transforms
// in/out arrays are [nel*NC][...] contiguous per (element, variable); all
// threads of the block participate; each call ends with a barrier.  Every
// thread produces a whole line of outputs from one set of LDS loads
// (register blocking along the contracted direction).
template <int DIM, int P>
__device__ void xform_V(const double* uh, double* T1, double* T2, double* out, const DevTables& T, int nec) {
  using S = Shape<DIM, P>;
  constexpr int Q = S::Q;
  constexpr int XU = Q <= 7 ? Q : 1;   // unroll the contraction while its table fits scalar registers
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
    __syncthreads();
    // out[ec][i1 + Q i2] = sum_a1 psi1[a1][i1] T1[ec][a1][i2]
    for (int o = tid; o < nec * Q; o += nth) {
      const int i2 = o % Q, ec = o / Q;
      double acc[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) acc[i] = 0.0;
#pragma unroll XU
      for (int a1 = 0; a1 <= P; ++a1) {
        const double x = T1[(ec * (P + 1) + a1) * Q + i2];
#pragma unroll
        for (int i = 0; i < Q; ++i) acc[i] += T.psi1[a1 * Q + i] * x;
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) out[ec * S::NQ + i + Q * i2] = acc[i];
    }
    __syncthreads();
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
#pragma unroll XU
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
    __syncthreads();
    // T2[ec][a1][i2 + Q i3] = sum_a2 psi2[a1][a2][i2] T1[ec][(a1,a2)][i3]
    for (int o = tid; o < nec * (P + 1) * Q; o += nth) {
      const int i3 = o % Q, a1 = (o / Q) % (P + 1), ec = o / (Q * (P + 1));
      const int pb = pair_index(P, a1, 0);
      double acc[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) acc[i] = 0.0;
#pragma unroll XU
      for (int a2 = 0; a2 <= P; ++a2) {
        if (a2 <= P - a1) {
          const double x = T1[(ec * S::NPAIR + pb + a2) * Q + i3];
          const double* ps = T.psi2 + (a1 * (P + 1) + a2) * Q;
#pragma unroll
          for (int i = 0; i < Q; ++i) acc[i] += ps[i] * x;
        }
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) T2[(ec * (P + 1) + a1) * Q * Q + i + Q * i3] = acc[i];
    }
    __syncthreads();
    // out[ec][i1 + Q i2 + Q^2 i3] = sum_a1 psi1[a1][i1] T2[ec][a1][i2 + Q i3]
    for (int o = tid; o < nec * Q * Q; o += nth) {
      const int i23 = o % (Q * Q), ec = o / (Q * Q);
      double acc[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) acc[i] = 0.0;
#pragma unroll XU
      for (int a1 = 0; a1 <= P; ++a1) {
        const double x = T2[(ec * (P + 1) + a1) * Q * Q + i23];
#pragma unroll
        for (int i = 0; i < Q; ++i) acc[i] += T.psi1[a1 * Q + i] * x;
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) out[ec * S::NQ + i + Q * i23] = acc[i];
    }
    __syncthreads();
  }
}

template <int DIM, int P>
__device__ void xform_Vt(const double* in, double* T1, double* T2, double* out, const DevTables& T, int nec) {
  using S = Shape<DIM, P>;
  constexpr int Q = S::Q;
  constexpr int XU = Q <= 7 ? Q : 1;   // unroll the contraction while its table fits scalar registers
  const int tid = threadIdx.x, nth = blockDim.x;
  if constexpr (DIM == 2) {
    // T1[ec][a1][i2] = sum_i1 psi1[a1][i1] in[ec][i1 + Q i2]
    for (int o = tid; o < nec * Q; o += nth) {
      const int i2 = o % Q, ec = o / Q;
      double acc[P + 1];
#pragma unroll
      for (int a = 0; a <= P; ++a) acc[a] = 0.0;
#pragma unroll XU
      for (int i1 = 0; i1 < Q; ++i1) {
        const double x = in[ec * S::NQ + i1 + Q * i2];
#pragma unroll
        for (int a = 0; a <= P; ++a) acc[a] += T.psi1[a * Q + i1] * x;
      }
#pragma unroll
      for (int a = 0; a <= P; ++a) T1[(ec * (P + 1) + a) * Q + i2] = acc[a];
    }
    __syncthreads();
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
    __syncthreads();
  } else {
    // T2[ec][a1][i2 + Q i3] = sum_i1 psi1[a1][i1] in[ec][i1 + Q i2 + Q^2 i3]
    for (int o = tid; o < nec * Q * Q; o += nth) {
      const int i23 = o % (Q * Q), ec = o / (Q * Q);
      double acc[P + 1];
#pragma unroll
      for (int a = 0; a <= P; ++a) acc[a] = 0.0;
#pragma unroll XU
      for (int i1 = 0; i1 < Q; ++i1) {
        const double x = in[ec * S::NQ + i1 + Q * i23];
#pragma unroll
        for (int a = 0; a <= P; ++a) acc[a] += T.psi1[a * Q + i1] * x;
      }
#pragma unroll
      for (int a = 0; a <= P; ++a) T2[(ec * (P + 1) + a) * Q * Q + i23] = acc[a];
    }
    __syncthreads();
    // T1[ec][(a1,a2)][i3] = sum_i2 psi2[a1][a2][i2] T2[ec][a1][i2 + Q i3]
    for (int o = tid; o < nec * (P + 1) * Q; o += nth) {
      const int i3 = o % Q, a1 = (o / Q) % (P + 1), ec = o / (Q * (P + 1));
      const int pb = pair_index(P, a1, 0);
      double acc[P + 1];
#pragma unroll
      for (int a = 0; a <= P; ++a) acc[a] = 0.0;
#pragma unroll XU
      for (int i2 = 0; i2 < Q; ++i2) {
        const double x = T2[(ec * (P + 1) + a1) * Q * Q + i2 + Q * i3];
#pragma unroll
        for (int a = 0; a <= P; ++a) acc[a] += T.psi2[(a1 * (P + 1) + a) * Q + i2] * x;
      }
#pragma unroll
      for (int a = 0; a <= P; ++a)
        if (a <= P - a1) T1[(ec * S::NPAIR + pb + a) * Q + i3] = acc[a];
    }
    __syncthreads();
    // out[ec][(a1,a2,a3)] = sum_i3 psi3[s][a3][i3] T1[ec][(a1,a2)][i3]
    for (int o = tid; o < nec * S::NPAIR; o += nth) {
      const int pr = o % S::NPAIR, ec = o / S::NPAIR;
      int a1, a2;
      decode_pair(P, pr, a1, a2);
      const int s = a1 + a2, mb = tet_mode_base(P, a1, a2);
      double acc[P + 1];
#pragma unroll
      for (int a = 0; a <= P; ++a) acc[a] = 0.0;
#pragma unroll XU
      for (int i3 = 0; i3 < Q; ++i3) {
        const double x = T1[(ec * S::NPAIR + pr) * Q + i3];
#pragma unroll
        for (int a = 0; a <= P; ++a) acc[a] += T.psi3[(s * (P + 1) + a) * Q + i3] * x;
      }
#pragma unroll
      for (int a = 0; a <= P; ++a)
        if (a <= P - s) out[ec * S::NP + mb + a] = acc[a];
    }
    __syncthreads();
  }
}

// 1/x: hardware reciprocal estimate refined by two Newton-Raphson steps
// (each squares the relative error), correctly rounded to within an ulp
__device__ __forceinline__ double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

// ------------------------------------------------------------------ physics
template <int DIM>
struct Node {
  double rho, lnrho, b, lnb, p, v[DIM];
};

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

// entropy-projected conservative state U(w) (inverse of W = dS/dU, Sec. 7.1)
template <int DIM>
__device__ __forceinline__ bool from_entropy(const double* w, const Scheme& S, Node<DIM>& n) {
  const double b = -w[DIM + 1];
  const double ib = frcp(b);
  double v2 = 0.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    n.v[i] = w[1 + i] * ib;
    v2 += n.v[i] * n.v[i];
  }
  const double s = S.gamma - (S.gamma - 1.0) * (w[0] + 0.5 * b * v2);
  n.b = b;
  n.lnb = log(b);
  n.lnrho = -(s + n.lnb) * S.gm1_inv;
  n.rho = exp(n.lnrho);
  n.p = n.rho * ib;
  return (b > 0.0) && isfinite(n.rho) && isfinite(n.p) && (n.rho > 0.0);
}

constexpr double LOG_SERIES_THRESHOLD = 1.0e-4;

// The logarithmic mean (a+ - a-)/(ln a+ - ln a-) and the reciprocal of the
// logarithmic mean, from precomputed logs.  With f = (a+ - a-)/(a+ + a-) and
// ln(a+/a-) = 2 atanh f, nearly equal arguments (f^2 < 1e-4) use the series
//   {a}_ln     = (a- + a+)/2 * f/atanh f,  f/atanh f = 1 - u/3 - 4u^2/45 - 44u^3/945 + O(u^4)
//   1/{a}_ln   = 2 (1 + u/3 + u^2/5 + u^3/7) / (a- + a+) + O(u^4),   u = f^2,
// whose truncation is below 3e-18 relative.  inv_s = 1/(a- + a+) is passed in.
__device__ __forceinline__ double log_mean(double a, double b, double la, double lb, double inv_s) {
  const double d = b - a;
  const double f = d * inv_s, u = f * f;
  if (u < LOG_SERIES_THRESHOLD)
    return 0.5 * (a + b) * (1.0 - u * (1.0 / 3.0 + u * (4.0 / 45.0 + u * (44.0 / 945.0))));
  return d / (lb - la);
}
__device__ __forceinline__ double inv_log_mean(double a, double b, double la, double lb, double inv_s) {
  const double d = b - a;
  const double f = d * inv_s, u = f * f;
  if (u < LOG_SERIES_THRESHOLD) return 2.0 * (1.0 + u * (1.0 / 3.0 + u * (1.0 / 5.0 + u * (1.0 / 7.0)))) * inv_s;
  return (lb - la) / d;
}

// directional entropy-conservative flux f#(A, B, n) = sum_m n_m f#_m(A, B)
template <int DIM, int FLUX>
__device__ __forceinline__ void ec_flux(const Node<DIM>& A, const Node<DIM>& B, const double* n, const Scheme& S,
                                        double* F) {
  // one reciprocal serves both means: 1/(sr sb) -> 1/sr = sb/(sr sb), 1/sb = sr/(sr sb)
  const double sr = A.rho + B.rho, sb = A.b + B.b;
  const double rr = frcp(sr * sb);
  const double rho_ln = log_mean(A.rho, B.rho, A.lnrho, B.lnrho, sb * rr);
  const double ib_ln = inv_log_mean(A.b, B.b, A.lnb, B.lnb, sr * rr);   // 1 / {rho/p}_ln
  double vavg[DIM];
  double vn = 0.0, vab = 0.0, van = 0.0, vbn = 0.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    vavg[i] = 0.5 * (A.v[i] + B.v[i]);
    vn += vavg[i] * n[i];
    vab += A.v[i] * B.v[i];
    van += A.v[i] * n[i];
    vbn += B.v[i] * n[i];
  }
  const double frho = rho_ln * vn;
  F[0] = frho;
  if constexpr (FLUX == FLUX_RANOCHA) {
    const double pavg = 0.5 * (A.p + B.p);
#pragma unroll
    for (int i = 0; i < DIM; ++i) F[1 + i] = frho * vavg[i] + pavg * n[i];
    F[DIM + 1] = frho * (0.5 * vab + ib_ln * S.gm1_inv) + 0.5 * (A.p * vbn + B.p * van);
  } else {
    const double phat = sr * sr * rr;                        // {rho} / (2 {beta}) = sr/sb, beta = b/2
#pragma unroll
    for (int i = 0; i < DIM; ++i) F[1 + i] = frho * vavg[i] + phat * n[i];
    F[DIM + 1] = frho * (0.5 * vab + ib_ln * S.gm1_inv) + phat * vn;
  }
}

// ------------------------------------------------------------------ K1: entropy projection
template <int DIM, int P, bool PROJECT_ONLY>
__global__ void __launch_bounds__((Launch<DIM, P>::BS))
k_entropy_projection(const double* __restrict__ u, double* __restrict__ wt, double* __restrict__ wf,
                     const double* __restrict__ gvol, DevTables T, Scheme S, int64_t ne, int* flag) {
  using Sh = Shape<DIM, P>;
  constexpr int EPB = Launch<DIM, P>::EPB;
  constexpr int Q = Sh::Q, NC = Sh::NC, NQ = Sh::NQ, NP = Sh::NP, NQF = Sh::NQF, NFQ = Sh::NFQ, NGV = Sh::NGV;
  __shared__ double sM[EPB * NC * NP];
  __shared__ double sA[EPB * NC * NQ];
  __shared__ double sS[EPB * Sh::SCR];
  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const int nel = (int)((ne - e0) < EPB ? (ne - e0) : EPB);
  const int nec = nel * NC;
  const int tid = threadIdx.x, nth = blockDim.x;
  double* T1 = sS;
  double* T2 = sS + EPB * Sh::T1;
  if constexpr (PROJECT_ONLY) {
    // u holds nodal values [e][node][var]; b = w J u
    for (int o = tid; o < nel * NQ * NC; o += nth) {
      const int c = o % NC, k = (o / NC) % NQ, el = o / (NC * NQ);
      const double wJ = gvol[((e0 + el) * NGV + NGV - 2) * NQ + k];
      sA[(el * NC + c) * NQ + k] = wJ * u[(e0 * NQ) * NC + o];
    }
    __syncthreads();
  } else {
    for (int o = tid; o < nec * NP; o += nth) sM[o] = u[e0 * NC * NP + o];
    __syncthreads();
    xform_V<DIM, P>(sM, T1, T2, sA, T, nec);
    // entropy variables times w J at every volume node
    for (int o = tid; o < nel * NQ; o += nth) {
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
      if (!(rho > 0.0) || !(p > 0.0) || !isfinite(rho) || !isfinite(p)) atomicOr(flag, 1);
      const double s = log(p) - S.gamma * log(rho);
      const double wJ = gvol[((e0 + el) * NGV + NGV - 2) * NQ + k];
      a[k] = wJ * ((S.gamma - s) * S.gm1_inv - 0.5 * rho * v2 / p);
#pragma unroll
      for (int i = 0; i < DIM; ++i) a[(1 + i) * NQ + k] = wJ * (rho * v[i] / p);
      a[(DIM + 1) * NQ + k] = wJ * (-rho / p);
    }
    __syncthreads();
  }
  // weight-adjusted projection: V^T (w/J) V V^T (w J W)
  xform_Vt<DIM, P>(sA, T1, T2, sM, T, nec);
  xform_V<DIM, P>(sM, T1, T2, sA, T, nec);
  for (int o = tid; o < nec * NQ; o += nth) {
    const int k = o % NQ, el = o / (NC * NQ);
    sA[o] *= gvol[((e0 + el) * NGV + NGV - 1) * NQ + k];
  }
  __syncthreads();
  xform_Vt<DIM, P>(sA, T1, T2, sM, T, nec);
  for (int o = tid; o < nec * NP; o += nth) wt[e0 * NC * NP + o] = sM[o];
  if constexpr (PROJECT_ONLY) return;
  else {
    // facet values of the projected entropy variables, w^z = R^z V w~
    xform_V<DIM, P>(sM, T1, T2, sA, T, nec);
    if constexpr (DIM == 3) {
      // face 4: contract eta3 -> -1 first
      for (int o = tid; o < nec * Q * Q; o += nth) {
        const int a1 = o % Q, k2 = (o / Q) % Q, ec = o / (Q * Q);
        double acc = 0.0;
#pragma unroll
        for (int k3 = 0; k3 < Q; ++k3) acc += T.gjm1[k3] * sA[ec * NQ + a1 + Q * k2 + Q * Q * k3];
        sS[o] = acc;
      }
      __syncthreads();
    }
    for (int o = tid; o < nec * NFQ; o += nth) {
      const int jj = o % NFQ, ec = o / NFQ, f = jj / NQF, j = jj % NQF;
      const double* w = sA + ec * NQ;
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
          for (int k = 0; k < Q; ++k) acc += T.I42[a2 * Q + k] * sS[ec * Q * Q + a1 + Q * k];
        } else {
          const double* l = (f == 1) ? T.lgp1 : T.lgm1;
#pragma unroll
          for (int k = 0; k < Q; ++k) acc += l[k] * w[k + Q * a1 + Q * Q * a2];
        }
      }
      wf[e0 * NC * NFQ + o] = acc;
    }
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
    ec_flux<DIM, FLUX>(Na, Nb, n, S, F);
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

// One facet-correction pair (eq. facet_correction): C = coef f#(u_i, u^z_j, (gn_i + nJ_j)/2);
// r_i -= C (registers), t_j += C (LDS atomics).
template <int DIM, int P, int FLUX>
__device__ __forceinline__ void facet_task(const Node<DIM>& Vi, const double* gn_i, const double* sF, double* sT,
                                           const double* __restrict__ gf, int j, double coef, const Scheme& S,
                                           double* racc) {
  constexpr int NC = DIM + 2, NFQ = Shape<DIM, P>::NFQ;
  const Node<DIM> Fj = load_node<DIM>(sF, NFQ, j);
  double n[DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i) n[i] = 0.5 * (gn_i[i] + gf[i * NFQ + j]);
  double F[NC];
  ec_flux<DIM, FLUX>(Vi, Fj, n, S, F);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double C = coef * F[c];
    racc[c] -= C;
    atomicAdd(&sT[c * NFQ + j], C);
  }
}

// ------------------------------------------------------------------ K2: right-hand side
template <int DIM, int P, int FLUX>
__global__ void __launch_bounds__((Launch<DIM, P>::BS))
k_rhs(const double* __restrict__ wt, const double* __restrict__ wfb, double* __restrict__ dudt,
      const double* __restrict__ gvol, const double* __restrict__ gfac, const int32_t* __restrict__ conn,
      DevTables T, Scheme S, int64_t ne, int* flag) {
  using Sh = Shape<DIM, P>;
  constexpr int EPB = Launch<DIM, P>::EPB;
  constexpr int Q = Sh::Q, NC = Sh::NC, NQ = Sh::NQ, NP = Sh::NP, NQF = Sh::NQF, NFQ = Sh::NFQ, NGV = Sh::NGV;
  constexpr int LPF = Sh::LPF;
  __shared__ double sM[EPB * NC * NP];
  __shared__ double sN[EPB * Sh::SCR];      // node data [el][8][NQ]; transform scratch
  __shared__ double sR[EPB * NC * NQ];      // w at nodes, then r
  __shared__ double sF[EPB * 8 * NFQ];      // own facet node data; later R^T scratch
  __shared__ double sT[EPB * NC * NFQ];     // C^T 1, then s = B J_f f* - C^T 1
  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const int nel = (int)((ne - e0) < EPB ? (ne - e0) : EPB);
  const int nec = nel * NC;
  const int tid = threadIdx.x, nth = blockDim.x;
  double* T1 = sN;
  double* T2 = sN + EPB * Sh::T1;

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
    bad |= !from_entropy<DIM>(w, S, nd);
    store_node<DIM>(sN + el * Sh::SCR, NQ, k, nd);
  }
  for (int o = tid; o < nel * NFQ; o += nth) {
    const int j = o % NFQ, el = o / NFQ;
    double w[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) w[c] = wfb[((e0 + el) * NC + c) * NFQ + j];
    Node<DIM> nd;
    bad |= !from_entropy<DIM>(w, S, nd);
    store_node<DIM>(sF + el * 8 * NFQ, NFQ, j, nd);
  }
  for (int o = tid; o < nec * NFQ; o += nth) sT[o] = 0.0;
  if (bad) atomicOr(flag, 1);
  __syncthreads();

  // ---- volume flux differencing: one task per (line family, line, node a);
  //      task a evaluates the pairs (a, a+k mod Q), k = 1..(Q-1)/2 (and k = Q/2
  //      for a < Q/2 when Q is even), so every unordered pair of a line is
  //      evaluated once and every task does the same work.  r_a accumulates in
  //      registers, r_b through LDS atomics.
  for (int o = tid; o < nec * NQ; o += nth) sR[o] = 0.0;
  for (int o = tid; o < nec * NFQ; o += nth) sT[o] = 0.0;
  __syncthreads();
  {
    constexpr int TPE = DIM * NQ;           // volume tasks per element
    for (int task = tid; task < nel * TPE; task += nth) {
      const int el = task / TPE, lt = task % TPE;
      const int fam = lt / NQ, rem = lt % NQ, L = rem / Q, a = rem % Q;
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
    const double* sFe = sF + el * 8 * NFQ;
    double* sTe = sT + el * NC * NFQ;
    const double* g = gvol + (e0 + el) * NGV * NQ;
    const double* gf = gfac + (e0 + el) * (DIM + 1) * NFQ;
    double racc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) racc[c] = 0.0;
    int i;
    if constexpr (DIM == 2) {
      const int b2 = t % Q, b1 = t / Q;     // b2 fastest: neighbouring lanes hit different facet nodes
      i = b1 + Q * b2;
      const Node<DIM> Vi = load_node<DIM>(sNe, NQ, i);
      const double w1 = T.wl[b1], w2 = T.wl[b2];
      double gA[2], gB[2], gC[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const double g1 = g[(0 + m) * NQ + i] / w2;
        const double g2 = 2.0 * g[(2 + m) * NQ + i] / w2;
        gA[m] = (g1 + g2) * 0.70710678118654752440;     // facet 2: G^T nhat, nhat = (1,1)/sqrt 2
        gB[m] = -g1;                                     // facet 3: nhat = (-1, 0)
        gC[m] = -2.0 * g[(4 + m) * NQ + i] / w1;         // facet 1: nhat = (0, -1)
      }
      facet_task<DIM, P, FLUX>(Vi, gA, sFe, sTe, gf, 1 * NQF + b2, T.lgp1[b1] * T.wf[1 * NQF + b2], S, racc);
      facet_task<DIM, P, FLUX>(Vi, gB, sFe, sTe, gf, 2 * NQF + b2, T.lgm1[b1] * T.wf[2 * NQF + b2], S, racc);
      facet_task<DIM, P, FLUX>(Vi, gC, sFe, sTe, gf, 0 * NQF + b1, T.lgm1[b2] * T.wf[0 * NQF + b1], S, racc);
    } else {
      const int b3 = t % Q, b2 = (t / Q) % Q, b1 = t / (Q * Q);
      i = b1 + Q * (b2 + Q * b3);
      const Node<DIM> Vi = load_node<DIM>(sNe, NQ, i);
      const double inv23 = 1.0 / (T.wl[b2] * T.wj[b3]);
      const double inv13 = 1.0 / (T.wl[b1] * T.wj[b3]);
      const double inv12 = 1.0 / (T.wl[b1] * T.wl[b2] * (1.0 - T.xl[b2]));
      double gA[3], gB[3], gC[3], gD[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const double g1 = 2.0 * g[(0 + m) * NQ + i] * inv23;
        const double g23 = 4.0 * g[(3 + m) * NQ + i] * inv23;
        gA[m] = (g1 + g23) * 0.57735026918962576451;    // facet 2: nhat = (1,1,1)/sqrt 3
        gB[m] = -g1;                                     // facet 3: nhat = (-1,0,0)
        gC[m] = -4.0 * g[(6 + m) * NQ + i] * inv13;      // facet 1: nhat = (0,-1,0)
        gD[m] = -8.0 * g[(12 + m) * NQ + i] * inv12;     // facet 4: nhat = (0,0,-1)
      }
      const int j23 = b2 + Q * b3;
      facet_task<DIM, P, FLUX>(Vi, gA, sFe, sTe, gf, 1 * NQF + j23, T.lgp1[b1] * T.wf[1 * NQF + j23], S, racc);
      facet_task<DIM, P, FLUX>(Vi, gB, sFe, sTe, gf, 2 * NQF + j23, T.lgm1[b1] * T.wf[2 * NQF + j23], S, racc);
      const int j13 = b1 + Q * b3;
      facet_task<DIM, P, FLUX>(Vi, gC, sFe, sTe, gf, 0 * NQF + j13, T.lgm1[b2] * T.wf[0 * NQF + j13], S, racc);
      const double cz = T.gjm1[b3];
#pragma unroll
      for (int m = 0; m < Q; ++m) {
        int a2 = m + b2 + b3;                 // rotated so that neighbouring lanes hit different facet nodes
        a2 = a2 % Q;
        const int j = 3 * NQF + b1 + Q * a2;
        facet_task<DIM, P, FLUX>(Vi, gD, sFe, sTe, gf, j, cz * T.I42[a2 * Q + b2] * T.wf[j], S, racc);
      }
    }
    double* r = sR + el * NC * NQ;
#pragma unroll
    for (int c = 0; c < NC; ++c) r[c * NQ + i] += racc[c];
  }
  __syncthreads();

  // ---- interface flux and s = B J_f f* - C^T 1
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
    bad |= !from_entropy<DIM>(w, S, Up);
    double nJ[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) nJ[i] = gfac[(e * (DIM + 1) + i) * NFQ + j];
    double F[NC];
    ec_flux<DIM, FLUX>(Um, Up, nJ, S, F);
    if (S.dissipation) {
      const double Jf = gfac[(e * (DIM + 1) + DIM) * NFQ + j];
      double vmn = 0.0, vpn = 0.0, vm2 = 0.0, vp2 = 0.0;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        vmn += Um.v[i] * nJ[i];
        vpn += Up.v[i] * nJ[i];
        vm2 += Um.v[i] * Um.v[i];
        vp2 += Up.v[i] * Up.v[i];
      }
      const double am = fabs(vmn), ap = fabs(vpn);
      const double cm = sqrt(S.gamma * Um.p / Um.rho), cp = sqrt(S.gamma * Up.p / Up.rho);
      const double lam = (am >= ap ? am : ap) + Jf * (cm >= cp ? cm : cp);   // J_f * lambda
      const double h = 0.5 * lam;
      F[0] -= h * (Up.rho - Um.rho);
#pragma unroll
      for (int i = 0; i < DIM; ++i) F[1 + i] -= h * (Up.rho * Up.v[i] - Um.rho * Um.v[i]);
      const double Em = Um.p * S.gm1_inv + 0.5 * Um.rho * vm2;
      const double Ep = Up.p * S.gm1_inv + 0.5 * Up.rho * vp2;
      F[DIM + 1] -= h * (Ep - Em);
    }
    const double wj = T.wf[j];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double* t = sT + (le * NC + c) * NFQ + j;
      *t = wj * F[c] - *t;
    }
  }
  if (bad) atomicOr(flag, 1);
  __syncthreads();

  // ---- r -= R^T s
  if constexpr (DIM == 3) {
    for (int o = tid; o < nec * Q * Q; o += nth) {
      const int b1 = o % Q, b2 = (o / Q) % Q, ec = o / (Q * Q);
      double acc4 = 0.0;
#pragma unroll
      for (int a2 = 0; a2 < Q; ++a2) acc4 += T.I42[a2 * Q + b2] * sT[ec * NFQ + 3 * NQF + b1 + Q * a2];
      sF[o] = acc4;
    }
    __syncthreads();
  }
  for (int o = tid; o < nec * NQ; o += nth) {
    const int k = o % NQ, ec = o / NQ;
    const double* s = sT + ec * NFQ;
    double d;
    if constexpr (DIM == 2) {
      const int b1 = k % Q, b2 = k / Q;
      d = T.lgm1[b2] * s[0 * NQF + b1] + T.lgp1[b1] * s[1 * NQF + b2] + T.lgm1[b1] * s[2 * NQF + b2];
    } else {
      const int b1 = k % Q, b2 = (k / Q) % Q, b3 = k / (Q * Q);
      d = T.lgm1[b2] * s[0 * NQF + b1 + Q * b3] + T.lgp1[b1] * s[1 * NQF + b2 + Q * b3] +
          T.lgm1[b1] * s[2 * NQF + b2 + Q * b3] + T.gjm1[b3] * sF[ec * Q * Q + b1 + Q * b2];
    }
    sR[o] -= d;
  }
  __syncthreads();

  // ---- du~/dt = V^T (w/J) V V^T r
  xform_Vt<DIM, P>(sR, T1, T2, sM, T, nec);
  xform_V<DIM, P>(sM, T1, T2, sR, T, nec);
  for (int o = tid; o < nec * NQ; o += nth) {
    const int k = o % NQ, le = o / (NC * NQ);
    sR[o] *= gvol[((e0 + le) * NGV + NGV - 1) * NQ + k];
  }
  __syncthreads();
  xform_Vt<DIM, P>(sR, T1, T2, sM, T, nec);
  for (int o = tid; o < nec * NP; o += nth) dudt[e0 * NC * NP + o] = sM[o];
}

// ------------------------------------------------------------------ RK4 helpers
__global__ void k_rk_stage(double* __restrict__ acc, double* __restrict__ U, const double* __restrict__ u,
                           const double* __restrict__ k, double ca, double cu, int first, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ki = k[i], ui = u[i];
    acc[i] = (first ? ui : acc[i]) + ca * ki;
    if (U) U[i] = ui + cu * ki;
  }
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, const double* __restrict__ z,
                       int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i] + a * z[i];
}

// ------------------------------------------------------------------ dispatch
static hipEvent_t timing_event(const esd_plan* pl, hipStream_t s) {
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
static int run_residual(const esd_plan* pl, const double* u, double* dudt, Workspace ws, hipStream_t s) {
  using L = Launch<DIM, P>;
  const int64_t nb = (pl->ne + L::EPB - 1) / L::EPB;
  if (pl->timing) timing_event(pl, s);
  hipLaunchKernelGGL((k_entropy_projection<DIM, P, false>), dim3(nb), dim3(L::BS), 0, s, u, ws.wt, ws.wf,
                     pl->d_gvol, pl->tab, pl->scheme, pl->ne, pl->d_flag);
  if (pl->timing) timing_event(pl, s);
  if (pl->scheme.ecflux == FLUX_RANOCHA)
    hipLaunchKernelGGL((k_rhs<DIM, P, FLUX_RANOCHA>), dim3(nb), dim3(L::BS), 0, s, ws.wt, ws.wf, dudt, pl->d_gvol,
                       pl->d_gfac, pl->d_conn, pl->tab, pl->scheme, pl->ne, pl->d_flag);
  else
    hipLaunchKernelGGL((k_rhs<DIM, P, FLUX_CHANDRASHEKAR>), dim3(nb), dim3(L::BS), 0, s, ws.wt, ws.wf, dudt,
                       pl->d_gvol, pl->d_gfac, pl->d_conn, pl->tab, pl->scheme, pl->ne, pl->d_flag);
  if (pl->timing) timing_event(pl, s);
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

#define ESD_TRI_DEGREES(X) X(2, 1) X(2, 2) X(2, 3) X(2, 4) X(2, 5) X(2, 6) X(2, 7) X(2, 8) X(2, 9) X(2, 10)
#define ESD_TET_DEGREES(X) X(3, 1) X(3, 2) X(3, 3) X(3, 4) X(3, 5) X(3, 6) X(3, 7) X(3, 8)

bool degree_supported(int dim, int p) {
  if (dim == 2) return p >= 1 && p <= 10;
  if (dim == 3) return p >= 1 && p <= 8;
  return false;
}

int launch_residual(const esd_plan* pl, const double* u, double* dudt, Workspace ws, hipStream_t s) {
#define X(D, PP) \
  if (pl->dim == D && pl->p == PP) return run_residual<D, PP>(pl, u, dudt, ws, s);
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

int launch_rk_stage(double* acc, double* U, const double* u, const double* k, double ca, double cu, int first,
                    int64_t n, hipStream_t s) {
  const int bs = 256;
  int64_t nb = (n + bs - 1) / bs;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_rk_stage, dim3(nb), dim3(bs), 0, s, acc, U, u, k, ca, cu, first, n);
  return (int)hipGetLastError();
}

int launch_axpy(double* y, const double* x, double a, const double* z, int64_t n, hipStream_t s) {
  const int bs = 256;
  int64_t nb = (n + bs - 1) / bs;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_axpy, dim3(nb), dim3(bs), 0, s, y, x, a, z, n);
  return (int)hipGetLastError();
}

int launch_vjp(const esd_plan*, const double*, const double*, double*, Workspace, hipStream_t) { return -1; }

}  // namespace esd
