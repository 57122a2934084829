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
  static constexpr int EPB = 1;
  static constexpr int BS = (3 * (P + 1) * (P + 1) <= 128) ? 128 : ((3 * (P + 1) * (P + 1) + 63) / 64) * 64;
};
template <int P>
struct Launch<2, P> {
  static constexpr int LINES = 2 * (P + 1);
  static constexpr int EPB = (P <= 4) ? 12 : ((P <= 7) ? 8 : 6);
  static constexpr int BS = ((EPB * LINES + 63) / 64) * 64 < 128 ? 128 : ((EPB * LINES + 63) / 64) * 64;
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
// threads of the block participate; each call ends with a barrier.
template <int DIM, int P>
__device__ void xform_V(const double* uh, double* T1, double* T2, double* out, const DevTables& T, int nec) {
  using S = Shape<DIM, P>;
  constexpr int Q = S::Q;
  const int tid = threadIdx.x, nth = blockDim.x;
  if constexpr (DIM == 2) {
    for (int o = tid; o < nec * (P + 1) * Q; o += nth) {
      const int i2 = o % Q, a1 = (o / Q) % (P + 1), ec = o / (Q * (P + 1));
      const int mb = a1 * (P + 1) - a1 * (a1 - 1) / 2;
      double acc = 0.0;
      for (int a2 = 0; a2 <= P - a1; ++a2) acc += T.psi2[(a1 * (P + 1) + a2) * Q + i2] * uh[ec * S::NP + mb + a2];
      T1[o] = acc;
    }
    __syncthreads();
    for (int o = tid; o < nec * S::NQ; o += nth) {
      const int i1 = o % Q, i2 = (o / Q) % Q, ec = o / S::NQ;
      double acc = 0.0;
#pragma unroll
      for (int a1 = 0; a1 <= P; ++a1) acc += T.psi1[a1 * Q + i1] * T1[(ec * (P + 1) + a1) * Q + i2];
      out[o] = acc;
    }
    __syncthreads();
  } else {
    for (int o = tid; o < nec * S::NPAIR * Q; o += nth) {
      const int i3 = o % Q, r = o / Q, pr = r % S::NPAIR, ec = r / S::NPAIR;
      int a1, a2;
      decode_pair(P, pr, a1, a2);
      const int s = a1 + a2, mb = tet_mode_base(P, a1, a2);
      double acc = 0.0;
      for (int a3 = 0; a3 <= P - s; ++a3) acc += T.psi3[(s * (P + 1) + a3) * Q + i3] * uh[ec * S::NP + mb + a3];
      T1[o] = acc;
    }
    __syncthreads();
    for (int o = tid; o < nec * (P + 1) * Q * Q; o += nth) {
      const int i3 = o % Q, i2 = (o / Q) % Q, a1 = (o / (Q * Q)) % (P + 1), ec = o / (Q * Q * (P + 1));
      const int pb = pair_index(P, a1, 0);
      double acc = 0.0;
      for (int a2 = 0; a2 <= P - a1; ++a2)
        acc += T.psi2[(a1 * (P + 1) + a2) * Q + i2] * T1[(ec * S::NPAIR + pb + a2) * Q + i3];
      T2[o] = acc;
    }
    __syncthreads();
    for (int o = tid; o < nec * S::NQ; o += nth) {
      const int i1 = o % Q, i2 = (o / Q) % Q, i3 = (o / (Q * Q)) % Q, ec = o / S::NQ;
      double acc = 0.0;
#pragma unroll
      for (int a1 = 0; a1 <= P; ++a1) acc += T.psi1[a1 * Q + i1] * T2[((ec * (P + 1) + a1) * Q + i2) * Q + i3];
      out[o] = acc;
    }
    __syncthreads();
  }
}

template <int DIM, int P>
__device__ void xform_Vt(const double* in, double* T1, double* T2, double* out, const DevTables& T, int nec) {
  using S = Shape<DIM, P>;
  constexpr int Q = S::Q;
  const int tid = threadIdx.x, nth = blockDim.x;
  if constexpr (DIM == 2) {
    for (int o = tid; o < nec * (P + 1) * Q; o += nth) {
      const int i2 = o % Q, a1 = (o / Q) % (P + 1), ec = o / (Q * (P + 1));
      double acc = 0.0;
#pragma unroll
      for (int i1 = 0; i1 < Q; ++i1) acc += T.psi1[a1 * Q + i1] * in[ec * S::NQ + i1 + Q * i2];
      T1[o] = acc;
    }
    __syncthreads();
    for (int o = tid; o < nec * S::NP; o += nth) {
      const int m = o % S::NP, ec = o / S::NP;
      int a1, a2;
      decode_tri_mode(P, m, a1, a2);
      double acc = 0.0;
#pragma unroll
      for (int i2 = 0; i2 < Q; ++i2) acc += T.psi2[(a1 * (P + 1) + a2) * Q + i2] * T1[(ec * (P + 1) + a1) * Q + i2];
      out[o] = acc;
    }
    __syncthreads();
  } else {
    for (int o = tid; o < nec * (P + 1) * Q * Q; o += nth) {
      const int i3 = o % Q, i2 = (o / Q) % Q, a1 = (o / (Q * Q)) % (P + 1), ec = o / (Q * Q * (P + 1));
      double acc = 0.0;
#pragma unroll
      for (int i1 = 0; i1 < Q; ++i1) acc += T.psi1[a1 * Q + i1] * in[ec * S::NQ + i1 + Q * (i2 + Q * i3)];
      T2[o] = acc;
    }
    __syncthreads();
    for (int o = tid; o < nec * S::NPAIR * Q; o += nth) {
      const int i3 = o % Q, r = o / Q, pr = r % S::NPAIR, ec = r / S::NPAIR;
      int a1, a2;
      decode_pair(P, pr, a1, a2);
      double acc = 0.0;
#pragma unroll
      for (int i2 = 0; i2 < Q; ++i2)
        acc += T.psi2[(a1 * (P + 1) + a2) * Q + i2] * T2[((ec * (P + 1) + a1) * Q + i2) * Q + i3];
      T1[o] = acc;
    }
    __syncthreads();
    for (int o = tid; o < nec * S::NP; o += nth) {
      const int m = o % S::NP, ec = o / S::NP;
      int a1, a2, a3;
      decode_tet_mode(P, m, a1, a2, a3);
      const int s = a1 + a2, pr = pair_index(P, a1, a2);
      double acc = 0.0;
#pragma unroll
      for (int i3 = 0; i3 < Q; ++i3) acc += T.psi3[(s * (P + 1) + a3) * Q + i3] * T1[(ec * S::NPAIR + pr) * Q + i3];
      out[o] = acc;
    }
    __syncthreads();
  }
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
  double v2 = 0.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    n.v[i] = w[1 + i] / b;
    v2 += n.v[i] * n.v[i];
  }
  const double s = S.gamma - (S.gamma - 1.0) * (w[0] + 0.5 * b * v2);
  n.b = b;
  n.lnb = log(b);
  n.lnrho = -(s + n.lnb) * S.gm1_inv;
  n.rho = exp(n.lnrho);
  n.p = n.rho / b;
  return (b > 0.0) && isfinite(n.rho) && isfinite(n.p) && (n.rho > 0.0);
}

constexpr double LOG_SERIES_THRESHOLD = 1.0e-4;

// logarithmic mean (a+ - a-)/(ln a+ - ln a-) from precomputed logs; series in
// f = (a+ - a-)/(a+ + a-) through f^6/7 when f^2 < 1e-4
__device__ __forceinline__ double log_mean(double a, double b, double la, double lb) {
  const double d = b - a, s = a + b;
  if (d * d < LOG_SERIES_THRESHOLD * s * s) {
    const double u = (d * d) / (s * s);
    return s / (2.0 * (1.0 + u * (1.0 / 3.0 + u * (1.0 / 5.0 + u * (1.0 / 7.0)))));
  }
  return d / (lb - la);
}
__device__ __forceinline__ double inv_log_mean(double a, double b, double la, double lb) {
  const double d = b - a, s = a + b;
  if (d * d < LOG_SERIES_THRESHOLD * s * s) {
    const double u = (d * d) / (s * s);
    return 2.0 * (1.0 + u * (1.0 / 3.0 + u * (1.0 / 5.0 + u * (1.0 / 7.0)))) / s;
  }
  return (lb - la) / d;
}

// directional entropy-conservative flux f#(A, B, n) = sum_m n_m f#_m(A, B)
template <int DIM, int FLUX>
__device__ __forceinline__ void ec_flux(const Node<DIM>& A, const Node<DIM>& B, const double* n, const Scheme& S,
                                        double* F) {
  const double rho_ln = log_mean(A.rho, B.rho, A.lnrho, B.lnrho);
  const double ib_ln = inv_log_mean(A.b, B.b, A.lnb, B.lnb);   // 1 / {rho/p}_ln
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
    const double phat = (A.rho + B.rho) / (A.b + B.b);      // {rho} / (2 {beta}), beta = b/2
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

// ------------------------------------------------------------------ K2 helpers: one collapsed line
// Pairs (a < b) of the line with nodes base + stride*k: F = f#(u_a, u_b, n_ab),
// n_ab = A0_ab (h0_a + h0_b) [+ A1_ab (h1_a + h1_b)], r_a -= F, r_b += F.
template <int DIM, int P, int FLUX, int NA>
__device__ __forceinline__ void line_pairs(const double* sN, const double* __restrict__ g, int base, int stride,
                                           const double* __restrict__ A0, const double* __restrict__ A1, int hc0,
                                           int hc1, const Scheme& S, double (&acc)[P + 1][DIM + 2]) {
  using Sh = Shape<DIM, P>;
  constexpr int Q = Sh::Q, NQ = Sh::NQ, NC = Sh::NC;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const int na = base + stride * a;
    const Node<DIM> NAa = load_node<DIM>(sN, NQ, na);
    double h0a[DIM], h1a[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      h0a[i] = g[(hc0 + i) * NQ + na];
      if constexpr (NA == 2) h1a[i] = g[(hc1 + i) * NQ + na];
    }
#pragma unroll
    for (int b = a + 1; b < Q; ++b) {
      const int nb = base + stride * b;
      const Node<DIM> NBb = load_node<DIM>(sN, NQ, nb);
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
      ec_flux<DIM, FLUX>(NAa, NBb, n, S, F);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        acc[a][c] -= F[c];
        acc[b][c] += F[c];
      }
    }
  }
}

// facet-correction pair: C = coef * f#(u_i, u^z_j, (gn_i + nJ_j)/2); r_i -= C, t_j += C
template <int DIM, int FLUX>
__device__ __forceinline__ void facet_pair(const Node<DIM>& Vi, const double* gn_i, const Node<DIM>& Fj,
                                           const double* nJ_j, double coef, const Scheme& S, double* racc,
                                           double* tacc) {
  double n[DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i) n[i] = 0.5 * (gn_i[i] + nJ_j[i]);
  double F[DIM + 2];
  ec_flux<DIM, FLUX>(Vi, Fj, n, S, F);
#pragma unroll
  for (int c = 0; c < DIM + 2; ++c) {
    const double C = coef * F[c];
    racc[c] -= C;
    tacc[c] += C;
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

  // ---- flux differencing along lines + facet corrections
  const int el = tid / Sh::NLINES;
  const int lt = tid % Sh::NLINES;
  const int fam = lt / LPF, L = lt % LPF;
  const bool active = el < nel;
  double acc[Q][NC];
#pragma unroll
  for (int k = 0; k < Q; ++k)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[k][c] = 0.0;
  int base = 0, stride = 1;
  if (active) {
    const double* sNe = sN + el * Sh::SCR;
    const double* sFe = sF + el * 8 * NFQ;
    double* sTe = sT + el * NC * NFQ;
    const double* g = gvol + (e0 + el) * NGV * NQ;
    const double* gf = gfac + (e0 + el) * (DIM + 1) * NFQ;
    if constexpr (DIM == 2) {
      if (fam == 0) {
        base = Q * L;
        stride = 1;
        line_pairs<DIM, P, FLUX, 2>(sNe, g, base, stride, T.A + 0 * Q * Q, T.A + 1 * Q * Q, 0, 2, S, acc);
        // facets 1 (eta1 = +1) and 2 (eta1 = -1) on this eta1-line
        const double w2 = T.wl[L];
        const Node<DIM> F1 = load_node<DIM>(sFe, NFQ, 1 * NQF + L);
        const Node<DIM> F2 = load_node<DIM>(sFe, NFQ, 2 * NQF + L);
        double nJ1[2], nJ2[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          nJ1[i] = gf[i * NFQ + 1 * NQF + L];
          nJ2[i] = gf[i * NFQ + 2 * NQF + L];
        }
        double t1[NC] = {0}, t2[NC] = {0};
        const double cw1 = T.wf[1 * NQF + L], cw2 = T.wf[2 * NQF + L];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          const int nk = base + k;
          const Node<DIM> Vk = load_node<DIM>(sNe, NQ, nk);
          double gA[2], gB[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const double g1 = g[(0 + i) * NQ + nk] / w2;
            const double g2 = 2.0 * g[(2 + i) * NQ + nk] / w2;
            gA[i] = (g1 + g2) * 0.70710678118654752440;
            gB[i] = -g1;
          }
          facet_pair<DIM, FLUX>(Vk, gA, F1, nJ1, T.lgp1[k] * cw1, S, acc[k], t1);
          facet_pair<DIM, FLUX>(Vk, gB, F2, nJ2, T.lgm1[k] * cw2, S, acc[k], t2);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          sTe[c * NFQ + 1 * NQF + L] += t1[c];
          sTe[c * NFQ + 2 * NQF + L] += t2[c];
        }
      } else {
        base = L;
        stride = Q;
        line_pairs<DIM, P, FLUX, 1>(sNe, g, base, stride, T.A + 2 * Q * Q, nullptr, 4, 0, S, acc);
        // facet 0 (eta2 = -1) on this eta2-line
        const double w1 = T.wl[L];
        const Node<DIM> F0 = load_node<DIM>(sFe, NFQ, 0 * NQF + L);
        double nJ0[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) nJ0[i] = gf[i * NFQ + 0 * NQF + L];
        double t0[NC] = {0};
        const double cw0 = T.wf[0 * NQF + L];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          const int nk = base + stride * k;
          const Node<DIM> Vk = load_node<DIM>(sNe, NQ, nk);
          double gA[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) gA[i] = -2.0 * g[(4 + i) * NQ + nk] / w1;
          facet_pair<DIM, FLUX>(Vk, gA, F0, nJ0, T.lgm1[k] * cw0, S, acc[k], t0);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) sTe[c * NFQ + 0 * NQF + L] += t0[c];
      }
    } else {
      if (fam == 0) {
        // eta1-line (a2, a3)
        const int a2 = L % Q, a3 = L / Q;
        base = Q * L;
        stride = 1;
        line_pairs<DIM, P, FLUX, 2>(sNe, g, base, stride, T.A + 0 * Q * Q, T.A + 1 * Q * Q, 0, 3, S, acc);
        const double inv23 = 1.0 / (T.wl[a2] * T.wj[a3]);
        const Node<DIM> F1 = load_node<DIM>(sFe, NFQ, 1 * NQF + L);
        const Node<DIM> F2 = load_node<DIM>(sFe, NFQ, 2 * NQF + L);
        double nJ1[3], nJ2[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          nJ1[i] = gf[i * NFQ + 1 * NQF + L];
          nJ2[i] = gf[i * NFQ + 2 * NQF + L];
        }
        double t1[NC] = {0}, t2[NC] = {0};
        const double cw1 = T.wf[1 * NQF + L], cw2 = T.wf[2 * NQF + L];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          const int nk = base + k;
          const Node<DIM> Vk = load_node<DIM>(sNe, NQ, nk);
          double gA[3], gB[3];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            const double g1 = 2.0 * g[(0 + i) * NQ + nk] * inv23;
            const double g23 = 4.0 * g[(3 + i) * NQ + nk] * inv23;
            gA[i] = (g1 + g23) * 0.57735026918962576451;
            gB[i] = -g1;
          }
          facet_pair<DIM, FLUX>(Vk, gA, F1, nJ1, T.lgp1[k] * cw1, S, acc[k], t1);
          facet_pair<DIM, FLUX>(Vk, gB, F2, nJ2, T.lgm1[k] * cw2, S, acc[k], t2);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          sTe[c * NFQ + 1 * NQF + L] += t1[c];
          sTe[c * NFQ + 2 * NQF + L] += t2[c];
        }
      } else if (fam == 1) {
        // eta2-line (a1, a3)
        const int a1 = L % Q, a3 = L / Q;
        base = a1 + Q * Q * a3;
        stride = Q;
        line_pairs<DIM, P, FLUX, 2>(sNe, g, base, stride, T.A + 2 * Q * Q, T.A + 3 * Q * Q, 6, 9, S, acc);
        const double inv13 = 1.0 / (T.wl[a1] * T.wj[a3]);
        const Node<DIM> F0 = load_node<DIM>(sFe, NFQ, 0 * NQF + L);
        double nJ0[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) nJ0[i] = gf[i * NFQ + 0 * NQF + L];
        double t0[NC] = {0};
        const double cw0 = T.wf[0 * NQF + L];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          const int nk = base + stride * k;
          const Node<DIM> Vk = load_node<DIM>(sNe, NQ, nk);
          double gA[3];
#pragma unroll
          for (int i = 0; i < 3; ++i) gA[i] = -4.0 * g[(6 + i) * NQ + nk] * inv13;
          facet_pair<DIM, FLUX>(Vk, gA, F0, nJ0, T.lgm1[k] * cw0, S, acc[k], t0);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) sTe[c * NFQ + 0 * NQF + L] += t0[c];
      } else {
        // eta3-line (a1, a2)
        const int a1 = L % Q, a2 = L / Q;
        base = L;
        stride = Q * Q;
        line_pairs<DIM, P, FLUX, 1>(sNe, g, base, stride, T.A + 4 * Q * Q, nullptr, 12, 0, S, acc);
        // face 4 (xi3 = -1): facet nodes (a1, b) for every b, volume nodes of this line
        const double inv12 = 1.0 / (T.wl[a1] * T.wl[a2] * (1.0 - T.xl[a2]));
        double gA[Q][3];
#pragma unroll
        for (int k = 0; k < Q; ++k)
#pragma unroll
          for (int i = 0; i < 3; ++i) gA[k][i] = -8.0 * g[(12 + i) * NQ + base + stride * k] * inv12;
        for (int bq = 0; bq < Q; ++bq) {
          const int j = 3 * NQF + a1 + Q * bq;
          const Node<DIM> Fj = load_node<DIM>(sFe, NFQ, j);
          double nJ[3];
#pragma unroll
          for (int i = 0; i < 3; ++i) nJ[i] = gf[i * NFQ + j];
          const double cw = T.wf[j] * T.I42[bq * Q + a2];
          double tj[NC] = {0};
#pragma unroll
          for (int k = 0; k < Q; ++k) {
            const Node<DIM> Vk = load_node<DIM>(sNe, NQ, base + stride * k);
            facet_pair<DIM, FLUX>(Vk, gA[k], Fj, nJ, cw * T.gjm1[k], S, acc[k], tj);
          }
#pragma unroll
          for (int c = 0; c < NC; ++c) atomicAdd(&sTe[c * NFQ + j], tj[c]);
        }
      }
    }
  }
  // ordered accumulation of the line families into r (deterministic)
#pragma unroll
  for (int ph = 0; ph < DIM; ++ph) {
    if (active && fam == ph) {
      double* r = sR + el * NC * NQ;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const int nk = base + stride * k;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (ph == 0)
            r[c * NQ + nk] = acc[k][c];
          else
            r[c * NQ + nk] += acc[k][c];
        }
      }
    }
    __syncthreads();
  }

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
