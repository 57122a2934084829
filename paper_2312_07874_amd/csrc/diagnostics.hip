// Global diagnostics of a state (gfx950, FP64): the conserved integrals
// sum_k w_k J_k u_k per variable (Theorem on conservation), the entropy
// integral sum_k w_k J_k S(u_k) with S = -rho s/(gamma-1) (eq. euler_entropy),
// and its semi-discrete rate sum_k w_k J_k W(u_k) . (V du~/dt)_k (Theorem on
// entropy conservation/stability), u = V u~.
//
// One kernel forms per-element partial sums (LDS tree over the volume nodes;
// the rate as V^T (w J W(u)) . du~/dt in modal space), a second one reduces
// them over the elements in a fixed order, so the result is bitwise
// reproducible.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.hpp"

namespace esd {

// sum over the threads of a workgroup of nv values per thread, red [nv][nth];
// result in red[c * nth]; any block size (folded to a power of two first)
__device__ void block_sum(double* red, const double* acc, int nv) {
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int c = 0; c < nv; ++c) red[c * nth + tid] = acc[c];
  __syncthreads();
  int pw = 1;
  while (pw * 2 <= nth) pw *= 2;
  if (tid >= pw)
    for (int c = 0; c < nv; ++c) red[c * nth + tid - pw] += red[c * nth + tid];
  __syncthreads();
  for (int h = pw / 2; h > 0; h >>= 1) {
    if (tid < h)
      for (int c = 0; c < nv; ++c) red[c * nth + tid] += red[c * nth + tid + h];
    __syncthreads();
  }
}

template <int DIM, int P>
__global__ void __launch_bounds__((Launch<DIM, P>::BS))
k_diag_partials(const double* __restrict__ u, const double* __restrict__ dudt, const double* __restrict__ gvol,
                double* __restrict__ part, DevTables T0, Scheme S, int64_t ne) {
  using Sh = Shape<DIM, P>;
  constexpr int EPB = Launch<DIM, P>::EPB;
  constexpr int NC = Sh::NC, NQ = Sh::NQ, NP = Sh::NP, NGV = Sh::NGV, NO = NC + 2;
  constexpr int RED = Launch<DIM, P>::BS * (NC + 1);
  __shared__ double sM[EPB * NC * NP];
  __shared__ double sU[EPB * NC * NQ];
  __shared__ double sS[EPB * Sh::SCR > RED ? EPB * Sh::SCR : RED];   // transform scratch, then reductions
  constexpr int NS = EPB * Sh::SCR > RED ? EPB * Sh::SCR : RED;
  constexpr unsigned TM = tab_mask<DIM, P, TAB_PSI>(8 * (EPB * NC * NP + EPB * NC * NQ + NS));
  __shared__ double sTab[TM ? TabLds<DIM, P, TM>::SIZE : 1];
  const DevTables T = stage_tables<DIM, P, TM>(T0, sTab);
  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const int nel = (int)((ne - e0) < EPB ? (ne - e0) : EPB);
  const int nec = nel * NC;
  const int tid = threadIdx.x, nth = blockDim.x;
  double* T1 = sS;
  double* T2 = sS + EPB * Sh::T1;
  for (int o = tid; o < nec * NP; o += nth) sM[o] = u[e0 * NC * NP + o];
  __syncthreads();
  xform_V<DIM, P>(sM, T1, T2, sU, T, nec);
  // conserved integrals and entropy; sU is overwritten by w J W(u)
  for (int el = 0; el < nel; ++el) {
    double acc[NC + 1];
#pragma unroll
    for (int c = 0; c <= NC; ++c) acc[c] = 0.0;
    double* a = sU + el * NC * NQ;
    for (int k = tid; k < NQ; k += nth) {
      const double wJ = gvol[((e0 + el) * NGV + NGV - 2) * NQ + k];
      const double rho = a[k];
      double m2 = 0.0;
#pragma unroll
      for (int i = 0; i < DIM; ++i) m2 += a[(1 + i) * NQ + k] * a[(1 + i) * NQ + k];
      const double p = (S.gamma - 1.0) * (a[(DIM + 1) * NQ + k] - 0.5 * m2 / rho);
      const double s = log(p) - S.gamma * log(rho);
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] += wJ * a[c * NQ + k];
      acc[NC] += wJ * (-rho * s * S.gm1_inv);
      a[k] = wJ * ((S.gamma - s) * S.gm1_inv - 0.5 * m2 / (rho * p));
#pragma unroll
      for (int i = 0; i < DIM; ++i) a[(1 + i) * NQ + k] *= wJ / p;
      a[(DIM + 1) * NQ + k] = wJ * (-rho / p);
    }
    block_sum(sS, acc, NC + 1);
    if (tid <= NC) part[(e0 + el) * NO + tid] = sS[tid * nth];
    __syncthreads();
  }
  // entropy rate: (V^T w J W(u)) . du~/dt in modal space
  xform_Vt<DIM, P>(sU, T1, T2, sM, T, nec);
  for (int el = 0; el < nel; ++el) {
    double acc = 0.0;
    for (int o = tid; o < NC * NP; o += nth)
      acc += sM[el * NC * NP + o] * dudt[(e0 + el) * NC * NP + o];
    block_sum(sS, &acc, 1);
    if (tid == 0) part[(e0 + el) * NO + NC + 1] = sS[0];
    __syncthreads();
  }
}

// out[c] = sum_e part[e][c], c < no; one workgroup of 1024 threads, fixed order
__global__ void __launch_bounds__(1024) k_diag_reduce(const double* __restrict__ part, double* __restrict__ out,
                                                      int64_t ne, int no) {
  __shared__ double sRed[1024];
  const int tid = threadIdx.x;
  for (int c = 0; c < no; ++c) {
    double acc = 0.0;
    for (int64_t e = tid; e < ne; e += 1024) acc += part[e * no + c];
    sRed[tid] = acc;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
      if (tid < h) sRed[tid] += sRed[tid + h];
      __syncthreads();
    }
    if (tid == 0) out[c] = sRed[0];
    __syncthreads();
  }
}

template <int DIM, int P>
static int run_diag(const esd_plan* pl, const double* u, const double* dudt, double* part, double* out,
                    hipStream_t s) {
  using L = Launch<DIM, P>;
  const int64_t nb = (pl->ne + L::EPB - 1) / L::EPB;
  hipLaunchKernelGGL((k_diag_partials<DIM, P>), dim3(nb), dim3(L::BS), 0, s, u, dudt, pl->d_gvol, part, pl->tab,
                     pl->scheme, pl->ne);
  hipLaunchKernelGGL(k_diag_reduce, dim3(1), dim3(1024), 0, s, part, out, pl->ne, DIM + 4);
  return (int)hipGetLastError();
}

int launch_diagnostics(const esd_plan* pl, const double* u, const double* dudt, double* part, double* out,
                       hipStream_t s) {
#define X(D, PP) \
  if (pl->dim == D && pl->p == PP) return run_diag<D, PP>(pl, u, dudt, part, out, s);
  ESD_TRI_DEGREES(X)
  ESD_TET_DEGREES(X)
#undef X
  return -1;
}

}  // namespace esd
