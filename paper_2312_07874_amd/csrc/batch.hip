// Exterior facet values across interfaces between elements of different
// degree (gfx950, FP64), and their adjoint.
//
// Each facet of an element whose neighbour has another degree:
//   w+[c][j] = sum_k I[j][k] w~_nb[c][k],   j < NQF (this degree), k < NP (neighbour's),
// I the neighbour's PKD basis at the reference points of this facet's nodes
// (built on the host).  The result lands in the element's exterior slot, laid
// out like its own facet values, where the right-hand-side kernel reads it
// through the facet permutation table like any other neighbour value.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace esd {

// Matrices are stored transposed, I^T [k][j], so that the threads of a facet
// (one per facet node j) read consecutive words.
constexpr int MIX_MAX_NP = 286;    // PKD modes of a degree-10 tetrahedron
constexpr int MIX_MAX_NQF = 121;   // facet nodes of a degree-10 tetrahedron
constexpr int MIX_BLOCK = 128;

// The facets are grouped by the element whose w~ they read (up to one per
// face of it, in the records of adjoint below): one workgroup per such
// element stages its w~ (at most 5 x 286 values) in LDS once and evaluates
// every facet of the group, instead of one workgroup per facet staging it
// again (measured on the batch of 35,904 tetrahedra: K1 with the interface
// kernels 3.02 -> 2.96 ms per residual).  NC (variables) is fixed at compile time
// and the contraction unrolled, so that several matrix rows are in flight per
// thread.  A facet of few nodes (nqf <= 42: tetrahedra up to p = 5, every
// triangle) would leave most of the 128 lanes idle and one lane walking all np
// modes; there the lanes split into S = 128 / nqf >= 3 slices, slice s summing
// the modes k = s, s + S, ..., and the slices' partial sums are added in LDS.
// Record, int32 [8]: destination bucket b, destination slot e, face f,
// matrix, source slot (the element whose w~ is read), NQF of b, NFQ of b,
// unused.
template <int NC>
__global__ void __launch_bounds__(MIX_BLOCK)
k_mixed_exterior(const int32_t* __restrict__ segs, const int32_t* __restrict__ recs, const double* __restrict__ ws_base,
                 const int64_t* __restrict__ wt_off, const int64_t* __restrict__ wext_off,
                 const double* __restrict__ mats, const int64_t* __restrict__ mat_off, int src_bucket, int np) {
  __shared__ double sW[5 * MIX_MAX_NP];
  __shared__ double sR[NC * MIX_BLOCK];
  const int first = segs[2 * blockIdx.x], count = segs[2 * blockIdx.x + 1];
  const int slot = recs[8 * first + 4];
  const double* wtn = ws_base + wt_off[src_bucket] + (int64_t)slot * NC * np;
  for (int o = threadIdx.x; o < NC * np; o += MIX_BLOCK) sW[o] = wtn[o];
  __syncthreads();
  for (int r = first; r < first + count; ++r) {
    const int32_t* t = recs + 8 * (int64_t)r;
    const int b = t[0], e = t[1], f = t[2], m = t[3], nqf = t[5], nfq = t[6];
    const double* IT = mats + mat_off[m];
    double* dst = const_cast<double*>(ws_base) + wext_off[b] + (int64_t)e * NC * nfq + f * nqf;
    if (3 * nqf > MIX_BLOCK) {
      for (int j = threadIdx.x; j < nqf; j += MIX_BLOCK) {
        double acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = 0.0;
#pragma unroll 8
        for (int k = 0; k < np; ++k) {
          const double a = IT[(int64_t)k * nqf + j];
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[c] += a * sW[c * np + k];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) dst[c * nfq + j] = acc[c];
      }
      continue;
    }
    // nqf <= 42: thread = (slice s, node j), s < S = MIX_BLOCK / nqf
    const int S = MIX_BLOCK / nqf;
    const int sl = threadIdx.x / nqf, j = threadIdx.x - sl * nqf;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    if (sl < S) {
#pragma unroll 4
      for (int k = sl; k < np; k += S) {
        const double a = IT[(int64_t)k * nqf + j];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += a * sW[c * np + k];
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) sR[c * MIX_BLOCK + threadIdx.x] = acc[c];
    __syncthreads();
    if (threadIdx.x < nqf) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double v = 0.0;
        for (int q = 0; q < S; ++q) v += sR[c * MIX_BLOCK + q * nqf + threadIdx.x];
        dst[c * nfq + threadIdx.x] = v;
      }
    }
    __syncthreads();   // sR is reused by the next facet
  }
}

// Adjoint of the facet evaluation above: w~_bar_nb[c][k] += sum_j I[j][k] x_bar_e[c][j],
// x_bar_e the cotangent of the exterior values of facet f of element e (the
// right-hand side's adjoint writes it at e's own facet nodes).  One workgroup
// per element nb of this bucket whose w~ some task reads; it walks the
// records of those tasks (one per facet of nb with a neighbour of another
// degree) in a fixed order and adds the sum to nb's w~_bar once, so there is
// no atomic and the result does not depend on scheduling.  Record, int32 [8]:
// source bucket, source slot e, face f, matrix, target slot nb, source NQF,
// source NFQ, unused.
constexpr int MIX_KMAX = (MIX_MAX_NP + MIX_BLOCK - 1) / MIX_BLOCK;

template <int NC>
__global__ void __launch_bounds__(MIX_BLOCK)
k_mixed_exterior_vjp(const int32_t* __restrict__ segs, const int32_t* __restrict__ recs,
                     const double* __restrict__ ws_base, const int64_t* __restrict__ xbar_off,
                     const double* __restrict__ mats, const int64_t* __restrict__ mat_off, double* __restrict__ grad,
                     int np) {
  __shared__ double sX[NC * MIX_MAX_NQF];
  const int first = segs[2 * blockIdx.x], count = segs[2 * blockIdx.x + 1];
  const int slot = recs[8 * first + 4];
  double acc[MIX_KMAX][NC];
#pragma unroll
  for (int q = 0; q < MIX_KMAX; ++q)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[q][c] = 0.0;
  for (int r = first; r < first + count; ++r) {
    const int32_t* t = recs + 8 * (int64_t)r;
    const int b = t[0], e = t[1], f = t[2], m = t[3], nqf = t[5], nfq = t[6];
    const double* xb = ws_base + xbar_off[b] + (int64_t)e * NC * nfq + f * nqf;
    __syncthreads();   // the previous record's values are read
    for (int o = threadIdx.x; o < NC * nqf; o += MIX_BLOCK) {
      const int c = o / nqf, j = o - c * nqf;
      sX[o] = xb[c * nfq + j];
    }
    __syncthreads();
    const double* IT = mats + mat_off[m];   // [k][j]
#pragma unroll
    for (int q = 0; q < MIX_KMAX; ++q) {
      const int k = threadIdx.x + q * MIX_BLOCK;
      if (k < np) {
        const double* row = IT + (int64_t)k * nqf;
#pragma unroll 4
        for (int j = 0; j < nqf; ++j) {
          const double a = row[j];
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[q][c] += a * sX[c * nqf + j];
        }
      }
    }
  }
  double* g = grad + (int64_t)slot * NC * np;
#pragma unroll
  for (int q = 0; q < MIX_KMAX; ++q) {
    const int k = threadIdx.x + q * MIX_BLOCK;
    if (k < np) {
#pragma unroll
      for (int c = 0; c < NC; ++c) g[c * np + k] += acc[q][c];
    }
  }
}

int launch_mixed_exterior_vjp(const esd_plan* b, const esd_plan* top, const double* ws_base, double* grad,
                              hipStream_t s) {
  if (b->n_asegs == 0) return 0;
  if (b->ref.NP > MIX_MAX_NP) return -1;
  if (b->nc == 5)
    hipLaunchKernelGGL(k_mixed_exterior_vjp<5>, dim3((unsigned)b->n_asegs), dim3(MIX_BLOCK), 0, s, b->d_asegs,
                       b->d_arecs, ws_base, top->d_xbar_off, top->d_mats, top->d_mat_off, grad, b->ref.NP);
  else
    hipLaunchKernelGGL(k_mixed_exterior_vjp<4>, dim3((unsigned)b->n_asegs), dim3(MIX_BLOCK), 0, s, b->d_asegs,
                       b->d_arecs, ws_base, top->d_xbar_off, top->d_mats, top->d_mat_off, grad, b->ref.NP);
  return (int)hipGetLastError();
}

int launch_mixed_exterior(const esd_plan* b, int bi, const esd_plan* top, const double* ws_base, hipStream_t s) {
  if (b->n_asegs == 0) return 0;
  if (b->ref.NP > MIX_MAX_NP) return -1;
  if (b->nc == 5)
    hipLaunchKernelGGL(k_mixed_exterior<5>, dim3((unsigned)b->n_asegs), dim3(MIX_BLOCK), 0, s, b->d_asegs, b->d_arecs,
                       ws_base, top->d_wt_off, top->d_wext_off, top->d_mats, top->d_mat_off, bi, b->ref.NP);
  else
    hipLaunchKernelGGL(k_mixed_exterior<4>, dim3((unsigned)b->n_asegs), dim3(MIX_BLOCK), 0, s, b->d_asegs, b->d_arecs,
                       ws_base, top->d_wt_off, top->d_wext_off, top->d_mats, top->d_mat_off, bi, b->ref.NP);
  return (int)hipGetLastError();
}

}  // namespace esd
