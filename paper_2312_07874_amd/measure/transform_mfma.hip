// FP64 VALU against v_mfma_f64_16x16x4 on the largest stage of the
// sum-factorised PKD transform (Sec. 5.2), on gfx950.
//
// The stage: out[c][i + Q l] = sum_a psi1[a][i] X[c][l][a] for the N = 5 Q^2
// lines (c, l) of one tetrahedron's five variables (the last stage of V at
// degree p = Q - 1), the lines' values staged in LDS as the library's kernels
// stage them.  One element per workgroup of 256 threads.
//   k_valu: one lane per line, its Q inputs read from LDS once, Q accumulators
//           in registers, psi1 read uniformly (scalar loads), as the library.
//   k_mfma: one wave per tile of 16 lines; A = psi1^T (16 x 4 per step, zero
//           beyond Q), B = 4 inputs of each of the 16 lines per step, D the
//           16 x 16 outputs of the tile, ceil(Q / 4) steps.
// The program first checks the MFMA register layout it assumes (A[m][k]:
// lane m + 16 k; B[k][n]: lane n + 16 k; D[m][n]: lane n + 16 (m % 4),
// element m / 4, as measured with one-hot inputs) on one tile against a host
// product, then times both kernels on the same data and compares their
// results.
//
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//       -o transform_mfma transform_mfma.hip && ./transform_mfma
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                  \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));               \
      std::exit(1);                                                               \
    }                                                                             \
  } while (0)

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NC = 5;
constexpr int BLOCK = 256;

// one tile: D = A B with A 16 x 4, B 4 x 16 given in row-major host order
__global__ void k_layout(const double* A, const double* B, double* D) {
  const int lane = threadIdx.x;
  const double a = A[(lane % 16) * 4 + lane / 16];
  const double b = B[(lane / 16) * 16 + lane % 16];
  d4 d = {0.0, 0.0, 0.0, 0.0};
  d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d, 0, 0, 0);
  for (int i = 0; i < 4; ++i) D[(4 * i + lane / 16) * 16 + lane % 16] = d[i];
}

template <int Q>
__global__ void __launch_bounds__(BLOCK) k_valu(const double* __restrict__ X, double* __restrict__ Y,
                                                const double* __restrict__ psi1) {
  constexpr int N = NC * Q * Q;
  __shared__ double s[N * Q];
  const double* x = X + (size_t)blockIdx.x * N * Q;
  for (int o = threadIdx.x; o < N * Q; o += BLOCK) s[o] = x[o];
  __syncthreads();
  double* y = Y + (size_t)blockIdx.x * N * Q;
  for (int col = threadIdx.x; col < N; col += BLOCK) {
    double acc[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) acc[i] = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const double v = s[col * Q + a];
#pragma unroll
      for (int i = 0; i < Q; ++i) acc[i] += psi1[a * Q + i] * v;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) y[col * Q + i] = acc[i];
  }
}

template <int Q>
__global__ void __launch_bounds__(BLOCK) k_mfma(const double* __restrict__ X, double* __restrict__ Y,
                                                const double* __restrict__ psi1) {
  constexpr int N = NC * Q * Q, KS = (Q + 3) / 4, TILES = (N + 15) / 16;
  __shared__ double s[N * Q];
  const double* x = X + (size_t)blockIdx.x * N * Q;
  for (int o = threadIdx.x; o < N * Q; o += BLOCK) s[o] = x[o];
  __syncthreads();
  double* y = Y + (size_t)blockIdx.x * N * Q;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, m = lane % 16, kq = lane / 16;
  double a[KS];
#pragma unroll
  for (int st = 0; st < KS; ++st) {
    const int k = 4 * st + kq;
    a[st] = (m < Q && k < Q) ? psi1[k * Q + m] : 0.0;
  }
  for (int t = wave; t < TILES; t += BLOCK / 64) {
    const int col = t * 16 + lane % 16;
    const bool valid = col < N;
    d4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      const int k = 4 * st + kq;
      const double b = (valid && k < Q) ? s[col * Q + k] : 0.0;
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b, d, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 4 * i + kq;
      if (valid && row < Q) y[col * Q + row] = d[i];
    }
  }
}

template <int Q>
static void run(int ne, int reps) {
  constexpr int N = NC * Q * Q;
  const size_t n = (size_t)ne * N * Q;
  std::vector<double> hx(n), hp(Q * Q);
  unsigned s = 12345u;
  auto rnd = [&]() {
    s = s * 1664525u + 1013904223u;
    return (double)(s >> 8) / 16777216.0 - 0.5;
  };
  for (auto& v : hx) v = rnd();
  for (auto& v : hp) v = rnd();
  double *X, *Y1, *Y2, *psi;
  CHECK(hipMalloc(&X, n * sizeof(double)));
  CHECK(hipMalloc(&Y1, n * sizeof(double)));
  CHECK(hipMalloc(&Y2, n * sizeof(double)));
  CHECK(hipMalloc(&psi, Q * Q * sizeof(double)));
  CHECK(hipMemcpy(X, hx.data(), n * sizeof(double), hipMemcpyHostToDevice));
  CHECK(hipMemcpy(psi, hp.data(), Q * Q * sizeof(double), hipMemcpyHostToDevice));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  float ms[2];
  for (int which = 0; which < 2; ++which) {
    auto launch = [&]() {
      if (which == 0) hipLaunchKernelGGL(k_valu<Q>, dim3(ne), dim3(BLOCK), 0, 0, X, Y1, psi);
      else hipLaunchKernelGGL(k_mfma<Q>, dim3(ne), dim3(BLOCK), 0, 0, X, Y2, psi);
    };
    launch();
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e0));
    for (int r = 0; r < reps; ++r) launch();
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    CHECK(hipEventElapsedTime(&ms[which], e0, e1));
    ms[which] /= reps;
  }
  std::vector<double> y1(n), y2(n);
  CHECK(hipMemcpy(y1.data(), Y1, n * sizeof(double), hipMemcpyDeviceToHost));
  CHECK(hipMemcpy(y2.data(), Y2, n * sizeof(double), hipMemcpyDeviceToHost));
  double err = 0.0, scale = 0.0;
  for (size_t i = 0; i < n; ++i) {
    err = std::fmax(err, std::fabs(y1[i] - y2[i]));
    scale = std::fmax(scale, std::fabs(y1[i]));
  }
  const double flops = 2.0 * N * Q * Q * (double)ne;   // useful multiply-adds x 2
  std::printf("{\"p\": %d, \"elements\": %d, \"valu_ms\": %.4f, \"mfma_ms\": %.4f, \"valu_tflops\": %.2f, "
              "\"mfma_tflops\": %.2f, \"max_rel_diff\": %.2e}\n",
              Q - 1, ne, ms[0], ms[1], flops / (ms[0] * 1e-3) / 1e12, flops / (ms[1] * 1e-3) / 1e12, err / scale);
  std::fflush(stdout);
  CHECK(hipFree(X));
  CHECK(hipFree(Y1));
  CHECK(hipFree(Y2));
  CHECK(hipFree(psi));
}

int main() {
  // register layout of the MFMA on one tile
  std::vector<double> A(64), B(64), D(256), R(256, 0.0);
  for (int i = 0; i < 64; ++i) {
    A[i] = 1.0 + i;
    B[i] = 0.5 * i - 7.0;
  }
  for (int mm = 0; mm < 16; ++mm)
    for (int nn = 0; nn < 16; ++nn)
      for (int k = 0; k < 4; ++k) R[mm * 16 + nn] += A[mm * 4 + k] * B[k * 16 + nn];
  double *dA, *dB, *dD;
  CHECK(hipMalloc(&dA, 64 * sizeof(double)));
  CHECK(hipMalloc(&dB, 64 * sizeof(double)));
  CHECK(hipMalloc(&dD, 256 * sizeof(double)));
  CHECK(hipMemcpy(dA, A.data(), 64 * sizeof(double), hipMemcpyHostToDevice));
  CHECK(hipMemcpy(dB, B.data(), 64 * sizeof(double), hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_layout, dim3(1), dim3(64), 0, 0, dA, dB, dD);
  CHECK(hipGetLastError());
  CHECK(hipMemcpy(D.data(), dD, 256 * sizeof(double), hipMemcpyDeviceToHost));
  double lerr = 0.0;
  for (int i = 0; i < 256; ++i) lerr = std::fmax(lerr, std::fabs(D[i] - R[i]));
  std::printf("{\"layout_max_abs_err\": %.3e}\n", lerr);
  std::fflush(stdout);
  if (lerr > 1e-9) {
    std::printf("{\"error\": \"MFMA register layout differs from the assumed one\"}\n");
    return 1;
  }
  run<7>(4096, 20);
  run<9>(4096, 20);
  run<11>(4096, 20);
  CHECK(hipFree(dA));
  CHECK(hipFree(dB));
  CHECK(hipFree(dD));
  return 0;
}
