// Probe kernels whose gfx950 code gives the FP64 instruction cost of one
// logarithm, exponential, square root and division as the compiler emits them
// for the library (same flags).  Never launched: paper_2312_07874_amd/flopweights.py
// compiles this file and counts the instructions of each kernel body against
// the baseline kernel's.
#include <hip/hip_runtime.h>

#include <cmath>

extern "C" __global__ void k_base(double* x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = x[i] * 1.5;
}
extern "C" __global__ void k_log(double* x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = log(x[i]);
}
extern "C" __global__ void k_exp(double* x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = exp(x[i]);
}
extern "C" __global__ void k_sqrt(double* x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = sqrt(x[i]);
}
extern "C" __global__ void k_div(double* x, const double* y, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = x[i] / y[i];
}
