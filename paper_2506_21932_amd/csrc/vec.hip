// Vector kernels of the outer Krylov iterations (FP64) and precision casts.
// Dot products are deterministic: a fixed grid of partial sums, each a
// wavefront-shuffle then LDS reduction, then one workgroup summing the
// partials in a fixed order.
#include "smg_kernels.h"

namespace smg {

__global__ __launch_bounds__(256) void k_axpy(long n, double a, const double* __restrict__ x, double* __restrict__ y) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = fma(a, x[i], y[i]);
}
__global__ __launch_bounds__(256) void k_xpby(long n, const double* __restrict__ x, double b, double* __restrict__ y) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = fma(b, y[i], x[i]);
}
__global__ __launch_bounds__(256) void k_scale(long n, double s, const double* __restrict__ x, double* __restrict__ y) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = x[i] * s;
}
__global__ __launch_bounds__(256) void k_add(long n, const double* __restrict__ a, const double* __restrict__ b,
                                             double* __restrict__ y) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = a[i] + b[i];
}
__global__ __launch_bounds__(256) void k_d2f(long n, const double* __restrict__ x, float* __restrict__ y) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}
__global__ __launch_bounds__(256) void k_f2d(long n, const float* __restrict__ x, double* __restrict__ y) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}

__device__ inline double block_sum(double v) {
  __shared__ double red[4];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = (red[0] + red[1]) + (red[2] + red[3]);
  return s;
}

__global__ __launch_bounds__(256) void k_dot_partial(long n, const double* __restrict__ x,
                                                     const double* __restrict__ y, double* __restrict__ part) {
  const long chunk = (n + DOT_BLOCKS - 1) / DOT_BLOCKS;
  const long lo = (long)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
  double acc = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += 256) acc = fma(x[i], y[i], acc);
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ __launch_bounds__(256) void k_dot_final(const double* __restrict__ part, double* __restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < DOT_BLOCKS; i += 256) acc += part[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) *out = s;
}

static dim3 g1(long n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_axpy(long n, double a, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, g1(n), dim3(256), 0, st, n, a, x, y);
  return hipGetLastError();
}
hipError_t launch_xpby(long n, const double* x, double b, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_xpby, g1(n), dim3(256), 0, st, n, x, b, y);
  return hipGetLastError();
}
hipError_t launch_scale(long n, double s, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_scale, g1(n), dim3(256), 0, st, n, s, x, y);
  return hipGetLastError();
}
hipError_t launch_dot(long n, const double* x, const double* y, double* partial, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_partial, dim3(DOT_BLOCKS), dim3(256), 0, st, n, x, y, partial);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, (const double*)partial, out);
  return hipGetLastError();
}
hipError_t launch_cast_d2f(long n, const double* x, float* y, hipStream_t st) {
  hipLaunchKernelGGL(k_d2f, g1(n), dim3(256), 0, st, n, x, y);
  return hipGetLastError();
}
hipError_t launch_cast_f2d(long n, const float* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_f2d, g1(n), dim3(256), 0, st, n, x, y);
  return hipGetLastError();
}
hipError_t launch_add(long n, const double* a, const double* b, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_add, g1(n), dim3(256), 0, st, n, a, b, y);
  return hipGetLastError();
}

template <class V>
__global__ __launch_bounds__(256) void k_vfma(long n, const V* __restrict__ a, const V* __restrict__ x,
                                              V* __restrict__ y) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = fma(a[i], x[i], y[i]);
}
template <class V>
hipError_t launch_vfma(long n, const V* a, const V* x, V* y, hipStream_t st) {
  hipLaunchKernelGGL((k_vfma<V>), g1(n), dim3(256), 0, st, n, a, x, y);
  return hipGetLastError();
}
template hipError_t launch_vfma<double>(long, const double*, const double*, double*, hipStream_t);
template hipError_t launch_vfma<float>(long, const float*, const float*, float*, hipStream_t);

}  // namespace smg
