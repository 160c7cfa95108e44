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

__global__ __launch_bounds__(256) void k_dot_partial(long n, const double* __restrict__ x,
                                                     const double* __restrict__ y, double* __restrict__ part,
                                                     const double* gate) {
  if (gate != nullptr && *gate == 0.0) return;
  const long chunk = (n + DOT_BLOCKS - 1) / DOT_BLOCKS;
  const long lo = (long)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
  double acc = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += 256) acc = fma(x[i], y[i], acc);
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ __launch_bounds__(256) void k_dot_final(const double* __restrict__ part, double* __restrict__ out,
                                                   const double* gate) {
  if (gate != nullptr && *gate == 0.0) return;
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
hipError_t launch_dot_gated(long n, const double* x, const double* y, double* partial, double* out,
                            const double* gate, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_partial, dim3(DOT_BLOCKS), dim3(256), 0, st, n, x, y, partial, gate);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, (const double*)partial, out, gate);
  return hipGetLastError();
}
hipError_t launch_dot(long n, const double* x, const double* y, double* partial, double* out, hipStream_t st) {
  return launch_dot_gated(n, x, y, partial, out, nullptr, st);
}

// ---- device-resident PCG scalars: one thread each, the host loop's formulas
__global__ void k_pcg_start(double* s, double bn, int it, int maxit, double rtol) {
  s[PS_BN] = bn;
  s[PS_IT] = it;
  s[PS_MAXIT] = maxit;
  s[PS_RTOL] = rtol;
  s[PS_STATE] = PCG_ITERATING;
  s[PS_GATE] = 0.0;
}
__global__ void k_pcg_alpha(double* s) {
  if (s[PS_STATE] != PCG_ITERATING) return;
  if (s[PS_IT] >= s[PS_MAXIT]) {
    s[PS_STATE] = PCG_LIMIT;
    return;
  }
  const double pq = s[PS_PQ];
  if (!(pq > 0.0)) {
    s[PS_STATE] = PCG_BREAKDOWN;
    return;
  }
  const double alpha = s[PS_RHO] / pq;
  s[PS_ALPHA] = alpha;
  s[PS_NALPHA] = -alpha;
}
__global__ void k_pcg_recur(double* s) {
  if (s[PS_STATE] != PCG_ITERATING) return;
  s[PS_IT] = s[PS_IT] + 1.0;
  const double rel = sqrt(s[PS_RR]) / s[PS_BN];
  s[PS_RECUR] = rel;
  s[PS_REL] = rel;
  if (rel < s[PS_RTOL]) {
    s[PS_STATE] = PCG_CHECK;
    s[PS_GATE] = 1.0;
  }
}
__global__ void k_pcg_true(double* s) {
  if (s[PS_STATE] != PCG_CHECK) return;
  const double rel = sqrt(s[PS_RR]) / s[PS_BN];
  s[PS_REL] = rel;
  s[PS_STATE] = rel < s[PS_RTOL] ? PCG_DONE : PCG_ITERATING;
  s[PS_GATE] = 0.0;
}
__global__ void k_pcg_beta(double* s) {
  if (s[PS_STATE] != PCG_ITERATING) return;
  const double rho1 = s[PS_RZ];
  s[PS_BETA] = rho1 / s[PS_RHO];
  s[PS_RHO] = rho1;
}
__global__ __launch_bounds__(256) void k_xpby_dev(long n, const double* __restrict__ x, const double* __restrict__ b,
                                                  const double* __restrict__ state, double* __restrict__ y) {
  if (*state != PCG_ITERATING) return;
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = fma(*b, y[i], x[i]);
}

// x += alpha p, r -= alpha q (skipped unless the state is ITERATING) and the
// partial sums of r.r in one pass: the element-to-thread mapping and the
// order of the fmas are those of k_dot_partial, so r.r has the same bits as a
// separate dot after the two updates.
__global__ __launch_bounds__(256) void k_pcg_update(long n, const double* __restrict__ s, const double* __restrict__ p,
                                                    const double* __restrict__ q, double* __restrict__ x,
                                                    double* __restrict__ r, double* __restrict__ part) {
  const bool upd = s[PS_STATE] == PCG_ITERATING;
  const double a = s[PS_ALPHA], na = s[PS_NALPHA];
  const long chunk = (n + DOT_BLOCKS - 1) / DOT_BLOCKS;
  const long lo = (long)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
  double acc = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += 256) {
    double ri = r[i];
    if (upd) {
      x[i] = fma(a, p[i], x[i]);
      ri = fma(na, q[i], ri);
      r[i] = ri;
    }
    acc = fma(ri, ri, acc);
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

hipError_t launch_pcg_update(long n, const double* s, const double* p, const double* q, double* x, double* r,
                             double* partial, double* rr, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_update, dim3(DOT_BLOCKS), dim3(256), 0, st, n, s, p, q, x, r, partial);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, (const double*)partial, rr, (const double*)nullptr);
  return hipGetLastError();
}

hipError_t launch_pcg_start(double* s, double bn, int it, int maxit, double rtol, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_start, dim3(1), dim3(1), 0, st, s, bn, it, maxit, rtol);
  return hipGetLastError();
}
hipError_t launch_pcg_alpha(double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(1), 0, st, s);
  return hipGetLastError();
}
hipError_t launch_pcg_recur(double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_recur, dim3(1), dim3(1), 0, st, s);
  return hipGetLastError();
}
hipError_t launch_pcg_true(double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_true, dim3(1), dim3(1), 0, st, s);
  return hipGetLastError();
}
hipError_t launch_pcg_beta(double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(1), 0, st, s);
  return hipGetLastError();
}
hipError_t launch_xpby_dev(long n, const double* x, const double* b, const double* state, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_xpby_dev, g1(n), dim3(256), 0, st, n, x, b, state, y);
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
