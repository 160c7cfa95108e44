// Coarsest level: dense FP64 operator assembled from the 27-point SG-DIA
// level, explicit inverse by Gauss-Jordan elimination with partial pivoting
// at setup, and an FP64 matrix-vector product per V-cycle (the paper leaves
// the coarsest solver unspecified; an exact solve is used).
#include "smg_group.h"
#include "smg_kernels.h"

namespace smg {

// M (row-major, leading dimension ld) = dense form of an operator of pattern
// pat (the finest pattern when the hierarchy has one level, else 27) with bs
// unknowns per node; M must be zeroed beforehand.
__global__ __launch_bounds__(256) void k_dense_assemble(Grid g, int pat, int bs, const double* __restrict__ A,
                                                        double* __restrict__ M, int ld) {
  const long N = g.N();
  const long k = (long)blockIdx.x * 256 + threadIdx.x;
  const int be = bs * bs;
  if (k >= N * pat * be) return;
  const long i = k % N;
  const int se = (int)(k / N);
  const int s = se / be, e = se % be;
  const int X = (int)(i / ((long)g.ny * g.nz)), Y = (int)((i / g.nz) % g.ny), Z = (int)(i % g.nz);
  const int ax = X + pat_off(pat, s, 0), ay = Y + pat_off(pat, s, 1), az = Z + pat_off(pat, s, 2);
  if (!in_grid(g, ax, ay, az)) return;
  const long j = ((long)ax * g.ny + ay) * g.nz + az;
  const int r = e / bs, c = e % bs;
  M[(i * bs + r) * ld + j * bs + c] = A[(long)se * N + i];
}

hipError_t launch_dense_assemble(const Grid& g, int pat, int bs, const double* A, double* M, int ld,
                                 hipStream_t st) {
  const long n = g.N() * pat * bs * bs;
  hipLaunchKernelGGL(k_dense_assemble, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, pat, bs, A, M, ld);
  return hipGetLastError();
}

// Pivot step k of Gauss-Jordan on aug = [A | I] (n x 2n, row-major): find the
// row of largest |a_rk| (first on ties), swap it into row k, keep the column
// of multipliers in fac, and scale row k by 1/pivot.
__global__ __launch_bounds__(256) void k_gj_pivot(int n, double* __restrict__ aug, int k, double* __restrict__ fac,
                                                  int* info) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const int ld = 2 * n;
  double best = -1.0;
  int bidx = n;
  for (int r = k + threadIdx.x; r < n; r += 256) {
    const double v = fabs(aug[(long)r * ld + k]);
    if (v > best || (v == best && r < bidx)) {
      best = v;
      bidx = r;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double ov = bv[threadIdx.x + w];
      const int oi = bi[threadIdx.x + w];
      if (ov > bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = ov;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const int p = bi[0];
  if (bv[0] == 0.0 || p >= n) {
    if (threadIdx.x == 0) atomicOr(info, 1);
    return;
  }
  if (p != k)
    for (int j = threadIdx.x; j < ld; j += 256) {
      const double t = aug[(long)k * ld + j];
      aug[(long)k * ld + j] = aug[(long)p * ld + j];
      aug[(long)p * ld + j] = t;
    }
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += 256) fac[r] = aug[(long)r * ld + k];
  __syncthreads();
  const double piv = fac[k];
  for (int j = threadIdx.x; j < ld; j += 256) aug[(long)k * ld + j] = aug[(long)k * ld + j] / piv;
}

// Eliminate column k from every other row: a_rj = fma(-fac_r, a_kj, a_rj).
__global__ __launch_bounds__(256) void k_gj_elim(int n, double* __restrict__ aug, int k,
                                                 const double* __restrict__ fac) {
  const int ld = 2 * n;
  const int w = ld - k;
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long)n * w) return;
  const int r = (int)(t / w), j = k + (int)(t % w);
  if (r == k) return;
  // zero entries of the pivot row (most of the right half while k is small)
  // leave the column unchanged (up to the sign of a zero): skip their traffic
  const double pk = aug[(long)k * ld + j];
  if (pk == 0.0) return;
  aug[(long)r * ld + j] = fma(-fac[r], pk, aug[(long)r * ld + j]);
}

hipError_t coarse_invert(int n, double* aug, int* info_dev, hipStream_t st) {
  double* fac = aug + (long)n * 2 * n;  // n extra doubles after the augmented matrix
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, st, n, aug, k, fac, info_dev);
    const long work = (long)n * (2 * n - k);
    hipLaunchKernelGGL(k_gj_elim, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, st, n, aug, k,
                       (const double*)fac);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// u = Ainv f in FP64 (input/output in the V-cycle precision); one wavefront
// per row, lanes strided over columns, then a fixed-order lane reduction.
template <class V>
struct GemvOp {
  using Args = GemvArgs<V>;
  __device__ static void run(const Args& a, unsigned bid) {
    const int row = (int)bid * 4 + (int)(threadIdx.x / 64);
    const int lane = threadIdx.x % 64;
    if (row >= a.n) return;
    const double* __restrict__ Ainv = a.ainv;
    const V* __restrict__ f = a.f;
    double acc = 0.0;
    for (int j = lane; j < a.n; j += 64) acc = fma(Ainv[(long)row * a.ld + j], (double)f[j], acc);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) a.u[row] = (V)acc;
  }
};

unsigned gemv_blocks(int n) { return (unsigned)((n + 3) / 4); }

template <class V>
hipError_t launch_coarse_gemv(int n, const double* Ainv, int ld, const V* f, V* u, hipStream_t st) {
  const GemvArgs<V> a{n, ld, Ainv, f, u, 0};
  hipLaunchKernelGGL((k_one<GemvOp<V>>), dim3(gemv_blocks(n)), dim3(256), 0, st, a);
  return hipGetLastError();
}
template <class V>
hipError_t launch_gemv_group(const GemvArgs<V>* segs, const unsigned* bmap, unsigned nblocks, const int* live,
                             hipStream_t st) {
  if (nblocks == 0) return hipSuccess;
  hipLaunchKernelGGL((k_group<GemvOp<V>>), dim3(nblocks), dim3(256), 0, st, segs, bmap, live);
  return hipGetLastError();
}
template hipError_t launch_gemv_group<double>(const GemvArgs<double>*, const unsigned*, unsigned, const int*,
                                              hipStream_t);
template hipError_t launch_gemv_group<float>(const GemvArgs<float>*, const unsigned*, unsigned, const int*,
                                             hipStream_t);
template hipError_t launch_coarse_gemv<double>(int, const double*, int, const double*, double*, hipStream_t);
template hipError_t launch_coarse_gemv<float>(int, const double*, int, const float*, float*, hipStream_t);

}  // namespace smg

namespace smg {
// aug = [0 | I] (n x 2n) followed by n spare doubles.
__global__ __launch_bounds__(256) void k_aug_init(int n, double* __restrict__ aug) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  const long tot = (long)n * 2 * n + n;
  if (t >= tot) return;
  double v = 0.0;
  if (t < (long)n * 2 * n) {
    const long r = t / (2 * n), c = t % (2 * n);
    if (c == n + r) v = 1.0;
  }
  aug[t] = v;
}
hipError_t launch_aug_init(int n, double* aug, hipStream_t st) {
  const long tot = (long)n * 2 * n + n;
  hipLaunchKernelGGL(k_aug_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, aug);
  return hipGetLastError();
}
}  // namespace smg
