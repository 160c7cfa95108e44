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

// Blocked form of the same steps, B pivot steps per pair of launches.
// k_gj_panel: one workgroup holds the panel's columns k0..k0+B-1 of every row
// in LDS and runs its B steps on them (pivot search, row swap, division of
// the pivot row by the pivot, elimination), keeping each step's pivot row,
// pivot and column of multipliers (column k after the swap).  The panel's
// columns are not read after the panel.  k_gj_trail: column tiles of the
// remaining columns (the rest of the left half and all of the right half),
// held in LDS, go through the same B steps: swap, division of the pivot
// row's entry by the pivot, then a_rj = fma(-m_r, a_kj, a_rj) for the other
// rows, skipped where a_kj is zero.  Every element meets the operations of
// the one-step-per-launch form in the same order, so the inverse has the
// same bits.  A singular pivot sets *info and ends the remaining launches.
// Thread t owns rows t + GJ_THREADS * i, i < R (n <= R * GJ_THREADS).
constexpr int GJ_THREADS = 1024;
constexpr int GJ_BMAX = 32;
constexpr int GJ_TCMAX = 8;
constexpr long GJ_LDS_BYTES = 128 * 1024;
constexpr int GJ_NMAX = 2 * GJ_THREADS;  // larger inverses take one step per pair of launches
                                         // (their panels would be narrower than 8 columns)

template <int R>
__global__ __launch_bounds__(GJ_THREADS) void k_gj_panel(int n, const double* __restrict__ aug, int k0, int B,
                                                         double* __restrict__ F, double* __restrict__ piv,
                                                         int* __restrict__ perm, int* info) {
  extern __shared__ double P[];  // P[c * n + r]: panel column k0 + c of row r
  __shared__ double wv[GJ_THREADS / 64];
  __shared__ int wi[GJ_THREADS / 64];
  __shared__ double qrow[GJ_BMAX], krow[GJ_BMAX];  // the step's scaled pivot row; row k before the swap
  if (*info) return;
  const int ld = 2 * n, tid = threadIdx.x;
  for (long e = tid; e < (long)n * B; e += GJ_THREADS) {
    const int r = (int)(e / B), c = (int)(e % B);
    P[(long)c * n + r] = aug[(long)r * ld + k0 + c];
  }
  __syncthreads();
  for (int c = 0; c < B; ++c) {
    const int k = k0 + c;
    const double* col = P + (long)c * n;
    // largest |a_rk| over rows r >= k, the first of equal ones
    double best = -1.0;
    int bidx = n;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = tid + GJ_THREADS * i;
      if (r >= k && r < n) {
        const double v = fabs(col[r]);
        if (v > best || (v == best && r < bidx)) {
          best = v;
          bidx = r;
        }
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o);
      const int oi = __shfl_xor(bidx, o);
      if (ov > best || (ov == best && oi < bidx)) {
        best = ov;
        bidx = oi;
      }
    }
    if ((tid & 63) == 0) {
      wv[tid >> 6] = best;
      wi[tid >> 6] = bidx;
    }
    __syncthreads();
    // every thread reduces the wave results (read only until the next barrier)
    best = wv[0];
    bidx = wi[0];
    for (int w = 1; w < GJ_THREADS / 64; ++w)
      if (wv[w] > best || (wv[w] == best && wi[w] < bidx)) {
        best = wv[w];
        bidx = wi[w];
      }
    if (best == 0.0 || bidx >= n) {
      if (tid == 0) atomicOr(info, 1);
      return;
    }
    const int p = bidx;
    const double pv = col[p];  // the pivot: row p's entry, row k after the swap
    if (tid == 0) {
      perm[c] = p;
      piv[c] = pv;
    }
    // multipliers: column k after the swap
    double m[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = tid + GJ_THREADS * i;
      m[i] = r < n ? (r == k ? pv : (r == p ? col[k] : col[r])) : 0.0;
      if (r < n) F[(long)c * n + r] = m[i];
    }
    if (tid >= c + 1 && tid < B) {
      krow[tid] = P[(long)tid * n + k];
      qrow[tid] = P[(long)tid * n + p] / pv;
    }
    __syncthreads();
    // row k takes the scaled pivot row, row p the old row k, and every row
    // other than k is eliminated (columns after c; column c is not read again)
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = tid + GJ_THREADS * i;
      if (r >= n) continue;
      if (r == k) {
        for (int cc = c + 1; cc < B; ++cc) P[(long)cc * n + k] = qrow[cc];
        continue;
      }
      for (int cc = c + 1; cc < B; ++cc) {
        const double q = qrow[cc];
        const double a = r == p ? krow[cc] : P[(long)cc * n + r];
        P[(long)cc * n + r] = q != 0.0 ? fma(-m[i], q, a) : a;
      }
    }
    __syncthreads();
  }
}

template <int R>
__global__ __launch_bounds__(GJ_THREADS) void k_gj_trail(int n, double* __restrict__ aug, int k0, int B, int j0,
                                                         int tc_max, const double* __restrict__ F,
                                                         const double* __restrict__ piv,
                                                         const int* __restrict__ perm, const int* info) {
  extern __shared__ double T[];  // T[cc * (n + 1) + r]: tile column cc of row r
  __shared__ double pk[GJ_TCMAX], spiv[GJ_BMAX];
  __shared__ int sperm[GJ_BMAX];
  if (*info) return;
  const int ld = 2 * n, tid = threadIdx.x, np = n + 1;
  const int ja = j0 + (int)blockIdx.x * tc_max;
  const int tc = ld - ja < tc_max ? ld - ja : tc_max;
  if (tid < B) {
    spiv[tid] = piv[tid];
    sperm[tid] = perm[tid];
  }
  for (long e = tid; e < (long)n * tc; e += GJ_THREADS) {
    const int r = (int)(e / tc), cc = (int)(e % tc);
    T[(long)cc * np + r] = aug[(long)r * ld + ja + cc];
  }
  double m[R];  // the multipliers of the current step for the owned rows
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int r = tid + GJ_THREADS * i;
    m[i] = r < n ? F[r] : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < B; ++c) {
    const int k = k0 + c;
    if (tid < tc) {
      const int p = sperm[c];
      double a = T[(long)tid * np + k];
      if (p != k) {
        const double b = T[(long)tid * np + p];
        T[(long)tid * np + p] = a;
        a = b;
      }
      a = a / spiv[c];
      T[(long)tid * np + k] = a;
      pk[tid] = a;
    }
    // the next step's multipliers load while this step computes
    double mn[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = tid + GJ_THREADS * i;
      mn[i] = (r < n && c + 1 < B) ? F[(long)(c + 1) * n + r] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int r = tid + GJ_THREADS * i;
      if (r >= n || r == k) continue;
      for (int cc = 0; cc < tc; ++cc) {
        const double q = pk[cc];
        if (q != 0.0) T[(long)cc * np + r] = fma(-m[i], q, T[(long)cc * np + r]);
      }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) m[i] = mn[i];
    __syncthreads();
  }
  for (long e = tid; e < (long)n * tc; e += GJ_THREADS) {
    const int r = (int)(e / tc), cc = (int)(e % tc);
    aug[(long)r * ld + ja + cc] = T[(long)cc * np + r];
  }
}

template <int R>
static hipError_t gj_blocked(int n, double* aug, int* info_dev, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gj_panel<R>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)GJ_LDS_BYTES);
    if (e == hipSuccess)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gj_trail<R>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)GJ_LDS_BYTES);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const long bl = GJ_LDS_BYTES / 8 / n, tl = GJ_LDS_BYTES / 8 / (n + 1);
  const int B = (int)(bl < GJ_BMAX ? bl : GJ_BMAX), TC = (int)(tl < GJ_TCMAX ? tl : GJ_TCMAX);
  double* F = aug + (long)n * 2 * n;
  double* piv = F + (long)n * GJ_BMAX;
  int* perm = reinterpret_cast<int*>(piv + GJ_BMAX);
  for (int k0 = 0; k0 < n; k0 += B) {
    const int Bp = n - k0 < B ? n - k0 : B;
    hipLaunchKernelGGL(k_gj_panel<R>, dim3(1), dim3(GJ_THREADS), (size_t)n * Bp * 8, st, n, (const double*)aug, k0,
                       Bp, F, piv, perm, info_dev);
    const int j0 = k0 + Bp, tiles = (2 * n - j0 + TC - 1) / TC;
    hipLaunchKernelGGL(k_gj_trail<R>, dim3((unsigned)tiles), dim3(GJ_THREADS), (size_t)TC * (n + 1) * 8, st, n, aug,
                       k0, Bp, j0, TC, (const double*)F, (const double*)piv, (const int*)perm,
                       (const int*)info_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

long coarse_invert_extra(int n) { return (long)n * GJ_BMAX + 2L * GJ_BMAX; }

hipError_t coarse_invert(int n, double* aug, int* info_dev, hipStream_t st) {
  if (n <= GJ_THREADS) return gj_blocked<1>(n, aug, info_dev, st);
  if (n <= GJ_NMAX) return gj_blocked<2>(n, aug, info_dev, st);
  double* fac = aug + (long)n * 2 * n;
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
