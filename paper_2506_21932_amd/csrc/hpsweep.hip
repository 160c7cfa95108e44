// Gauss-Seidel sweep of a small level in one workgroup, hyperplane by
// hyperplane (Sec. 4.4: the lexicographic dependence graph; a point depends
// only on points of smaller wx*x + wy*y + z).
//
// The tiled wavefront sweep needs at least (tile skew + nz) steps per tile,
// which on a level of a few thousand points is two to three times the number
// of hyperplanes, and its steps are paced by global memory.  Here the whole
// level lives in LDS: the right-hand side and the result in a zero-padded box
// (nx+2)(ny+2)(nz+2), so that out-of-grid neighbours read as zero without a
// test.  Step k handles every point of hyperplane k (one per thread; at most
// 256), reading its neighbours from LDS, with one barrier per step.  The
// coefficients come from a setup-time copy in step order, 16 bytes per load
// (triangle coefficients in canonical order, then the diagonal scaling),
// prefetched HP_P steps ahead.  Per point the arithmetic is that of the tiled
// sweep: t = h_i, t = fma(-c_s, x_nb, t) over the triangle in canonical
// order, x_i = t * d_i.
#include <vector>

#include "smg_kernels.h"

namespace smg {

constexpr int HP_NL = 256;  // threads; also the most points a hyperplane may hold
constexpr int HP_P = 8;     // steps of coefficients prefetched

typedef unsigned hp_u32x4 __attribute__((ext_vector_type(4)));
// entries per 16-byte pack and packs per point
template <class V>
__host__ __device__ constexpr int hp_k() { return 16 / (int)sizeof(V); }
template <class V>
__host__ __device__ constexpr int hp_npk(int pat) { return (pat / 2 + 1 + hp_k<V>() - 1) / hp_k<V>(); }

__host__ __device__ inline int hp_box(const Grid& g) { return (g.nx + 2) * (g.ny + 2) * (g.nz + 2); }
__host__ __device__ inline int hp_boxidx(const Grid& g, int x, int y, int z) {
  return ((x + 1) * (g.ny + 2) + (y + 1)) * (g.nz + 2) + (z + 1);
}

// Schedule of a level: number of hyperplanes (steps), or 0 when the level is
// not handled here (LDS or points per hyperplane too large).  pts (if not
// null) receives [step][slot] box indices of the points, -1 for none.
int hp_plan(const Grid& g, int pat, int vbytes, std::vector<int>* pts) {
  const long N = g.N();
  if (N > 65536 || 2L * hp_box(g) * vbytes > 128 * 1024) return 0;
  const int wx = hp_wx(pat), wy = hp_wy(pat);
  const int H = wx * (g.nx - 1) + wy * (g.ny - 1) + g.nz;
  std::vector<int> cnt(H, 0);
  for (int x = 0; x < g.nx; ++x)
    for (int y = 0; y < g.ny; ++y)
      for (int z = 0; z < g.nz; ++z)
        if (++cnt[wx * x + wy * y + z] > HP_NL) return 0;
  if (pts) {
    pts->assign((size_t)H * HP_NL, -1);
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int x = 0; x < g.nx; ++x)
      for (int y = 0; y < g.ny; ++y)
        for (int z = 0; z < g.nz; ++z) {
          const int h = wx * x + wy * y + z;
          (*pts)[(size_t)h * HP_NL + cnt[h]++] = hp_boxidx(g, x, y, z);
        }
  }
  return H;
}

// Coefficient copy of direction dir in step order (step k is hyperplane k
// forward, nsteps-1-k backward), 16-byte packs per point: element e of pack
// p of slot t of step k at ((k * NPK + p) * 256 + t) * K + e holds entry
// p*K + e of [triangle coefficients in canonical order, diagonal scaling].
// SRC 0: FP64 A / 1/a_ii; 1: the same rounded to FP32; 2: FP16 storage, coefficient = row scale * float(half) formed in
// FP32 and the FP32 diagonal scaling (the values the tiled sweep forms).
template <int PAT, int SRC, class V>
__global__ __launch_bounds__(256) void k_hp_pack(Grid g, int nsteps, int dir, const int* __restrict__ pts,
                                                 const double* __restrict__ A, const double* __restrict__ rd,
                                                 const __half* __restrict__ a16, const float* __restrict__ sc,
                                                 const float* __restrict__ rd32, V* __restrict__ out) {
  constexpr int C = PAT / 2, NT = PAT / 2, NV = NT + 1, K = hp_k<V>(), NPK = hp_npk<V>(PAT);
  const long q = (long)blockIdx.x * 256 + threadIdx.x;
  if (q >= (long)nsteps * HP_NL) return;
  const int k = (int)(q / HP_NL), slot = (int)(q % HP_NL);
  const int hp = dir > 0 ? k : nsteps - 1 - k;
  const int b = pts[(long)hp * HP_NL + slot];
  const long N = g.N();
  long i = -1;
  if (b >= 0) {
    const int bz = g.nz + 2, by = g.ny + 2;
    const int z = b % bz - 1, y = (b / bz) % by - 1, x = b / (bz * by) - 1;
    i = ((long)x * g.ny + y) * g.nz + z;
  }
#pragma unroll
  for (int m = 0; m < NPK * K; ++m) {
    V v = V(0);
    if (i >= 0 && m < NV) {
      const int s = m < NT ? (dir > 0 ? m : C + 1 + m) : C;
      if (SRC == 0) v = (V)(m < NT ? A[(long)s * N + i] : rd[i]);
      if (SRC == 1) v = (V)(float)(m < NT ? A[(long)s * N + i] : rd[i]);
      if (SRC == 2) v = (V)(m < NT ? sc[i] * __half2float(a16[(long)s * N + i]) : rd32[i]);
    }
    out[(((long)k * NPK + m / K) * HP_NL + slot) * K + m % K] = v;
  }
}

template <class V>
__device__ inline V hp_get(const hp_u32x4* pk, int m);
template <>
__device__ inline double hp_get<double>(const hp_u32x4* pk, int m) {
  const hp_u32x4 w = pk[m / 2];
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  return m % 2 == 0 ? __builtin_bit_cast(double, u2{w.x, w.y}) : __builtin_bit_cast(double, u2{w.z, w.w});
}
template <>
__device__ inline float hp_get<float>(const hp_u32x4* pk, int m) {
  return __uint_as_float(pk[m / 4][m % 4]);
}

template <int PAT, int DIR, class V>
__global__ __launch_bounds__(HP_NL) void k_hpsweep(Grid g, int nsteps, const int* __restrict__ pts,
                                                   const V* __restrict__ cf, const V* __restrict__ h,
                                                   V* __restrict__ x) {
  constexpr int C = PAT / 2, NT = PAT / 2, NV = NT + 1;
  extern __shared__ __align__(16) unsigned char hp_dyn[];
  const int box = hp_box(g);
  V* xb = reinterpret_cast<V*>(hp_dyn);
  V* hb = xb + box;
  const int tid = threadIdx.x;
  const int N = (int)g.N();
  for (int k = tid; k < box; k += HP_NL) xb[k] = V(0);
  for (int k = tid; k < N; k += HP_NL) {
    const int z = k % g.nz, y = (k / g.nz) % g.ny, xx = k / (g.nz * g.ny);
    hb[hp_boxidx(g, xx, y, z)] = h[k];
  }
  // neighbour offsets in the box, in the triangle's canonical order
  const int sy = g.nz + 2, sx = (g.ny + 2) * (g.nz + 2);
  int noff[NT];
#pragma unroll
  for (int m = 0; m < NT; ++m) {
    const int so = DIR > 0 ? m : C + 1 + m;
    noff[m] = pat_off(PAT, so, 0) * sx + pat_off(PAT, so, 1) * sy + pat_off(PAT, so, 2);
  }
  constexpr int NPK = hp_npk<V>(PAT);
  const hp_u32x4* cfp = reinterpret_cast<const hp_u32x4*>(cf);
  int pb[HP_P];
  hp_u32x4 pc[HP_P][NPK];
  // branch-free prefetch (steps past the end reload the last step, unused):
  // the loads stay in flight across the following steps
  auto fetch = [&](int k, int j) {
    const int kk = k < nsteps ? k : nsteps - 1;
    const int b = pts[(long)(DIR > 0 ? kk : nsteps - 1 - kk) * HP_NL + tid];
    pb[j] = k < nsteps ? b : -1;
#pragma unroll
    for (int p = 0; p < NPK; ++p) pc[j][p] = cfp[((long)kk * NPK + p) * HP_NL + tid];
  };
#pragma unroll
  for (int j = 0; j < HP_P; ++j) fetch(j, j);
  __syncthreads();
  for (int k0 = 0; k0 < nsteps; k0 += HP_P) {
#pragma unroll
    for (int j = 0; j < HP_P; ++j) {
      const int b = pb[j];
      if (b >= 0) {
        V t = hb[b];
#pragma unroll
        for (int m = 0; m < NT; ++m) t = fma(-hp_get<V>(pc[j], m), xb[b + noff[m]], t);
        xb[b] = t * hp_get<V>(pc[j], NT);
      }
      fetch(k0 + j + HP_P, j);
      __syncthreads();
    }
  }
  for (int k = tid; k < N; k += HP_NL) {
    const int z = k % g.nz, y = (k / g.nz) % g.ny, xx = k / (g.nz * g.ny);
    x[k] = xb[hp_boxidx(g, xx, y, z)];
  }
}

hipError_t launch_hp_pack(int pat, int src, const Grid& g, int nsteps, int dir, const int* pts, const double* A,
                          const double* rd, const __half* a16, const float* sc, const float* rd32, void* out,
                          hipStream_t st) {
  const dim3 grid((unsigned)(((long)nsteps * HP_NL + 255) / 256)), blk(256);
#define SMG_HPP(P)                                                                                               \
  if (pat == P) {                                                                                                \
    if (src == 0)                                                                                                \
      hipLaunchKernelGGL((k_hp_pack<P, 0, double>), grid, blk, 0, st, g, nsteps, dir, pts, A, rd, a16, sc, rd32, \
                         (double*)out);                                                                          \
    else if (src == 1)                                                                                           \
      hipLaunchKernelGGL((k_hp_pack<P, 1, float>), grid, blk, 0, st, g, nsteps, dir, pts, A, rd, a16, sc, rd32,  \
                         (float*)out);                                                                           \
    else                                                                                                         \
      hipLaunchKernelGGL((k_hp_pack<P, 2, float>), grid, blk, 0, st, g, nsteps, dir, pts, A, rd, a16, sc, rd32,  \
                         (float*)out);                                                                           \
    return hipGetLastError();                                                                                    \
  }
  SMG_HPP(7)
  SMG_HPP(19)
  SMG_HPP(27)
#undef SMG_HPP
  return hipErrorInvalidValue;
}

template <int PAT, int DIR, class V>
static hipError_t launch_hp_t(const Grid& g, int nsteps, const int* pts, const V* cf, const V* h, V* x,
                              hipStream_t st) {
  static bool attr = false;
  const size_t lds = 2 * (size_t)hp_box(g) * sizeof(V);
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hpsweep<PAT, DIR, V>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((k_hpsweep<PAT, DIR, V>), dim3(1), dim3(HP_NL), lds, st, g, nsteps, pts, cf, h, x);
  return hipGetLastError();
}

template <class V>
hipError_t launch_hpsweep(int pat, int dir, const Grid& g, int nsteps, const int* pts, const V* cf, const V* h, V* x,
                          hipStream_t st) {
#define SMG_HPS(P)                                                                              \
  if (pat == P) return dir > 0 ? launch_hp_t<P, 1, V>(g, nsteps, pts, cf, h, x, st)             \
                               : launch_hp_t<P, -1, V>(g, nsteps, pts, cf, h, x, st);
  SMG_HPS(7)
  SMG_HPS(19)
  SMG_HPS(27)
#undef SMG_HPS
  return hipErrorInvalidValue;
}
template hipError_t launch_hpsweep<double>(int, int, const Grid&, int, const int*, const double*, const double*,
                                           double*, hipStream_t);
template hipError_t launch_hpsweep<float>(int, int, const Grid&, int, const int*, const float*, const float*, float*,
                                          hipStream_t);

}  // namespace smg
