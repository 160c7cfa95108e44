// Setup-phase kernels: level-0 copy with Dirichlet masking (Sec. 4.1 P1
// zero padding), reciprocal diagonal, 3x3 diagonal-block inverses, ILU(0)
// factorisation on the level's own mask (Sec. 4.2.3, Sec. 4.4 ILU), and
// truncation of FP64 level data to FP32 or FP16 with a per-row FP32 scale.
#include <utility>

#include "smg_group.h"
#include "smg_kernels.h"

namespace smg {

__device__ inline void unflat3(unsigned i, int ny, int nz, int& x, int& y, int& z) {
  unsigned nyz = (unsigned)ny * (unsigned)nz;
  x = (int)(i / nyz);
  unsigned r = i - (unsigned)x * nyz;
  y = (int)(r / (unsigned)nz);
  z = (int)(r - (unsigned)y * (unsigned)nz);
}

// dst[s*be+e][i] = src[...] for in-grid couplings, 0 otherwise.
template <int PAT>
__global__ __launch_bounds__(256) void k_copy_masked(Grid g, int be, const double* __restrict__ src,
                                                     double* __restrict__ dst) {
  const unsigned N = (unsigned)g.N();
  const unsigned i = blockIdx.x * 256u + threadIdx.x;
  if (i >= N) return;
  int X, Y, Z;
  unflat3(i, g.ny, g.nz, X, Y, Z);
#pragma unroll
  for (int s = 0; s < PAT; ++s) {
    const bool in = in_grid(g, X + pat_off(PAT, s, 0), Y + pat_off(PAT, s, 1), Z + pat_off(PAT, s, 2));
    for (int e = 0; e < be; ++e) {
      const long k = ((long)s * be + e) * N + i;
      dst[k] = in ? src[k] : 0.0;
    }
  }
}

hipError_t launch_copy_masked(int pat, const Grid& g, int be, const double* src, double* dst, hipStream_t st) {
  const unsigned N = (unsigned)g.N();
  dim3 grid((N + 255) / 256), blk(256);
  if (pat == 7)
    hipLaunchKernelGGL((k_copy_masked<7>), grid, blk, 0, st, g, be, src, dst);
  else if (pat == 19)
    hipLaunchKernelGGL((k_copy_masked<19>), grid, blk, 0, st, g, be, src, dst);
  else if (pat == 27)
    hipLaunchKernelGGL((k_copy_masked<27>), grid, blk, 0, st, g, be, src, dst);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// rd_i = 1 / a_ii (IEEE division); a zero diagonal raises err bit 1.
__global__ __launch_bounds__(256) void k_recip_diag(long N, const double* __restrict__ ac, double w,
                                                    double* __restrict__ rd, unsigned* err) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const double a = ac[i];
  if (a == 0.0) atomicOr(err, 2u);
  rd[i] = w / a;
}

hipError_t launch_recip_diag(int pat, const Grid& g, const double* A, double w, double* rd, unsigned* err,
                             hipStream_t st) {
  const long N = g.N();
  hipLaunchKernelGGL(k_recip_diag, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N, A + (long)(pat / 2) * N,
                     w, rd, err);
  return hipGetLastError();
}

template <class V>
__global__ __launch_bounds__(256) void k_centre_scaled(long N, const double* __restrict__ ac, double q,
                                                       V* __restrict__ qa) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < N) qa[i] = (V)(q * ac[i]);
}

template <class V>
hipError_t launch_centre_scaled(int pat, const Grid& g, const double* A, double q, V* qa, hipStream_t st) {
  const long N = g.N();
  hipLaunchKernelGGL((k_centre_scaled<V>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N,
                     A + (long)(pat / 2) * N, q, qa);
  return hipGetLastError();
}
template hipError_t launch_centre_scaled<double>(int, const Grid&, const double*, double, double*, hipStream_t);
template hipError_t launch_centre_scaled<float>(int, const Grid&, const double*, double, float*, hipStream_t);

// Coupling strength per axis: sums of |a| over the two face offsets of x, y
// and z whose neighbour lies in the grid.  Workgroup b of the fixed grid
// takes every AXIS_BLOCKS-th chunk of 256 points; lane sums are combined in
// a fixed order, so the result does not depend on timing.
__global__ __launch_bounds__(256) void k_axis_coupling(Grid g, const double* __restrict__ A, int sxm, int sxp,
                                                       int sym, int syp, int szm, int szp, double* __restrict__ part) {
  const long N = g.N();
  const long nyz = (long)g.ny * g.nz;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < N; i += (long)AXIS_BLOCKS * 256) {
    const int X = (int)(i / nyz), Y = (int)((i / g.nz) % g.ny), Z = (int)(i % g.nz);
    if (X > 0) sx += fabs(A[(long)sxm * N + i]);
    if (X + 1 < g.nx) sx += fabs(A[(long)sxp * N + i]);
    if (Y > 0) sy += fabs(A[(long)sym * N + i]);
    if (Y + 1 < g.ny) sy += fabs(A[(long)syp * N + i]);
    if (Z > 0) sz += fabs(A[(long)szm * N + i]);
    if (Z + 1 < g.nz) sz += fabs(A[(long)szp * N + i]);
  }
  __shared__ double red[3][256];
  red[0][threadIdx.x] = sx;
  red[1][threadIdx.x] = sy;
  red[2][threadIdx.x] = sz;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 3) part[3 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_axis_coupling(int pat, const Grid& g, const double* A, double* part, hipStream_t st) {
  const int sxm = pat_slot(pat, -1, 0, 0), sxp = pat_slot(pat, 1, 0, 0), sym = pat_slot(pat, 0, -1, 0),
            syp = pat_slot(pat, 0, 1, 0), szm = pat_slot(pat, 0, 0, -1), szp = pat_slot(pat, 0, 0, 1);
  if (sxm < 0 || sxp < 0 || sym < 0 || syp < 0 || szm < 0 || szp < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_axis_coupling, dim3(AXIS_BLOCKS), dim3(256), 0, st, g, A, sxm, sxp, sym, syp, szm, szp, part);
  return hipGetLastError();
}

// Inverse of the centre 3x3 block of each node: Gauss-Jordan with partial
// pivoting on [D | I]; pivot row divided by the pivot, other rows updated
// with fma(-f, pivot_row, row).
__global__ __launch_bounds__(256) void k_block_dinv(long N, const double* __restrict__ Ac, double* __restrict__ Dinv,
                                                    unsigned* err) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  double m[3][6];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      m[r][k] = Ac[(long)(r * 3 + k) * N + i];
      m[r][3 + k] = r == k ? 1.0 : 0.0;
    }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int p = k;
#pragma unroll
    for (int r = k + 1; r < 3; ++r)
      if (fabs(m[r][k]) > fabs(m[p][k])) p = r;
    if (m[p][k] == 0.0) {
      atomicOr(err, 2u);
      return;
    }
    if (p != k) {
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const double t = m[k][j];
        m[k][j] = m[p][j];
        m[p][j] = t;
      }
    }
    const double piv = m[k][k];
#pragma unroll
    for (int j = 0; j < 6; ++j) m[k][j] = m[k][j] / piv;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      if (r == k) continue;
      const double f = m[r][k];
#pragma unroll
      for (int j = 0; j < 6; ++j) m[r][j] = fma(-f, m[k][j], m[r][j]);
    }
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) Dinv[(long)(r * 3 + k) * N + i] = m[r][3 + k];
}

hipError_t launch_block_dinv(const Grid& g, const double* A, double* Dinv, unsigned* err, hipStream_t st) {
  const long N = g.N();
  hipLaunchKernelGGL(k_block_dinv, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N, A + 13L * 9 * N, Dinv,
                     err);
  return hipGetLastError();
}

// Which of a point's 26 neighbours lie in the grid: every offset that the
// elimination of one row touches (its own slots, the rows of its lower
// neighbours and the fill kept on the mask) lies within one step of the point
// on each axis, so six comparisons per point decide them all.
struct IluNb {
  bool xl, xh, yl, yh, zl, zh;  // neighbour at -1 / +1 on x, y, z in the grid
};

template <int DX, int DY, int DZ>
__device__ __forceinline__ bool ilu_nb(const IluNb& b) {
  static_assert(DX >= -1 && DX <= 1 && DY >= -1 && DY <= 1 && DZ >= -1 && DZ <= 1, "offset beyond one step");
  bool r = true;
  if constexpr (DX < 0) r = r & b.xl;
  if constexpr (DX > 0) r = r & b.xh;
  if constexpr (DY < 0) r = r & b.yl;
  if constexpr (DY > 0) r = r & b.yh;
  if constexpr (DZ < 0) r = r & b.zl;
  if constexpr (DZ > 0) r = r & b.zh;
  return r;
}

// Flat index offset of the neighbour at (dx, dy, dz).
__device__ __forceinline__ long ilu_flat(const Grid& g, int dx, int dy, int dz) {
  return ((long)dx * g.ny + dy) * g.nz + dz;
}

// Compile-time unrolled elimination of one ILU(0) row (all slot indices are
// constants): for lower slot S (canonical order) of the row, with the row k
// of that neighbour: w[S] /= U_C[k], then for each upper slot T of row k in
// canonical order whose combined offset lies in the mask and in the grid,
// w[slot] = fma(-w[S], U_T[k], w[slot]).
// The elimination runs in two phases: every pivot and coupling it uses is
// loaded first (ilu_load), then the arithmetic runs on registers (ilu_elim),
// so all loads of the row are in flight together.  Fill outside the mask is
// dropped at compile time; every other update is performed, with the pivot 1
// and the coupling 0 where the neighbour row or the coupled point lies
// outside the grid; those constants are read from
// one = U[PAT*N+1] and zero = U[PAT*N] through a selected address (a select
// of a loaded value instead lets the compiler move the load into a branch
// that waits for it alone).  An address is a per-launch constant
// (U + T*N + the neighbour's flat offset) plus the point's index i.
template <int PAT>
struct IluRowVals {
  double ud[PAT / 2];               // pivot U_C of lower neighbour S
  double uf[PAT / 2][PAT / 2];      // coupling U_T of lower neighbour S, T = C + 1 + t
};

// combined offset of lower slot S and upper slot T: its slot in the mask, or
// -1 if the fill is dropped
template <int PAT, int S, int T>
__host__ __device__ constexpr int ilu_fill_slot() {
  constexpr int dx = pat_off(PAT, S, 0) + pat_off(PAT, T, 0), dy = pat_off(PAT, S, 1) + pat_off(PAT, T, 1),
                dz = pat_off(PAT, S, 2) + pat_off(PAT, T, 2);
  if constexpr (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1)
    return pat_slot(PAT, dx, dy, dz);
  else
    return -1;
}

template <int PAT, int S, int T>
__device__ __forceinline__ void ilu_load_fill(IluRowVals<PAT>& v, const double* __restrict__ U, const double* zero,
                                              long N, long koff, long i, bool vs, const IluNb& nb) {
  constexpr int sl = ilu_fill_slot<PAT, S, T>();
  if constexpr (sl >= 0) {
    constexpr int dx = pat_off(PAT, sl, 0), dy = pat_off(PAT, sl, 1), dz = pat_off(PAT, sl, 2);
    const bool in = vs & ilu_nb<dx, dy, dz>(nb);
    v.uf[S][T - PAT / 2 - 1] = *(in ? U + ((long)T * N + koff) + i : zero);
  }
}

template <int PAT, int S, int... T>
__device__ __forceinline__ void ilu_load(IluRowVals<PAT>& v, const Grid& g, long i, const IluNb& nb,
                                         const double* __restrict__ U, const double* zero,
                                         std::integer_sequence<int, T...>) {
  constexpr int C = PAT / 2;
  constexpr int ox = pat_off(PAT, S, 0), oy = pat_off(PAT, S, 1), oz = pat_off(PAT, S, 2);
  const long N = g.N();
  const bool vs = ilu_nb<ox, oy, oz>(nb);
  const long koff = ilu_flat(g, ox, oy, oz);
  v.ud[S] = *(vs ? U + ((long)C * N + koff) + i : zero + 1);  // the stored 1 outside the grid
  (ilu_load_fill<PAT, S, C + 1 + T>(v, U, zero, N, koff, i, vs, nb), ...);
}

template <int PAT, int S, int T>
__device__ __forceinline__ void ilu_elim_fill(double (&w)[PAT], const IluRowVals<PAT>& v) {
  constexpr int sl = ilu_fill_slot<PAT, S, T>();
  // unused couplings are the stored zero: w + (-w_S * 0) = w up to the sign
  // of a zero result
  if constexpr (sl >= 0) w[sl] = fma(-w[S], v.uf[S][T - PAT / 2 - 1], w[sl]);
}

template <int PAT, int S, int... T>
__device__ __forceinline__ void ilu_elim(double (&w)[PAT], const IluRowVals<PAT>& v,
                                         std::integer_sequence<int, T...>) {
  w[S] = w[S] / v.ud[S];
  (ilu_elim_fill<PAT, S, PAT / 2 + 1 + T>(w, v), ...);
}

template <int PAT, int... S>
__device__ __forceinline__ void ilu_rows(double (&w)[PAT], const Grid& g, long i, const IluNb& nb,
                                         const double* __restrict__ U, const double* zero,
                                         std::integer_sequence<int, S...>) {
  using Up = std::make_integer_sequence<int, PAT - PAT / 2 - 1>;
  IluRowVals<PAT> v;
  (ilu_load<PAT, S>(v, g, i, nb, U, zero, Up{}), ...);
  (ilu_elim<PAT, S>(w, v, Up{}), ...);
}

// ILU(0) rows on one hyperplane wx*x + wy*y + z = tau (all their lower
// neighbours lie on earlier hyperplanes).  Doolittle IKJ on the mask:
// lower slots in canonical (= ascending column) order, w[s] /= U_c[k], then
// w[slot(off_s+off_t)] = fma(-w[s], U_t[k], w[...]) for the upper slots t of
// row k in canonical order, dropping fill outside the mask.
// Threads cover only the points that can meet the hyperplane: the x range
// [x0, x0 + nxr) where it crosses the grid, and for each x the kb = nz / wy + 2
// largest y with z = tau - wx*x - wy*y >= 0.  The rows of one hyperplane are
// scattered in memory (every load of a wave touches 64 lines), so the launch
// uses one-wave workgroups to spread them over all compute units.
__host__ __device__ constexpr int ilu_band(int nz, int wy) { return nz / wy + 2; }
constexpr int ILU_WG = 64;

// x range [x0, x0 + nxr) of the points on hyperplane tau (nxr <= 0: none)
__host__ __device__ inline void ilu_xrange(const Grid& g, int wx, int wy, int tau, int* x0, int* nxr) {
  // wx*x <= tau and wx*x >= tau - wy*(ny-1) - (nz-1)
  const int lo = tau - wy * (g.ny - 1) - (g.nz - 1);
  *x0 = lo <= 0 ? 0 : (lo + wx - 1) / wx;
  const int x1 = tau / wx < g.nx - 1 ? tau / wx : g.nx - 1;
  *nxr = x1 - *x0 + 1;
}

// Point of band thread t of hyperplane tau (x range starting at x0, nxr
// columns); false if the thread has none.
template <int WX, int WY>
__device__ __forceinline__ bool ilu_point(const Grid& g, int tau, int x0, int nxr, int kb, int t, int& X, int& Y,
                                          int& Z) {
  if (t < 0 || t >= nxr * kb) return false;
  X = x0 + t / kb;
  if (X >= g.nx) return false;
  const int rem = tau - WX * X;
  if (rem < 0) return false;
  Y = rem / WY - t % kb;
  if (Y < 0 || Y >= g.ny) return false;
  Z = rem - WY * Y;
  return Z >= 0 && Z < g.nz;
}

// Row i of A on the factor mask PAT: A's coefficient of the same offset in
// its own pattern PA where there is one and the neighbour is in the grid,
// else 0 (a mask larger than A's pattern keeps fill there, a smaller one
// drops A's other entries).  Outside the grid the slot reads the stored zero
// through a selected address: a select of the loaded value instead lets the
// compiler move each load into a branch that waits for it alone, one memory
// round trip per slot.
template <int PAT, int PA, int S>
__device__ __forceinline__ void ilu_init(double (&w)[PAT], const double* __restrict__ A, const double* zero, long N,
                                         long i, const IluNb& nb) {
  constexpr int dx = pat_off(PAT, S, 0), dy = pat_off(PAT, S, 1), dz = pat_off(PAT, S, 2);
  constexpr int sa = pat_slot(PA, dx, dy, dz);
  if constexpr (sa >= 0) {
    w[S] = *(ilu_nb<dx, dy, dz>(nb) ? A + (long)sa * N + i : zero);
  } else {
    w[S] = 0.0;
  }
}

template <int PAT, int PA, int... S>
__device__ __forceinline__ void ilu_init_row(double (&w)[PAT], const double* __restrict__ A, const double* zero,
                                             long N, long i, const IluNb& nb, std::integer_sequence<int, S...>) {
  (ilu_init<PAT, PA, S>(w, A, zero, N, i, nb), ...);
}

// PAT: the factor mask (its hyperplanes order the rows); PA: A's pattern.
template <int PAT, int PA>
__global__ __launch_bounds__(ILU_WG) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_ilu0_plane(Grid g, int tau, int x0, int nxr,
                                                       const double* __restrict__ A, double* __restrict__ L,
                                                       double* __restrict__ U, double* __restrict__ rU,
                                                       unsigned* err) {
  constexpr int C = PAT / 2, WX = hp_wx(PAT), WY = hp_wy(PAT);
  const long N = g.N();
  const int kb = ilu_band(g.nz, WY);
  int X, Y, Z;
  // neighbouring band slots read overlapping U lines: keep them on one XCD
  const unsigned slot = xcd_block(blockIdx.x, gridDim.x) * (unsigned)ILU_WG + threadIdx.x;
  if (!ilu_point<WX, WY>(g, tau, x0, nxr, kb, (int)slot, X, Y, Z)) return;
  const long i = ((long)X * g.ny + Y) * g.nz + Z;
  const IluNb nb{X > 0, X < g.nx - 1, Y > 0, Y < g.ny - 1, Z > 0, Z < g.nz - 1};
  const double* zero = U + (long)PAT * N;  // U[PAT*N] = 0, U[PAT*N+1] = 1
  double w[PAT];
  ilu_init_row<PAT, PA>(w, A, zero, N, i, nb, std::make_integer_sequence<int, PAT>{});
  ilu_rows<PAT>(w, g, i, nb, U, zero, std::make_integer_sequence<int, C>{});
#pragma unroll
  for (int s = 0; s < PAT; ++s) {
    L[(long)s * N + i] = s < C ? w[s] : 0.0;
    U[(long)s * N + i] = s >= C ? w[s] : 0.0;
  }
  if (w[C] == 0.0) atomicOr(err, 2u);
  rU[i] = 1.0 / w[C];
}

// The factorisation of a small level in one workgroup: hyperplane after
// hyperplane, its band slots dealt to the workgroup's threads, one barrier
// between hyperplanes (which makes the rows just stored visible to every
// thread of the workgroup).  Each row takes the operations of k_ilu0_plane
// in the same order.
constexpr int ILU_WG1 = 256;

template <int PAT, int PA>
__global__ __launch_bounds__(ILU_WG1) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_ilu0_small(
    Grid g, const double* __restrict__ A, double* __restrict__ L, double* __restrict__ U, double* __restrict__ rU,
    unsigned* err) {
  constexpr int C = PAT / 2, WX = hp_wx(PAT), WY = hp_wy(PAT);
  const long N = g.N();
  const int kb = ilu_band(g.nz, WY);
  const int D = WX * (g.nx - 1) + WY * (g.ny - 1) + g.nz;
  const double* zero = U + (long)PAT * N;
  for (int tau = 0; tau < D; ++tau) {
    int x0, nxr;
    ilu_xrange(g, WX, WY, tau, &x0, &nxr);
    for (int slot = threadIdx.x; slot < nxr * kb; slot += ILU_WG1) {
      int X, Y, Z;
      if (!ilu_point<WX, WY>(g, tau, x0, nxr, kb, slot, X, Y, Z)) continue;
      const long i = ((long)X * g.ny + Y) * g.nz + Z;
      const IluNb nb{X > 0, X < g.nx - 1, Y > 0, Y < g.ny - 1, Z > 0, Z < g.nz - 1};
      double w[PAT];
      ilu_init_row<PAT, PA>(w, A, zero, N, i, nb, std::make_integer_sequence<int, PAT>{});
      ilu_rows<PAT>(w, g, i, nb, U, zero, std::make_integer_sequence<int, C>{});
#pragma unroll
      for (int s = 0; s < PAT; ++s) {
        L[(long)s * N + i] = s < C ? w[s] : 0.0;
        U[(long)s * N + i] = s >= C ? w[s] : 0.0;
      }
      if (w[C] == 0.0) atomicOr(err, 2u);
      rU[i] = 1.0 / w[C];
    }
    __syncthreads();
  }
}

template <int PAT, int PA>
static hipError_t launch_ilu0_t(const Grid& g, const double* A, double* L, double* U, double* rU, unsigned* err,
                                hipStream_t st) {
  constexpr int wx = hp_wx(PAT), wy = hp_wy(PAT);
  const int D = wx * (g.nx - 1) + wy * (g.ny - 1) + g.nz;
  const long N = g.N();
  hipError_t e = launch_fill_bits<double>(U + (long)PAT * N, 1, 0.0, st);
  if (e == hipSuccess) e = launch_fill_bits<double>(U + (long)PAT * N + 1, 1, 1.0, st);
  if (e != hipSuccess) return e;
  if (N <= ILU_SMALL_POINTS) {
    hipLaunchKernelGGL((k_ilu0_small<PAT, PA>), dim3(1), dim3(ILU_WG1), 0, st, g, A, L, U, rU, err);
    return hipGetLastError();
  }
  const int kb = ilu_band(g.nz, wy);
  for (int tau = 0; tau < D; ++tau) {
    int x0, nxr;
    ilu_xrange(g, wx, wy, tau, &x0, &nxr);
    if (nxr <= 0) continue;
    const dim3 grid((unsigned)((nxr * kb + ILU_WG - 1) / ILU_WG)), blk(ILU_WG);
    hipLaunchKernelGGL((k_ilu0_plane<PAT, PA>), grid, blk, 0, st, g, tau, x0, nxr, A, L, U, rU, err);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int PAT>
static hipError_t launch_ilu0_m(int pa, const Grid& g, const double* A, double* L, double* U, double* rU,
                                unsigned* err, hipStream_t st) {
  if (pa == 7) return launch_ilu0_t<PAT, 7>(g, A, L, U, rU, err, st);
  if (pa == 19) return launch_ilu0_t<PAT, 19>(g, A, L, U, rU, err, st);
  if (pa == 27) return launch_ilu0_t<PAT, 27>(g, A, L, U, rU, err, st);
  return hipErrorInvalidValue;
}

hipError_t launch_ilu0_factor(int pa, int pm, const Grid& g, const double* A, double* L, double* U, double* rU,
                              unsigned* err, hipStream_t st) {
  if (pm == 7) return launch_ilu0_m<7>(pa, g, A, L, U, rU, err, st);
  if (pm == 19) return launch_ilu0_m<19>(pa, g, A, L, U, rU, err, st);
  if (pm == 27) return launch_ilu0_m<27>(pa, g, A, L, U, rU, err, st);
  return hipErrorInvalidValue;
}

__global__ __launch_bounds__(256) void k_to_f32(const double* __restrict__ s, float* __restrict__ d, long n) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = (float)s[i];
}

hipError_t launch_to_f32(const double* src, float* dst, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

// Per scalar row (node i, block row r): s = float(max |a|), h = half(float(a / s)).
__global__ __launch_bounds__(256) void k_to_f16(const double* __restrict__ A, long N, int S, int bs,
                                                __half* __restrict__ h, float* __restrict__ sc) {
  const long k = (long)blockIdx.x * 256 + threadIdx.x;
  if (k >= N * bs) return;
  const long i = k % N;
  const int r = (int)(k / N);
  const int be = bs * bs;
  double mx = 0.0;
  for (int s = 0; s < S; ++s)
    for (int c = 0; c < bs; ++c) {
      const double v = fabs(A[((long)s * be + r * bs + c) * N + i]);
      if (v > mx) mx = v;
    }
  const float s32 = (float)mx;
  sc[(long)r * N + i] = s32;
  for (int s = 0; s < S; ++s)
    for (int c = 0; c < bs; ++c) {
      const long q = ((long)s * be + r * bs + c) * N + i;
      h[q] = s32 == 0.0f ? __float2half_rn(0.0f) : __float2half_rn((float)(A[q] / (double)s32));
    }
}

hipError_t launch_to_f16_rowscale(const double* A, long N, int S, int bs, __half* h, float* sc, hipStream_t st) {
  const long n = N * bs;
  hipLaunchKernelGGL(k_to_f16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, N, S, bs, h, sc);
  return hipGetLastError();
}

// out = scale * float(h), the value the kernels use for an FP16 coefficient.
__global__ __launch_bounds__(256) void k_dequant(const __half* __restrict__ h, const float* __restrict__ sc, long N,
                                                 int S, int bs, float* __restrict__ out) {
  const long k = (long)blockIdx.x * 256 + threadIdx.x;
  const int be = bs * bs;
  if (k >= (long)S * be * N) return;
  const long i = k % N;
  const int e = (int)((k / N) % be);
  out[k] = sc[(long)(e / bs) * N + i] * __half2float(h[k]);
}

hipError_t launch_dequant_f16(const __half* h, const float* sc, long N, int S, int bs, float* out, hipStream_t st) {
  const long n = (long)S * bs * bs * N;
  hipLaunchKernelGGL(k_dequant, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, h, sc, N, S, bs, out);
  return hipGetLastError();
}

template <class V>
__global__ __launch_bounds__(256) void k_fill(V* p, long n, V v) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

template <class V>
hipError_t launch_fill_bits(V* p, long n, V v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill<V>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
template hipError_t launch_fill_bits<double>(double*, long, double, hipStream_t);
template hipError_t launch_fill_bits<float>(float*, long, float, hipStream_t);
template hipError_t launch_fill_bits<unsigned>(unsigned*, long, unsigned, hipStream_t);

}  // namespace smg
