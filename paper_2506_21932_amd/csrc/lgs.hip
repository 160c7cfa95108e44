// Line Gauss-Seidel over z-columns (Sec. 4.4, "For LGS" paragraph): the
// unknowns of one column (x, y) are updated together.  The right-hand side of
// a column is assembled from the neighbouring columns, then the column's
// tridiagonal system (couplings (0,0,-1), centre, (0,0,+1)) is solved by the
// Thomas algorithm.  Columns are visited in lexicographic (x, y) order
// (forward) or in reverse (backward), as in the GS formulas with the column
// blocks as D.
//
// Setup: k_tri_factor forms the Thomas pivots once per hierarchy (FP64, one
// thread per column): p_0 = b_0, p_z = fma(-a_z, cp_{z-1}, b_z),
// rden_z = 1/p_z, cp_z = c_z * rden_z.
//
// Sweep (k_lgs): a column depends only on columns whose (x, y) come earlier
// in the visiting order and are stencil neighbours (the projected 2D pattern:
// 2d5 for 3d7, 2d9 for 3d19 / 3d27).  In the sheared coordinates
// (x, y' = y + sh*x), sh = 0 for 3d7 and 1 otherwise (the neighbour
// (x-1, y+1) must come first), every such neighbour lies at (dx, dy') with
// dx <= 0, dy' <= 0 and dx + dy' <= -1.  The columns are cut into K x K tiles
// in (x, y'); a tile depends only on the tiles (bx-1, by'), (bx-1, by'-1) and
// (bx, by'-1), so tiles listed by diagonal bx + by' (setup-time table, empty
// tiles left out) are in dependence order.  Persistent workgroups take tiles
// by atomic ticket (every tile's producers hold smaller tickets and are
// already running: the grid always makes progress) and walk a tile's local
// hyperplanes lx + ly' = k, at most K columns each (K*nz <= 256 points, one
// per thread, unless a column is longer); every column of this sweep is read
// back device-coherently, a column of another tile after its sentinel has
// gone.  The backward sweep takes the table and the local
// hyperplanes in reverse.
// For each local hyperplane a workgroup
//   A. assembles the right-hand side of its columns, one point per thread:
//      t = f_i; the terms of columns not yet visited (values from before the
//      sweep, plain loads); then the terms of columns of this sweep, whose
//      values are read device-coherently from the output and awaited while
//      they still hold the sentinel; each group in canonical order with fma.
//      Every load of a point is issued before its first wait.  The Thomas
//      factors of the columns are staged in LDS with the sums;
//   B. solves each column in one lane (forward elimination, back
//      substitution), in the oracle's order of operations;
//   C. stores the column device-coherently and, if asked, writes the sentinel
//      into `next` (the buffer the following sweep will fill).  Every reader
//      of `next` at these points is a column this one waited for, so those
//      reads are complete.
// Waits are bounded: after LGS_SPIN_LIMIT polls, bit 0 of err is set and
// every waiting lane gives up.
#include <utility>
#include <vector>

#include "smg_kernels.h"

namespace smg {

namespace {

constexpr int LGS_NT = 256;                 // threads per workgroup
constexpr int LGS_PTS = LGS_NT;             // points per chunk (K * nz), unless nz is larger
constexpr unsigned LGS_SPIN_LIMIT = 1u << 21;

__host__ __device__ constexpr int lgs_cwx(int pat) { return pat == 7 ? 1 : 2; }

// does the column at (dx, dy) come later than the current one in the
// visiting order of direction DIR?
__host__ __device__ constexpr bool lgs_later(int dir, int dx, int dy) {
  return dir > 0 ? (dx > 0 || (dx == 0 && dy > 0)) : (dx < 0 || (dx == 0 && dy < 0));
}

template <class V>
__device__ inline V cload(const V* p) {
  using U = typename VBits<V>::U;
  return VBits<V>::val(__hip_atomic_load(reinterpret_cast<const U*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

template <class V>
__device__ inline void cstore(V* p, V v) {
  using U = typename VBits<V>::U;
  __hip_atomic_store(reinterpret_cast<U*>(p), VBits<V>::bits(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait until *p no longer holds the sentinel.
template <class V>
__device__ inline V await_value(const V* p, V v, unsigned* err) {
  unsigned spins = 0;
  while (VBits<V>::bits(v) == VBits<V>::sent) {
    if (++spins >= LGS_SPIN_LIMIT) {
      atomicOr(err, 1u);
      break;
    }
    if ((spins & 1023u) == 1023u && (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1u)) break;
    __builtin_amdgcn_s_sleep(2);
    v = cload(p);
  }
  return v;
}

// Loads of the term of slot S (off-column slots only), issued for all slots
// before any wait: in-grid flag, coefficient, and the neighbour's value (from
// before the sweep for a column later in the order, else device-coherently
// from the output).  A neighbour outside the grid loads the row's own
// position instead; its term is not used.
template <int PAT, int DIR, bool ZG, int S, class V>
__device__ __forceinline__ void lgs_load(bool (&in)[PAT], V (&av)[PAT], V (&uv)[PAT], const LgsArgs<V>& a, long N,
                                         long i, int X, int Y, int Z) {
  constexpr int dx = pat_off(PAT, S, 0), dy = pat_off(PAT, S, 1), dz = pat_off(PAT, S, 2);
  if constexpr (!(dx == 0 && dy == 0) && !(ZG && lgs_later(DIR, dx, dy))) {
    in[S] = in_grid(a.g, X + dx, Y + dy, Z + dz);
    const long j = in[S] ? i + dx * ((long)a.g.ny * a.g.nz) + dy * (long)a.g.nz + dz : i;
    av[S] = a.A[(long)S * N + i];
    if constexpr (lgs_later(DIR, dx, dy))
      uv[S] = a.uold[j];
    else
      uv[S] = cload(a.x + j);
  }
}

// Bounded wait for the value of a column of this sweep that is still the
// sentinel.
template <int PAT, int DIR, int S, class V>
__device__ __forceinline__ void lgs_wait(const bool (&in)[PAT], V (&uv)[PAT], const LgsArgs<V>& a, long i) {
  constexpr int dx = pat_off(PAT, S, 0), dy = pat_off(PAT, S, 1), dz = pat_off(PAT, S, 2);
  if constexpr (!(dx == 0 && dy == 0) && !lgs_later(DIR, dx, dy)) {
    if (in[S] && VBits<V>::bits(uv[S]) == VBits<V>::sent)
      uv[S] = await_value(a.x + i + dx * ((long)a.g.ny * a.g.nz) + dy * (long)a.g.nz + dz, uv[S], a.err);
  }
}

// t = fma(-a_s, u_nbr, t) for slot S if it belongs to the group (OLD: columns
// later in the order) and its neighbour is in the grid.
template <int PAT, int DIR, bool OLD, int S, class V>
__device__ __forceinline__ void lgs_acc(V& t, const bool (&in)[PAT], const V (&av)[PAT], const V (&uv)[PAT]) {
  constexpr int dx = pat_off(PAT, S, 0), dy = pat_off(PAT, S, 1);
  if constexpr (!(dx == 0 && dy == 0) && lgs_later(DIR, dx, dy) == OLD) t = in[S] ? fma(-av[S], uv[S], t) : t;
}

// Right-hand side of point i: f_i, then the group of columns not yet visited
// (omitted for the zero initial guess), then the columns of this sweep, each
// in canonical order.
template <int PAT, int DIR, bool ZG, class V, int... S>
__device__ __forceinline__ V lgs_rhs(const LgsArgs<V>& a, long N, long i, int X, int Y, int Z,
                                     std::integer_sequence<int, S...>) {
  bool in[PAT];
  V av[PAT], uv[PAT];
  V t = a.f[i];
  (lgs_load<PAT, DIR, ZG, S, V>(in, av, uv, a, N, i, X, Y, Z), ...);
  if constexpr (!ZG) (lgs_acc<PAT, DIR, true, S, V>(t, in, av, uv), ...);
  (lgs_wait<PAT, DIR, S, V>(in, uv, a, i), ...);
  (lgs_acc<PAT, DIR, false, S, V>(t, in, av, uv), ...);
  return t;
}

__device__ inline unsigned lgs_take_ticket(unsigned* ctr) {
  __shared__ unsigned s_ticket;
  if (threadIdx.x == 0) s_ticket = atomicAdd(&ctr[0], 1u);
  __syncthreads();
  const unsigned t = s_ticket;
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(t);
}

// The last workgroup to finish resets the ticket counters for the next launch.
__device__ inline void lgs_retire(unsigned* ctr) {
  if (threadIdx.x == 0) {
    const unsigned o = atomicAdd(&ctr[1], 1u);
    if (o == gridDim.x - 1) {
      __hip_atomic_store(&ctr[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctr[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <int PAT, int DIR, class V, bool ZG>
__global__ __launch_bounds__(LGS_NT) void k_lgs(LgsArgs<V> a) {
  constexpr int CWX = lgs_cwx(PAT);
  constexpr int SLO = pat_slot(PAT, 0, 0, -1);
  extern __shared__ __align__(16) unsigned char lgs_smem[];
  const Grid g = a.g;
  const long N = g.N();
  const int nz = g.nz, K = a.K, LD = nz + 1;
  V* ld = reinterpret_cast<V*>(lgs_smem);  // right-hand side, then d', then x
  V* la = ld + K * LD;                      // coupling to z-1
  V* lr = la + K * LD;                      // 1 / pivot
  V* lc = lr + K * LD;                      // c / pivot
  const int SH = CWX - 1;
  const int nsteps = 2 * K - 1;
  for (;;) {
    const unsigned ticket = lgs_take_ticket(a.ctr);
    if (ticket >= (unsigned)a.ntile) break;
    const int e = a.tmap[DIR > 0 ? (int)ticket : a.ntile - 1 - (int)ticket];
    const int bx = e >> 16, by = e & 0xffff;
    for (int st = 0; st < nsteps; ++st) {
      const int kh = DIR > 0 ? st : nsteps - 1 - st;  // local hyperplane lx + ly' = kh
      const int lx0 = kh - (K - 1) > 0 ? kh - (K - 1) : 0;
      const int ncol = (kh < K - 1 ? kh : K - 1) - lx0 + 1;  // columns of this hyperplane in the tile
      // column c of the hyperplane: (lx, ly') = (lx0 + c, kh - lx0 - c); it
      // exists if it falls inside the grid
      auto column = [&](int c, int& X, int& Y) {
        X = bx * K + lx0 + c;
        Y = by * K + (kh - lx0 - c) - SH * X;
        return X < g.nx && Y >= 0 && Y < g.ny;
      };
      // A. right-hand sides and staged factors (one point per thread unless
      // the column is longer than a workgroup)
      for (int q = threadIdx.x; q < ncol * nz; q += LGS_NT) {
        const int c = q / nz, Z = q - c * nz;
        int X, Y;
        if (!column(c, X, Y)) continue;
        const long i = ((long)X * g.ny + Y) * nz + Z;
        const int o = c * LD + Z;
        la[o] = Z > 0 ? a.A[(long)SLO * N + i] : V(0);
        lr[o] = a.rden[i];
        lc[o] = a.cp[i];
        ld[o] = lgs_rhs<PAT, DIR, ZG, V>(a, N, i, X, Y, Z, std::make_integer_sequence<int, PAT>{});
      }
      __syncthreads();
      // B. Thomas solve, one lane per column, in blocks of 8 points whose LDS
      // reads are issued together.  d'_0 = t_0 * rden_0 comes out of the same
      // formula: the stored coupling to z-1 at z = 0 is +0 and d' starts at +0,
      // so fma(-0, +0, t_0) = t_0 exactly.
      int cX, cY;
      if ((int)threadIdx.x < ncol && column((int)threadIdx.x, cX, cY)) {
        const int b = (int)threadIdx.x * LD;
        V dp = V(0);
        for (int z0 = 0; z0 < nz; z0 += 8) {
          V a8[8], r8[8], d8[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int z = z0 + k < nz ? z0 + k : nz - 1;
            a8[k] = la[b + z];
            r8[k] = lr[b + z];
            d8[k] = ld[b + z];
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            if (z0 + k < nz) {
              dp = fma(-a8[k], dp, d8[k]) * r8[k];
              ld[b + z0 + k] = dp;
            }
          }
        }
        V xv = dp;
        for (int z1 = nz - 2; z1 >= 0; z1 -= 8) {
          V c8[8], d8[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int z = z1 - k >= 0 ? z1 - k : 0;
            c8[k] = lc[b + z];
            d8[k] = ld[b + z];
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            if (z1 - k >= 0) {
              xv = fma(-c8[k], xv, d8[k]);
              ld[b + z1 - k] = xv;
            }
          }
        }
      }
      __syncthreads();
      // C. results out, sentinels for the next sweep
      for (int q = threadIdx.x; q < ncol * nz; q += LGS_NT) {
        const int c = q / nz, Z = q - c * nz;
        int X, Y;
        if (!column(c, X, Y)) continue;
        const long i = ((long)X * g.ny + Y) * nz + Z;
        cstore(a.x + i, ld[c * LD + Z]);
        if (a.next) a.next[i] = VBits<V>::val(VBits<V>::sent);
      }
      __syncthreads();  // LDS is refilled by the next local hyperplane
    }
  }
  lgs_retire(a.ctr);
}

// Thomas pivots of every z-column (FP64, one thread per column).
__global__ __launch_bounds__(256) void k_tri_factor(Grid g, int slo, int sc, int sup, const double* __restrict__ A,
                                                     double* __restrict__ rden, double* __restrict__ cp,
                                                     unsigned* err) {
  const long col = (long)blockIdx.x * 256 + threadIdx.x;
  if (col >= (long)g.nx * g.ny) return;
  const long N = g.N();
  const long i0 = col * g.nz;
  double cprev = 0.0;
  for (int Z = 0; Z < g.nz; ++Z) {
    const long i = i0 + Z;
    const double az = Z > 0 ? A[(long)slo * N + i] : 0.0;
    const double cz = Z < g.nz - 1 ? A[(long)sup * N + i] : 0.0;
    const double piv = Z == 0 ? A[(long)sc * N + i] : fma(-az, cprev, A[(long)sc * N + i]);
    if (piv == 0.0) atomicOr(err, 2u);
    const double r = 1.0 / piv;
    rden[i] = r;
    cprev = cz * r;
    cp[i] = cprev;
  }
}

template <int PAT, int DIR, class V, bool ZG>
hipError_t launch_lgs_t(const LgsArgs<V>& a, hipStream_t st) {
  const unsigned total = (unsigned)a.ntile;
  const unsigned grid = total < (unsigned)LGS_MAX_GRID ? total : (unsigned)LGS_MAX_GRID;
  const size_t lds = lgs_lds_bytes(a.g, a.K, (int)sizeof(V));
  hipLaunchKernelGGL((k_lgs<PAT, DIR, V, ZG>), dim3(grid), dim3(LGS_NT), lds, st, a);
  return hipGetLastError();
}

template <int PAT, class V>
hipError_t launch_lgs_p(int dir, bool zg, const LgsArgs<V>& a, hipStream_t st) {
  if (dir > 0) return zg ? launch_lgs_t<PAT, 1, V, true>(a, st) : launch_lgs_t<PAT, 1, V, false>(a, st);
  if (zg) return hipErrorInvalidValue;  // the zero-guess sweep is the forward pre-smoother
  return launch_lgs_t<PAT, -1, V, false>(a, st);
}

}  // namespace

int lgs_plan(const Grid& g, int pat, int* K, std::vector<int>* tmap) {
  const int k = g.nz >= LGS_PTS ? 1 : (LGS_PTS / g.nz < 8 ? LGS_PTS / g.nz : 8);
  const int sh = lgs_cwx(pat) - 1;
  const int ntx = (g.nx + k - 1) / k, nty = (g.ny + sh * (g.nx - 1) + k - 1) / k;
  *K = k;
  int n = 0;
  for (int d = 0; d < ntx + nty - 1; ++d)
    for (int bx = 0; bx < ntx; ++bx) {
      const int by = d - bx;
      if (by < 0 || by >= nty) continue;
      // the tile holds a column if some x of it has y = y' - sh*x in [0, ny)
      bool any = false;
      for (int x = bx * k; x < bx * k + k && x < g.nx && !any; ++x) {
        const int y0 = by * k - sh * x, y1 = y0 + k - 1;
        any = y1 >= 0 && y0 < g.ny;
      }
      if (!any) continue;
      if (tmap) tmap->push_back((bx << 16) | by);
      ++n;
    }
  return n;
}

size_t lgs_lds_bytes(const Grid& g, int K, int vbytes) { return (size_t)4 * K * (g.nz + 1) * vbytes; }

hipError_t launch_tri_factor(int pat, const Grid& g, const double* A, double* rden, double* cp, unsigned* err,
                             hipStream_t st) {
  const int slo = pat_slot(pat, 0, 0, -1), sc = pat_slot(pat, 0, 0, 0), sup = pat_slot(pat, 0, 0, 1);
  if (slo < 0 || sc < 0 || sup < 0) return hipErrorInvalidValue;
  const long ncol = (long)g.nx * g.ny;
  hipLaunchKernelGGL(k_tri_factor, dim3((unsigned)((ncol + 255) / 256)), dim3(256), 0, st, g, slo, sc, sup, A, rden,
                     cp, err);
  return hipGetLastError();
}

template <class V>
hipError_t launch_lgs(int pat, int dir, bool zero_guess, const LgsArgs<V>& a, hipStream_t st) {
  if (a.K < 1 || a.ntile < 1 || !a.tmap || a.g.nz > LGS_MAX_NZ || lgs_lds_bytes(a.g, a.K, (int)sizeof(V)) > 65536 ||
      (!zero_guess && a.uold == nullptr))
    return hipErrorInvalidValue;
  if (pat == 7) return launch_lgs_p<7, V>(dir, zero_guess, a, st);
  if (pat == 19) return launch_lgs_p<19, V>(dir, zero_guess, a, st);
  if (pat == 27) return launch_lgs_p<27, V>(dir, zero_guess, a, st);
  return hipErrorInvalidValue;
}

template hipError_t launch_lgs<double>(int, int, bool, const LgsArgs<double>&, hipStream_t);
template hipError_t launch_lgs<float>(int, int, bool, const LgsArgs<float>&, hipStream_t);

}  // namespace smg
