// Dependence-preserving structured triangular sweep (Sec. 3.4): point
// Gauss-Seidel and the ILU(0) factor solves, computed in exactly the order of
// the sequential lexicographic sweep, so the result equals the serial one.
//
// Row update (T = lower offsets for a forward sweep, upper for a backward one):
//     t = h_i;  for s in T (canonical order): t = fma(-c_s[i], x[i+off_s], t);
//     x_i = t * d_i          (or x_i = t for a unit diagonal)
//
// GPU design (replaces the CPU design of the paper, which projects the grid
// onto x-y columns, runs level-scheduled column tasks and synchronises
// threads point-to-point through a shared counter array):
//  * The z-column is the unit.  A workgroup owns a TX x TY tile of columns,
//    one column per lane: tile (X, Y) holds x in [X*TX, X*TX+TX) and
//    y + sh*(x - X*TX) in [Y*TY, Y*TY+TY) (sheared so that no dependence
//    points from a tile to a later one).
//  * Lane (lx, ly) handles point z at step s = z + skew(lx, ly), with
//    skew = (wx - sh*wy)*lx + wy*ly + PRE and the hyperplane weights
//    (wx, wy, 1) of the pattern; every lower neighbour is then handled at an
//    earlier step.  A forward sweep runs tiles (x-tiles outer) and steps in
//    ascending order; a backward sweep runs the very same tiles and steps in
//    descending order, which orders every upper neighbour first.
//  * The coefficients and the diagonal scaling are read from a copy stored
//    in this schedule order ([tile][step][lane], built at setup), so every
//    step reads them with contiguous, coalesced loads.
//  * Lanes exchange fresh values through an LDS ring of the last 8 steps and
//    one workgroup barrier per step.
//  * Columns owned by other tiles are read from global memory.  The output
//    vector holds a signalling-NaN sentinel at every position that another
//    tile reads; a value is ready when it is no longer the sentinel.  These
//    positions are written and read with device-coherent (agent-scope)
//    atomic stores and loads, so no fences or flag counters are needed.  The
//    sentinels for the next sweep on the same level are written by this
//    sweep into that sweep's output buffer.
//  * Tiles are handed out by an atomic ticket in dependence order, so a
//    persistent grid of any size always makes progress.  Waits are bounded
//    by a watchdog that raises an error flag instead of hanging.
//  * Every lane issues the same loads and stores at every step (inactive
//    lanes use valid dummy addresses), and all per-point inputs are
//    prefetched P steps ahead, so each load is waited for only when used.
#include "smg_common.h"
#include "smg_kernels.h"

namespace smg {

constexpr int WF_HIST = 8;
constexpr unsigned WF_SPIN_LIMIT = 1u << 21;

// Neighbour columns holding lower neighbours (forward-frame offsets); a
// backward sweep uses the negated offsets.
__host__ __device__ constexpr int col_dx(int c) { return c == 3 ? 0 : -1; }
__host__ __device__ constexpr int col_dy(int c) { return c == 3 ? -1 : c - 1; }
__host__ __device__ constexpr bool col_used(int pat, int c) {
  return pat_has(pat, col_dx(c), col_dy(c), -1) || pat_has(pat, col_dx(c), col_dy(c), 0) ||
         pat_has(pat, col_dx(c), col_dy(c), 1);
}
__host__ __device__ constexpr int col_maxdz(int pat, int c) {
  return pat_has(pat, col_dx(c), col_dy(c), 1) ? 1 : 0;
}
__host__ __device__ constexpr int col_of(int dx, int dy) {
  return dx == -1 ? dy + 1 : (dy == -1 ? 3 : -1);
}
// One extra step at both ends of the step range when a neighbour column is
// read one point ahead (dz = +1), so every lane can fill its window first.
__host__ __device__ constexpr int wf_pre(int pat) {
  return (col_used(pat, 0) && col_maxdz(pat, 0)) || (col_used(pat, 1) && col_maxdz(pat, 1)) ||
                 (col_used(pat, 2) && col_maxdz(pat, 2)) || (col_used(pat, 3) && col_maxdz(pat, 3))
             ? 1
             : 0;
}

void wf_tiling(const Grid& g, int pat, WfTiling* t) {
  t->sh = g.ny <= WF_TY ? 0 : 1;
  t->ntx = (g.nx + WF_TX - 1) / WF_TX;
  t->nty = (g.ny + t->sh * (WF_TX - 1) + WF_TY - 1) / WF_TY;
  const int pre = wf_pre(pat);
  t->ns = g.nz + (hp_wx(pat) - t->sh * hp_wy(pat)) * (WF_TX - 1) + hp_wy(pat) * (WF_TY - 1) + 2 * pre;
  t->nsk = (long)t->ntx * t->nty * t->ns * (WF_TX * WF_TY);
}

// Is lane (lx, ly)'s column read by a lane of another tile in a sweep of
// direction dir?
__device__ inline bool wf_exported(int pat, int dir, int lx, int ly, int sh) {
  for (int c = 0; c < 4; ++c) {
    if (!col_used(pat, c)) continue;
    const int cx = dir * col_dx(c), cy = dir * col_dy(c);
    const int qx = lx - cx, qy = ly - cy - sh * cx;
    if (qx < 0 || qx >= WF_TX || qy < 0 || qy >= WF_TY) return true;
  }
  return false;
}

template <class V>
__device__ inline V ld_coherent(const V* p) {
  using U = typename VBits<V>::U;
  U b = __hip_atomic_load(reinterpret_cast<const U*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return VBits<V>::val(b);
}
template <class V>
__device__ inline void st_coherent(V* p, V v) {
  using U = typename VBits<V>::U;
  __hip_atomic_store(reinterpret_cast<U*>(p), VBits<V>::bits(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int PAT, int DIR, int P, class SK, bool UNITD, bool ADD>
__global__ __launch_bounds__(WF_TX* WF_TY) void k_wavefront(WfArgs<typename SK::V> a, SK sk) {
  using V = typename SK::V;
  using B = VBits<V>;
  constexpr int C = PAT / 2;
  constexpr int NT = PAT / 2;
  constexpr int WX = hp_wx(PAT), WY = hp_wy(PAT);
  constexpr int NL = WF_TX * WF_TY;
  constexpr int PRE = wf_pre(PAT);
  __shared__ V ring[WF_HIST][NL];
  __shared__ unsigned s_ticket;

  const int tid = threadIdx.x;
  const int lx = tid / WF_TY, ly = tid % WF_TY;
  const int sh = a.t.sh;
  const int skew = (WX - sh * WY) * lx + WY * ly + PRE;
  const Grid g = a.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int NS = a.t.ns;
  const unsigned ntiles = (unsigned)(a.t.ntx * a.t.nty);
  const bool exported = wf_exported(PAT, DIR, lx, ly, sh);
  const bool exp_next = a.next != nullptr && wf_exported(PAT, a.next_dir, lx, ly, sh);

  // Neighbour lanes / remoteness of the four candidate columns (their
  // offsets are mirrored for a backward sweep).
  int nlane[4];
  int nskew[4];
  bool remote[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int cx = DIR * col_dx(c), cy = DIR * col_dy(c);
    const int qx = lx + cx, qy = ly + cy + sh * cx;
    remote[c] = qx < 0 || qx >= WF_TX || qy < 0 || qy >= WF_TY;
    nlane[c] = remote[c] ? 0 : qx * WF_TY + qy;
    nskew[c] = (WX - sh * WY) * qx + WY * qy + PRE;
  }

  for (;;) {
    if (tid == 0) s_ticket = atomicAdd(&a.ctr[0], 1u);
    __syncthreads();
    const unsigned ticket = s_ticket;
    __syncthreads();
    if (ticket >= ntiles) break;
    const unsigned tile = DIR > 0 ? ticket : ntiles - 1u - ticket;
    const int X = (int)(tile / (unsigned)a.t.nty), Y = (int)(tile % (unsigned)a.t.nty);
    const int xt = X * WF_TX + lx;
    const int yt = Y * WF_TY + ly - sh * lx;
    const bool colv = xt < nx && yt >= 0 && yt < ny;
    const long cb = colv ? ((long)xt * ny + yt) * nz : 0;
    const long kb = (long)tile * NS * NL + tid;  // skewed index of (tile, step 0, lane)

    bool cin[4];
    long ncb[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int qx = xt + DIR * col_dx(c), qy = yt + DIR * col_dy(c);
      cin[c] = colv && qx >= 0 && qx < nx && qy >= 0 && qy < ny;
      ncb[c] = cin[c] ? ((long)qx * ny + qy) * nz : 0;
    }

    // step count rounded up to a multiple of P (the extra steps find every
    // lane inactive): the unrolled loop below then has no early exit
    const int nsteps = (NS + P - 1) / P * P;

    V cf[P][NT > 0 ? NT : 1];
    V hv[P], dv[P], av[P];
    V rb[P][4];
    V win[4][3];
    V own_prev = V(0);
#pragma unroll
    for (int c = 0; c < 4; ++c) win[c][0] = win[c][1] = win[c][2] = V(0);
    V* const nbuf = a.next != nullptr ? a.next : a.dump;

    auto prefetch = [&](int k, int j) {
      const int s = DIR > 0 ? k : NS - 1 - k;
      const int z = s - skew;
      const bool act = colv && z >= 0 && z < nz;
      const long q = act ? kb + (long)s * NL : kb;
      const long i = act ? cb + z : 0;
#pragma unroll
      for (int t = 0; t < NT; ++t) cf[j][t] = sk(DIR > 0 ? t : C + 1 + t, q);
      if (!UNITD) dv[j] = sk(C, q);
      hv[j] = a.h[i];
      if (ADD) av[j] = a.addv[i];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (!col_used(PAT, c)) continue;
        const int zn = z + DIR * col_maxdz(PAT, c);
        const bool ok = remote[c] && cin[c] && zn >= 0 && zn < nz;
        rb[j][c] = ld_coherent(a.x + (ok ? ncb[c] + zn : 0));
      }
    };

#pragma unroll
    for (int j = 0; j < P; ++j) prefetch(j, j);

    for (int k0 = 0; k0 < nsteps; k0 += P) {
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int k = k0 + j;
        const int s = DIR > 0 ? k : NS - 1 - k;
        const int z = s - skew;
        // 1. slide the neighbour windows by one point and fetch the newest
        //    (win[c][e] holds the value at z + DIR*(e-1))
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (!col_used(PAT, c)) continue;
          const int md = col_maxdz(PAT, c);
          win[c][0] = win[c][1];
          win[c][1] = win[c][2];
          const int zn = z + DIR * md;
          const bool valid = cin[c] && zn >= 0 && zn < nz;
          const V vl = ring[(zn + nskew[c] + 64 * WF_HIST) % WF_HIST][nlane[c]];
          V v = remote[c] ? rb[j][c] : vl;
          if (valid && remote[c] && B::bits(v) == B::sent) {
            const V* p = a.x + ncb[c] + zn;
            unsigned spins = 0;
            do {
              __builtin_amdgcn_s_sleep(1);
              v = ld_coherent(p);
              // once any wait has timed out, stop waiting anywhere
              if ((spins & 1023u) == 1023u &&
                  (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1u))
                spins = WF_SPIN_LIMIT;
            } while (B::bits(v) == B::sent && ++spins < WF_SPIN_LIMIT);
            if (spins >= WF_SPIN_LIMIT) atomicOr(a.err, 1u);
          }
          win[c][md + 1] = valid ? v : V(0);
        }
        // 2. the row update (computed by every lane, stored by active ones)
        const bool act = colv && z >= 0 && z < nz;
        V t = hv[j];
#pragma unroll
        for (int m = 0; m < NT; ++m) {
          const int so = DIR > 0 ? m : C + 1 + m;
          const int dx = pat_off(PAT, so, 0), dy = pat_off(PAT, so, 1), dz = pat_off(PAT, so, 2);
          V val;
          bool ok;
          if (dx == 0 && dy == 0) {
            val = own_prev;
            ok = z + dz >= 0 && z + dz < nz;
          } else {
            const int c = col_of(DIR * dx, DIR * dy);
            val = win[c][DIR * dz + 1];
            ok = cin[c] && z + dz >= 0 && z + dz < nz;
          }
          if (ok) t = fma(-cf[j][m], val, t);
        }
        const V xv = UNITD ? t : t * dv[j];
        own_prev = xv;
        ring[(s + 64 * WF_HIST) % WF_HIST][tid] = xv;
        const long i = cb + z;
        *((act && !exported) ? a.x + i : a.dump + tid) = xv;
        st_coherent((act && exported) ? a.x + i : a.dump + NL + tid, xv);
        *((act && exp_next) ? nbuf + i : a.dump + 2 * NL + tid) = B::val(B::sent);
        if (ADD) *(act ? a.addout + i : a.dump + 3 * NL + tid) = av[j] + xv;
        // 3. refill this register slot for step k + P
        prefetch(k + P, j);
        __syncthreads();
      }
    }
  }
  if (tid == 0) {
    unsigned o = atomicAdd(&a.ctr[1], 1u);
    if (o == gridDim.x - 1) {
      __hip_atomic_store(&a.ctr[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&a.ctr[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// Builds the schedule-ordered copy of a level's sweep data: slot s < C from
// lo[s], slot C from dg, slot s > C from up[s] (natural SG-DIA arrays of N
// entries per slot); positions that hold no point are zero.
template <class T>
__device__ inline T conv(double v);
template <>
__device__ inline double conv<double>(double v) {
  return v;
}
template <>
__device__ inline float conv<float>(double v) {
  return (float)v;
}

__device__ inline long skew_point(const Grid& g, const WfTiling& tl, int pat, long q) {
  constexpr int NL = WF_TX * WF_TY;
  const int l = (int)(q % NL);
  const long r = q / NL;
  const int s = (int)(r % tl.ns);
  const int tile = (int)(r / tl.ns);
  const int X = tile / tl.nty, Y = tile % tl.nty;
  const int lx = l / WF_TY, ly = l % WF_TY;
  const int x = X * WF_TX + lx, y = Y * WF_TY + ly - tl.sh * lx;
  const int z = s - ((hp_wx(pat) - tl.sh * hp_wy(pat)) * lx + hp_wy(pat) * ly + wf_pre(pat));
  const bool v = x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
  return v ? ((long)x * g.ny + y) * g.nz + z : -1;
}

template <int PAT, class T>
__global__ __launch_bounds__(256) void k_skew_pack(Grid g, WfTiling tl, const double* __restrict__ lo,
                                                   const double* __restrict__ dg, const double* __restrict__ up,
                                                   T* __restrict__ out) {
  constexpr int C = PAT / 2;
  const long q = (long)blockIdx.x * 256 + threadIdx.x;
  if (q >= tl.nsk) return;
  const long i = skew_point(g, tl, PAT, q);
  const long N = g.N();
#pragma unroll
  for (int sl = 0; sl < PAT; ++sl) {
    double val = 0.0;
    if (i >= 0) val = sl < C ? lo[(long)sl * N + i] : (sl == C ? dg[i] : up[(long)sl * N + i]);
    out[(long)sl * tl.nsk + q] = conv<T>(val);
  }
}

// FP16 storage: halves and row scales copied from the natural FP16 arrays,
// the diagonal scaling (FP32) into its own array.
template <int PAT>
__global__ __launch_bounds__(256) void k_skew_pack_h(Grid g, WfTiling tl, const __half* __restrict__ a16,
                                                     const float* __restrict__ sc, const float* __restrict__ rd,
                                                     __half* __restrict__ o16, float* __restrict__ osc,
                                                     float* __restrict__ ord) {
  const long q = (long)blockIdx.x * 256 + threadIdx.x;
  if (q >= tl.nsk) return;
  const long i = skew_point(g, tl, PAT, q);
  const long N = g.N();
#pragma unroll
  for (int sl = 0; sl < PAT; ++sl)
    o16[(long)sl * tl.nsk + q] = i >= 0 ? a16[(long)sl * N + i] : __float2half_rn(0.0f);
  osc[q] = i >= 0 ? sc[i] : 0.0f;
  ord[q] = i >= 0 ? rd[i] : 0.0f;
}

template <class T>
hipError_t launch_skew_pack(int pat, const Grid& g, const WfTiling& tl, const double* lo, const double* dg,
                            const double* up, T* out, hipStream_t st) {
  const dim3 grid((unsigned)((tl.nsk + 255) / 256)), blk(256);
  if (pat == 7)
    hipLaunchKernelGGL((k_skew_pack<7, T>), grid, blk, 0, st, g, tl, lo, dg, up, out);
  else if (pat == 19)
    hipLaunchKernelGGL((k_skew_pack<19, T>), grid, blk, 0, st, g, tl, lo, dg, up, out);
  else if (pat == 27)
    hipLaunchKernelGGL((k_skew_pack<27, T>), grid, blk, 0, st, g, tl, lo, dg, up, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
template hipError_t launch_skew_pack<double>(int, const Grid&, const WfTiling&, const double*, const double*,
                                             const double*, double*, hipStream_t);
template hipError_t launch_skew_pack<float>(int, const Grid&, const WfTiling&, const double*, const double*,
                                            const double*, float*, hipStream_t);

hipError_t launch_skew_pack_h(int pat, const Grid& g, const WfTiling& tl, const __half* a16, const float* sc,
                              const float* rd, __half* o16, float* osc, float* ord, hipStream_t st) {
  const dim3 grid((unsigned)((tl.nsk + 255) / 256)), blk(256);
  if (pat == 7)
    hipLaunchKernelGGL((k_skew_pack_h<7>), grid, blk, 0, st, g, tl, a16, sc, rd, o16, osc, ord);
  else if (pat == 19)
    hipLaunchKernelGGL((k_skew_pack_h<19>), grid, blk, 0, st, g, tl, a16, sc, rd, o16, osc, ord);
  else if (pat == 27)
    hipLaunchKernelGGL((k_skew_pack_h<27>), grid, blk, 0, st, g, tl, a16, sc, rd, o16, osc, ord);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <int PAT, int DIR, int P, class SK, bool UNITD, bool ADD>
static hipError_t launch_wf_t(const WfArgs<typename SK::V>& a, const SK& m, hipStream_t st) {
  const unsigned ntiles = (unsigned)(a.t.ntx * a.t.nty);
  const unsigned grid = ntiles < 2048u ? ntiles : 2048u;
  hipLaunchKernelGGL((k_wavefront<PAT, DIR, P, SK, UNITD, ADD>), dim3(grid), dim3(WF_TX * WF_TY), 0, st, a, m);
  return hipGetLastError();
}

template <class SK>
hipError_t launch_wavefront(int pat, int dir, bool unitd, bool add, const WfArgs<typename SK::V>& a, const SK& m,
                            hipStream_t st) {
#define SMG_WF_CASE(PATV, PV)                                                                           \
  if (pat == PATV) {                                                                                    \
    if (dir > 0 && !unitd && !add) return launch_wf_t<PATV, 1, PV, SK, false, false>(a, m, st);         \
    if (dir < 0 && !unitd && !add) return launch_wf_t<PATV, -1, PV, SK, false, false>(a, m, st);        \
    if (dir > 0 && unitd && !add) return launch_wf_t<PATV, 1, PV, SK, true, false>(a, m, st);           \
    if (dir < 0 && !unitd && add) return launch_wf_t<PATV, -1, PV, SK, false, true>(a, m, st);          \
  }
  SMG_WF_CASE(7, 6)
  SMG_WF_CASE(19, 3)
  SMG_WF_CASE(27, 2)
#undef SMG_WF_CASE
  return hipErrorInvalidValue;
}

template hipError_t launch_wavefront<SkD>(int, int, bool, bool, const WfArgs<double>&, const SkD&, hipStream_t);
template hipError_t launch_wavefront<SkF>(int, int, bool, bool, const WfArgs<float>&, const SkF&, hipStream_t);
template hipError_t launch_wavefront<SkH>(int, int, bool, bool, const WfArgs<float>&, const SkH&, hipStream_t);

}  // namespace smg
