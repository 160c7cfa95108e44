// Dependence-preserving structured triangular sweep (Sec. 3.4): point
// Gauss-Seidel and the ILU(0) factor solves, computed in exactly the order of
// the sequential lexicographic sweep, so the result equals the serial one.
//
// Row update (sweep frame, the "lower" offsets of the sweep direction T):
//     t = h_i;  for s in T (canonical order): t = fma(-c_s[i], x[i+off_s], t);
//     x_i = t * d_i          (or x_i = t for a unit diagonal)
//
// GPU design (replaces the CPU design of the paper, which projects the grid
// onto x-y columns, runs level-scheduled column tasks and synchronises
// threads point-to-point through a shared counter array):
//  * The z-column is the unit.  A workgroup owns a TX x TY tile of columns,
//    one column per lane.  In the sweep frame, column (x, y) is sheared so a
//    tile covers x in [X*TX, X*TX+TX) and y + sh*(x - X*TX) in [Y*TY, Y*TY+TY).
//  * Lane (lx, ly) processes point z at local step z + skew(lx, ly), with
//    skew = (wx - sh*wy)*lx + wy*ly and the hyperplane weights (wx, wy, 1) of
//    the pattern.  All lanes of a tile then sit on one global hyperplane per
//    step, and every dependence points to an earlier step.
//  * Lanes exchange fresh values through an LDS ring of the last 8 steps and
//    one workgroup barrier per step.
//  * Columns owned by other tiles are read from global memory.  The output
//    vector holds a signalling-NaN sentinel at every position that another
//    tile reads; a value is ready when it is no longer the sentinel.  These
//    positions are written and read with device-coherent (agent-scope)
//    atomic stores and loads, so no fences or flag counters are needed.  The
//    sentinels for the next sweep on the same level are written by this
//    sweep into that sweep's output buffer.
//  * Tiles are handed out by an atomic ticket in an order in which every
//    dependence has a smaller ticket (x-tiles outer, y-tiles inner), so a
//    persistent grid of any size always makes progress.  Waits are bounded
//    by a watchdog that raises an error flag instead of hanging.
//  * Coefficients, right-hand side and diagonal are prefetched P steps ahead
//    in registers; values from other tiles are prefetched P steps ahead too.
#include "smg_common.h"
#include "smg_kernels.h"

namespace smg {

constexpr int WF_TX = 16, WF_TY = 16, WF_HIST = 8;
constexpr unsigned WF_SPIN_LIMIT = 1u << 21;

// Sweep-frame neighbour columns that can hold lower neighbours.
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

// Is column (lx, ly) read by a lane of another tile?
__device__ inline bool wf_exported(int pat, int lx, int ly, int sh) {
  for (int c = 0; c < 4; ++c) {
    if (!col_used(pat, c)) continue;
    int cx = lx - col_dx(c), cy = ly - col_dy(c) - sh * col_dx(c);
    if (cx < 0 || cx >= WF_TX || cy < 0 || cy >= WF_TY) return true;
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

template <int PAT, int DIR, int P, class M, bool UNITD, bool ADD>
__global__ __launch_bounds__(WF_TX* WF_TY) void k_wavefront(WfArgs<typename M::V> a, M mat) {
  using V = typename M::V;
  using B = VBits<V>;
  constexpr int C = PAT / 2;
  constexpr int NT = PAT / 2;
  constexpr int WX = hp_wx(PAT), WY = hp_wy(PAT);
  constexpr int NL = WF_TX * WF_TY;
  __shared__ V ring[WF_HIST][NL];
  __shared__ unsigned s_ticket;

  const int tid = threadIdx.x;
  const int lx = tid / WF_TY, ly = tid % WF_TY;
  const int sh = a.sh;
  // PRE = 1 when a neighbour column is read one point ahead (dz = +1): every
  // lane then starts one step early to fill its window.
  constexpr int PRE = (col_used(PAT, 0) && col_maxdz(PAT, 0)) || (col_used(PAT, 1) && col_maxdz(PAT, 1)) ||
                              (col_used(PAT, 2) && col_maxdz(PAT, 2)) || (col_used(PAT, 3) && col_maxdz(PAT, 3))
                          ? 1
                          : 0;
  const int skew = (WX - sh * WY) * lx + WY * ly + PRE;
  const Grid g = a.g;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const unsigned ntiles = (unsigned)(a.ntx * a.nty);
  const bool exported = wf_exported(PAT, lx, ly, sh);

  // Neighbour lanes / remoteness of the four candidate columns.
  int nlane[4];
  int nskew[4];
  bool remote[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int qx = lx + col_dx(c), qy = ly + col_dy(c) + sh * col_dx(c);
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
    const int X = (int)(ticket / (unsigned)a.nty), Y = (int)(ticket % (unsigned)a.nty);
    const int xt = X * WF_TX + lx;
    const int yt = Y * WF_TY + ly - sh * lx;
    const bool colv = xt < nx && yt >= 0 && yt < ny;
    const int xo = DIR > 0 ? xt : nx - 1 - xt;
    const int yo = DIR > 0 ? yt : ny - 1 - yt;
    const long cb = colv ? ((long)xo * ny + yo) * nz : 0;

    // column validity of the neighbour columns and their global bases
    bool cin[4];
    long ncb[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int qx = xt + col_dx(c), qy = yt + col_dy(c);
      cin[c] = colv && qx >= 0 && qx < nx && qy >= 0 && qy < ny;
      int qxo = DIR > 0 ? qx : nx - 1 - qx, qyo = DIR > 0 ? qy : ny - 1 - qy;
      ncb[c] = cin[c] ? ((long)qxo * ny + qyo) * nz : 0;
    }

    // exported flag of this column for the next sweep (its own frame)
    bool pref = false;
    if (a.next != nullptr && colv) {
      int x2 = a.next_dir > 0 ? xo : nx - 1 - xo;
      int y2 = a.next_dir > 0 ? yo : ny - 1 - yo;
      int lx2 = x2 % WF_TX;
      int ly2 = (y2 + a.next_sh * lx2) % WF_TY;
      pref = wf_exported(PAT, lx2, ly2, a.next_sh);
    }

    const int nsteps = nz + (WX - sh * WY) * (WF_TX - 1) + WY * (WF_TY - 1) + PRE;

    V cf[P][NT > 0 ? NT : 1];
    V hv[P], dv[P], av[P];
    V rb[P][4];
    V win[4][3];
    V own_prev = V(0);
#pragma unroll
    for (int c = 0; c < 4; ++c) win[c][0] = win[c][1] = win[c][2] = V(0);

    auto prefetch = [&](int s, int j) {
      const int z = s - skew;
      if (colv && z >= 0 && z < nz) {
        const long i = cb + (DIR > 0 ? z : nz - 1 - z);
#pragma unroll
        for (int t = 0; t < NT; ++t) cf[j][t] = mat(DIR > 0 ? t : C + 1 + t, i);
        hv[j] = a.h[i];
        if (!UNITD) dv[j] = a.d[i];
        if (ADD) av[j] = a.addv[i];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (!col_used(PAT, c) || !remote[c]) continue;
        const int zn = z + col_maxdz(PAT, c);
        if (cin[c] && zn >= 0 && zn < nz) rb[j][c] = ld_coherent(a.x + ncb[c] + (DIR > 0 ? zn : nz - 1 - zn));
      }
    };

#pragma unroll
    for (int j = 0; j < P; ++j) prefetch(j, j);

    for (int s0 = 0; s0 < nsteps; s0 += P) {
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int s = s0 + j;
        if (s >= nsteps) break;
        const int z = s - skew;
        // 1. slide the neighbour windows by one point and fetch the newest
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (!col_used(PAT, c)) continue;
          const int md = col_maxdz(PAT, c);
          win[c][0] = win[c][1];
          win[c][1] = win[c][2];
          const int zn = z + md;
          V v = V(0);
          if (cin[c] && zn >= 0 && zn < nz) {
            if (!remote[c]) {
              v = ring[(zn + nskew[c]) % WF_HIST][nlane[c]];
            } else {
              v = rb[j][c];
              if (B::bits(v) == B::sent) {
                const V* p = a.x + ncb[c] + (DIR > 0 ? zn : nz - 1 - zn);
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
            }
          }
          win[c][md + 1] = v;
        }
        // 2. the row update
        if (colv && z >= 0 && z < nz) {
          V t = hv[j];
#pragma unroll
          for (int k = 0; k < NT; ++k) {
            const int so = DIR > 0 ? k : C + 1 + k;
            const int dx = DIR * pat_off(PAT, so, 0), dy = DIR * pat_off(PAT, so, 1),
                      dz = DIR * pat_off(PAT, so, 2);
            V val;
            bool ok;
            if (dx == 0 && dy == 0) {
              val = own_prev;
              ok = z >= 1;
            } else {
              const int c = col_of(dx, dy);
              val = win[c][dz + 1];
              ok = cin[c] && z + dz >= 0 && z + dz < nz;
            }
            if (ok) t = fma(-cf[j][k], val, t);
          }
          const V xv = UNITD ? t : t * dv[j];
          own_prev = xv;
          ring[s % WF_HIST][tid] = xv;
          const long i = cb + (DIR > 0 ? z : nz - 1 - z);
          if (exported)
            st_coherent(a.x + i, xv);
          else
            a.x[i] = xv;
          if (pref) a.next[i] = B::val(B::sent);
          if (ADD) a.addout[i] = av[j] + xv;
        }
        // 3. refill this register slot for step s + P
        prefetch(s + P, j);
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
template <int PAT, int DIR, int P, class M, bool UNITD, bool ADD>
static hipError_t launch_wf_t(const WfArgs<typename M::V>& a, const M& m, hipStream_t st) {
  unsigned ntiles = (unsigned)(a.ntx * a.nty);
  unsigned grid = ntiles < 2048u ? ntiles : 2048u;
  hipLaunchKernelGGL((k_wavefront<PAT, DIR, P, M, UNITD, ADD>), dim3(grid), dim3(WF_TX * WF_TY), 0, st, a, m);
  return hipGetLastError();
}

void wf_tiling(const Grid& g, int* sh, int* ntx, int* nty) {
  *sh = g.ny <= WF_TY ? 0 : 1;
  *ntx = (g.nx + WF_TX - 1) / WF_TX;
  *nty = (g.ny + (*sh) * (WF_TX - 1) + WF_TY - 1) / WF_TY;
}

template <class M>
hipError_t launch_wavefront(int pat, int dir, bool unitd, bool add, const WfArgs<typename M::V>& a, const M& m,
                            hipStream_t st) {
#define SMG_WF_CASE(PATV, PV)                                                                           \
  if (pat == PATV) {                                                                                    \
    if (dir > 0 && !unitd && !add) return launch_wf_t<PATV, 1, PV, M, false, false>(a, m, st);          \
    if (dir < 0 && !unitd && !add) return launch_wf_t<PATV, -1, PV, M, false, false>(a, m, st);         \
    if (dir > 0 && unitd && !add) return launch_wf_t<PATV, 1, PV, M, true, false>(a, m, st);            \
    if (dir < 0 && !unitd && add) return launch_wf_t<PATV, -1, PV, M, false, true>(a, m, st);           \
  }
  SMG_WF_CASE(7, 8)
  SMG_WF_CASE(19, 4)
  SMG_WF_CASE(27, 4)
#undef SMG_WF_CASE
  return hipErrorInvalidValue;
}

template hipError_t launch_wavefront<MatD>(int, int, bool, bool, const WfArgs<double>&, const MatD&, hipStream_t);
template hipError_t launch_wavefront<MatF>(int, int, bool, bool, const WfArgs<float>&, const MatF&, hipStream_t);
template hipError_t launch_wavefront<MatH>(int, int, bool, bool, const WfArgs<float>&, const MatH&, hipStream_t);

}  // namespace smg
