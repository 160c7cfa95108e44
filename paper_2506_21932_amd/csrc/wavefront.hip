// Dependence-preserving structured triangular sweep (Sec. 4.4): point
// Gauss-Seidel and the ILU(0) factor solves, computed in exactly the order of
// the sequential lexicographic sweep, so the result equals the serial one.
//
// Row update (T = lower offsets for a forward sweep, upper for a backward one):
//     t = h_i;  for s in T (canonical order): t = fma(-c_s[i], x[i+off_s], t);
//     x_i = t * d_i          (or x_i = t for a unit diagonal)
// Couplings to points outside the grid are stored as zero and their values
// read as zero, so every term is applied unconditionally.
//
// GPU design (replaces the CPU design of the paper, which projects the grid
// onto x-y columns, runs level-scheduled column tasks and synchronises
// threads point-to-point through a shared counter array):
//  * The z-column is the unit.  A workgroup owns a TX x TY tile of columns,
//    one column per lane: tile (X, Y) holds x in [X*TX, X*TX+TX) and
//    y + sh*(x - X*TX) in [Y*TY, Y*TY+TY) (sheared so that no dependence
//    points from a tile to a later one).
//  * Lane (lx, ly) handles point z at step s = z + skew(lx, ly), with
//    skew = (wx - sh*wy)*lx + wy*ly + KB and the hyperplane weights
//    (wx, wy, 1) of the pattern; a neighbour at offset (dx, dy, dz) is then
//    handled exactly wx*dx + wy*dy + dz steps away, the same for every lane,
//    which is earlier for every lower neighbour.  A backward sweep runs the
//    same tiles and steps in reverse order, which orders upper neighbours
//    first.  KB pads both ends of the step range so that values of
//    neighbouring tiles referenced at the first and last steps have a step.
//  * The coefficients and the diagonal scaling are read from a copy stored
//    in this schedule order, one copy per direction, packed 16 bytes per lane
//    ([tile][step][pack][lane]): each step loads them with a few wide,
//    fully coalesced loads.
//  * Values are exchanged through an LDS ring of 16 steps holding the tile's
//    columns plus a halo of neighbouring tiles' columns, with one workgroup
//    barrier per step.  Because step distances do not depend on the lane,
//    every neighbour read is one LDS load at a compile-time row.
//  * Halo values are fetched by a few loader lanes from the output vector,
//    which holds a signalling-NaN sentinel at every position read by another
//    tile until that tile writes it; a value is ready when it is no longer
//    the sentinel.  These accesses are device-coherent (agent scope), so no
//    fences or flag counters are needed.  The sentinels for the next sweep on
//    the same level are written by this sweep into that sweep's output.
//  * Halo values are prefetched PH = 4 steps ahead: enough to cover a
//    device-coherent load (about a microsecond), while a tile must run only
//    that far behind its producer for the prefetch to find them written.
//    A loader lane that finds a value not yet written first waits for the
//    value WF_AHEAD steps further along the same column and then refetches
//    its other prefetched halo values: the tile then runs far enough behind
//    its producer that later prefetches find their values written, instead
//    of paying one coherent round trip per step.
//  * The right-hand side is staged through LDS in chunks of 16 steps, loaded
//    one chunk ahead as runs of 16 consecutive z per column (two runs per
//    step in the first half of a chunk, each placed in LDS four steps after
//    its load); each lane writes its result over the right-hand-side slot it
//    has just used, and the chunk's results leave the same way, two runs per
//    step in the first half of the following chunk (before their slots are
//    refilled), together with the sentinels for the next sweep.  Per-step accesses to the natural-order vectors would touch one
//    element of a different cache line per lane and keep hundreds of lines
//    per tile alive in the L2 cache; spreading the runs over the steps keeps
//    them from holding up the in-order completion of the coefficient loads.
//    Only columns read by other tiles are also stored at once,
//    device-coherently.
//  * Tiles are handed out by an atomic ticket in dependence order, so a
//    persistent grid of any size always makes progress.  Waits are bounded
//    by a watchdog that raises an error flag instead of hanging.
//  * All per-point accesses use buffer instructions; lanes without a point
//    at a step use an offset outside the buffer, for which loads return zero
//    and stores are dropped.  Tile inputs are prefetched P steps ahead.
#include "smg_common.h"
#include "smg_kernels.h"

namespace smg {

constexpr int WF_HIST = 16;                // LDS ring rows (steps)
constexpr int WF_CH = 16;                  // steps per chunk of right-hand side / results
constexpr int WF_NL = WF_TX * WF_TY;       // lanes (columns) per tile
constexpr int WF_NH = 104;                 // halo slots around a tile
constexpr unsigned WF_SPIN_LIMIT = 1u << 21;
#ifndef WF_LAG_EXTRA
#define WF_LAG_EXTRA 2
#endif
#ifndef WF_PH
#define WF_PH 4
#endif
constexpr unsigned WF_OOB = 0x80000000u;   // buffer offset outside every range
constexpr int WF_SC1 = 16;                 // cache policy of device-coherent accesses

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Neighbour columns holding lower neighbours (forward-frame offsets); a
// backward sweep uses the negated offsets.
__host__ __device__ constexpr int col_dx(int c) { return c == 3 ? 0 : -1; }
__host__ __device__ constexpr int col_dy(int c) { return c == 3 ? -1 : c - 1; }
__host__ __device__ constexpr bool col_used(int pat, int c) {
  return pat_has(pat, col_dx(c), col_dy(c), -1) || pat_has(pat, col_dx(c), col_dy(c), 0) ||
         pat_has(pat, col_dx(c), col_dy(c), 1);
}
__host__ __device__ constexpr int col_of(int dx, int dy) {
  return dx == -1 ? dy + 1 : (dy == -1 ? 3 : -1);
}

// Largest step distance of a lower neighbour: max over lower offsets of
// -(wx*dx + wy*dy + dz).
__host__ __device__ constexpr int wf_kb(int pat) {
  int m = 0;
  for (int s = 0; s < pat / 2; ++s) {
    const int d = -(hp_wx(pat) * pat_off(pat, s, 0) + hp_wy(pat) * pat_off(pat, s, 1) + pat_off(pat, s, 2));
    m = d > m ? d : m;
  }
  return m;
}

// 16-byte packs per point and direction: the pat/2 coefficients of the
// sweep's triangle followed (except for FP16 storage, which keeps it apart)
// by the diagonal scaling.
__host__ __device__ constexpr int wf_npk(int pat, int ebytes) {
  return (pat / 2 + (ebytes == 2 ? 0 : 1) + 16 / ebytes - 1) / (16 / ebytes);
}

void wf_tiling(const Grid& g, int pat, WfTiling* t) {
  t->sh = g.ny <= WF_TY ? 0 : 1;
  t->ntx = (g.nx + WF_TX - 1) / WF_TX;
  t->nty = (g.ny + t->sh * (WF_TX - 1) + WF_TY - 1) / WF_TY;
  const int kb = wf_kb(pat);
  t->ns = g.nz + (hp_wx(pat) - t->sh * hp_wy(pat)) * (WF_TX - 1) + hp_wy(pat) * (WF_TY - 1) + 2 * kb;
  t->nsk = (long)t->ntx * t->nty * t->ns * WF_NL;
}

int wf_pack_count(int pat, int ebytes) { return wf_npk(pat, ebytes); }

bool wf_ranges_ok(const Grid& g, const WfTiling& t, int pat, int vbytes, int ebytes) {
  const double vec = (double)(WF_TX + 2) * g.ny * g.nz * vbytes;
  const double tile = (double)t.ns * wf_npk(pat, ebytes) * WF_NL * 16;
  return vec < 2147483647.0 && tile < 2147483647.0;
}

// Halo slot of column (qx, qy) relative to a tile (outside [0,TX) x [0,TY)):
// the columns x-1 and x+TX with y in [-2, TY+2), and for x inside the tile the
// rows y in {-2, -1, TY, TY+1}.  Every neighbour column of a tile lies there.
__host__ __device__ constexpr int wf_halo_slot(int qx, int qy) {
  return qx == -1 ? qy + 2
                  : (qx == WF_TX ? 22 + qy
                                 : (qy < 0 ? 40 + 2 * qx + (qy + 2) : 72 + 2 * qx + (qy - WF_TY)));
}
__device__ inline void wf_halo_pos(int hs, int* qx, int* qy) {
  if (hs < 20) {
    *qx = -1;
    *qy = hs - 2;
  } else if (hs < 40) {
    *qx = WF_TX;
    *qy = hs - 22;
  } else if (hs < 72) {
    *qx = (hs - 40) / 2;
    *qy = (hs - 40) % 2 - 2;
  } else {
    *qx = (hs - 72) / 2;
    *qy = WF_TY + (hs - 72) % 2;
  }
}

// Is halo column (qx, qy) a neighbour column of some lane of the tile in a
// sweep of direction dir?
__device__ inline bool wf_halo_used(int pat, int dir, int sh, int qx, int qy) {
  for (int c = 0; c < 4; ++c) {
    if (!col_used(pat, c)) continue;
    const int cx = dir * col_dx(c), cy = dir * col_dy(c);
    const int lx = qx - cx, ly = qy - cy - sh * cx;
    if (lx >= 0 && lx < WF_TX && ly >= 0 && ly < WF_TY) return true;
  }
  return false;
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

// ---- buffer access helpers -------------------------------------------------
__device__ inline __amdgpu_buffer_rsrc_t wf_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <class V, int CP>
__device__ inline V bld(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ inline double bld<double, 0>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ inline double bld<double, WF_SC1>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, WF_SC1));
}
template <>
__device__ inline float bld<float, 0>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ inline float bld<float, WF_SC1>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, WF_SC1));
}
template <int CP>
__device__ inline void bst(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, CP);
}
template <int CP>
__device__ inline void bst(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, CP);
}

// Storage element traits: arithmetic type V, elements per 16-byte pack K,
// and element m of a run of packs.
template <class E>
struct WfE;
template <>
struct WfE<double> {
  using V = double;
  static constexpr int K = 2;
  static constexpr bool HALF = false;
  __device__ static double get(const u32x4* pk, int m) {
    const u32x4 w = pk[m / 2];
    return m % 2 == 0 ? __builtin_bit_cast(double, u32x2{w.x, w.y}) : __builtin_bit_cast(double, u32x2{w.z, w.w});
  }
};
template <>
struct WfE<float> {
  using V = float;
  static constexpr int K = 4;
  static constexpr bool HALF = false;
  __device__ static float get(const u32x4* pk, int m) { return __uint_as_float(pk[m / 4][m % 4]); }
};
template <>
struct WfE<__half> {
  using V = float;
  static constexpr int K = 8;
  static constexpr bool HALF = true;
  __device__ static float get(const u32x4* pk, int m) {
    const unsigned w = pk[m / 8][(m % 8) / 2];
    return __half2float(__ushort_as_half((unsigned short)(m % 2 == 0 ? (w & 0xffffu) : (w >> 16))));
  }
};

// One tile of a sweep (tile numbers in forward dependence order).  err
// receives the watchdog flag.
template <int PAT, int DIR, int P, class E, bool UNITD, bool ADD>
__device__ __forceinline__ void wf_tile(const WfArgs<typename WfVal<E>::V>& a, unsigned tile, unsigned* err) {
  using T = WfE<E>;
  using V = typename T::V;
  using B = VBits<V>;
  constexpr int C = PAT / 2;
  constexpr int NT = PAT / 2;
  constexpr int WX = hp_wx(PAT), WY = hp_wy(PAT);
  constexpr int KB = wf_kb(PAT);
  constexpr int NPK = wf_npk(PAT, sizeof(E));
  constexpr int RW = WF_NL + WF_NH + 1;  // ring row length (padded: column runs hit distinct banks)
  constexpr int HRW = WF_NL + 1;         // right-hand-side chunk row length (padded likewise)
  constexpr unsigned PACKB = WF_NL * 16u;
  constexpr int PH = WF_PH;                    // prefetch distance of halo values
  constexpr int WF_AHEAD = PH + WF_LAG_EXTRA;  // steps a stalled tile falls back behind its producer
  static_assert(WF_HIST % P == 0 && WF_HIST % PH == 0 && PH >= 2 && WF_HIST > KB + 1, "ring too short");
  __shared__ V ring[WF_HIST * RW];
  __shared__ V hbuf[2 * WF_CH * HRW];  // right-hand side then results, two chunks of 16 steps

  const int tid = threadIdx.x;
  const int lx = tid / WF_TY, ly = tid % WF_TY;
  const int sh = a.t.sh;
  const int skew = (WX - sh * WY) * lx + WY * ly + KB;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int NS = a.t.ns;
  const bool exported = wf_exported(PAT, DIR, lx, ly, sh);

  // LDS index of each neighbour column (its offsets mirrored for a backward
  // sweep): a lane of this tile or a halo slot
  int nidx[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int cx = DIR * col_dx(c), cy = DIR * col_dy(c);
    const int qx = lx + cx, qy = ly + cy + sh * cx;
    const bool in = qx >= 0 && qx < WF_TX && qy >= 0 && qy < WF_TY;
    nidx[c] = !col_used(PAT, c) ? 0 : (in ? qx * WF_TY + qy : WF_NL + wf_halo_slot(qx, qy));
  }
  // halo loader role: slot hs, spread over the four waves
  const int hs = (tid % 64) * 4 + tid / 64;
  int hqx = 0, hqy = 0;
  bool hrole = false;
  if (hs < WF_NH) {
    wf_halo_pos(hs, &hqx, &hqy);
    hrole = wf_halo_used(PAT, DIR, sh, hqx, hqy);
  }
  const int hskew = (WX - sh * WY) * hqx + WY * hqy + KB;
  // column runs: in chunk transfers this thread moves step (tid % 16) of the
  // columns of lanes (lx = i, ly = tid / 16), i = 0..15
  const int cy = tid / WF_CH;
  const int cr = tid % WF_CH;
  unsigned cexp = 0, cnext = 0;  // bit i: that column is read by other tiles in this / the next sweep
#pragma unroll
  for (int i = 0; i < WF_TX; ++i) {
    cexp |= wf_exported(PAT, DIR, i, cy, sh) ? 1u << i : 0u;
    cnext |= (a.next != nullptr && wf_exported(PAT, a.next_dir, i, cy, sh)) ? 1u << i : 0u;
  }

  {
    const int X = (int)(tile / (unsigned)a.t.nty), Y = (int)(tile % (unsigned)a.t.nty);
    const int xt = X * WF_TX + lx;
    const int yt = Y * WF_TY + ly - sh * lx;
    const bool colv = xt < nx && yt >= 0 && yt < ny;

    // buffers over the planes x in [X*TX - 1, X*TX + TX + 1) of the vectors
    const int p0 = X * WF_TX > 0 ? X * WF_TX - 1 : 0;
    const int p1 = X * WF_TX + WF_TX + 1 < nx ? X * WF_TX + WF_TX + 1 : nx;
    const long pl = (long)ny * nz;
    const unsigned vbytes = (unsigned)((p1 - p0) * pl * (long)sizeof(V));
    const long vb = p0 * pl;
    const auto rh = wf_rsrc(a.h + vb, vbytes);
    const auto rx = wf_rsrc(a.x + vb, vbytes);
    const auto rn = wf_rsrc((a.next != nullptr ? a.next : a.x) + vb, a.next != nullptr ? vbytes : 0u);
    const auto rav = wf_rsrc((ADD ? a.addv : a.h) + vb, ADD ? vbytes : 0u);
    const auto rao = wf_rsrc((ADD ? a.addout : a.x) + vb, ADD ? vbytes : 0u);
    const unsigned vo = colv ? (unsigned)(((xt - p0) * (long)ny + yt) * nz) : 0u;
    const int gx = X * WF_TX + hqx, gy = Y * WF_TY + hqy - sh * hqx;
    const bool hcolv = hrole && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    const unsigned hvo = hcolv ? (unsigned)(((gx - p0) * (long)ny + gy) * nz) : 0u;
    const unsigned tbytes = (unsigned)NS * NPK * PACKB;
    const auto rp = wf_rsrc((const char*)a.pk + (size_t)tile * tbytes, tbytes);
    const unsigned sdbytes = T::HALF ? (unsigned)NS * WF_NL * 8u : 0u;
    const auto rs = wf_rsrc(T::HALF ? (const char*)a.sd + (size_t)tile * sdbytes : (const char*)a.pk, sdbytes);

    const int nsteps = (NS + WF_HIST - 1) / WF_HIST * WF_HIST;
    u32x4 cf[P][NPK];
    u32x2 sdv[P];
    V hb[PH], hc[WF_TX / 2];
    V own_prev = V(0);

    auto step_of = [&](int k) { return DIR > 0 ? k : NS - 1 - k; };
    auto prefetch = [&](int k, int j) {
      const int s = step_of(k);
      const bool sin = s >= 0 && s < NS;
      const unsigned so = sin ? (unsigned)s * (NPK * PACKB) : WF_OOB;
#pragma unroll
      for (int p = 0; p < NPK; ++p)
        cf[j][p] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rp, tid * 16u, so + p * PACKB, 0));
      if (T::HALF)
        sdv[j] = __builtin_amdgcn_raw_buffer_load_b64(rs, tid * 8u, sin ? (unsigned)s * (WF_NL * 8u) : WF_OOB, 0);
    };
    // byte offset of step s of the column of lane (i, cy), or WF_OOB.  The
    // column's element offset and skew are linear in i; which columns lie in
    // the grid is fixed per tile (bit i of rmask).
    const unsigned rb0 = (unsigned)(((X * WF_TX - p0) * (long)ny + (Y * WF_TY + cy)) * nz);
    const unsigned rdi = (unsigned)((long)ny * nz - (long)sh * nz);
    const int rsk0 = WY * cy + KB;
    unsigned rmask = 0;
#pragma unroll
    for (int i = 0; i < WF_TX; ++i) {
      const int xx = X * WF_TX + i, yy = Y * WF_TY + cy - sh * i;
      rmask |= (xx < nx && yy >= 0 && yy < ny) ? 1u << i : 0u;
    }
    auto run_off = [&](int i, int s) {
      const int z = s - rsk0 - (WX - sh * WY) * i;
      // branch-free: both tests as bits
      const unsigned ok = ((rmask >> i) & 1u) & (unsigned)((unsigned)z < (unsigned)nz);
      return ok ? (rb0 + (unsigned)i * rdi + (unsigned)z) * (unsigned)sizeof(V) : WF_OOB;
    };
    // right-hand side of chunk c: column runs i loaded into hc[i], then
    // placed in LDS
    auto hrun_load = [&](int c, int i) { hc[i % (WF_TX / 2)] = bld<V, 0>(rh, run_off(i, step_of(c * WF_CH + cr))); };
    auto hrun_put = [&](int c, int i) { hbuf[((c & 1) * WF_CH + cr) * HRW + i * WF_TY + cy] = hc[i % (WF_TX / 2)]; };
    // results of chunk c (in its hbuf half): column run i out, with the
    // sentinels of the next sweep
    auto xrun_out = [&](int c, int i) {
      const unsigned off = run_off(i, step_of(c * WF_CH + cr));
      const V xo = hbuf[((c & 1) * WF_CH + cr) * HRW + i * WF_TY + cy];
      bst<0>(xo, rx, (cexp >> i) & 1u ? WF_OOB : off);
      bst<0>(B::val(B::sent), rn, (cnext >> i) & 1u ? off : WF_OOB);
    };
    // ADD: addout = addv + x for all runs of chunk c
    auto add_out = [&](int c) {
      V av[WF_TX];
      unsigned off[WF_TX];
#pragma unroll
      for (int i = 0; i < WF_TX; ++i) {
        off[i] = run_off(i, step_of(c * WF_CH + cr));
        av[i] = bld<V, 0>(rav, off[i]);
      }
#pragma unroll
      for (int i = 0; i < WF_TX; ++i) bst<0>(av[i] + hbuf[((c & 1) * WF_CH + cr) * HRW + i * WF_TY + cy], rao, off[i]);
    };
    auto halo_fetch = [&](int k, int j) {
      const int s = step_of(k);
      const int hz = s - hskew;
      const bool hok = s >= 0 && s < NS && hcolv && hz >= 0 && hz < nz;
      hb[j] = bld<V, WF_SC1>(rx, hok ? (hvo + (unsigned)hz) * (unsigned)sizeof(V) : WF_OOB);
    };
    // Bounded wait until the halo value at byte offset off is no longer the
    // sentinel (v: its last loaded value).
    auto wait_value = [&](unsigned off, V v) {
      unsigned spins = 0;
      while (B::bits(v) == B::sent && spins < WF_SPIN_LIMIT) {
        __builtin_amdgcn_s_sleep(1);
        v = bld<V, WF_SC1>(rx, off);
        ++spins;
        // once any wait has timed out, stop waiting anywhere
        if ((spins & 1023u) == 1023u && (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1u))
          spins = WF_SPIN_LIMIT;
      }
      if (spins >= WF_SPIN_LIMIT) atomicOr(err, 1u);
      return v;
    };
    // halo value of iteration k (held in slot j): wait for it if it is still
    // the sentinel, then publish it in the ring
    auto halo_put = [&](int k, int j) {
      const int s = step_of(k);
      const int hz = s - hskew;
      const bool hok = s >= 0 && s < NS && hcolv && hz >= 0 && hz < nz;
      V v = hb[j];
      if (hok && B::bits(v) == B::sent) {
        // fall back behind the producer: wait for the value WF_AHEAD steps on
        // (clamped to the column), then for this one
        int zf = hz + DIR * WF_AHEAD;
        zf = zf < 0 ? 0 : (zf >= nz ? nz - 1 : zf);
        const unsigned offf = (hvo + (unsigned)zf) * (unsigned)sizeof(V);
        wait_value(offf, bld<V, WF_SC1>(rx, offf));
        v = wait_value((hvo + (unsigned)hz) * (unsigned)sizeof(V), v);
        // the other prefetched halo values were fetched too early: fetch again
#pragma unroll
        for (int d = 1; d < PH - 1; ++d) halo_fetch(k + d, (j + d) % PH);
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the refetched values are in
      }
      if (hrole) ring[(k % WF_HIST) * RW + WF_NL + hs] = hok ? v : V(0);
    };

#pragma unroll
    for (int j = 0; j < P; ++j) prefetch(j, j);
#pragma unroll
    for (int j = 0; j < PH; ++j) halo_fetch(j, j);
#pragma unroll
    for (int i = 0; i < WF_TX; ++i) {
      hrun_load(0, i);
      hrun_put(0, i);
    }
    halo_put(0, 0);
    __syncthreads();

    for (int k0 = 0; k0 < nsteps; k0 += WF_HIST) {
#pragma unroll
      for (int j = 0; j < WF_HIST; ++j) {
        const int k = k0 + j;
        const int jp = j % P;
        const int jj = j % WF_CH;
        const int ch = k / WF_CH;
        // the previous chunk's results, runs 2jj and 2jj+1 (a chunk before the
        // first maps every run outside the buffers), out before their slots
        // are refilled below
        if (jj < WF_CH / 2) {
          if (ADD && jj == 0) add_out(ch - 1);
          xrun_out(ch - 1, 2 * jj);
          xrun_out(ch - 1, 2 * jj + 1);
        }
        // the next chunk's right-hand side: runs 2(jj-4), 2(jj-4)+1 into LDS,
        // then runs 2jj, 2jj+1 from HBM (their registers were just freed)
        if (jj >= 4 && jj < WF_CH / 2 + 4) {
          hrun_put(ch + 1, 2 * (jj - 4));
          hrun_put(ch + 1, 2 * (jj - 4) + 1);
        }
        if (jj < WF_CH / 2) {
          hrun_load(ch + 1, 2 * jj);
          hrun_load(ch + 1, 2 * jj + 1);
        }
        const int s = step_of(k);
        const int z = s - skew;
        const bool act = colv && z >= 0 && z < nz;
        // the row update, in canonical order of the triangle's offsets
        const V sc = T::HALF ? __uint_as_float(sdv[jp].x) : V(1);
        V& hslot = hbuf[((ch & 1) * WF_CH + jj) * HRW + tid];
        V t = hslot;
        // all neighbour values first (one wait), then the chain of fmas
        V val[NT];
#pragma unroll
        for (int m = 0; m < NT; ++m) {
          const int so = DIR > 0 ? m : C + 1 + m;
          const int dx = pat_off(PAT, so, 0), dy = pat_off(PAT, so, 1), dz = pat_off(PAT, so, 2);
          if (dx == 0 && dy == 0) {
            val[m] = own_prev;
          } else {
            const int c = col_of(DIR * dx, DIR * dy);
            const int back = DIR * (WX * dx + WY * dy + dz);  // in [-KB, -1]
            val[m] = ring[((j + back + WF_HIST) % WF_HIST) * RW + nidx[c]];
          }
        }
#pragma unroll
        for (int m = 0; m < NT; ++m) {
          const V cm = T::HALF ? sc * T::get(cf[jp], m) : T::get(cf[jp], m);
          t = fma(-cm, val[m], t);
        }
        const V dv = T::HALF ? __uint_as_float(sdv[jp].y) : T::get(cf[jp], NT);
        const V xv = UNITD ? t : t * dv;
        const V xr = act ? xv : V(0);
        own_prev = xr;
        ring[j * RW + tid] = xr;
        hslot = xr;
        // columns read by other tiles leave at once, device-coherently
        bst<WF_SC1>(xv, rx, exported && act ? (vo + (unsigned)z) * (unsigned)sizeof(V) : WF_OOB);
        halo_put(k + 1, (j + 1) % PH);
        halo_fetch(k + PH, j % PH);
        prefetch(k + P, jp);
        __syncthreads();
      }
    }
    // the last chunk's results
    {
      const int cl = nsteps / WF_CH - 1;
#pragma unroll
      for (int i = 0; i < WF_TX; ++i) xrun_out(cl, i);
      if (ADD) add_out(cl);
    }
  }
}

// The last workgroup to finish resets the ticket counters for the next launch.
__device__ inline void wf_retire(unsigned* ctr) {
  if (threadIdx.x == 0) {
    unsigned o = atomicAdd(&ctr[1], 1u);
    if (o == gridDim.x - 1) {
      __hip_atomic_store(&ctr[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctr[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__device__ inline unsigned wf_take_ticket(unsigned* ctr) {
  __shared__ unsigned s_ticket;
  if (threadIdx.x == 0) s_ticket = atomicAdd(&ctr[0], 1u);
  __syncthreads();
  const unsigned t = s_ticket;
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(t);
}

// One sweep over one grid: persistent workgroups take tiles by ticket.
template <int PAT, int DIR, int P, class E, bool UNITD, bool ADD>
__global__ __launch_bounds__(WF_NL) void k_wavefront(WfArgs<typename WfVal<E>::V> a) {
  const unsigned ntiles = (unsigned)(a.t.ntx * a.t.nty);
  for (;;) {
    const unsigned ticket = wf_take_ticket(a.ctr);
    if (ticket >= ntiles) break;
    wf_tile<PAT, DIR, P, E, UNITD, ADD>(a, DIR > 0 ? ticket : ntiles - 1u - ticket, a.err);
  }
  wf_retire(a.ctr);
}

// One sweep over many independent grids of the same pattern and precision in
// one launch.  Ticket k names entry tmap[k] = (segment << 20) | r: the r-th
// tile of segment seg in that segment's own dependence order, so every
// tile's producers hold smaller tickets whatever the merge of the segments.
template <int PAT, int DIR, int P, class E, bool UNITD, bool ADD>
__global__ __launch_bounds__(WF_NL) void k_wavefront_group(const WfArgs<typename WfVal<E>::V>* __restrict__ segs,
                                                           const unsigned* __restrict__ tmap, unsigned total,
                                                           const int* __restrict__ live, unsigned* ctr,
                                                           unsigned* err) {
  for (;;) {
    const unsigned ticket = wf_take_ticket(ctr);
    if (ticket >= total) break;
    const unsigned e = __builtin_amdgcn_readfirstlane(tmap[ticket]);
    const WfArgs<typename WfVal<E>::V> a = segs[e >> 20];
    if (live != nullptr && live[a.sys] == 0) continue;
    const unsigned r = e & 0xFFFFFu, nt = (unsigned)(a.t.ntx * a.t.nty);
    wf_tile<PAT, DIR, P, E, UNITD, ADD>(a, DIR > 0 ? r : nt - 1u - r, err);
  }
  wf_retire(ctr);
}

// ---------------------------------------------------------------------------
// Builds the packed schedule-ordered sweep data of one direction.  Position
// q = (tile*NS + s)*NL + lane holds the point handled there (or none); its
// element e of pack p is entry p*K + e of the list [triangle coefficients in
// canonical order, diagonal scaling] (lower triangle for dir > 0, upper for
// dir < 0); missing entries are zero.
__device__ inline long wf_point(const Grid& g, const WfTiling& tl, int pat, long q) {
  const int l = (int)(q % WF_NL);
  const long r = q / WF_NL;
  const int s = (int)(r % tl.ns);
  const int tile = (int)(r / tl.ns);
  const int X = tile / tl.nty, Y = tile % tl.nty;
  const int lx = l / WF_TY, ly = l % WF_TY;
  const int x = X * WF_TX + lx, y = Y * WF_TY + ly - tl.sh * lx;
  const int z = s - ((hp_wx(pat) - tl.sh * hp_wy(pat)) * lx + hp_wy(pat) * ly + wf_kb(pat));
  const bool v = x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
  return v ? ((long)x * g.ny + y) * g.nz + z : -1;
}

template <class E>
__device__ inline E to_e(double v);
template <>
__device__ inline double to_e<double>(double v) {
  return v;
}
template <>
__device__ inline float to_e<float>(double v) {
  return (float)v;
}

template <int PAT, class E>
__global__ __launch_bounds__(256) void k_wf_pack(Grid g, WfTiling tl, int dir, const double* __restrict__ lo,
                                                 const double* __restrict__ dg, const double* __restrict__ up,
                                                 E* __restrict__ out) {
  constexpr int C = PAT / 2, NT = PAT / 2, K = 16 / (int)sizeof(E), NPK = wf_npk(PAT, sizeof(E));
  const long q = (long)blockIdx.x * 256 + threadIdx.x;
  if (q >= tl.nsk) return;
  const long i = wf_point(g, tl, PAT, q);
  const long N = g.N();
  const long row = q / WF_NL;
  const int lane = (int)(q % WF_NL);
  // positions without a point read point 0 and store zeros: every load is
  // unconditional and all of them come before the first store, so a
  // thread's loads are in flight together
  const long ic = i >= 0 ? i : 0;
  E v[NPK * K];
#pragma unroll
  for (int m = 0; m < NPK * K; ++m) {
    double x = 0.0;
    if (m < NT) x = (dir > 0 ? lo + (long)m * N : up + (long)(C + 1 + m) * N)[ic];
    if (m == NT) x = dg[ic];
    v[m] = to_e<E>(i >= 0 ? x : 0.0);
  }
#pragma unroll
  for (int p = 0; p < NPK; ++p) {
    E* o = out + ((row * NPK + p) * WF_NL + lane) * K;
#pragma unroll
    for (int e = 0; e < K; ++e) o[e] = v[p * K + e];
  }
}

// FP16 storage: the halves of the natural FP16 matrix, and (dir > 0 call)
// the pair {row scale, diagonal scaling} per position.
template <int PAT>
__global__ __launch_bounds__(256) void k_wf_pack_h(Grid g, WfTiling tl, int dir, const __half* __restrict__ a16,
                                                   const float* __restrict__ sc, const float* __restrict__ rd,
                                                   __half* __restrict__ out, float* __restrict__ sd) {
  constexpr int C = PAT / 2, NT = PAT / 2, K = 8, NPK = wf_npk(PAT, 2);
  const long q = (long)blockIdx.x * 256 + threadIdx.x;
  if (q >= tl.nsk) return;
  const long i = wf_point(g, tl, PAT, q);
  const long N = g.N();
  const long row = q / WF_NL;
  const int lane = (int)(q % WF_NL);
  // unconditional loads (point 0 for positions without a point), all before
  // the first store
  const long ic = i >= 0 ? i : 0;
  __half v[NPK * K];
#pragma unroll
  for (int m = 0; m < NPK * K; ++m) {
    __half x = __float2half_rn(0.0f);
    if (m < NT) x = (a16 + (long)(dir > 0 ? m : C + 1 + m) * N)[ic];
    v[m] = i >= 0 ? x : __float2half_rn(0.0f);
  }
  const float s0 = sc[ic], s1 = rd[ic];
#pragma unroll
  for (int p = 0; p < NPK; ++p) {
    __half* o = out + ((row * NPK + p) * WF_NL + lane) * K;
#pragma unroll
    for (int e = 0; e < K; ++e) o[e] = v[p * K + e];
  }
  if (dir > 0) {
    sd[2 * q] = i >= 0 ? s0 : 0.0f;
    sd[2 * q + 1] = i >= 0 ? s1 : 0.0f;
  }
}

template <class E>
hipError_t launch_wf_pack(int pat, const Grid& g, const WfTiling& tl, int dir, const double* lo, const double* dg,
                          const double* up, E* out, hipStream_t st) {
  const dim3 grid((unsigned)((tl.nsk + 255) / 256)), blk(256);
  if (pat == 7)
    hipLaunchKernelGGL((k_wf_pack<7, E>), grid, blk, 0, st, g, tl, dir, lo, dg, up, out);
  else if (pat == 19)
    hipLaunchKernelGGL((k_wf_pack<19, E>), grid, blk, 0, st, g, tl, dir, lo, dg, up, out);
  else if (pat == 27)
    hipLaunchKernelGGL((k_wf_pack<27, E>), grid, blk, 0, st, g, tl, dir, lo, dg, up, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
template hipError_t launch_wf_pack<double>(int, const Grid&, const WfTiling&, int, const double*, const double*,
                                           const double*, double*, hipStream_t);
template hipError_t launch_wf_pack<float>(int, const Grid&, const WfTiling&, int, const double*, const double*,
                                          const double*, float*, hipStream_t);

hipError_t launch_wf_pack_h(int pat, const Grid& g, const WfTiling& tl, int dir, const __half* a16, const float* sc,
                            const float* rd, __half* out, float* sd, hipStream_t st) {
  const dim3 grid((unsigned)((tl.nsk + 255) / 256)), blk(256);
  if (pat == 7)
    hipLaunchKernelGGL((k_wf_pack_h<7>), grid, blk, 0, st, g, tl, dir, a16, sc, rd, out, sd);
  else if (pat == 19)
    hipLaunchKernelGGL((k_wf_pack_h<19>), grid, blk, 0, st, g, tl, dir, a16, sc, rd, out, sd);
  else if (pat == 27)
    hipLaunchKernelGGL((k_wf_pack_h<27>), grid, blk, 0, st, g, tl, dir, a16, sc, rd, out, sd);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <int PAT, int DIR, int P, class E, bool UNITD, bool ADD>
static hipError_t launch_wf_t(const WfArgs<typename WfVal<E>::V>& a, hipStream_t st) {
  const unsigned ntiles = (unsigned)(a.t.ntx * a.t.nty);
  const unsigned grid = ntiles < (unsigned)WF_MAX_GRID ? ntiles : (unsigned)WF_MAX_GRID;
  hipLaunchKernelGGL((k_wavefront<PAT, DIR, P, E, UNITD, ADD>), dim3(grid), dim3(WF_NL), 0, st, a);
  return hipGetLastError();
}

template <int PAT, int DIR, int P, class E, bool UNITD, bool ADD>
static hipError_t launch_wfg_t(const WfArgs<typename WfVal<E>::V>* segs, const unsigned* tmap, unsigned total,
                               unsigned grid, const int* live, unsigned* ctr, unsigned* err, hipStream_t st) {
  hipLaunchKernelGGL((k_wavefront_group<PAT, DIR, P, E, UNITD, ADD>), dim3(grid), dim3(WF_NL), 0, st, segs, tmap,
                     total, live, ctr, err);
  return hipGetLastError();
}

template <class E>
hipError_t launch_wavefront_group(int pat, int dir, const WfArgs<typename WfVal<E>::V>* segs, const unsigned* tmap,
                                  unsigned total, unsigned grid, const int* live, unsigned* ctr, unsigned* err,
                                  hipStream_t st) {
  if (total == 0) return hipSuccess;
  if (grid == 0 || grid > total) grid = total;
  if (pat == 7 && dir > 0) return launch_wfg_t<7, 1, 8, E, false, false>(segs, tmap, total, grid, live, ctr, err, st);
  if (pat == 7 && dir < 0) return launch_wfg_t<7, -1, 8, E, false, false>(segs, tmap, total, grid, live, ctr, err, st);
  if (pat == 19 && dir > 0) return launch_wfg_t<19, 1, 4, E, false, false>(segs, tmap, total, grid, live, ctr, err, st);
  if (pat == 19 && dir < 0) return launch_wfg_t<19, -1, 4, E, false, false>(segs, tmap, total, grid, live, ctr, err, st);
  if (pat == 27 && dir > 0) return launch_wfg_t<27, 1, 4, E, false, false>(segs, tmap, total, grid, live, ctr, err, st);
  if (pat == 27 && dir < 0) return launch_wfg_t<27, -1, 4, E, false, false>(segs, tmap, total, grid, live, ctr, err, st);
  return hipErrorInvalidValue;
}
template hipError_t launch_wavefront_group<double>(int, int, const WfArgs<double>*, const unsigned*, unsigned,
                                                   unsigned, const int*, unsigned*, unsigned*, hipStream_t);
template hipError_t launch_wavefront_group<float>(int, int, const WfArgs<float>*, const unsigned*, unsigned, unsigned,
                                                  const int*, unsigned*, unsigned*, hipStream_t);
template hipError_t launch_wavefront_group<__half>(int, int, const WfArgs<float>*, const unsigned*, unsigned,
                                                   unsigned, const int*, unsigned*, unsigned*, hipStream_t);

template <class E>
hipError_t launch_wavefront(int pat, int dir, bool unitd, bool add, const WfArgs<typename WfVal<E>::V>& a,
                            hipStream_t st) {
#define SMG_WF_CASE(PATV, PV)                                                                  \
  if (pat == PATV) {                                                                           \
    if (dir > 0 && !unitd && !add) return launch_wf_t<PATV, 1, PV, E, false, false>(a, st);    \
    if (dir < 0 && !unitd && !add) return launch_wf_t<PATV, -1, PV, E, false, false>(a, st);   \
    if (dir > 0 && unitd && !add) return launch_wf_t<PATV, 1, PV, E, true, false>(a, st);      \
    if (dir < 0 && !unitd && add) return launch_wf_t<PATV, -1, PV, E, false, true>(a, st);     \
  }
  SMG_WF_CASE(7, 8)
  SMG_WF_CASE(19, 4)
  SMG_WF_CASE(27, 4)
#undef SMG_WF_CASE
  return hipErrorInvalidValue;
}

template hipError_t launch_wavefront<double>(int, int, bool, bool, const WfArgs<double>&, hipStream_t);
template hipError_t launch_wavefront<float>(int, int, bool, bool, const WfArgs<float>&, hipStream_t);
template hipError_t launch_wavefront<__half>(int, int, bool, bool, const WfArgs<float>&, hipStream_t);

}  // namespace smg
