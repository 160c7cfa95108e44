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
//  * The z-column is the unit.  A workgroup owns a TX x TY tile of columns:
//    tile (X, Y) holds x in [X*TX, X*TX+TX) and y + sh*(x - X*TX) in
//    [Y*TY, Y*TY+TY) (sheared so that no dependence points from a tile to a
//    later one).
//  * Column (lx, ly) of the tile handles point z at step s = z + skew(lx, ly),
//    skew = (wx - sh*wy)*lx + wy*ly + KB with the hyperplane weights
//    (wx, wy, 1) of the pattern; a neighbour at offset (dx, dy, dz) is then
//    handled exactly wx*dx + wy*dy + dz steps away, the same for every
//    column, which is earlier for every lower neighbour.  A backward sweep
//    runs the same tiles and steps in reverse order.  KB pads both ends of
//    the step range so that values referenced at the first and last steps
//    have a step.
//  * A step costs the time a wave needs to issue its instructions (one per
//    four cycles at best) plus one exchange of values through LDS, so the
//    workgroup splits the work by role, each role in waves of its own, and
//    all waves meet at one workgroup barrier per step:
//      - four compute waves, one column per lane: per step they read the
//        right-hand side and the neighbours' values from LDS, run the chain
//        of fmas, write the result to LDS, and prefetch the step's packed
//        coefficients (a schedule-ordered copy, 16-byte coalesced loads,
//        P steps ahead) -- about twenty instructions, no global stores and
//        no waits on memory other than their own coefficient loads;
//      - a halo wave: fetches the values of neighbouring tiles' columns
//        (device-coherent loads PH steps ahead, checked against the
//        sentinel) into the LDS ring;
//      - a load wave: streams the right-hand side into LDS as runs of 16
//        consecutive z per column, two chunks of 16 steps ahead;
//      - a store wave: stores the tile's own columns that other tiles read
//        (device-coherent, one step after they are computed), and streams
//        the results out of LDS as runs one chunk behind, together with the
//        sentinels for the next sweep on the level.
//    Loads and stores never share a wave: a wave's vector memory operations
//    retire in issue order, so a wave that waits for a load would also wait
//    for every store issued before it, whose acknowledgement is slow.
//    Values that cross waves move through an LDS ring of 16 steps (the tile's
//    columns plus a halo of neighbouring tiles' columns) and three chunk
//    buffers (one filled, one computed, one drained).
//  * Inactive positions (a column outside the grid, or z outside [0, nz) at
//    that step) have zero coefficients, scaling and right-hand side, so
//    their result is zero without a test: the LDS is zeroed once per launch
//    and every value in it stays finite.
//  * Every position read by another tile holds a signalling-NaN sentinel
//    until it is written; a value is ready when it is no longer the
//    sentinel.  The sentinels for the next sweep on the same level are
//    written by this sweep into that sweep's output.
//  * A halo wave that finds a value not yet written first waits for the value
//    WF_AHEAD steps further along the same column and then refetches its
//    other prefetched halo values: the tile then runs far enough behind its
//    producer that later prefetches find their values written, instead of
//    paying one coherent round trip per step.
//  * Tiles are handed out by an atomic ticket in dependence order, so a
//    persistent grid of any size always makes progress.  Waits are bounded
//    by a watchdog that raises an error flag instead of hanging.
//  * All per-point accesses use buffer instructions; positions without a
//    point use an offset outside the buffer, for which loads return zero
//    and stores are dropped.
#include "smg_common.h"
#include "smg_group.h"
#include "smg_kernels.h"

namespace smg {

constexpr int WF_HIST = 16;                  // LDS ring rows (steps)
constexpr int WF_CH = 16;                    // steps per chunk of right-hand side / results
constexpr int WF_NL = WF_TX * WF_TY;         // compute lanes (columns) per tile
constexpr int WF_NH = 104;                   // halo slots around a tile
constexpr int WF_NB = 3;                     // chunk buffers: filled, computed, drained
constexpr int WF_NW = 7;                     // waves: 4 compute, halo, load, store
constexpr int WF_THREADS = 64 * WF_NW;
constexpr int WF_GRP = WF_NL * WF_CH / 64;   // column-run groups per chunk (4 columns x 16 steps)
constexpr int WF_GPS = WF_GRP / WF_CH;       // groups moved per step
constexpr int WF_RW = WF_NL + WF_NH + 1;     // ring row length (padded)
constexpr int WF_HRW = WF_NL + 1;            // chunk buffer row length (padded)
constexpr unsigned WF_SPIN_LIMIT = 1u << 21;
#ifndef WF_LAG_EXTRA
#define WF_LAG_EXTRA 2
#endif
#ifndef WF_PH
#define WF_PH 4
#endif
constexpr unsigned WF_OOB = 0x80000000u;     // buffer offset outside every range
constexpr int WF_SC1 = 16;                   // cache policy of device-coherent accesses

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
// FP16 storage: do the position's FP32 {row scale, diagonal scaling} fit in
// the last two words of its packs (after the pattern's lower halves)?  Then a
// step loads them with the coefficients (7- and 19-point: one load per step
// instead of two); otherwise (27-point) they come from a separate array.
__host__ __device__ constexpr bool wf_sd_in_pack(int pat) { return pat / 2 + 4 <= 8 * wf_npk(pat, 2); }

void wf_tiling(const Grid& g, int pat, WfTiling* t, int shape) {
  // Default: tiles are sheared (y + x offset) when a lower neighbour column
  // lies at (x-1, y+1) (19- and 27-point patterns), so that every dependence
  // points to an earlier tile in x and y; otherwise, and when a single tile
  // row covers y, plain rectangles, which give fewer tile hand-offs on the
  // critical path.  Shears are valid for every pattern (a point's step is its
  // hyperplane index minus a per-tile offset either way).  Rectangles are not
  // for 19/27-point sweeps with more than one tile row: column (x, y) of a
  // tile's top row then reads (x-1, y+1) in the tile above, which reads the
  // tile below through (x, y-1), and two tiles waiting on each other stall
  // (retile_level refuses that case).  shape 1 / 2 forces sheared /
  // rectangular tiles.
  t->sh = shape == 1 ? 1 : (shape == 2 ? 0 : ((pat == 7 || g.ny <= WF_TY) ? 0 : 1));
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
  // the row-scaled coefficient float(h_m) * sc in one instruction
  __device__ static float scaled(const u32x4* pk, int m, float sc) {
    const unsigned w = pk[m / 8][(m % 8) / 2];
    return m % 2 == 0 ? half_times<0>(w, sc) : half_times<1>(w, sc);
  }
};

// Columns of a tile that no lane of another tile reads in a sweep of
// direction dir: the lanes whose consumers (lane - neighbour-column offset,
// sheared) all lie inside the tile, an intersection of shifted copies of the
// tile, hence a rectangle [xl, xh) x [yl, yh).
struct WfRect {
  int xl, xh, yl, yh;
};
__host__ __device__ constexpr WfRect wf_inner(int pat, int dir, int sh) {
  WfRect r{0, WF_TX, 0, WF_TY};
  for (int c = 0; c < 4; ++c) {
    if (!col_used(pat, c)) continue;
    const int cx = dir * col_dx(c), cy = dir * col_dy(c) + sh * dir * col_dx(c);
    r.xl = r.xl > cx ? r.xl : cx;
    r.xh = r.xh < WF_TX + cx ? r.xh : WF_TX + cx;
    r.yl = r.yl > cy ? r.yl : cy;
    r.yh = r.yh < WF_TY + cy ? r.yh : WF_TY + cy;
  }
  return r;
}
__host__ __device__ constexpr int wf_exported_count(const WfRect& r) {
  return WF_NL - (r.xh - r.xl) * (r.yh - r.yl);
}
// Lane (lx*TY + ly) of the e-th column outside the rectangle, in lane order.
__device__ inline int wf_exported_lane(const WfRect& r, int e) {
  const int nm = WF_TY - (r.yh - r.yl);  // outside columns per row inside [xl, xh)
  int lx, ly;
  if (e < WF_TY * r.xl) {
    lx = e / WF_TY;
    ly = e % WF_TY;
  } else if (e < WF_TY * r.xl + nm * (r.xh - r.xl)) {
    const int q = e - WF_TY * r.xl;
    lx = r.xl + q / nm;
    const int w = q % nm;
    ly = w < r.yl ? w : r.yh + (w - r.yl);
  } else {
    const int q = e - WF_TY * r.xl - nm * (r.xh - r.xl);
    lx = r.xh + q / WF_TY;
    ly = q % WF_TY;
  }
  return lx * WF_TY + ly;
}

// Geometry of one tile shared by all roles.
struct WfGeo {
  int X, Y, sh, NS, nsteps;
  int p0;             // first x plane of the vector buffers
  unsigned vbytes;    // bytes of the vector buffers (planes p0 .. p1-1)
  long vb;            // element offset of plane p0
};

template <class V>
__device__ inline WfGeo wf_geo(const WfArgs<V>& a, unsigned tile) {
  WfGeo q;
  q.X = (int)(tile / (unsigned)a.t.nty);
  q.Y = (int)(tile % (unsigned)a.t.nty);
  q.sh = a.t.sh;
  q.NS = a.t.ns;
  q.nsteps = (q.NS + WF_CH - 1) / WF_CH * WF_CH;
  q.p0 = q.X * WF_TX > 0 ? q.X * WF_TX - 1 : 0;
  const int p1 = q.X * WF_TX + WF_TX + 1 < a.g.nx ? q.X * WF_TX + WF_TX + 1 : a.g.nx;
  const long pl = (long)a.g.ny * a.g.nz;
  q.vbytes = (unsigned)((p1 - q.p0) * pl * (long)sizeof(V));
  q.vb = q.p0 * pl;
  return q;
}

template <int DIR>
__device__ inline int wf_step(int NS, int k) {
  return DIR > 0 ? k : NS - 1 - k;
}

// ---- compute role (waves 0-3) ----------------------------------------------
template <int PAT, int DIR, int P, class E, bool UNITD>
__device__ __forceinline__ void wf_compute(const WfArgs<typename WfVal<E>::V>& a, const WfGeo& q, unsigned tile,
                                           typename WfVal<E>::V* ring, typename WfVal<E>::V* hbuf) {
  using T = WfE<E>;
  using V = typename T::V;
  constexpr int C = PAT / 2;
  constexpr int NT = PAT / 2;
  constexpr int WX = hp_wx(PAT), WY = hp_wy(PAT);
  constexpr int NPK = wf_npk(PAT, sizeof(E));
  constexpr unsigned PACKB = WF_NL * 16u;
  static_assert(WF_HIST % P == 0 && WF_HIST > wf_kb(PAT) + 1, "ring too short");
  const int tid = threadIdx.x;
  const int lx = tid / WF_TY, ly = tid % WF_TY;
  const int NS = q.NS;

  // LDS index of each neighbour column within a ring row (offsets mirrored
  // for a backward sweep): a lane of this tile or a halo slot
  int nidx[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int cx = DIR * col_dx(c), cy = DIR * col_dy(c);
    const int qx = lx + cx, qy = ly + cy + q.sh * cx;
    const bool in = qx >= 0 && qx < WF_TX && qy >= 0 && qy < WF_TY;
    nidx[c] = !col_used(PAT, c) ? 0 : (in ? qx * WF_TY + qy : WF_NL + wf_halo_slot(qx, qy));
  }
  const unsigned tbytes = (unsigned)NS * NPK * PACKB;
  const auto rp = wf_rsrc((const char*)a.pk + (size_t)tile * tbytes, tbytes);
  const unsigned sdbytes = T::HALF ? (unsigned)NS * WF_NL * 8u : 0u;
  const auto rs = wf_rsrc(T::HALF ? (const char*)a.sd + (size_t)tile * sdbytes : (const char*)a.pk, sdbytes);

  // Positions without a point (z outside [0, nz) or the column outside the
  // grid) take an offset outside the buffer: their coefficients read as zero
  // without a memory access, so the copy's padding costs no traffic.
  const int skew = (WX - q.sh * WY) * lx + WY * ly + wf_kb(PAT);
  const int xt = q.X * WF_TX + lx, yt = q.Y * WF_TY + ly - q.sh * lx;
  const unsigned zlim = xt < a.g.nx && yt >= 0 && yt < a.g.ny ? (unsigned)a.g.nz : 0u;
  u32x4 cf[P][NPK];
  u32x2 sdv[P];
  auto prefetch = [&](int k, int j) {
    const int s = wf_step<DIR>(NS, k);
    const bool sin = s >= 0 && s < NS;
    const unsigned so = sin ? (unsigned)s * (NPK * PACKB) : WF_OOB;
    const bool pt = (unsigned)(s - skew) < zlim;
    const unsigned vo = pt ? tid * 16u : WF_OOB;
#pragma unroll
    for (int p = 0; p < NPK; ++p)
      cf[j][p] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rp, vo, so + p * PACKB, 0));
    if (T::HALF && !wf_sd_in_pack(PAT))
      sdv[j] = __builtin_amdgcn_raw_buffer_load_b64(rs, pt ? tid * 8u : WF_OOB,
                                                    sin ? (unsigned)s * (WF_NL * 8u) : WF_OOB, 0);
  };
#pragma unroll
  for (int j = 0; j < P; ++j) prefetch(j, j);
  V own_prev = V(0);
  __syncthreads();  // prologue: the first chunk is in LDS

  for (int k0 = 0; k0 < q.nsteps; k0 += WF_HIST) {
    V* hb = hbuf + ((k0 / WF_CH) % WF_NB) * (WF_CH * WF_HRW) + tid;
#pragma unroll
    for (int j = 0; j < WF_HIST; ++j) {
      const int jp = j % P;
      constexpr bool SDP = T::HALF && wf_sd_in_pack(PAT);
      const V sc = T::HALF ? __uint_as_float(SDP ? cf[jp][NPK - 1][2] : sdv[jp].x) : V(1);
      V t = hb[j * WF_HRW];
      // all neighbour values first (one wait), then the chain of fmas in
      // canonical order of the triangle's offsets
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
          val[m] = ring[((j + back + WF_HIST) % WF_HIST) * WF_RW + nidx[c]];
        }
      }
#pragma unroll
      for (int m = 0; m < NT; ++m) {
        V cm;
        if constexpr (T::HALF)
          cm = T::scaled(cf[jp], m, sc);
        else
          cm = T::get(cf[jp], m);
        t = fma(-cm, val[m], t);
      }
      const V dv = T::HALF ? __uint_as_float(SDP ? cf[jp][NPK - 1][3] : sdv[jp].y) : T::get(cf[jp], NT);
      const V xv = UNITD ? t : t * dv;
      own_prev = xv;
      ring[j * WF_RW + tid] = xv;
      hb[j * WF_HRW] = xv;
      prefetch(k0 + j + P, jp);
      __syncthreads();
    }
  }
  __syncthreads();  // tail: the last chunk is drained and the last step exported
  __syncthreads();
}

// ---- halo role (wave 4) ------------------------------------------------------
template <int PAT, int DIR, class V>
__device__ __forceinline__ void wf_halo(const WfArgs<V>& a, const WfGeo& q, V* ring, unsigned* err) {
  using B = VBits<V>;
  constexpr int WX = hp_wx(PAT), WY = hp_wy(PAT);
  constexpr int KB = wf_kb(PAT);
  constexpr int PH = WF_PH;
  constexpr int WF_AHEAD = PH + WF_LAG_EXTRA;  // steps a stalled tile falls back behind its producer
  static_assert(WF_HIST % PH == 0 && PH >= 2, "halo prefetch distance");
  const int t = threadIdx.x - 4 * 64;
  const int NS = q.NS, nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const long vb = q.vb;
  const auto rx = wf_rsrc(a.x + vb, q.vbytes);

  // halo slots t and 64 + t
  bool hrole[2];
  int hs[2], hskew[2];
  unsigned hvo[2];
  bool hcolv[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    hs[i] = t + 64 * i;
    int hqx = 0, hqy = 0;
    hrole[i] = false;
    if (hs[i] < WF_NH) {
      wf_halo_pos(hs[i], &hqx, &hqy);
      hrole[i] = wf_halo_used(PAT, DIR, q.sh, hqx, hqy);
    }
    hskew[i] = (WX - q.sh * WY) * hqx + WY * hqy + KB;
    const int gx = q.X * WF_TX + hqx, gy = q.Y * WF_TY + hqy - q.sh * hqx;
    hcolv[i] = hrole[i] && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    hvo[i] = hcolv[i] ? (unsigned)(((gx - q.p0) * (long)ny + gy) * nz) : 0u;
  }
  V hb[2][PH];
  auto halo_off = [&](int i, int k) {
    const int s = wf_step<DIR>(NS, k);
    const int hz = s - hskew[i];
    const bool ok = s >= 0 && s < NS && hcolv[i] && hz >= 0 && hz < nz;
    return ok ? (hvo[i] + (unsigned)hz) * (unsigned)sizeof(V) : WF_OOB;
  };
  auto halo_fetch = [&](int k, int j) {
#pragma unroll
    for (int i = 0; i < 2; ++i) hb[i][j] = bld<V, WF_SC1>(rx, halo_off(i, k));
  };
  // Bounded wait until the value at byte offset off is no longer the
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
  // halo values of step k (slot j): wait for any that is still the sentinel,
  // then publish them in ring row k
  auto halo_put = [&](int k, int j) {
    bool miss = false;
#pragma unroll
    for (int i = 0; i < 2; ++i) miss |= B::bits(hb[i][j]) == B::sent;
    if (__builtin_amdgcn_ballot_w64(miss) != 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (B::bits(hb[i][j]) == B::sent) {
          // fall back behind the producer: wait for the value WF_AHEAD steps
          // on (clamped to the column), then for this one
          const int s = wf_step<DIR>(NS, k);
          const int hz = s - hskew[i];
          int zf = hz + DIR * WF_AHEAD;
          zf = zf < 0 ? 0 : (zf >= nz ? nz - 1 : zf);
          const unsigned offf = (hvo[i] + (unsigned)zf) * (unsigned)sizeof(V);
          wait_value(offf, bld<V, WF_SC1>(rx, offf));
          hb[i][j] = wait_value(halo_off(i, k), hb[i][j]);
        }
      }
      // the other prefetched halo values were fetched too early: fetch again
#pragma unroll
      for (int d = 1; d < PH; ++d) halo_fetch(k + d, (j + d) % PH);
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the refetched values are in
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
      if (hrole[i]) ring[(k % WF_HIST) * WF_RW + WF_NL + hs[i]] = hb[i][j];
  };
#pragma unroll
  for (int j = 0; j < PH; ++j) halo_fetch(j, j);
  __syncthreads();  // prologue

  for (int k0 = 0; k0 < q.nsteps; k0 += WF_HIST) {
#pragma unroll
    for (int j = 0; j < WF_HIST; ++j) {
      const int k = k0 + j;
      halo_put(k, j % PH);
      halo_fetch(k + PH, j % PH);
      __syncthreads();
    }
  }
  __syncthreads();
  __syncthreads();
}

// ---- column runs (load and store roles) --------------------------------------
// Group r of a chunk moves columns 4r + cq (cq = lane / 16), steps m = lane %
// 16 of the chunk: each column's 16 consecutive z values are one coalesced run.
// Per chunk a lane forms its base offsets once, per step the step's bases; a
// group then adds a uniform term.  The bases pass through wf_keep, which the
// compiler may not move across the step's memory operations, so that it does
// not compute every step's offsets ahead (they would hold dozens of
// registers for the whole chunk or sweep).
__device__ inline int wf_keep(int v) {
  asm volatile("" : "+v"(v) : : "memory");
  return v;
}
__device__ inline int wf_keep_s(int v) {
  asm volatile("" : "+s"(v) : : "memory");
  return v;
}

template <int PAT, int DIR, class V>
struct WfRuns {
  static constexpr int WX = hp_wx(PAT), WY = hp_wy(PAT), KB = wf_kb(PAT);
  int cq, m;
  int lds;        // LDS index of (step m, column cq) within a chunk buffer
  int a0;         // element offset of column cq of group 0 minus its skew
  int y0;         // y of column cq of group 0
  int skq;        // skew of column cq of group 0
  int gx, gy;     // element offset steps per group row (r / 4) and per group (r % 4)
  int sx;         // skew step per group row
  int nx;
  __device__ void init(const WfArgs<V>& a, const WfGeo& q, int lane) {
    nx = a.g.nx;
    cq = lane / 16;
    m = lane % 16;
    lds = m * WF_HRW + cq;
    const int ny = a.g.ny, nz = a.g.nz;
    skq = WY * cq + KB;
    y0 = q.Y * WF_TY + cq;
    a0 = ((q.X * WF_TX - q.p0) * ny + y0) * nz - skq;
    sx = WX - q.sh * WY;
    gx = (ny - q.sh) * nz - sx;
    gy = 4 * (nz - WY);
  }
  // Per-chunk bases of this lane's step s of the chunk.
  struct Base {
    int e;    // element offset of group 0
    int z;    // z of group 0
    int gx, gy, sx;
  };
  __device__ Base base(int s) const { return Base{wf_keep(a0 + s), wf_keep(s - skq), wf_keep_s(gx), wf_keep_s(gy),
                                                  wf_keep_s(sx)}; }
  // Per-step bases: the four groups 4j .. 4j+3 moved at step j of a chunk
  // share the column row lx = j.
  struct Step {
    int e, z, y, lx;
  };
  __device__ Step step(const Base& b, const WfGeo& q, int j) const {
    // a column row beyond the grid in x takes y = -1 - 16 (outside for every group)
    const int y = q.X * WF_TX + j < nx ? y0 - q.sh * j : -WF_TY - 1;
    return Step{wf_keep(b.e + j * b.gx), wf_keep(b.z - j * b.sx), wf_keep(y), j};
  }
  // byte offset of group 4*lx + g with every position in the grid
  __device__ static unsigned off_in(const Base& b, const Step& t, int g) {
    return (unsigned)(t.e + g * b.gy) * (unsigned)sizeof(V);
  }
  // byte offset of group 4*lx + g, or WF_OOB where the position is outside the grid
  __device__ static unsigned off_any(const WfArgs<V>& a, const WfGeo& q, const Base& b, const Step& t, int g) {
    const int yt = t.y + 4 * g;
    const int z = t.z - 4 * WY * g;
    const bool ok = (unsigned)yt < (unsigned)a.g.ny && (unsigned)z < (unsigned)a.g.nz;
    return ok ? off_in(b, t, g) : WF_OOB;
  }
};

// ---- load role (wave 5): right-hand side, two chunks ahead --------------------
template <int PAT, int DIR, class V>
__device__ __forceinline__ void wf_load(const WfArgs<V>& a, const WfGeo& q, V* hbuf) {
  using RU = WfRuns<PAT, DIR, V>;
  const int lane = threadIdx.x - 5 * 64;
  RU R;
  R.init(a, q, lane);
  const auto rh = wf_rsrc(a.h + q.vb, q.vbytes);
  V reg[WF_GRP];
  // Per step j of a chunk: the registers of groups 4j .. 4j+3 (a chunk's
  // runs) go to the chunk buffer hb, then take the runs of the chunk with
  // bases b.
  auto advance = [&](V* hb, const typename RU::Base& b, bool sync) {
#pragma unroll
    for (int j = 0; j < WF_HIST; ++j) {
#pragma unroll
      for (int g = 0; g < WF_GPS; ++g) hb[4 * (j * WF_GPS + g)] = reg[j * WF_GPS + g];
      const typename RU::Step t = R.step(b, q, j);
#pragma unroll
      for (int g = 0; g < WF_GPS; ++g) reg[j * WF_GPS + g] = bld<V, 0>(rh, RU::off_any(a, q, b, t, g));
      if (sync)
        __syncthreads();
      else
        __builtin_amdgcn_sched_barrier(0);  // keep the refill behind this step's LDS writes
    }
  };
  auto bases = [&](int c) { return R.base(wf_step<DIR>(q.NS, c * WF_CH + R.m)); };
  // prologue: chunk 0 into buffer 0, chunk 1 into the registers
  {
    const typename RU::Base b = bases(0);
#pragma unroll
    for (int j = 0; j < WF_HIST; ++j) {
      const typename RU::Step t = R.step(b, q, j);
#pragma unroll
      for (int g = 0; g < WF_GPS; ++g) reg[j * WF_GPS + g] = bld<V, 0>(rh, RU::off_any(a, q, b, t, g));
    }
  }
  advance(hbuf + R.lds, bases(1), false);
  __syncthreads();

  for (int k0 = 0; k0 < q.nsteps; k0 += WF_HIST) {
    const int c = k0 / WF_CH;
    // chunk c+1's groups into LDS, then chunk c+2's into the registers freed
    advance(hbuf + ((c + 1) % WF_NB) * (WF_CH * WF_HRW) + R.lds, bases(c + 2), true);
  }
  __syncthreads();
  __syncthreads();
}

// ---- store role (wave 6): exports, results one chunk behind, sentinels -------
template <int PAT, int DIR, class V>
__device__ __forceinline__ void wf_store(const WfArgs<V>& a, const WfGeo& q, const V* ring, V* hbuf) {
  using B = VBits<V>;
  using RU = WfRuns<PAT, DIR, V>;
  constexpr int WX = hp_wx(PAT), WY = hp_wy(PAT), KB = wf_kb(PAT);
  const int lane = threadIdx.x - 6 * 64;
  const int NS = q.NS, nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  RU R;
  R.init(a, q, lane);
  const auto rx = wf_rsrc(a.x + q.vb, q.vbytes);
  const auto rn = wf_rsrc((a.next != nullptr ? a.next : a.x) + q.vb, a.next != nullptr ? q.vbytes : 0u);
  // Columns read by other tiles in this sweep (exported below) and in the
  // next sweep (given the sentinel) lie outside the inner rectangles.  Bit r
  // of xm / nm: is column 4r + cq outside (its run store dropped / its
  // sentinel written)?  A set bit 31 puts an offset outside the buffer.
  const WfRect ix = wf_inner(PAT, DIR, q.sh);
  const WfRect inx = wf_inner(PAT, a.next_dir, q.sh);
  unsigned long long xm = 0, nm = 0;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int ly = 4 * g + R.cq;
    xm |= (ly < ix.yl || ly >= ix.yh) ? 0x1111111111111111ull << g : 0ull;
    nm |= (ly < inx.yl || ly >= inx.yh) ? 0x1111111111111111ull << g : 0ull;
  }
#pragma unroll
  for (int lx = 0; lx < WF_TX; ++lx) {
    xm |= (lx < ix.xl || lx >= ix.xh) ? 0xFull << (4 * lx) : 0ull;
    nm |= (lx < inx.xl || lx >= inx.xh) ? 0xFull << (4 * lx) : 0ull;
  }
  const unsigned xm0 = (unsigned)xm, xm1 = (unsigned)(xm >> 32);
  const unsigned nm0 = ~(unsigned)nm, nm1 = ~(unsigned)(nm >> 32);  // set: no sentinel
  // does group r hold a column that gets the sentinel (the same for all lanes)?
  auto gsent = [&](int r) {
    const int lx = r / 4, g = r % 4;
    return lx < inx.xl || lx >= inx.xh || 4 * g < inx.yl || 4 * g + 3 >= inx.yh;
  };
  auto bit31 = [](unsigned w, int r) { return ((w >> (r % 32)) & 1u) << 31; };
  auto put = [&](unsigned off, int r, const V* hb, bool nxt) {
    const V v = hb[4 * r];
    bst<0>(v, rx, off | bit31(r < 32 ? xm0 : xm1, r));
    if (nxt && gsent(r)) bst<0>(B::val(B::sent), rn, off | bit31(r < 32 ? nm0 : nm1, r));
  };
  // exported column `lane` (in lane order) of the tile
  const bool erole = lane < wf_exported_count(ix);
  const int el = erole ? wf_exported_lane(ix, lane) : 0;
  const int elx = el / WF_TY, ely = el % WF_TY;
  const int exx = q.X * WF_TX + elx, eyy = q.Y * WF_TY + ely - q.sh * elx;
  const bool ecolv = erole && exx < nx && eyy >= 0 && eyy < ny;
  const unsigned evo = ecolv ? (unsigned)(((exx - q.p0) * (long)ny + eyy) * nz) : 0u;
  const int eskew = (WX - q.sh * WY) * elx + WY * ely + KB;
  // the exported columns' values of step k (ring row j = k mod 16), device-coherently
  auto export_step = [&](int k, int j) {
    const int s = wf_step<DIR>(NS, k);
    const int z = s - eskew;
    const bool ok = ecolv && k >= 0 && s >= 0 && s < NS && z >= 0 && z < nz;
    const V v = ring[((j + WF_HIST) % WF_HIST) * WF_RW + el];
    bst<WF_SC1>(v, rx, ok ? (evo + (unsigned)z) * (unsigned)sizeof(V) : WF_OOB);
  };
  auto chunk = [&](int k0, const typename RU::Base& b, int mode, const V* hb) {
#pragma unroll
    for (int j = 0; j < WF_HIST; ++j) {
      export_step(k0 + j - 1, j - 1);
      if (mode > 0) {
        const typename RU::Step t = R.step(b, q, j);
#pragma unroll
        for (int g = 0; g < WF_GPS; ++g) put(RU::off_any(a, q, b, t, g), j * WF_GPS + g, hb, mode == 2);
      }
      __syncthreads();
    }
  };
  __syncthreads();  // prologue

  for (int k0 = 0; k0 < q.nsteps; k0 += WF_HIST) {
    const int c = k0 / WF_CH;
    const V* hb = hbuf + ((c + WF_NB - 1) % WF_NB) * (WF_CH * WF_HRW) + R.lds;
    const typename RU::Base b = R.base(wf_step<DIR>(q.NS, (c - 1) * WF_CH + R.m));
    if (c == 0)
      chunk(k0, b, 0, hb);
    else if (a.next != nullptr)
      chunk(k0, b, 2, hb);
    else
      chunk(k0, b, 1, hb);
  }
  __syncthreads();
  export_step(q.nsteps - 1, WF_HIST - 1);
  {
    const int c = q.nsteps / WF_CH - 1;
    const V* hb = hbuf + (c % WF_NB) * (WF_CH * WF_HRW) + R.lds;
    const typename RU::Base b = R.base(wf_step<DIR>(q.NS, c * WF_CH + R.m));
#pragma unroll 4
    for (int r = 0; r < WF_GRP; ++r) {
      const unsigned off = RU::off_any(a, q, b, R.step(b, q, r / 4), r % 4);
      const V v = hb[4 * r];
      const unsigned xw = r < 32 ? xm0 : xm1, nw = r < 32 ? nm0 : nm1;
      bst<0>(v, rx, off | (((xw >> (r % 32)) & 1u) << 31));
      if (a.next != nullptr) bst<0>(B::val(B::sent), rn, off | (((nw >> (r % 32)) & 1u) << 31));
    }
  }
  __syncthreads();
}

// The LDS of a sweep workgroup: the value ring and the chunk buffers, zeroed
// once per launch (inactive positions then compute zeros from zeros).
template <class V>
struct WfLds {
  V ring[WF_HIST * WF_RW];
  V hbuf[WF_NB * WF_CH * WF_HRW];
};
template <class V>
__device__ inline void wf_zero_lds(WfLds<V>* L) {
  constexpr int n = (int)(sizeof(WfLds<V>) / 4);
  unsigned* p = reinterpret_cast<unsigned*>(L);
  for (int i = threadIdx.x; i < n; i += WF_THREADS) p[i] = 0u;
  __syncthreads();
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

// Every role of a sweep workgroup runs its own loop over the workgroup's
// tiles (values a role keeps across tiles then stay out of the other roles'
// code); next(&a, &tile) takes the next ticket, the same for all waves.
template <int PAT, int DIR, int P, class E, bool UNITD, class Next>
__device__ __forceinline__ void wf_roles(Next next, unsigned* err, WfLds<typename WfVal<E>::V>* L) {
  using V = typename WfVal<E>::V;
  WfArgs<V> a;
  unsigned tile;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64);
  if (wave < 4) {
    while (next(&a, &tile)) wf_compute<PAT, DIR, P, E, UNITD>(a, wf_geo(a, tile), tile, L->ring, L->hbuf);
  } else if (wave == 4) {
    while (next(&a, &tile)) wf_halo<PAT, DIR, V>(a, wf_geo(a, tile), L->ring, err);
  } else if (wave == 5) {
    while (next(&a, &tile)) wf_load<PAT, DIR, V>(a, wf_geo(a, tile), L->hbuf);
  } else {
    while (next(&a, &tile)) wf_store<PAT, DIR, V>(a, wf_geo(a, tile), L->ring, L->hbuf);
  }
}

// One sweep over one grid: persistent workgroups take tiles by ticket.
template <int PAT, int DIR, int P, class E, bool UNITD>
__global__ __launch_bounds__(WF_THREADS) void k_wavefront(WfArgs<typename WfVal<E>::V> a) {
  using V = typename WfVal<E>::V;
  __shared__ WfLds<V> L;
  wf_zero_lds(&L);
  const unsigned ntiles = (unsigned)(a.t.ntx * a.t.nty);
  auto next = [&](WfArgs<V>* pa, unsigned* tile) {
    const unsigned ticket = wf_take_ticket(a.ctr);
    if (ticket >= ntiles) return false;
    *pa = a;
    *tile = DIR > 0 ? ticket : ntiles - 1u - ticket;
    return true;
  };
  wf_roles<PAT, DIR, P, E, UNITD>(next, a.err, &L);
  wf_retire(a.ctr);
}

// One sweep over many independent grids of the same pattern and precision in
// one launch.  Ticket k names entry tmap[k] = (segment << 20) | r: the r-th
// tile of segment seg in that segment's own dependence order, so every
// tile's producers hold smaller tickets whatever the merge of the segments.
template <int PAT, int DIR, int P, class E>
__global__ __launch_bounds__(WF_THREADS) void k_wavefront_group(const WfArgs<typename WfVal<E>::V>* __restrict__ segs,
                                                                const unsigned* __restrict__ tmap, unsigned total,
                                                                const int* __restrict__ live, unsigned* ctr,
                                                                unsigned* err) {
  using V = typename WfVal<E>::V;
  __shared__ WfLds<V> L;
  wf_zero_lds(&L);
  auto next = [&](WfArgs<V>* pa, unsigned* tile) {
    for (;;) {
      const unsigned ticket = wf_take_ticket(ctr);
      if (ticket >= total) return false;
      const unsigned e = __builtin_amdgcn_readfirstlane(tmap[ticket]);
      *pa = segs[e >> 20];
      if (live != nullptr && live[pa->sys] == 0) continue;
      const unsigned r = e & 0xFFFFFu, nt = (unsigned)(pa->t.ntx * pa->t.nty);
      *tile = DIR > 0 ? r : nt - 1u - r;
      return true;
    }
  };
  wf_roles<PAT, DIR, P, E, false>(next, err, &L);
  wf_retire(ctr);
}

// addout = addv + x (the correction step after an ILU(0) upper sweep)
template <class V>
__global__ __launch_bounds__(256) void k_wf_add(const V* __restrict__ addv, const V* __restrict__ x,
                                                V* __restrict__ addout, long n) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) addout[i] = addv[i] + x[i];
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
  // consecutive steps of a tile read the same column lines: keep them on one
  // XCD's L2 (contiguous block ranges per XCD)
  const long q = (long)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
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
  // consecutive steps of a tile read the same column lines: keep them on one
  // XCD's L2 (contiguous block ranges per XCD)
  const long q = (long)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
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
  const unsigned b0 = i >= 0 ? __float_as_uint(s0) : 0u, b1 = i >= 0 ? __float_as_uint(s1) : 0u;
  if constexpr (wf_sd_in_pack(PAT)) {
    // the scalars take the last two words: halves NPK*K-4 .. NPK*K-1
    v[NPK * K - 4] = __ushort_as_half((unsigned short)(b0 & 0xffffu));
    v[NPK * K - 3] = __ushort_as_half((unsigned short)(b0 >> 16));
    v[NPK * K - 2] = __ushort_as_half((unsigned short)(b1 & 0xffffu));
    v[NPK * K - 1] = __ushort_as_half((unsigned short)(b1 >> 16));
  }
#pragma unroll
  for (int p = 0; p < NPK; ++p) {
    __half* o = out + ((row * NPK + p) * WF_NL + lane) * K;
#pragma unroll
    for (int e = 0; e < K; ++e) o[e] = v[p * K + e];
  }
  if (!wf_sd_in_pack(PAT) && dir > 0) {
    sd[2 * q] = __uint_as_float(b0);
    sd[2 * q + 1] = __uint_as_float(b1);
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
template <int PAT, int DIR, int P, class E, bool UNITD>
static hipError_t launch_wf_t(const WfArgs<typename WfVal<E>::V>& a, hipStream_t st) {
  const unsigned ntiles = (unsigned)(a.t.ntx * a.t.nty);
  const unsigned grid = ntiles < (unsigned)WF_MAX_GRID ? ntiles : (unsigned)WF_MAX_GRID;
  hipLaunchKernelGGL((k_wavefront<PAT, DIR, P, E, UNITD>), dim3(grid), dim3(WF_THREADS), 0, st, a);
  return hipGetLastError();
}

template <int PAT, int DIR, int P, class E>
static hipError_t launch_wfg_t(const WfArgs<typename WfVal<E>::V>* segs, const unsigned* tmap, unsigned total,
                               unsigned grid, const int* live, unsigned* ctr, unsigned* err, hipStream_t st) {
  hipLaunchKernelGGL((k_wavefront_group<PAT, DIR, P, E>), dim3(grid), dim3(WF_THREADS), 0, st, segs, tmap, total,
                     live, ctr, err);
  return hipGetLastError();
}

// Coefficient prefetch distance (steps) per pattern and storage type: as deep
// as the compute waves' registers allow (NPK 16-byte packs per step).
template <int PAT, class E>
constexpr int wf_prefetch() {
  return wf_npk(PAT, sizeof(E)) * 4 * 16 <= 160 ? 16 : (wf_npk(PAT, sizeof(E)) * 4 * 8 <= 160 ? 8 : 4);
}

template <class E>
hipError_t launch_wavefront_group(int pat, int dir, const WfArgs<typename WfVal<E>::V>* segs, const unsigned* tmap,
                                  unsigned total, unsigned grid, const int* live, unsigned* ctr, unsigned* err,
                                  hipStream_t st) {
  if (total == 0) return hipSuccess;
  if (grid == 0 || grid > total) grid = total;
  if (grid > (unsigned)WF_MAX_GRID) grid = WF_MAX_GRID;
#define SMG_WFG_CASE(PATV)                                                                                       \
  if (pat == PATV && dir > 0)                                                                                    \
    return launch_wfg_t<PATV, 1, wf_prefetch<PATV, E>(), E>(segs, tmap, total, grid, live, ctr, err, st);         \
  if (pat == PATV && dir < 0)                                                                                    \
    return launch_wfg_t<PATV, -1, wf_prefetch<PATV, E>(), E>(segs, tmap, total, grid, live, ctr, err, st);
  SMG_WFG_CASE(7)
  SMG_WFG_CASE(19)
  SMG_WFG_CASE(27)
#undef SMG_WFG_CASE
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
  using V = typename WfVal<E>::V;
  hipError_t e = hipErrorInvalidValue;
#define SMG_WF_CASE(PATV)                                                                           \
  if (pat == PATV) {                                                                                \
    constexpr int PV = wf_prefetch<PATV, E>();                                                      \
    if (dir > 0 && !unitd) e = launch_wf_t<PATV, 1, PV, E, false>(a, st);                           \
    if (dir < 0 && !unitd) e = launch_wf_t<PATV, -1, PV, E, false>(a, st);                          \
    if (dir > 0 && unitd) e = launch_wf_t<PATV, 1, PV, E, true>(a, st);                             \
  }
  SMG_WF_CASE(7)
  SMG_WF_CASE(19)
  SMG_WF_CASE(27)
#undef SMG_WF_CASE
  if (e != hipSuccess || !add) return e;
  // addout = addv + x once the sweep has finished
  const long n = a.g.N();
  hipLaunchKernelGGL((k_wf_add<V>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a.addv,
                     (const V*)a.x, a.addout, n);
  return hipGetLastError();
}

template hipError_t launch_wavefront<double>(int, int, bool, bool, const WfArgs<double>&, hipStream_t);
template hipError_t launch_wavefront<float>(int, int, bool, bool, const WfArgs<float>&, hipStream_t);
template hipError_t launch_wavefront<__half>(int, int, bool, bool, const WfArgs<float>&, hipStream_t);

}  // namespace smg
