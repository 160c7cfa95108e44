// 3x3 block systems (vector PDEs, the block operators of Sec. 4.2.3 and the
// elasticity problem of Sec. 5.1): point-block SpMV and residual, the input
// of the backward post-smoothing sweep, and the dependence-preserving
// point-block Gauss-Seidel sweep (Sec. 4.4 with 3x3 blocks).
//
// Storage: entry (r, c) of the block of offset s at A[(s*9 + r*3 + c)*N + i];
// vectors interleaved v[i*3 + c].  Per scalar row r of a block row the
// accumulation runs over neighbour blocks in canonical order and, inside a
// block, over columns c in order, with fma.
//
// The block sweep follows the scalar wavefront design (csrc/wavefront.hip):
// z-columns as lanes, sheared tiles in dependence order taken by atomic
// ticket, per-lane skew with the 3d27 hyperplane weights (4, 2, 1), an LDS
// ring for neighbour values plus a halo of other tiles' columns fetched
// device-coherently and checked against a signalling-NaN sentinel.  A node
// carries 3 values and needs 13 coefficient blocks and the inverse diagonal
// block per step (126 numbers, ~1 KB in FP64): more memory operations than a
// single wavefront may have in flight (63).  So a tile of 8 x 8 columns has
// three wavefronts, wavefront r computing scalar row r of every node: it
// loads only that row of the blocks (42 numbers), accumulates the row's sum
// in the oracle's order, the three sums meet in LDS, and each wavefront
// applies its row of the inverse diagonal block.
#include "smg_common.h"
#include "smg_group.h"
#include "smg_kernels.h"

namespace smg {

// ------------------------------------------------------------ SpMV / residual
template <class M, bool RES>
__global__ __launch_bounds__(256) void k_bspmv(Grid g, M m, const typename M::V* __restrict__ x,
                                               const typename M::V* __restrict__ b, typename M::V* __restrict__ y,
                                               const double* gate) {
  using V = typename M::V;
  if (gate != nullptr && *gate == 0.0) return;
  const long N = g.N();
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int X = (int)(i / ((long)g.ny * g.nz)), Y = (int)((i / g.nz) % g.ny), Z = (int)(i % g.nz);
  const long nyz = (long)g.ny * g.nz;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    V acc = V(0);
#pragma unroll
    for (int s = 0; s < 27; ++s) {
      const int dx = pat_off(27, s, 0), dy = pat_off(27, s, 1), dz = pat_off(27, s, 2);
      if (!in_grid(g, X + dx, Y + dy, Z + dz)) continue;
      const long j = i + dx * nyz + dy * g.nz + dz;
#pragma unroll
      for (int c = 0; c < 3; ++c) acc = fma(m(s * 9 + r * 3 + c, r, i), x[j * 3 + c], acc);
    }
    y[i * 3 + r] = RES ? b[i * 3 + r] - acc : acc;
  }
}

template <class M>
hipError_t launch_bspmv(const Grid& g, const M& m, const typename M::V* x, const typename M::V* b,
                        typename M::V* y, bool res, hipStream_t st) {
  const dim3 grid((unsigned)((g.N() + 255) / 256)), blk(256);
  if (res)
    hipLaunchKernelGGL((k_bspmv<M, true>), grid, blk, 0, st, g, m, x, b, y, (const double*)nullptr);
  else
    hipLaunchKernelGGL((k_bspmv<M, false>), grid, blk, 0, st, g, m, x, b, y, (const double*)nullptr);
  return hipGetLastError();
}

hipError_t launch_bspmv_res_gated(const Grid& g, const BMatD& m, const double* x, const double* b, double* y,
                                  const double* gate, hipStream_t st) {
  const dim3 grid((unsigned)((g.N() + 255) / 256)), blk(256);
  hipLaunchKernelGGL((k_bspmv<BMatD, true>), grid, blk, 0, st, g, m, x, b, y, gate);
  return hipGetLastError();
}

// h = f - sum over lower (UP = false) or upper (UP = true) neighbour blocks
// of A_ij u_j (old values): the terms a backward or forward sweep takes from
// before the sweep, in the order the sequential sweep applies them (first
// group of the row update).
template <class M, bool UP>
__global__ __launch_bounds__(256) void k_btri(Grid g, M m, const typename M::V* __restrict__ f,
                                              const typename M::V* __restrict__ u, typename M::V* __restrict__ h) {
  using V = typename M::V;
  const long N = g.N();
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int X = (int)(i / ((long)g.ny * g.nz)), Y = (int)((i / g.nz) % g.ny), Z = (int)(i % g.nz);
  const long nyz = (long)g.ny * g.nz;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    V t = f[i * 3 + r];
#pragma unroll
    for (int s = UP ? 14 : 0; s < (UP ? 27 : 13); ++s) {
      const int dx = pat_off(27, s, 0), dy = pat_off(27, s, 1), dz = pat_off(27, s, 2);
      if (!in_grid(g, X + dx, Y + dy, Z + dz)) continue;
      const long j = i + dx * nyz + dy * g.nz + dz;
#pragma unroll
      for (int c = 0; c < 3; ++c) t = fma(-m(s * 9 + r * 3 + c, r, i), u[j * 3 + c], t);
    }
    h[i * 3 + r] = t;
  }
}

template <class M>
hipError_t launch_blower(const Grid& g, const M& m, const typename M::V* f, const typename M::V* u,
                         typename M::V* h, hipStream_t st) {
  hipLaunchKernelGGL((k_btri<M, false>), dim3((unsigned)((g.N() + 255) / 256)), dim3(256), 0, st, g, m, f, u, h);
  return hipGetLastError();
}

template <class M>
hipError_t launch_bupper(const Grid& g, const M& m, const typename M::V* f, const typename M::V* u,
                         typename M::V* h, hipStream_t st) {
  hipLaunchKernelGGL((k_btri<M, true>), dim3((unsigned)((g.N() + 255) / 256)), dim3(256), 0, st, g, m, f, u, h);
  return hipGetLastError();
}

#define SMG_BINST(M)                                                                                           \
  template hipError_t launch_bspmv<M>(const Grid&, const M&, const M::V*, const M::V*, M::V*, bool, hipStream_t); \
  template hipError_t launch_blower<M>(const Grid&, const M&, const M::V*, const M::V*, M::V*, hipStream_t); \
  template hipError_t launch_bupper<M>(const Grid&, const M&, const M::V*, const M::V*, M::V*, hipStream_t);
SMG_BINST(BMatD)
SMG_BINST(BMatF)
SMG_BINST(BMatH)
#undef SMG_BINST

// ------------------------------------------------------------ block sweep
constexpr int BW_TX = 8, BW_TY = 8, BW_NL = 64;
constexpr int BW_NH = 56;    // halo slots around an 8 x 8 tile
constexpr int BW_HIST = 16;  // LDS ring rows (steps)
constexpr int BW_PH = 4;     // prefetch distance (steps) of right-hand side and halo values
constexpr int BW_UNROLL = 4;
constexpr int BW_WX = 4, BW_WY = 2, BW_KB = 7;  // 3d27 hyperplane weights, largest lower step distance
constexpr unsigned BW_SPIN_LIMIT = 1u << 21;
constexpr unsigned BW_OOB = 0x80000000u;
constexpr int BW_SC1 = 16;

typedef unsigned bu32x2 __attribute__((ext_vector_type(2)));
typedef unsigned bu32x4 __attribute__((ext_vector_type(4)));

void bwf_tiling(const Grid& g, WfTiling* t) {
  t->sh = g.ny <= BW_TY ? 0 : 1;
  t->ntx = (g.nx + BW_TX - 1) / BW_TX;
  t->nty = (g.ny + t->sh * (BW_TX - 1) + BW_TY - 1) / BW_TY;
  t->ns = g.nz + (BW_WX - t->sh * BW_WY) * (BW_TX - 1) + BW_WY * (BW_TY - 1) + 2 * BW_KB;
  t->nsk = (long)t->ntx * t->nty * t->ns * BW_NL;
}

// Sweep data per node position and scalar row r (each of the tile's three
// waves handles one row of every node): the row's 13 triangle blocks (3
// entries each, canonical order) then row r of the inverse diagonal block.
// FP64: 42 doubles = 21 packs; FP32: 42 floats in 11 packs; FP16: 39 halves
// (bytes 0..77), the FP32 row scale (byte 80) and the FP32 inverse row
// (bytes 84..95) = 6 packs.  Layout [tile][step][row][pack][lane].
__host__ __device__ constexpr int bwf_npr(int ebytes) { return ebytes == 8 ? 21 : (ebytes == 4 ? 11 : 6); }
__host__ __device__ constexpr int bwf_npk(int ebytes) { return 3 * bwf_npr(ebytes); }
int bwf_pack_count(int ebytes) { return bwf_npk(ebytes); }

__host__ __device__ constexpr int bw_col_dx(int c) { return c == 3 ? 0 : -1; }
__host__ __device__ constexpr int bw_col_dy(int c) { return c == 3 ? -1 : c - 1; }
__host__ __device__ constexpr int bw_col_of(int dx, int dy) { return dx == -1 ? dy + 1 : (dy == -1 ? 3 : -1); }

__host__ __device__ constexpr int bwf_halo_slot(int qx, int qy) {
  return qx == -1 ? qy + 2
                  : (qx == BW_TX ? 14 + qy
                                 : (qy < 0 ? 24 + 2 * qx + (qy + 2) : 40 + 2 * qx + (qy - BW_TY)));
}
__device__ inline void bwf_halo_pos(int hs, int* qx, int* qy) {
  if (hs < 12) {
    *qx = -1;
    *qy = hs - 2;
  } else if (hs < 24) {
    *qx = BW_TX;
    *qy = hs - 14;
  } else if (hs < 40) {
    *qx = (hs - 24) / 2;
    *qy = (hs - 24) % 2 - 2;
  } else {
    *qx = (hs - 40) / 2;
    *qy = BW_TY + (hs - 40) % 2;
  }
}
__device__ inline bool bwf_halo_used(int dir, int sh, int qx, int qy) {
  for (int c = 0; c < 4; ++c) {
    const int cx = dir * bw_col_dx(c), cy = dir * bw_col_dy(c);
    const int lx = qx - cx, ly = qy - cy - sh * cx;
    if (lx >= 0 && lx < BW_TX && ly >= 0 && ly < BW_TY) return true;
  }
  return false;
}
__device__ inline bool bwf_exported(int dir, int lx, int ly, int sh) {
  for (int c = 0; c < 4; ++c) {
    const int cx = dir * bw_col_dx(c), cy = dir * bw_col_dy(c);
    const int qx = lx - cx, qy = ly - cy - sh * cx;
    if (qx < 0 || qx >= BW_TX || qy < 0 || qy >= BW_TY) return true;
  }
  return false;
}

__device__ inline __amdgpu_buffer_rsrc_t bw_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <class V, int CP>
__device__ inline V bw_ld(__amdgpu_buffer_rsrc_t r, unsigned off) {
  if constexpr (sizeof(V) == 8)
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, CP));
  else
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, CP));
}
template <int CP, class V>
__device__ inline void bw_st(V v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  if constexpr (sizeof(V) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bu32x2, v), r, off, 0, CP);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, CP);
}

// entry e (0..41) of a row's sweep data held in packs p[]: e < 39 are the
// triangle coefficients (block e / 3, column e % 3), e = 39 + c the inverse
// row's column c
template <class E>
__device__ inline typename WfVal<E>::V bw_row(const bu32x4* p, int e);
template <>
__device__ inline double bw_row<double>(const bu32x4* p, int e) {
  const bu32x4 w = p[e / 2];
  return e % 2 == 0 ? __builtin_bit_cast(double, bu32x2{w.x, w.y}) : __builtin_bit_cast(double, bu32x2{w.z, w.w});
}
template <>
__device__ inline float bw_row<float>(const bu32x4* p, int e) {
  return __uint_as_float(p[e / 4][e % 4]);
}
template <>
__device__ inline float bw_row<__half>(const bu32x4* p, int e) {
  if (e >= 39) return __uint_as_float(p[(84 + 4 * (e - 39)) / 16][((84 + 4 * (e - 39)) % 16) / 4]);
  // row scale (byte 80) times the half, rounded once
  const unsigned w = p[e / 8][(e % 8) / 2];
  const float sc = __uint_as_float(p[5][0]);
  return e % 2 == 0 ? half_times<0>(w, sc) : half_times<1>(w, sc);
}

constexpr int BW_NT = 3 * BW_NL;  // threads: one wave per scalar row

template <int DIR, class E>
__global__ __launch_bounds__(BW_NT) void k_bwavefront(WfArgs<typename WfVal<E>::V> a) {
  using V = typename WfVal<E>::V;
  using B = VBits<V>;
  constexpr int NPR = bwf_npr(sizeof(E)), NPK = bwf_npk(sizeof(E));
  constexpr int P = sizeof(E) == 2 ? 4 : 2;  // steps of row data fetched ahead
  static_assert(BW_UNROLL % P == 0 && BW_UNROLL % BW_PH == 0, "unroll");
  constexpr int RW = (BW_NL + BW_NH) * 3 + 1;
  constexpr unsigned PACKB = BW_NL * 16u;
  constexpr int VS = (int)sizeof(V);
  __shared__ V ring[BW_HIST * RW];
  __shared__ V tx[3 * BW_NL];  // the three rows' sums of the current step
  __shared__ unsigned s_ticket;

  const int tid = threadIdx.x;
  const int r = tid / BW_NL;    // scalar row of this wave
  const int lane = tid % BW_NL;  // column of the tile
  const int lx = lane / BW_TY, ly = lane % BW_TY;
  const int sh = a.t.sh;
  const int skew = (BW_WX - sh * BW_WY) * lx + BW_WY * ly + BW_KB;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int NS = a.t.ns;
  const unsigned ntiles = (unsigned)(a.t.ntx * a.t.nty);
  const bool exported = bwf_exported(DIR, lx, ly, sh);
  const bool exp_next = a.next != nullptr && bwf_exported(a.next_dir, lx, ly, sh);
  int nidx[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int cx = DIR * bw_col_dx(c), cy = DIR * bw_col_dy(c);
    const int qx = lx + cx, qy = ly + cy + sh * cx;
    const bool in = qx >= 0 && qx < BW_TX && qy >= 0 && qy < BW_TY;
    nidx[c] = in ? qx * BW_TY + qy : BW_NL + bwf_halo_slot(qx, qy);
  }
  // halo loading: lane hs of wave r loads component r of halo slot hs
  const int hs = lane;
  int hqx = 0, hqy = 0;
  bool hrole = false;
  if (hs < BW_NH) {
    bwf_halo_pos(hs, &hqx, &hqy);
    hrole = bwf_halo_used(DIR, sh, hqx, hqy);
  }
  const int hskew = (BW_WX - sh * BW_WY) * hqx + BW_WY * hqy + BW_KB;

  for (;;) {
    if (tid == 0) s_ticket = atomicAdd(&a.ctr[0], 1u);
    __syncthreads();
    const unsigned ticket = s_ticket;
    __syncthreads();
    if (ticket >= ntiles) break;
    const unsigned tile = DIR > 0 ? ticket : ntiles - 1u - ticket;
    const int X = (int)(tile / (unsigned)a.t.nty), Y = (int)(tile % (unsigned)a.t.nty);
    const int xt = X * BW_TX + lx, yt = Y * BW_TY + ly - sh * lx;
    const bool colv = xt < nx && yt >= 0 && yt < ny;
    const int p0 = X * BW_TX > 0 ? X * BW_TX - 1 : 0;
    const int p1 = X * BW_TX + BW_TX + 1 < nx ? X * BW_TX + BW_TX + 1 : nx;
    const long pl = (long)ny * nz;
    const unsigned vbytes = (unsigned)((p1 - p0) * pl * 3 * (long)VS);
    const long vb = p0 * pl * 3;
    const auto rh = bw_rsrc(a.h + vb, vbytes);
    const auto rx = bw_rsrc(a.x + vb, vbytes);
    const auto rn = bw_rsrc((a.next != nullptr ? a.next : a.x) + vb, a.next != nullptr ? vbytes : 0u);
    const unsigned vo = colv ? (unsigned)(((xt - p0) * (long)ny + yt) * nz) : 0u;
    const int gx = X * BW_TX + hqx, gy = Y * BW_TY + hqy - sh * hqx;
    const bool hcolv = hrole && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    const unsigned hvo = hcolv ? (unsigned)(((gx - p0) * (long)ny + gy) * nz) : 0u;
    const unsigned tbytes = (unsigned)NS * NPK * PACKB;
    const auto rp = bw_rsrc((const char*)a.pk + (size_t)tile * tbytes, tbytes);
    const int nsteps = (NS + BW_UNROLL - 1) / BW_UNROLL * BW_UNROLL;

    auto step_of = [&](int k) { return DIR > 0 ? k : NS - 1 - k; };
    // byte offset of component r of the node of this lane at iteration k
    auto node_off = [&](int k) {
      const int z = step_of(k) - skew;
      return colv && z >= 0 && z < nz ? ((vo + (unsigned)z) * 3u + (unsigned)r) * (unsigned)VS : BW_OOB;
    };
    auto halo_off = [&](int k) {
      const int s = step_of(k);
      const int hz = s - hskew;
      return s >= 0 && s < NS && hcolv && hz >= 0 && hz < nz ? ((hvo + (unsigned)hz) * 3u + (unsigned)r) * (unsigned)VS
                                                             : BW_OOB;
    };
    // this row's sweep data of iteration k
    bu32x4 cf[P][NPR];
    auto row_fetch = [&](int k, int j) {
      const int s = step_of(k);
      const unsigned so = s >= 0 && s < NS ? ((unsigned)s * 3u + (unsigned)r) * (NPR * PACKB) : BW_OOB;
#pragma unroll
      for (int p = 0; p < NPR; ++p)
        cf[j][p] =
            __builtin_bit_cast(bu32x4, __builtin_amdgcn_raw_buffer_load_b128(rp, lane * 16u, so + p * PACKB, 0));
    };
    V hv[BW_PH], hb[BW_PH];
    auto h_fetch = [&](int k, int j) { hv[j] = bw_ld<V, 0>(rh, node_off(k)); };
    auto halo_fetch = [&](int k, int j) { hb[j] = bw_ld<V, BW_SC1>(rx, halo_off(k)); };
    auto halo_put = [&](int k, int j) {
      const unsigned off = halo_off(k);
      V v = hb[j];
      if (off != BW_OOB && B::bits(v) == B::sent) {
        unsigned spins = 0;
        do {
          __builtin_amdgcn_s_sleep(1);
          v = bw_ld<V, BW_SC1>(rx, off);
          // once any wait has timed out, stop waiting anywhere
          if ((spins & 1023u) == 1023u && (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1u))
            spins = BW_SPIN_LIMIT;
        } while (B::bits(v) == B::sent && ++spins < BW_SPIN_LIMIT);
        if (spins >= BW_SPIN_LIMIT) atomicOr(a.err, 1u);
      }
      if (hrole) ring[(k % BW_HIST) * RW + (BW_NL + hs) * 3 + r] = off != BW_OOB ? v : V(0);
    };

#pragma unroll
    for (int j = 0; j < P; ++j) row_fetch(j, j);
#pragma unroll
    for (int j = 0; j < BW_PH; ++j) {
      h_fetch(j, j);
      halo_fetch(j, j);
    }
    halo_put(0, 0);
    __syncthreads();

    for (int k0 = 0; k0 < nsteps; k0 += BW_UNROLL) {
#pragma unroll
      for (int j = 0; j < BW_UNROLL; ++j) {
        const int k = k0 + j;
        const int jh = j % BW_PH, jc = j % P;
        // this row's sum over the 13 triangle blocks, canonical order,
        // columns in order: t = h_r - sum A[m][r][c] u_m[c]
        V t = hv[jh];
#pragma unroll
        for (int m = 0; m < 13; ++m) {
          const int so = DIR > 0 ? m : 14 + m;
          const int dx = pat_off(27, so, 0), dy = pat_off(27, so, 1), dz = pat_off(27, so, 2);
          const V* rr;
          if (dx == 0 && dy == 0) {
            rr = ring + ((k - 1 + BW_HIST) % BW_HIST) * RW + lane * 3;  // this column, previous step
          } else {
            const int c = bw_col_of(DIR * dx, DIR * dy);
            const int back = DIR * (BW_WX * dx + BW_WY * dy + dz);  // in [-KB, -1]
            rr = ring + ((k + back + BW_HIST) % BW_HIST) * RW + nidx[c] * 3;
          }
          const V u0 = rr[0], u1 = rr[1], u2 = rr[2];
          t = fma(-bw_row<E>(cf[jc], 3 * m + 0), u0, t);
          t = fma(-bw_row<E>(cf[jc], 3 * m + 1), u1, t);
          t = fma(-bw_row<E>(cf[jc], 3 * m + 2), u2, t);
        }
        tx[r * BW_NL + lane] = t;
        __syncthreads();
        const V t0 = tx[lane], t1 = tx[BW_NL + lane], t2 = tx[2 * BW_NL + lane];
        const V xv = fma(bw_row<E>(cf[jc], 41), t2, fma(bw_row<E>(cf[jc], 40), t1, bw_row<E>(cf[jc], 39) * t0));
        const unsigned off = node_off(k);
        const bool act = off != BW_OOB;
        ring[(k % BW_HIST) * RW + lane * 3 + r] = act ? xv : V(0);
        bw_st<BW_SC1>(xv, rx, exported ? off : BW_OOB);
        bw_st<0>(xv, rx, exported ? BW_OOB : off);
        if (exp_next) bw_st<0>(B::val(B::sent), rn, off);
        halo_put(k + 1, (j + 1) % BW_PH);
        halo_fetch(k + BW_PH, jh);
        h_fetch(k + BW_PH, jh);
        row_fetch(k + P, jc);
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

template <class E>
hipError_t launch_bwavefront(int dir, const WfArgs<typename WfVal<E>::V>& a, hipStream_t st) {
  const unsigned ntiles = (unsigned)(a.t.ntx * a.t.nty);
  const unsigned grid = ntiles < 2048u ? ntiles : 2048u;
  if (dir > 0)
    hipLaunchKernelGGL((k_bwavefront<1, E>), dim3(grid), dim3(BW_NT), 0, st, a);
  else
    hipLaunchKernelGGL((k_bwavefront<-1, E>), dim3(grid), dim3(BW_NT), 0, st, a);
  return hipGetLastError();
}
template hipError_t launch_bwavefront<double>(int, const WfArgs<double>&, hipStream_t);
template hipError_t launch_bwavefront<float>(int, const WfArgs<float>&, hipStream_t);
template hipError_t launch_bwavefront<__half>(int, const WfArgs<float>&, hipStream_t);

// ------------------------------------------------------------ packing (setup)
__device__ inline long bwf_point(const Grid& g, const WfTiling& tl, long q) {
  const int l = (int)(q % BW_NL);
  const long r = q / BW_NL;
  const int s = (int)(r % tl.ns);
  const int tile = (int)(r / tl.ns);
  const int X = tile / tl.nty, Y = tile % tl.nty;
  const int lx = l / BW_TY, ly = l % BW_TY;
  const int x = X * BW_TX + lx, y = Y * BW_TY + ly - tl.sh * lx;
  const int z = s - ((BW_WX - tl.sh * BW_WY) * lx + BW_WY * ly + BW_KB);
  const bool v = x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
  return v ? ((long)x * g.ny + y) * g.nz + z : -1;
}

// FP64 / FP32: row r of position q: entries 3m + c = block (dir > 0 ? m :
// 14 + m) entry (r, c), m < 13; entries 39 + c = inverse diagonal entry
// (r, c); padding zero.
template <class E>
__global__ __launch_bounds__(256) void k_bwf_pack(Grid g, WfTiling tl, int dir, const double* __restrict__ A,
                                                  const double* __restrict__ Dinv, E* __restrict__ out) {
  constexpr int K = 16 / (int)sizeof(E), NPR = bwf_npr(sizeof(E));
  // consecutive steps of a tile read the same column lines: keep them on one
  // XCD's L2 (contiguous block ranges per XCD)
  const long q = (long)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (q >= tl.nsk) return;
  const long i = bwf_point(g, tl, q);
  const long N = g.N();
  const long pos = q / BW_NL;
  const int lane = (int)(q % BW_NL);
  for (int r = 0; r < 3; ++r)
    for (int p = 0; p < NPR; ++p) {
      E* o = out + (((pos * 3 + r) * NPR + p) * BW_NL + lane) * K;
      for (int e = 0; e < K; ++e) {
        const int v = p * K + e;
        double x = 0.0;
        if (i >= 0 && v < 39)
          x = A[((long)(dir > 0 ? v / 3 : 14 + v / 3) * 9 + r * 3 + v % 3) * N + i];
        else if (i >= 0 && v < 42)
          x = Dinv[(long)(r * 3 + v - 39) * N + i];
        o[e] = (E)x;
      }
    }
}

// FP16: row r of position q: the 39 halves of the row's triangle entries
// (bytes 0..77), the FP32 row scale (bytes 80..83), the FP32 inverse row
// (bytes 84..95).
__global__ __launch_bounds__(256) void k_bwf_pack_h(Grid g, WfTiling tl, int dir, const __half* __restrict__ a16,
                                                    const float* __restrict__ sc, const float* __restrict__ rd,
                                                    unsigned char* __restrict__ out) {
  constexpr int NPR = bwf_npr(2);
  // consecutive steps of a tile read the same column lines: keep them on one
  // XCD's L2 (contiguous block ranges per XCD)
  const long q = (long)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (q >= tl.nsk) return;
  const long i = bwf_point(g, tl, q);
  const long N = g.N();
  const long pos = q / BW_NL;
  const int lane = (int)(q % BW_NL);
  for (int r = 0; r < 3; ++r) {
    unsigned char bytes[16 * NPR];
    for (int b = 0; b < 16 * NPR; ++b) bytes[b] = 0;
    for (int v = 0; v < 39; ++v) {
      const __half h = i >= 0 ? a16[((long)(dir > 0 ? v / 3 : 14 + v / 3) * 9 + r * 3 + v % 3) * N + i]
                              : __float2half_rn(0.0f);
      const unsigned short u = __half_as_ushort(h);
      bytes[2 * v] = (unsigned char)(u & 0xff);
      bytes[2 * v + 1] = (unsigned char)(u >> 8);
    }
    const unsigned us = __float_as_uint(i >= 0 ? sc[(long)r * N + i] : 0.0f);
    for (int b = 0; b < 4; ++b) bytes[80 + b] = (unsigned char)(us >> (8 * b));
    for (int c = 0; c < 3; ++c) {
      const unsigned u = __float_as_uint(i >= 0 ? rd[(long)(r * 3 + c) * N + i] : 0.0f);
      for (int b = 0; b < 4; ++b) bytes[84 + 4 * c + b] = (unsigned char)(u >> (8 * b));
    }
    for (int p = 0; p < NPR; ++p) {
      unsigned char* o = out + (((pos * 3 + r) * NPR + p) * BW_NL + lane) * 16;
      for (int b = 0; b < 16; ++b) o[b] = bytes[16 * p + b];
    }
  }
}

template <class E>
hipError_t launch_bwf_pack(const Grid& g, const WfTiling& tl, int dir, const double* A, const double* Dinv, E* out,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_bwf_pack<E>), dim3((unsigned)((tl.nsk + 255) / 256)), dim3(256), 0, st, g, tl, dir, A, Dinv,
                     out);
  return hipGetLastError();
}
template hipError_t launch_bwf_pack<double>(const Grid&, const WfTiling&, int, const double*, const double*, double*,
                                            hipStream_t);
template hipError_t launch_bwf_pack<float>(const Grid&, const WfTiling&, int, const double*, const double*, float*,
                                           hipStream_t);

hipError_t launch_bwf_pack_h(const Grid& g, const WfTiling& tl, int dir, const __half* a16, const float* sc,
                             const float* rd, void* out, hipStream_t st) {
  hipLaunchKernelGGL(k_bwf_pack_h, dim3((unsigned)((tl.nsk + 255) / 256)), dim3(256), 0, st, g, tl, dir, a16, sc,
                     rd, (unsigned char*)out);
  return hipGetLastError();
}

}  // namespace smg
