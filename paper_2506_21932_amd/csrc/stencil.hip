// Parallel stencil kernels on SG-DIA storage: SpMV / residual (Sec. 4.1 P1),
// the fused residual + restriction of the downward V-cycle leg, and the fused
// prolongation + correction feeding the post-smoother of the upward leg
// (Sec. 2, V-cycle).  Interpolation P is vertex-centred trilinear with the
// grid map of Sec. 4.3 (coarse X <-> fine 2X+1, stride 2, base offset 1);
// restriction is R = P^T.
//
// Every output element is produced with the same operations in the same
// order as the definition it implements: accumulations run over stencil
// offsets (or restriction offsets, or interpolation parents) in canonical
// lexicographic order with explicit fma, and out-of-grid terms are skipped.
#include "smg_group.h"
#include "smg_kernels.h"

namespace smg {

__device__ inline void unflat(unsigned i, int ny, int nz, int& x, int& y, int& z) {
  unsigned nyz = (unsigned)ny * (unsigned)nz;
  x = (int)(i / nyz);
  unsigned r = i - (unsigned)x * nyz;
  y = (int)(r / (unsigned)nz);
  z = (int)(r - (unsigned)y * (unsigned)nz);
}

// ---------------------------------------------------------------- SpMV
template <int PAT, class M, bool RES>
struct SpmvOp {
  using Args = SpmvArgs<M>;
  __device__ static void run(const Args& a, unsigned bid) {
    using V = typename M::V;
    const Grid g = a.g;
    const M m = a.m;
    const V* __restrict__ x = a.x;
    const unsigned N = (unsigned)g.N();
    const unsigned i = bid * 256u + threadIdx.x;
    if (i >= N) return;
    int X, Y, Z;
    unflat(i, g.ny, g.nz, X, Y, Z);
    const long nyz = (long)g.ny * g.nz;
    V acc = V(0);
#pragma unroll
    for (int s = 0; s < PAT; ++s) {
      const int dx = pat_off(PAT, s, 0), dy = pat_off(PAT, s, 1), dz = pat_off(PAT, s, 2);
      if (in_grid(g, X + dx, Y + dy, Z + dz)) acc = fma(m(s, i), x[(long)i + dx * nyz + dy * g.nz + dz], acc);
    }
    a.y[i] = RES ? a.b[i] - acc : acc;
  }
};

unsigned spmv_blocks(const Grid& g) { return (unsigned)((g.N() + 255) / 256); }

template <class M>
hipError_t launch_spmv(int pat, const Grid& g, const M& m, const typename M::V* x, const typename M::V* b,
                       typename M::V* y, bool res, hipStream_t st) {
  const SpmvArgs<M> a{g, m, x, b, y, 0};
  const dim3 grid(spmv_blocks(g)), blk(256);
#define SMG_SPMV(P)                                                                      \
  if (pat == P) {                                                                        \
    if (res)                                                                             \
      hipLaunchKernelGGL((k_one<SpmvOp<P, M, true>>), grid, blk, 0, st, a);             \
    else                                                                                 \
      hipLaunchKernelGGL((k_one<SpmvOp<P, M, false>>), grid, blk, 0, st, a);            \
    return hipGetLastError();                                                            \
  }
  SMG_SPMV(7)
  SMG_SPMV(19)
  SMG_SPMV(27)
#undef SMG_SPMV
  return hipErrorInvalidValue;
}

// The residual of the true-residual check of the device-resident PCG: runs
// only where *gate != 0 (the same operations as SpmvOp otherwise).
template <class OP>
__global__ __launch_bounds__(256) void k_one_gated(const typename OP::Args a, const double* gate) {
  if (*gate == 0.0) return;
  OP::run(a, blockIdx.x);
}
hipError_t launch_spmv_res_gated(int pat, const Grid& g, const MatD& m, const double* x, const double* b, double* y,
                                 const double* gate, hipStream_t st) {
  const SpmvArgs<MatD> a{g, m, x, b, y, 0};
  const dim3 grid(spmv_blocks(g)), blk(256);
  if (pat == 7)
    hipLaunchKernelGGL((k_one_gated<SpmvOp<7, MatD, true>>), grid, blk, 0, st, a, gate);
  else if (pat == 19)
    hipLaunchKernelGGL((k_one_gated<SpmvOp<19, MatD, true>>), grid, blk, 0, st, a, gate);
  else if (pat == 27)
    hipLaunchKernelGGL((k_one_gated<SpmvOp<27, MatD, true>>), grid, blk, 0, st, a, gate);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class M>
hipError_t launch_spmv_group(int pat, bool res, const SpmvArgs<M>* segs, const unsigned* bmap, unsigned nblocks,
                             const int* live, hipStream_t st) {
  if (nblocks == 0) return hipSuccess;
  const dim3 grid(nblocks), blk(256);
#define SMG_SPMV(P)                                                                          \
  if (pat == P) {                                                                            \
    if (res)                                                                                 \
      hipLaunchKernelGGL((k_group<SpmvOp<P, M, true>>), grid, blk, 0, st, segs, bmap, live); \
    else                                                                                     \
      hipLaunchKernelGGL((k_group<SpmvOp<P, M, false>>), grid, blk, 0, st, segs, bmap, live);\
    return hipGetLastError();                                                                \
  }
  SMG_SPMV(7)
  SMG_SPMV(19)
  SMG_SPMV(27)
#undef SMG_SPMV
  return hipErrorInvalidValue;
}

// ------------------------------------------ one-triangle residual
// h = f - sum over the lower (UP = false) or upper (UP = true) offsets s, in
// canonical order, of a_s u[nbr]: the old-value terms of a backward or a
// forward Gauss-Seidel row (t = f; t = fma(-a, u, t)).
template <int PAT, class M, bool UP>
struct TriOp {
  using Args = SpmvArgs<M>;  // x = u, b = f, y = h
  __device__ static void run(const Args& a, unsigned bid) {
    using V = typename M::V;
    const Grid g = a.g;
    const M m = a.m;
    const unsigned i = bid * 256u + threadIdx.x;
    if (i >= (unsigned)g.N()) return;
    int X, Y, Z;
    unflat(i, g.ny, g.nz, X, Y, Z);
    const long nyz = (long)g.ny * g.nz;
    V t = a.b[i];
#pragma unroll
    for (int s = UP ? PAT / 2 + 1 : 0; s < (UP ? PAT : PAT / 2); ++s) {
      const int dx = pat_off(PAT, s, 0), dy = pat_off(PAT, s, 1), dz = pat_off(PAT, s, 2);
      if (in_grid(g, X + dx, Y + dy, Z + dz)) t = fma(-m(s, i), a.x[(long)i + dx * nyz + dy * g.nz + dz], t);
    }
    a.y[i] = t;
  }
};

template <class M, bool UP>
static hipError_t launch_tri(int pat, const Grid& g, const M& m, const typename M::V* f, const typename M::V* u,
                             typename M::V* h, hipStream_t st) {
  const SpmvArgs<M> a{g, m, u, f, h, 0};
  const dim3 grid(spmv_blocks(g)), blk(256);
  if (pat == 7)
    hipLaunchKernelGGL((k_one<TriOp<7, M, UP>>), grid, blk, 0, st, a);
  else if (pat == 19)
    hipLaunchKernelGGL((k_one<TriOp<19, M, UP>>), grid, blk, 0, st, a);
  else if (pat == 27)
    hipLaunchKernelGGL((k_one<TriOp<27, M, UP>>), grid, blk, 0, st, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class M>
hipError_t launch_lower(int pat, const Grid& g, const M& m, const typename M::V* f, const typename M::V* u,
                        typename M::V* h, hipStream_t st) {
  return launch_tri<M, false>(pat, g, m, f, u, h, st);
}

template <class M>
hipError_t launch_upper(int pat, const Grid& g, const M& m, const typename M::V* f, const typename M::V* u,
                        typename M::V* h, hipStream_t st) {
  return launch_tri<M, true>(pat, g, m, f, u, h, st);
}

// ------------------------------------------------ residual + restriction
// One workgroup per coarse block of RB_X x RB_Y x RB_Z coarse points.
// Phase 1 computes the fine residuals of the block's footprint into LDS;
// phase 2 restricts them.  A residual shared by two blocks is recomputed
// (identically) by both.
// Coarse block per workgroup: 4 x 4 x 16 on large levels; 2 x 2 x 4 where
// the large blocks would leave most compute units idle (small levels), so
// that each thread computes about one residual and the kernel's latency is
// one round of loads.  Results do not depend on the block shape.
template <bool SMALL>
struct RBT {
  static constexpr int X = SMALL ? 2 : 4, Y = SMALL ? 2 : 4, Z = SMALL ? 4 : 16;
};

__host__ __device__ inline int rr_ext(int cm, int cb) { return cm ? 2 * cb + 1 : cb; }

template <int PAT, class M, bool SMALL>
struct RROp {
  static constexpr int RB_X = RBT<SMALL>::X, RB_Y = RBT<SMALL>::Y, RB_Z = RBT<SMALL>::Z;
  using Args = RRArgs<M>;
  __device__ static void run(const Args& a, unsigned bid_) {
  const Grid gf = a.g;
  const int cmask = a.cmask;
  const M m = a.m;
  const typename M::V* __restrict__ f = a.f;
  const typename M::V* __restrict__ u = a.u;
  typename M::V* __restrict__ rc = a.rc;
  using V = typename M::V;
  constexpr int MAXE = (2 * RB_X + 1) * (2 * RB_Y + 1) * (2 * RB_Z + 1);
  __shared__ V rs[MAXE];
  const int cmx = cmask & 1, cmy = (cmask >> 1) & 1, cmz = (cmask >> 2) & 1;
  const Grid gc{cmx ? gf.nx / 2 : gf.nx, cmy ? gf.ny / 2 : gf.ny, cmz ? gf.nz / 2 : gf.nz};
  const int nbz = (gc.nz + RB_Z - 1) / RB_Z, nby = (gc.ny + RB_Y - 1) / RB_Y;
  const int bid = (int)bid_;
  const int bz = bid % nbz, by = (bid / nbz) % nby, bx = bid / (nbz * nby);
  const int C0x = bx * RB_X, C0y = by * RB_Y, C0z = bz * RB_Z;
  const int lox = cmx ? 2 * C0x : C0x, loy = cmy ? 2 * C0y : C0y, loz = cmz ? 2 * C0z : C0z;
  const int ex = rr_ext(cmx, RB_X), ey = rr_ext(cmy, RB_Y), ez = rr_ext(cmz, RB_Z);
  const long nyz = (long)gf.ny * gf.nz;
  const int ne = ex * ey * ez;
  for (int k = threadIdx.x; k < ne; k += 256) {
    const int fz = loz + k % ez, fy = loy + (k / ez) % ey, fx = lox + k / (ez * ey);
    if (fx >= gf.nx || fy >= gf.ny || fz >= gf.nz) continue;
    const long i = ((long)fx * gf.ny + fy) * gf.nz + fz;
    V acc = V(0);
#pragma unroll
    for (int s = 0; s < PAT; ++s) {
      const int dx = pat_off(PAT, s, 0), dy = pat_off(PAT, s, 1), dz = pat_off(PAT, s, 2);
      if (in_grid(gf, fx + dx, fy + dy, fz + dz)) acc = fma(m(s, i), u[i + dx * nyz + dy * gf.nz + dz], acc);
    }
    rs[k] = f[i] - acc;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < RB_X * RB_Y * RB_Z; k += 256) {
    const int Z = C0z + k % RB_Z, Yc = C0y + (k / RB_Z) % RB_Y, Xc = C0x + k / (RB_Z * RB_Y);
    if (Xc >= gc.nx || Yc >= gc.ny || Z >= gc.nz) continue;
    const int fx0 = cmx ? 2 * Xc + 1 : Xc, fy0 = cmy ? 2 * Yc + 1 : Yc, fz0 = cmz ? 2 * Z + 1 : Z;
    V acc = V(0);
#pragma unroll
    for (int r = 0; r < 27; ++r) {
      const int dx = r / 9 - 1, dy = (r / 3) % 3 - 1, dz = r % 3 - 1;
      if ((!cmx && dx) || (!cmy && dy) || (!cmz && dz)) continue;
      const int ux = fx0 + dx, uy = fy0 + dy, uz = fz0 + dz;
      if (!in_grid(gf, ux, uy, uz)) continue;
      const V w = V((dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0));
      acc = fma(w, rs[((ux - lox) * ey + (uy - loy)) * ez + (uz - loz)], acc);
    }
    rc[((long)Xc * gc.ny + Yc) * gc.nz + Z] = acc;
  }
  }
};

template <bool SMALL>
static unsigned rr_blocks_t(const Grid& g, int cmask) {
  constexpr int BX = RBT<SMALL>::X, BY = RBT<SMALL>::Y, BZ = RBT<SMALL>::Z;
  const int cx = (cmask & 1) ? g.nx / 2 : g.nx, cy = (cmask & 2) ? g.ny / 2 : g.ny, cz = (cmask & 4) ? g.nz / 2 : g.nz;
  return (unsigned)(((cx + BX - 1) / BX) * ((cy + BY - 1) / BY) * ((cz + BZ - 1) / BZ));
}
unsigned rr_blocks(const Grid& g, int cmask, bool small) {
  return small ? rr_blocks_t<true>(g, cmask) : rr_blocks_t<false>(g, cmask);
}
bool rr_small(unsigned big_blocks) { return big_blocks < 1024; }

template <class M>
hipError_t launch_resid_restrict(int pat, const Grid& g, int cmask, const M& m, const typename M::V* f,
                                 const typename M::V* u, typename M::V* rc, hipStream_t st) {
  const RRArgs<M> a{g, cmask, m, f, u, rc, 0};
  const bool small = rr_small(rr_blocks(g, cmask, false));
  const unsigned nb = rr_blocks(g, cmask, small);
#define SMG_RR(P)                                                                          \
  if (pat == P) {                                                                          \
    if (small)                                                                             \
      hipLaunchKernelGGL((k_one_xcd<RROp<P, M, true>>), dim3(nb), dim3(256), 0, st, a);       \
    else                                                                                   \
      hipLaunchKernelGGL((k_one_xcd<RROp<P, M, false>>), dim3(nb), dim3(256), 0, st, a);      \
    return hipGetLastError();                                                              \
  }
  SMG_RR(7)
  SMG_RR(19)
  SMG_RR(27)
#undef SMG_RR
  return hipErrorInvalidValue;
}

template <class M>
hipError_t launch_rr_group(int pat, bool small, const RRArgs<M>* segs, const unsigned* bmap, unsigned nblocks,
                           const int* live, hipStream_t st) {
  if (nblocks == 0) return hipSuccess;
#define SMG_RR(P)                                                                                              \
  if (pat == P) {                                                                                              \
    if (small)                                                                                                 \
      hipLaunchKernelGGL((k_group<RROp<P, M, true>>), dim3(nblocks), dim3(256), 0, st, segs, bmap, live);     \
    else                                                                                                       \
      hipLaunchKernelGGL((k_group<RROp<P, M, false>>), dim3(nblocks), dim3(256), 0, st, segs, bmap, live);    \
    return hipGetLastError();                                                                                  \
  }
  SMG_RR(7)
  SMG_RR(19)
  SMG_RR(27)
#undef SMG_RR
  return hipErrorInvalidValue;
}

// --------------------------------------- interpolation of one fine point
// pe = sum over parents (lexicographic) of w * e_J via fma, from zero.
template <class V, class EC>
__device__ inline V interp_point_at(const EC& ec_at, const Grid& gc, int cmx, int cmy, int cmz, int fx, int fy,
                                    int fz) {
  int par[3][2], np[3];
  V wt[3][2];
  const int f[3] = {fx, fy, fz}, cm[3] = {cmx, cmy, cmz}, nc[3] = {gc.nx, gc.ny, gc.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    np[a] = 0;
    par[a][0] = par[a][1] = 0;
    wt[a][0] = wt[a][1] = V(0);
    if (!cm[a]) {
      par[a][0] = f[a];
      wt[a][0] = V(1);
      np[a] = 1;
    } else if (f[a] & 1) {
      const int J = (f[a] - 1) / 2;
      if (J < nc[a]) {
        par[a][0] = J;
        wt[a][0] = V(1);
        np[a] = 1;
      }
    } else {
      const int J0 = f[a] / 2 - 1, J1 = f[a] / 2;
      if (J0 >= 0 && J0 < nc[a]) {
        par[a][np[a]] = J0;
        wt[a][np[a]] = V(0.5);
        np[a]++;
      }
      if (J1 < nc[a]) {
        par[a][np[a]] = J1;
        wt[a][np[a]] = V(0.5);
        np[a]++;
      }
    }
  }
  // parents in lexicographic order; fixed trip counts, absent parents
  // predicated off (the same terms in the same order as a loop to np[a])
  V pe = V(0);
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        if (p < np[0] && q < np[1] && r < np[2]) {
          const V w = wt[0][p] * wt[1][q] * wt[2][r];
          pe = fma(w, ec_at(par[0][p], par[1][q], par[2][r]), pe);
        }
      }
  return pe;
}

template <class V>
__device__ inline V interp_point(const V* __restrict__ ec, const Grid& gc, int cmx, int cmy, int cmz, int fx, int fy,
                                 int fz, int bs, int comp) {
  auto at = [&](int X, int Y, int Z) { return ec[(((long)X * gc.ny + Y) * gc.nz + Z) * bs + comp]; };
  return interp_point_at<V>(at, gc, cmx, cmy, cmz, fx, fy, fz);
}

// --------------------------------- prolongation + post-smoother input
// Fine block per workgroup: 8 x 8 x 32 on large levels, 4 x 4 x 8 on small
// ones (as for the restriction).
template <bool SMALL>
struct PBT {
  static constexpr int X = SMALL ? 4 : 8, Y = SMALL ? 4 : 8, Z = SMALL ? 8 : 32;
};

template <int PAT, class M, bool FULL, bool SMALL>
struct PPOp {
  static constexpr int PP_X = PBT<SMALL>::X, PP_Y = PBT<SMALL>::Y, PP_Z = PBT<SMALL>::Z;
  using Args = PPArgs<M>;
  __device__ static void run(const Args& a, unsigned bid_) {
  const Grid gf = a.g;
  const int cmask = a.cmask;
  const M m = a.m;
  const typename M::V* __restrict__ f = a.f;
  const typename M::V* __restrict__ u = a.u;
  const typename M::V* __restrict__ ec = a.ec;
  typename M::V* __restrict__ h = a.h;
  typename M::V* __restrict__ uo = a.uo;
  using V = typename M::V;
  constexpr int HX = PP_X + 2, HY = PP_Y + 2, HZ = PP_Z + 2;
  __shared__ V us[HX * HY * HZ];
  const int cmx = cmask & 1, cmy = (cmask >> 1) & 1, cmz = (cmask >> 2) & 1;
  const Grid gc{cmx ? gf.nx / 2 : gf.nx, cmy ? gf.ny / 2 : gf.ny, cmz ? gf.nz / 2 : gf.nz};
  const int nbz = (gf.nz + PP_Z - 1) / PP_Z, nby = (gf.ny + PP_Y - 1) / PP_Y;
  const int bid = (int)bid_;
  const int bz = bid % nbz, by = (bid / nbz) % nby, bx = bid / (nbz * nby);
  const int x0 = bx * PP_X - 1, y0 = by * PP_Y - 1, z0 = bz * PP_Z - 1;
  // the coarse values interpolated into this block's fine region, staged in
  // LDS: parents of fine x in [x0, x0+HX) lie in [floor((x0-1)/2), floor((x0+HX-1)/2)]
  // staging buffer: dynamic LDS sized by the launch for the coarsening masks
  // of its grids (pp_stage_elems)
  extern __shared__ __align__(16) unsigned char pp_dyn[];
  V* ecs = reinterpret_cast<V*>(pp_dyn);
  auto fdiv2 = [](int v) { return v >= 0 ? v / 2 : -((1 - v) / 2); };
  const int c0x = cmx ? fdiv2(x0 - 1) : x0, c0y = cmy ? fdiv2(y0 - 1) : y0, c0z = cmz ? fdiv2(z0 - 1) : z0;
  const int ecx = cmx ? HX / 2 + 1 : HX, ecy = cmy ? HY / 2 + 1 : HY, ecz = cmz ? HZ / 2 + 1 : HZ;
  const bool staged = ec != nullptr;
  if (staged) {
    for (int k = threadIdx.x; k < ecx * ecy * ecz; k += 256) {
      const int cz = c0z + k % ecz, cy = c0y + (k / ecz) % ecy, cx = c0x + k / (ecz * ecy);
      if (in_grid(gc, cx, cy, cz)) ecs[k] = ec[((long)cx * gc.ny + cy) * gc.nz + cz];
    }
    __syncthreads();
  }
  auto ec_at = [&](int X, int Y, int Z) { return ecs[((X - c0x) * ecy + (Y - c0y)) * ecz + (Z - c0z)]; };
  for (int k = threadIdx.x; k < HX * HY * HZ; k += 256) {
    const int fz = z0 + k % HZ, fy = y0 + (k / HZ) % HY, fx = x0 + k / (HZ * HY);
    if (!in_grid(gf, fx, fy, fz)) continue;
    const long i = ((long)fx * gf.ny + fy) * gf.nz + fz;
    V v = u[i];
    if (staged) v = v + interp_point_at<V>(ec_at, gc, cmx, cmy, cmz, fx, fy, fz);
    us[k] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < PP_X * PP_Y * PP_Z; k += 256) {
    const int lz = k % PP_Z, ly = (k / PP_Z) % PP_Y, lx = k / (PP_Z * PP_Y);
    const int fx = x0 + 1 + lx, fy = y0 + 1 + ly, fz = z0 + 1 + lz;
    if (!in_grid(gf, fx, fy, fz)) continue;
    const long i = ((long)fx * gf.ny + fy) * gf.nz + fz;
    const int c = ((lx + 1) * HY + (ly + 1)) * HZ + (lz + 1);
    // the row's coefficients are loaded unconditionally (row i's own slots)
    // before the sums, so a thread's loads are in flight together; terms of
    // neighbours outside the grid leave the sums unchanged
    constexpr int NS = FULL ? PAT : PAT / 2;
    V a[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) a[s] = m(s, i);
    if (!FULL) {
      V t = f[i];
#pragma unroll
      for (int s = 0; s < PAT / 2; ++s) {
        const int dx = pat_off(PAT, s, 0), dy = pat_off(PAT, s, 1), dz = pat_off(PAT, s, 2);
        const V un = us[c + (dx * HY + dy) * HZ + dz];
        t = in_grid(gf, fx + dx, fy + dy, fz + dz) ? fma(-a[s], un, t) : t;
      }
      h[i] = t;
    } else {
      V acc = V(0);
#pragma unroll
      for (int s = 0; s < PAT; ++s) {
        const int dx = pat_off(PAT, s, 0), dy = pat_off(PAT, s, 1), dz = pat_off(PAT, s, 2);
        const V un = us[c + (dx * HY + dy) * HZ + dz];
        acc = in_grid(gf, fx + dx, fy + dy, fz + dz) ? fma(a[s], un, acc) : acc;
      }
      h[i] = f[i] - acc;
      uo[i] = us[c];
    }
  }
  }
};

template <bool SMALL>
static unsigned pp_blocks_t(const Grid& g) {
  constexpr int BX = PBT<SMALL>::X, BY = PBT<SMALL>::Y, BZ = PBT<SMALL>::Z;
  return (unsigned)(((g.nx + BX - 1) / BX) * ((g.ny + BY - 1) / BY) * ((g.nz + BZ - 1) / BZ));
}
unsigned pp_blocks(const Grid& g, bool small) { return small ? pp_blocks_t<true>(g) : pp_blocks_t<false>(g); }
unsigned pp_stage_elems(int cmask, bool small) {
  const int hx = (small ? PBT<true>::X : PBT<false>::X) + 2, hy = (small ? PBT<true>::Y : PBT<false>::Y) + 2,
            hz = (small ? PBT<true>::Z : PBT<false>::Z) + 2;
  return (unsigned)(((cmask & 1) ? hx / 2 + 1 : hx) * ((cmask & 2) ? hy / 2 + 1 : hy) *
                    ((cmask & 4) ? hz / 2 + 1 : hz));
}
bool pp_small(unsigned big_blocks) { return big_blocks < 1024; }

template <class M>
hipError_t launch_prolong_post(int pat, const Grid& g, int cmask, const M& m, const typename M::V* f,
                               const typename M::V* u, const typename M::V* ec, typename M::V* h,
                               typename M::V* uold_out, bool full, hipStream_t st) {
  const PPArgs<M> a{g, cmask, m, f, u, ec, h, uold_out, 0};
  const bool small = pp_small(pp_blocks(g, false));
  const unsigned nb = pp_blocks(g, small);
  const size_t dyn = ec != nullptr ? pp_stage_elems(cmask, small) * sizeof(typename M::V) : 0;
#define SMG_PP2(P, F)                                                                          \
  if (small)                                                                                   \
    hipLaunchKernelGGL((k_one_xcd<PPOp<P, M, F, true>>), dim3(nb), dim3(256), dyn, st, a);    \
  else                                                                                         \
    hipLaunchKernelGGL((k_one_xcd<PPOp<P, M, F, false>>), dim3(nb), dim3(256), dyn, st, a);
#define SMG_PP(P)                                                                              \
  if (pat == P) {                                                                              \
    if (full) {                                                                                \
      SMG_PP2(P, true)                                                                         \
    } else {                                                                                   \
      SMG_PP2(P, false)                                                                        \
    }                                                                                          \
    return hipGetLastError();                                                                  \
  }
  SMG_PP(7)
  SMG_PP(19)
  SMG_PP(27)
#undef SMG_PP
#undef SMG_PP2
  return hipErrorInvalidValue;
}

template <class M>
hipError_t launch_pp_group(int pat, bool full, bool small, unsigned stage_elems, const PPArgs<M>* segs,
                           const unsigned* bmap, unsigned nblocks, const int* live, hipStream_t st) {
  if (nblocks == 0) return hipSuccess;
  const size_t dyn = stage_elems * sizeof(typename M::V);
#define SMG_PP2(P, F)                                                                                             \
  if (small)                                                                                                      \
    hipLaunchKernelGGL((k_group<PPOp<P, M, F, true>>), dim3(nblocks), dim3(256), dyn, st, segs, bmap, live);     \
  else                                                                                                            \
    hipLaunchKernelGGL((k_group<PPOp<P, M, F, false>>), dim3(nblocks), dim3(256), dyn, st, segs, bmap, live);
#define SMG_PP(P)                                                                                               \
  if (pat == P) {                                                                                               \
    if (full) {                                                                                                 \
      SMG_PP2(P, true)                                                                                          \
    } else {                                                                                                    \
      SMG_PP2(P, false)                                                                                         \
    }                                                                                                           \
    return hipGetLastError();                                                                                   \
  }
  SMG_PP(7)
  SMG_PP(19)
  SMG_PP(27)
#undef SMG_PP
#undef SMG_PP2
  return hipErrorInvalidValue;
}

// -------------------------------------- plain restriction / prolongation
template <class V>
__global__ __launch_bounds__(256) void k_restrict(Grid gf, int cmask, int bs, const V* __restrict__ rf,
                                                  V* __restrict__ rc) {
  const int cmx = cmask & 1, cmy = (cmask >> 1) & 1, cmz = (cmask >> 2) & 1;
  const Grid gc{cmx ? gf.nx / 2 : gf.nx, cmy ? gf.ny / 2 : gf.ny, cmz ? gf.nz / 2 : gf.nz};
  const unsigned k = blockIdx.x * 256u + threadIdx.x;
  if (k >= (unsigned)(gc.N() * bs)) return;
  const unsigned ic = k / bs;
  const int comp = k % bs;
  int Xc, Yc, Z;
  unflat(ic, gc.ny, gc.nz, Xc, Yc, Z);
  const int fx0 = cmx ? 2 * Xc + 1 : Xc, fy0 = cmy ? 2 * Yc + 1 : Yc, fz0 = cmz ? 2 * Z + 1 : Z;
  V acc = V(0);
  for (int r = 0; r < 27; ++r) {
    const int dx = r / 9 - 1, dy = (r / 3) % 3 - 1, dz = r % 3 - 1;
    if ((!cmx && dx) || (!cmy && dy) || (!cmz && dz)) continue;
    const int ux = fx0 + dx, uy = fy0 + dy, uz = fz0 + dz;
    if (!in_grid(gf, ux, uy, uz)) continue;
    const V w = V((dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0));
    acc = fma(w, rf[(((long)ux * gf.ny + uy) * gf.nz + uz) * bs + comp], acc);
  }
  rc[k] = acc;
}

template <class V>
__global__ __launch_bounds__(256) void k_prolong_add(Grid gf, int cmask, int bs, const V* __restrict__ ec,
                                                     V* __restrict__ uf) {
  const int cmx = cmask & 1, cmy = (cmask >> 1) & 1, cmz = (cmask >> 2) & 1;
  const Grid gc{cmx ? gf.nx / 2 : gf.nx, cmy ? gf.ny / 2 : gf.ny, cmz ? gf.nz / 2 : gf.nz};
  const unsigned k = blockIdx.x * 256u + threadIdx.x;
  if (k >= (unsigned)(gf.N() * bs)) return;
  const unsigned i = k / bs;
  const int comp = k % bs;
  int X, Y, Z;
  unflat(i, gf.ny, gf.nz, X, Y, Z);
  uf[k] = uf[k] + interp_point(ec, gc, cmx, cmy, cmz, X, Y, Z, bs, comp);
}

template <class V>
hipError_t launch_restrict(const Grid& g, int cmask, int bs, const V* rf, V* rc, hipStream_t st) {
  const long nc = (long)((cmask & 1) ? g.nx / 2 : g.nx) * ((cmask & 2) ? g.ny / 2 : g.ny) *
                  ((cmask & 4) ? g.nz / 2 : g.nz) * bs;
  hipLaunchKernelGGL((k_restrict<V>), dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, g, cmask, bs, rf, rc);
  return hipGetLastError();
}
template <class V>
hipError_t launch_prolong_add(const Grid& g, int cmask, int bs, const V* ec, V* uf, hipStream_t st) {
  const long n = g.N() * bs;
  hipLaunchKernelGGL((k_prolong_add<V>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, cmask, bs, ec, uf);
  return hipGetLastError();
}

#define SMG_INST(M)                                                                                              \
  template hipError_t launch_spmv<M>(int, const Grid&, const M&, const M::V*, const M::V*, M::V*, bool,          \
                                     hipStream_t);                                                               \
  template hipError_t launch_resid_restrict<M>(int, const Grid&, int, const M&, const M::V*, const M::V*, M::V*, \
                                               hipStream_t);                                                     \
  template hipError_t launch_prolong_post<M>(int, const Grid&, int, const M&, const M::V*, const M::V*,          \
                                             const M::V*, M::V*, M::V*, bool, hipStream_t);
SMG_INST(MatD)
SMG_INST(MatF)
SMG_INST(MatH)
#undef SMG_INST
#define SMG_GINST(M)                                                                                           \
  template hipError_t launch_spmv_group<M>(int, bool, const SpmvArgs<M>*, const unsigned*, unsigned, const int*, \
                                           hipStream_t);                                                       \
  template hipError_t launch_rr_group<M>(int, bool, const RRArgs<M>*, const unsigned*, unsigned, const int*,     \
                                         hipStream_t);                                                         \
  template hipError_t launch_pp_group<M>(int, bool, bool, unsigned, const PPArgs<M>*, const unsigned*, unsigned, \
                                         const int*, hipStream_t);
SMG_GINST(MatD)
SMG_GINST(MatF)
SMG_GINST(MatH)
#undef SMG_GINST
template hipError_t launch_lower<MatD>(int, const Grid&, const MatD&, const double*, const double*, double*,
                                       hipStream_t);
template hipError_t launch_lower<MatF>(int, const Grid&, const MatF&, const float*, const float*, float*, hipStream_t);
template hipError_t launch_lower<MatH>(int, const Grid&, const MatH&, const float*, const float*, float*, hipStream_t);
template hipError_t launch_upper<MatD>(int, const Grid&, const MatD&, const double*, const double*, double*,
                                       hipStream_t);
template hipError_t launch_upper<MatF>(int, const Grid&, const MatF&, const float*, const float*, float*, hipStream_t);
template hipError_t launch_upper<MatH>(int, const Grid&, const MatH&, const float*, const float*, float*, hipStream_t);
template hipError_t launch_restrict<double>(const Grid&, int, int, const double*, double*, hipStream_t);
template hipError_t launch_restrict<float>(const Grid&, int, int, const float*, float*, hipStream_t);
template hipError_t launch_prolong_add<double>(const Grid&, int, int, const double*, double*, hipStream_t);
template hipError_t launch_prolong_add<float>(const Grid&, int, int, const float*, float*, hipStream_t);

}  // namespace smg
