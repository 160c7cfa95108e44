// Operator-dependent vertex interpolation (P and R = P^T varying from point
// to point, as in the caption of the generated-code listing, after Dendy's
// black-box multigrid): weights from the level's own stencil, the transfers
// that apply them, and the stencil Galerkin product A_c = P^T A P.
//
// Grid map of the vertex hierarchy: coarse X <-> fine 2X+1 on coarsened axes.
// A fine point f that is even on the coarsened axes of E(f) lies between
// coarse points; its corner on such an axis is lo = f/2 - 1 (c_a = 0) or
// hi = f/2 (c_a = 1), elsewhere the single parent (c_a = 0).  W[c*N + f]
// holds the weight of corner c = (cx*2 + cy)*2 + cz.  Points with E(f) empty
// are coarse points (weight 1).  The others, in order of |E(f)| = 1, 2, 3
// (one launch each), collapse their stencil onto the axes of E(f),
//   Abar(d) = sum of A(f, s) over the canonical s with s_a = d_a on E(f),
// and take W(f, c) = -r * sum over the neighbours g = f + d (d != 0 in the
// box of E(f), lexicographic, g in the grid, on the line of corner c) of
// fma(Abar(d), W(g, c'), .), r = 1 / Abar(0), c'_a = (d_a == 0 ? c_a : 0).
#include <utility>

#include "smg_group.h"
#include "smg_kernels.h"

namespace smg {

namespace {

__device__ inline bool od_even(int f, int cm) { return cm && !(f & 1); }

// index on one axis of corner bit b of fine coordinate f (-1: none)
__device__ inline int od_corner_index(int f, int cm, int b) {
  if (!cm) return b ? -1 : f;
  if (f & 1) return b ? -1 : (f - 1) / 2;
  return f / 2 - 1 + b;
}

template <int PAT>
__global__ __launch_bounds__(256) void k_od_weights(Grid g, int cmask, int k, const double* __restrict__ A,
                                                    double* __restrict__ W, unsigned* err) {
  const long N = g.N();
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int Z = (int)(i % g.nz), Y = (int)((i / g.nz) % g.ny), X = (int)(i / ((long)g.nz * g.ny));
  const int f[3] = {X, Y, Z};
  int ev[3], ne = 0;
  for (int a = 0; a < 3; ++a) ne += ev[a] = od_even(f[a], (cmask >> a) & 1);
  if (ne != k) return;
  if (k == 0) {
    for (int c = 0; c < 8; ++c) W[(long)c * N + i] = c == 0 ? 1.0 : 0.0;
    return;
  }
  double Ab[27];
  for (int d = 0; d < 27; ++d) {
    const int dd[3] = {d / 9 - 1, (d / 3) % 3 - 1, d % 3 - 1};
    bool box = true;
    for (int a = 0; a < 3; ++a)
      if (!ev[a] && dd[a] != 0) box = false;
    double acc = 0.0;
    if (box)
#pragma unroll
      for (int s = 0; s < PAT; ++s) {
        const int o[3] = {pat_off(PAT, s, 0), pat_off(PAT, s, 1), pat_off(PAT, s, 2)};
        bool match = true;
        for (int a = 0; a < 3; ++a)
          if (ev[a] && o[a] != dd[a]) match = false;
        if (match) acc = acc + A[(long)s * N + i];
      }
    Ab[d] = acc;
  }
  if (Ab[13] == 0.0) {
    atomicOr(err, 2u);
    return;
  }
  const double r = 1.0 / Ab[13];
  for (int c = 0; c < 8; ++c) {
    const int cc[3] = {c / 4, (c / 2) % 2, c % 2};
    bool used = true;
    for (int a = 0; a < 3; ++a)
      if (!ev[a] && cc[a]) used = false;
    double acc = 0.0;
    if (used)
      for (int d = 0; d < 27; ++d) {
        if (d == 13) continue;
        const int dd[3] = {d / 9 - 1, (d / 3) % 3 - 1, d % 3 - 1};
        bool ok = true;
        int gg[3], cp = 0;
        for (int a = 0; a < 3; ++a) {
          if (!ev[a] && dd[a] != 0) ok = false;
          if (dd[a] == 1 && cc[a] != 1) ok = false;
          if (dd[a] == -1 && cc[a] != 0) ok = false;
          gg[a] = f[a] + dd[a];
        }
        if (!ok || !in_grid(g, gg[0], gg[1], gg[2])) continue;
        for (int a = 0; a < 3; ++a) cp = cp * 2 + (dd[a] == 0 ? cc[a] : 0);
        const long j = ((long)gg[0] * g.ny + gg[1]) * g.nz + gg[2];
        acc = fma(Ab[d], W[(long)cp * N + j], acc);
      }
    W[(long)c * N + i] = used ? -acc * r : 0.0;
  }
}

// r_c[I] = sum over u = fine(I) + rho (rho lexicographic, u in the grid) of
// fma(W(u, corner I), r_f[u], acc) from zero (R = P^T).
template <class V>
__global__ __launch_bounds__(256) void k_restrict_od(Grid gf, int cmask, const V* __restrict__ W,
                                                     const V* __restrict__ rf, V* __restrict__ rc) {
  const int cx = cmask & 1, cy = (cmask >> 1) & 1, cz = (cmask >> 2) & 1;
  const Grid gc{cx ? gf.nx / 2 : gf.nx, cy ? gf.ny / 2 : gf.ny, cz ? gf.nz / 2 : gf.nz};
  const long Nf = gf.N();
  const long ic = (long)blockIdx.x * 256 + threadIdx.x;
  if (ic >= gc.N()) return;
  const int Z = (int)(ic % gc.nz), Y = (int)((ic / gc.nz) % gc.ny), X = (int)(ic / ((long)gc.nz * gc.ny));
  const int fx = cx ? 2 * X + 1 : X, fy = cy ? 2 * Y + 1 : Y, fz = cz ? 2 * Z + 1 : Z;
  // all 27 candidate fine points, lexicographic; the loads are
  // unconditional (a point outside the grid or on an uncoarsened axis offset
  // reads the centre point fine(I), c = 0) so a thread's loads are in flight
  // together, and such points leave the sum unchanged
  const long i0 = ((long)fx * gf.ny + fy) * gf.nz + fz;
  V w[27], r[27];
  bool ok[27];
#pragma unroll
  for (int d = 0; d < 27; ++d) {
    const int dx = d / 9 - 1, dy = (d / 3) % 3 - 1, dz = d % 3 - 1;
    const int ux = fx + dx, uy = fy + dy, uz = fz + dz;
    ok[d] = (cx || dx == 0) && (cy || dy == 0) && (cz || dz == 0) && in_grid(gf, ux, uy, uz);
    // I is the hi corner of an even coordinate reached from below
    const int c = ((dx < 0 ? 1 : 0) * 2 + (dy < 0 ? 1 : 0)) * 2 + (dz < 0 ? 1 : 0);
    const long iu = ok[d] ? ((long)ux * gf.ny + uy) * gf.nz + uz : i0;
    w[d] = W[(ok[d] ? (long)c * Nf : 0L) + iu];
    r[d] = rf[iu];
  }
  V acc = V(0);
#pragma unroll
  for (int d = 0; d < 27; ++d) acc = ok[d] ? fma(w[d], r[d], acc) : acc;
  rc[ic] = acc;
}

// uout[f] = uin[f] + pe, pe = sum over the corners c in order of
// fma(W(f, c), e_c[corner], pe) from zero (uout may be uin).
template <class V>
__global__ __launch_bounds__(256) void k_prolong_od(Grid gf, int cmask, const V* __restrict__ W,
                                                    const V* __restrict__ ec, const V* uin, V* uout) {
  const int cx = cmask & 1, cy = (cmask >> 1) & 1, cz = (cmask >> 2) & 1;
  const Grid gc{cx ? gf.nx / 2 : gf.nx, cy ? gf.ny / 2 : gf.ny, cz ? gf.nz / 2 : gf.nz};
  const long Nf = gf.N();
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= Nf) return;
  const int Z = (int)(i % gf.nz), Y = (int)((i / gf.nz) % gf.ny), X = (int)(i / ((long)gf.nz * gf.ny));
  // every load is unconditional so that a thread's loads are in flight
  // together: a corner the point does not have reads the point's corner-0
  // weight (a line the thread reads anyway) and coarse entry 0, and leaves
  // the sum unchanged
  V w[8], e[8];
  bool ok[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int jx = od_corner_index(X, cx, c / 4), jy = od_corner_index(Y, cy, (c / 2) % 2),
              jz = od_corner_index(Z, cz, c % 2);
    ok[c] = in_grid(gc, jx, jy, jz);
    w[c] = W[(ok[c] ? (long)c * Nf : 0L) + i];
    e[c] = ec[ok[c] ? ((long)jx * gc.ny + jy) * gc.nz + jz : 0L];
  }
  V pe = V(0);
#pragma unroll
  for (int c = 0; c < 8; ++c) pe = ok[c] ? fma(w[c], e[c], pe) : pe;
  uout[i] = uin[i] + pe;
}

// A_c = P^T A P, 27-point: one thread per coarse point I computes all 27
// coarse offsets n.  Over the fine points u = fine(I) + rho (rho
// lexicographic, u in the grid; I is always a corner of u) the partial sums
// t[n] collect fma(A(u, s), W(g, corner c), t[n]) over the canonical s with
// g = u + s in the grid and the corners c of g, n = J_c - I; then
// acc[n] = fma(W(u, corner I), t[n], acc[n]).  rho, s and c are unrolled at
// compile time, so every coarse offset is a constant and the sums stay in
// registers; offsets whose J lies outside the coarse grid are stored as 0.
// CM: the coarsening mask.
// offset component of corner bit c on one axis for q = rho_a + s_a (-1: none)
__host__ __device__ constexpr int od_noff(bool cm, int rho, int s, int c) {
  return !cm ? (c ? -9 : s)
             : (((rho + s) % 2 == 0) ? (c ? -9 : (rho + s) / 2) : ((rho + s + 2 - 1) / 2 - 1 + c));
}

template <int PAT, int CM, int RHO, int S>
__device__ __forceinline__ void od_rap_s(double (&t)[27], const double* __restrict__ A, const double* __restrict__ W,
                                         long Nf, long iu, const Grid& gf, int ux, int uy, int uz) {
  constexpr int rx = RHO / 9 - 1, ry = (RHO / 3) % 3 - 1, rz = RHO % 3 - 1;
  constexpr int sx = pat_off(PAT, S, 0), sy = pat_off(PAT, S, 1), sz = pat_off(PAT, S, 2);
  const int gx = ux + sx, gy = uy + sy, gz = uz + sz;
  if (!in_grid(gf, gx, gy, gz)) return;
  const double a = A[(long)S * Nf + iu];
  const long ig = ((long)gx * gf.ny + gy) * gf.nz + gz;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int nx = od_noff(CM & 1, rx, sx, c / 4), ny = od_noff((CM >> 1) & 1, ry, sy, (c / 2) % 2),
              nz = od_noff((CM >> 2) & 1, rz, sz, c % 2);
    if (nx < -1 || ny < -1 || nz < -1 || nx > 1 || ny > 1 || nz > 1) continue;
    const int n = (nx + 1) * 9 + (ny + 1) * 3 + (nz + 1);
    t[n] = fma(a, W[(long)c * Nf + ig], t[n]);
  }
}

template <int PAT, int CM, int RHO, int... S>
__device__ __forceinline__ void od_rap_rho(double (&acc)[27], const double* __restrict__ A,
                                           const double* __restrict__ W, long Nf, const Grid& gf, int fx, int fy,
                                           int fz, std::integer_sequence<int, S...>) {
  constexpr int rx = RHO / 9 - 1, ry = (RHO / 3) % 3 - 1, rz = RHO % 3 - 1;
  if constexpr ((rx != 0 && !(CM & 1)) || (ry != 0 && !(CM & 2)) || (rz != 0 && !(CM & 4))) {
    return;
  } else {
    const int ux = fx + rx, uy = fy + ry, uz = fz + rz;
    if (!in_grid(gf, ux, uy, uz)) return;
    const long iu = ((long)ux * gf.ny + uy) * gf.nz + uz;
    // corner of u that is I: hi (1) where u is even below fine(I), else 0
    constexpr int cu = ((rx < 0 ? 1 : 0) * 2 + (ry < 0 ? 1 : 0)) * 2 + (rz < 0 ? 1 : 0);
    double t[27];
#pragma unroll
    for (int n = 0; n < 27; ++n) t[n] = 0.0;
    (od_rap_s<PAT, CM, RHO, S>(t, A, W, Nf, iu, gf, ux, uy, uz), ...);
    const double wu = W[(long)cu * Nf + iu];
#pragma unroll
    for (int n = 0; n < 27; ++n) acc[n] = fma(wu, t[n], acc[n]);
  }
}

template <int PAT, int CM, int... RHO>
__device__ __forceinline__ void od_rap_all(double (&acc)[27], const double* __restrict__ A,
                                           const double* __restrict__ W, long Nf, const Grid& gf, int fx, int fy,
                                           int fz, std::integer_sequence<int, RHO...>) {
  (od_rap_rho<PAT, CM, RHO>(acc, A, W, Nf, gf, fx, fy, fz, std::make_integer_sequence<int, PAT>{}), ...);
}

template <int PAT, int CM>
__global__ __launch_bounds__(256) void k_rap_od_all(Grid gf, const double* __restrict__ A,
                                                    const double* __restrict__ W, double* __restrict__ Ac) {
  constexpr int cx = CM & 1, cy = (CM >> 1) & 1, cz = (CM >> 2) & 1;
  const Grid gc{cx ? gf.nx / 2 : gf.nx, cy ? gf.ny / 2 : gf.ny, cz ? gf.nz / 2 : gf.nz};
  const long Nf = gf.N(), Nc = gc.N();
  // contiguous coarse lines per XCD: neighbouring lines share most of their
  // fine neighbourhood, which then stays in one L2
  const long ic = (long)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (ic >= Nc) return;
  const int Z = (int)(ic % gc.nz), Y = (int)((ic / gc.nz) % gc.ny), X = (int)(ic / ((long)gc.nz * gc.ny));
  double acc[27];
#pragma unroll
  for (int n = 0; n < 27; ++n) acc[n] = 0.0;
  od_rap_all<PAT, CM>(acc, A, W, Nf, gf, cx ? 2 * X + 1 : X, cy ? 2 * Y + 1 : Y, cz ? 2 * Z + 1 : Z,
                      std::make_integer_sequence<int, 27>{});
#pragma unroll
  for (int n = 0; n < 27; ++n) {
    const bool inJ = in_grid(gc, X + n / 9 - 1, Y + (n / 3) % 3 - 1, Z + n % 3 - 1);
    Ac[(long)n * Nc + ic] = inJ ? acc[n] : 0.0;
  }
}

template <int PAT, int CM>
hipError_t launch_rap_od_all_t(const Grid& gf, const double* A, const double* W, double* Ac, hipStream_t st) {
  const long nc = (long)((CM & 1) ? gf.nx / 2 : gf.nx) * ((CM & 2) ? gf.ny / 2 : gf.ny) * ((CM & 4) ? gf.nz / 2 : gf.nz);
  hipLaunchKernelGGL((k_rap_od_all<PAT, CM>), dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, gf, A, W, Ac);
  return hipGetLastError();
}

template <int PAT>
hipError_t launch_rap_od_all_p(int cmask, const Grid& gf, const double* A, const double* W, double* Ac,
                               hipStream_t st) {
  switch (cmask) {
    case 1: return launch_rap_od_all_t<PAT, 1>(gf, A, W, Ac, st);
    case 2: return launch_rap_od_all_t<PAT, 2>(gf, A, W, Ac, st);
    case 3: return launch_rap_od_all_t<PAT, 3>(gf, A, W, Ac, st);
    case 4: return launch_rap_od_all_t<PAT, 4>(gf, A, W, Ac, st);
    case 5: return launch_rap_od_all_t<PAT, 5>(gf, A, W, Ac, st);
    case 6: return launch_rap_od_all_t<PAT, 6>(gf, A, W, Ac, st);
    case 7: return launch_rap_od_all_t<PAT, 7>(gf, A, W, Ac, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_od_weights(int pat, const Grid& g, int cmask, const double* A, double* W, unsigned* err,
                             hipStream_t st) {
  const dim3 grid((unsigned)((g.N() + 255) / 256)), blk(256);
  for (int k = 0; k <= 3; ++k) {
    if (pat == 7)
      hipLaunchKernelGGL(k_od_weights<7>, grid, blk, 0, st, g, cmask, k, A, W, err);
    else if (pat == 19)
      hipLaunchKernelGGL(k_od_weights<19>, grid, blk, 0, st, g, cmask, k, A, W, err);
    else if (pat == 27)
      hipLaunchKernelGGL(k_od_weights<27>, grid, blk, 0, st, g, cmask, k, A, W, err);
    else
      return hipErrorInvalidValue;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <class V>
hipError_t launch_restrict_od(const Grid& gf, int cmask, const V* W, const V* rf, V* rc, hipStream_t st) {
  const long n = (long)((cmask & 1) ? gf.nx / 2 : gf.nx) * ((cmask & 2) ? gf.ny / 2 : gf.ny) *
                 ((cmask & 4) ? gf.nz / 2 : gf.nz);
  hipLaunchKernelGGL(k_restrict_od<V>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, gf, cmask, W, rf, rc);
  return hipGetLastError();
}

template <class V>
hipError_t launch_prolong_od(const Grid& gf, int cmask, const V* W, const V* ec, const V* uin, V* uout,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_prolong_od<V>, dim3((unsigned)((gf.N() + 255) / 256)), dim3(256), 0, st, gf, cmask, W, ec, uin,
                     uout);
  return hipGetLastError();
}

hipError_t launch_rap_od(int pat, int cmask, const Grid& gf, const double* A, const double* W, double* Ac,
                         hipStream_t st) {
  if (pat == 7) return launch_rap_od_all_p<7>(cmask, gf, A, W, Ac, st);
  if (pat == 19) return launch_rap_od_all_p<19>(cmask, gf, A, W, Ac, st);
  if (pat == 27) return launch_rap_od_all_p<27>(cmask, gf, A, W, Ac, st);
  return hipErrorInvalidValue;
}

template hipError_t launch_restrict_od<double>(const Grid&, int, const double*, const double*, double*, hipStream_t);
template hipError_t launch_restrict_od<float>(const Grid&, int, const float*, const float*, float*, hipStream_t);
template hipError_t launch_prolong_od<double>(const Grid&, int, const double*, const double*, const double*, double*,
                                              hipStream_t);
template hipError_t launch_prolong_od<float>(const Grid&, int, const float*, const float*, const float*, float*,
                                             hipStream_t);

}  // namespace smg
