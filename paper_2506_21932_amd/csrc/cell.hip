// Cell-centred transfer operators and their stencil Galerkin products (the
// Cell_3d8 interpolation / restriction pair of the R/A/P combinations table,
// suffix "c", and the Cell_3d8 restriction with the cell-centred trilinear
// Cell_3d64 interpolation).  Coarse cell I owns the fine cells 2I + d, d in {0,1} on each
// coarsened axis (0 on the others); a coarsened axis keeps ceil(n_f / 2)
// cells.  P is piecewise constant (a fine cell takes its parent's value),
// R = P^T sums a coarse cell's children.  With these, A_c = R A P keeps the
// fine pattern: a fine coupling of offset s can only connect a child of I to
// a child of I + n with n inside the same pattern.  With the trilinear
// interpolation instead the coarse operators are 27-point.
#include "smg_kernels.h"

namespace smg {

namespace {

__host__ __device__ inline Grid cc_coarse(const Grid& gf, int cmask) {
  return Grid{(cmask & 1) ? (gf.nx + 1) / 2 : gf.nx, (cmask & 2) ? (gf.ny + 1) / 2 : gf.ny,
              (cmask & 4) ? (gf.nz + 1) / 2 : gf.nz};
}

// r_c[I] = sum over the children of I in lexicographic order of d, from zero.
template <class V>
__global__ __launch_bounds__(256) void k_restrict_cc(Grid gf, int cmask, int bs, const V* __restrict__ rf,
                                                     V* __restrict__ rc) {
  const Grid gc = cc_coarse(gf, cmask);
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= gc.N() * bs) return;
  const long ic = t / bs;
  const int comp = (int)(t - ic * bs);
  const int Z = (int)(ic % gc.nz), Y = (int)((ic / gc.nz) % gc.ny), X = (int)(ic / ((long)gc.nz * gc.ny));
  const int cx = cmask & 1, cy = (cmask >> 1) & 1, cz = (cmask >> 2) & 1;
  V acc = V(0);
  for (int dx = 0; dx <= cx; ++dx)
    for (int dy = 0; dy <= cy; ++dy)
      for (int dz = 0; dz <= cz; ++dz) {
        const int fx = cx ? 2 * X + dx : X, fy = cy ? 2 * Y + dy : Y, fz = cz ? 2 * Z + dz : Z;
        if (fx < gf.nx && fy < gf.ny && fz < gf.nz) acc = acc + rf[(((long)fx * gf.ny + fy) * gf.nz + fz) * bs + comp];
      }
  rc[t] = acc;
}

// uout[f] = uin[f] + ec[parent(f)]  (uout may be uin)
template <class V>
__global__ __launch_bounds__(256) void k_prolong_cc(Grid gf, int cmask, int bs, const V* __restrict__ ec,
                                                    const V* uin, V* uout) {
  const Grid gc = cc_coarse(gf, cmask);
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= gf.N() * bs) return;
  const long i = t / bs;
  const int comp = (int)(t - i * bs);
  const int Z = (int)(i % gf.nz), Y = (int)((i / gf.nz) % gf.ny), X = (int)(i / ((long)gf.nz * gf.ny));
  const int JX = (cmask & 1) ? X / 2 : X, JY = (cmask & 2) ? Y / 2 : Y, JZ = (cmask & 4) ? Z / 2 : Z;
  uout[t] = uin[t] + ec[(((long)JX * gc.ny + JY) * gc.nz + JZ) * bs + comp];
}

// A_c(I, n) = sum of A(f, s) over the children f of I (lexicographic d) and
// the fine offsets s (canonical order) with f + s in the grid and
// parent(f + s) = I + n; plain additions from zero.  One thread per coarse
// point and coarse offset n.
template <int PAT>
__global__ __launch_bounds__(256) void k_rap_cc(Grid gf, int cmask, const double* __restrict__ A, long sA,
                                                double* __restrict__ Ac, long sAc) {
  const Grid gc = cc_coarse(gf, cmask);
  const long Nc = gc.N();
  // block b: coarse points [256*(b/PAT), +256) for offset n = b % PAT (the
  // PAT blocks of one tile run together and share their fine reads)
  const int n = (int)(blockIdx.x % (unsigned)PAT);
  const long ic = (long)(blockIdx.x / (unsigned)PAT) * 256 + threadIdx.x;
  if (ic >= Nc) return;
  const int Z = (int)(ic % gc.nz), Y = (int)((ic / gc.nz) % gc.ny), X = (int)(ic / ((long)gc.nz * gc.ny));
  const int cx = cmask & 1, cy = (cmask >> 1) & 1, cz = (cmask >> 2) & 1;
  const int nx = pat_off(PAT, n, 0), ny = pat_off(PAT, n, 1), nz = pat_off(PAT, n, 2);
  double acc = 0.0;
  for (int dx = 0; dx <= cx; ++dx)
    for (int dy = 0; dy <= cy; ++dy)
      for (int dz = 0; dz <= cz; ++dz) {
        const int fx = cx ? 2 * X + dx : X, fy = cy ? 2 * Y + dy : Y, fz = cz ? 2 * Z + dz : Z;
        if (fx >= gf.nx || fy >= gf.ny || fz >= gf.nz) continue;
        const long i = ((long)fx * gf.ny + fy) * gf.nz + fz;
#pragma unroll
        for (int s = 0; s < PAT; ++s) {
          const int gx = fx + pat_off(PAT, s, 0), gy = fy + pat_off(PAT, s, 1), gz = fz + pat_off(PAT, s, 2);
          if (!in_grid(gf, gx, gy, gz)) continue;
          if ((cx ? gx / 2 : gx) - X == nx && (cy ? gy / 2 : gy) - Y == ny && (cz ? gz / 2 : gz) - Z == nz)
            acc = acc + A[(long)s * sA + i];
        }
      }
  Ac[(long)n * sAc + ic] = acc;
}

// Contributors of fine index g on one axis for the cell-centred trilinear
// interpolation (3d64c): parent I = g/2 with 3/4 and the neighbour on g's
// side (I-1 for even g, I+1 for odd g) with 1/4, ascending index, those
// outside [0, nc) dropped; a non-coarsened axis has the single contributor g.
template <class V>
__device__ inline int c64_axis(int g, int cm, int nc, int (&par)[2], V (&wt)[2]) {
  if (!cm) {
    par[0] = g;
    wt[0] = V(1);
    return 1;
  }
  const int I = g / 2, J = (g & 1) ? I + 1 : I - 1;
  const int lo = J < I ? J : I, hi = J < I ? I : J;
  int n = 0;
  if (lo >= 0 && lo < nc) {
    par[n] = lo;
    wt[n] = lo == I ? V(0.75) : V(0.25);
    ++n;
  }
  if (hi >= 0 && hi < nc) {
    par[n] = hi;
    wt[n] = hi == I ? V(0.75) : V(0.25);
    ++n;
  }
  return n;
}

// uout[f] = uin[f] + sum_J w_J ec[J] (contributors in lexicographic order,
// pe = fma(w, e_J, pe) from zero); uout may be uin.
template <class V>
__global__ __launch_bounds__(256) void k_prolong_c64(Grid gf, int cmask, int bs, const V* __restrict__ ec,
                                                     const V* uin, V* uout) {
  const Grid gc = cc_coarse(gf, cmask);
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= gf.N() * bs) return;
  const long i = t / bs;
  const int comp = (int)(t - i * bs);
  const int Z = (int)(i % gf.nz), Y = (int)((i / gf.nz) % gf.ny), X = (int)(i / ((long)gf.nz * gf.ny));
  int px[2], py[2], pz[2];
  V wx[2], wy[2], wz[2];
  const int nx = c64_axis<V>(X, cmask & 1, gc.nx, px, wx), ny = c64_axis<V>(Y, (cmask >> 1) & 1, gc.ny, py, wy),
            nz = c64_axis<V>(Z, (cmask >> 2) & 1, gc.nz, pz, wz);
  V pe = V(0);
  for (int p = 0; p < nx; ++p)
    for (int q = 0; q < ny; ++q)
      for (int r = 0; r < nz; ++r)
        pe = fma(wx[p] * wy[q] * wz[r], ec[(((long)px[p] * gc.ny + py[q]) * gc.nz + pz[r]) * bs + comp], pe);
  uout[t] = uin[t] + pe;
}

// A_c(I, n) for the 27 coarse offsets n: over the children f of I
// (lexicographic d), the fine offsets s (canonical) with g = f + s in the
// grid and the interpolation contributors J of g with J - I = n:
// acc = fma(A(f, s), w_J, acc) from zero.  One thread per (coarse point, n).
template <int PAT>
__global__ __launch_bounds__(256) void k_rap_c64(Grid gf, int cmask, const double* __restrict__ A, long sA,
                                                 double* __restrict__ Ac, long sAc) {
  const Grid gc = cc_coarse(gf, cmask);
  const long Nc = gc.N();
  // block b: coarse points [256*(b/27), +256) for offset n = b % 27
  const int n = (int)(blockIdx.x % 27u);
  const long ic = (long)(blockIdx.x / 27u) * 256 + threadIdx.x;
  if (ic >= Nc) return;
  const int Z = (int)(ic % gc.nz), Y = (int)((ic / gc.nz) % gc.ny), X = (int)(ic / ((long)gc.nz * gc.ny));
  const int cx = cmask & 1, cy = (cmask >> 1) & 1, cz = (cmask >> 2) & 1;
  const int JX = X + pat_off(27, n, 0), JY = Y + pat_off(27, n, 1), JZ = Z + pat_off(27, n, 2);
  double acc = 0.0;
  for (int dx = 0; dx <= cx; ++dx)
    for (int dy = 0; dy <= cy; ++dy)
      for (int dz = 0; dz <= cz; ++dz) {
        const int fx = cx ? 2 * X + dx : X, fy = cy ? 2 * Y + dy : Y, fz = cz ? 2 * Z + dz : Z;
        if (fx >= gf.nx || fy >= gf.ny || fz >= gf.nz) continue;
        const long i = ((long)fx * gf.ny + fy) * gf.nz + fz;
#pragma unroll
        for (int s = 0; s < PAT; ++s) {
          const int gx = fx + pat_off(PAT, s, 0), gy = fy + pat_off(PAT, s, 1), gz = fz + pat_off(PAT, s, 2);
          if (!in_grid(gf, gx, gy, gz)) continue;
          int px[2], py[2], pz[2];
          double wx[2], wy[2], wz[2];
          const int nx = c64_axis<double>(gx, cx, gc.nx, px, wx), ny = c64_axis<double>(gy, cy, gc.ny, py, wy),
                    nz = c64_axis<double>(gz, cz, gc.nz, pz, wz);
          const double av = A[(long)s * sA + i];
          for (int p = 0; p < nx; ++p)
            for (int q = 0; q < ny; ++q)
              for (int r = 0; r < nz; ++r)
                if (px[p] == JX && py[q] == JY && pz[r] == JZ) acc = fma(av, wx[p] * wy[q] * wz[r], acc);
        }
      }
  Ac[(long)n * sAc + ic] = acc;
}

}  // namespace

template <class V>
hipError_t launch_prolong_c64(const Grid& gf, int cmask, int bs, const V* ec, const V* uin, V* uout,
                              hipStream_t st) {
  const long n = gf.N() * bs;
  hipLaunchKernelGGL(k_prolong_c64<V>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, gf, cmask, bs, ec, uin,
                     uout);
  return hipGetLastError();
}

hipError_t launch_rap_c64(int pat, int cmask, const Grid& gf, const double* A, long sA, double* Ac, long sAc,
                          hipStream_t st) {
  const long n = cc_coarse(gf, cmask).N();
  const dim3 grid((unsigned)((n + 255) / 256 * 27)), blk(256);
  if (pat == 7)
    hipLaunchKernelGGL(k_rap_c64<7>, grid, blk, 0, st, gf, cmask, A, sA, Ac, sAc);
  else if (pat == 19)
    hipLaunchKernelGGL(k_rap_c64<19>, grid, blk, 0, st, gf, cmask, A, sA, Ac, sAc);
  else if (pat == 27)
    hipLaunchKernelGGL(k_rap_c64<27>, grid, blk, 0, st, gf, cmask, A, sA, Ac, sAc);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class V>
hipError_t launch_restrict_cc(const Grid& gf, int cmask, int bs, const V* rf, V* rc, hipStream_t st) {
  const long n = cc_coarse(gf, cmask).N() * bs;
  hipLaunchKernelGGL(k_restrict_cc<V>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, gf, cmask, bs, rf, rc);
  return hipGetLastError();
}

template <class V>
hipError_t launch_prolong_cc(const Grid& gf, int cmask, int bs, const V* ec, const V* uin, V* uout, hipStream_t st) {
  const long n = gf.N() * bs;
  hipLaunchKernelGGL(k_prolong_cc<V>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, gf, cmask, bs, ec, uin,
                     uout);
  return hipGetLastError();
}

hipError_t launch_rap_cc(int pat, int cmask, const Grid& gf, const double* A, long sA, double* Ac, long sAc,
                         hipStream_t st) {
  const long n = cc_coarse(gf, cmask).N();
  const dim3 grid((unsigned)((n + 255) / 256 * pat)), blk(256);
  if (pat == 7)
    hipLaunchKernelGGL(k_rap_cc<7>, grid, blk, 0, st, gf, cmask, A, sA, Ac, sAc);
  else if (pat == 19)
    hipLaunchKernelGGL(k_rap_cc<19>, grid, blk, 0, st, gf, cmask, A, sA, Ac, sAc);
  else if (pat == 27)
    hipLaunchKernelGGL(k_rap_cc<27>, grid, blk, 0, st, gf, cmask, A, sA, Ac, sAc);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template hipError_t launch_restrict_cc<double>(const Grid&, int, int, const double*, double*, hipStream_t);
template hipError_t launch_restrict_cc<float>(const Grid&, int, int, const float*, float*, hipStream_t);
template hipError_t launch_prolong_cc<double>(const Grid&, int, int, const double*, const double*, double*,
                                              hipStream_t);
template hipError_t launch_prolong_cc<float>(const Grid&, int, int, const float*, const float*, float*, hipStream_t);
template hipError_t launch_prolong_c64<double>(const Grid&, int, int, const double*, const double*, double*,
                                               hipStream_t);
template hipError_t launch_prolong_c64<float>(const Grid&, int, int, const float*, const float*, float*,
                                              hipStream_t);

}  // namespace smg
