/*
 * CPU ORACLE — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential FP64 implementation of the structured multigrid
 * preconditioner of "StructMG: A Fast and Scalable Structured Algebraic
 * Multigrid" (arXiv 2506.21932): SG-DIA stencil SpMV and residual
 * (Sec. 4.1 P1), lexicographic Gauss-Seidel and ILU(0) (Sec. 4.4 formulas),
 * vertex-centred trilinear restriction / prolongation with the grid map of
 * Sec. 4.3, the stencil Galerkin triple product A^C = R A^F P in its
 * influence-chain form (Sec. 4.3, Eq. for A^C(i,j) as a sum over chains),
 * the V-cycle (Sec. 2), and the outer CG and GMRES iterations (Sec. 5.2).
 *
 * Only tests, the smoke check and the CPU-baseline leg of the benchmark load
 * this library.  It shares no code, header or table with the GPU library;
 * both follow the same written conventions (lexicographic offset order,
 * z-fastest linear index, fma accumulation in the stated order).
 *
 * Build: gcc -O2 -mfma -ffp-contract=off -fPIC -shared oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- precision-generic kernels (scalar and 3x3-block) ---------------- */
#define REAL double
#define FMA fma
#define SFX _f64
#include "oracle_kernels.inc"
#undef REAL
#undef FMA
#undef SFX

#define REAL float
#define FMA fmaf
#define SFX _f32
#include "oracle_kernels.inc"
#undef REAL
#undef FMA
#undef SFX

/* ---- IEEE binary16 conversion (round to nearest even), written from the
 * IEEE 754 definition; used for the FP16 row-scaled truncation. ---------- */
uint16_t orc_f32_to_f16(float f) {
  uint32_t x;
  memcpy(&x, &f, 4);
  uint32_t sign = (x >> 16) & 0x8000u;
  uint32_t ax = x & 0x7fffffffu;
  if (ax >= 0x7f800000u) /* inf / nan */
    return (uint16_t)(sign | 0x7c00u | (ax > 0x7f800000u ? (0x200u | ((ax >> 13) & 0x3ffu)) : 0u));
  if (ax >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u); /* >= 65520 rounds to inf */
  int e = (int)(ax >> 23) - 127;
  if (e >= -14) {
    uint32_t mant = ax & 0x7fffffu;
    uint32_t h = ((uint32_t)(e + 15) << 10) | (mant >> 13);
    uint32_t rem = mant & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) h += 1u;
    return (uint16_t)(sign | h);
  }
  if (e < -25) return (uint16_t)sign;
  uint32_t mant = (ax & 0x7fffffu) | 0x800000u;
  int shift = -e - 1; /* 14..24 */
  uint32_t hm = mant >> shift, rem = mant & ((1u << shift) - 1u), half = 1u << (shift - 1);
  if (rem > half || (rem == half && (hm & 1u))) hm += 1u;
  return (uint16_t)(sign | hm);
}

float orc_f16_to_f32(uint16_t h) {
  uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
  int e = (h >> 10) & 0x1f;
  uint32_t m = h & 0x3ffu, bits;
  float out;
  if (e == 0) {
    out = ldexpf((float)m, -24);
    return sign ? -out : out;
  }
  if (e == 31)
    bits = sign | 0x7f800000u | (m << 13);
  else
    bits = sign | ((uint32_t)(e - 15 + 127) << 23) | (m << 13);
  memcpy(&out, &bits, 4);
  return out;
}

/* ---- stencil patterns ------------------------------------------------- */
/* Fills off[] with the offsets of a 3D pattern (7, 19 or 27 points) in
 * lexicographic (dx slowest) order; returns the number of points. */
int orc_pattern(int npts, int* off) {
  int S = 0;
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dz = -1; dz <= 1; ++dz) {
        int m = abs(dx) + abs(dy) + abs(dz);
        int keep = npts == 27 || (npts == 19 && m <= 2) || (npts == 7 && m <= 1);
        if (!keep) continue;
        off[3 * S] = dx; off[3 * S + 1] = dy; off[3 * S + 2] = dz;
        ++S;
      }
  return S;
}

/* ---- Galerkin triple product ----------------------------------------- */
static int rap_chain_ok(const int* rho, const int* a, const int* n, int cmask, double* wR, double* wP) {
  /* R(I, fine(I)+rho) and P(fine(I)+rho+a, I+n) both nonzero? */
  double r = 1.0, p = 1.0;
  for (int ax = 0; ax < 3; ++ax) {
    int cm = (cmask >> ax) & 1;
    if (!cm) {
      if (rho[ax] != 0) return 0;
      if (a[ax] != n[ax]) return 0;
    } else {
      int d = rho[ax] + a[ax] - 2 * n[ax]; /* v - fine(J) along this axis */
      if (d < -1 || d > 1) return 0;
      if (rho[ax] != 0) r *= 0.5;
      if (d != 0) p *= 0.5;
    }
  }
  *wR = r;
  *wP = p;
  return 1;
}

/*
 * A^C = R A^F P, stencil form (Sec. 4.3): for each coarse element I and each
 * of the 27 coarse offsets n (canonical order), the entry A^C(I, I+n) is the
 * sum over influence chains I <- u <- v <- I+n of R(I,u) A^F(u,v) P(v,I+n),
 * grouped per fine element u as
 *     tmp = sum_a A^F[a][u] * P(u+a, J);  res += tmp * R(I, u).
 * u runs over fine(I)+rho (rho canonical), a over the fine pattern
 * (canonical); only in-grid u, v and J contribute.  bs = 3 treats each of
 * the 9 block entries as an independent scalar field (P, R act per unknown).
 * Output Ac[(n*bs*bs + e)*Nc + I], with Nc the coarse grid size.
 */
/* The 27 * bs^2 entries of coarse row I, written to Ac[(n * be + e) * ldc]. */
static void rap_row(const int* nf, const int* nc, int S, const int* off, int bs, const double* Af, int cmask,
                    const int* I, double* Ac, long ldc) {
  int cm[3], fI[3];
  long Nf = (long)nf[0] * nf[1] * nf[2];
  int be = bs * bs;
  for (int a = 0; a < 3; ++a) {
    cm[a] = (cmask >> a) & 1;
    fI[a] = cm[a] ? 2 * I[a] + 1 : I[a];
  }
  int ni = 0;
  for (int nx_ = -1; nx_ <= 1; ++nx_)
    for (int ny_ = -1; ny_ <= 1; ++ny_)
      for (int nz_ = -1; nz_ <= 1; ++nz_, ++ni) {
        int n[3] = {nx_, ny_, nz_}, J[3], inJ = 1;
        for (int a = 0; a < 3; ++a) {
          J[a] = I[a] + n[a];
          if (J[a] < 0 || J[a] >= nc[a]) inJ = 0;
        }
        for (int e = 0; e < be; ++e) {
          double res = 0.0;
          if (inJ) {
            for (int rx = -1; rx <= 1; ++rx)
              for (int ry = -1; ry <= 1; ++ry)
                for (int rz = -1; rz <= 1; ++rz) {
                  int rho[3] = {rx, ry, rz}, u[3], inU = 1;
                  for (int a = 0; a < 3; ++a) {
                    u[a] = fI[a] + rho[a];
                    if (u[a] < 0 || u[a] >= nf[a]) inU = 0;
                  }
                  if (!inU) continue;
                  int anyc = 0;
                  double wR = 1.0, tmp = 0.0;
                  long iu = ((long)u[0] * nf[1] + u[1]) * nf[2] + u[2];
                  for (int s = 0; s < S; ++s) {
                    double wr, wp;
                    if (!rap_chain_ok(rho, &off[3 * s], n, cmask, &wr, &wp)) continue;
                    int v0 = u[0] + off[3 * s], v1 = u[1] + off[3 * s + 1], v2 = u[2] + off[3 * s + 2];
                    if (v0 < 0 || v0 >= nf[0] || v1 < 0 || v1 >= nf[1] || v2 < 0 || v2 >= nf[2]) continue;
                    wR = wr;
                    anyc = 1;
                    tmp = fma(Af[((long)s * be + e) * Nf + iu], wp, tmp);
                  }
                  if (anyc) res = fma(tmp, wR, res);
                }
          }
          Ac[((long)ni * be + e) * ldc] = res;
        }
      }
}

void orc_rap(int nxf, int nyf, int nzf, int S, const int* off, int bs, const double* Af, int cmask,
             double* Ac) {
  int nf[3] = {nxf, nyf, nzf}, nc[3];
  for (int a = 0; a < 3; ++a) nc[a] = (cmask >> a) & 1 ? nf[a] / 2 : nf[a];
  long Nc = (long)nc[0] * nc[1] * nc[2];
  for (int X = 0; X < nc[0]; ++X)
    for (int Y = 0; Y < nc[1]; ++Y)
      for (int Z = 0; Z < nc[2]; ++Z) {
        int I[3] = {X, Y, Z};
        long ic = ((long)X * nc[1] + Y) * nc[2] + Z;
        rap_row(nf, nc, S, off, bs, Af, cmask, I, Ac + ic, Nc);
      }
}

/* The same rows at npts listed coarse points (flat coarse indices pts[k]):
 * Ac[(n * be + e) * npts + k]. */
void orc_rap_points(int nxf, int nyf, int nzf, int S, const int* off, int bs, const double* Af, int cmask,
                    int npts, const long* pts, double* Ac) {
  int nf[3] = {nxf, nyf, nzf}, nc[3];
  for (int a = 0; a < 3; ++a) nc[a] = (cmask >> a) & 1 ? nf[a] / 2 : nf[a];
  for (int k = 0; k < npts; ++k) {
    long ic = pts[k];
    int I[3] = {(int)(ic / ((long)nc[1] * nc[2])), (int)((ic / nc[2]) % nc[1]), (int)(ic % nc[2])};
    rap_row(nf, nc, S, off, bs, Af, cmask, I, Ac + k, npts);
  }
}

/*
 * Influence chains of one coarse offset n for an interior coarse element:
 * writes triples (rho index in the 27-point fine neighbourhood, fine-pattern
 * index, P index in the 27-point neighbourhood of fine(J)) and returns their
 * number (Table of chain counts; Listing of the generated 2D code).
 */
int orc_rap_chains(int S, const int* off, int cmask, int n_index, int* out, int max_out) {
  int n[3] = {n_index / 9 - 1, (n_index / 3) % 3 - 1, n_index % 3 - 1};
  int cnt = 0;
  for (int ri = 0; ri < 27; ++ri) {
    int rho[3] = {ri / 9 - 1, (ri / 3) % 3 - 1, ri % 3 - 1};
    for (int s = 0; s < S; ++s) {
      double wr, wp;
      if (!rap_chain_ok(rho, &off[3 * s], n, cmask, &wr, &wp)) continue;
      int d[3];
      for (int a = 0; a < 3; ++a) {
        int cm = (cmask >> a) & 1;
        d[a] = cm ? rho[a] + off[3 * s + a] - 2 * n[a] : 0;
      }
      if (cnt < max_out) {
        out[3 * cnt] = ri;
        out[3 * cnt + 1] = s;
        out[3 * cnt + 2] = (d[0] + 1) * 9 + (d[1] + 1) * 3 + (d[2] + 1);
      }
      ++cnt;
    }
  }
  return cnt;
}

/* ---- ILU(0) factorisation (Sec. 4.2.3 mask flexibility; Sec. 4.4 ILU) ---
 * Doolittle (unit lower factor), IKJ order, restricted to a mask (offsets
 * off[0..S), which may differ from A's pattern offA[0..SA): entries of A
 * outside the mask are dropped, fill inside the mask is kept).
 * Row i: w = row i of A on the mask; for each lower slot s in canonical
 * order (= ascending column k = i+off_s): w[s] = w[s] / U_c[k]; then for
 * each upper slot t of row k in canonical order with j = k+off_t in the grid
 * and off_s+off_t in the mask: w[slot] = fma(-w[s], U_t[k], w[slot]).
 * The lower slots of w go to L, centre and upper slots to U; rU = 1/U_c.
 * Returns 0, or -1 on a zero pivot. */
int orc_ilu0_mask(int nx, int ny, int nz, int SA, const int* offA, const double* A, int S, const int* off,
                  double* L, double* U, double* rU) {
  long N = (long)nx * ny * nz;
  int slot[27], aslot[27], c = -1;
  for (int k = 0; k < 27; ++k) slot[k] = aslot[k] = -1;
  for (int s = 0; s < S; ++s) {
    slot[(off[3 * s] + 1) * 9 + (off[3 * s + 1] + 1) * 3 + (off[3 * s + 2] + 1)] = s;
    if (off[3 * s] == 0 && off[3 * s + 1] == 0 && off[3 * s + 2] == 0) c = s;
  }
  for (int s = 0; s < SA; ++s) aslot[(offA[3 * s] + 1) * 9 + (offA[3 * s + 1] + 1) * 3 + (offA[3 * s + 2] + 1)] = s;
  double w[27];
  for (long i = 0; i < N; ++i) {
    int X = (int)(i / ((long)ny * nz)), Y = (int)((i / nz) % ny), Z = (int)(i % nz);
    for (int s = 0; s < S; ++s) {
      /* row i of A on the mask: zero where A's pattern has no such offset */
      int a = X + off[3 * s], b = Y + off[3 * s + 1], cc = Z + off[3 * s + 2];
      int in = !(a < 0 || a >= nx || b < 0 || b >= ny || cc < 0 || cc >= nz);
      int sa = aslot[(off[3 * s] + 1) * 9 + (off[3 * s + 1] + 1) * 3 + (off[3 * s + 2] + 1)];
      w[s] = in && sa >= 0 ? A[sa * N + i] : 0.0;
    }
    for (int s = 0; s < c; ++s) {
      int a = X + off[3 * s], b = Y + off[3 * s + 1], cc = Z + off[3 * s + 2];
      if (a < 0 || a >= nx || b < 0 || b >= ny || cc < 0 || cc >= nz) continue;
      long k = ((long)a * ny + b) * nz + cc;
      w[s] = w[s] / U[c * N + k];
      for (int t = c + 1; t < S; ++t) {
        int ja = a + off[3 * t], jb = b + off[3 * t + 1], jc = cc + off[3 * t + 2];
        if (ja < 0 || ja >= nx || jb < 0 || jb >= ny || jc < 0 || jc >= nz) continue;
        int dx = off[3 * s] + off[3 * t], dy = off[3 * s + 1] + off[3 * t + 1], dz = off[3 * s + 2] + off[3 * t + 2];
        if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) continue;
        int sl = slot[(dx + 1) * 9 + (dy + 1) * 3 + (dz + 1)];
        if (sl < 0) continue;
        w[sl] = fma(-w[s], U[t * N + k], w[sl]);
      }
    }
    for (int s = 0; s < S; ++s) {
      L[s * N + i] = s < c ? w[s] : 0.0;
      U[s * N + i] = s >= c ? w[s] : 0.0;
    }
    if (w[c] == 0.0) return -1;
    rU[i] = 1.0 / w[c];
  }
  return 0;
}

/* ILU(0) on the matrix's own pattern. */
int orc_ilu0(int nx, int ny, int nz, int S, const int* off, const double* A, double* L, double* U,
             double* rU) {
  return orc_ilu0_mask(nx, ny, nz, S, off, A, S, off, L, U, rU);
}

/* ---- dense LU with partial pivoting (coarsest level) ------------------ */
int orc_lu_factor(int n, double* M, int* piv) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = fabs(M[(long)k * n + k]);
    for (int r = k + 1; r < n; ++r)
      if (fabs(M[(long)r * n + k]) > best) { best = fabs(M[(long)r * n + k]); p = r; }
    piv[k] = p;
    if (best == 0.0) return -1;
    if (p != k)
      for (int j = 0; j < n; ++j) {
        double t = M[(long)k * n + j];
        M[(long)k * n + j] = M[(long)p * n + j];
        M[(long)p * n + j] = t;
      }
    for (int r = k + 1; r < n; ++r) {
      double l = M[(long)r * n + k] / M[(long)k * n + k];
      M[(long)r * n + k] = l;
      for (int j = k + 1; j < n; ++j) M[(long)r * n + j] = fma(-l, M[(long)k * n + j], M[(long)r * n + j]);
    }
  }
  return 0;
}

void orc_lu_solve(int n, const double* M, const int* piv, double* b) {
  for (int k = 0; k < n; ++k) {
    double t = b[k];
    b[k] = b[piv[k]];
    b[piv[k]] = t;
  }
  for (int r = 0; r < n; ++r) {
    double t = b[r];
    for (int j = 0; j < r; ++j) t = fma(-M[(long)r * n + j], b[j], t);
    b[r] = t;
  }
  for (int r = n - 1; r >= 0; --r) {
    double t = b[r];
    for (int j = r + 1; j < n; ++j) t = fma(-M[(long)r * n + j], b[j], t);
    b[r] = t / M[(long)r * n + r];
  }
}

/* Dense matrix of an SG-DIA operator (row-major, n = N*bs). */
void orc_dense_from_sgdia(int nx, int ny, int nz, int S, const int* off, int bs, const double* A, double* M) {
  long N = (long)nx * ny * nz, n = N * bs;
  memset(M, 0, sizeof(double) * n * n);
  for (long i = 0; i < N; ++i) {
    int X = (int)(i / ((long)ny * nz)), Y = (int)((i / nz) % ny), Z = (int)(i % nz);
    for (int s = 0; s < S; ++s) {
      int a = X + off[3 * s], b = Y + off[3 * s + 1], c = Z + off[3 * s + 2];
      if (a < 0 || a >= nx || b < 0 || b >= ny || c < 0 || c >= nz) continue;
      long j = ((long)a * ny + b) * nz + c;
      for (int r = 0; r < bs; ++r)
        for (int cc = 0; cc < bs; ++cc)
          M[(i * bs + r) * n + j * bs + cc] = A[((long)s * bs * bs + r * bs + cc) * N + i];
    }
  }
}

/* Inverse of each 3x3 diagonal block by Gauss-Jordan with partial pivoting.
 * Returns -1 if a block is singular. */
int orc_block_dinv(int nx, int ny, int nz, int S, const int* off, const double* A, double* Dinv) {
  long N = (long)nx * ny * nz;
  int c = -1;
  for (int s = 0; s < S; ++s)
    if (off[3 * s] == 0 && off[3 * s + 1] == 0 && off[3 * s + 2] == 0) c = s;
  for (long i = 0; i < N; ++i) {
    double m[3][6];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) {
        m[r][k] = A[((long)c * 9 + r * 3 + k) * N + i];
        m[r][3 + k] = r == k ? 1.0 : 0.0;
      }
    for (int k = 0; k < 3; ++k) {
      int p = k;
      for (int r = k + 1; r < 3; ++r)
        if (fabs(m[r][k]) > fabs(m[p][k])) p = r;
      if (m[p][k] == 0.0) return -1;
      if (p != k)
        for (int j = 0; j < 6; ++j) { double t = m[k][j]; m[k][j] = m[p][j]; m[p][j] = t; }
      double piv = m[k][k];
      for (int j = 0; j < 6; ++j) m[k][j] = m[k][j] / piv;
      for (int r = 0; r < 3; ++r) {
        if (r == k) continue;
        double f = m[r][k];
        for (int j = 0; j < 6; ++j) m[r][j] = fma(-f, m[k][j], m[r][j]);
      }
    }
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) Dinv[(long)(r * 3 + k) * N + i] = m[r][3 + k];
  }
  return 0;
}

/* ---- stencil Galerkin product for the cell-centred pair (Cell_3d8
 * restriction and interpolation; Table of R/A/P combinations, 3d8c columns)
 * With piecewise-constant P and R = P^T, A_c(I, n) is the sum of A(f, s)
 * over the children f of coarse cell I (lexicographic order of the child
 * offset d) and the fine offsets s (canonical order) with f + s in the grid
 * and parent(f + s) = I + n; plain additions from zero.  A coupling of the
 * fine pattern can only reach coarse offsets of that pattern, so the coarse
 * operator keeps the fine pattern (off, S); Ac holds S*bs*bs coarse
 * diagonals. */
void orc_rap_cc(int nxf, int nyf, int nzf, int S, const int* off, int bs, const double* Af, int cmask, double* Ac) {
  int nf[3] = {nxf, nyf, nzf}, nc[3], cm[3];
  for (int a = 0; a < 3; ++a) {
    cm[a] = (cmask >> a) & 1;
    nc[a] = cm[a] ? (nf[a] + 1) / 2 : nf[a];
  }
  long Nf = (long)nf[0] * nf[1] * nf[2], Nc = (long)nc[0] * nc[1] * nc[2];
  int be = bs * bs;
  for (int X = 0; X < nc[0]; ++X)
    for (int Y = 0; Y < nc[1]; ++Y)
      for (int Z = 0; Z < nc[2]; ++Z) {
        int I[3] = {X, Y, Z};
        long ic = ((long)X * nc[1] + Y) * nc[2] + Z;
        for (int n = 0; n < S; ++n)
          for (int e = 0; e < be; ++e) {
            double acc = 0.0;
            for (int dx = 0; dx <= cm[0]; ++dx)
              for (int dy = 0; dy <= cm[1]; ++dy)
                for (int dz = 0; dz <= cm[2]; ++dz) {
                  int d[3] = {dx, dy, dz}, f[3], skip = 0;
                  for (int a = 0; a < 3; ++a) {
                    f[a] = cm[a] ? 2 * I[a] + d[a] : I[a];
                    if (f[a] >= nf[a]) skip = 1;
                  }
                  if (skip) continue;
                  long i = ((long)f[0] * nf[1] + f[1]) * nf[2] + f[2];
                  for (int s = 0; s < S; ++s) {
                    int g[3], hit = 1;
                    for (int a = 0; a < 3; ++a) {
                      g[a] = f[a] + off[3 * s + a];
                      if (g[a] < 0 || g[a] >= nf[a]) hit = 0;
                      else if ((cm[a] ? g[a] / 2 : g[a]) - I[a] != off[3 * n + a]) hit = 0;
                    }
                    if (hit) acc = acc + Af[((long)s * be + e) * Nf + i];
                  }
                }
            Ac[((long)n * be + e) * Nc + ic] = acc;
          }
      }
}

/* Influence chains of the cell-centred product for an interior coarse cell
 * and full coarsening: the (child, fine offset) pairs, each of which lands on
 * exactly one coarse offset (Table of chain counts, 3d8c columns). */
int orc_rap_cc_chains(int S, const int* off, int cmask) {
  int cnt = 0, I[3] = {4, 4, 4}, cm[3];
  for (int a = 0; a < 3; ++a) cm[a] = (cmask >> a) & 1;
  for (int n = 0; n < S; ++n)
    for (int dx = 0; dx <= cm[0]; ++dx)
      for (int dy = 0; dy <= cm[1]; ++dy)
        for (int dz = 0; dz <= cm[2]; ++dz) {
          int d[3] = {dx, dy, dz};
          for (int s = 0; s < S; ++s) {
            int hit = 1;
            for (int a = 0; a < 3; ++a) {
              int f = cm[a] ? 2 * I[a] + d[a] : I[a], g = f + off[3 * s + a];
              if ((cm[a] ? g / 2 : g) - I[a] != off[3 * n + a]) hit = 0;
            }
            cnt += hit;
          }
        }
  return cnt;
}

/* ---- stencil Galerkin product of Cell_3d8 restriction and Cell_3d64
 * interpolation (table of R/A/P combinations: R 3d8c, P 3d64c) ------------
 * A_c(I, n) for the 27 coarse offsets n (canonical order): over the children
 * f of I (lexicographic d), the fine offsets s (canonical) with g = f + s in
 * the grid, and the interpolation contributors J of g (lexicographic, as in
 * orc_prolong_add_c64) with J - I = n: acc = fma(A(f, s), w_J, acc) from
 * zero.  Coarse operators are 27-point. */
static int c64_parents(int g, int cm, int nc, int* par, double* wt) {
  if (!cm) { par[0] = g; wt[0] = 1.0; return 1; }
  int I = g / 2, J = (g & 1) ? I + 1 : I - 1, n = 0;
  int lo = J < I ? J : I, hi = J < I ? I : J;
  if (lo >= 0 && lo < nc) { par[n] = lo; wt[n] = lo == I ? 0.75 : 0.25; ++n; }
  if (hi >= 0 && hi < nc) { par[n] = hi; wt[n] = hi == I ? 0.75 : 0.25; ++n; }
  return n;
}

void orc_rap_c64(int nxf, int nyf, int nzf, int S, const int* off, int bs, const double* Af, int cmask, double* Ac) {
  int nf[3] = {nxf, nyf, nzf}, nc[3], cm[3];
  for (int a = 0; a < 3; ++a) {
    cm[a] = (cmask >> a) & 1;
    nc[a] = cm[a] ? (nf[a] + 1) / 2 : nf[a];
  }
  long Nf = (long)nf[0] * nf[1] * nf[2], Nc = (long)nc[0] * nc[1] * nc[2];
  int be = bs * bs, off27[81];
  orc_pattern(27, off27);
  for (int X = 0; X < nc[0]; ++X)
    for (int Y = 0; Y < nc[1]; ++Y)
      for (int Z = 0; Z < nc[2]; ++Z) {
        int I[3] = {X, Y, Z};
        long ic = ((long)X * nc[1] + Y) * nc[2] + Z;
        for (int n = 0; n < 27; ++n)
          for (int e = 0; e < be; ++e) {
            double acc = 0.0;
            for (int dx = 0; dx <= cm[0]; ++dx)
              for (int dy = 0; dy <= cm[1]; ++dy)
                for (int dz = 0; dz <= cm[2]; ++dz) {
                  int d[3] = {dx, dy, dz}, f[3], skip = 0;
                  for (int a = 0; a < 3; ++a) {
                    f[a] = cm[a] ? 2 * I[a] + d[a] : I[a];
                    if (f[a] >= nf[a]) skip = 1;
                  }
                  if (skip) continue;
                  long i = ((long)f[0] * nf[1] + f[1]) * nf[2] + f[2];
                  for (int s = 0; s < S; ++s) {
                    int g[3], par[3][2], np[3], out = 0;
                    double wt[3][2];
                    for (int a = 0; a < 3; ++a) {
                      g[a] = f[a] + off[3 * s + a];
                      if (g[a] < 0 || g[a] >= nf[a]) out = 1;
                    }
                    if (out) continue;
                    for (int a = 0; a < 3; ++a) np[a] = c64_parents(g[a], cm[a], nc[a], par[a], wt[a]);
                    double av = Af[((long)s * be + e) * Nf + i];
                    for (int p = 0; p < np[0]; ++p)
                      for (int q = 0; q < np[1]; ++q)
                        for (int r = 0; r < np[2]; ++r)
                          if (par[0][p] - X == off27[3 * n] && par[1][q] - Y == off27[3 * n + 1] &&
                              par[2][r] - Z == off27[3 * n + 2])
                            acc = fma(av, wt[0][p] * wt[1][q] * wt[2][r], acc);
                  }
                }
            Ac[((long)n * be + e) * Nc + ic] = acc;
          }
      }
}

/* Influence chains of the (3d8c, A, 3d64c) product for an interior coarse
 * cell: (child, fine offset, interpolation contributor) triples summed over
 * the 27 coarse offsets (Table of chain counts). */
int orc_rap_c64_chains(int S, const int* off, int cmask) {
  int cnt = 0, I[3] = {4, 4, 4}, cm[3], off27[81];
  orc_pattern(27, off27);
  for (int a = 0; a < 3; ++a) cm[a] = (cmask >> a) & 1;
  for (int n = 0; n < 27; ++n)
    for (int dx = 0; dx <= cm[0]; ++dx)
      for (int dy = 0; dy <= cm[1]; ++dy)
        for (int dz = 0; dz <= cm[2]; ++dz) {
          int d[3] = {dx, dy, dz};
          for (int s = 0; s < S; ++s) {
            int par[3][2], np[3];
            double wt[3][2];
            for (int a = 0; a < 3; ++a) {
              int f = cm[a] ? 2 * I[a] + d[a] : I[a];
              np[a] = c64_parents(f + off[3 * s + a], cm[a], 64, par[a], wt[a]);
            }
            for (int p = 0; p < np[0]; ++p)
              for (int q = 0; q < np[1]; ++q)
                for (int r = 0; r < np[2]; ++r)
                  cnt += par[0][p] - I[0] == off27[3 * n] && par[1][q] - I[1] == off27[3 * n + 1] &&
                         par[2][r] - I[2] == off27[3 * n + 2];
          }
        }
  return cnt;
}

/* ---- operator-dependent vertex interpolation (Listing 1 caption: P and R
 * vary from element to element; Dendy's black-box collapse) -------------
 * Grid map of the vertex hierarchy (coarse X <-> fine 2X+1 on coarsened
 * axes).  For fine point f let E(f) be the coarsened axes on which f is even
 * (between two coarse points); its corners on such an axis are lo = f/2 - 1
 * and hi = f/2, on the other axes the single parent.  W[c*N + f], c =
 * (cx*2 + cy)*2 + cz in {0..7} with c_a = 0 for lo or the single parent, 1
 * for hi: the weight of f's corner c.  Points with E(f) empty have W = 1 at
 * c = 0.  Otherwise, in order of |E(f)| = 1, 2, 3, with the stencil collapsed
 * onto the axes of E(f):
 *   Abar(f, d) = sum over the offsets s (canonical) with s_a = d_a on the
 *                axes a of E(f) of A(f, s)  (plain additions from zero),
 *   W(f, c) = -( sum over d != 0 in the box of E(f) (lexicographic), with
 *              g = f + d in the grid, of fma(Abar(f, d), W(g, c'), .) ) * r,
 *   r = 1 / Abar(f, 0),
 * where g contributes to c only if c_a = 1 when d_a = +1 and c_a = 0 when
 * d_a = -1 (g sits on that corner's line), and c'_a = (d_a == 0 ? c_a : 0).
 * Returns 0, or -1 on a zero collapsed diagonal. */
static int od_nbits(int f, int cm) { return cm && !(f & 1); }

int orc_od_weights(int nxf, int nyf, int nzf, int S, const int* off, const double* A, int cmask, double* W) {
  int nf[3] = {nxf, nyf, nzf}, cm[3];
  long N = (long)nxf * nyf * nzf;
  for (int a = 0; a < 3; ++a) cm[a] = (cmask >> a) & 1;
  for (int k = 0; k <= 3; ++k)
    for (int X = 0; X < nf[0]; ++X)
      for (int Y = 0; Y < nf[1]; ++Y)
        for (int Z = 0; Z < nf[2]; ++Z) {
          int f[3] = {X, Y, Z}, ev[3], ne = 0;
          for (int a = 0; a < 3; ++a) ne += ev[a] = od_nbits(f[a], cm[a]);
          if (ne != k) continue;
          long i = ((long)X * nf[1] + Y) * nf[2] + Z;
          if (k == 0) {
            for (int c = 0; c < 8; ++c) W[(long)c * N + i] = c == 0 ? 1.0 : 0.0;
            continue;
          }
          double Ab[27];
          for (int d = 0; d < 27; ++d) {
            int dd[3] = {d / 9 - 1, (d / 3) % 3 - 1, d % 3 - 1}, skip = 0;
            for (int a = 0; a < 3; ++a)
              if (!ev[a] && dd[a] != 0) skip = 1;
            Ab[d] = 0.0;
            if (skip) continue;
            for (int s2 = 0; s2 < S; ++s2) {
              int match = 1;
              for (int a = 0; a < 3; ++a)
                if (ev[a] && off[3 * s2 + a] != dd[a]) match = 0;
              if (match) Ab[d] = Ab[d] + A[(long)s2 * N + i];
            }
          }
          if (Ab[13] == 0.0) return -1;
          double r = 1.0 / Ab[13];
          for (int c = 0; c < 8; ++c) {
            int cc[3] = {c / 4, (c / 2) % 2, c % 2}, used = 1;
            for (int a = 0; a < 3; ++a)
              if (!ev[a] && cc[a]) used = 0;
            double acc = 0.0;
            if (used)
              for (int d = 0; d < 27; ++d) {
                int dd[3] = {d / 9 - 1, (d / 3) % 3 - 1, d % 3 - 1}, g[3], ok = 1, cp = 0;
                if (d == 13) continue;
                for (int a = 0; a < 3; ++a) {
                  if (!ev[a] && dd[a] != 0) ok = 0;
                  if (dd[a] == 1 && cc[a] != 1) ok = 0;
                  if (dd[a] == -1 && cc[a] != 0) ok = 0;
                  g[a] = f[a] + dd[a];
                  if (g[a] < 0 || g[a] >= nf[a]) ok = 0;
                }
                if (!ok) continue;
                for (int a = 0; a < 3; ++a) cp = cp * 2 + (dd[a] == 0 ? cc[a] : 0);
                long j = ((long)g[0] * nf[1] + g[1]) * nf[2] + g[2];
                acc = fma(Ab[d], W[(long)cp * N + j], acc);
              }
            W[(long)c * N + i] = used ? -acc * r : 0.0;
          }
        }
  return 0;
}

/* Corner c' of fine point g that is coarse point J (per axis: the single
 * parent, or lo / hi of an even coordinate), or -1 if J is not a corner. */
static int od_corner(const int* g, const int* cm, const int* J) {
  int c = 0;
  for (int a = 0; a < 3; ++a) {
    int b;
    if (!cm[a]) b = J[a] == g[a] ? 0 : -1;
    else if (g[a] & 1) b = J[a] == (g[a] - 1) / 2 ? 0 : -1;
    else b = J[a] == g[a] / 2 - 1 ? 0 : (J[a] == g[a] / 2 ? 1 : -1);
    if (b < 0) return -1;
    c = c * 2 + b;
  }
  return c;
}

/* Galerkin product with the operator-dependent P and R = P^T: for coarse I
 * and the 27 coarse offsets n (J = I + n in the coarse grid), over the fine
 * points u = fine(I) + rho (rho lexicographic over the box of the coarsened
 * axes, u in the grid) of which I is a corner:
 * t = sum over the canonical s with g = u + s in the grid and J a corner of g
 * of fma(A(u, s), W(g, corner J), t) from zero; then
 * acc = fma(W(u, corner I), t, acc) (the per-u partial sum times R(I, u), as
 * in the grouping of Listing 1).  Coarse operators are 27-point. */
/* The 27 entries of coarse row I (coarse grid nc, 27-point offsets off27),
 * written to Ac[n * ldc] for n = 0..26. */
static void od_rap_row(const int* nf, const int* nc, const int* cm, int S, const int* off, const int* off27,
                       const double* Af, const double* W, const int* I, double* Ac, long ldc) {
  long Nf = (long)nf[0] * nf[1] * nf[2];
  int fI[3];
  for (int a = 0; a < 3; ++a) fI[a] = cm[a] ? 2 * I[a] + 1 : I[a];
  for (int n = 0; n < 27; ++n) {
    int J[3], inJ = 1;
    for (int a = 0; a < 3; ++a) {
      J[a] = I[a] + off27[3 * n + a];
      if (J[a] < 0 || J[a] >= nc[a]) inJ = 0;
    }
    double acc = 0.0;
    if (inJ)
      for (int rho = 0; rho < 27; ++rho) {
        int rr[3] = {rho / 9 - 1, (rho / 3) % 3 - 1, rho % 3 - 1}, u[3], ok = 1;
        for (int a = 0; a < 3; ++a) {
          if (!cm[a] && rr[a] != 0) ok = 0;
          u[a] = fI[a] + rr[a];
          if (u[a] < 0 || u[a] >= nf[a]) ok = 0;
        }
        if (!ok) continue;
        int cu = od_corner(u, cm, I);
        if (cu < 0) continue;
        long iu = ((long)u[0] * nf[1] + u[1]) * nf[2] + u[2];
        double t = 0.0;
        for (int s2 = 0; s2 < S; ++s2) {
          int g[3], in = 1;
          for (int a = 0; a < 3; ++a) {
            g[a] = u[a] + off[3 * s2 + a];
            if (g[a] < 0 || g[a] >= nf[a]) in = 0;
          }
          if (!in) continue;
          int cg = od_corner(g, cm, J);
          if (cg < 0) continue;
          long ig = ((long)g[0] * nf[1] + g[1]) * nf[2] + g[2];
          t = fma(Af[(long)s2 * Nf + iu], W[(long)cg * Nf + ig], t);
        }
        acc = fma(W[(long)cu * Nf + iu], t, acc);
      }
    Ac[(long)n * ldc] = acc;
  }
}

void orc_rap_od(int nxf, int nyf, int nzf, int S, const int* off, const double* Af, int cmask, const double* W,
                double* Ac) {
  int nf[3] = {nxf, nyf, nzf}, nc[3], cm[3];
  for (int a = 0; a < 3; ++a) {
    cm[a] = (cmask >> a) & 1;
    nc[a] = cm[a] ? nf[a] / 2 : nf[a];
  }
  long Nc = (long)nc[0] * nc[1] * nc[2];
  int off27[81];
  orc_pattern(27, off27);
  for (int X = 0; X < nc[0]; ++X)
    for (int Y = 0; Y < nc[1]; ++Y)
      for (int Z = 0; Z < nc[2]; ++Z) {
        int I[3] = {X, Y, Z};
        long ic = ((long)X * nc[1] + Y) * nc[2] + Z;
        od_rap_row(nf, nc, cm, S, off, off27, Af, W, I, Ac + ic, Nc);
      }
}

/* The same rows at npts listed coarse points (flat coarse indices pts[k]):
 * Ac[n * npts + k].  For checks of a large grid's product at sampled points
 * without forming the whole coarse operator. */
void orc_rap_od_points(int nxf, int nyf, int nzf, int S, const int* off, const double* Af, int cmask,
                       const double* W, int npts, const long* pts, double* Ac) {
  int nf[3] = {nxf, nyf, nzf}, nc[3], cm[3];
  for (int a = 0; a < 3; ++a) {
    cm[a] = (cmask >> a) & 1;
    nc[a] = cm[a] ? nf[a] / 2 : nf[a];
  }
  int off27[81];
  orc_pattern(27, off27);
  for (int k = 0; k < npts; ++k) {
    long ic = pts[k];
    int I[3] = {(int)(ic / ((long)nc[1] * nc[2])), (int)((ic / nc[2]) % nc[1]), (int)(ic % nc[2])};
    od_rap_row(nf, nc, cm, S, off, off27, Af, W, I, Ac + k, npts);
  }
}

/* ---- Thomas factorisation of the z-columns (Sec. 4.4, LGS paragraph) ---
 * For every column (x, y) the tridiagonal block of A on that column: a_z =
 * coupling to z-1, b_z = centre, c_z = coupling to z+1 (zero at the column
 * ends).  Pivots of the Thomas algorithm:
 *   p_0 = b_0,  p_z = fma(-a_z, cp_{z-1}, b_z);  rden_z = 1/p_z;
 *   cp_z = c_z * rden_z.
 * Returns 0, or -1 on a zero pivot. */
int orc_tri_factor(int nx, int ny, int nz, int S, const int* off, const double* A, double* rden, double* cp) {
  long N = (long)nx * ny * nz;
  int slo = -1, sc = -1, sup = -1;
  for (int s = 0; s < S; ++s)
    if (off[3 * s] == 0 && off[3 * s + 1] == 0) {
      if (off[3 * s + 2] == -1) slo = s;
      if (off[3 * s + 2] == 0) sc = s;
      if (off[3 * s + 2] == 1) sup = s;
    }
  for (long col = 0; col < (long)nx * ny; ++col) {
    long i0 = col * nz;
    for (int Z = 0; Z < nz; ++Z) {
      long i = i0 + Z;
      double az = Z > 0 ? A[slo * N + i] : 0.0;
      double cz = Z < nz - 1 ? A[sup * N + i] : 0.0;
      double p = Z == 0 ? A[sc * N + i] : fma(-az, cp[i - 1], A[sc * N + i]);
      if (p == 0.0) return -1;
      rden[i] = 1.0 / p;
      cp[i] = cz * rden[i];
    }
  }
  return 0;
}

/* ---- multigrid hierarchy ---------------------------------------------- */
typedef struct {
  int nx, ny, nz, S, cmask;
  long N;
  int off[81];
  int Sm, offm[81]; /* ILU(0) mask (the level's own pattern unless chosen) */
  double *A, *rd, *L, *U, *rU;           /* FP64 level data */
  double *tr, *tc;                       /* Thomas factors rden, cp (line GS) */
  double* W;                             /* operator-dependent interpolation weights (8 x N) */
  double* qa;                            /* weighted GS: ((1 - w) / w) a_ii (NULL for w = 1) */
  float* qa32;
  float* W32;
  float *A32, *rd32, *L32, *U32, *rU32;  /* truncated level data */
  float *tr32, *tc32;
  double *f, *u, *r, *w, *d;             /* FP64 work vectors (d: one column) */
  float *f32, *u32, *r32, *w32, *d32;    /* reduced-precision work vectors */
} olev;

typedef struct {
  int nlev, bs, smoother, prec, cell;
  int npre, npost, zero_guess; /* smoothing steps per level; ZeroGuess on the first */
  double w;                    /* GS weight */
  olev lev[48];
  int nc;
  double *LU, *cw;
  int* piv;
  double *kr, *kz, *kp, *kq, *kt; /* Krylov work */
  float *k32a, *k32b;
} omg;

/* Axes coarsened to go from level `lev` with dims n[] to the next level:
 * every allowed axis whose size is at least nmin = 2 * min_coarse (8 by
 * default: coarse size >= 4).  Allowed axes are x and y on the first
 * `semi_levels` levels (or always, for the semi mode), all three otherwise.
 * A level of the first `semi_levels` whose x and y can no longer be coarsened
 * takes all three axes instead (the switch to full coarsening comes early
 * rather than the hierarchy ending). */
static int orc_next_cmask(int lev, const int* n, int semi_mode, int semi_levels, int nmin) {
  int allowed = (semi_mode || lev < semi_levels) ? 3 : 7, m = 0;
  for (int a = 0; a < 3; ++a)
    if (((allowed >> a) & 1) && n[a] >= nmin) m |= 1 << a;
  if (m == 0 && !semi_mode && allowed == 3)
    for (int a = 0; a < 3; ++a)
      if (n[a] >= nmin) m |= 1 << a;
  return m;
}

/* Automatic choice of the x,y-only levels (fixed-stride coarsening per
 * level, Sec. 4.1 P2): rho = (sum over points of |a| of the two z-face
 * couplings) / (mean of the same sums along x and along y), in-grid
 * neighbours only.  Coarsening x and y by 2 makes the z coupling of the next
 * level relatively 4 times stronger, so level l coarsens x,y only while
 * rho * 4^l < 1/4. */
int orc_auto_semi_levels(int nx, int ny, int nz, int S, const int* off, const double* A) {
  long N = (long)nx * ny * nz;
  double sum[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < S; ++s) {
    int d[3] = {off[3 * s], off[3 * s + 1], off[3 * s + 2]};
    int axis = -1;
    for (int a = 0; a < 3; ++a)
      if (abs(d[a]) == 1 && d[(a + 1) % 3] == 0 && d[(a + 2) % 3] == 0) axis = a;
    if (axis < 0) continue;
    for (long i = 0; i < N; ++i) {
      int X = (int)(i / ((long)ny * nz)), Y = (int)((i / nz) % ny), Z = (int)(i % nz);
      int a = X + d[0], b = Y + d[1], c = Z + d[2];
      if (a < 0 || a >= nx || b < 0 || b >= ny || c < 0 || c >= nz) continue;
      sum[axis] += fabs(A[(long)s * N + i]);
    }
  }
  double sxy = 0.5 * (sum[0] + sum[1]);
  int lev = 0;
  if (sxy > 0.0)
    for (double r = sum[2] / sxy; lev < 40 && r < 0.25; r *= 4.0) ++lev;
  return lev;
}

static float* to_f32(const double* a, long n) {
  float* o = (float*)malloc(sizeof(float) * (n > 0 ? n : 1));
  for (long k = 0; k < n; ++k) o[k] = (float)a[k];
  return o;
}

/* FP16 with per-scalar-row FP32 scale: s = float(max |a| over the row),
 * h = half(float(a / s)), stored value used by the kernels = s * float(h). */
static float* to_f16_rowscaled(const double* A, long N, int S, int bs) {
  int be = bs * bs;
  float* o = (float*)malloc(sizeof(float) * (long)S * be * N);
  for (long i = 0; i < N; ++i)
    for (int r = 0; r < bs; ++r) {
      double mx = 0.0;
      for (int s = 0; s < S; ++s)
        for (int c = 0; c < bs; ++c) {
          double v = fabs(A[((long)s * be + r * bs + c) * N + i]);
          if (v > mx) mx = v;
        }
      float sc = (float)mx;
      for (int s = 0; s < S; ++s)
        for (int c = 0; c < bs; ++c) {
          long k = ((long)s * be + r * bs + c) * N + i;
          float hv = orc_f16_to_f32(orc_f32_to_f16((float)(A[k] / (double)sc)));
          o[k] = sc == 0.0f ? 0.0f : sc * hv;
        }
    }
  return o;
}

void orc_mg_destroy(omg* mg);

/*
 * Builds the hierarchy from the finest matrix only (Sec. 4.2.2 input).
 * pattern: 7/19/27 (level 0); coarse levels are 27-point.  bs: 1 or 3.
 * smoother: 0 = symmetric GS, 1 = ILU(0), 2 = symmetric line GS over
 * z-columns (scalar systems; FP64 and FP32).  prec: 0 FP64, 1 FP32,
 * 2 FP16 row-scaled.  ilu_mask: 0 = ILU(0) on each level's own pattern, or
 * 7 / 19 / 27 = that mask for the finest matrix (coarse levels keep their
 * own 27-point pattern).  cell = 0: vertex-centred trilinear P, R = P^T,
 * coarse levels 27-point; cell = 1: cell-centred piecewise-constant P and
 * R = P^T (Cell_3d8), every level keeps the finest pattern; cell = 2:
 * Cell_3d8 restriction with cell-centred trilinear interpolation (3d64c),
 * coarse levels 27-point; cell = 3: operator-dependent vertex interpolation
 * (orc_od_weights) with R = P^T, coarse levels 27-point.  A0 is copied;
 * out-of-grid couplings are zeroed.  semi_mode: 0 = full coarsening after
 * semi_levels x,y-only levels, 1 = x,y only, 2 = the automatic choice of
 * orc_auto_semi_levels.  npre / npost: smoothing steps before / after the
 * coarse correction (GS directions alternate, post-steps starting opposite
 * to the last pre-step); w: GS weight (point GS, scalar systems);
 * zero_guess: the first pre-step uses ZeroGuess (else it runs on u = 0 in
 * full); an axis of n points is coarsened while n >= 2 * min_coarse.
 * Returns NULL on error (zero pivot, coarsest level too large).
 */
omg* orc_mg_create_ex(int nx, int ny, int nz, int pattern, int bs, const double* A0, int smoother, int semi_mode,
                      int semi_levels, int prec, int max_coarse, int ilu_mask, int cell, int npre, int npost,
                      double w, int zero_guess, int min_coarse) {
  if (smoother == 2 && (bs != 1 || prec == 2)) return NULL;
  if (ilu_mask != 0 && (smoother != 1 || (ilu_mask != 7 && ilu_mask != 19 && ilu_mask != 27))) return NULL;
  if (cell == 3 && bs != 1) return NULL;
  if (npre < 1 || npost < 1 || !(w > 0.0 && w < 2.0) || min_coarse < 2) return NULL;
  if (w != 1.0 && (smoother != 0 || bs != 1)) return NULL;
  if (semi_mode == 2 && bs != 1) return NULL;
  omg* mg = (omg*)calloc(1, sizeof(omg));
  mg->bs = bs;
  mg->cell = cell;
  mg->smoother = smoother;
  mg->prec = prec;
  mg->npre = npre;
  mg->npost = npost;
  mg->w = w;
  mg->zero_guess = zero_guess;
  int be = bs * bs, l = 0;
  int n[3] = {nx, ny, nz};
  for (;;) {
    olev* v = &mg->lev[l];
    v->nx = n[0]; v->ny = n[1]; v->nz = n[2];
    v->N = (long)n[0] * n[1] * n[2];
    v->S = orc_pattern(l == 0 || cell == 1 ? pattern : 27, v->off);
    v->A = (double*)malloc(sizeof(double) * v->S * be * v->N);
    if (l == 0) {
      for (int s = 0; s < v->S; ++s)
        for (long i = 0; i < v->N; ++i) {
          int X = (int)(i / ((long)n[1] * n[2])), Y = (int)((i / n[2]) % n[1]), Z = (int)(i % n[2]);
          int a = X + v->off[3 * s], b = Y + v->off[3 * s + 1], c = Z + v->off[3 * s + 2];
          int in = !(a < 0 || a >= n[0] || b < 0 || b >= n[1] || c < 0 || c >= n[2]);
          for (int e = 0; e < be; ++e)
            v->A[((long)s * be + e) * v->N + i] = in ? A0[((long)s * be + e) * v->N + i] : 0.0;
        }
    } else {
      olev* p = &mg->lev[l - 1];
      if (cell == 3)
        orc_rap_od(p->nx, p->ny, p->nz, p->S, p->off, p->A, p->cmask, p->W, v->A);
      else if (cell == 1)
        orc_rap_cc(p->nx, p->ny, p->nz, p->S, p->off, bs, p->A, p->cmask, v->A);
      else if (cell == 2)
        orc_rap_c64(p->nx, p->ny, p->nz, p->S, p->off, bs, p->A, p->cmask, v->A);
      else
        orc_rap(p->nx, p->ny, p->nz, p->S, p->off, bs, p->A, p->cmask, v->A);
    }
    long nvec = v->N * bs;
    v->f = (double*)calloc(nvec, sizeof(double));
    v->u = (double*)calloc(nvec, sizeof(double));
    v->r = (double*)calloc(nvec, sizeof(double));
    v->w = (double*)calloc(nvec, sizeof(double));
    v->f32 = (float*)calloc(nvec, sizeof(float));
    v->u32 = (float*)calloc(nvec, sizeof(float));
    v->r32 = (float*)calloc(nvec, sizeof(float));
    v->w32 = (float*)calloc(nvec, sizeof(float));
    v->d = (double*)calloc(n[2], sizeof(double));
    v->d32 = (float*)calloc(n[2], sizeof(float));
    mg->nlev = l + 1;
    if (l == 0 && semi_mode == 2) {
      semi_levels = orc_auto_semi_levels(nx, ny, nz, v->S, v->off, v->A);
      semi_mode = 0;
    }
    v->cmask = orc_next_cmask(l, n, semi_mode, semi_levels, 2 * min_coarse);
    if (v->cmask == 0 || l == 47) {
      v->cmask = 0;
      break;
    }
    if (cell == 3) {
      v->W = (double*)malloc(sizeof(double) * 8 * v->N);
      if (orc_od_weights(v->nx, v->ny, v->nz, v->S, v->off, v->A, v->cmask, v->W)) {
        orc_mg_destroy(mg);
        return NULL;
      }
    }
    for (int a = 0; a < 3; ++a)
      if ((v->cmask >> a) & 1) n[a] = cell == 1 || cell == 2 ? (n[a] + 1) / 2 : n[a] / 2;
    ++l;
  }
  /* smoother data on all but the coarsest level */
  for (l = 0; l < mg->nlev - 1; ++l) {
    olev* v = &mg->lev[l];
    int c = (v->S - 1) / 2;
    if (bs == 3) {
      v->rd = (double*)malloc(sizeof(double) * 9 * v->N);
      if (orc_block_dinv(v->nx, v->ny, v->nz, v->S, v->off, v->A, v->rd)) { orc_mg_destroy(mg); return NULL; }
    } else {
      v->rd = (double*)malloc(sizeof(double) * v->N);
      for (long i = 0; i < v->N; ++i) v->rd[i] = w / v->A[c * v->N + i];
      if (w != 1.0) {
        double q = (1.0 - w) / w;
        v->qa = (double*)malloc(sizeof(double) * v->N);
        for (long i = 0; i < v->N; ++i) v->qa[i] = q * v->A[c * v->N + i];
      }
      if (smoother == 1) {
        v->Sm = ilu_mask && l == 0 ? orc_pattern(ilu_mask, v->offm) : orc_pattern(v->S, v->offm);
        v->L = (double*)malloc(sizeof(double) * v->Sm * v->N);
        v->U = (double*)malloc(sizeof(double) * v->Sm * v->N);
        v->rU = (double*)malloc(sizeof(double) * v->N);
        if (orc_ilu0_mask(v->nx, v->ny, v->nz, v->S, v->off, v->A, v->Sm, v->offm, v->L, v->U, v->rU)) {
          orc_mg_destroy(mg);
          return NULL;
        }
      }
      if (smoother == 2) {
        v->tr = (double*)malloc(sizeof(double) * v->N);
        v->tc = (double*)malloc(sizeof(double) * v->N);
        if (orc_tri_factor(v->nx, v->ny, v->nz, v->S, v->off, v->A, v->tr, v->tc)) { orc_mg_destroy(mg); return NULL; }
      }
    }
    if (prec != 0) {
      long na = (long)v->S * be * v->N;
      v->A32 = prec == 2 ? to_f16_rowscaled(v->A, v->N, v->S, bs) : to_f32(v->A, na);
      v->rd32 = to_f32(v->rd, (bs == 3 ? 9 : 1) * v->N);
      if (smoother == 1 && bs == 1) {
        v->L32 = to_f32(v->L, (long)v->Sm * v->N);
        v->U32 = to_f32(v->U, (long)v->Sm * v->N);
        v->rU32 = to_f32(v->rU, v->N);
      }
      if (smoother == 2) {
        v->tr32 = to_f32(v->tr, v->N);
        v->tc32 = to_f32(v->tc, v->N);
      }
      if (cell == 3) v->W32 = to_f32(v->W, 8 * v->N);
      if (v->qa) v->qa32 = to_f32(v->qa, v->N);
    }
  }
  /* coarsest: dense FP64 LU */
  olev* cl = &mg->lev[mg->nlev - 1];
  long nc = cl->N * bs;
  if (nc > max_coarse) { orc_mg_destroy(mg); return NULL; }
  mg->nc = (int)nc;
  mg->LU = (double*)malloc(sizeof(double) * nc * nc);
  mg->piv = (int*)malloc(sizeof(int) * nc);
  mg->cw = (double*)malloc(sizeof(double) * nc);
  orc_dense_from_sgdia(cl->nx, cl->ny, cl->nz, cl->S, cl->off, bs, cl->A, mg->LU);
  if (orc_lu_factor((int)nc, mg->LU, mg->piv)) { orc_mg_destroy(mg); return NULL; }
  long n0 = mg->lev[0].N * bs;
  mg->kr = (double*)calloc(n0, sizeof(double));
  mg->kz = (double*)calloc(n0, sizeof(double));
  mg->kp = (double*)calloc(n0, sizeof(double));
  mg->kq = (double*)calloc(n0, sizeof(double));
  mg->kt = (double*)calloc(n0, sizeof(double));
  mg->k32a = (float*)calloc(n0, sizeof(float));
  mg->k32b = (float*)calloc(n0, sizeof(float));
  return mg;
}

omg* orc_mg_create(int nx, int ny, int nz, int pattern, int bs, const double* A0, int smoother, int semi_mode,
                   int semi_levels, int prec, int max_coarse, int ilu_mask, int cell) {
  return orc_mg_create_ex(nx, ny, nz, pattern, bs, A0, smoother, semi_mode, semi_levels, prec, max_coarse, ilu_mask,
                          cell, 1, 1, 1.0, 1, 4);
}

void orc_mg_destroy(omg* mg) {
  if (!mg) return;
  for (int l = 0; l < mg->nlev; ++l) {
    olev* v = &mg->lev[l];
    free(v->qa); free(v->qa32);
    free(v->A); free(v->rd); free(v->L); free(v->U); free(v->rU);
    free(v->A32); free(v->rd32); free(v->L32); free(v->U32); free(v->rU32);
    free(v->tr); free(v->tc); free(v->tr32); free(v->tc32); free(v->W); free(v->W32);
    free(v->f); free(v->u); free(v->r); free(v->w); free(v->d);
    free(v->f32); free(v->u32); free(v->r32); free(v->w32); free(v->d32);
  }
  free(mg->LU); free(mg->piv); free(mg->cw);
  free(mg->kr); free(mg->kz); free(mg->kp); free(mg->kq); free(mg->kt);
  free(mg->k32a); free(mg->k32b);
  free(mg);
}

int orc_mg_nlev(const omg* mg) { return mg->nlev; }

/* dims[0..2], S, cmask, ILU mask points of level l */
void orc_mg_level_info(const omg* mg, int l, int* info) {
  const olev* v = &mg->lev[l];
  info[0] = v->nx; info[1] = v->ny; info[2] = v->nz; info[3] = v->S; info[4] = v->cmask; info[5] = v->Sm;
}

/* Copies out level data: what = 0 A, 1 rd (or block Dinv), 2 L, 3 U, 4 rU,
 * 5 truncated A (as float), 6 truncated rd, 7 Thomas rden, 8 Thomas cp,
 * 9 operator-dependent interpolation weights (8 x N). */
void orc_mg_level_data(const omg* mg, int l, int what, void* out) {
  const olev* v = &mg->lev[l];
  long be = (long)mg->bs * mg->bs;
  switch (what) {
    case 0: memcpy(out, v->A, sizeof(double) * v->S * be * v->N); break;
    case 1: memcpy(out, v->rd, sizeof(double) * (mg->bs == 3 ? 9 : 1) * v->N); break;
    case 2: memcpy(out, v->L, sizeof(double) * v->Sm * v->N); break;
    case 3: memcpy(out, v->U, sizeof(double) * v->Sm * v->N); break;
    case 4: memcpy(out, v->rU, sizeof(double) * v->N); break;
    case 5: memcpy(out, v->A32, sizeof(float) * v->S * be * v->N); break;
    case 6: memcpy(out, v->rd32, sizeof(float) * (mg->bs == 3 ? 9 : 1) * v->N); break;
    case 7: memcpy(out, v->tr, sizeof(double) * v->N); break;
    case 8: memcpy(out, v->tc, sizeof(double) * v->N); break;
    case 9: memcpy(out, v->W, sizeof(double) * 8 * v->N); break;
  }
}

#define FF f
#define FU_ u
#define FR r
#define FW w
#define FA A
#define FRD rd
#define FL L
#define FU U
#define FRU rU
#define FTR tr
#define FTC tc
#define FD d
#define FPW W
#define FQA qa
#define REAL double
#define SFX _f64
#include "oracle_vcycle.inc"
#undef REAL
#undef SFX
#undef FF
#undef FU_
#undef FR
#undef FW
#undef FA
#undef FRD
#undef FL
#undef FU
#undef FRU
#undef FTR
#undef FTC
#undef FD
#undef FPW
#undef FQA

#define FF f32
#define FU_ u32
#define FR r32
#define FW w32
#define FA A32
#define FRD rd32
#define FL L32
#define FU U32
#define FRU rU32
#define FTR tr32
#define FTC tc32
#define FD d32
#define FPW W32
#define FQA qa32
#define REAL float
#define SFX _f32
#include "oracle_vcycle.inc"
#undef REAL
#undef SFX

/* z = M r: one V-cycle in the hierarchy's precision (FP64 in, FP64 out). */
void orc_mg_apply(omg* mg, const double* r, double* z) {
  long n = mg->lev[0].N * mg->bs;
  if (mg->prec == 0) {
    vcycle_f64(mg, 0, r, z);
  } else {
    for (long k = 0; k < n; ++k) mg->k32a[k] = (float)r[k];
    vcycle_f32(mg, 0, mg->k32a, mg->k32b);
    for (long k = 0; k < n; ++k) z[k] = (double)mg->k32b[k];
  }
}

/* Single-precision V-cycle on float input/output (for kernel-level parity). */
void orc_mg_apply_f32(omg* mg, const float* r, float* z) { vcycle_f32(mg, 0, r, z); }

static void op0(omg* mg, const double* x, double* y) {
  olev* v = &mg->lev[0];
  if (mg->bs == 3)
    orc_bspmv_f64(v->nx, v->ny, v->nz, v->S, v->off, v->A, x, y);
  else
    orc_spmv_f64(v->nx, v->ny, v->nz, v->S, v->off, v->A, x, y);
}

static double dot(const double* a, const double* b, long n) {
  double s = 0.0;
  for (long k = 0; k < n; ++k) s = fma(a[k], b[k], s);
  return s;
}

/*
 * Preconditioned CG (Sec. 5.2; stopping rule ||r||_2/||b||_2 < tol from the
 * settings table).  x holds x0 on entry.  When the recursive residual meets
 * the tolerance the true residual b - A x is formed; the iteration stops only
 * if the true residual also meets it, otherwise continues from it.
 * Returns 0 converged, 1 not converged, -4 breakdown (p.Ap <= 0).
 * out[0] = iterations, out[1] = final true relative residual.
 */
int orc_pcg(omg* mg, const double* b, double* x, double tol, int maxit, double* out) {
  long n = mg->lev[0].N * mg->bs;
  double *r = mg->kr, *z = mg->kz, *p = mg->kp, *q = mg->kq;
  double bn = sqrt(dot(b, b, n));
  if (bn == 0.0) bn = 1.0;
  op0(mg, x, q);
  for (long k = 0; k < n; ++k) r[k] = b[k] - q[k];
  int it = 0, status = 1;
  double rel = sqrt(dot(r, r, n)) / bn;
  if (rel < tol) { out[0] = 0; out[1] = rel; return 0; }
  orc_mg_apply(mg, r, z);
  memcpy(p, z, sizeof(double) * n);
  double rho = dot(r, z, n);
  while (it < maxit) {
    op0(mg, p, q);
    double pq = dot(p, q, n);
    if (!(pq > 0.0)) { status = -4; break; }
    double alpha = rho / pq;
    for (long k = 0; k < n; ++k) { x[k] = fma(alpha, p[k], x[k]); r[k] = fma(-alpha, q[k], r[k]); }
    ++it;
    rel = sqrt(dot(r, r, n)) / bn;
    if (rel < tol) {
      op0(mg, x, q);
      for (long k = 0; k < n; ++k) r[k] = b[k] - q[k];
      rel = sqrt(dot(r, r, n)) / bn;
      if (rel < tol) { status = 0; break; }
    }
    orc_mg_apply(mg, r, z);
    double rho1 = dot(r, z, n);
    double beta = rho1 / rho;
    rho = rho1;
    for (long k = 0; k < n; ++k) p[k] = fma(beta, p[k], z[k]);
  }
  op0(mg, x, q);
  for (long k = 0; k < n; ++k) r[k] = b[k] - q[k];
  out[0] = it;
  out[1] = sqrt(dot(r, r, n)) / bn;
  return status;
}

/*
 * Right-preconditioned restarted GMRES(m) with modified Gram-Schmidt and
 * Givens rotations (Sec. 5.2).  Converges when the Givens residual estimate
 * over ||b|| is below tol and the true residual confirms it; restarts from
 * the true residual.  out as for orc_pcg.
 */
int orc_gmres(omg* mg, const double* b, double* x, double tol, int maxit, int m, double* out) {
  long n = mg->lev[0].N * mg->bs;
  double* V = (double*)malloc(sizeof(double) * n * (m + 1));
  double* H = (double*)calloc((size_t)(m + 1) * m, sizeof(double));
  double *cs = (double*)calloc(m, sizeof(double)), *sn = (double*)calloc(m, sizeof(double));
  double *g = (double*)calloc(m + 1, sizeof(double)), *y = (double*)calloc(m, sizeof(double));
  double *r = mg->kr, *z = mg->kz, *w = mg->kq, *t = mg->kt;
  double bn = sqrt(dot(b, b, n));
  if (bn == 0.0) bn = 1.0;
  int it = 0, status = 1;
  op0(mg, x, w);
  for (long k = 0; k < n; ++k) r[k] = b[k] - w[k];
  double beta = sqrt(dot(r, r, n));
  if (beta / bn < tol) status = 0;
  while (status == 1 && it < maxit) {
    for (long k = 0; k < n; ++k) V[k] = r[k] / beta;
    for (int k = 0; k <= m; ++k) g[k] = 0.0;
    g[0] = beta;
    int j, jdone = 0;
    for (j = 0; j < m && it < maxit; ++j) {
      double* vj = V + (long)j * n;
      double* vn = V + (long)(j + 1) * n;
      orc_mg_apply(mg, vj, z);
      op0(mg, z, w);
      for (int i = 0; i <= j; ++i) {
        double* vi = V + (long)i * n;
        double h = dot(w, vi, n);
        H[i * m + j] = h;
        for (long k = 0; k < n; ++k) w[k] = fma(-h, vi[k], w[k]);
      }
      double hn = sqrt(dot(w, w, n));
      H[(j + 1) * m + j] = hn;
      if (hn != 0.0)
        for (long k = 0; k < n; ++k) vn[k] = w[k] / hn;
      for (int i = 0; i < j; ++i) {
        double a = H[i * m + j], bb = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * bb;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
      }
      double a = H[j * m + j], bb = H[(j + 1) * m + j];
      double den = sqrt(a * a + bb * bb);
      cs[j] = den == 0.0 ? 1.0 : a / den;
      sn[j] = den == 0.0 ? 0.0 : bb / den;
      H[j * m + j] = den;
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      jdone = j + 1;
      if (fabs(g[j + 1]) / bn < tol || hn == 0.0) break;
    }
    for (int i = jdone - 1; i >= 0; --i) {
      double s = g[i];
      for (int k = i + 1; k < jdone; ++k) s -= H[i * m + k] * y[k];
      y[i] = s / H[i * m + i];
    }
    for (long k = 0; k < n; ++k) t[k] = 0.0;
    for (int i = 0; i < jdone; ++i)
      for (long k = 0; k < n; ++k) t[k] = fma(y[i], V[(long)i * n + k], t[k]);
    orc_mg_apply(mg, t, z);
    for (long k = 0; k < n; ++k) x[k] += z[k];
    op0(mg, x, w);
    for (long k = 0; k < n; ++k) r[k] = b[k] - w[k];
    beta = sqrt(dot(r, r, n));
    if (beta / bn < tol) status = 0;
  }
  out[0] = it;
  out[1] = beta / bn;
  free(V); free(H); free(cs); free(sn); free(g); free(y);
  return status;
}
