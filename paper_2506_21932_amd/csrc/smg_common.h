// Shared device definitions of the structured multigrid library (gfx950).
//
// Grid (nx, ny, nz), linear index i = (x*ny + y)*nz + z (z contiguous).
// Stencil offsets are enumerated in lexicographic order (dx slowest), which
// is the numbering of the paper's Offset(2d9) / Offset(2d5) lists extended to
// 3D (Sec. 4.3).  A level matrix is stored diagonal-major ("SG-DIA",
// Sec. 4.1 P1): coefficient of row i for offset s at A[s*N + i]; couplings to
// neighbours outside the grid are stored as zero.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smg {

__host__ __device__ constexpr int iabs(int v) { return v < 0 ? -v : v; }

__host__ __device__ constexpr bool pat_has(int pat, int dx, int dy, int dz) {
  return pat == 27 || (pat == 19 && iabs(dx) + iabs(dy) + iabs(dz) <= 2) ||
         (pat == 7 && iabs(dx) + iabs(dy) + iabs(dz) <= 1);
}

// Component `axis` of offset number s of a pattern in canonical order.
__host__ __device__ constexpr int pat_off(int pat, int s, int axis) {
  int k = 0;
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dz = -1; dz <= 1; ++dz)
        if (pat_has(pat, dx, dy, dz)) {
          if (k == s) return axis == 0 ? dx : (axis == 1 ? dy : dz);
          ++k;
        }
  return 0;
}

// Slot of offset (dx,dy,dz) in a pattern, or -1.
__host__ __device__ constexpr int pat_slot(int pat, int dx, int dy, int dz) {
  int k = 0;
  for (int a = -1; a <= 1; ++a)
    for (int b = -1; b <= 1; ++b)
      for (int c = -1; c <= 1; ++c)
        if (pat_has(pat, a, b, c)) {
          if (a == dx && b == dy && c == dz) return k;
          ++k;
        }
  return -1;
}

// Hyperplane weights of the lexicographic dependence graph: a unit (x,y,z)
// depends only on units with smaller wx*x + wy*y + z.  3d7: (1,1,1);
// 3d19: (3,2,1); 3d27: (4,2,1).
__host__ __device__ constexpr int hp_wx(int pat) { return pat == 7 ? 1 : (pat == 19 ? 3 : 4); }
__host__ __device__ constexpr int hp_wy(int pat) { return pat == 7 ? 1 : 2; }

// Sentinels marking "not yet written in this sweep" in wavefront outputs:
// signalling NaNs with a fixed payload.  Arithmetic never produces a
// signalling NaN, so a computed value can never equal them.
constexpr uint64_t SENT64 = 0xFFF5A5A55A5AA5A5ull;
constexpr uint32_t SENT32 = 0xFFA5A55Au;

template <class V> struct VBits;
template <> struct VBits<double> {
  using U = unsigned long long;
  static constexpr U sent = SENT64;
  __device__ static U bits(double v) { return (U)__double_as_longlong(v); }
  __device__ static double val(U b) { return __longlong_as_double((long long)b); }
};
template <> struct VBits<float> {
  using U = unsigned int;
  static constexpr U sent = SENT32;
  __device__ static U bits(float v) { return (U)__float_as_uint(v); }
  __device__ static float val(U b) { return __uint_as_float(b); }
};

// Coefficient accessors of a level matrix in the three storage precisions.
// FP16 storage keeps one FP32 scale per (scalar) row; the kernel value of a
// coefficient is scale * float(h), formed in FP32.
struct MatD {
  const double* a;
  long n;
  using V = double;
  __device__ double operator()(int s, long i) const { return a[(long)s * n + i]; }
};
struct MatF {
  const float* a;
  long n;
  using V = float;
  __device__ float operator()(int s, long i) const { return a[(long)s * n + i]; }
};
struct MatH {
  const __half* a;
  const float* sc;
  long n;
  using V = float;
  __device__ float operator()(int s, long i) const { return sc[i] * __half2float(a[(long)s * n + i]); }
};

// 3x3 block matrices: entry e = s*9 + r*3 + c of node i at a[e*N + i]; FP16
// storage scales scalar row r of node i by sc[r*N + i].
struct BMatD {
  const double* a;
  long n;
  using V = double;
  __device__ double operator()(int e, int r, long i) const { return a[(long)e * n + i]; }
};
struct BMatF {
  const float* a;
  long n;
  using V = float;
  __device__ float operator()(int e, int r, long i) const { return a[(long)e * n + i]; }
};
// float(half m of the packed pair w) * sc rounded once, as the product of the
// converted half and sc: a mixed-precision fma (the half operand converted
// exactly) with addend -0, which keeps the product's sign of zero.  M = 0:
// low half, 1: high half.
template <int M>
__device__ __forceinline__ float half_times(unsigned w, float sc) {
  float r;
  if constexpr (M == 0)
    asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(sc), "v"(-0.0f));
  else
    asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(sc), "v"(-0.0f));
  return r;
}

struct BMatH {
  const __half* a;
  const float* sc;
  long n;
  using V = float;
  __device__ float operator()(int e, int r, long i) const {
    return sc[(long)r * n + i] * __half2float(a[(long)e * n + i]);
  }
};

constexpr int WF_TX = 16, WF_TY = 16;  // columns per wavefront tile (256 lanes)

struct WfTiling {
  int sh, ntx, nty, ns;  // shear, tiles in x / y, steps per tile
  long nsk;              // schedule positions (tiles * steps * lanes)
};

struct Grid {
  int nx, ny, nz;
  __host__ __device__ long N() const { return (long)nx * ny * nz; }
};

__device__ inline bool in_grid(const Grid& g, int x, int y, int z) {
  return x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
}

}  // namespace smg
