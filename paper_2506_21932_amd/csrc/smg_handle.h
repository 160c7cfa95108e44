// Internal layout of a libstructmg handle and the precision traits of the
// V-cycle (shared by the single-system and the batched host code).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/structmg.h"
#include "smg_kernels.h"

#define SMG_TIMING_CAP 16384
#define SMG_TIMING_KINDS 8

namespace smg {

constexpr int MAXLEV = 40;

struct Level {
  Grid g;
  int S = 0;      // pattern points
  int Ssw = 0;    // pattern of the triangular sweeps and their data (ILU: the factor mask; else S)
  int cmask = 0;  // axes coarsened to reach the next level (0: coarsest)
  long N = 0;
  double *A64 = nullptr, *rd64 = nullptr, *L64 = nullptr, *U64 = nullptr, *rU64 = nullptr;
  float *A32 = nullptr, *rd32 = nullptr, *L32 = nullptr, *U32 = nullptr, *rU32 = nullptr;
  __half* A16 = nullptr;
  float* sc16 = nullptr;
  void *f = nullptr, *ua = nullptr, *ub = nullptr, *h = nullptr;
  void *y1 = nullptr, *y2 = nullptr, *zz = nullptr, *uo = nullptr;
  WfTiling tl{};                    // wavefront tiling
  long nsk_cap = 0;                 // schedule positions the packed sweep data has room for (either tile shape)
  void* pk[2] = {nullptr, nullptr};  // packed sweep data, forward / backward (V-cycle precision; FP16: halves)
  float* psd = nullptr;             // FP16: {row scale, diagonal scaling} per schedule position
  int hp_steps = 0;                 // small level: hyperplanes of the one-workgroup sweep (0: tiled sweep)
  int* hp_pts = nullptr;            // its point schedule [step][256]
  void* hp_cf[2] = {nullptr, nullptr};  // its step-ordered coefficients, forward / backward
  double *tr64 = nullptr, *tc64 = nullptr;  // line GS: Thomas 1/pivot and c/pivot per point
  float *tr32 = nullptr, *tc32 = nullptr;
  int lg_K = 0, lg_nt = 0;                  // line GS tiles: side (columns) and number
  int* lg_map = nullptr;                    // their dependence order (bx << 16 | by')
  double* W64 = nullptr;                    // operator-dependent interpolation weights to the next level (8 x N)
  float* W32 = nullptr;                     // their FP32 copy for reduced-precision V-cycles
  // non-default smoothing settings only
  void* ux = nullptr;  // third sweep output when a cycle has an odd number of sweeps per level
  void* uz = nullptr;  // zeros: the old values of the first step without ZeroGuess
  void* qa = nullptr;  // weighted GS: ((1 - w) / w) a_ii, the old-centre term of a full sweep
};

// Smoothing settings of a configuration with the defaults of zero fields
// filled in.
inline int cfg_pre(const smg_config& c) { return c.pre_sweeps > 0 ? c.pre_sweeps : 1; }
inline int cfg_post(const smg_config& c) { return c.post_sweeps > 0 ? c.post_sweeps : 1; }
inline double cfg_weight(const smg_config& c) { return c.relax_weight != 0.0 ? c.relax_weight : 1.0; }
inline bool cfg_zero_guess(const smg_config& c) { return c.zero_guess >= 0; }
inline int cfg_min_coarse(const smg_config& c) { return c.min_coarse > 0 ? c.min_coarse : 4; }
// one ZeroGuess step before and one step after the coarse correction, w = 1
inline bool cfg_default_smoothing(const smg_config& c) {
  return cfg_pre(c) == 1 && cfg_post(c) == 1 && cfg_weight(c) == 1.0 && cfg_zero_guess(c);
}

}  // namespace smg

struct smg_handle_s {
  smg_config cfg{};
  int bs = 1, nlev = 0, nc = 0;
  smg::Level lev[smg::MAXLEV];
  double* aug = nullptr;  // coarsest [.. | A^-1] (n x 2n) + the inversion's work space
  unsigned* ctr = nullptr;
  unsigned* err = nullptr;
  int* info = nullptr;
  double *dpart = nullptr, *dout = nullptr;
  double *kr = nullptr, *kz = nullptr, *kp = nullptr, *kq = nullptr, *kt = nullptr, *kw = nullptr;
  double* kV = nullptr;
  double* kZ = nullptr;  // flexible GMRES: preconditioned basis vectors
  int kV_m = 0;
  double t_setup_ms = 0.0;
  char msg[512] = {0};
  // kernel timing (profiling aid): event pairs per (level, kind)
  // captured graph of the V-cycle on the solver's own vectors (kr -> kz)
  bool use_graph = true;
  bool side_ok = true;  // setup may run per-level work on the library's side streams
  bool hp_on = true;  // small levels use the one-workgroup sweep (off inside batches)
  hipStream_t cap = nullptr;
  hipGraph_t vgraph = nullptr;
  hipGraphExec_t vexec = nullptr;
  bool timing = false;
  int tm_level = -1;      // record only this level (-1: all)
  unsigned tm_kinds = ~0u;  // bit mask of recorded kinds
  int ev_used = 0;
  int ev_tag[SMG_TIMING_CAP];
  hipEvent_t ev0[SMG_TIMING_CAP], ev1[SMG_TIMING_CAP];
};

namespace smg {

// ---- precision traits of the V-cycle ---------------------------------
struct P64 {
  using V = double;
  using M = MatD;
  using MF = MatD;
  using E = double;
  using BM = BMatD;
  static BM BA(const Level& l) { return BMatD{l.A64, l.N}; }
  static M A(const Level& l) { return MatD{l.A64, l.N}; }
  static MF Lf(const Level& l) { return MatD{l.L64, l.N}; }
  static MF Uf(const Level& l) { return MatD{l.U64, l.N}; }
  static const V* rd(const Level& l) { return l.rd64; }
  static const V* rU(const Level& l) { return l.rU64; }
  static const V* Araw(const Level& l) { return l.A64; }
  static const V* tr(const Level& l) { return l.tr64; }
  static const V* tc(const Level& l) { return l.tc64; }
};
struct P32 {
  using V = float;
  using M = MatF;
  using MF = MatF;
  using E = float;
  using BM = BMatF;
  static BM BA(const Level& l) { return BMatF{l.A32, l.N}; }
  static M A(const Level& l) { return MatF{l.A32, l.N}; }
  static MF Lf(const Level& l) { return MatF{l.L32, l.N}; }
  static MF Uf(const Level& l) { return MatF{l.U32, l.N}; }
  static const V* rd(const Level& l) { return l.rd32; }
  static const V* rU(const Level& l) { return l.rU32; }
  static const V* Araw(const Level& l) { return l.A32; }
  static const V* tr(const Level& l) { return l.tr32; }
  static const V* tc(const Level& l) { return l.tc32; }
};
struct P16 {
  using V = float;
  using M = MatH;
  using MF = MatF;
  using E = __half;
  using BM = BMatH;
  static BM BA(const Level& l) { return BMatH{l.A16, l.sc16, l.N}; }
  static M A(const Level& l) { return MatH{l.A16, l.sc16, l.N}; }
  static MF Lf(const Level& l) { return MatF{l.L32, l.N}; }
  static MF Uf(const Level& l) { return MatF{l.U32, l.N}; }
  static const V* rd(const Level& l) { return l.rd32; }
  static const V* rU(const Level& l) { return l.rU32; }
  // line GS keeps no FP16 storage (the configuration is rejected)
  static const V* Araw(const Level&) { return nullptr; }
  static const V* tr(const Level&) { return nullptr; }
  static const V* tc(const Level&) { return nullptr; }
};

// Validation of a configuration (null when supported) and the level shapes
// (grids, patterns, coarsening masks, sweep tilings; no memory) it leads to.
// plan_shapes returns the workspace bytes, or 0 when the coarsest level is
// too large; L holds MAXLEV entries.
const char* config_error(const smg_config* cfg);
size_t plan_shapes(const smg_config& cfg, Level* L, int* nlev, int* nc);

// Re-tiles the sweep of level l (shape 0 default, 1 sheared, 2 rectangular):
// new schedule-ordered sweep data and sentinel state for the level; *why is
// set when the request is refused (hipErrorInvalidValue).
hipError_t retile_level(smg_handle_s* H, int l, int shape, hipStream_t st, const char** why);

}  // namespace smg
