// libstructmg host side: hierarchy setup, V-cycle orchestration, outer
// Krylov solvers and the C ABI declared in include/structmg.h.
//
// Setup builds the hierarchy from the finest matrix only (Sec. 4.2.2):
// multi-dimensional coarsening by fixed stride 2 (Sec. 4.1 P2), coarse
// operators from the generated stencil triple product (Sec. 4.3), smoother
// data per level, then the dense coarsest inverse.  The V-cycle (Sec. 2) runs
// a zero-initial-guess forward GS sweep (or ILU(0) solve) before the coarse
// correction and a backward GS sweep (or ILU(0) correction) after it, the
// symmetric PGS / ILU settings of the paper's configuration table.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <mutex>
#include <vector>

#include "smg_handle.h"

using namespace smg;

static char g_setup_msg[512] = "no error";

// Brackets the launches of one (level, kind) with events on `st` when timing
// is enabled.
struct Timed {
  smg_handle_s* H;
  int slot;
  hipStream_t st;
  Timed(smg_handle_s* h, int level, int kind, hipStream_t s) : H(h), slot(-1), st(s) {
    if (H->timing && H->ev_used < SMG_TIMING_CAP && (H->tm_level < 0 || H->tm_level == level) &&
        ((H->tm_kinds >> kind) & 1u)) {
      slot = H->ev_used++;
      H->ev_tag[slot] = level * SMG_TIMING_KINDS + kind;
      (void)hipEventRecord(H->ev0[slot], st);
    }
  }
  ~Timed() {
    if (slot >= 0) (void)hipEventRecord(H->ev1[slot], st);
  }
};

static smg_status fail(smg_handle h, smg_status st, const char* fmt, ...) {
  char* dst = h ? h->msg : g_setup_msg;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  return st;
}

#define HIPCHK(h, expr)                                                                         \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return fail(h, SMG_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));  \
  } while (0)

namespace {

struct Arena {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Axes coarsened from level lev (dims n): the allowed axes with at least
// nmin points; x,y only on the first semi_levels levels (or always in semi
// mode), where a level whose x and y cannot be coarsened any more switches to
// all axes.
int next_cmask(int lev, const int* n, int semi, int semi_levels, int nmin) {
  int allowed = (semi || lev < semi_levels) ? 3 : 7, m = 0;
  for (int a = 0; a < 3; ++a)
    if (((allowed >> a) & 1) && n[a] >= nmin) m |= 1 << a;
  if (m == 0 && !semi && allowed == 3)
    for (int a = 0; a < 3; ++a)
      if (n[a] >= nmin) m |= 1 << a;
  return m;
}

bool cell_centred(const smg_config& c) {
  return c.interp == SMG_INTERP_CELL || c.interp == SMG_INTERP_CELL_TRILINEAR;
}

const char* check_cfg(const smg_config* c) {
  if (!c) return "null config";
  if (c->nx < 1 || c->ny < 1 || c->nz < 1) return "grid dimensions must be >= 1";
  if ((double)c->nx * c->ny * c->nz * (c->block > 1 ? c->block : 1) >= 2147483647.0) return "grid too large";
  // sweep buffers address 18 x-planes and one tile's steps with 31-bit byte offsets
  if ((double)(WF_TX + 2) * c->ny * c->nz * 8 >= 2147483647.0) return "ny * nz too large (limit 14.9e6)";
  if (c->nz > 65536) return "nz too large (limit 65536)";
  if (c->block == 3 && (double)10 * c->ny * c->nz * 3 * 8 >= 2147483647.0) return "ny * nz too large for 3x3 blocks";
  if (c->block != 1 && c->block != 3) return "block must be 1 or 3";
  if (c->pattern != 7 && c->pattern != 19 && c->pattern != 27) return "pattern must be 7, 19 or 27";
  if (c->block == 3 && c->pattern != 27) return "block systems use the 27-point pattern";
  if (c->smoother != SMG_SMOOTH_GS && c->smoother != SMG_SMOOTH_ILU0 && c->smoother != SMG_SMOOTH_LGS)
    return "unknown smoother";
  if (c->smoother == SMG_SMOOTH_LGS && c->block != 1) return "line GS is implemented for scalar systems";
  if (c->smoother == SMG_SMOOTH_LGS && c->prec == SMG_FP16_ROWSCALE) return "line GS supports FP64 and FP32";
  if (c->smoother == SMG_SMOOTH_LGS && c->nz > LGS_MAX_NZ) return "line GS: nz too large (limit 2047)";
  if (c->smoother == SMG_SMOOTH_ILU0 && c->block != 1) return "ILU(0) is implemented for scalar systems";
  if (c->smoother == SMG_SMOOTH_ILU0 && c->prec == SMG_FP16_ROWSCALE) return "ILU(0) supports FP64 and FP32";
  if (c->coarsen != SMG_COARSEN_FULL && c->coarsen != SMG_COARSEN_SEMI_XY && c->coarsen != SMG_COARSEN_AUTO)
    return "unknown coarsening";
  if (c->coarsen == SMG_COARSEN_AUTO && c->block != 1) return "automatic coarsening takes scalar systems";
  if (c->semi_levels < 0) return "semi_levels must be >= 0";
  if (c->prec < SMG_FP64 || c->prec > SMG_FP16_ROWSCALE) return "unknown precision";
  if (c->max_coarse < 0 || c->gmres_restart < 0 || c->gmres_restart > 200) return "bad max_coarse / gmres_restart";
  if (c->ilu_mask != 0 && c->ilu_mask != 7 && c->ilu_mask != 19 && c->ilu_mask != 27)
    return "ilu_mask must be 0, 7, 19 or 27";
  if (c->ilu_mask != 0 && c->smoother != SMG_SMOOTH_ILU0) return "ilu_mask applies to the ILU(0) smoother only";
  if (c->interp < SMG_INTERP_VERTEX || c->interp > SMG_INTERP_OPERATOR) return "unknown interpolation";
  if (c->interp != SMG_INTERP_VERTEX && c->block != 1)
    return "cell-centred and operator-dependent transfers are implemented for scalar systems";
  if (c->pre_sweeps < 0 || c->pre_sweeps > 8 || c->post_sweeps < 0 || c->post_sweeps > 8)
    return "pre_sweeps / post_sweeps must be 0..8 (0: 1)";
  if (!(c->relax_weight == 0.0 || (c->relax_weight > 0.0 && c->relax_weight < 2.0)))
    return "relax_weight must lie in (0, 2) (0: 1.0)";
  if (cfg_weight(*c) != 1.0 && (c->smoother != SMG_SMOOTH_GS || c->block != 1))
    return "relax_weight other than 1 applies to point GS on scalar systems";
  if (c->zero_guess < -1 || c->zero_guess > 1) return "zero_guess must be -1, 0 or 1";
  if (c->min_coarse != 0 && (c->min_coarse < 2 || c->min_coarse > 4096)) return "min_coarse must be 2..4096 (0: 4)";
  return nullptr;
}

// Lays out every device array of the handle in the workspace (base == null:
// size only).  Returns the number of bytes.
size_t plan(const smg_config& cfg, smg_handle_s* H, char* base, int* nlev_out, int* nc_out, Level* Lext = nullptr) {
  Arena ar{base};
  const int bs = cfg.block, be = bs * bs;
  const int maxc = cfg.max_coarse > 0 ? cfg.max_coarse : 4096;
  const size_t vsz = cfg.prec == SMG_FP64 ? 8 : 4;
  int n[3] = {cfg.nx, cfg.ny, cfg.nz};
  int nlev = 0;
  Level tmp[MAXLEV];
  Level* L = H ? H->lev : (Lext ? Lext : tmp);
  for (;;) {
    Level& v = L[nlev];
    v.g = Grid{n[0], n[1], n[2]};
    v.N = v.g.N();
    v.S = nlev == 0 || cfg.interp == SMG_INTERP_CELL ? cfg.pattern : 27;
    v.Ssw = cfg.smoother == SMG_SMOOTH_ILU0 && nlev == 0 && cfg.ilu_mask ? cfg.ilu_mask : v.S;
    v.cmask = next_cmask(nlev, n, cfg.coarsen == SMG_COARSEN_SEMI_XY, cfg.semi_levels, 2 * cfg_min_coarse(cfg));
    ++nlev;
    if (v.cmask == 0 || nlev == MAXLEV) {
      v.cmask = 0;
      break;
    }
    for (int a = 0; a < 3; ++a)
      if ((v.cmask >> a) & 1) n[a] = cell_centred(cfg) ? (n[a] + 1) / 2 : n[a] / 2;
  }
  const long nc = L[nlev - 1].N * bs;
  if (nlev_out) *nlev_out = nlev;
  if (nc_out) *nc_out = (int)nc;
  if (nc > maxc) return 0;
  for (int l = 0; l < nlev; ++l) {
    Level& v = L[l];
    const long N = v.N;
    const bool last = l == nlev - 1;
    v.A64 = ar.take<double>((size_t)v.S * be * N);
    auto vec = [&](void** p) { *p = ar.take<char>((size_t)N * bs * vsz); };
    vec(&v.f);
    vec(&v.ub);
    if (last) continue;
    vec(&v.ua);
    vec(&v.h);
    if ((cfg_pre(cfg) + cfg_post(cfg)) % 2 == 1 && cfg.smoother != SMG_SMOOTH_ILU0) vec(&v.ux);
    if (!cfg_zero_guess(cfg)) vec(&v.uz);
    if (cfg_weight(cfg) != 1.0) v.qa = ar.take<char>((size_t)N * vsz);
    v.rd64 = ar.take<double>((size_t)(bs == 3 ? 9 : 1) * N);
    if (cfg.interp == SMG_INTERP_OPERATOR) {
      v.W64 = ar.take<double>((size_t)8 * N);
      if (cfg.prec != SMG_FP64) v.W32 = ar.take<float>((size_t)8 * N);
    }
    if (cfg.smoother == SMG_SMOOTH_ILU0) {
      v.L64 = ar.take<double>((size_t)v.Ssw * N);
      v.U64 = ar.take<double>((size_t)v.Ssw * N + 2);  // + the factorisation's {0, 1}
      v.rU64 = ar.take<double>((size_t)N);
      vec(&v.y1);
      vec(&v.y2);
      vec(&v.zz);
      vec(&v.uo);
    }
    const int eb = cfg.prec == SMG_FP16_ROWSCALE ? 2 : (int)vsz;
    if (cfg.smoother == SMG_SMOOTH_LGS) {
      v.lg_nt = lgs_plan(v.g, v.S, &v.lg_K, nullptr);
      v.lg_map = ar.take<int>((size_t)v.lg_nt);
      v.tr64 = ar.take<double>((size_t)N);
      v.tc64 = ar.take<double>((size_t)N);
      if (cfg.prec == SMG_FP32) {
        v.tr32 = ar.take<float>((size_t)N);
        v.tc32 = ar.take<float>((size_t)N);
      }
    } else if (bs == 1) {
      // room for the sweep data of either tile shape (smg_set_tile_shape)
      WfTiling t1, t2;
      wf_tiling(v.g, v.Ssw, &t1, 1);
      wf_tiling(v.g, v.Ssw, &t2, 2);
      wf_tiling(v.g, v.Ssw, &v.tl);
      v.nsk_cap = std::max(t1.nsk, t2.nsk);
      const size_t pbytes = (size_t)wf_pack_count(v.Ssw, eb) * 16 * v.nsk_cap;
      v.pk[0] = ar.take<char>(pbytes);
      v.pk[1] = ar.take<char>(pbytes);
      if (cfg.prec == SMG_FP16_ROWSCALE) v.psd = ar.take<float>((size_t)2 * v.nsk_cap);
      v.hp_steps = cfg.smoother == SMG_SMOOTH_GS ? hp_plan(v.g, v.S, (int)vsz, nullptr) : 0;
      if (v.hp_steps > 0) {
        v.hp_pts = ar.take<int>((size_t)v.hp_steps * 256);
        const size_t kv = 16 / vsz, npk = (v.S / 2 + 1 + kv - 1) / kv;  // 16-byte packs per point
        v.hp_cf[0] = ar.take<char>((size_t)v.hp_steps * npk * 256 * 16);
        v.hp_cf[1] = ar.take<char>((size_t)v.hp_steps * npk * 256 * 16);
      }
    } else {
      bwf_tiling(v.g, &v.tl);
      const size_t pbytes = (size_t)bwf_pack_count(eb) * 16 * v.tl.nsk;
      v.pk[0] = ar.take<char>(pbytes);
      v.pk[1] = ar.take<char>(pbytes);
    }
    if (cfg.prec == SMG_FP32) {
      v.A32 = ar.take<float>((size_t)v.S * be * N);
      v.rd32 = ar.take<float>((size_t)(bs == 3 ? 9 : 1) * N);
      if (cfg.smoother == SMG_SMOOTH_ILU0) {
        v.L32 = ar.take<float>((size_t)v.Ssw * N);
        v.U32 = ar.take<float>((size_t)v.Ssw * N);
        v.rU32 = ar.take<float>((size_t)N);
      }
    } else if (cfg.prec == SMG_FP16_ROWSCALE) {
      v.A16 = ar.take<__half>((size_t)v.S * be * N);
      v.sc16 = ar.take<float>((size_t)bs * N);
      v.rd32 = ar.take<float>((size_t)(bs == 3 ? 9 : 1) * N);
    }
  }
  double* aug = ar.take<double>((size_t)nc * 2 * nc + coarse_invert_extra(nc));
  unsigned* ctr = ar.take<unsigned>(64);
  unsigned* err = ar.take<unsigned>(64);
  int* info = ar.take<int>(64);
  double* dpart = ar.take<double>(DOT_BLOCKS);
  double* dout = ar.take<double>(64);
  const long n0 = L[0].N * bs;
  double* kr = ar.take<double>(n0);
  double* kz = ar.take<double>(n0);
  double* kp = ar.take<double>(n0);
  double* kq = ar.take<double>(n0);
  double* kt = ar.take<double>(n0);
  double* kw = ar.take<double>(n0);
  double* kV = cfg.gmres_restart > 0 ? ar.take<double>((size_t)n0 * (cfg.gmres_restart + 1)) : nullptr;
  double* kZ = cfg.gmres_restart > 0 ? ar.take<double>((size_t)n0 * cfg.gmres_restart) : nullptr;
  if (H) {
    H->aug = aug;
    H->ctr = ctr;
    H->err = err;
    H->info = info;
    H->dpart = dpart;
    H->dout = dout;
    H->kr = kr;
    H->kz = kz;
    H->kp = kp;
    H->kq = kq;
    H->kt = kt;
    H->kw = kw;
    H->kV = kV;
    H->kZ = kZ;
    H->kV_m = cfg.gmres_restart;
  }
  return ar.off + 256;
}

template <class E, class V>
hipError_t sweep(smg_handle_s* H, const Level& L, int dir, bool unitd, const V* hin, V* x, V* next, int next_dir,
                 const V* addv, V* addout, hipStream_t st) {
  // small level: every sweep on it runs in one workgroup (no sentinels used)
  if (L.hp_steps > 0 && H->hp_on && !unitd && addout == nullptr)
    return launch_hpsweep<V>(L.S, dir, L.g, L.hp_steps, L.hp_pts, (const V*)L.hp_cf[dir > 0 ? 0 : 1], hin, x, st);
  WfArgs<V> a{};
  a.g = L.g;
  a.t = L.tl;
  a.pk = L.pk[dir > 0 ? 0 : 1];
  a.sd = L.psd;
  a.h = hin;
  a.x = x;
  a.next = next;
  a.next_dir = next_dir;
  a.addv = addv;
  a.addout = addout;
  a.ctr = H->ctr;
  a.err = H->err;
  return launch_wavefront<E>(L.Ssw, dir, unitd, addout != nullptr, a, st);
}

template <class E, class V>
hipError_t bsweep(smg_handle_s* H, const Level& L, int dir, const V* hin, V* x, V* next, int next_dir,
                  hipStream_t st) {
  WfArgs<V> a{};
  a.g = L.g;
  a.t = L.tl;
  a.pk = L.pk[dir > 0 ? 0 : 1];
  a.h = hin;
  a.x = x;
  a.next = next;
  a.next_dir = next_dir;
  a.ctr = H->ctr;
  a.err = H->err;
  return launch_bwavefront<E>(dir, a, st);
}

// V-cycle of a 3x3 block system: point-block GS before and after the coarse
// correction; residual, restriction and prolongation per component.
template <class PT>
hipError_t bvcycle_t(smg_handle_s* H, const typename PT::V* f0, typename PT::V* z0, hipStream_t st) {
  using V = typename PT::V;
  using E = typename PT::E;
  const int NL = H->nlev;
  auto F = [&](int l) -> const V* { return l == 0 ? f0 : (const V*)H->lev[l].f; };
  auto UB = [&](int l) -> V* { return l == 0 ? z0 : (V*)H->lev[l].ub; };
  hipError_t e;
  for (int l = 0; l < NL - 1; ++l) {
    const Level& v = H->lev[l];
    {
      Timed t(H, l, 0, st);
      e = bsweep<E, V>(H, v, +1, F(l), (V*)v.ua, UB(l), -1, st);
    }
    if (e != hipSuccess) return e;
    Timed t(H, l, 2, st);
    e = launch_bspmv(v.g, PT::BA(v), (const V*)v.ua, F(l), (V*)v.h, true, st);
    if (e == hipSuccess) e = launch_restrict<V>(v.g, v.cmask, 3, (const V*)v.h, (V*)H->lev[l + 1].f, st);
    if (e != hipSuccess) return e;
  }
  {
    Timed t(H, NL - 1, 3, st);
    e = launch_coarse_gemv<V>(H->nc, H->aug + H->nc, 2 * H->nc, F(NL - 1), UB(NL - 1), st);
  }
  if (e != hipSuccess) return e;
  for (int l = NL - 2; l >= 0; --l) {
    const Level& v = H->lev[l];
    {
      Timed t(H, l, 4, st);
      e = launch_prolong_add<V>(v.g, v.cmask, 3, (const V*)UB(l + 1), (V*)v.ua, st);
      if (e == hipSuccess) e = launch_blower(v.g, PT::BA(v), F(l), (const V*)v.ua, (V*)v.h, st);
    }
    if (e != hipSuccess) return e;
    Timed t(H, l, 5, st);
    e = bsweep<E, V>(H, v, -1, (const V*)v.h, UB(l), (V*)v.ua, +1, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Scalar levels of at least this many points run the residual + restriction
// and the prolongation + lower-triangle terms as two plain passes each (more
// workgroups, no halo recomputation); smaller levels use the fused one-launch
// kernels, whose single launch costs less there.  Both forms give identical
// bits.
constexpr long SPLIT_MIN_POINTS = 1L << 17;
static bool split_rp(const Level& v) { return v.N >= SPLIT_MIN_POINTS; }

// One line GS sweep on level v: x = LGS(f) from the values uold (null: zero
// initial guess, forward only); next receives the sentinel (or null).
template <class PT>
hipError_t lgs_sweep(smg_handle_s* H, const Level& v, int dir, const typename PT::V* f, const typename PT::V* uold,
                     typename PT::V* x, typename PT::V* next, hipStream_t st) {
  using V = typename PT::V;
  LgsArgs<V> a{};
  a.g = v.g;
  a.A = PT::Araw(v);
  a.rden = PT::tr(v);
  a.cp = PT::tc(v);
  if (!a.A || !a.rden || !a.cp) return hipErrorInvalidValue;
  a.f = f;
  a.uold = uold;
  a.x = x;
  a.next = next;
  a.K = v.lg_K;
  a.ntile = v.lg_nt;
  a.tmap = v.lg_map;
  a.ctr = H->ctr;
  a.err = H->err;
  return launch_lgs<V>(v.S, dir, uold == nullptr, a, st);
}

// operator-dependent interpolation weights of level v in precision V
template <class V>
const V* od_weights(const Level& v) {
  return sizeof(V) == 8 ? reinterpret_cast<const V*>(v.W64) : reinterpret_cast<const V*>(v.W32);
}

// uout = uin + P ec for the cell-centred and operator-dependent
// interpolations (uout may be uin).
template <class V>
hipError_t prolong_cell(const smg_handle_s* H, const Level& v, const V* ec, const V* uin, V* uout, hipStream_t st) {
  if (H->cfg.interp == SMG_INTERP_OPERATOR)
    return launch_prolong_od<V>(v.g, v.cmask, od_weights<V>(v), ec, uin, uout, st);
  if (H->cfg.interp == SMG_INTERP_CELL_TRILINEAR)
    return launch_prolong_c64<V>(v.g, v.cmask, H->bs, ec, uin, uout, st);
  return launch_prolong_cc<V>(v.g, v.cmask, H->bs, ec, uin, uout, st);
}

// rc = R rf with the handle's restriction (bs components per point).
template <class V>
hipError_t restrict_any(const smg_handle_s* H, const Level& v, const V* rf, V* rc, hipStream_t st) {
  if (H->cfg.interp == SMG_INTERP_OPERATOR)
    return launch_restrict_od<V>(v.g, v.cmask, od_weights<V>(v), rf, rc, st);
  if (H->cfg.interp != SMG_INTERP_VERTEX) return launch_restrict_cc<V>(v.g, v.cmask, H->bs, rf, rc, st);
  return launch_restrict<V>(v.g, v.cmask, H->bs, rf, rc, st);
}

// uf += P ec with the handle's interpolation (bs components per point).
template <class V>
hipError_t prolong_in_place(const smg_handle_s* H, const Level& v, const V* ec, V* uf, hipStream_t st) {
  if (H->cfg.interp != SMG_INTERP_VERTEX) return prolong_cell<V>(H, v, ec, uf, uf, st);
  return launch_prolong_add<V>(v.g, v.cmask, H->bs, ec, uf, st);
}

// h = f minus the terms a GS sweep in direction dir takes from the values u
// of before the sweep (upper neighbours forward, lower backward), plus, for
// weight w != 1, the old-centre term ((1 - w) / w) a_ii u_i: with the
// diagonal factor w / a_ii of the packed sweep data this makes the sweep the
// weighted one of the GS formulas (Sec. 4.4).
template <class PT>
hipError_t old_terms(smg_handle_s* H, const Level& v, int dir, const typename PT::V* f, const typename PT::V* u,
                     typename PT::V* h, hipStream_t st) {
  using V = typename PT::V;
  hipError_t e;
  if (H->bs == 3)
    e = dir > 0 ? launch_bupper(v.g, PT::BA(v), f, u, h, st) : launch_blower(v.g, PT::BA(v), f, u, h, st);
  else
    e = dir > 0 ? launch_upper(v.S, v.g, PT::A(v), f, u, h, st) : launch_lower(v.S, v.g, PT::A(v), f, u, h, st);
  if (e == hipSuccess && v.qa) e = launch_vfma<V>(v.N, (const V*)v.qa, u, h, st);
  return e;
}

// V-cycle with the smoothing settings of the configuration (pre_sweeps and
// post_sweeps steps per level, GS weight, ZeroGuess on or off), from plain
// passes: every GS step is "old-value terms, then the triangular sweep";
// every ILU(0) step is "residual, L solve, U solve, add".  The default
// settings take vcycle_t's fused forms instead; both apply the same
// operations to each value.
//
// GS step k of a level (0 <= k < T = pre + post) runs in direction D(k) and
// writes X(k); the step before it left the sentinels of direction D(k) in
// X(k) (the last step of a cycle prepares X(0) of the next cycle, setup
// prepares every buffer once).  X alternates between u_a and the level's
// output, so X(k + 1) = X(k - 1): that buffer's old values were consumed by
// the old-value pass (GS) or are read only by columns this sweep waits for
// (line GS) before it receives sentinels.  With T odd, X(0) is a third
// buffer u_x so that the last step still ends in the level's output.
template <class PT>
hipError_t vcycle_gen_t(smg_handle_s* H, const typename PT::V* f0, typename PT::V* z0, hipStream_t st) {
  using V = typename PT::V;
  using E = typename PT::E;
  const int NL = H->nlev, bs = H->bs;
  const int m = cfg_pre(H->cfg), T = m + cfg_post(H->cfg);
  const bool zg = cfg_zero_guess(H->cfg);
  const bool ilu = H->cfg.smoother == SMG_SMOOTH_ILU0;
  const bool lgs = H->cfg.smoother == SMG_SMOOTH_LGS;
  auto F = [&](int l) -> const V* { return l == 0 ? f0 : (const V*)H->lev[l].f; };
  auto UB = [&](int l) -> V* { return l == 0 ? z0 : (V*)H->lev[l].ub; };
  auto X = [&](int l, int k) -> V* {
    const Level& v = H->lev[l];
    if (T % 2 == 1 && k == 0) return (V*)v.ux;
    return (k % 2 == 0) == (T % 2 == 0) ? (V*)v.ua : UB(l);
  };
  // pre-steps alternate forward, backward, ...; post-steps start opposite to the last pre-step
  auto D = [&](int k) {
    if (k < m) return k % 2 == 0 ? 1 : -1;
    const int last = (m - 1) % 2 == 0 ? 1 : -1;
    return (k - m) % 2 == 0 ? -last : last;
  };
  // GS / line GS step k of level l
  auto gs_step = [&](int l, int k) -> hipError_t {
    const Level& v = H->lev[l];
    const int kn = (k + 1) % T;
    V* x = X(l, k);
    V* nx = X(l, kn);
    const bool first_zg = k == 0 && zg;
    const V* uold = k == 0 ? (zg ? nullptr : (const V*)v.uz) : X(l, k - 1);
    Timed t(H, l, k < m ? 0 : 5, st);
    if (lgs) return lgs_sweep<PT>(H, v, D(k), F(l), uold, x, nx, st);
    const V* hin = F(l);
    if (!first_zg) {
      hipError_t e = old_terms<PT>(H, v, D(k), F(l), uold, (V*)v.h, st);
      if (e != hipSuccess) return e;
      hin = (const V*)v.h;
    }
    if (bs == 3) return bsweep<E, V>(H, v, D(k), hin, x, nx, D(kn), st);
    return sweep<E, V>(H, v, D(k), false, hin, x, nx, D(kn), nullptr, nullptr, st);
  };
  // ILU(0) step k: out = u + U^-1 L^-1 (f - A u) (u null: the ZeroGuess
  // solve into u_a).  The L solve of step k writes LB(k), alternately y1 and
  // y2, whose sentinels the U solve of step k - 1 (which reads the other one)
  // has written; the U solve writes zz (sentinels from the L solve) or u_a.
  // With T odd the last step would have to prepare the buffer it reads, so
  // the cycle refills y1 before its first step instead.
  auto LB = [&](const Level& v, int k) -> V* { return k % 2 == 0 ? (V*)v.y1 : (V*)v.y2; };
  auto ilu_step = [&](int l, int k, const V* u, V* out, int kind) -> hipError_t {
    const Level& v = H->lev[l];
    const auto A = PT::A(v);
    V* nxt = k + 1 < T ? LB(v, k + 1) : (T % 2 == 0 ? LB(v, 0) : nullptr);
    hipError_t e;
    Timed t(H, l, kind, st);
    if (!u) {
      e = sweep<E, V>(H, v, +1, true, F(l), LB(v, k), (V*)v.ua, -1, nullptr, nullptr, st);
      if (e == hipSuccess) e = sweep<E, V>(H, v, -1, false, (const V*)LB(v, k), (V*)v.ua, nxt, +1, nullptr, nullptr, st);
      return e;
    }
    e = launch_spmv(v.S, v.g, A, u, F(l), (V*)v.h, true, st);
    if (e == hipSuccess) e = sweep<E, V>(H, v, +1, true, (const V*)v.h, LB(v, k), (V*)v.zz, -1, nullptr, nullptr, st);
    if (e == hipSuccess) e = sweep<E, V>(H, v, -1, false, (const V*)LB(v, k), (V*)v.zz, nxt, +1, u, out, st);
    return e;
  };
  V sent;
  if (sizeof(V) == 8) {
    uint64_t b = SENT64;
    memcpy(&sent, &b, 8);
  } else {
    uint32_t b = SENT32;
    memcpy(&sent, &b, 4);
  }
  hipError_t e;
  std::vector<V*> upre(NL);  // each level's pre-smoothed values
  for (int l = 0; l < NL - 1; ++l) {
    const Level& v = H->lev[l];
    if (ilu) {
      if (T % 2 == 1) {
        e = launch_fill_bits<V>((V*)v.y1, v.N, sent, st);
        if (e != hipSuccess) return e;
      }
      V* u = nullptr;
      for (int k = 0; k < m; ++k) {
        V* out = (u == (V*)v.ua) ? (V*)v.uo : (V*)v.ua;
        e = ilu_step(l, k, k == 0 ? (zg ? nullptr : (const V*)v.uz) : u, out, 0);
        if (e != hipSuccess) return e;
        u = (k == 0 && zg) ? (V*)v.ua : out;
      }
      upre[l] = u;
    } else {
      for (int k = 0; k < m; ++k) {
        e = gs_step(l, k);
        if (e != hipSuccess) return e;
      }
      upre[l] = X(l, m - 1);
    }
    Timed t(H, l, 2, st);
    if (bs == 3) {
      e = launch_bspmv(v.g, PT::BA(v), (const V*)upre[l], F(l), (V*)v.h, true, st);
      if (e == hipSuccess) e = launch_restrict<V>(v.g, v.cmask, 3, (const V*)v.h, (V*)H->lev[l + 1].f, st);
    } else {
      e = launch_spmv(v.S, v.g, PT::A(v), (const V*)upre[l], F(l), (V*)v.h, true, st);
      if (e == hipSuccess) e = restrict_any<V>(H, v, (const V*)v.h, (V*)H->lev[l + 1].f, st);
    }
    if (e != hipSuccess) return e;
  }
  {
    Timed t(H, NL - 1, 3, st);
    e = launch_coarse_gemv<V>(H->nc, H->aug + H->nc, 2 * H->nc, F(NL - 1), UB(NL - 1), st);
  }
  if (e != hipSuccess) return e;
  for (int l = NL - 2; l >= 0; --l) {
    const Level& v = H->lev[l];
    {
      Timed t(H, l, 4, st);
      e = bs == 3 ? launch_prolong_add<V>(v.g, v.cmask, 3, (const V*)UB(l + 1), upre[l], st)
                  : prolong_in_place<V>(H, v, (const V*)UB(l + 1), upre[l], st);
    }
    if (e != hipSuccess) return e;
    if (ilu) {
      const int p = T - m;
      V* u = upre[l];
      for (int k = 0; k < p; ++k) {
        V* out = k == p - 1 ? UB(l) : (u == (V*)v.ua ? (V*)v.uo : (V*)v.ua);
        e = ilu_step(l, m + k, u, out, 5);
        if (e != hipSuccess) return e;
        u = out;
      }
    } else {
      for (int k = m; k < T; ++k) {
        e = gs_step(l, k);
        if (e != hipSuccess) return e;
      }
    }
  }
  return hipSuccess;
}

// One V-cycle on internal or caller vectors: f0 = level-0 right-hand side,
// z0 = level-0 output (its positions read across tiles are given sentinels by
// the pre-smoothing sweep).
template <class PT>
hipError_t vcycle_t(smg_handle_s* H, const typename PT::V* f0, typename PT::V* z0, hipStream_t st) {
  using V = typename PT::V;
  if (!cfg_default_smoothing(H->cfg)) return vcycle_gen_t<PT>(H, f0, z0, st);
  if (H->bs == 3) return bvcycle_t<PT>(H, f0, z0, st);
  const int NL = H->nlev;
  const bool ilu = H->cfg.smoother == SMG_SMOOTH_ILU0;
  const bool lgs = H->cfg.smoother == SMG_SMOOTH_LGS;
  // transfers other than the vertex trilinear ones run as separate passes
  const bool sep = H->cfg.interp != SMG_INTERP_VERTEX;
  auto F = [&](int l) -> const V* { return l == 0 ? f0 : (const V*)H->lev[l].f; };
  auto UB = [&](int l) -> V* { return l == 0 ? z0 : (V*)H->lev[l].ub; };
  hipError_t e;
  for (int l = 0; l < NL - 1; ++l) {
    const Level& v = H->lev[l];
    const auto A = PT::A(v);
    if (lgs) {
      // forward line GS from zero into u_a; the level's output gets sentinels
      Timed t(H, l, 0, st);
      e = lgs_sweep<PT>(H, v, +1, F(l), nullptr, (V*)v.ua, UB(l), st);
    } else if (!ilu) {
      Timed t(H, l, 0, st);
      e = sweep<typename PT::E, V>(H, v, +1, false, F(l), (V*)v.ua, UB(l), -1, nullptr, nullptr, st);
    } else {
      {
        Timed t(H, l, 0, st);
        e = sweep<typename PT::E, V>(H, v, +1, true, F(l), (V*)v.y1, (V*)v.ua, -1, nullptr, nullptr, st);
      }
      if (e != hipSuccess) return e;
      Timed t(H, l, 1, st);
      e = sweep<typename PT::E, V>(H, v, -1, false, (const V*)v.y1, (V*)v.ua, (V*)v.y2, +1, nullptr, nullptr, st);
    }
    if (e != hipSuccess) return e;
    {
      Timed t(H, l, 2, st);
      if (sep) {
        e = launch_spmv(v.S, v.g, A, (const V*)v.ua, F(l), (V*)v.h, true, st);
        if (e == hipSuccess) e = restrict_any<V>(H, v, (const V*)v.h, (V*)H->lev[l + 1].f, st);
      } else if (split_rp(v)) {
        // residual into the level's h (free until the upward leg), then R
        e = launch_spmv(v.S, v.g, A, (const V*)v.ua, F(l), (V*)v.h, true, st);
        if (e == hipSuccess) e = launch_restrict<V>(v.g, v.cmask, 1, (const V*)v.h, (V*)H->lev[l + 1].f, st);
      } else {
        e = launch_resid_restrict(v.S, v.g, v.cmask, A, F(l), (const V*)v.ua, (V*)H->lev[l + 1].f, st);
      }
    }
    if (e != hipSuccess) return e;
  }
  {
    Timed t(H, NL - 1, 3, st);
    e = launch_coarse_gemv<V>(H->nc, H->aug + H->nc, 2 * H->nc, F(NL - 1), UB(NL - 1), st);
  }
  if (e != hipSuccess) return e;
  for (int l = NL - 2; l >= 0; --l) {
    const Level& v = H->lev[l];
    const auto A = PT::A(v);
    if (lgs) {
      {
        Timed t(H, l, 4, st);
        e = prolong_in_place<V>(H, v, (const V*)UB(l + 1), (V*)v.ua, st);
      }
      if (e != hipSuccess) return e;
      // backward line GS from u_a + P e_c; u_a gets its sentinels back
      Timed t(H, l, 5, st);
      e = lgs_sweep<PT>(H, v, -1, F(l), (const V*)v.ua, UB(l), (V*)v.ua, st);
    } else if (!ilu) {
      {
        Timed t(H, l, 4, st);
        if (sep || split_rp(v)) {
          // u_old = u + P e_c in place (u_a is refilled by the sweep below),
          // then the backward sweep's old-value terms
          e = prolong_in_place<V>(H, v, (const V*)UB(l + 1), (V*)v.ua, st);
          if (e == hipSuccess) e = launch_lower(v.S, v.g, A, F(l), (const V*)v.ua, (V*)v.h, st);
        } else {
          e = launch_prolong_post(v.S, v.g, v.cmask, A, F(l), (const V*)v.ua, (const V*)UB(l + 1), (V*)v.h,
                                  (V*)nullptr, false, st);
        }
      }
      if (e != hipSuccess) return e;
      Timed t(H, l, 5, st);
      e = sweep<typename PT::E, V>(H, v, -1, false, (const V*)v.h, UB(l), (V*)v.ua, +1, nullptr, nullptr, st);
    } else {
      {
        Timed t(H, l, 4, st);
        if (sep) {
          // u_old = u_a + P e_c into u_o, then h = f - A u_old
          e = prolong_cell<V>(H, v, (const V*)UB(l + 1), (const V*)v.ua, (V*)v.uo, st);
          if (e == hipSuccess) e = launch_spmv(v.S, v.g, A, (const V*)v.uo, F(l), (V*)v.h, true, st);
        } else {
          e = launch_prolong_post(v.S, v.g, v.cmask, A, F(l), (const V*)v.ua, (const V*)UB(l + 1), (V*)v.h,
                                  (V*)v.uo, true, st);
        }
      }
      if (e != hipSuccess) return e;
      {
        Timed t(H, l, 5, st);
        e = sweep<typename PT::E, V>(H, v, +1, true, (const V*)v.h, (V*)v.y2, (V*)v.zz, -1, nullptr, nullptr, st);
      }
      if (e != hipSuccess) return e;
      Timed t(H, l, 6, st);
      e = sweep<typename PT::E, V>(H, v, -1, false, (const V*)v.y2, (V*)v.zz, (V*)v.y1, +1, (const V*)v.uo, UB(l), st);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t vcycle(smg_handle_s* H, const double* r, double* z, hipStream_t st) {
  const Level& l0 = H->lev[0];
  const long n0 = l0.N * H->bs;
  switch (H->cfg.prec) {
    case SMG_FP64:
      return vcycle_t<P64>(H, r, z, st);
    case SMG_FP32: {
      hipError_t e = launch_cast_d2f(n0, r, (float*)l0.f, st);
      if (e == hipSuccess) e = vcycle_t<P32>(H, (const float*)l0.f, (float*)l0.ub, st);
      if (e == hipSuccess) e = launch_cast_f2d(n0, (const float*)l0.ub, z, st);
      return e;
    }
    default: {
      hipError_t e = launch_cast_d2f(n0, r, (float*)l0.f, st);
      if (e == hipSuccess) e = vcycle_t<P16>(H, (const float*)l0.f, (float*)l0.ub, st);
      if (e == hipSuccess) e = launch_cast_f2d(n0, (const float*)l0.ub, z, st);
      return e;
    }
  }
}

hipError_t spmv64(smg_handle_s* H, const double* x, const double* b, double* y, bool res, hipStream_t st) {
  const Level& l0 = H->lev[0];
  Timed t(H, 0, 7, st);
  if (H->bs == 3) return launch_bspmv(l0.g, BMatD{l0.A64, l0.N}, x, b, y, res, st);
  return launch_spmv(l0.S, l0.g, MatD{l0.A64, l0.N}, x, b, y, res, st);
}

void drop_vgraph(smg_handle_s* H) {
  if (H->vexec) (void)hipGraphExecDestroy(H->vexec);
  if (H->vgraph) (void)hipGraphDestroy(H->vgraph);
  H->vexec = nullptr;
  H->vgraph = nullptr;
}

// z = M r on the solver's vectors: replays a captured graph of the whole
// V-cycle (one launch for all its kernels) unless graphs are off or kernel
// timing is on; the graph is captured at the first use.
hipError_t vcycle_solver(smg_handle_s* H, hipStream_t st) {
  if (!H->use_graph || H->timing) return vcycle(H, H->kr, H->kz, st);
  if (!H->vexec) {
    hipError_t e = hipSuccess;
    if (!H->cap) e = hipStreamCreateWithFlags(&H->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(H->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t ev = vcycle(H, H->kr, H->kz, H->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(H->cap, &g);
    if (ev != hipSuccess) e = ev;
    if (e == hipSuccess) {
      H->vgraph = g;
      e = hipGraphInstantiate(&H->vexec, g, nullptr, nullptr, 0);
      if (e != hipSuccess) drop_vgraph(H);
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
    if (e != hipSuccess) return e;
  }
  return hipGraphLaunch(H->vexec, st);
}

smg_status check_err(smg_handle_s* H, hipStream_t st) {
  unsigned e = 0;
  HIPCHK(H, hipMemcpyAsync(&e, H->err, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  HIPCHK(H, hipStreamSynchronize(st));
  if (e & 1u) return fail(H, SMG_EDEADLOCK, "wavefront watchdog fired");
  if (e & 2u) return fail(H, SMG_EBREAKDOWN, "zero pivot or zero diagonal");
  return SMG_OK;
}

double dot(smg_handle_s* H, const double* x, const double* y, long n, hipStream_t st, hipError_t* e) {
  double v = 0.0;
  *e = launch_dot(n, x, y, H->dpart, H->dout, st);
  if (*e != hipSuccess) return 0.0;
  *e = hipMemcpyAsync(&v, H->dout, sizeof(double), hipMemcpyDeviceToHost, st);
  if (*e != hipSuccess) return 0.0;
  *e = hipStreamSynchronize(st);
  return v;
}


}  // namespace

namespace smg {
const char* config_error(const smg_config* cfg) { return check_cfg(cfg); }
size_t plan_shapes(const smg_config& cfg, Level* L, int* nlev, int* nc) {
  return plan(cfg, nullptr, nullptr, nlev, nc, L);
}
}  // namespace smg

namespace {

// Streams for the setup work of different levels, which is independent once
// the triple products are done (the ILU(0) factorisation in particular is
// bound by the latency of one hyperplane after another and occupies few
// compute units).  One pool per device for the life of the process, at the
// default priority.
constexpr int SETUP_SIDE = 3;
constexpr int SETUP_DEVICES = 64;
static hipStream_t g_side[SETUP_DEVICES][SETUP_SIDE];
static std::mutex g_side_mu;

static hipError_t side_streams(hipStream_t* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= SETUP_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_side_mu);
  for (int k = 0; k < SETUP_SIDE; ++k) {
    if (!g_side[dev][k]) {
      e = hipStreamCreateWithFlags(&g_side[dev][k], hipStreamNonBlocking);
      if (e != hipSuccess) return e;
    }
    out[k] = g_side[dev][k];
  }
  return hipSuccess;
}

constexpr long SETUP_SIDE_POINTS = 1L << 21;  // finest levels from this size use the side streams

// Events that join the side streams back into the caller's stream; on an
// early return the side streams are drained before the events go.
struct SideJoin {
  hipEvent_t ev[SETUP_SIDE + 1] = {};
  hipStream_t* side = nullptr;
  bool joined = false;
  ~SideJoin() {
    if (side && !joined)
      for (int k = 0; k < SETUP_SIDE; ++k) (void)hipStreamSynchronize(side[k]);
    for (hipEvent_t& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

// Scalar point-smoother levels: the sweep data of both directions in the
// schedule order of the level's current tiling.
hipError_t pack_sweep_data(smg_handle_s* H, Level& v, hipStream_t st) {
  const smg_config* cfg = &H->cfg;
  const bool ilu = cfg->smoother == SMG_SMOOTH_ILU0;
  const double* lo = ilu ? v.L64 : v.A64;
  const double* up = ilu ? v.U64 : v.A64;
  const double* dg = ilu ? v.rU64 : v.rd64;
  for (int d = 0; d < 2; ++d) {
    const int dir = d == 0 ? 1 : -1;
    hipError_t e;
    if (cfg->prec == SMG_FP64)
      e = launch_wf_pack<double>(v.Ssw, v.g, v.tl, dir, lo, dg, up, (double*)v.pk[d], st);
    else if (cfg->prec == SMG_FP32)
      e = launch_wf_pack<float>(v.Ssw, v.g, v.tl, dir, lo, dg, up, (float*)v.pk[d], st);
    else
      e = launch_wf_pack_h(v.S, v.g, v.tl, dir, v.A16, v.sc16, v.rd32, (__half*)v.pk[d], v.psd, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Every smoothing buffer of a level filled with the sentinel: the state the
// first sweep of a cycle expects whatever the tiling (each sweep then hands
// the next one its sentinels).
hipError_t fill_sentinels(smg_handle_s* H, Level& v, hipStream_t st) {
  const long nv = v.N * H->bs;
  void* bufs[] = {v.ua, v.ub, v.y1, v.y2, v.zz, v.ux};
  for (void* p : bufs) {
    if (!p) continue;
    hipError_t e;
    if (H->cfg.prec == SMG_FP64) {
      double s;
      uint64_t b = SENT64;
      memcpy(&s, &b, 8);
      e = launch_fill_bits<double>((double*)p, nv, s, st);
    } else {
      float s;
      uint32_t b = SENT32;
      memcpy(&s, &b, 4);
      e = launch_fill_bits<float>((float*)p, nv, s, st);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Setup pipeline on an already planned handle (used by smg_setup and
// smg_resetup): level-0 copy, triple products, smoother data, truncation,
// sentinel fills, coarsest inverse.  Large hierarchies build the smoother
// data of level 0, level 1 and the remaining levels on three side streams
// that start after the triple products and join the caller's stream before
// the final synchronisation.
smg_status build_hierarchy(smg_handle_s* H, const double* coeffs, hipStream_t st) {
  const smg_config* cfg = &H->cfg;
  const int bs = H->bs, be = bs * bs;
#define SCHK(expr)                                                                            \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(H, SMG_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)
  SCHK(launch_fill_bits<unsigned>(H->ctr, 64, 0u, st));
  SCHK(launch_fill_bits<unsigned>(H->err, 64, 0u, st));
  SCHK(launch_fill_bits<unsigned>((unsigned*)H->info, 64, 0u, st));
  // level 0 copy (Dirichlet couplings zeroed), coarse operators by RAP
  SCHK(launch_copy_masked(H->lev[0].S, H->lev[0].g, be, coeffs, H->lev[0].A64, st));
  for (int l = 0; l + 1 < H->nlev; ++l) {
    const Level& f = H->lev[l];
    Level& c = H->lev[l + 1];
    for (int e = 0; e < be; ++e) {
      if (cfg->interp == SMG_INTERP_CELL)
        SCHK(launch_rap_cc(f.S, f.cmask, f.g, f.A64 + (long)e * f.N, (long)be * f.N, c.A64 + (long)e * c.N,
                           (long)be * c.N, st));
      else if (cfg->interp == SMG_INTERP_CELL_TRILINEAR)
        SCHK(launch_rap_c64(f.S, f.cmask, f.g, f.A64 + (long)e * f.N, (long)be * f.N, c.A64 + (long)e * c.N,
                            (long)be * c.N, st));
      else if (cfg->interp == SMG_INTERP_OPERATOR) {
        SCHK(launch_od_weights(f.S, f.g, f.cmask, f.A64, f.W64, H->err, st));
        SCHK(launch_rap_od(f.S, f.cmask, f.g, f.A64, f.W64, c.A64, st));
      }
      else
        SCHK(launch_rap(f.S, f.cmask, f.g, f.A64 + (long)e * f.N, (long)be * f.N, c.A64 + (long)e * c.N,
                        (long)be * c.N, st));
    }
  }
  // smoother data, truncation, wavefront tiling and sentinel fills
  hipStream_t side[SETUP_SIDE] = {st, st, st};
  SideJoin join;
  const bool par = H->side_ok && H->nlev >= 3 && H->lev[0].N >= SETUP_SIDE_POINTS;
  if (par) {
    SCHK(side_streams(side));
    join.side = side;
    SCHK(hipEventCreateWithFlags(&join.ev[SETUP_SIDE], hipEventDisableTiming));
    SCHK(hipEventRecord(join.ev[SETUP_SIDE], st));
    for (int k = 0; k < SETUP_SIDE; ++k) {
      SCHK(hipEventCreateWithFlags(&join.ev[k], hipEventDisableTiming));
      SCHK(hipStreamWaitEvent(side[k], join.ev[SETUP_SIDE], 0));
    }
  }
  const hipStream_t st0 = st;
  for (int l = 0; l + 1 < H->nlev; ++l) {
    Level& v = H->lev[l];
    const hipStream_t st = side[l < SETUP_SIDE ? l : SETUP_SIDE - 1];
    if (bs == 3)
      SCHK(launch_block_dinv(v.g, v.A64, v.rd64, H->err, st));
    else
      SCHK(launch_recip_diag(v.S, v.g, v.A64, cfg_weight(*cfg), v.rd64, H->err, st));
    if (v.qa) {
      const double w = cfg_weight(*cfg), q = (1.0 - w) / w;
      if (cfg->prec == SMG_FP64)
        SCHK(launch_centre_scaled<double>(v.S, v.g, v.A64, q, (double*)v.qa, st));
      else
        SCHK(launch_centre_scaled<float>(v.S, v.g, v.A64, q, (float*)v.qa, st));
    }
    if (v.uz) {
      if (cfg->prec == SMG_FP64)
        SCHK(launch_fill_bits<double>((double*)v.uz, v.N * bs, 0.0, st));
      else
        SCHK(launch_fill_bits<float>((float*)v.uz, v.N * bs, 0.0f, st));
    }
    if (cfg->smoother == SMG_SMOOTH_ILU0)
      SCHK(launch_ilu0_factor(v.S, v.Ssw, v.g, v.A64, v.L64, v.U64, v.rU64, H->err, st));
    if (v.W32) SCHK(launch_to_f32(v.W64, v.W32, 8 * v.N, st));
    if (cfg->smoother == SMG_SMOOTH_LGS) {
      std::vector<int> tiles;
      int kside = 0;
      lgs_plan(v.g, v.S, &kside, &tiles);
      SCHK(hipMemcpy(v.lg_map, tiles.data(), sizeof(int) * tiles.size(), hipMemcpyHostToDevice));
      SCHK(launch_tri_factor(v.S, v.g, v.A64, v.tr64, v.tc64, H->err, st));
      if (cfg->prec == SMG_FP32) {
        SCHK(launch_to_f32(v.tr64, v.tr32, v.N, st));
        SCHK(launch_to_f32(v.tc64, v.tc32, v.N, st));
      }
    }
    const long na = (long)v.S * be * v.N;
    if (cfg->prec == SMG_FP32) {
      SCHK(launch_to_f32(v.A64, v.A32, na, st));
      SCHK(launch_to_f32(v.rd64, v.rd32, (bs == 3 ? 9 : 1) * v.N, st));
      if (cfg->smoother == SMG_SMOOTH_ILU0) {
        SCHK(launch_to_f32(v.L64, v.L32, (long)v.Ssw * v.N, st));
        SCHK(launch_to_f32(v.U64, v.U32, (long)v.Ssw * v.N, st));
        SCHK(launch_to_f32(v.rU64, v.rU32, v.N, st));
      }
    } else if (cfg->prec == SMG_FP16_ROWSCALE) {
      SCHK(launch_to_f16_rowscale(v.A64, v.N, v.S, bs, v.A16, v.sc16, st));
      SCHK(launch_to_f32(v.rd64, v.rd32, (bs == 3 ? 9 : 1) * v.N, st));
    }
    // sweep data in wavefront schedule order
    if (bs == 3) {
      for (int d = 0; d < 2; ++d) {
        const int dir = d == 0 ? 1 : -1;
        if (cfg->prec == SMG_FP64)
          SCHK(launch_bwf_pack<double>(v.g, v.tl, dir, v.A64, v.rd64, (double*)v.pk[d], st));
        else if (cfg->prec == SMG_FP32)
          SCHK(launch_bwf_pack<float>(v.g, v.tl, dir, v.A64, v.rd64, (float*)v.pk[d], st));
        else
          SCHK(launch_bwf_pack_h(v.g, v.tl, dir, v.A16, v.sc16, v.rd32, v.pk[d], st));
      }
    }
    if (bs == 1 && cfg->smoother != SMG_SMOOTH_LGS) {
      SCHK(pack_sweep_data(H, v, st));
      if (v.hp_steps > 0) {
        std::vector<int> pts;
        hp_plan(v.g, v.S, cfg->prec == SMG_FP64 ? 8 : 4, &pts);
        SCHK(hipMemcpy(v.hp_pts, pts.data(), sizeof(int) * pts.size(), hipMemcpyHostToDevice));
        const int src = cfg->prec == SMG_FP64 ? 0 : (cfg->prec == SMG_FP32 ? 1 : 2);
        for (int d = 0; d < 2; ++d)
          SCHK(launch_hp_pack(v.S, src, v.g, v.hp_steps, d == 0 ? 1 : -1, v.hp_pts, v.A64, v.rd64, v.A16, v.sc16,
                              v.rd32, v.hp_cf[d], st));
      }
    }
    SCHK(fill_sentinels(H, v, st));
  }
  // coarsest: dense FP64 inverse
  {
    const Level& c = H->lev[H->nlev - 1];
    SCHK(launch_aug_init(H->nc, H->aug, st0));
    SCHK(launch_dense_assemble(c.g, c.S, bs, c.A64, H->aug, 2 * H->nc, st0));
    SCHK(coarse_invert(H->nc, H->aug, H->info, st0));
  }
  if (par) {
    for (int k = 0; k < SETUP_SIDE; ++k) {
      SCHK(hipEventRecord(join.ev[k], side[k]));
      SCHK(hipStreamWaitEvent(st0, join.ev[k], 0));
    }
    join.joined = true;
  }
  SCHK(hipStreamSynchronize(st));
  unsigned errv = 0;
  int infov = 0;
  SCHK(hipMemcpy(&errv, H->err, sizeof errv, hipMemcpyDeviceToHost));
  SCHK(hipMemcpy(&infov, H->info, sizeof infov, hipMemcpyDeviceToHost));
  if (errv & 2u) return fail(H, SMG_EBREAKDOWN, "zero diagonal or zero ILU pivot during setup");
  if (infov) return fail(H, SMG_EBREAKDOWN, "singular coarsest operator");
#undef SCHK
  return SMG_OK;
}

}  // namespace

namespace smg {
// Re-tiles level l of a handle (shape 0 default, 1 sheared, 2 rectangular)
// and rebuilds what depends on the tiling: the packed sweep data of both
// directions and the sentinel state of the level's buffers.  The captured
// V-cycle graph is dropped (its launches carry the old tiling).  *why names
// the reason of a refusal.
hipError_t retile_level(smg_handle_s* H, int l, int shape, hipStream_t st, const char** why) {
  *why = nullptr;
  if (l < 0 || l >= H->nlev - 1) {
    *why = "the level has no smoothing sweep";
    return hipErrorInvalidValue;
  }
  if (shape < 0 || shape > 2) {
    *why = "tile shape must be 0 (default), 1 (sheared) or 2 (rectangular)";
    return hipErrorInvalidValue;
  }
  if (H->bs != 1 || H->cfg.smoother == SMG_SMOOTH_LGS) {
    *why = "tile shapes apply to the point GS and ILU(0) sweeps of scalar systems";
    return hipErrorInvalidValue;
  }
  Level& v = H->lev[l];
  WfTiling t;
  wf_tiling(v.g, v.Ssw, &t, shape);
  if (t.sh == 0 && v.Ssw != 7 && t.nty > 1) {
    *why = "rectangular tiles of a 19/27-point sweep need a single tile row (ny <= 16)";
    return hipErrorInvalidValue;
  }
  const int vb = H->cfg.prec == SMG_FP64 ? 8 : 4, eb = H->cfg.prec == SMG_FP16_ROWSCALE ? 2 : vb;
  if (t.nsk > v.nsk_cap || !wf_ranges_ok(v.g, t, v.Ssw, vb, eb)) {
    *why = "the tiling does not fit the level's sweep buffers";
    return hipErrorInvalidValue;
  }
  if (t.sh == v.tl.sh) return hipSuccess;
  v.tl = t;
  hipError_t e = pack_sweep_data(H, v, st);
  if (e == hipSuccess) e = fill_sentinels(H, v, st);
  drop_vgraph(H);
  return e;
}
}  // namespace smg

namespace {

}  // namespace

extern "C" {

// Workspace bytes of cfg; with automatic coarsening the largest over the
// possible numbers of leading x,y-only levels.
size_t plan_bytes(const smg_config& cfg, int* nlev, int* nc) {
  if (cfg.coarsen != SMG_COARSEN_AUTO) return plan(cfg, nullptr, nullptr, nlev, nc);
  size_t best = 0;
  for (int s = MAXLEV; s >= 0; --s) {
    smg_config e = cfg;
    e.coarsen = SMG_COARSEN_FULL;
    e.semi_levels = s;
    int nl = 0, ncc = 0;
    const size_t b = plan(e, nullptr, nullptr, &nl, &ncc);
    if (b > best || s == MAXLEV) {
      *nlev = nl;
      *nc = ncc;
    }
    if (b > best) best = b;
  }
  return best;
}

// Leading x,y-only levels of the automatic coarsening for the finest
// coefficients: rho = sum |z couplings| / mean(sum |x couplings|, sum |y
// couplings|); level l coarsens x,y only while rho * 4^l < 1/4.  part holds
// 3 * AXIS_BLOCKS doubles of device scratch.  Synchronises st.
hipError_t auto_semi_levels(const smg_config& cfg, const double* coeffs, double* part, hipStream_t st, int* out) {
  const Grid g{cfg.nx, cfg.ny, cfg.nz};
  hipError_t e = launch_axis_coupling(cfg.pattern, g, coeffs, part, st);
  std::vector<double> h(3 * AXIS_BLOCKS);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int b = 0; b < AXIS_BLOCKS; ++b) {
    sx += h[3 * b];
    sy += h[3 * b + 1];
    sz += h[3 * b + 2];
  }
  const double sxy = 0.5 * (sx + sy);
  int s = 0;
  if (sxy > 0.0)
    for (double r = sz / sxy; s < MAXLEV && r < 0.25; r *= 4.0) ++s;
  *out = s;
  return hipSuccess;
}

smg_status smg_workspace_size(const smg_config* cfg, size_t* bytes) {
  const char* why = check_cfg(cfg);
  if (why) return fail(nullptr, SMG_EINVAL, "%s", why);
  if (!bytes) return fail(nullptr, SMG_EINVAL, "null bytes pointer");
  int nlev = 0, nc = 0;
  size_t b = plan_bytes(*cfg, &nlev, &nc);
  if (b == 0) return fail(nullptr, SMG_EINVAL, "coarsest level has %d unknowns (> max_coarse)", nc);
  *bytes = b;
  return SMG_OK;
}

static smg_status setup_impl(const smg_config* cfg, const double* coeffs, void* workspace, size_t bytes,
                             void* stream, smg_handle* out, bool side_ok);

smg_status smg_setup(const smg_config* cfg, const double* coeffs, void* workspace, size_t bytes, void* stream,
                     smg_handle* out) {
  return setup_impl(cfg, coeffs, workspace, bytes, stream, out, true);
}

// side_ok: the setup may use the library's side streams (not for callers
// that cannot allocate)
static smg_status setup_impl(const smg_config* cfg, const double* coeffs, void* workspace, size_t bytes,
                             void* stream, smg_handle* out, bool side_ok) {
  if (!out) return fail(nullptr, SMG_EINVAL, "null output handle");
  *out = nullptr;
  const char* why = check_cfg(cfg);
  if (why) return fail(nullptr, SMG_EINVAL, "%s", why);
  if (!coeffs || !workspace) return fail(nullptr, SMG_EINVAL, "null coefficient or workspace pointer");
  int nlev = 0, nc = 0;
  const size_t need = plan_bytes(*cfg, &nlev, &nc);
  if (need == 0) return fail(nullptr, SMG_EINVAL, "coarsest level has %d unknowns (> max_coarse)", nc);
  if (bytes < need) return fail(nullptr, SMG_ENOMEM, "workspace of %zu bytes, %zu needed", bytes, need);
  hipStream_t st = (hipStream_t)stream;
  auto t0 = std::chrono::steady_clock::now();
  char* base = (char*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
  smg_config eff = *cfg;
  if (cfg->coarsen == SMG_COARSEN_AUTO) {
    // the rule needs the coefficients: the workspace serves as scratch first
    int s = 0;
    const hipError_t e = auto_semi_levels(*cfg, coeffs, (double*)base, st, &s);
    if (e != hipSuccess) return fail(nullptr, SMG_EDEVICE, "automatic coarsening: %s", hipGetErrorString(e));
    eff.coarsen = SMG_COARSEN_FULL;
    eff.semi_levels = s;
    if (plan(eff, nullptr, nullptr, &nlev, &nc) == 0)
      return fail(nullptr, SMG_EINVAL, "automatic coarsening (%d x,y levels): coarsest level has %d unknowns "
                  "(> max_coarse)", s, nc);
  }
  smg_handle_s* H = new smg_handle_s();
  H->cfg = eff;
  H->bs = cfg->block;
  H->side_ok = side_ok;
  plan(eff, H, base, &H->nlev, &H->nc);
  auto bail = [&](smg_status s) {
    if (s != SMG_OK) {
      snprintf(g_setup_msg, sizeof g_setup_msg, "%s", H->msg);
      delete H;
    }
    return s;
  };
  {
    smg_status bs_ = build_hierarchy(H, coeffs, st);
    if (bs_ != SMG_OK) return bail(bs_);
  }
  H->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = H;
  return SMG_OK;
}

// ---- setup into a static device array (callers that cannot allocate) ----
// The hierarchy of smg_setup_noalloc lives in `scratch`, a file-scope device
// array (each GPU the library runs on holds its own copy until the process
// ends).  Host code never passes the array's name to a kernel or copy: its
// device address is taken once per device with hipGetSymbolAddress and kept
// in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[SMG_SCRATCH_BYTES];
constexpr int SMG_SCRATCH_DEVICES = 64;
static void* g_scratch_ptr[SMG_SCRATCH_DEVICES];
static std::mutex g_scratch_mu;

static smg_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, SMG_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= SMG_SCRATCH_DEVICES)
    return fail(nullptr, SMG_EDEVICE, "device %d beyond the %d devices the scratch table holds", dev,
                SMG_SCRATCH_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(nullptr, SMG_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SMG_OK;
}

smg_status smg_setup_noalloc(const smg_config* cfg, const double* coeffs, void* stream, smg_handle* out) {
  if (!out) return fail(nullptr, SMG_EINVAL, "null output handle");
  *out = nullptr;
  const char* why = check_cfg(cfg);
  if (why) return fail(nullptr, SMG_EINVAL, "%s", why);
  int nlev = 0, nc = 0;
  const size_t need = plan_bytes(*cfg, &nlev, &nc);
  if (need == 0) return fail(nullptr, SMG_EINVAL, "coarsest level has %d unknowns (> max_coarse)", nc);
  if (need > SMG_SCRATCH_BYTES)
    return fail(nullptr, SMG_ENOMEM,
                "hierarchy needs %zu bytes; the static scratch array holds %zu (use smg_setup with a workspace)", need,
                (size_t)SMG_SCRATCH_BYTES);
  void* p = nullptr;
  const smg_status s = scratch_address(&p);
  if (s != SMG_OK) return s;
  return setup_impl(cfg, coeffs, p, SMG_SCRATCH_BYTES, stream, out, false);
}

smg_status smg_resetup(smg_handle h, const double* coeffs, void* stream) {
  if (!h) return fail(nullptr, SMG_EINVAL, "null handle");
  if (!coeffs) return fail(h, SMG_EINVAL, "null coefficient pointer");
  auto t0 = std::chrono::steady_clock::now();
  smg_status s = build_hierarchy(h, coeffs, (hipStream_t)stream);
  if (s != SMG_OK) return s;
  h->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return SMG_OK;
}

smg_status smg_precondition(smg_handle h, const double* r, double* z, void* stream) {
  if (!h) return fail(nullptr, SMG_EINVAL, "null handle");
  if (!r || !z) return fail(h, SMG_EINVAL, "null vector");
  const long n0 = h->lev[0].N * h->bs;
  if ((const char*)z < (const char*)(r + n0) && (const char*)r < (const char*)(z + n0))
    return fail(h, SMG_EINVAL, "r and z overlap");
  HIPCHK(h, vcycle(h, r, z, (hipStream_t)stream));
  return SMG_OK;
}

smg_status smg_solve(smg_handle H, const double* b, double* x, double rtol, int maxit, int krylov, smg_result* res,
                     void* stream) {
  if (!H) return fail(nullptr, SMG_EINVAL, "null handle");
  if (!b || !x) return fail(H, SMG_EINVAL, "null vector");
  if (!(rtol > 0.0) || maxit < 0 || krylov < 0) return fail(H, SMG_EINVAL, "bad rtol / maxit / krylov");
  if (krylov > 0 && krylov > H->kV_m) return fail(H, SMG_EINVAL, "GMRES(%d) needs cfg.gmres_restart >= %d", krylov, krylov);
  hipStream_t st = (hipStream_t)stream;
  const long n = H->lev[0].N * H->bs;
  hipError_t e = hipSuccess;
  auto t0 = std::chrono::steady_clock::now();
#define KCHK(expr)                                                                       \
  do {                                                                                   \
    e = (expr);                                                                          \
    if (e != hipSuccess) return fail(H, SMG_EDEVICE, "%s: %s", #expr, hipGetErrorString(e)); \
  } while (0)
  int waits = 0;  // host waits for the device (reported in the result)
#define KDOT(a, b_) (++waits, dot(H, a, b_, n, st, &e))
  double *r = H->kr, *z = H->kz, *p = H->kp, *q = H->kq;
  double bn = sqrt(KDOT(b, b));
  KCHK(e);
  if (bn == 0.0) bn = 1.0;
  KCHK(spmv64(H, x, b, r, true, st));
  double rel = sqrt(KDOT(r, r)) / bn;
  KCHK(e);
  int it = 0;
  double recur = rel;  // the method's own residual estimate
  smg_status status = SMG_ENOTCONV;
  if (rel < rtol) status = SMG_OK;
  if (krylov == 0 && status != SMG_OK) {
    // PCG with its scalars on the device (rho, p.q, r.r, r.z, alpha, beta and
    // the convergence tests of the host formulation, in the same order and
    // arithmetic, so the iterates are the same).  The host enqueues several
    // iterations between reads of the state: as many as the recurrence
    // residual's recent rate predicts before convergence (one at a time near
    // it); an iteration enqueued after convergence changes nothing (its
    // vector updates are skipped on the device).
    double* sc = H->dout;
    KCHK(vcycle_solver(H, st));
    KCHK(hipMemcpyAsync(p, z, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    KCHK(launch_dot(n, r, z, H->dpart, sc + PS_RHO, st));
    KCHK(launch_pcg_start(sc, bn, it, maxit, rtol, st));
    double hs[PS_END];
    double rel_prev = rel;
    int it_prev = it, batch = 1;
    // first half of an iteration: q = A p, alpha, the updates of x and r and
    // the convergence tests; second half: the V-cycle, beta and p
    auto first_half = [&]() -> hipError_t {
      hipError_t e2 = spmv64(H, p, nullptr, q, false, st);
      if (e2 == hipSuccess) e2 = launch_dot(n, p, q, H->dpart, sc + PS_PQ, st);
      if (e2 == hipSuccess) e2 = launch_pcg_alpha(sc, st);
      if (e2 == hipSuccess) e2 = launch_pcg_update(n, sc, p, q, x, r, H->dpart, sc + PS_RR, st);
      if (e2 == hipSuccess) e2 = launch_pcg_recur(sc, st);
      // the true residual where the recurrence residual is below tolerance
      const Level& l0 = H->lev[0];
      if (e2 == hipSuccess)
        e2 = H->bs == 3 ? launch_bspmv_res_gated(l0.g, BMatD{l0.A64, l0.N}, x, b, r, sc + PS_GATE, st)
                        : launch_spmv_res_gated(l0.S, l0.g, MatD{l0.A64, l0.N}, x, b, r, sc + PS_GATE, st);
      if (e2 == hipSuccess) e2 = launch_dot_gated(n, r, r, H->dpart, sc + PS_RR, sc + PS_GATE, st);
      if (e2 == hipSuccess) e2 = launch_pcg_true(sc, st);
      return e2;
    };
    auto second_half = [&]() -> hipError_t {
      hipError_t e2 = vcycle_solver(H, st);
      if (e2 == hipSuccess) e2 = launch_dot(n, r, z, H->dpart, sc + PS_RZ, st);
      if (e2 == hipSuccess) e2 = launch_pcg_beta(sc, st);
      if (e2 == hipSuccess) e2 = launch_xpby_dev(n, z, sc + PS_BETA, sc + PS_STATE, p, st);
      return e2;
    };
    for (;;) {
      // the state is read after the last iteration's tests, before its
      // V-cycle, so no V-cycle runs after convergence is seen
      for (int k = 0; k < batch; ++k) {
        KCHK(first_half());
        if (k + 1 < batch) KCHK(second_half());
      }
      KCHK(hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, st));
      KCHK(hipStreamSynchronize(st));
      ++waits;
      it = (int)hs[PS_IT];
      if (it > it_prev) {
        recur = hs[PS_RECUR];
        rel = hs[PS_REL];
      }
      const double state = hs[PS_STATE];
      if (state == PCG_DONE) {
        status = SMG_OK;
        break;
      }
      if (state == PCG_BREAKDOWN) {
        status = SMG_EBREAKDOWN;
        fail(H, SMG_EBREAKDOWN, "p.Ap = %g <= 0", hs[PS_PQ]);
        break;
      }
      if (state == PCG_LIMIT || it >= maxit) break;
      KCHK(second_half());
      // iterations to enqueue next: one fewer than the recurrence's rate
      // over the last batch predicts to reach the tolerance, 1 to 8
      batch = 1;
      if (it > it_prev && recur < rel_prev && recur > 0.0) {
        const double rate = log(recur / rel_prev) / (it - it_prev);
        const double need = log(rtol / recur) / rate;
        if (need > 2.0) batch = need > 9.0 ? 8 : (int)need - 1;
      }
      if (batch > maxit - it) batch = maxit - it;
      rel_prev = recur;
      it_prev = it;
    }
  } else if (status != SMG_OK) {
    // right-preconditioned GMRES(m) in its flexible form: the preconditioned
    // basis vectors z_j = M v_j are kept (Z) and the update is x += Z y, so
    // no further V-cycle runs per cycle and the recurrence residual stays
    // the true one when M is not exactly linear (V-cycle in FP32 / FP16);
    // modified Gram-Schmidt, Givens rotations
    const int m = krylov;
    double* V = H->kV;
    double* Z = H->kZ;
    double *w = H->kw, *t = H->kt;
    double Hm[201 * 200];
    double cs[200], sn[200], g[201], y[200];
    double beta = rel * bn;
    while (status != SMG_OK && it < maxit) {
      KCHK(launch_scale(n, 1.0 / beta, r, V, st));
      for (int k = 0; k <= m; ++k) g[k] = 0.0;
      g[0] = beta;
      int jdone = 0;
      for (int j = 0; j < m && it < maxit; ++j) {
        double* vj = V + (long)j * n;
        double* vn = V + (long)(j + 1) * n;
        double* zj = Z + (long)j * n;
        KCHK(vcycle(H, vj, zj, st));
        KCHK(spmv64(H, zj, nullptr, w, false, st));
        for (int i = 0; i <= j; ++i) {
          double* vi = V + (long)i * n;
          const double hij = KDOT(w, vi);
          KCHK(e);
          Hm[i * m + j] = hij;
          KCHK(launch_axpy(n, -hij, vi, w, st));
        }
        const double hn = sqrt(KDOT(w, w));
        KCHK(e);
        Hm[(j + 1) * m + j] = hn;
        if (hn != 0.0) KCHK(launch_scale(n, 1.0 / hn, w, vn, st));
        for (int i = 0; i < j; ++i) {
          const double a = Hm[i * m + j], bb = Hm[(i + 1) * m + j];
          Hm[i * m + j] = cs[i] * a + sn[i] * bb;
          Hm[(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
        }
        const double a = Hm[j * m + j], bb = Hm[(j + 1) * m + j];
        const double den = sqrt(a * a + bb * bb);
        cs[j] = den == 0.0 ? 1.0 : a / den;
        sn[j] = den == 0.0 ? 0.0 : bb / den;
        Hm[j * m + j] = den;
        Hm[(j + 1) * m + j] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++it;
        jdone = j + 1;
        recur = fabs(g[j + 1]) / bn;
        if (recur < rtol || hn == 0.0) break;
      }
      for (int i = jdone - 1; i >= 0; --i) {
        double s = g[i];
        for (int k = i + 1; k < jdone; ++k) s -= Hm[i * m + k] * y[k];
        y[i] = s / Hm[i * m + i];
      }
      for (int i = 0; i < jdone; ++i) KCHK(launch_axpy(n, y[i], Z + (long)i * n, x, st));
      KCHK(spmv64(H, x, b, r, true, st));
      beta = sqrt(KDOT(r, r));
      KCHK(e);
      rel = beta / bn;
      if (rel < rtol) status = SMG_OK;
    }
  }
  // final true residual in FP64
  KCHK(spmv64(H, x, b, r, true, st));
  rel = sqrt(KDOT(r, r)) / bn;
  KCHK(e);
  smg_status es = check_err(H, st);
  ++waits;
  if (es != SMG_OK) return es;
#undef KDOT
#undef KCHK
  if (res) {
    res->iters = it;
    res->levels = H->nlev;
    res->rel_resid_true = rel;
    res->rel_resid_recur = recur;
    res->host_waits = waits;
    double sn0 = 0, sn = 0, so0 = 0, so = 0;
    for (int l = 0; l < H->nlev; ++l) {
      sn += (double)H->lev[l].N;
      so += (double)H->lev[l].N * H->lev[l].S;
    }
    sn0 = (double)H->lev[0].N;
    so0 = (double)H->lev[0].N * H->lev[0].S;
    res->grid_complexity = sn / sn0;
    res->op_complexity = so / so0;
    res->t_setup_ms = H->t_setup_ms;
    res->t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (status == SMG_ENOTCONV) fail(H, SMG_ENOTCONV, "not converged after %d iterations (rel %g)", it, rel);
  return status;
}

smg_status smg_set_timing(smg_handle h, int enable, int level, unsigned kinds);

smg_status smg_destroy(smg_handle h) {
  if (h && h->timing) smg_set_timing(h, 0, -1, 0);
  if (h) {
    drop_vgraph(h);
    if (h->cap) (void)hipStreamDestroy(h->cap);
  }
  delete h;
  return SMG_OK;
}

smg_status smg_set_graph(smg_handle h, int enable) {
  if (!h) return fail(nullptr, SMG_EINVAL, "null handle");
  h->use_graph = enable != 0;
  drop_vgraph(h);
  return SMG_OK;
}

smg_status smg_set_tile_shape(smg_handle h, int level, int shape, void* stream) {
  if (!h) return fail(nullptr, SMG_EINVAL, "null handle");
  const char* why = nullptr;
  const hipError_t e = retile_level(h, level, shape, (hipStream_t)stream, &why);
  if (why) return fail(h, SMG_EINVAL, "level %d: %s", level, why);
  HIPCHK(h, e);
  HIPCHK(h, hipStreamSynchronize((hipStream_t)stream));
  return SMG_OK;
}

int smg_tile_shape(smg_handle h, int level) {
  if (!h || level < 0 || level >= h->nlev - 1 || h->bs != 1 || h->cfg.smoother == SMG_SMOOTH_LGS) return 0;
  return h->lev[level].tl.sh ? 1 : 2;
}

const char* smg_last_error(smg_handle h) { return h ? h->msg : g_setup_msg; }

int smg_num_levels(smg_handle h) { return h ? h->nlev : 0; }

smg_status smg_level_info(smg_handle h, int level, int* info) {
  if (!h || !info) return fail(h, SMG_EINVAL, "null argument");
  if (level < 0 || level >= h->nlev) return fail(h, SMG_EINVAL, "level %d out of range", level);
  const Level& v = h->lev[level];
  info[0] = v.g.nx;
  info[1] = v.g.ny;
  info[2] = v.g.nz;
  info[3] = v.S;
  info[4] = v.cmask;
  info[5] = h->bs;
  return SMG_OK;
}

smg_status smg_level_export(smg_handle h, int level, int what, void* dst, void* stream) {
  if (!h || !dst) return fail(h, SMG_EINVAL, "null argument");
  if (level < 0 || level >= h->nlev) return fail(h, SMG_EINVAL, "level %d out of range", level);
  const Level& v = h->lev[level];
  hipStream_t st = (hipStream_t)stream;
  const long be = (long)h->bs * h->bs, nd = (h->bs == 3 ? 9 : 1) * v.N;
  const void* src = nullptr;
  size_t bytes = 0;
  const bool last = level == h->nlev - 1;
  switch (what) {
    case 0: src = v.A64; bytes = sizeof(double) * v.S * be * v.N; break;
    case 1: src = v.rd64; bytes = sizeof(double) * nd; break;
    case 2: src = v.L64; bytes = sizeof(double) * v.Ssw * v.N; break;
    case 3: src = v.U64; bytes = sizeof(double) * v.Ssw * v.N; break;
    case 4: src = v.rU64; bytes = sizeof(double) * v.N; break;
    case 5:
      if (last || h->cfg.prec == SMG_FP64) return fail(h, SMG_EINVAL, "no reduced-precision matrix on this level");
      if (h->cfg.prec == SMG_FP32) {
        src = v.A32;
        bytes = sizeof(float) * v.S * be * v.N;
        break;
      }
      HIPCHK(h, launch_dequant_f16(v.A16, v.sc16, v.N, v.S, h->bs, (float*)dst, st));
      return SMG_OK;
    case 6:
      if (last || h->cfg.prec == SMG_FP64) return fail(h, SMG_EINVAL, "no reduced-precision diagonal on this level");
      src = v.rd32;
      bytes = sizeof(float) * nd;
      break;
    case 7: src = v.tr64; bytes = sizeof(double) * v.N; break;
    case 8: src = v.tc64; bytes = sizeof(double) * v.N; break;
    case 9: src = v.W64; bytes = sizeof(double) * 8 * v.N; break;
    default: return fail(h, SMG_EINVAL, "unknown export %d", what);
  }
  if (!src) return fail(h, SMG_EINVAL, "level %d has no data %d", level, what);
  HIPCHK(h, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
  return SMG_OK;
}

int smg_rap_chain_count(int pattern, int cmask) { return rap_chain_count(pattern, cmask); }

}  // extern "C"

// ---- single-step entry points (C linkage from the header declarations) ---
static smg_status op_level_check(smg_handle h, int level, bool need_next) {
  if (!h) return fail(nullptr, SMG_EINVAL, "null handle");
  if (level < 0 || level >= h->nlev) return fail(h, SMG_EINVAL, "level %d out of range", level);
  if (need_next && level + 1 >= h->nlev) return fail(h, SMG_EINVAL, "level %d is the coarsest", level);
  return SMG_OK;
}

template <class PT>
static hipError_t op_presmooth_t(smg_handle_s* H, const Level& v, const void* f, void* u, hipStream_t st) {
  using V = typename PT::V;
  V sent;
  if (sizeof(V) == 8) {
    uint64_t b = SENT64;
    memcpy(&sent, &b, 8);
  } else {
    uint32_t b = SENT32;
    memcpy(&sent, &b, 4);
  }
  const long nv = v.N * H->bs;
  hipError_t e;
  if (H->bs == 3) {
    e = launch_fill_bits<V>((V*)u, nv, sent, st);
    if (e == hipSuccess) e = bsweep<typename PT::E, V>(H, v, +1, (const V*)f, (V*)u, nullptr, 0, st);
    return e;
  }
  if (H->cfg.smoother == SMG_SMOOTH_GS) {
    e = launch_fill_bits<V>((V*)u, nv, sent, st);
    if (e == hipSuccess)
      e = sweep<typename PT::E, V>(H, v, +1, false, (const V*)f, (V*)u, nullptr, 0, nullptr, nullptr, st);
    return e;
  }
  if (H->cfg.smoother == SMG_SMOOTH_LGS) {
    e = launch_fill_bits<V>((V*)u, nv, sent, st);
    if (e == hipSuccess) e = lgs_sweep<PT>(H, v, +1, (const V*)f, nullptr, (V*)u, nullptr, st);
    return e;
  }
  e = launch_fill_bits<V>((V*)v.h, nv, sent, st);
  if (e == hipSuccess) e = launch_fill_bits<V>((V*)u, nv, sent, st);
  if (e == hipSuccess)
    e = sweep<typename PT::E, V>(H, v, +1, true, (const V*)f, (V*)v.h, nullptr, 0, nullptr, nullptr, st);
  if (e == hipSuccess)
    e = sweep<typename PT::E, V>(H, v, -1, false, (const V*)v.h, (V*)u, nullptr, 0, nullptr, nullptr, st);
  return e;
}

template <class PT>
static hipError_t op_postsmooth_t(smg_handle_s* H, const Level& v, const void* f, const void* uin, const void* ec,
                                  void* uout, hipStream_t st) {
  using V = typename PT::V;
  V sent;
  if (sizeof(V) == 8) {
    uint64_t b = SENT64;
    memcpy(&sent, &b, 8);
  } else {
    uint32_t b = SENT32;
    memcpy(&sent, &b, 4);
  }
  const long nv = v.N * H->bs;
  const auto A = PT::A(v);
  hipError_t e;
  if (H->bs == 3) {
    // u_old = u_in + P ec in the level's u_a buffer (its sentinels restored after)
    e = hipMemcpyAsync(v.ua, uin, sizeof(V) * nv, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && ec != nullptr) e = launch_prolong_add<V>(v.g, v.cmask, 3, (const V*)ec, (V*)v.ua, st);
    if (e == hipSuccess) e = launch_blower(v.g, PT::BA(v), (const V*)f, (const V*)v.ua, (V*)v.h, st);
    if (e == hipSuccess) e = launch_fill_bits<V>((V*)uout, nv, sent, st);
    if (e == hipSuccess) e = bsweep<typename PT::E, V>(H, v, -1, (const V*)v.h, (V*)uout, nullptr, 0, st);
    if (e == hipSuccess) e = launch_fill_bits<V>((V*)v.ua, nv, sent, st);
    return e;
  }
  if (H->cfg.smoother == SMG_SMOOTH_LGS) {
    // u_old = u_in + P ec in the level's u_a buffer, then the backward line GS
    // sweep, which gives u_a its sentinels back
    e = hipMemcpyAsync(v.ua, uin, sizeof(V) * nv, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && ec != nullptr) e = prolong_in_place<V>(H, v, (const V*)ec, (V*)v.ua, st);
    if (e == hipSuccess) e = launch_fill_bits<V>((V*)uout, nv, sent, st);
    if (e == hipSuccess) e = lgs_sweep<PT>(H, v, -1, (const V*)f, (const V*)v.ua, (V*)uout, (V*)v.ua, st);
    return e;
  }
  if (H->cfg.smoother == SMG_SMOOTH_GS) {
    // the V-cycle's kernels for this level: h = f - lower(A) u_old with
    // u_old = u_in + P ec (large levels: formed in u_a, whose sentinels are
    // restored after)
    if (split_rp(v) || H->cfg.interp != SMG_INTERP_VERTEX || v.qa) {
      e = hipMemcpyAsync(v.ua, uin, sizeof(V) * nv, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess && ec != nullptr) e = prolong_in_place<V>(H, v, (const V*)ec, (V*)v.ua, st);
      if (e == hipSuccess) e = old_terms<PT>(H, v, -1, (const V*)f, (const V*)v.ua, (V*)v.h, st);
      if (e == hipSuccess) e = launch_fill_bits<V>((V*)v.ua, nv, sent, st);
    } else {
      e = launch_prolong_post(v.S, v.g, v.cmask, A, (const V*)f, (const V*)uin, (const V*)ec, (V*)v.h,
                              (V*)nullptr, false, st);
    }
    if (e == hipSuccess) e = launch_fill_bits<V>((V*)uout, nv, sent, st);
    if (e == hipSuccess)
      e = sweep<typename PT::E, V>(H, v, -1, false, (const V*)v.h, (V*)uout, nullptr, 0, nullptr, nullptr, st);
    return e;
  }
  // ILU correction: r = f - A u_old; u_out = u_old + U^-1 L^-1 r.  Scratch: the
  // level's y1/y2/zz buffers, whose sentinel state is restored afterwards.
  if (H->cfg.interp != SMG_INTERP_VERTEX) {
    e = ec ? prolong_cell<V>(H, v, (const V*)ec, (const V*)uin, (V*)v.uo, st)
           : hipMemcpyAsync(v.uo, uin, sizeof(V) * nv, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = launch_spmv(v.S, v.g, A, (const V*)v.uo, (const V*)f, (V*)v.h, true, st);
  } else {
    e = launch_prolong_post(v.S, v.g, v.cmask, A, (const V*)f, (const V*)uin, (const V*)ec, (V*)v.h, (V*)v.uo,
                            true, st);
  }
  if (e == hipSuccess) e = launch_fill_bits<V>((V*)v.y2, nv, sent, st);
  if (e == hipSuccess) e = launch_fill_bits<V>((V*)v.zz, nv, sent, st);
  if (e == hipSuccess)
    e = sweep<typename PT::E, V>(H, v, +1, true, (const V*)v.h, (V*)v.y2, nullptr, 0, nullptr, nullptr, st);
  if (e == hipSuccess)
    e = sweep<typename PT::E, V>(H, v, -1, false, (const V*)v.y2, (V*)v.zz, nullptr, 0, (const V*)v.uo, (V*)uout, st);
  if (e == hipSuccess) e = launch_fill_bits<V>((V*)v.y2, nv, sent, st);
  if (e == hipSuccess) e = launch_fill_bits<V>((V*)v.zz, nv, sent, st);
  return e;
}

template <template <class> class OP, class... Args>
static hipError_t by_prec(smg_handle_s* H, Args... args) {
  switch (H->cfg.prec) {
    case SMG_FP64: return OP<P64>::run(H, args...);
    case SMG_FP32: return OP<P32>::run(H, args...);
    default: return OP<P16>::run(H, args...);
  }
}

template <class PT>
struct OpSpmv {
  static hipError_t run(smg_handle_s* H, int l, const void* x, void* y, hipStream_t st) {
    const Level& v = H->lev[l];
    using V = typename PT::V;
    if (l == H->nlev - 1 && H->cfg.prec != SMG_FP64) return hipErrorInvalidValue;
    if (H->bs == 3) {
      if (l == H->nlev - 1 || H->cfg.prec == SMG_FP64)
        return launch_bspmv(v.g, BMatD{v.A64, v.N}, (const double*)x, (const double*)nullptr, (double*)y, false, st);
      return launch_bspmv(v.g, PT::BA(v), (const V*)x, (const V*)nullptr, (V*)y, false, st);
    }
    if (l == H->nlev - 1 || H->cfg.prec == SMG_FP64)
      return launch_spmv(v.S, v.g, MatD{v.A64, v.N}, (const double*)x, nullptr, (double*)y, false, st);
    return launch_spmv(v.S, v.g, PT::A(v), (const V*)x, (const V*)nullptr, (V*)y, false, st);
  }
};
template <class PT>
struct OpPre {
  static hipError_t run(smg_handle_s* H, int l, const void* f, void* u, hipStream_t st) {
    return op_presmooth_t<PT>(H, H->lev[l], f, u, st);
  }
};
template <class PT>
struct OpPost {
  static hipError_t run(smg_handle_s* H, int l, const void* f, const void* ui, const void* ec, void* uo,
                        hipStream_t st) {
    return op_postsmooth_t<PT>(H, H->lev[l], f, ui, ec, uo, st);
  }
};
template <class PT>
struct OpRR {
  static hipError_t run(smg_handle_s* H, int l, const void* f, const void* u, void* rc, hipStream_t st) {
    const Level& v = H->lev[l];
    using V = typename PT::V;
    if (H->bs == 3) {
      hipError_t e = launch_bspmv(v.g, PT::BA(v), (const V*)u, (const V*)f, (V*)v.h, true, st);
      if (e == hipSuccess) e = launch_restrict<V>(v.g, v.cmask, 3, (const V*)v.h, (V*)rc, st);
      return e;
    }
    if (!split_rp(v) && H->cfg.interp == SMG_INTERP_VERTEX)
      return launch_resid_restrict(v.S, v.g, v.cmask, PT::A(v), (const V*)f, (const V*)u, (V*)rc, st);
    hipError_t e = launch_spmv(v.S, v.g, PT::A(v), (const V*)u, (const V*)f, (V*)v.h, true, st);
    if (e == hipSuccess)
      e = restrict_any<V>(H, v, (const V*)v.h, (V*)rc, st);
    return e;
  }
};

smg_status smg_op_spmv(smg_handle h, int level, const void* x, void* y, void* stream) {
  smg_status s = op_level_check(h, level, false);
  if (s != SMG_OK) return s;
  if (!x || !y) return fail(h, SMG_EINVAL, "null vector");
  if (level == h->nlev - 1 && h->cfg.prec != SMG_FP64)
    return fail(h, SMG_EINVAL, "the coarsest level is kept in FP64 only");
  HIPCHK(h, (by_prec<OpSpmv>(h, level, x, y, (hipStream_t)stream)));
  return SMG_OK;
}

smg_status smg_op_spmv_fp64(smg_handle h, const double* x, double* y, void* stream) {
  if (!h || !x || !y) return fail(h, SMG_EINVAL, "null argument");
  HIPCHK(h, spmv64(h, x, nullptr, y, false, (hipStream_t)stream));
  return SMG_OK;
}

smg_status smg_op_presmooth(smg_handle h, int level, const void* f, void* u, void* stream) {
  smg_status s = op_level_check(h, level, true);
  if (s != SMG_OK) return s;
  if (!f || !u || f == u) return fail(h, SMG_EINVAL, "null or aliased vectors");
  HIPCHK(h, (by_prec<OpPre>(h, level, f, u, (hipStream_t)stream)));
  return check_err(h, (hipStream_t)stream);
}

smg_status smg_op_postsmooth(smg_handle h, int level, const void* f, const void* u_in, const void* ec, void* u_out,
                             void* stream) {
  smg_status s = op_level_check(h, level, true);
  if (s != SMG_OK) return s;
  if (!f || !u_in || !u_out || u_out == u_in || u_out == f) return fail(h, SMG_EINVAL, "null or aliased vectors");
  HIPCHK(h, (by_prec<OpPost>(h, level, f, u_in, ec, u_out, (hipStream_t)stream)));
  return check_err(h, (hipStream_t)stream);
}

smg_status smg_op_resid_restrict(smg_handle h, int level, const void* f, const void* u, void* rc, void* stream) {
  smg_status s = op_level_check(h, level, true);
  if (s != SMG_OK) return s;
  if (!f || !u || !rc) return fail(h, SMG_EINVAL, "null vector");
  HIPCHK(h, (by_prec<OpRR>(h, level, f, u, rc, (hipStream_t)stream)));
  return SMG_OK;
}

smg_status smg_op_restrict(smg_handle h, int level, const void* rf, void* rc, void* stream) {
  if (!h) return fail(nullptr, SMG_EINVAL, "null handle");
  if (level < 0 || level + 1 >= h->nlev) return fail(h, SMG_EINVAL, "level %d has no coarser level", level);
  if (!rf || !rc) return fail(h, SMG_EINVAL, "null vector");
  const Level& v = h->lev[level];
  const hipStream_t st = (hipStream_t)stream;
  if (h->cfg.prec == SMG_FP64)
    HIPCHK(h, restrict_any<double>(h, v, (const double*)rf, (double*)rc, st));
  else
    HIPCHK(h, restrict_any<float>(h, v, (const float*)rf, (float*)rc, st));
  return SMG_OK;
}

smg_status smg_op_prolong_add(smg_handle h, int level, const void* ec, void* uf, void* stream) {
  if (!h) return fail(nullptr, SMG_EINVAL, "null handle");
  if (level < 0 || level + 1 >= h->nlev) return fail(h, SMG_EINVAL, "level %d has no coarser level", level);
  if (!ec || !uf) return fail(h, SMG_EINVAL, "null vector");
  const Level& v = h->lev[level];
  if (h->cfg.prec == SMG_FP64)
    HIPCHK(h, prolong_in_place<double>(h, v, (const double*)ec, (double*)uf, (hipStream_t)stream));
  else
    HIPCHK(h, prolong_in_place<float>(h, v, (const float*)ec, (float*)uf, (hipStream_t)stream));
  return SMG_OK;
}

smg_status smg_op_coarse_solve(smg_handle h, const void* f, void* u, void* stream) {
  if (!h || !f || !u) return fail(h, SMG_EINVAL, "null argument");
  if (h->cfg.prec == SMG_FP64)
    HIPCHK(h, launch_coarse_gemv<double>(h->nc, h->aug + h->nc, 2 * h->nc, (const double*)f, (double*)u,
                                         (hipStream_t)stream));
  else
    HIPCHK(h, launch_coarse_gemv<float>(h->nc, h->aug + h->nc, 2 * h->nc, (const float*)f, (float*)u,
                                        (hipStream_t)stream));
  return SMG_OK;
}

smg_status smg_set_timing(smg_handle h, int enable, int level, unsigned kinds) {
  if (!h) return fail(nullptr, SMG_EINVAL, "null handle");
  h->tm_level = level;
  h->tm_kinds = kinds;
  if (enable && !h->timing) {
    for (int k = 0; k < SMG_TIMING_CAP; ++k) {
      HIPCHK(h, hipEventCreate(&h->ev0[k]));
      HIPCHK(h, hipEventCreate(&h->ev1[k]));
    }
  }
  if (!enable && h->timing) {
    for (int k = 0; k < SMG_TIMING_CAP; ++k) {
      (void)hipEventDestroy(h->ev0[k]);
      (void)hipEventDestroy(h->ev1[k]);
    }
  }
  h->timing = enable != 0;
  h->ev_used = 0;
  return SMG_OK;
}

smg_status smg_timing_report(smg_handle h, double* ms, int* counts, int max_levels, int* dropped) {
  if (!h || !ms || !counts || max_levels < 1) return fail(h, SMG_EINVAL, "bad arguments");
  const int nk = SMG_TIMING_KINDS;
  for (int k = 0; k < max_levels * nk; ++k) {
    ms[k] = 0.0;
    counts[k] = 0;
  }
  for (int k = 0; k < h->ev_used; ++k) {
    HIPCHK(h, hipEventSynchronize(h->ev1[k]));
    float t = 0.0f;
    HIPCHK(h, hipEventElapsedTime(&t, h->ev0[k], h->ev1[k]));
    const int tag = h->ev_tag[k];
    if (tag / nk < max_levels) {
      ms[tag] += t;
      counts[tag] += 1;
    }
  }
  if (dropped) *dropped = h->ev_used >= SMG_TIMING_CAP;
  h->ev_used = 0;
  return SMG_OK;
}
