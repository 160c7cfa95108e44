// Batched solve of many independent structured systems.
//
// Every system gets its own hierarchy, built by the single-system setup in
// its own slice of one workspace (the method is per system: Sec. 4.2.2 input,
// Sec. 4.3 coarse operators, Sec. 2 V-cycle).  The systems then advance in
// lockstep through preconditioned CG: each step of an iteration -- every
// V-cycle kernel of every level, the outer FP64 operator, the vector updates
// and the dot products -- is one grouped launch over all systems, so a batch
// of small grids occupies the GPU like one large grid instead of a long
// series of small launches.
//  * Grouped stencil kernels map each block to (system, block) through a
//    block map; grouped sweeps hand out tiles by ticket over a merged tile
//    map that keeps every system's own dependence order.
//  * Per-system scalars (rho, alpha, beta, residual norms) and the flags
//    "still iterating" / "convergence claimed" live in device memory; a
//    finished system is skipped by every later launch.  Dot products are
//    deterministic: fixed blocks of 2048 elements, then a fixed-order sum.
//  * BATCH_K lockstep iterations are captured into one HIP graph once and
//    replayed; the host reads the flags once per replay, and each system
//    stops on the device at its convergence or its iteration limit.
//  * The merge order of the systems' sweep tiles (system after system, or
//    round robin) and the size of the persistent sweep grid are chosen by
//    timing whole batched V-cycles (smg_batch_tune).
// Each system's V-cycle runs exactly the kernels of its single-system
// V-cycle on the same data, so a batched preconditioner application equals
// the single-system one bit for bit.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "smg_group.h"
#include "smg_handle.h"

namespace smg {
namespace {

constexpr int BV = 2048;       // vector elements per block of the vector kernels (256 threads x 8)
constexpr int MAXSYS = 4095;   // systems per batch (12 bits of a map entry)
constexpr long MAXMAP = 1L << 20;  // blocks or tiles per system and launch (20 bits of a map entry)

struct SysVec {
  long n;             // unknowns
  long pbase;         // first slot of this system's partial sums
  long nb;            // vector blocks of BV elements
  double* x;          // solution (caller's)
  const double* b;    // right-hand side (caller's)
  double *r, *z, *p, *q;
  void* vin;          // reduced precision: level-0 right-hand side of the V-cycle
  const void* vout;   // reduced precision: level-0 result of the V-cycle
  const double* rin;  // preconditioner entry: caller's r
  double* zout;       // preconditioner entry: caller's z
};

struct Scal {
  double bn, rho, alpha, beta, rel;
  double recur;  // recursively updated residual norm / ||b|| of the last iteration
  int iters, status;
};

// ---------------------------------------------------------------- kernels
__device__ inline double bsum256(double v) {
  __shared__ double red[4];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

enum { D_BB = 0, D_RR = 1, D_PQ = 2, D_RZ = 3 };

// Partial dot products of one vector block per workgroup.
template <int W>
__global__ __launch_bounds__(256) void k_bdot(const SysVec* __restrict__ sv, const unsigned* __restrict__ bmap,
                                              const int* __restrict__ gate, double* __restrict__ part) {
  const unsigned e = bmap[blockIdx.x];
  const int s = (int)(e >> 20);
  const long blk = e & 0xFFFFFu;
  if (gate != nullptr && gate[s] == 0) return;
  const SysVec& v = sv[s];
  const double* __restrict__ a = W == D_BB ? v.b : (W == D_PQ ? v.p : v.r);
  const double* __restrict__ c = W == D_BB ? v.b : (W == D_RR ? v.r : (W == D_PQ ? v.q : v.z));
  const long i0 = blk * BV + threadIdx.x;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < BV / 256; ++k) {
    const long i = i0 + k * 256;
    if (i < v.n) acc = fma(a[i], c[i], acc);
  }
  const double t = bsum256(acc);
  if (threadIdx.x == 0) part[v.pbase + blk] = t;
}

enum { S_BN, S_REL0, S_RHO, S_ALPHA, S_REL, S_CLAIM, S_BETA, S_FINAL };

// Per-system scalar step after a dot product: one wavefront per system sums
// the system's partials in a fixed order, then lane 0 updates its scalars.
template <int OP>
__global__ __launch_bounds__(64) void k_bscal(const SysVec* __restrict__ sv, const double* __restrict__ part,
                                              Scal* __restrict__ sc, int* __restrict__ live, int* __restrict__ claim,
                                              const double* __restrict__ prm) {
  const int s = blockIdx.x;
  const bool need = (OP == S_BN || OP == S_REL0 || OP == S_FINAL) ? true
                                                                    : (OP == S_CLAIM ? claim[s] != 0 : live[s] != 0);
  if (!need) return;
  const SysVec& v = sv[s];
  double acc = 0.0;
  for (long k = threadIdx.x; k < v.nb; k += 64) acc += part[v.pbase + k];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (threadIdx.x != 0) return;
  Scal& c = sc[s];
  const double tol = prm[0];
  switch (OP) {
    case S_BN:
      c.bn = sqrt(acc);
      if (c.bn == 0.0) c.bn = 1.0;
      break;
    case S_REL0:
      c.rel = sqrt(acc) / c.bn;
      c.recur = c.rel;
      c.iters = 0;
      claim[s] = 0;
      if (c.rel < tol) {
        live[s] = 0;
        c.status = SMG_OK;
      } else {
        live[s] = 1;
        c.status = SMG_ENOTCONV;
      }
      break;
    case S_RHO:
      c.rho = acc;
      break;
    case S_ALPHA:
      if (!(acc > 0.0)) {
        c.status = SMG_EBREAKDOWN;
        live[s] = 0;
      } else {
        c.alpha = c.rho / acc;
      }
      break;
    case S_REL:
      c.iters += 1;
      c.rel = sqrt(acc) / c.bn;
      c.recur = c.rel;
      claim[s] = c.rel < tol ? 1 : 0;
      break;
    case S_CLAIM:
      c.rel = sqrt(acc) / c.bn;
      claim[s] = 0;
      if (c.rel < tol) {
        live[s] = 0;
        c.status = SMG_OK;
      }
      break;
    case S_BETA:
      c.beta = acc / c.rho;
      c.rho = acc;
      // the iteration limit: the system stops here, as the single-system
      // solver's loop does after maxit iterations
      if (c.iters >= (int)prm[1]) live[s] = 0;
      break;
    case S_FINAL:
      c.rel = sqrt(acc) / c.bn;
      break;
  }
}

enum { U_AXPY2, U_XPBY, U_COPYZP, U_IN, U_OUT, U_D2F, U_F2D, U_AXPY2RR };

// Vector updates of one block of BV elements per workgroup (same arithmetic
// as the single-system vector kernels).
template <int OP, class V>
// U_AXPY2RR: U_AXPY2 with the partial sums of r.r over the same elements in
// the same order as k_bdot<D_RR>, written where k_bdot writes them (the same
// bits as the update followed by that dot).
__global__ __launch_bounds__(256) void k_bvec(const SysVec* __restrict__ sv, const unsigned* __restrict__ bmap,
                                              const int* __restrict__ gate, const Scal* __restrict__ sc,
                                              double* __restrict__ part) {
  const unsigned e = bmap[blockIdx.x];
  const int s = (int)(e >> 20);
  const long blk = e & 0xFFFFFu;
  if (gate != nullptr && gate[s] == 0) return;
  const SysVec& v = sv[s];
  const double alpha = (OP == U_AXPY2 || OP == U_AXPY2RR) ? sc[s].alpha : 0.0;
  const double beta = OP == U_XPBY ? sc[s].beta : 0.0;
  const long i0 = blk * BV + threadIdx.x;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < BV / 256; ++k) {
    const long i = i0 + k * 256;
    if (i >= v.n) break;
    if (OP == U_AXPY2 || OP == U_AXPY2RR) {
      v.x[i] = fma(alpha, v.p[i], v.x[i]);
      const double ri = fma(-alpha, v.q[i], v.r[i]);
      v.r[i] = ri;
      if (OP == U_AXPY2RR) acc = fma(ri, ri, acc);
    } else if (OP == U_XPBY) {
      v.p[i] = fma(beta, v.p[i], v.z[i]);
    } else if (OP == U_COPYZP) {
      v.p[i] = v.z[i];
    } else if (OP == U_IN) {
      v.r[i] = v.rin[i];
    } else if (OP == U_OUT) {
      v.zout[i] = v.z[i];
    } else if (OP == U_D2F) {
      ((V*)v.vin)[i] = (V)v.r[i];
    } else {
      v.z[i] = (double)((const V*)v.vout)[i];
    }
  }
  if (OP == U_AXPY2RR) {
    const double t = bsum256(acc);
    if (threadIdx.x == 0) part[v.pbase + blk] = t;
  }
}

// ---------------------------------------------------------------- host side
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

// One grouped sweep: segments (one per system taking part), merged tile map.
struct WfGrp {
  int pat = 0;
  void* segs = nullptr;
  unsigned* tmap = nullptr;
  unsigned total = 0;
  std::vector<int> nt;  // tiles per segment
};
// One grouped stencil launch: segments, block map.
struct Grp {
  int pat = 0;
  bool small = false;  // small block shape (residual + restriction, prolongation)
  unsigned stage = 0;  // prolongation: LDS-staged coarse values per block
  void* segs = nullptr;
  unsigned* bmap = nullptr;
  unsigned nblocks = 0;
};
struct LevelPh {
  WfGrp pre, post;
  Grp rr, pp;
  std::vector<int> sys;  // systems with a smoothing step on this level
};

constexpr size_t SEGB = 160;  // bytes reserved per segment of any argument struct
static_assert(sizeof(WfArgs<double>) <= SEGB && sizeof(WfArgs<float>) <= SEGB, "segment size");
static_assert(sizeof(RRArgs<MatH>) <= SEGB && sizeof(PPArgs<MatH>) <= SEGB && sizeof(SpmvArgs<MatD>) <= SEGB,
              "segment size");

}  // namespace
}  // namespace smg

using namespace smg;

struct smg_batch_s {
  int nsys = 0, maxlev = 0, prec = 0, pat0 = 0;
  std::vector<smg_handle_s*> h;
  std::vector<SysVec> sv_host;
  // device tables
  SysVec* sv = nullptr;
  Scal* sc = nullptr;
  int *live = nullptr, *claim = nullptr;
  double *part = nullptr, *prm = nullptr;  // prm: {rtol, maxit} of the running solve
  unsigned *ctr = nullptr, *err = nullptr;
  unsigned* vbmap = nullptr;
  unsigned vblocks = 0;
  std::vector<LevelPh> lv;
  Grp gemv, spmv_ap, spmv_res;
  // sweep schedule (smg_batch_tune)
  int order = 1;
  unsigned grid = WF_MAX_GRID;
  double prm_host[2] = {0.0, 0.0};
  // graph of BATCH_K lockstep CG iterations
  bool use_graph = true;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double t_setup_ms = 0.0;
  char msg[512] = {0};
};

static char g_batch_msg[512] = "no error";

static smg_status bfail(smg_batch B, smg_status st, const char* fmt, ...) {
  char* dst = B ? B->msg : g_batch_msg;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  return st;
}

#define BCHK(B, expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return bfail(B, SMG_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

namespace {

// Shapes of one system's hierarchy (grids, patterns, masks, tilings).
struct Shape {
  int nlev = 0, nc = 0;
  std::vector<Level> lev;
};

// Lays out the batch's device tables in `base` (null: size only).
size_t layout(smg_batch_s* B, const std::vector<Shape>& sh, char* base) {
  Arena ar{base};
  const int ns = B->nsys;
  B->sv = ar.take<SysVec>(ns);
  B->sc = ar.take<Scal>(ns);
  B->live = ar.take<int>(ns);
  B->claim = ar.take<int>(ns);
  B->prm = ar.take<double>(2);
  B->ctr = ar.take<unsigned>(2);
  B->err = ar.take<unsigned>(1);
  long vb = 0, sb = 0;
  for (int s = 0; s < ns; ++s) {
    const long n = sh[s].lev[0].N;
    vb += (n + BV - 1) / BV;
    sb += spmv_blocks(sh[s].lev[0].g);
  }
  B->part = ar.take<double>(vb);
  B->vbmap = ar.take<unsigned>(vb);
  B->vblocks = (unsigned)vb;
  B->maxlev = 0;
  for (int s = 0; s < ns; ++s) B->maxlev = std::max(B->maxlev, sh[s].nlev);
  B->lv.assign(std::max(B->maxlev - 1, 0), LevelPh{});
  for (int l = 0; l + 1 < B->maxlev; ++l) {
    LevelPh& L = B->lv[l];
    long tiles = 0, rrb = 0, ppb = 0;
    for (int s = 0; s < ns; ++s) {
      if (l + 1 >= sh[s].nlev) continue;
      const Level& v = sh[s].lev[l];
      L.sys.push_back(s);
      // room in the tile maps for either tile shape (smg_batch_set_tile_shape)
      WfTiling t1, t2;
      wf_tiling(v.g, v.Ssw, &t1, 1);
      wf_tiling(v.g, v.Ssw, &t2, 2);
      tiles += std::max((long)t1.ntx * t1.nty, (long)t2.ntx * t2.nty);
      rrb += rr_blocks(v.g, v.cmask, false);
      ppb += pp_blocks(v.g, false);
      L.pre.pat = L.post.pat = L.rr.pat = L.pp.pat = v.S;
    }
    // the block shape of a level's grouped launches follows their total size
    L.rr.small = rr_small((unsigned)rrb);
    L.pp.small = pp_small((unsigned)ppb);
    rrb = ppb = 0;
    L.pp.stage = 0;
    for (int s : L.sys) {
      const Level& v = sh[s].lev[l];
      rrb += rr_blocks(v.g, v.cmask, L.rr.small);
      ppb += pp_blocks(v.g, L.pp.small);
      L.pp.stage = std::max(L.pp.stage, pp_stage_elems(v.cmask, L.pp.small));
    }
    const size_t k = L.sys.size();
    L.pre.segs = ar.take<char>(k * SEGB);
    L.post.segs = ar.take<char>(k * SEGB);
    L.pre.tmap = ar.take<unsigned>(tiles);
    L.post.tmap = ar.take<unsigned>(tiles);
    L.rr.segs = ar.take<char>(k * SEGB);
    L.rr.bmap = ar.take<unsigned>(rrb);
    L.rr.nblocks = (unsigned)rrb;
    L.pp.segs = ar.take<char>(k * SEGB);
    L.pp.bmap = ar.take<unsigned>(ppb);
    L.pp.nblocks = (unsigned)ppb;
  }
  long gb = 0;
  for (int s = 0; s < ns; ++s) gb += gemv_blocks(sh[s].nc);
  B->gemv.segs = ar.take<char>(ns * SEGB);
  B->gemv.bmap = ar.take<unsigned>(gb);
  B->gemv.nblocks = (unsigned)gb;
  B->spmv_ap.segs = ar.take<char>(ns * SEGB);
  B->spmv_ap.bmap = ar.take<unsigned>(sb);
  B->spmv_ap.nblocks = (unsigned)sb;
  B->spmv_ap.pat = B->pat0;
  B->spmv_res.segs = ar.take<char>(ns * SEGB);
  B->spmv_res.bmap = B->spmv_ap.bmap;  // same blocks
  B->spmv_res.nblocks = (unsigned)sb;
  B->spmv_res.pat = B->pat0;
  return ar.off + 256;
}

template <class T>
hipError_t upload(T* dst, const std::vector<T>& v) {
  if (v.empty()) return hipSuccess;
  return hipMemcpy(dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}
// Segment tables are dense arrays of one argument type (the grouped kernels
// index them as such); SEGB bytes per segment are reserved for any type.
template <class T>
hipError_t upload_typed(void* dst, const std::vector<T>& v) {
  if (v.empty()) return hipSuccess;
  return hipMemcpy(dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

std::vector<unsigned> block_map(const std::vector<unsigned>& nb) {
  std::vector<unsigned> m;
  for (size_t k = 0; k < nb.size(); ++k)
    for (unsigned b = 0; b < nb[k]; ++b) m.push_back((unsigned)(k << 20) | b);
  return m;
}

// Merged tile map: order 0 = system after system, 1 = round robin over the
// systems' r-th tiles.  Both keep each system's tiles in increasing order.
std::vector<unsigned> tile_map(const std::vector<int>& nt, int order) {
  std::vector<unsigned> m;
  if (order == 0) {
    for (size_t k = 0; k < nt.size(); ++k)
      for (int r = 0; r < nt[k]; ++r) m.push_back((unsigned)(k << 20) | (unsigned)r);
  } else {
    int mx = 0;
    for (int v : nt) mx = std::max(mx, v);
    for (int r = 0; r < mx; ++r)
      for (size_t k = 0; k < nt.size(); ++k)
        if (r < nt[k]) m.push_back((unsigned)(k << 20) | (unsigned)r);
  }
  return m;
}

hipError_t upload_tile_maps(smg_batch_s* B) {
  for (auto& L : B->lv) {
    const std::vector<unsigned> m = tile_map(L.pre.nt, B->order);
    hipError_t e = upload(L.pre.tmap, m);
    if (e == hipSuccess) e = upload(L.post.tmap, m);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <class PT>
const typename PT::V* Fp(const smg_batch_s* B, int s, int l) {
  const smg_handle_s* H = B->h[s];
  if (l > 0) return (const typename PT::V*)H->lev[l].f;
  return B->prec == SMG_FP64 ? (const typename PT::V*)H->kr : (const typename PT::V*)H->lev[0].f;
}
template <class PT>
typename PT::V* UBp(const smg_batch_s* B, int s, int l) {
  const smg_handle_s* H = B->h[s];
  if (l > 0) return (typename PT::V*)H->lev[l].ub;
  return B->prec == SMG_FP64 ? (typename PT::V*)H->kz : (typename PT::V*)H->lev[0].ub;
}

// Fills every table that does not depend on caller vectors.
template <class PT>
hipError_t fill_tables(smg_batch_s* B) {
  using V = typename PT::V;
  using M = typename PT::M;
  const int ns = B->nsys;
  hipError_t e;
  // vector blocks
  std::vector<unsigned> nbv(ns);
  long pb = 0;
  B->sv_host.assign(ns, SysVec{});
  for (int s = 0; s < ns; ++s) {
    smg_handle_s* H = B->h[s];
    SysVec& v = B->sv_host[s];
    v.n = H->lev[0].N;
    v.nb = (v.n + BV - 1) / BV;
    v.pbase = pb;
    pb += v.nb;
    v.r = H->kr;
    v.z = H->kz;
    v.p = H->kp;
    v.q = H->kq;
    v.vin = H->lev[0].f;
    v.vout = H->lev[0].ub;
    nbv[s] = (unsigned)v.nb;
  }
  if ((e = upload(B->vbmap, block_map(nbv))) != hipSuccess) return e;
  if ((e = upload(B->sv, B->sv_host)) != hipSuccess) return e;
  // levels
  for (int l = 0; l + 1 < B->maxlev; ++l) {
    LevelPh& L = B->lv[l];
    std::vector<WfArgs<V>> pre, post;
    std::vector<RRArgs<M>> rr;
    std::vector<PPArgs<M>> pp;
    std::vector<unsigned> rrb, ppb;
    L.pre.nt.clear();
    for (int s : L.sys) {
      smg_handle_s* H = B->h[s];
      const Level& v = H->lev[l];
      WfArgs<V> a{};
      a.g = v.g;
      a.t = v.tl;
      a.pk = v.pk[0];
      a.sd = v.psd;
      a.h = Fp<PT>(B, s, l);
      a.x = (V*)v.ua;
      a.next = UBp<PT>(B, s, l);
      a.next_dir = -1;
      a.sys = s;
      pre.push_back(a);
      WfArgs<V> c = a;
      c.pk = v.pk[1];
      c.h = (const V*)v.h;
      c.x = UBp<PT>(B, s, l);
      c.next = (V*)v.ua;
      c.next_dir = +1;
      post.push_back(c);
      L.pre.nt.push_back(v.tl.ntx * v.tl.nty);
      rr.push_back(RRArgs<M>{v.g, v.cmask, PT::A(v), Fp<PT>(B, s, l), (const V*)v.ua, (V*)H->lev[l + 1].f, s});
      pp.push_back(PPArgs<M>{v.g, v.cmask, PT::A(v), Fp<PT>(B, s, l), (const V*)v.ua, (const V*)UBp<PT>(B, s, l + 1),
                             (V*)v.h, nullptr, s});
      rrb.push_back(rr_blocks(v.g, v.cmask, L.rr.small));
      ppb.push_back(pp_blocks(v.g, L.pp.small));
    }
    L.post.nt = L.pre.nt;
    unsigned tiles = 0;
    for (int t : L.pre.nt) tiles += (unsigned)t;
    L.pre.total = L.post.total = tiles;
    if ((e = upload_typed(L.pre.segs, pre)) != hipSuccess) return e;
    if ((e = upload_typed(L.post.segs, post)) != hipSuccess) return e;
    if ((e = upload_typed(L.rr.segs, rr)) != hipSuccess) return e;
    if ((e = upload_typed(L.pp.segs, pp)) != hipSuccess) return e;
    if ((e = upload(L.rr.bmap, block_map(rrb))) != hipSuccess) return e;
    if ((e = upload(L.pp.bmap, block_map(ppb))) != hipSuccess) return e;
  }
  if ((e = upload_tile_maps(B)) != hipSuccess) return e;
  // coarsest solves
  std::vector<GemvArgs<V>> gm;
  std::vector<unsigned> gmb;
  for (int s = 0; s < ns; ++s) {
    smg_handle_s* H = B->h[s];
    const int L = H->nlev - 1;
    gm.push_back(GemvArgs<V>{H->nc, 2 * H->nc, H->aug + H->nc, Fp<PT>(B, s, L), UBp<PT>(B, s, L), s});
    gmb.push_back(gemv_blocks(H->nc));
  }
  if ((e = upload_typed(B->gemv.segs, gm)) != hipSuccess) return e;
  if ((e = upload(B->gemv.bmap, block_map(gmb))) != hipSuccess) return e;
  // outer operator q = A p
  std::vector<SpmvArgs<MatD>> ap;
  std::vector<unsigned> apb;
  for (int s = 0; s < ns; ++s) {
    smg_handle_s* H = B->h[s];
    const Level& v = H->lev[0];
    ap.push_back(SpmvArgs<MatD>{v.g, MatD{v.A64, v.N}, H->kp, nullptr, H->kq, s});
    apb.push_back(spmv_blocks(v.g));
  }
  if ((e = upload_typed(B->spmv_ap.segs, ap)) != hipSuccess) return e;
  return upload(B->spmv_ap.bmap, block_map(apb));
}

hipError_t fill_tables_any(smg_batch_s* B) {
  switch (B->prec) {
    case SMG_FP64: return fill_tables<P64>(B);
    case SMG_FP32: return fill_tables<P32>(B);
    default: return fill_tables<P16>(B);
  }
}

// One batched V-cycle z = M r on the systems with gate[s] != 0 (null: all),
// on the internal vectors r (kr) and z (kz) of every system.
template <class PT>
hipError_t bvcycle(smg_batch_s* B, const int* gate, hipStream_t st) {
  using V = typename PT::V;
  using E = typename PT::E;
  using M = typename PT::M;
  hipError_t e = hipSuccess;
  const dim3 vg(B->vblocks), vb(256);
  if (B->prec != SMG_FP64) {
    hipLaunchKernelGGL((k_bvec<U_D2F, float>), vg, vb, 0, st, B->sv, B->vbmap, gate, B->sc, (double*)nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int l = 0; l + 1 < B->maxlev; ++l) {
    const LevelPh& L = B->lv[l];
    e = launch_wavefront_group<E>(L.pre.pat, +1, (const WfArgs<V>*)L.pre.segs, L.pre.tmap, L.pre.total, B->grid,
                                  gate, B->ctr, B->err, st);
    if (e == hipSuccess) e = launch_rr_group<M>(L.rr.pat, L.rr.small, (const RRArgs<M>*)L.rr.segs, L.rr.bmap, L.rr.nblocks, gate, st);
    if (e != hipSuccess) return e;
  }
  e = launch_gemv_group<V>((const GemvArgs<V>*)B->gemv.segs, B->gemv.bmap, B->gemv.nblocks, gate, st);
  if (e != hipSuccess) return e;
  for (int l = B->maxlev - 2; l >= 0; --l) {
    const LevelPh& L = B->lv[l];
    e = launch_pp_group<M>(L.pp.pat, false, L.pp.small, L.pp.stage, (const PPArgs<M>*)L.pp.segs, L.pp.bmap, L.pp.nblocks, gate, st);
    if (e == hipSuccess)
      e = launch_wavefront_group<E>(L.post.pat, -1, (const WfArgs<V>*)L.post.segs, L.post.tmap, L.post.total, B->grid,
                                    gate, B->ctr, B->err, st);
    if (e != hipSuccess) return e;
  }
  if (B->prec != SMG_FP64) {
    hipLaunchKernelGGL((k_bvec<U_F2D, float>), vg, vb, 0, st, B->sv, B->vbmap, gate, B->sc, (double*)nullptr);
    e = hipGetLastError();
  }
  return e;
}

hipError_t vcycle_any(smg_batch_s* B, const int* gate, hipStream_t st) {
  switch (B->prec) {
    case SMG_FP64: return bvcycle<P64>(B, gate, st);
    case SMG_FP32: return bvcycle<P32>(B, gate, st);
    default: return bvcycle<P16>(B, gate, st);
  }
}

template <int W>
hipError_t dot(smg_batch_s* B, const int* gate, hipStream_t st) {
  hipLaunchKernelGGL((k_bdot<W>), dim3(B->vblocks), dim3(256), 0, st, B->sv, B->vbmap, gate, B->part);
  return hipGetLastError();
}
template <int OP>
hipError_t scal(smg_batch_s* B, hipStream_t st) {
  hipLaunchKernelGGL((k_bscal<OP>), dim3(B->nsys), dim3(64), 0, st, B->sv, B->part, B->sc, B->live, B->claim,
                     B->prm);
  return hipGetLastError();
}
template <int OP>
hipError_t vec(smg_batch_s* B, const int* gate, hipStream_t st) {
  hipLaunchKernelGGL((k_bvec<OP, float>), dim3(B->vblocks), dim3(256), 0, st, B->sv, B->vbmap, gate, B->sc, B->part);
  return hipGetLastError();
}
hipError_t spmv(smg_batch_s* B, const Grp& g, bool res, const int* gate, hipStream_t st) {
  return launch_spmv_group<MatD>(g.pat, res, (const SpmvArgs<MatD>*)g.segs, g.bmap, g.nblocks, gate, st);
}

// One lockstep CG iteration of every live system (the order of the
// single-system solver: q = A p, alpha, x and r updates, residual norm, true
// residual on a convergence claim, V-cycle, beta, p update).
hipError_t iteration(smg_batch_s* B, hipStream_t st) {
  hipError_t e;
#define ICHK(x)                           \
  if ((e = (x)) != hipSuccess) return e;
  ICHK(spmv(B, B->spmv_ap, false, B->live, st));
  ICHK(dot<D_PQ>(B, B->live, st));
  ICHK(scal<S_ALPHA>(B, st));
  ICHK(vec<U_AXPY2RR>(B, B->live, st));
  ICHK(scal<S_REL>(B, st));
  ICHK(spmv(B, B->spmv_res, true, B->claim, st));
  ICHK(dot<D_RR>(B, B->claim, st));
  ICHK(scal<S_CLAIM>(B, st));
  ICHK(vcycle_any(B, B->live, st));
  ICHK(dot<D_RZ>(B, B->live, st));
  ICHK(scal<S_BETA>(B, st));
  ICHK(vec<U_XPBY>(B, B->live, st));
#undef ICHK
  return hipSuccess;
}

void drop_graph(smg_batch_s* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
}

// Lockstep iterations per graph launch: the host reads the systems' flags
// once per launch.  A system that converges (or reaches maxit, or breaks
// down) inside a launch is skipped by the rest of its kernels.
constexpr int BATCH_K = 4;

hipError_t ensure_graph(smg_batch_s* B) {
  if (B->exec) return hipSuccess;
  hipError_t e = hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t ei = hipSuccess;
  for (int k = 0; k < BATCH_K && ei == hipSuccess; ++k) ei = iteration(B, B->cap);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(B->cap, &g);
  if (ei != hipSuccess) e = ei;
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return e;
  }
  B->graph = g;
  e = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) drop_graph(B);
  return e;
}

}  // namespace

extern "C" {

smg_status smg_batch_workspace_size(int nsys, const smg_config* cfgs, size_t* bytes) {
  if (nsys < 1 || nsys > MAXSYS) return bfail(nullptr, SMG_EINVAL, "nsys = %d outside [1, %d]", nsys, MAXSYS);
  if (!cfgs || !bytes) return bfail(nullptr, SMG_EINVAL, "null argument");
  std::vector<Shape> sh(nsys);
  size_t total = 0;
  for (int s = 0; s < nsys; ++s) {
    const smg_config& c = cfgs[s];
    const char* why = config_error(&c);
    if (why) return bfail(nullptr, SMG_EINVAL, "system %d: %s", s, why);
    if (c.block != 1 || c.smoother != SMG_SMOOTH_GS || c.interp != SMG_INTERP_VERTEX)
      return bfail(nullptr, SMG_EINVAL,
                   "system %d: batches take scalar systems, the GS smoother and vertex-centred transfers", s);
    if (!cfg_default_smoothing(c) || c.coarsen == SMG_COARSEN_AUTO)
      return bfail(nullptr, SMG_EINVAL,
                   "system %d: batches take one ZeroGuess GS step before and after the coarse correction "
                   "(weight 1) and a fixed coarsening", s);
    if (c.prec != cfgs[0].prec || c.pattern != cfgs[0].pattern)
      return bfail(nullptr, SMG_EINVAL, "system %d: every system of a batch has the same pattern and precision", s);
    sh[s].lev.resize(MAXLEV);
    const size_t b = plan_shapes(c, sh[s].lev.data(), &sh[s].nlev, &sh[s].nc);
    if (b == 0) return bfail(nullptr, SMG_EINVAL, "system %d: coarsest level too large", s);
    if ((sh[s].lev[0].N + BV - 1) / BV >= MAXMAP || spmv_blocks(sh[s].lev[0].g) >= MAXMAP)
      return bfail(nullptr, SMG_EINVAL, "system %d: grid too large for a batch", s);
    total += (b + 255) & ~(size_t)255;
  }
  smg_batch_s tmp;
  tmp.nsys = nsys;
  tmp.pat0 = cfgs[0].pattern;
  total += layout(&tmp, sh, nullptr);
  *bytes = total + 512;  // alignment of the workspace and of the table region
  return SMG_OK;
}

smg_status smg_batch_setup(int nsys, const smg_config* cfgs, const double* const* coeffs, void* workspace,
                           size_t bytes, void* stream, smg_batch* out) {
  if (!out) return bfail(nullptr, SMG_EINVAL, "null output handle");
  *out = nullptr;
  size_t need = 0;
  smg_status s0 = smg_batch_workspace_size(nsys, cfgs, &need);
  if (s0 != SMG_OK) return s0;
  if (!coeffs || !workspace) return bfail(nullptr, SMG_EINVAL, "null coefficient or workspace pointer");
  if (bytes < need) return bfail(nullptr, SMG_ENOMEM, "workspace of %zu bytes, %zu needed", bytes, need);
  for (int s = 0; s < nsys; ++s)
    if (!coeffs[s]) return bfail(nullptr, SMG_EINVAL, "null coefficients of system %d", s);
  hipStream_t st = (hipStream_t)stream;
  auto t0 = std::chrono::steady_clock::now();
  smg_batch_s* B = new smg_batch_s();
  B->nsys = nsys;
  B->prec = cfgs[0].prec;
  B->pat0 = cfgs[0].pattern;
  auto bail = [&](smg_status s) {
    snprintf(g_batch_msg, sizeof g_batch_msg, "%s", B->msg);
    for (smg_handle_s* H : B->h) smg_destroy(H);
    if (B->cap) (void)hipStreamDestroy(B->cap);
    delete B;
    return s;
  };
  char* base = (char*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
  std::vector<Shape> sh(nsys);
  for (int s = 0; s < nsys; ++s) {
    sh[s].lev.resize(MAXLEV);
    plan_shapes(cfgs[s], sh[s].lev.data(), &sh[s].nlev, &sh[s].nc);
  }
  const size_t tb = layout(B, sh, base);
  size_t off = (tb + 255) & ~(size_t)255;
  for (int s = 0; s < nsys; ++s) {
    size_t b = 0;
    smg_workspace_size(&cfgs[s], &b);
    smg_handle H = nullptr;
    smg_status ss = smg_setup(&cfgs[s], coeffs[s], base + off, b, stream, &H);
    if (ss != SMG_OK) {
      bfail(B, ss, "system %d: %s", s, smg_last_error(nullptr));
      return bail(ss);
    }
    // the batch's sweeps are tiled on every level; keep the system's own
    // sweeps on the same data (sentinel protocol) when it is used alone
    H->hp_on = false;
    B->h.push_back(H);
    off += (b + 255) & ~(size_t)255;
  }
  hipError_t e = fill_tables_any(B);
  // ticket counters and the watchdog flag start at zero (the workspace is
  // the caller's memory, not cleared; a stale flag read as a fired watchdog)
  if (e == hipSuccess) e = hipMemsetAsync(B->ctr, 0, 2 * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMemsetAsync(B->err, 0, sizeof(unsigned), st);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    bfail(B, SMG_EDEVICE, "batch tables: %s", hipGetErrorString(e));
    return bail(SMG_EDEVICE);
  }
  B->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = B;
  return SMG_OK;
}

// Tile shape of level l in every system that sweeps there, and the batch's
// tables that depend on the tilings.
smg_status set_tile_shape(smg_batch_s* B, int l, int shape, hipStream_t st) {
  if (l < 0 || l + 1 >= B->maxlev) return bfail(B, SMG_EINVAL, "level %d has no smoothing sweep", l);
  for (int s : B->lv[l].sys) {
    const char* why = nullptr;
    const hipError_t e = retile_level(B->h[s], l, shape, st, &why);
    if (why) return bfail(B, SMG_EINVAL, "system %d level %d: %s", s, l, why);
    BCHK(B, e);
  }
  BCHK(B, hipStreamSynchronize(st));
  drop_graph(B);
  BCHK(B, fill_tables_any(B));
  return SMG_OK;
}

smg_status smg_batch_set_schedule(smg_batch B, int order, int grid) {
  if (!B) return bfail(nullptr, SMG_EINVAL, "null batch");
  if (order < 0 || order > 1 || grid < 0) return bfail(B, SMG_EINVAL, "bad schedule (%d, %d)", order, grid);
  B->order = order;
  B->grid = grid == 0 ? WF_MAX_GRID : (unsigned)grid;
  drop_graph(B);
  BCHK(B, upload_tile_maps(B));
  return SMG_OK;
}

smg_status smg_batch_set_graph(smg_batch B, int enable) {
  if (!B) return bfail(nullptr, SMG_EINVAL, "null batch");
  B->use_graph = enable != 0;
  drop_graph(B);
  return SMG_OK;
}

smg_status smg_batch_precondition(smg_batch B, const double* const* r, double* const* z, void* stream) {
  if (!B) return bfail(nullptr, SMG_EINVAL, "null batch");
  if (!r || !z) return bfail(B, SMG_EINVAL, "null vector array");
  hipStream_t st = (hipStream_t)stream;
  for (int s = 0; s < B->nsys; ++s) {
    if (!r[s] || !z[s]) return bfail(B, SMG_EINVAL, "null vector of system %d", s);
    B->sv_host[s].rin = r[s];
    B->sv_host[s].zout = z[s];
  }
  BCHK(B, hipMemcpyAsync(B->sv, B->sv_host.data(), sizeof(SysVec) * B->nsys, hipMemcpyHostToDevice, st));
  BCHK(B, vec<U_IN>(B, nullptr, st));
  BCHK(B, vcycle_any(B, nullptr, st));
  BCHK(B, vec<U_OUT>(B, nullptr, st));
  // the host array is read by the copy above before it may change
  BCHK(B, hipStreamSynchronize(st));
  return SMG_OK;
}

smg_status smg_batch_tune(smg_batch B, void* stream, int* order_out, int* grid_out, double* ms_out) {
  if (!B) return bfail(nullptr, SMG_EINVAL, "null batch");
  hipStream_t st = (hipStream_t)stream;
  for (int s = 0; s < B->nsys; ++s) BCHK(B, hipMemsetAsync(B->h[s]->kr, 0, sizeof(double) * B->sv_host[s].n, st));
  // persistent sweep grids (one sweep workgroup fits a CU: at most WF_MAX_GRID)
  const unsigned grids[] = {128, 192, WF_MAX_GRID};
  hipEvent_t e0, e1;
  BCHK(B, hipEventCreate(&e0));
  BCHK(B, hipEventCreate(&e1));
  double best = 1e300;
  int bo = B->order;
  unsigned bg = B->grid;
  for (int order = 0; order < 2; ++order) {
    B->order = order;
    BCHK(B, upload_tile_maps(B));
    for (unsigned g : grids) {
      B->grid = g;
      BCHK(B, vcycle_any(B, nullptr, st));
      BCHK(B, hipEventRecord(e0, st));
      for (int k = 0; k < 3; ++k) BCHK(B, vcycle_any(B, nullptr, st));
      BCHK(B, hipEventRecord(e1, st));
      BCHK(B, hipEventSynchronize(e1));
      float ms = 0.f;
      BCHK(B, hipEventElapsedTime(&ms, e0, e1));
      if (ms / 3.0 < best) {
        best = ms / 3.0;
        bo = order;
        bg = g;
      }
    }
  }
  smg_status s = smg_batch_set_schedule(B, bo, (int)bg);
  if (s != SMG_OK) return s;
  // then the tile shape of each level's sweeps (sheared / rectangular),
  // level by level with the others fixed
  auto time_cycles = [&](double* ms_out) -> smg_status {
    BCHK(B, vcycle_any(B, nullptr, st));
    BCHK(B, hipEventRecord(e0, st));
    for (int k = 0; k < 3; ++k) BCHK(B, vcycle_any(B, nullptr, st));
    BCHK(B, hipEventRecord(e1, st));
    BCHK(B, hipEventSynchronize(e1));
    float ms = 0.f;
    BCHK(B, hipEventElapsedTime(&ms, e0, e1));
    *ms_out = ms / 3.0;
    return SMG_OK;
  };
  for (int l = 0; l + 1 < B->maxlev; ++l) {
    if (B->lv[l].sys.empty()) continue;
    // rectangles only where every system's level allows them
    bool rect_ok = true;
    for (int sy : B->lv[l].sys) {
      const Level& v = B->h[sy]->lev[l];
      WfTiling t;
      wf_tiling(v.g, v.Ssw, &t, 2);
      rect_ok = rect_ok && (v.Ssw == 7 || t.nty == 1);
    }
    int bshape = 0;
    double bms = 1e300;
    for (int shape = 1; shape <= (rect_ok ? 2 : 1); ++shape) {
      if ((s = set_tile_shape(B, l, shape, st)) != SMG_OK) return s;
      double ms = 0.0;
      if ((s = time_cycles(&ms)) != SMG_OK) return s;
      if (ms < bms) {
        bms = ms;
        bshape = shape;
      }
    }
    if ((s = set_tile_shape(B, l, bshape, st)) != SMG_OK) return s;
    best = bms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  unsigned ef = 0;
  BCHK(B, hipMemcpy(&ef, B->err, sizeof ef, hipMemcpyDeviceToHost));
  if (ef & 1u) return bfail(B, SMG_EDEADLOCK, "wavefront watchdog fired");
  if (order_out) *order_out = bo;
  if (grid_out) *grid_out = (int)bg;
  if (ms_out) *ms_out = best;
  return SMG_OK;
}

smg_status smg_batch_solve(smg_batch B, const double* const* b, double* const* x, double rtol, int maxit,
                           smg_result* results, int* status, void* stream) {
  if (!B) return bfail(nullptr, SMG_EINVAL, "null batch");
  if (!b || !x) return bfail(B, SMG_EINVAL, "null vector array");
  if (!(rtol > 0.0) || maxit < 0) return bfail(B, SMG_EINVAL, "bad rtol / maxit");
  hipStream_t st = (hipStream_t)stream;
  auto t0 = std::chrono::steady_clock::now();
  const int ns = B->nsys;
  std::vector<SpmvArgs<MatD>> res(ns);
  for (int s = 0; s < ns; ++s) {
    if (!b[s] || !x[s]) return bfail(B, SMG_EINVAL, "null vector of system %d", s);
    smg_handle_s* H = B->h[s];
    const Level& v = H->lev[0];
    B->sv_host[s].x = x[s];
    B->sv_host[s].b = b[s];
    res[s] = SpmvArgs<MatD>{v.g, MatD{v.A64, v.N}, x[s], b[s], H->kr, s};
  }
  BCHK(B, hipMemcpyAsync(B->sv, B->sv_host.data(), sizeof(SysVec) * ns, hipMemcpyHostToDevice, st));
  BCHK(B, hipMemcpyAsync(B->spmv_res.segs, res.data(), sizeof(SpmvArgs<MatD>) * ns, hipMemcpyHostToDevice, st));
  B->prm_host[0] = rtol;
  B->prm_host[1] = (double)maxit;
  BCHK(B, hipMemcpyAsync(B->prm, B->prm_host, sizeof B->prm_host, hipMemcpyHostToDevice, st));
  // start: |b|, r = b - A x, first residual, z = M r, p = z, rho = r.z
  BCHK(B, dot<D_BB>(B, nullptr, st));
  BCHK(B, scal<S_BN>(B, st));
  BCHK(B, spmv(B, B->spmv_res, true, nullptr, st));
  BCHK(B, dot<D_RR>(B, nullptr, st));
  BCHK(B, scal<S_REL0>(B, st));
  BCHK(B, vcycle_any(B, B->live, st));
  BCHK(B, vec<U_COPYZP>(B, B->live, st));
  BCHK(B, dot<D_RZ>(B, B->live, st));
  BCHK(B, scal<S_RHO>(B, st));
  if (B->use_graph) BCHK(B, ensure_graph(B));
  // BATCH_K iterations per host check of the flags (one graph launch, or
  // the same launches one by one); every system stops at its own
  // convergence or at maxit on the device
  std::vector<int> live(ns);
  int waits = 0;
  for (int it = 0; it < maxit; it += BATCH_K) {
    BCHK(B, hipMemcpyAsync(live.data(), B->live, sizeof(int) * ns, hipMemcpyDeviceToHost, st));
    BCHK(B, hipStreamSynchronize(st));
    ++waits;
    int nl = 0;
    for (int v : live) nl += v != 0;
    if (nl == 0) break;
    if (B->use_graph) {
      BCHK(B, hipGraphLaunch(B->exec, st));
    } else {
      for (int k = 0; k < BATCH_K; ++k) BCHK(B, iteration(B, st));
    }
  }
  // final true residuals
  BCHK(B, spmv(B, B->spmv_res, true, nullptr, st));
  BCHK(B, dot<D_RR>(B, nullptr, st));
  BCHK(B, scal<S_FINAL>(B, st));
  std::vector<Scal> sc(ns);
  unsigned ef = 0;
  BCHK(B, hipMemcpyAsync(sc.data(), B->sc, sizeof(Scal) * ns, hipMemcpyDeviceToHost, st));
  BCHK(B, hipMemcpyAsync(&ef, B->err, sizeof ef, hipMemcpyDeviceToHost, st));
  BCHK(B, hipStreamSynchronize(st));
  ++waits;
  if (ef & 1u) return bfail(B, SMG_EDEADLOCK, "wavefront watchdog fired");
  const double tsolve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  smg_status worst = SMG_OK;
  for (int s = 0; s < ns; ++s) {
    const smg_handle_s* H = B->h[s];
    const int stt = sc[s].status;
    if (status) status[s] = stt;
    if (stt == SMG_EBREAKDOWN) worst = SMG_EBREAKDOWN;
    else if (stt != SMG_OK && worst == SMG_OK) worst = SMG_ENOTCONV;
    if (results) {
      smg_result& r = results[s];
      r.iters = sc[s].iters;
      r.levels = H->nlev;
      r.rel_resid_true = sc[s].rel;
      r.rel_resid_recur = sc[s].recur;
      double sn = 0, so = 0;
      for (int l = 0; l < H->nlev; ++l) {
        sn += (double)H->lev[l].N;
        so += (double)H->lev[l].N * H->lev[l].S;
      }
      r.grid_complexity = sn / (double)H->lev[0].N;
      r.op_complexity = so / ((double)H->lev[0].N * H->lev[0].S);
      r.t_setup_ms = B->t_setup_ms;
      r.t_solve_ms = tsolve;
      r.host_waits = waits;
    }
  }
  if (worst == SMG_ENOTCONV) bfail(B, worst, "some systems did not converge in %d iterations", maxit);
  if (worst == SMG_EBREAKDOWN) bfail(B, worst, "breakdown (p.Ap <= 0) in some system");
  return worst;
}

smg_status smg_batch_set_tile_shape(smg_batch B, int level, int shape, void* stream) {
  if (!B) return bfail(nullptr, SMG_EINVAL, "null batch");
  return set_tile_shape(B, level, shape, (hipStream_t)stream);
}

int smg_batch_tile_shape(smg_batch B, int level) {
  if (!B || level < 0 || level + 1 >= B->maxlev || B->lv[level].sys.empty()) return 0;
  return smg_tile_shape(B->h[B->lv[level].sys[0]], level);
}

int smg_batch_num_systems(smg_batch B) { return B ? B->nsys : 0; }

smg_handle smg_batch_system(smg_batch B, int s) { return (B && s >= 0 && s < B->nsys) ? B->h[s] : nullptr; }

smg_status smg_batch_destroy(smg_batch B) {
  if (!B) return SMG_OK;
  drop_graph(B);
  for (smg_handle_s* H : B->h) smg_destroy(H);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  delete B;
  return SMG_OK;
}

const char* smg_batch_last_error(smg_batch B) { return B ? B->msg : g_batch_msg; }

}  // extern "C"
