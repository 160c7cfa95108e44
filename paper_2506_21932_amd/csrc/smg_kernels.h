// Host-side launchers of the device kernels (internal to libstructmg).
#pragma once
#include <vector>

#include "smg_common.h"

namespace smg {

// ---- wavefront triangular sweep --------------------------------------
// Persistent grid of at most WF_MAX_GRID workgroups (one resident sweep
// workgroup per CU: its LDS ring and chunk buffers take most of the CU's LDS).
constexpr int WF_MAX_GRID = 256;

template <class E>
struct WfVal {
  using V = E;  // arithmetic type of storage element E
};
template <>
struct WfVal<__half> {
  using V = float;
};

template <class V>
struct WfArgs {
  Grid g;
  WfTiling t;                // tiling of the level (wf_tiling)
  const void* pk;            // packed sweep data of this direction (launch_wf_pack)
  const float* sd;           // FP16 storage: {row scale, diagonal scaling} per position
  const V* h;                // right-hand side of the triangular system
  V* x;                      // output; positions read by other tiles hold the sentinel
  V* next;                   // output buffer of the next sweep on this level (sentinel prefill), or null
  int next_dir;              // direction of that next sweep
  const V* addv;             // optional: addout = addv + x
  V* addout;
  unsigned* ctr;             // [0] ticket counter, [1] exit counter; zero between launches
  unsigned* err;             // watchdog flag (bit 0)
  int sys;                   // grouped sweeps: system of this grid
};

// shape: 0 default (sheared for 19/27 points with more than one tile row),
// 1 sheared, 2 rectangular
void wf_tiling(const Grid& g, int pat, WfTiling* t, int shape = 0);
// 16-byte packs per schedule position and direction for storage elements of
// ebytes bytes; offsets within a tile must stay below 2^31 bytes.
int wf_pack_count(int pat, int ebytes);
bool wf_ranges_ok(const Grid& g, const WfTiling& t, int pat, int vbytes, int ebytes);

// E = double / float / __half (FP16 storage, FP32 arithmetic)
template <class E>
hipError_t launch_wavefront(int pat, int dir, bool unitd, bool add, const WfArgs<typename WfVal<E>::V>& a,
                            hipStream_t st);
// Packed sweep data of direction dir from natural SG-DIA arrays: lower
// (dir > 0) or upper (dir < 0) triangle of lo / up, then the diagonal scaling dg.
template <class E>
hipError_t launch_wf_pack(int pat, const Grid& g, const WfTiling& tl, int dir, const double* lo, const double* dg,
                          const double* up, E* out, hipStream_t st);
// FP16: halves of a16 per direction; sd (written by the dir > 0 call) holds
// {row scale, diagonal scaling} per position.
hipError_t launch_wf_pack_h(int pat, const Grid& g, const WfTiling& tl, int dir, const __half* a16, const float* sc,
                            const float* rd, __half* out, float* sd, hipStream_t st);

// One sweep over many independent grids of pattern pat in one launch.
// segs[k]: the arguments of grid k (their ctr / err are not used);
// tmap[t] = (k << 20) | r: ticket t is the r-th tile of grid k in its own
// forward dependence order (each grid's tiles appear in increasing r);
// total tickets; grid workgroups (0: one per tile); ctr / err as in WfArgs;
// tiles of a grid whose system is finished (live[sys] == 0) are skipped.
template <class E>
hipError_t launch_wavefront_group(int pat, int dir, const WfArgs<typename WfVal<E>::V>* segs, const unsigned* tmap,
                                  unsigned total, unsigned grid, const int* live, unsigned* ctr, unsigned* err,
                                  hipStream_t st);

// ---- small levels: one-workgroup hyperplane sweep (hpsweep.hip) ---------
// hp_plan: hyperplanes of the level, or 0 when it does not fit (pts: host
// schedule [step][256] of box indices, -1 padded).  launch_hp_pack builds the
// step-ordered coefficients of direction dir (src 0: FP64, 1: FP32 from the
// FP64 data, 2: FP16 row-scaled storage); launch_hpsweep runs a forward
// (dir > 0) or backward Gauss-Seidel sweep x = S(h) of the level.
int hp_plan(const Grid& g, int pat, int vbytes, std::vector<int>* pts);
hipError_t launch_hp_pack(int pat, int src, const Grid& g, int nsteps, int dir, const int* pts, const double* A,
                          const double* rd, const __half* a16, const float* sc, const float* rd32, void* out,
                          hipStream_t st);
template <class V>
hipError_t launch_hpsweep(int pat, int dir, const Grid& g, int nsteps, const int* pts, const V* cf, const V* h, V* x,
                          hipStream_t st);

// ---- grouped launches ---------------------------------------------------
// Arguments of one grid of a kernel that can also run grouped (smg_group.h):
// bmap[b] = (segment << 20) | (block of that segment), live[sys] == 0 skips
// a segment.  *_blocks give the blocks of one grid.
template <class M>
struct SpmvArgs {
  Grid g;
  M m;
  const typename M::V* x;
  const typename M::V* b;
  typename M::V* y;
  int sys;
};
template <class M>
struct RRArgs {
  Grid g;
  int cmask;
  M m;
  const typename M::V* f;
  const typename M::V* u;
  typename M::V* rc;
  int sys;
};
template <class M>
struct PPArgs {
  Grid g;
  int cmask;
  M m;
  const typename M::V* f;
  const typename M::V* u;
  const typename M::V* ec;
  typename M::V* h;
  typename M::V* uo;
  int sys;
};
template <class V>
struct GemvArgs {
  int n;
  int ld;
  const double* ainv;
  const V* f;
  V* u;
  int sys;
};
unsigned spmv_blocks(const Grid& g);
// residual + restriction and prolongation: large or small blocks (chosen by
// rr_small / pp_small from the large-block count of one grid or a group)
unsigned rr_blocks(const Grid& g, int cmask, bool small);
unsigned pp_blocks(const Grid& g, bool small);
bool rr_small(unsigned big_blocks);
bool pp_small(unsigned big_blocks);
// coarse values staged in LDS by one prolongation block (grid's mask)
unsigned pp_stage_elems(int cmask, bool small);
unsigned gemv_blocks(int n);
template <class M>
hipError_t launch_spmv_group(int pat, bool res, const SpmvArgs<M>* segs, const unsigned* bmap, unsigned nblocks,
                             const int* live, hipStream_t st);
template <class M>
hipError_t launch_rr_group(int pat, bool small, const RRArgs<M>* segs, const unsigned* bmap, unsigned nblocks,
                           const int* live, hipStream_t st);
// stage_elems: the largest pp_stage_elems of the segments (0 when every ec is null)
template <class M>
hipError_t launch_pp_group(int pat, bool full, bool small, unsigned stage_elems, const PPArgs<M>* segs,
                           const unsigned* bmap, unsigned nblocks, const int* live, hipStream_t st);
template <class V>
hipError_t launch_gemv_group(const GemvArgs<V>* segs, const unsigned* bmap, unsigned nblocks, const int* live,
                             hipStream_t st);

// ---- parallel stencil kernels (stencil.hip) ----------------------------
// y = A x   (res = false)   or   y = b - A x   (res = true)
template <class M>
hipError_t launch_spmv(int pat, const Grid& g, const M& m, const typename M::V* x, const typename M::V* b,
                       typename M::V* y, bool res, hipStream_t st);

// rc = R (f - A u), R = P^T trilinear, coarsening mask cmask
template <class M>
hipError_t launch_resid_restrict(int pat, const Grid& g, int cmask, const M& m, const typename M::V* f,
                                 const typename M::V* u, typename M::V* rc, hipStream_t st);

// With u_old = u + P ec (ec may be null: u_old = u):
//   full = false: h = f - sum_{lower s} a_s u_old[nbr]    (input of the backward GS sweep)
//   full = true : h = f - A u_old, and uold_out = u_old   (input of the ILU correction)
template <class M>
hipError_t launch_prolong_post(int pat, const Grid& g, int cmask, const M& m, const typename M::V* f,
                               const typename M::V* u, const typename M::V* ec, typename M::V* h,
                               typename M::V* uold_out, bool full, hipStream_t st);

// h = f - sum_{lower s} a_s u[nbr] (canonical order, fma): the input of a
// backward Gauss-Seidel sweep from the old values u
template <class M>
hipError_t launch_lower(int pat, const Grid& g, const M& m, const typename M::V* f, const typename M::V* u,
                        typename M::V* h, hipStream_t st);
// h = f - sum_{upper s} a_s u[nbr]: the input of a forward sweep from old values u
template <class M>
hipError_t launch_upper(int pat, const Grid& g, const M& m, const typename M::V* f, const typename M::V* u,
                        typename M::V* h, hipStream_t st);

// plain restriction / prolongation (kernel-level entry points)
template <class V>
hipError_t launch_restrict(const Grid& g, int cmask, int bs, const V* rf, V* rc, hipStream_t st);
template <class V>
hipError_t launch_prolong_add(const Grid& g, int cmask, int bs, const V* ec, V* uf, hipStream_t st);

// cell-centred piecewise-constant pair (cell.hip): coarse cell I owns fine
// cells 2I + {0,1} on coarsened axes, n_c = ceil(n_f / 2); rc = P^T rf,
// uout = uin + P ec (uout may be uin), A_c = R A P on the fine pattern
template <class V>
hipError_t launch_restrict_cc(const Grid& gf, int cmask, int bs, const V* rf, V* rc, hipStream_t st);
template <class V>
hipError_t launch_prolong_cc(const Grid& gf, int cmask, int bs, const V* ec, const V* uin, V* uout, hipStream_t st);
hipError_t launch_rap_cc(int pat, int cmask, const Grid& gf, const double* A, long sA, double* Ac, long sAc,
                         hipStream_t st);
// cell-centred trilinear interpolation (3d64c; same grid map): uout = uin + P ec,
// and the 27-point product of the Cell_3d8 restriction, A and this P
template <class V>
hipError_t launch_prolong_c64(const Grid& gf, int cmask, int bs, const V* ec, const V* uin, V* uout,
                              hipStream_t st);
hipError_t launch_rap_c64(int pat, int cmask, const Grid& gf, const double* A, long sA, double* Ac, long sAc,
                          hipStream_t st);

// operator-dependent vertex interpolation (od.hip): weights W (8 per fine
// point) from the level's stencil, rc = P^T rf, uout = uin + P ec (uout may
// be uin), and the 27-point product P^T A P (scalar systems)
hipError_t launch_od_weights(int pat, const Grid& g, int cmask, const double* A, double* W, unsigned* err,
                             hipStream_t st);
template <class V>
hipError_t launch_restrict_od(const Grid& gf, int cmask, const V* W, const V* rf, V* rc, hipStream_t st);
template <class V>
hipError_t launch_prolong_od(const Grid& gf, int cmask, const V* W, const V* ec, const V* uin, V* uout,
                             hipStream_t st);
hipError_t launch_rap_od(int pat, int cmask, const Grid& gf, const double* A, const double* W, double* Ac,
                         hipStream_t st);

// ---- block (3x3) variants (block.hip) --------------------------------
// y = A x or y = b - A x on 3x3 blocks (27-point pattern)
template <class M>
hipError_t launch_bspmv(const Grid& g, const M& m, const typename M::V* x, const typename M::V* b,
                        typename M::V* y, bool res, hipStream_t st);
// h = f - sum over lower neighbour blocks of A_ij u_j (input of the backward block sweep)
template <class M>
hipError_t launch_blower(const Grid& g, const M& m, const typename M::V* f, const typename M::V* u,
                         typename M::V* h, hipStream_t st);
// h = f - sum over upper neighbour blocks (input of a forward block sweep from old values u)
template <class M>
hipError_t launch_bupper(const Grid& g, const M& m, const typename M::V* f, const typename M::V* u,
                         typename M::V* h, hipStream_t st);
// point-block Gauss-Seidel sweep on 8 x 8-column tiles (WfArgs.pk: launch_bwf_pack data of this direction)
void bwf_tiling(const Grid& g, WfTiling* t);
int bwf_pack_count(int ebytes);
template <class E>
hipError_t launch_bwavefront(int dir, const WfArgs<typename WfVal<E>::V>& a, hipStream_t st);
template <class E>
hipError_t launch_bwf_pack(const Grid& g, const WfTiling& tl, int dir, const double* A, const double* Dinv, E* out,
                           hipStream_t st);
hipError_t launch_bwf_pack_h(const Grid& g, const WfTiling& tl, int dir, const __half* a16, const float* sc,
                             const float* rd, void* out, hipStream_t st);

// ---- setup (setup.hip) ------------------------------------------------
hipError_t launch_copy_masked(int pat, const Grid& g, int be, const double* src, double* dst, hipStream_t st);
// rd_i = w / a_ii (the diagonal factor of the GS sweeps with weight w)
hipError_t launch_recip_diag(int pat, const Grid& g, const double* A, double w, double* rd, unsigned* err,
                             hipStream_t st);
// qa_i = (V)(q * a_ii): the old-centre coefficient q = (1 - w) / w of a weighted sweep
template <class V>
hipError_t launch_centre_scaled(int pat, const Grid& g, const double* A, double q, V* qa, hipStream_t st);
// Sums of |a| over the couplings along x, y and z (the two face offsets of
// each axis, in-grid neighbours only): one triple per workgroup of a fixed
// grid of AXIS_BLOCKS, part[3 * b + axis]
constexpr int AXIS_BLOCKS = 256;
hipError_t launch_axis_coupling(int pat, const Grid& g, const double* A, double* part, hipStream_t st);
hipError_t launch_block_dinv(const Grid& g, const double* A, double* Dinv, unsigned* err, hipStream_t st);
// ILU(0) factors on the mask pattern pm of A (pattern pa); L and U hold the
// mask's slots, U holds pm*N + 2 doubles (the last two are set to {0, 1} and
// read where a coupling or pivot is unused)
// Levels of at most ILU_SMALL_POINTS points are factored in one
// workgroup (one launch), larger ones with one launch per hyperplane; both
// give the same bits.
constexpr long ILU_SMALL_POINTS = 4096;
hipError_t launch_ilu0_factor(int pa, int pm, const Grid& g, const double* A, double* L, double* U, double* rU,
                              unsigned* err, hipStream_t st);
// Line Gauss-Seidel over z-columns (lgs.hip).  Tiles of K x K columns in
// sheared (x, y + sh*x) coordinates are the work units, taken in the order of
// tmap (ntile entries bx << 16 | by'); x holds the sentinel until written;
// uold: values before the sweep (null for the zero-guess forward sweep);
// next: buffer given the sentinel (or null).
constexpr int LGS_MAX_GRID = 512;
constexpr int LGS_MAX_NZ = 2047;
template <class V>
struct LgsArgs {
  Grid g;
  const V* A;
  const V* rden;
  const V* cp;
  const V* f;
  const V* uold;
  V* x;
  V* next;
  int K, ntile;
  const int* tmap;
  unsigned* ctr;
  unsigned* err;
};
// tile side K and the tiles holding columns in dependence order (tmap may
// be null: count only); returns their number
int lgs_plan(const Grid& g, int pat, int* K, std::vector<int>* tmap);
size_t lgs_lds_bytes(const Grid& g, int K, int vbytes);
hipError_t launch_tri_factor(int pat, const Grid& g, const double* A, double* rden, double* cp, unsigned* err,
                             hipStream_t st);
template <class V>
hipError_t launch_lgs(int pat, int dir, bool zero_guess, const LgsArgs<V>& a, hipStream_t st);
hipError_t launch_to_f32(const double* src, float* dst, long n, hipStream_t st);
hipError_t launch_to_f16_rowscale(const double* A, long N, int S, int bs, __half* h, float* sc, hipStream_t st);
hipError_t launch_dequant_f16(const __half* h, const float* sc, long N, int S, int bs, float* out, hipStream_t st);
template <class V>
hipError_t launch_fill_bits(V* p, long n, V v, hipStream_t st);

// ---- RAP (rap.hip, generated chains) --------------------------------
// Ac[(n*be + e)*Nc + I] for the 27 coarse offsets; A entry stride sA elements.
hipError_t launch_rap(int pat, int cmask, const Grid& gf, const double* A, long sA, double* Ac, long sAc,
                      hipStream_t st);
int rap_chain_count(int pat, int cmask);

// ---- coarsest level (coarse.hip) ------------------------------------
hipError_t launch_dense_assemble(const Grid& g, int pat, int bs, const double* A, double* M, int ld,
                                 hipStream_t st);
hipError_t launch_aug_init(int n, double* aug, hipStream_t st);
// aug: n x 2n [A | I] followed by coarse_invert_extra(n) doubles of work
// space; the inverse ends in the right half (Gauss-Jordan, partial pivoting)
long coarse_invert_extra(int n);
hipError_t coarse_invert(int n, double* aug, int* info_dev, hipStream_t st);
template <class V>
hipError_t launch_coarse_gemv(int n, const double* Ainv, int ld, const V* f, V* u, hipStream_t st);

// ---- vectors and reductions (vec.hip) --------------------------------
hipError_t launch_axpy(long n, double a, const double* x, double* y, hipStream_t st);   // y = fma(a, x, y)
hipError_t launch_xpby(long n, const double* x, double b, double* y, hipStream_t st);   // y = fma(b, y, x)
hipError_t launch_scale(long n, double s, const double* x, double* y, hipStream_t st);  // y = s * x
hipError_t launch_dot(long n, const double* x, const double* y, double* partial, double* out, hipStream_t st);
hipError_t launch_cast_d2f(long n, const double* x, float* y, hipStream_t st);
hipError_t launch_cast_f2d(long n, const float* x, double* y, hipStream_t st);
hipError_t launch_add(long n, const double* a, const double* b, double* y, hipStream_t st);
template <class V>
hipError_t launch_vfma(long n, const V* a, const V* x, V* y, hipStream_t st);  // y_i = fma(a_i, x_i, y_i)
constexpr int DOT_BLOCKS = 1024;
// Sum over a 256-thread workgroup in a fixed order (wavefront shuffles, then
// the four wave sums pairwise); the result is valid in thread 0.
__device__ inline double block_sum(double v) {
  __shared__ double red[4];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = (red[0] + red[1]) + (red[2] + red[3]);
  return s;
}

// ---- device-resident PCG (vec.hip) ------------------------------------
// The scalars of preconditioned CG (Sec. 5.2) live in a small device block
// s[] so that an iteration needs no host round trip: alpha, beta and the
// convergence tests are formed on the device with the host loop's formulas,
// and the vector kernels below skip their work unless s[PS_STATE] == 0.
// States: iterating, recurrence residual below tolerance (the true residual
// is checked next), converged, iteration limit, breakdown (p.Ap <= 0).
enum PcgSlot {
  PS_RHO = 8, PS_PQ, PS_RR, PS_RZ, PS_BN, PS_ALPHA, PS_NALPHA, PS_BETA, PS_RECUR, PS_REL, PS_STATE, PS_IT,
  PS_MAXIT, PS_RTOL, PS_GATE, PS_END
};
constexpr double PCG_ITERATING = 0.0, PCG_CHECK = 1.0, PCG_DONE = 2.0, PCG_LIMIT = 3.0, PCG_BREAKDOWN = 4.0;
hipError_t launch_pcg_start(double* s, double bn, int it, int maxit, double rtol, hipStream_t st);
hipError_t launch_pcg_alpha(double* s, hipStream_t st);        // limit and breakdown tests, alpha = rho / p.q
hipError_t launch_pcg_recur(double* s, hipStream_t st);        // it += 1, recurrence residual test
hipError_t launch_pcg_true(double* s, hipStream_t st);         // true residual test after the check
hipError_t launch_pcg_beta(double* s, hipStream_t st);         // beta = r.z / rho, rho = r.z
// y = fma(*a, x, y) / y = fma(*b, y, x) where *state == 0
// x += alpha p, r -= alpha q (while iterating) and rr = r.r, with s the PCG
// slots (PS_ALPHA, PS_NALPHA, PS_STATE); the dot's bits equal launch_dot's
hipError_t launch_pcg_update(long n, const double* s, const double* p, const double* q, double* x, double* r,
                             double* partial, double* rr, hipStream_t st);

hipError_t launch_xpby_dev(long n, const double* x, const double* b, const double* state, double* y, hipStream_t st);
// launch_dot where *gate != 0 (out unchanged otherwise)
hipError_t launch_dot_gated(long n, const double* x, const double* y, double* partial, double* out,
                            const double* gate, hipStream_t st);
// residual y = b - A x of the finest level where *gate != 0 (y unchanged otherwise)
hipError_t launch_spmv_res_gated(int pat, const Grid& g, const MatD& m, const double* x, const double* b, double* y,
                                 const double* gate, hipStream_t st);
hipError_t launch_bspmv_res_gated(const Grid& g, const BMatD& m, const double* x, const double* b, double* y,
                                  const double* gate, hipStream_t st);

}  // namespace smg
