/*
 * structmg.h -- C ABI of libstructmg, an MI355X (gfx950) implementation of
 * the structured algebraic multigrid preconditioner of "StructMG: A Fast and
 * Scalable Structured Algebraic Multigrid" (arXiv 2506.21932).
 *
 * The user supplies only the finest-level matrix and right-hand sides
 * (Sec. 4.2.2, input data format); the hierarchy is built once and applied
 * many times (Sec. 2, total-time equation).  One application of the
 * preconditioner is one V-cycle (Sec. 2): pre-smoothing, residual and
 * restriction, coarse correction, prolongation, post-smoothing.
 *
 * Conventions shared by every entry point
 *   Grid (nx, ny, nz); linear index i = (x*ny + y)*nz + z (z contiguous).
 *   Stencil patterns 3d7 / 3d19 / 3d27 with offsets in {-1,0,1}^3 (Sec. 4.2.3
 *   masks), numbered lexicographically with dx slowest (the Offset(2d9) /
 *   Offset(2d5) numbering of Sec. 4.3 extended to 3D).
 *   Matrix storage "SG-DIA" (Sec. 4.1 P1): coefficient of row i for offset s
 *   at coeffs[s*N + i], N = nx*ny*nz.  Block systems (block = 3 unknowns per
 *   node): entry (r, c) of the 3x3 block of offset s at coeffs[(s*9 + r*3 + c)*N + i],
 *   vectors interleaved v[i*3 + c].  Couplings to neighbours outside the
 *   grid are ignored (Dirichlet elimination; the paper zero-pads them).
 *   Pointers named "device" are HIP device memory owned by the caller;
 *   "stream" is a hipStream_t (NULL = default stream).
 *
 * Ownership: the library never allocates device memory.  Every hierarchy
 *   array lives in the caller's workspace (size from smg_workspace_size),
 *   which the handle borrows until smg_destroy.  coeffs may be freed once
 *   smg_setup has returned.
 *
 * Errors: every call returns an smg_status; nothing aborts.  A failed call
 *   leaves a message for smg_last_error.  Handles are not thread-safe, and
 *   calls on one handle must not overlap in time (they share its workspace).
 */
#ifndef STRUCTMG_H
#define STRUCTMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smg_handle_s* smg_handle;

typedef enum {
  SMG_OK = 0,
  SMG_ENOTCONV = 1,    /* iteration limit reached; results still filled in */
  SMG_EINVAL = -1,     /* invalid argument or configuration */
  SMG_ENOMEM = -2,     /* workspace too small */
  SMG_EDEVICE = -3,    /* HIP runtime error */
  SMG_EBREAKDOWN = -4, /* zero pivot / zero diagonal, or p.Ap <= 0 in CG */
  SMG_EDEADLOCK = -5   /* wavefront watchdog fired (a wait did not finish) */
} smg_status;

typedef enum { SMG_SMOOTH_GS = 0, SMG_SMOOTH_ILU0 = 1, SMG_SMOOTH_LGS = 2 } smg_smoother;
typedef enum { SMG_COARSEN_FULL = 0, SMG_COARSEN_SEMI_XY = 1, SMG_COARSEN_AUTO = 2 } smg_coarsen;
typedef enum { SMG_FP64 = 0, SMG_FP32 = 1, SMG_FP16_ROWSCALE = 2 } smg_prec;
typedef enum {
  SMG_INTERP_VERTEX = 0,
  SMG_INTERP_CELL = 1,
  SMG_INTERP_CELL_TRILINEAR = 2,
  SMG_INTERP_OPERATOR = 3
} smg_interp;

typedef struct {
  int nx, ny, nz;      /* finest grid */
  int block;           /* unknowns per node: 1, or 3 (3x3 blocks, 27-point only) */
  int pattern;         /* finest-level pattern: 7, 19 or 27; coarse levels are 27-point */
  int smoother;        /* smg_smoother: symmetric point GS (forward before, backward
                          after the coarse correction), ILU(0) on each level's mask, or
                          symmetric line GS over z-columns (Sec. 4.4: column right-hand
                          side from the neighbouring columns, Thomas solve per column;
                          scalar systems, FP64 or FP32, nz <= 2047) */
  int coarsen;         /* smg_coarsen: coarsen x,y,z (full), only x,y (semi), or x,y while
                          the level's z coupling stays weak (auto, Sec. 4.1 P2 fixed-stride
                          coarsening chosen per level): with rho the ratio of the finest
                          matrix's summed |z-face couplings| to the mean of its summed
                          |x-face| and |y-face| couplings, level l coarsens x,y only while
                          rho * 4^l < 1/4 (x,y coarsening by 2 scales the relative z
                          coupling by 4), then x,y,z; scalar systems.  smg_workspace_size
                          then returns the largest size over the possible choices, and
                          smg_resetup keeps the coarsening chosen at setup */
  int semi_levels;     /* with SMG_COARSEN_FULL: the first semi_levels levels coarsen x,y only */
  int prec;            /* smg_prec of the V-cycle matrices and vectors; the outer
                          Krylov method, its operator, dot products, true residuals
                          and the coarsest solve stay FP64 */
  int max_coarse;      /* bound on the unknowns of the dense coarsest level (0: 4096) */
  int gmres_restart;   /* Krylov basis reserved in the workspace for GMRES (0: none) */
  int ilu_mask;        /* ILU(0) only: positions kept by the factorisation of the finest
                          matrix (Sec. 4.2.3 ILU masks): 0 = its own pattern, or the
                          7 / 19 / 27-point mask (fewer or more fill-ins than the
                          matrix pattern); coarse levels keep their 27-point pattern */
  int interp;          /* smg_interp: vertex-centred trilinear P with R = P^T, coarse
                          X <-> fine 2X+1, n_c = floor(n_f/2), 27-point coarse levels; or
                          the cell-centred piecewise-constant pair (table of R/A/P
                          combinations, Cell_3d8 interpolation and restriction): coarse
                          cell I owns fine cells 2I, 2I+1 per coarsened axis,
                          n_c = ceil(n_f/2), R = P^T, every level keeps the finest
                          pattern; or that restriction with cell-centred trilinear
                          interpolation (Cell_3d64: 3/4 from the parent cell, 1/4 from
                          the neighbour on the fine cell's side, per axis), 27-point
                          coarse levels, R != P^T (use GMRES unless A is benign); or
                          operator-dependent vertex interpolation (the weights of the
                          generated triple product vary per point, after Dendy): the
                          vertex grid map, each fine point between coarse points takes
                          its weights from its stencil collapsed onto the directions
                          it is not aligned with, R = P^T, 27-point coarse levels.
                          Cell-centred and operator-dependent transfers take scalar
                          systems. */
  /* Smoothing settings (Sec. 4.4 GS / ILU formulas; settings table: ZeroGuess,
   * relax weight 1.0).  Zero in any of these fields selects the default. */
  int pre_sweeps;      /* smoothing steps before the coarse correction, 1..8 (0: 1); GS
                          directions alternate forward, backward, ... */
  int post_sweeps;     /* after it, 1..8 (0: 1); GS directions alternate starting opposite
                          to the last pre-sweep, so pre_sweeps == post_sweeps gives a
                          symmetric V-cycle */
  double relax_weight; /* weight w of the point GS sweeps, 0 < w < 2 (0: 1.0):
                          u += w (D + w L)^-1 (b - A u) forward, (D + w U)^-1 backward.
                          Computed as a GS sweep with diagonal factor w / a_ii on the
                          right-hand side b + ((1 - w) / w) a_ii u_old (the same update in
                          exact arithmetic).  Point GS only (scalar systems); ILU(0) has
                          no weight, line GS and 3x3 blocks take w = 1 */
  int zero_guess;      /* 0 or 1 (default): the first pre-smoothing step starts from u = 0
                          and reads only the lower triangle and diagonal (ZeroGuess);
                          -1: that step applies the full stencil to u = 0 (same values up
                          to the sign of zero, more traffic) */
  int min_coarse;      /* an axis of n points is coarsened while n >= 2 * min_coarse,
                          2..4096 (0: 4) */
} smg_config;

typedef struct {
  int iters;               /* preconditioner applications in the Krylov loop */
  int levels;              /* multigrid levels */
  double rel_resid_true;   /* ||b - A x||_2 / ||b||_2 recomputed in FP64 at the end */
  double rel_resid_recur;  /* the Krylov method's own residual estimate at exit, over ||b||_2:
                              the recursively updated PCG residual, or |g_{j+1}| of the last
                              GMRES step (batched solves: the recursive PCG residual) */
  double grid_complexity;  /* sum n_l / n_0          (Sec. 2, complexity equation) */
  double op_complexity;    /* sum S_l n_l / (S_0 n_0): stored structured entries */
  double t_setup_ms;
  double t_solve_ms;
  int host_waits;          /* times the solve waited for the device: PCG keeps its scalars on
                              the device and reads its state once per batch of iterations
                              (one per iteration only near convergence); GMRES once per
                              inner product */
} smg_result;

/* Workspace bytes needed for cfg.  Returns SMG_EINVAL for an unsupported cfg. */
smg_status smg_workspace_size(const smg_config* cfg, size_t* bytes);

/* Builds the hierarchy: copies the finest matrix (device, FP64, SG-DIA as
 * above), forms every coarse operator with the stencil Galerkin product
 * A_c = R A P (Sec. 4.3; trilinear P, R = P^T), the smoother data (1/a_ii,
 * 3x3 block inverses or ILU(0) factors), truncated copies for reduced
 * V-cycle precision, and the inverse of the dense coarsest operator.
 * Synchronises `stream` before returning.  SMG_EBREAKDOWN on a zero pivot. */
smg_status smg_setup(const smg_config* cfg, const double* coeffs, void* workspace, size_t bytes, void* stream,
                     smg_handle* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): smg_setup with
 * the hierarchy placed in a static device array of SMG_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends, instead of a
 * caller workspace.  Calls no hipMalloc / hipFree.  SMG_ENOMEM (nothing
 * touched on the device) when smg_workspace_size(cfg) exceeds the array
 * (7-point scalar grids beyond about 40^3).  Every call on one device
 * builds its hierarchy in that device's one array: a call invalidates the
 * handles of earlier smg_setup_noalloc calls on the same device (destroy them
 * with smg_destroy), and calls or uses of such handles that overlap in time
 * race.  Synchronises `stream`. */
#define SMG_SCRATCH_BYTES ((size_t)64 << 20)
smg_status smg_setup_noalloc(const smg_config* cfg, const double* coeffs, void* stream, smg_handle* out);

/* Rebuilds the hierarchy of an existing handle for new finest-level
 * coefficients with the same grid, pattern and settings (same workspace).
 * Synchronises `stream`.  A failure leaves the handle unusable until the next
 * successful smg_resetup. */
smg_status smg_resetup(smg_handle h, const double* coeffs, void* stream);

/* z = M^-1 r: one V-cycle (device FP64 vectors of N*block entries; r and z
 * must not overlap).  Asynchronous on `stream`. */
smg_status smg_precondition(smg_handle h, const double* r, double* z, void* stream);

/* Solves A x = b with preconditioned CG (krylov = 0) or right-preconditioned
 * restarted GMRES(krylov) (krylov <= cfg.gmres_restart) in its flexible form
 * (the preconditioned basis vectors are kept and combined into the update;
 * for an exactly linear V-cycle this is plain right-preconditioned GMRES, and
 * with an FP32 / FP16 V-cycle the recurrence residual stays the true one).
 * PCG forms its scalars (rho, alpha, beta) and its convergence tests on the
 * device with the same arithmetic as a host loop, so the iterates do not
 * depend on how many iterations the host enqueues between reads of the
 * state.  x holds the initial
 * guess on entry.  Stops when ||r||_2 / ||b||_2 < rtol for the true residual
 * (settings table: relative tolerance).  Synchronises `stream`.
 * SMG_ENOTCONV when maxit is reached (res still filled in). */
smg_status smg_solve(smg_handle h, const double* b, double* x, double rtol, int maxit, int krylov, smg_result* res,
                     void* stream);

smg_status smg_destroy(smg_handle h);

/* PCG in smg_solve replays one captured HIP graph per V-cycle (1, default;
 * captured at the first solve, not used while kernel timing is on) or
 * launches the V-cycle's kernels one by one (0).  Results are identical. */
smg_status smg_set_graph(smg_handle h, int enable);

/* Tile shape of the wavefront sweep of one level (the columns a workgroup
 * owns): 1 sheared (y offset by x, the default for 19/27-point levels with
 * more than one tile row), 2 rectangular 16 x 16 (the default otherwise), 0
 * the default rule.  The sweep's results do not depend on it (every shape
 * runs the sequential lexicographic order; Sec. 4.4), only its time.
 * Rectangles of a 19/27-point sweep with more than one tile row are refused
 * (tiles of one tile column would wait on each other).  Re-packs the level's
 * sweep data and resets its sentinels; synchronises `stream`.  SMG_EINVAL for
 * the coarsest level, 3x3 block systems, line GS, a shape outside 0..2 or
 * that refused case. */
smg_status smg_set_tile_shape(smg_handle h, int level, int shape, void* stream);
/* Current tile shape of a level (1 or 2), 0 where the level has no tiled sweep. */
int smg_tile_shape(smg_handle h, int level);

/* Message of the last failed call on h (or of the last failed setup when h is
 * NULL).  Never NULL. */
const char* smg_last_error(smg_handle h);

/* ---- hierarchy introspection ------------------------------------------ */
/* info[0..5] = nx, ny, nz, pattern points, coarsening mask to the next level
 * (bit 0 x, bit 1 y, bit 2 z; 0 on the coarsest level), block. */
smg_status smg_level_info(smg_handle h, int level, int* info);
int smg_num_levels(smg_handle h);

/* Copies level data into device memory dst (stream-ordered):
 * what = 0 matrix (FP64, S*block^2*N), 1 reciprocal diagonal (FP64, N) or
 * 3x3 diagonal-block inverses (FP64, 9*N), 2 ILU lower factor (FP64, S*N),
 * 3 ILU upper factor (FP64, S*N; on the finest level S is the ILU mask's
 * points when cfg.ilu_mask is set), 4 reciprocal of the ILU diagonal (FP64, N),
 * 5 V-cycle matrix (FP32; FP16 storage is expanded to scale*float(h)),
 * 6 V-cycle reciprocal diagonal / block inverses (FP32), 7 line GS Thomas
 * reciprocal pivots (FP64, N), 8 line GS Thomas c/pivot (FP64, N),
 * 9 operator-dependent interpolation weights to the next level (FP64, 8*N:
 * weight c of fine point i at [c*N + i]). */
smg_status smg_level_export(smg_handle h, int level, int what, void* dst, void* stream);

/* Influence chains of the generated triple product for a (fine pattern,
 * coarsening mask) pair per interior coarse element (Table of chain counts). */
int smg_rap_chain_count(int pattern, int cmask);

/* ---- single V-cycle steps on one level --------------------------------
 * These run the same kernels as the V-cycle.  Vectors are device arrays in
 * the V-cycle precision (double for SMG_FP64, float otherwise) of the level's
 * size (times block).  Output arrays must not overlap inputs. */
smg_status smg_op_spmv(smg_handle h, int level, const void* x, void* y, void* stream);          /* y = A_l x */
smg_status smg_op_spmv_fp64(smg_handle h, const double* x, double* y, void* stream);           /* finest, FP64 */
/* One smoothing step with the handle's weight, whatever pre_sweeps and
 * post_sweeps hold.
 * u = S_pre(f): forward GS or line GS sweep from u = 0, or the ILU(0) solve. */
smg_status smg_op_presmooth(smg_handle h, int level, const void* f, void* u, void* stream);
/* u_out = S_post(f, u_in + P e_c): backward GS or line GS sweep, or the
 * ILU(0) correction, after prolongation of the coarse correction e_c (level
 * l+1 vector, NULL for none). */
smg_status smg_op_postsmooth(smg_handle h, int level, const void* f, const void* u_in, const void* ec, void* u_out,
                             void* stream);
/* rc = R (f - A_l u): fused residual and restriction to level l+1. */
smg_status smg_op_resid_restrict(smg_handle h, int level, const void* f, const void* u, void* rc, void* stream);
smg_status smg_op_restrict(smg_handle h, int level, const void* rf, void* rc, void* stream);
smg_status smg_op_prolong_add(smg_handle h, int level, const void* ec, void* uf, void* stream);
/* u = A_L^-1 f on the coarsest level (FP64 inverse). */
smg_status smg_op_coarse_solve(smg_handle h, const void* f, void* u, void* stream);

/* ---- kernel timing (profiling aid) --------------------------------------
 * When enabled, each kernel of the V-cycle and the outer FP64 SpMV on the
 * selected level and of the selected kinds (bit k of `kinds` for kind k) is
 * bracketed by HIP events on its launch stream (at most 16384 launches are
 * recorded between reports).  smg_timing_report synchronises on the events,
 * then fills ms[level*8 + kind] (milliseconds summed over launches) and
 * counts[...] (number of launches) for levels < max_levels, and clears the
 * record.  Kinds: 0 pre-smoothing sweep (GS forward / ILU lower), 1 ILU upper
 * pre-smoothing sweep, 2 residual + restriction, 3 coarsest solve,
 * 4 prolongation + post-smoother input, 5 post-smoothing sweep (GS backward /
 * ILU lower), 6 ILU upper post-smoothing sweep, 7 outer FP64 SpMV. */
smg_status smg_set_timing(smg_handle h, int enable, int level /* -1: all */, unsigned kinds /* bit mask */);
smg_status smg_timing_report(smg_handle h, double* ms, int* counts, int max_levels, int* dropped);

/* ---- batches of independent systems -------------------------------------
 * Many independent scalar systems (GS smoother; one pattern and one V-cycle
 * precision for all; grids may differ) solved together: each system has its
 * own hierarchy, built exactly as by smg_setup, and all systems advance in
 * lockstep through preconditioned CG, every step being one launch over all
 * systems; a system stops at its own convergence (per-system tolerance test
 * as in smg_solve).  Four lockstep iterations run as one captured HIP graph,
 * and the host reads the systems' flags once per graph; a system stops on the
 * device at its convergence or at maxit.
 * Pointer arrays are host arrays of nsys device pointers.  At most 4095
 * systems. */
typedef struct smg_batch_s* smg_batch;

/* Workspace bytes for the batch (every cfgs[k] as for smg_workspace_size). */
smg_status smg_batch_workspace_size(int nsys, const smg_config* cfgs, size_t* bytes);

/* Builds the nsys hierarchies into one workspace (borrowed until
 * smg_batch_destroy).  Synchronises `stream`. */
smg_status smg_batch_setup(int nsys, const smg_config* cfgs, const double* const* coeffs, void* workspace,
                           size_t bytes, void* stream, smg_batch* out);

/* z[k] = M_k^-1 r[k] for every system: one batched V-cycle (each system's
 * result equals smg_precondition on that system).  Synchronises `stream`. */
smg_status smg_batch_precondition(smg_batch b, const double* const* r, double* const* z, void* stream);

/* Solves A_k x[k] = bv[k] for all k by lockstep PCG (x[k]: initial guess on
 * entry).  results / status (optional host arrays of nsys) receive each
 * system's outcome: SMG_OK, SMG_ENOTCONV or SMG_EBREAKDOWN.  Returns SMG_OK
 * when all converged, otherwise the worst per-system status.  Synchronises. */
smg_status smg_batch_solve(smg_batch b, const double* const* bv, double* const* x, double rtol, int maxit,
                           smg_result* results, int* status, void* stream);

/* Sweep schedule: merge order of the systems' tiles (0: system after system,
 * 1: round robin) and persistent grid of the batched sweeps (workgroups, one
 * per CU at most: larger values act as 256; 0: 256). */
smg_status smg_batch_set_schedule(smg_batch b, int order, int grid);
/* Times batched V-cycles for every (order, grid) candidate and keeps the
 * fastest, then, level by level, the faster tile shape of the level's sweeps
 * (sheared or rectangular; smg_batch_tile_shape reports the choice); returns
 * the order, grid and time per V-cycle (ms) of the final choice.  Results
 * do not depend on any of these choices.  Overwrites the internal residual
 * vectors (not the caller's). */
smg_status smg_batch_tune(smg_batch b, void* stream, int* order, int* grid, double* ms_per_vcycle);
/* Tile shape of the sweeps of one level in every system (as
 * smg_set_tile_shape); synchronises `stream`. */
smg_status smg_batch_set_tile_shape(smg_batch b, int level, int shape, void* stream);
int smg_batch_tile_shape(smg_batch b, int level);
/* Replays a captured graph of four lockstep iterations (1, default) or
 * launches the iterations' kernels one by one (0). */
smg_status smg_batch_set_graph(smg_batch b, int enable);
int smg_batch_num_systems(smg_batch b);
/* The hierarchy of system k (owned by the batch; for introspection and the
 * single-system entry points). */
smg_handle smg_batch_system(smg_batch b, int k);
smg_status smg_batch_destroy(smg_batch b);
const char* smg_batch_last_error(smg_batch b);

#ifdef __cplusplus
}
#endif
#endif
