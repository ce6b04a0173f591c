/*
 * ell.h -- C ABI of an MI355X (gfx950) solver for the 3D anisotropic elliptic
 * pressure-correction equation of Mueller & Scheichl, "Massively parallel
 * solvers for elliptic PDEs in Numerical Weather- and Climate Prediction"
 * (arXiv:1307.2036):
 *
 *     -omega^2 ( Lap_2d u + d/dz( lambda^2(z) du/dz ) ) + u = f        (Sec. 3)
 *
 * on nx x ny x nz cells that are doubly periodic in the horizontal, with
 * homogeneous Neumann conditions at the bottom and top.  The discretisation
 * is the cell-centred finite-volume 7-point stencil (Sec. 3.1); the solver is
 * conjugate gradients (Appendix B, Alg. "Preconditioned Conjugate Gradient
 * method") preconditioned by one tensor-product multigrid V-cycle (Sec. 4.3,
 * Alg. "Multigrid V-cycle"; Sec. 4.3.1 and 6.2.1): vertical line relaxation
 * (block red/black SOR over columns, each column solved by the Thomas
 * algorithm of Appendix B), horizontal-only coarsening, sum restriction and
 * bilinear prolongation, re-discretised coarse operators.
 *
 * Conventions shared by every entry point
 *  - Vectors passed to ell_apply_A, ell_vcycle and ell_pcg_solve are DEVICE
 *    pointers to nx*ny*nz doubles in plane-major layout,
 *    idx = (k*ny + j)*nx + i.  The caller owns them.
 *  - "Level" entry points (ell_level_*) work on the library's internal
 *    colour-split layout of one multigrid level (see ell_to_split) and on the
 *    grid's internal element type: double for ELL_FP64, float otherwise.
 *  - The grid owns all of its hierarchy and workspace memory.  Calls on one
 *    grid must not overlap: they share that workspace.  Calls are enqueued on
 *    the given stream; ell_apply_A, ell_vcycle and the level entry points
 *    return without synchronising, ell_pcg_solve returns when the solve is
 *    complete because it fills host statistics.
 *  - Return value: ELL_OK (0) on success, a negative ELL_ERR_* code on error
 *    (outputs untouched or partially written; message in ell_last_error()),
 *    ELL_NOT_CONVERGED (+1) from ell_pcg_solve when maxiter was reached with a
 *    valid u.
 */
#ifndef ELL_H
#define ELL_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ell_grid ell_grid;

enum {
    ELL_OK = 0,
    ELL_NOT_CONVERGED = 1,
    ELL_PENDING = 2,
    ELL_ERR_INVALID = -1,   /* bad argument or descriptor                     */
    ELL_ERR_OOM = -2,       /* device allocation failed                       */
    ELL_ERR_HIP = -3,       /* a HIP runtime call failed                      */
    ELL_ERR_NUMERIC = -4,   /* non-finite alpha, beta or residual norm        */
    ELL_ERR_BUDGET = -5     /* request larger than a memory budget            */
};

/* Arithmetic of the V-cycle preconditioner.  The outer CG (dots, residual,
 * solution update) is always FP64. */
enum {
    ELL_FP64 = 0,           /* FP64 everywhere                                */
    ELL_FP32_PRECOND = 1,   /* FP32 V-cycle, FP64 coefficients rounded to FP32 */
    ELL_FP32_BF16COEF = 2   /* FP32 V-cycle, stencil coefficients rounded to
                               BF16, Thomas factors computed in FP32 from them */
};

/* Grid and multigrid description (Sec. 3, 3.1, 4.3, 6.2.1). */
typedef struct {
    int32_t nx, ny, nz;      /* cells; nx and ny must each be even or 1        */
    double hx, hy;           /* horizontal spacings (> 0)                      */
    double omega2;           /* omega^2 >= 0 (eq. omega2lambda2)               */
    const double *dz;        /* HOST array of nz layer thicknesses (> 0); copied */
    const double *lambda2;   /* HOST array of nz cell values of lambda^2 (> 0);
                                copied.  Vertical face coefficients use the
                                harmonic (series-resistance) rule.            */
    int32_t n_levels;        /* multigrid levels incl. the finest; 0 = standard
                                depth: halve nx, ny while both are even and each
                                half is even or 1                              */
    int32_t nu_pre, nu_post; /* red/black sweeps before / after the coarse
                                correction (paper: 1 and 1)                    */
    int32_t nu_coarse;       /* sweeps on the coarsest level (paper: 1, or 5
                                for its four-level variant, Sec. 7.3.1)        */
    double rho;              /* SOR relaxation factor, 0 < rho < 2 (1 = plain) */
    int32_t prolong;         /* 0 = bilinear (paper), 1 = piecewise constant   */
    int32_t precision;       /* ELL_FP64, ELL_FP32_PRECOND, ELL_FP32_BF16COEF  */
} ell_grid_desc;

typedef struct {
    double rtol;             /* stop when ||r_K|| < rtol * ||r_0|| ...         */
    double atol;             /* ... or ||r_K|| < atol (Appendix B, PCG)        */
    int32_t maxiter;         /* > 0                                            */
    int32_t flexible;        /* 1: beta = <z_K, r_K - r_{K-1}> / <z_{K-1}, r_{K-1}>
                                (robust to a non-symmetric V-cycle);
                                0: beta = <r_K,z_K>/<r_{K-1},z_{K-1}> as printed */
    int32_t rel_to_rhs;      /* 1: the relative test uses ||b|| = ||V f||
                                instead of ||r_0|| (warm starts)               */
    int32_t poll_every;      /* iterations enqueued between host polls of the
                                device-side convergence flag; 0 = default (4).
                                Does not change the result.                   */
} ell_solve_opts;

typedef struct {
    int32_t iters;           /* completed CG iterations K                      */
    int32_t status;          /* ELL_OK, ELL_NOT_CONVERGED or ELL_ERR_NUMERIC   */
    double r0_norm;          /* ||b - A u_0||                                  */
    double r_norm;           /* ||r_K|| of the CG recurrence                   */
    double true_r_norm;      /* ||b - A u_K|| recomputed in FP64 at the end    */
    double b_norm;           /* ||b||, b = V f                                 */
} ell_solve_stats;

/* Build the level hierarchy: coefficient tables and Thomas factors for every
 * level (Sec. 6.2.1: only O(nz) numbers per level, nothing per column) and
 * all device work space.  Synchronous.  *out receives the new grid. */
int ell_grid_create(const ell_grid_desc *desc, ell_grid **out);
int ell_grid_destroy(ell_grid *g);

/* A grid whose vertical coefficient lambda^2 varies horizontally too: the
 * model equation of Sec. 3 with lambda^2(x, y, z), a step from the paper's
 * lambda^2(r) toward its panel geometry, whose metric terms differ from column
 * to column (Sec. 3, Sec. 6.2.1).  lambda2_3d: HOST array of nx*ny*nz cell
 * values (> 0, finite), plane-major, copied; desc->lambda2 is not read (it may
 * be NULL).  Every column gets its own vertical faces (the harmonic rule of
 * ell_grid_desc.lambda2, column by column) and its own Thomas factors; a coarse
 * column's face is the sum of its four children's (parallel faces; for a
 * horizontally constant lambda^2 this is the re-discretised face exactly).
 * desc->precision is ELL_FP64 or ELL_FP32_PRECOND (ELL_BF16COEF returns
 * ELL_ERR_INVALID).  The grid works with every grid entry point (ell_apply_A,
 * ell_vcycle, ell_pcg_solve, ell_mg_solve, the level entry points); its sweeps
 * run k-segmented column kernels, which also carry the fused CG residual
 * update and dots (ELL_FEAT_FUSED_UPDATE, ELL_FEAT_FUSED_DOTS); the LDS-tiled
 * sweeps, the fused prolongation and the tiled ends do not apply.  It holds
 * three FP64 fields per level
 * (faces, 1/p_k, T_{k+1/2}/p_k) more than ell_grid_bytes reports, and with
 * ELL_FP32_PRECOND their FP32 copies too, which the FP32 sweeps and
 * restrictions read (the FP64 finest post-smoothing reads the FP64 fields);
 * the operator step and the solve's ends read the FP64 faces.  The batch engine does not take such
 * grids.  Synchronous; ELL_ERR_INVALID for a bad descriptor or field. */
int ell_grid_create_varying(const ell_grid_desc *desc, const double *lambda2_3d, ell_grid **out);

/* Device bytes ell_grid_create would allocate for desc (0 if invalid). */
size_t ell_grid_bytes(const ell_grid_desc *desc);

/* Number of multigrid levels of the grid (>= 1), or a negative error. */
int ell_grid_levels(const ell_grid *g);

/* Which fused forms the grid's CG solves (ell_pcg_solve) take, as a bit mask
 * in *mask: ELL_FEAT_TILED_SMOOTH (the finest level's half-sweeps after the
 * first stage neighbours in LDS tiles), ELL_FEAT_FUSED_DOTS (the CG inner
 * products ride on the last two post-smoothing half-sweeps),
 * ELL_FEAT_FUSED_UPDATE (the residual update r -= alpha q rides on the first
 * pre-smoothing pair), ELL_FEAT_FUSED_PROLONG (the finest prolongation rides
 * on the first post-smoothing sweep),
 * ELL_FEAT_TILED_ENDS (a solve's start, r = V f - A u0, and end, the final
 * update and true residual, run on LDS tiles), ELL_FEAT_COARSE_TAIL (the
 * coarsest level's sweeps run in one cooperative launch; cleared if the
 * runtime refused that launch, the sweeps then run one by one),
 * ELL_FEAT_COARSE_PROLONG (on at least one coarse level the bilinear
 * prolongation rides on the first post-smoothing sweep, as the finest one
 * does: FP64, rho = 1, LDS-tiled sweeps; any beta), ELL_FEAT_COARSE_PAIR (each
 * of the coarsest level's sweep pairs runs in one launch: every block sweeps
 * colour 0 on its 8 x 8 tile and the ring around it, keeps that in LDS and
 * sweeps colour 1 on the tile; rho = 1, constant coefficients, nx and ny
 * multiples of 8).  They change
 * where bytes move and how many launches there are, not what is computed;
 * a benchmark's byte model reads them.  Returns ELL_OK or a negative error. */
enum {
  ELL_FEAT_TILED_SMOOTH = 1,
  ELL_FEAT_FUSED_DOTS = 2,
  ELL_FEAT_FUSED_UPDATE = 4,
  ELL_FEAT_FUSED_PROLONG = 8,
  ELL_FEAT_TILED_ENDS = 16,
  ELL_FEAT_COARSE_TAIL = 32,
  ELL_FEAT_COARSE_PROLONG = 64,
  ELL_FEAT_COARSE_PAIR = 128
};
int ell_grid_features(const ell_grid *g, int32_t *mask);

/* y = A x: the operator of eq. ModelEquation integrated over every cell
 * (cell volume V = hx*hy*dz_k), so A is symmetric positive definite.
 * x, y: device, plane-major, nx*ny*nz doubles, must not alias. */
int ell_apply_A(ell_grid *g, const double *x, double *y, hipStream_t stream);

/* y = A x without a grid object and without allocating device memory, for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  desc describes the grid as for
 * ell_grid_create (validated the same way; its multigrid and precision fields
 * do not change the result); x, y: device, plane-major, nx*ny*nz doubles,
 * must not alias; the values are those ell_apply_A gives for a grid created
 * from desc.  The finest level's stencil coefficients (4 x (nz+1) doubles) go
 * into a fixed library-owned device area of 32.8 KB per GPU, held until the
 * process ends; nz > ELL_NOALLOC_MAX_NZ returns ELL_ERR_INVALID.  No hipMalloc,
 * hipFree, host-to-device copy or other allocating call is made: the
 * coefficients travel in kernel arguments.  All calls on one GPU share that
 * area: calls on one stream are ordered, calls that overlap on one GPU
 * (several streams or host threads) race.  Asynchronous like ell_apply_A. */
#define ELL_NOALLOC_MAX_NZ 1024
int ell_apply_A_noalloc(const ell_grid_desc *desc, const double *x, double *y, hipStream_t stream);

/* z = M^{-1} r: one V-cycle (Alg. "Multigrid V-cycle") from a zero initial
 * guess with right-hand side r.  Runs in the grid's precision; r and z are
 * FP64 device vectors, plane-major, must not alias. */
int ell_vcycle(ell_grid *g, const double *r, double *z, hipStream_t stream);

/* Solve A u = V f by preconditioned CG (Appendix B) with one V-cycle as the
 * preconditioner.  f: device, the per-volume right-hand side; u: device, the
 * initial guess on entry and the solution on return.  opts may be NULL
 * (rtol 1e-5, flexible, maxiter 500).  stats may be NULL. */
int ell_pcg_solve(ell_grid *g, const double *f, double *u, const ell_solve_opts *opts,
                  ell_solve_stats *stats, hipStream_t stream);

/* Stand-alone multigrid (Sec. 4.3, the V-cycle iterated as a solver, as the
 * paper runs its geometric multigrid in Sec. 7.3): u_K = u_{K-1} + M r_{K-1},
 * r_K = r_{K-1} - A M r_{K-1}, from the caller's u_0, stopped like
 * ell_pcg_solve (same options, opts->flexible ignored; same statistics,
 * return codes, ownership and synchronisation; true_r_norm is the FP64
 * ||b - A u|| of the returned u).  The residual is carried by the recurrence:
 * on strongly graded grids the recomputed b - A u has a rounding floor above
 * practical tolerances. */
int ell_mg_solve(ell_grid *g, const double *f, double *u, const ell_solve_opts *opts,
                 ell_solve_stats *stats, hipStream_t stream);

/* ---- level entry points (the V-cycle's kernels one at a time) ------------
 * Colour-split layout of level l (nx_l = nx >> l, ny_l = ny >> l): element
 * (i, j, k) of colour c = (i+j) mod 2 lives at c*C + k*S + m, where
 * m = j*(nx_l/2) + i/2 (m = j/2 when nx_l = 1) runs over the H =
 * ceil(nx_l*ny_l/2) columns of the colour, S >= H is the padded plane stride
 * and C >= nz*S the colour stride (see ell_level_layout).  Padding entries
 * are zero and never written.  Element type: double for ELL_FP64 grids,
 * float otherwise. */
size_t ell_level_elems(const ell_grid *g, int level);  /* 2*C; 0 if invalid */
int ell_level_layout(const ell_grid *g, int level, int64_t *cols, int64_t *plane_stride,
                     int64_t *colour_stride);

/* plane-major FP64 -> split / split -> plane-major FP64 conversion */
int ell_to_split(ell_grid *g, int level, const double *src, void *dst, hipStream_t stream);
int ell_from_split(ell_grid *g, int level, const void *src, double *dst, hipStream_t stream);

/* One colour of block SOR (Sec. 4.2 eq. BlockRBSOR) on level l: every column
 * of colour c gets its vertical tridiagonal system solved with the other
 * colour's values on the right-hand side.  zero_init = 1 asserts u = 0 on
 * entry (neighbour and old values are then not read). */
int ell_level_smooth(ell_grid *g, int level, int colour, int zero_init, const void *b, void *u,
                     hipStream_t stream);

/* bc = R (b - A_l u): residual on level l summed over each 2x2 block of
 * children into level l+1 (Alg. "Multigrid V-cycle", restriction step).
 * black_zero = 1 asserts that the residual vanishes on colour-1 columns (true
 * right after a colour-1 sweep with rho = 1); those columns are skipped. */
int ell_level_resid_restrict(ell_grid *g, int level, const void *b, const void *u, void *bc,
                             int black_zero, hipStream_t stream);

/* u += P uc: interpolation from level l+1 to level l (bilinear 9/3/3/1 or
 * piecewise constant, per the grid).  red_only = 1 updates colour-0 columns
 * only (the colour-1 values are about to be overwritten by a rho = 1 sweep). */
int ell_level_prolong_add(ell_grid *g, int level, const void *uc, void *u, int red_only,
                          hipStream_t stream);

/* y = A_l x on level l in the split layout. */
int ell_level_apply(ell_grid *g, int level, const void *x, void *y, hipStream_t stream);

/* ---- measurement -----------------------------------------------------------
 * Kernel timing with HIP events recorded on the launch stream around each
 * launch of one kernel family during subsequent calls (up to max_events
 * launches).  Families: ELL_K_SMOOTH0 (finest-level line relaxation),
 * ELL_K_APPLY (CG operator application), ELL_K_RESTRICT0, ELL_K_PROLONG0,
 * ELL_K_UPDATE (CG vector update). */
enum { ELL_K_SMOOTH0 = 0, ELL_K_APPLY = 1, ELL_K_RESTRICT0 = 2, ELL_K_PROLONG0 = 3,
       ELL_K_UPDATE = 4, ELL_K_COUNT = 5 };
int ell_profile_enable(ell_grid *g, int family, int max_events);
/* Pause (paused != 0) or resume the recording of a family enabled above; the
 * events already recorded are kept.  Each recorded launch costs two event
 * records on the stream (a few microseconds of idle GPU each), so a caller
 * that times a long run can record a sample of its launches. */
int ell_profile_pause(ell_grid *g, int family, int paused);
/* Synchronises the recorded events; *count launches, *total_ms summed time. */
int ell_profile_read(ell_grid *g, int family, int *count, double *total_ms);
/* Per-launch times in milliseconds of the recorded launches, in launch order:
 * writes min(count, cap) values to ms (host array) and returns the count, or a
 * negative error.  Launches enqueued after the solve converged return at once
 * and show up as near-zero times. */
int ell_profile_times(ell_grid *g, int family, float *ms, int cap);

/* Tuning for grids created afterwards (process-wide): padding, in elements,
 * added to the plane stride S and to the colour stride C; k-segments (1, 2
 * or 4) of the column-walking CG operator kernels; APPLY_TILE 1 (default) runs
 * the CG operator step of grids with nx, ny > 1 on LDS-staged horizontal
 * tiles, 0 on the column-walking kernel; BATCH_GRAPH 1 (default) makes batch
 * engines created afterwards replay each grouped step from a captured HIP
 * graph, 0 launches the kernels directly (same results, bitwise); SMOOTH_TILE
 * 1 (default) stages neighbour values in LDS tiles for the half-sweeps after
 * the first on every level (FP64, and FP32 on the coarse levels of the
 * mixed-precision V-cycle; rho = 1, nx/2 and ny even, even plane and colour
 * strides) and for the bilinear colour-0 prolongation (ny even), 0 uses the
 * column kernels (same values, bitwise); FUSED_DOT 1 (default) lets the finest level's last two
 * post-smoothing half-sweeps of a CG preconditioner application (tiled, with
 * at least two levels) also form the partial sums of <r, z> (and <z, q> for
 * the flexible beta) that the next CG scalar needs, in place of a separate
 * pass over r, z (and q); 0 always uses the separate pass (the same values up
 * to the order of the summation); FUSED_UPDATE 1 (default) lets the finest
 * level's first pre-smoothing pair of a CG preconditioner application also
 * carry the residual update r -= alpha q and the partial sums of ||r||^2 (the
 * convergence test runs between that pair and the rest of the V-cycle), in
 * place of a separate pass over r and q; 0 always uses the separate pass;
 * FUSED_PROLONG 1 (default) lets the finest level's first post-smoothing sweep
 * of an FP64 V-cycle (one post-smoothing sweep, bilinear prolongation, fused
 * dots, either beta) apply the coarse correction to the colour-0 values it
 * reads instead of a prolongation pass (the colour-0 sweep that follows
 * overwrites them), the colour-0 sweep then forming <r, z> (and, with the
 * flexible beta, <z, q>) of both colours, and does the same on every coarse FP64 level with
 * LDS-tiled sweeps and rho = 1 (any beta; same values, bitwise), and lets the
 * mixed-precision V-cycle's first FP64 post-smoothing sweep of the finest
 * level (colour 1, LDS-tiled, bilinear prolongation) read the FP32 colour-0
 * values and the FP32 coarse correction and form the values the prolongation
 * pass would write into the FP64 output (any beta; bitwise the same); 0 always
 * runs the prolongation pass; TILED_ENDS 1
 * (default) runs the start of a solve (us = u0, r = V f - A u0) and its end (u
 * = us + alpha p written plane-major, the true residual) on the LDS tiles of
 * the operator step for grids created afterwards with nx, ny > 1, 0 on the
 * column kernels (u and r the same bitwise, the norms up to summation
 * order); COARSE_TAIL 1 runs the coarsest level's nu_coarse sweep pairs of
 * every V-cycle (Alg. "Multigrid V-cycle", coarsest-level solve) in one
 * cooperative launch with grid-wide barriers between the half-sweeps, where
 * that level's sweeps are the 8- or 16-segment kernels (rho = 1, both
 * horizontal directions, segments of at most 16 levels); 0 (default) launches
 * them one by one (the same values, bitwise; on MI355X a barrier across the
 * eight XCDs costs more than a kernel boundary, so one launch per half-sweep
 * is faster); COARSE_PAIR 1 (default) runs each of those sweep pairs in one
 * launch where ELL_FEAT_COARSE_PAIR applies, 0 as two half-sweeps (the same
 * values, bitwise). */
enum {
  ELL_TUNE_PLANE_PAD = 0,
  ELL_TUNE_COLOUR_PAD = 1,
  ELL_TUNE_STENCIL_SEG = 2,
  ELL_TUNE_APPLY_TILE = 3,
  ELL_TUNE_BATCH_GRAPH = 4,
  ELL_TUNE_SMOOTH_TILE = 5,
  ELL_TUNE_FUSED_DOT = 6,
  ELL_TUNE_FUSED_UPDATE = 7,
  ELL_TUNE_FUSED_PROLONG = 8,
  ELL_TUNE_TILED_ENDS = 9,
  ELL_TUNE_COARSE_TAIL = 10,
  ELL_TUNE_COARSE_PAIR = 11
};
int ell_set_tuning(int key, int value);

/* ---- schedule autotuning (beyond the paper) ---------------------------------
 * A schedule fixes how a grid of one shape runs on the chip, not what it
 * computes (every schedule gives the same iterates up to rounding order): the
 * CG operator step's kernel (LDS-tiled or column-walking) and its k-segments,
 * and the line smoother's k-segments on every level (4 or 8 on the finest
 * level, 8 where a segment then holds at most 16 levels; 4, 8 or 16 on the
 * coarse ones).  Schedules are kept process-wide per shape (nx, ny, nz,
 * number of levels, FP64 or mixed precision); a grid created afterwards uses
 * the schedule recorded for its shape, else the built-in heuristics.  Batch
 * grids take the operator-step part only (their smoother layout is uniform).
 * Thread-safe. */
#define ELL_MAX_LEVELS 16
typedef struct {
  int32_t apply_tile;                  /* 1: LDS-tiled operator step, 0: column-walking */
  int32_t apply_nseg;                  /* k-segments of the operator step: 1, 2 or 4 */
  int32_t smooth_nseg[ELL_MAX_LEVELS]; /* per level: line-smoother k-segments, 4, 8 or 16
                                          (entry 0 is 4 or 8; entries past the last level 0) */
  double ms_per_iter;                  /* ell_autotune: measured milliseconds per PCG
                                          iteration of the chosen schedule; otherwise 0 */
} ell_schedule;
/* Autotuner: times fixed-iteration PCG solves (iters iterations from u = 0,
 * rtol 0, f a fixed pseudo-random field; median of three) of a grid of this
 * shape under candidate schedules, by coordinate descent: the operator step
 * first (tiled with 1, 2 or 4 segments, column-walking with 1, 2 or 4), then
 * each coarse level's smoother segments.  A candidate replaces the current
 * one only if it is at least 1% faster.  Records the winner for the shape and
 * writes it to *best (host struct).  iters <= 0 means 4.  Allocates and frees
 * its own device memory: one grid of the shape and two vectors at a time.
 * Synchronises the device. */
int ell_autotune(const ell_grid_desc *desc, int32_t iters, ell_schedule *best);
/* The schedule a grid of this shape would get now (recorded or heuristic). */
int ell_schedule_get(const ell_grid_desc *desc, ell_schedule *out);
/* Records a schedule for this shape after validating it; NULL clears the
 * record (back to the heuristics). */
int ell_schedule_set(const ell_grid_desc *desc, const ell_schedule *s);

/* ---- batched solves and serving (beyond the paper) ---------------------------
 * A batch engine advances many solves together: every stage of a CG iteration
 * (operator step, residual update, each V-cycle half-sweep, restriction and
 * prolongation, dots, scalar updates) is one launch covering all active grids,
 * each grid with its own CG state on the device.  A worker thread admits
 * submitted requests and retires finished ones between iterations, so requests
 * that arrive while others run join at the next iteration (continuous
 * batching).  Grids of a batch are created by the batch (four or eight
 * k-segments per coarse level, so a level's grouped launch takes at most two
 * block shapes), count against its HBM budget and must all be FP64 or all use the
 * FP32 preconditioner; they need rho = 1, nu >= 1, nx, ny > 1 on every level
 * and nz <= 256.  Requests on one grid run one after another (warm starts:
 * pass the previous solution as u). */
typedef struct ell_batch ell_batch;

/* hbm_budget_bytes: upper bound on the device bytes of the batch's grids. */
int ell_batch_create(size_t hbm_budget_bytes, ell_batch **out);
/* Create a grid owned by the batch; ELL_ERR_BUDGET if it does not fit. */
int ell_batch_grid(ell_batch *b, const ell_grid_desc *desc, ell_grid **out);
/* Destroy an idle grid of the batch and return its bytes to the budget. */
int ell_batch_release(ell_batch *b, ell_grid *g);
size_t ell_batch_bytes_in_use(const ell_batch *b);
/* Enqueue n solves A u_i = V f_i (device vectors, plane-major, valid until
 * the ticket completes); returns at once with a ticket. */
int ell_batch_submit(ell_batch *b, int32_t n, ell_grid *const *grids, const double *const *f,
                     double *const *u, const ell_solve_opts *opts, uint64_t *ticket_out);
/* ELL_PENDING while any solve of the ticket runs; otherwise the combined
 * status and n statistics (stats may be NULL). */
int ell_batch_poll(ell_batch *b, uint64_t ticket, ell_solve_stats *stats);
/* Block until the ticket completes, fill stats, release the ticket. */
int ell_batch_wait(ell_batch *b, uint64_t ticket, ell_solve_stats *stats);
/* Finish queued work, then free the batch and its grids. */
int ell_batch_destroy(ell_batch *b);

/* Message of the last error on the calling thread ("" if none). */
const char *ell_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ELL_H */
