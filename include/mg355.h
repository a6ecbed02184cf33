/*
 * mg355.h -- C ABI of the MI355X (gfx950) geometric multigrid Poisson solver.
 *
 * Solves  nabla^2 phi = 4 pi G rho  (eq. poisson of Tomida & Stone, arXiv:2302.13903,
 * Sec. 2.1) on a uniform cubic grid of n^3 cells with the 7-point cell-centred Laplacian
 * (eq. discretized2), by full multigrid (Alg. 2) followed by V(npre, npost) correction-
 * scheme cycles (Alg. 1) with the over-relaxed red-black Gauss-Seidel smoother
 * (eqs. rbsor1-2), 8-cell restriction (eq. restriction), trilinear correction
 * prolongation (eq. trilinear) and tricubic FMG prolongation (Sec. 2.3.1), the convergence
 * test of Sec. 2.3.7 and the boundary conditions of Sec. 2.3.6 and Appendix A.
 *
 * Conventions shared by every entry point:
 *   - Grid arrays are contiguous, x fastest: element (i, j, k) at ((k*n + j)*n + i);
 *     cell (i, j, k) is centred at ((i+1/2) dx, (j+1/2) dx, (k+1/2) dx); the domain is
 *     [0, n dx]^3.
 *   - Face order: -x, +x, -y, +y, -z, +z.  A face array is indexed [t2][t1] over the face's
 *     two transverse axes in increasing axis order (x faces: (y, z); y faces: (x, z);
 *     z faces: (x, y)), t1 fastest.
 *   - "Device" pointers are HIP device memory on the context's device; "host" pointers
 *     are ordinary host memory.  Every device pointer is caller-owned: the library neither
 *     frees nor retains it after the call returns.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on it; calls
 *     that return host values (residual history, moments) synchronise that stream.
 *   - Return value: MG_OK (0); a positive soft status (the output is valid, see below);
 *     or a negative error (nothing valid was written; mg_last_error() explains).
 *   - A context is not re-entrant: one host thread at a time per context.
 */
#ifndef MG355_H
#define MG355_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------- */
#define MG_OK 0
#define MG_NOT_CONVERGED 1   /* max_cycles reached above tol; phi holds the last iterate */
#define MG_STALLED 2         /* residual fell < 10 % per cycle twice in a row (round-off floor) */
#define MG_ERR_INVALID_ARG -1
#define MG_ERR_UNSUPPORTED -2
#define MG_ERR_OOM -3
#define MG_ERR_DEVICE -4
#define MG_ERR_NONFINITE -5  /* NaN/Inf in rho or in fixed face values */

/* ---- boundary kinds (Sec. 2.3.6, Appendix A) -------------------------------------- */
#define MG_BC_PERIODIC 0       /* ghost = opposite active cell; must be set on both faces of an axis */
#define MG_BC_ZERO_GRADIENT 1  /* ghost = adjacent active cell */
#define MG_BC_FIXED 2          /* ghost = 2 b - adjacent cell: the value on the face equals b */
#define MG_BC_MULTIPOLE 3      /* FIXED with b from the l <= lmax multipole expansion of rho */

#define MG_MODE_FMG 0          /* full multigrid start (Alg. 2), then V-cycles */
#define MG_MODE_MGI 1          /* V-cycles from the initial guess held in phi */

#define MG_PREC_FP64 0         /* every operator in FP64 */
#define MG_PREC_MIXED 1        /* FP32 smoothing / restriction / prolongation inside FP64
                                  defect-correction (FP64 residual and phi update) */

#define MG_SCHEME_CS 0         /* V-cycles in the correction scheme (Alg. 1)             */
#define MG_SCHEME_FAS 1        /* Full Approximation Scheme iterations (Alg. 3; FMG with FAS,
                                  Sec. 2.3.5): every level solves for the potential with its
                                  own physical boundary values; on this linear problem it
                                  reaches the correction scheme's iterates up to rounding.
                                  FP64 and the dense layout only (else MG_ERR_UNSUPPORTED). */

#define MG_LAYOUT_DENSE 0      /* one n^3 array per level, x fastest */
#define MG_LAYOUT_BLOCKS 1     /* MeshBlock decomposition (Sec. 3.2): rho and phi hold
                                  (n/block_n)^3 blocks of block_n^3 cells, blocks in Morton
                                  order of their coordinates (bits of bx, by, bz interleaved,
                                  x lowest), each block x fastest.  Block levels are coarsened
                                  to one cell per block; those cells form the dense root grid.
                                  block_n in {2, 4, 8, 16}. */

typedef struct mg_ctx mg_ctx;

/* Solver parameters.  mg_default_params() fills the defaults given in brackets. */
typedef struct {
  int n;            /* cells per side: a power of two, 2 <= n <= 2048                   [-] */
  double dx;        /* cell width, > 0                                                  [1/n] */
  double four_pi_g; /* 4 pi G; the source is f = four_pi_g * rho                        [4 pi] */
  int mode;         /* MG_MODE_FMG or MG_MODE_MGI                                       [FMG] */
  int npre, npost;  /* smoothing sweeps before / after the coarse correction, 0..4     [2, 2] */
  double omega;     /* over-relaxation factor of the smoother, 0 < omega < 2            [1.15] */
  double tol;       /* stop when RMS(defect)/RMS(f) <= tol (finest level)               [1e-10] */
  int max_cycles;   /* V-cycle cap after the FMG sweep, 0..1000                         [50] */
  int fixed_cycles; /* > 0: run exactly this many V-cycles and ignore tol               [0] */
  int precision;    /* MG_PREC_FP64 or MG_PREC_MIXED                                    [FP64] */
  int layout;       /* MG_LAYOUT_DENSE or MG_LAYOUT_BLOCKS                              [DENSE] */
  int block_n;      /* MeshBlock side for MG_LAYOUT_BLOCKS (2..16, power of two, < n)   [16] */
  int scheme;       /* MG_SCHEME_CS or MG_SCHEME_FAS                                    [CS] */
} mg_params;

/* Boundary description of a solve. */
typedef struct {
  int kind[6];               /* MG_BC_* per face */
  const double *fixed_b[6];  /* device, n*n face-centre values per FIXED face; NULL = 0 */
  int lmax;                  /* multipole order 0..4 (Appendix A)                        */
  int use_origin;            /* 0: expansion about the centre of mass; 1: about origin[] */
  double origin[3];
} mg_bc;

/* Boundary description of one level for the operator entry points: face kinds and
 * extended face arrays of (nl+2)^2 values (device, indexed [t2+1][t1+1], t = -1..nl;
 * the outer ring gives the values used for edge and corner ghosts); NULL = 0.
 * MG_BC_MULTIPOLE faces are treated as MG_BC_FIXED with the given arrays. */
typedef struct {
  int kind[6];
  const double *b[6];
} mg_level_bc;

void mg_default_params(mg_params *p);

/* Create a context on HIP device `device`.  The workspace grows on demand and is reused.
 * hbm_budget caps the device bytes the context may hold (hierarchy workspace, operator and
 * autotuner scratch, reduction scratch; mg_footprint_bytes gives what a solve needs): a call
 * that would need more returns MG_ERR_OOM without allocating.  0 = no cap.  Returns
 * MG_ERR_OOM when the budget cannot hold the context's fixed reduction scratch, and
 * MG_ERR_DEVICE when the device cannot be used. */
int mg_ctx_create(mg_ctx **ctx, int device, size_t hbm_budget);
void mg_ctx_destroy(mg_ctx *ctx);
const char *mg_last_error(const mg_ctx *ctx);

/* Device bytes a solve with these parameters keeps resident in its context (hierarchy,
 * boundary arrays, reduction scratch); 0 for invalid parameters.  Used for admission. */
size_t mg_footprint_bytes(const mg_params *p);

/* Size the context's workspace for solves with these parameters now (one allocation), so
 * that later solves of the same or smaller size allocate nothing.  MG_ERR_OOM when the
 * device cannot hold it (the previous workspace is then released). */
int mg_ctx_reserve(mg_ctx *ctx, const mg_params *p);

/* Autotuner.  For every level of a solve with these parameters it times the alternative
 * schedules over `reps` launches on scratch arrays and keeps the fastest in the context;
 * later solves use it.
 *   MG_LAYOUT_BLOCKS: the block sweep (threads per workgroup, blocks staged per workgroup,
 *     one or two sweeps fused per launch; every such schedule gives bitwise the same result)
 *     and, on the finest block level, whether the streaming passes that cross block
 *     boundaries replace the per-block halo-tile sweeps (with V(2,2) from 128 cells per side:
 *     the two-sweep down and up passes against four halo-tile sweeps; otherwise, from 256
 *     cells per side, the one-sweep passes against one halo-tile sweep).
 *   MG_LAYOUT_DENSE (n >= 64): whether the restricted defect (and, on the FP64 finest level,
 *     the residual norm) is fused into the last smoothing pass or runs as its own streaming
 *     pass, and whether sweeps run one per pass or two per pass (temporally blocked).  The
 *     alternatives differ only in floating-point contraction (same expressions).
 * Allocates and frees its own scratch (3.25 n^3 values); synchronises its own stream. */
int mg_autotune(mg_ctx *ctx, const mg_params *p, int reps);

/* The context's schedules as text, one line each: "blk fp64|fp32 Lm Lb threads G S"
 * (Lm = log2 block side on that level, Lb = log2 blocks per side) and
 * "pass fp64|fp32 l split" (level l = log2 n_l; split bit 0: defect pass separate, bit 1:
 * norm pass separate), "fusedmin fp64|fp32 n" (smallest level size swept by the fused
 * z-marching passes, a power of two >= 64; smaller levels run one launch per operator) and
 * "tail fp64|fp32 l" (highest level, 1..4, solved by the single-workgroup LDS tail) and
 * "tb fp64|fp32 0|1" (1: large-level sweeps two per pass over HBM) and "blkz fp64|fp32 0|1"
 * (MeshBlock layout, 1: streaming passes across blocks on the large block levels) and
 * "march fp64|fp32 0|1|2" (V(2,2) legs of the levels >= 128^3, or >= the fusedmin size when
 * that was set larger, as two streaming passes -- down: two sweeps + restricted defect; up:
 * prolongation + two sweeps + norm -- 0 off, 1 when every face is periodic, 2 always (default))
 * and "tile fp64|fp32 0|1" (1, the default: with V(2,2), each leg of the levels 32^3 .. 128^3
 * that the streaming passes do not take runs as one region-tile launch) and "split fp64 0|1"
 * (1, the default: an FP64 streaming pass of a level with x or y walls runs its interior tiles
 * and its wall tiles as two launches on the context's second stream and the caller's, joined
 * before the pass returns; 0: one launch; the serving runtime sets 0) and "inner fp32 k"
 * (precision MG_PREC_MIXED on grids above the LDS tail: k = 1..4 FP32 V-cycles per outer
 * defect-correction step, each outer step then contracting the residual as k V-cycles do;
 * unset: chosen per step, see mg_last_inner).  Writes at most cap bytes (NUL-terminated) and returns the length
 * needed including the NUL.  mg_tuning_set reads the same format (e.g. from a cache file)
 * and rejects schedules the device cannot run. */
int mg_tuning_get(const mg_ctx *ctx, char *buf, int cap);
int mg_tuning_set(mg_ctx *ctx, const char *text);

/* Full solve (Sec. 2.3.7, Alg. 1, Alg. 2).
 *   rho   device, n^3 FP64, read only.
 *   phi   device, n^3 FP64; output (and the initial guess when mode = MG_MODE_MGI).
 *         When no face is FIXED or MULTIPOLE the mean of f and of phi is removed.
 *   hist  host, capacity max(max_cycles, fixed_cycles) + 1: the relative residual after
 *         the FMG sweep (or of the initial guess) and after each V-cycle.
 *   n_hist host: number of entries written.
 * Waits once per cycle for the stopping test, which runs on the host: the device publishes the
 * cycle's norm to pinned host memory and the calling thread spins until it arrives (one CPU
 * core stays busy during the solve); the next cycle's first pass may already be queued on
 * `stream` by then.  Returns after synchronising `stream`. */
int mg_solve(mg_ctx *ctx, const mg_params *p, const mg_bc *bc, const double *rho, double *phi,
             double *hist, int *n_hist, void *stream);

/* mg_solve for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same solve, the same kernels and
 * the same results, but the hierarchy workspace, reduction partials and device scalars live
 * in the library's static device scratch -- one 64 MiB array per device, held until the
 * process ends -- and the call makes no hipMalloc/hipFree or other allocation (and records
 * no per-cycle or kernel timing events: mg_last_timing reports set-up and FMG only).  The
 * context must exist already (mg_ctx_create allocates).
 *   Limit: footprint + reduction scratch <= 64 MiB, which holds every precision, layout and
 *   scheme up to n = 128; larger solves return MG_ERR_OOM with nothing written.
 *   Every call on one device shares that device's scratch and leaves the last call's contents
 *   in it (each solve clears what must start at zero): calls that overlap on one device --
 *   on different streams, contexts or host threads -- race and give undefined results.
 * Arguments, outputs and status as for mg_solve. */
int mg_solve_noalloc(mg_ctx *ctx, const mg_params *p, const mg_bc *bc, const double *rho, double *phi,
                     double *hist, int *n_hist, void *stream);

/* Short form of mg_solve (Sec. 2.3.7, Alg. 1, Alg. 2) with the defaults of mg_default_params:
 * FMG start, V(2,2) cycles, omega = 1.15, four_pi_g = 4 pi, FP64, dense layout, at most 50
 * cycles.  All six faces take bc_kind (MG_BC_*): FIXED faces hold b = 0; MULTIPOLE faces the
 * l <= 4 expansion about the centre of mass (Appendix A).
 *   n     cells per side (power of two, 2..2048); dx > 0; tol > 0 (relative residual).
 *   rho   device, n^3 FP64, read only;  phi  device, n^3 FP64, output.
 *   hist  host, capacity 51: the relative residual after FMG and after each V-cycle;
 *   n_hist host: entries written.
 * Returns as mg_solve. */
int mg_solve_simple(mg_ctx *ctx, int n, const double *rho, int bc_kind, double dx, double tol, double *phi,
                    double *hist, int *n_hist, void *stream);

/* Timing of the last mg_solve on this context, from HIP events on its stream:
 * *fmg_ms = set-up + FMG sweep; cycle_ms[c] = wall time of V-cycle c (including its
 * residual norm); *n = number of cycles (up to cap). */
int mg_last_timing(const mg_ctx *ctx, double *setup_ms, double *fmg_ms, double *cycle_ms,
                   int cap, int *n);

/* FP32 V-cycles the last mg_solve on this context ran inside its outer defect-correction
 * steps (precision MG_PREC_MIXED; 0 for FP64).  Each outer step is one entry of the residual
 * history and runs "inner fp32 k" V-cycles when that tuning line is set; otherwise, in a
 * solve to a tolerance, as many as the residual contraction per V-cycle observed so far
 * (taken 1.5 times as slow) says are still needed to reach it, at most 3 (one per step in a
 * fixed-cycle solve).
 *   inner_cycles  host int, output.
 * Returns MG_ERR_INVALID_ARG for a null argument. */
int mg_last_inner(const mg_ctx *ctx, int *inner_cycles);

/* Kernel-level timing of the finest-level smoothing kernels of the V-cycles of the last
 * mg_solve, from HIP events on the solve stream: a pass that is one kernel carries its events
 * in its own dispatch (its start and end), a pass split over two streams has events recorded
 * around both launches.  Enabled by mg_set_kernel_timing(ctx, 1); off by default (each timed
 * dispatch costs the device a few microseconds between kernels).
 * Entry `index` (0-based, one per kernel name): launch count, summed duration (ms), the
 * algorithmic HBM bytes of one launch, and the kernel name (as the profiler lists it).
 * Returns MG_ERR_INVALID_ARG past the last entry. */
int mg_set_kernel_timing(mg_ctx *ctx, int on);
int mg_kernel_timing(const mg_ctx *ctx, int index, int *launches, double *total_ms,
                     double *bytes_per_launch, char *name, int name_cap);

/* Multipole set-up (Appendix A): centre of mass (unless use_origin) and the 25 moments
 * Q_lm, l <= lmax, of rho (device, n^3) with cell volume dx^3.  origin_out (host, 3) and
 * q_out (host, 25, index l*l + l + m) receive the results. */
int mg_multipole_moments(mg_ctx *ctx, int n, double dx, const double *rho, int lmax, int use_origin,
                         const double *origin, double *origin_out, double *q_out, void *stream);

/* Gravitational acceleration g = -grad phi (eq. acceleration) in the cell-centred
 * source-term scheme of Sec. 2.4, from the potential of a solve:
 *   face   g_{x,i-1/2} = (phi_{i-1} - phi_i) / dx   (likewise y, z), where a potential
 *          across the domain surface is the ghost of the solve's boundary rule: periodic
 *          -> the opposite cell; zero-gradient -> the adjacent cell (face value 0); fixed
 *          and multipole -> 2 b - adjacent cell (face value (b - phi_0) / (dx/2));
 *   cell   g_x = (g_{x,i-1/2} + g_{x,i+1/2}) / 2;
 *   source (rho g)_x = rho g_x   (the momentum source term).
 * For a power-of-two dx every value is the correctly rounded result of these formulas.
 *   p      n, dx, four_pi_g (multipole faces), layout, block_n; the iteration fields are
 *          validated as for mg_solve and otherwise ignored.
 *   bc     as for mg_solve; MULTIPOLE faces are recomputed from rho as the solve does.
 *   phi    device, n^3 FP64 in the layout of p; read only.
 *   rho    device, n^3 FP64 in the layout of p; required for rhog and MULTIPOLE faces,
 *          else may be NULL.
 *   g      device, 3 n^3 FP64 (g_x, g_y, g_z one after another, each in the layout of p),
 *          or NULL.
 *   rhog   device, 3 n^3 FP64 like g, or NULL.
 *   gface  device, 3 n^2 (n+1) FP64, or NULL; dense layout only (MG_ERR_UNSUPPORTED
 *          otherwise): x faces [k][j][i'] with i' = 0..n (face i' lies between cells i'-1
 *          and i'), then y faces [k][j'][i], then z faces [k'][j][i].
 * At least one output must be given.  Asynchronous on `stream` (no host synchronisation);
 * face arrays of FIXED/MULTIPOLE faces use the context's scratch. */
int mg_gravity(mg_ctx *ctx, const mg_params *p, const mg_bc *bc, const double *phi,
               const double *rho, double *g, double *rhog, double *gface, void *stream);

/* Name of the kernel mg_gravity launches for these parameters and outputs (nonzero
 * want_* = that output is given), as profilers list it, written to buf (cap bytes,
 * NUL-terminated); returns the length needed with the NUL. */
int mg_gravity_kernel_name(const mg_params *p, int want_g, int want_rhog, int want_gface, char *buf,
                           int cap);

/* ---- statically refined mesh (Sec. 3.3) --------------------------------------------
 *
 * The unit cube as NB^3 root MeshBlocks of nb^3 cells, with `levels` nested refinement
 * boxes: box lam (1..levels) is a box of level-(lam-1) MeshBlocks, [box_lo, box_hi) per axis
 * in level-(lam-1) block units, each refined into 2 x 2 x 2 level-lam MeshBlocks.  Box 1
 * lies inside the root grid and box lam inside box lam-1 (in level-(lam-1) units: inside
 * [2 lo_{lam-1}, 2 hi_{lam-1})), each with at least one block of margin (2:1 balance).
 * Refinement level lam is one dense patch per MeshBlock level: patch 0 is the root grid at
 * (NB nb)^3 cells; patch lam >= 1 covers box lam at cell width 1/(NB nb 2^lam); its dims come
 * from mg_amr_patch_dims.  Cells of a patch under the next finer box are covered: ignored on
 * input, 0 on output. */
#define MG_AMR_MAX_LEVELS 8
typedef struct {
  int NB;                               /* root blocks per side (power of two, <= 256)      */
  int nb;                               /* cells per block side (power of two, 2..64)       */
  int levels;                           /* refinement levels, 0..MG_AMR_MAX_LEVELS          */
  int box_lo[MG_AMR_MAX_LEVELS][3];     /* box of level lam at index lam-1, (x, y, z)       */
  int box_hi[MG_AMR_MAX_LEVELS][3];
} mg_amr_mesh;

/* Cells per axis (x, y, z) of patch lam (0..levels) at the finest MeshBlock level. */
int mg_amr_patch_dims(const mg_amr_mesh *mesh, int lam, int dims[3]);

/* Full multigrid (Alg. 2 with FAS; MG_MODE_FMG) or V-cycles from the initial guess in phi
 * (MG_MODE_MGI), then FAS V-cycles (Alg. 3) on the refined mesh:
 * MeshBlock levels with every refinement level smoothed together, the conservative level
 * boundary (eqs. masscons, transgrad, piint, lbint, lbext: interpolated fine ghosts, one
 * extrapolated coarse ghost per face of the refined region) before every colour and defect,
 * Octet levels finest first, a uniform FAS V-cycle on the NB^3 root grid, and corrections
 * prolongated through the normal level boundary (restriction into the covered coarse cells,
 * trilinear prolongation into the finer patch's ghost shell).  FMG restricts the source to
 * every level, solves the root cell, then starts root levels, Octet levels and MeshBlock
 * levels in turn from the tricubic prolongation of the solution below (the normal level
 * boundary with physical root conditions for the ghosts) and runs one V-cycle from each.
 *   p     dx = 1/(NB nb) (the unit cube); mode, four_pi_g, npre, npost, omega, tol,
 *         max_cycles, fixed_cycles as for mg_solve; precision FP64 (else MG_ERR_UNSUPPORTED).
 *   bc    periodic, zero-gradient, fixed (fixed_b: device (NB nb)^2 face-centre arrays;
 *         coarser levels take 2 x 2 area means) or multipole faces (Appendix A: moments up
 *         to lmax over the composite grid, every patch's active cells at their centres,
 *         about the composite centre of mass or origin; the expansion evaluated at the face
 *         centres of every root level).
 *   rho   host array of levels+1 device pointers, patch lam's density (dims of
 *         mg_amr_patch_dims, x fastest), read only.
 *   phi   host array of levels+1 device pointers, same shapes: the initial guess on input
 *         (MG_MODE_MGI; ignored by FMG), the potential on output (volume-weighted mean removed
 *         when no face is fixed).
 *   hist  host, relative composite residual RMS(f - L phi)/RMS(f) (cell-volume weighted) of
 *         the initial guess and after each cycle; n_hist its length.
 * The workspace is the context's: allocated on the first call, grown when a larger mesh needs
 * more (within the context's HBM budget, else MG_ERR_OOM), kept for later calls and freed by
 * mg_ctx_destroy.  Synchronises `stream`. */
int mg_amr_solve(mg_ctx *ctx, const mg_params *p, const mg_amr_mesh *mesh, const mg_bc *bc,
                 const double *const *rho, double *const *phi, double *hist, int *n_hist,
                 void *stream);

/* ---- operator entry points (each operator alone, for parity checks) ---------------- */

/* One colour (0 = red, (i+j+k) even; 1 = black) of the RB-SOR smoother, eqs. rbsor1-2:
 * u <- u + omega ((sum of 6 neighbours - h^2 f)/6 - u) on cells of that colour, with
 * ghosts from `bc` evaluated from u before the colour.  u, f: device, n^3 FP64. */
int mg_op_half_sweep(mg_ctx *ctx, int n, double h, double omega, int colour, const mg_level_bc *bc,
                     double *u, const double *f, void *stream);

/* `sweeps` full red-then-black smoothing sweeps in the bandwidth-optimised fused kernel
 * used by the solver on large levels; identical in result to 2*sweeps half-sweeps. */
int mg_op_smooth(mg_ctx *ctx, int n, double h, double omega, int sweeps, const mg_level_bc *bc,
                 double *u, const double *f, void *stream);

/* Ghost fill of one level (Sec. 2.3.6): out (device, (n+2)^3 FP64, x fastest) receives u
 * (device, n^3) at active index (i+1, j+1, k+1) and every ghost from bc: periodic faces the
 * opposite active cell, zero-gradient faces the adjacent cell, fixed (and multipole) faces
 * 2 b - adjacent cell.  Ghosts are filled axis by axis -- x, then y over the x ghosts, then z
 * over both -- which defines the edge and corner ghosts the 27-point prolongations read.
 * The operators evaluate these ghosts on the fly; this entry point exposes them. */
int mg_op_fill(mg_ctx *ctx, int n, const mg_level_bc *bc, const double *u, double *out, void *stream);

/* d = f - L_h u (eq. defect).  u, f, d: device, n^3 FP64. */
int mg_op_defect(mg_ctx *ctx, int n, double h, const mg_level_bc *bc, const double *u,
                 const double *f, double *d, void *stream);

/* uc = 8-cell mean of uf (eq. restriction).  uf: device (2nc)^3, uc: device nc^3. */
int mg_op_restrict(mg_ctx *ctx, int nc, const double *uf, double *uc, void *stream);

/* uf += trilinear prolongation of uc (eq. trilinear; Alg. 1 steps 5-6), ghosts of uc from bc. */
int mg_op_prolong_add(mg_ctx *ctx, int nc, const mg_level_bc *bc, const double *uc, double *uf,
                      void *stream);

/* uf = tricubic FMG prolongation of uc (Sec. 2.3.1; Alg. 2 step 3), ghosts of uc from bc. */
int mg_op_prolong_fmg(mg_ctx *ctx, int nc, const mg_level_bc *bc, const double *uc, double *uf,
                      void *stream);

/* Single-cell coarsest solve (Sec. 2.3.2): u (device, 1) from f (device, 1), cell width h. */
int mg_op_coarsest(mg_ctx *ctx, double h, const mg_level_bc *bc, double *u, const double *f,
                   void *stream);

/* Fused down step of a V-cycle level (Alg. 1 steps 1-3): `npre` smoothing sweeps of u,
 * then fc = restriction of the defect f - L u; uc = 0.  u, f: device n^3; fc, uc: (n/2)^3.
 * The kernels follow the context's schedule as the solver does: with npre = 2 on n >= 128 and
 * the "march" setting allowing it, one two-sweep streaming pass; otherwise the defect fused
 * into the last sweep or as its own pass ("pass" lines of mg_tuning_set). */
int mg_op_down(mg_ctx *ctx, int n, double h, double omega, int npre, const mg_level_bc *bc,
               double *u, const double *f, double *fc, double *uc, void *stream);

/* Fused up step of a V-cycle level (Alg. 1 steps 5-7): u += trilinear(uc) with uc's ghosts
 * from bc_coarse, then `npost` smoothing sweeps with bc (with npost = 2 on n >= 128 and the
 * "march" setting allowing it, in one two-sweep streaming pass). */
int mg_op_up(mg_ctx *ctx, int n, double h, double omega, int npost, const mg_level_bc *bc,
             const mg_level_bc *bc_coarse, double *u, const double *f, const double *uc,
             void *stream);

/* FP32 forms of mg_op_smooth, mg_op_down and mg_op_up: the same passes, in the single
 * precision the inner cycles of MG_PREC_MIXED run (u, f, fc, uc, uc: device FP32 arrays of
 * the same shapes; h, omega and face values as above, rounded to FP32 by the kernels).
 * zero_in != 0: u is zero on input and the first sweep does not read it (the first sweep of a
 * mixed-precision correction cycle). */
int mg_op_smooth_f32(mg_ctx *ctx, int n, double h, double omega, int sweeps, int zero_in, const mg_level_bc *bc,
                     float *u, const float *f, void *stream);
int mg_op_down_f32(mg_ctx *ctx, int n, double h, double omega, int npre, const mg_level_bc *bc, float *u,
                   const float *f, float *fc, float *uc, void *stream);
int mg_op_up_f32(mg_ctx *ctx, int n, double h, double omega, int npost, const mg_level_bc *bc,
                 const mg_level_bc *bc_coarse, float *u, const float *f, const float *uc, void *stream);

/* One smoothing sweep of u in place (eqs. rbsor1-2) and *sumsq = the sum over the level of
 * the squared defect f - L_h u of the INPUT u (Sec. 2.3.7): the solver's first pre-sweep of a
 * V-cycle, which also measures the residual of the iterate it starts from.  u: device n^3
 * FP64 (in and out); f: device n^3 FP64; sumsq: host.  Synchronises the stream. */
int mg_op_sweep_input_norm(mg_ctx *ctx, int n, double h, double omega, const mg_level_bc *bc, double *u,
                           const double *f, double *sumsq, void *stream);

/* FP64 half of one mixed-precision defect-correction step (the refinement around the FP32
 * cycle): phi <- phi + e, then the defect d = f - L_h phi (eq. defect) of the updated phi,
 * r32 = d rounded to FP32 (the next correction's right-hand side) and *sumsq = the sum of d^2
 * over the level (Sec. 2.3.7), all in one pass.  phi: device n^3 FP64 (in and out); e, r32:
 * device n^3 FP32; f: device n^3 FP64; sumsq: host.  Synchronises the stream. */
int mg_op_mixed_update(mg_ctx *ctx, int n, double h, const mg_level_bc *bc, double *phi, const float *e,
                       const double *f, float *r32, double *sumsq, void *stream);

/* ---- serving runtime ---------------------------------------------------------------
 *
 * A request stream of independent solves (different sizes, boundary kinds and precisions)
 * on one device.  `workers` host threads each drive one HIP stream of default priority, so
 * solves overlap on the device.  Admission is by HBM footprint: a request starts only when
 * its hierarchy (mg_footprint_bytes + one n^3 FP64 result slot) fits in `hbm_budget` next to
 * the hierarchies in use.  Hierarchies stay resident after a solve and are reused by the next
 * request of the same workspace class (n, precision, block_n of the MeshBlock layout, scheme);
 * each is a context whose HBM budget is that class's footprint, so a solve never grows it
 * beyond what admission counted.  Idle hierarchies of other classes are released (least
 * recently used first) only when a new one would not fit.  Every kernel of a solve is
 * deterministic, so a request's phi and history do not depend on what runs beside it. */

typedef struct mg_server mg_server;

typedef struct {
  int device;           /* HIP device                                                      */
  int workers;          /* host threads = concurrent solves, 1..64                         */
  size_t hbm_budget;    /* bytes for resident hierarchies; 0 = 80 % of the free memory     */
  int policy;           /* MG_SERVE_FIFO: strict arrival order; MG_SERVE_SKIP: a later
                           request that fits may start while the head waits for memory     */
  int simulate;         /* 1: no device work; a request occupies its worker for sim_ms
                           (tests of the scheduler without a GPU)                          */
} mg_server_config;

#define MG_SERVE_FIFO 0
#define MG_SERVE_SKIP 1

typedef struct {
  /* in */
  mg_params params;
  mg_bc bc;
  const double *rho;    /* device, n^3; read only                                          */
  double *phi;          /* device, n^3 output, or NULL: written to the hierarchy's result
                           slot and discarded (MG_MODE_MGI needs phi)                      */
  double arrival_ms;    /* submission time, ms after the start of mg_server_run            */
  double sim_ms;        /* simulate mode: service time                                     */
  int hist_cap;         /* capacity of hist (0: no history returned)                       */
  double *hist;         /* host, hist_cap entries, or NULL                                 */
  /* out */
  int status;           /* mg_solve's return value; MG_ERR_OOM if it can never fit         */
  int n_hist;
  double resid;         /* last relative residual                                          */
  double admit_ms;      /* picked by a worker (memory granted)                             */
  double start_ms;      /* hierarchy ready, solve enqueued                                 */
  double end_ms;        /* solve complete (result in phi)                                  */
  int worker;
  int reused;           /* 1 if a resident hierarchy was reused                            */
} mg_request;

typedef struct {
  int created;          /* hierarchies allocated                                           */
  int reused;           /* requests served by a resident hierarchy                         */
  int evicted;          /* idle hierarchies released to make room                          */
  int rejected;         /* requests larger than the whole budget                           */
  int max_concurrent;   /* most solves in flight at once                                   */
  size_t resident_bytes;  /* bytes held by hierarchies now                                 */
  size_t peak_bytes;    /* most bytes held at once                                         */
} mg_server_stats;

int mg_server_create(mg_server **srv, const mg_server_config *cfg);
void mg_server_destroy(mg_server *srv);
const char *mg_server_last_error(const mg_server *srv);

/* Allocate `count` resident hierarchies for requests like p (warm-up), within the budget. */
int mg_server_reserve(mg_server *srv, const mg_params *p, int count);

/* Serve `n` requests (host array): each is submitted at its arrival_ms (open loop; 0 for
 * all = closed batch), scheduled by the policy and solved on a worker's stream.  Blocks
 * until every request is complete; outputs are written into the array.  Per-request errors
 * are in reqs[i].status; the return value is MG_OK unless the run itself failed. */
int mg_server_run(mg_server *srv, mg_request *reqs, int n);

/* Counters since mg_server_create. */
int mg_server_get_stats(const mg_server *srv, mg_server_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* MG355_H */
