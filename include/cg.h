/*
 * cg.h - C ABI of the MI355X (gfx950) stencil conjugate-gradient library.
 *
 * The library solves A x = b where A is the Laplacian of Section II of
 * "Efficient FPGA Implementation of Conjugate Gradient Methods for Laplacian
 * System using HLS" (arXiv 1803.03797): an nx-by-ny interior grid with zero
 * Dirichlet boundary, discretised by the 5-point stencil the paper prints in
 * Section II-B (4 on the centre, -1 on the four compass neighbours), used
 * unscaled.  A is never assembled: every product A*u is the stencil applied on
 * the grid (Section II-B, "Parallel Matrix Vector Multiplication implemented as
 * Stencil operations").  Two iterations are offered, the paper's Algorithm 1
 * (stdCG, "classic") and Algorithm 2 (newCG, the pipelined CG that overlaps the
 * stencil with the two dot products, "pipelined").
 *
 * Vector layout at the boundary: nx*ny doubles, row-major, unknown (i, j) with
 * 0 <= i < nx, 0 <= j < ny at index j*nx + i.  Pointers are host or device
 * pointers as stated by cg_problem.mem; the caller owns them.
 *
 * Return convention of every int-returning call: a negative value means the
 * call was rejected and nothing happened (CG_E_*); a non-negative value is an
 * outcome (CG_OK, CG_PENDING, CG_NOT_CONVERGED, CG_BREAKDOWN).  No exception
 * and no errno crosses this boundary.  cg_status_str() names any code.
 *
 * Threading: calls on one context are serialised by the context; cg_submit
 * and cg_poll may be called from any thread.
 */
#ifndef CG_H
#define CG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cg_ctx cg_ctx; /* opaque: device workspace, streams, scheduler */

typedef enum { CG_VARIANT_CLASSIC = 0, CG_VARIANT_PIPELINED = 1 } cg_variant;
/* CG_PREC_FIXED: the paper's fixed-point format (Section II-B, the stencil
 * listing's 50-bit type with 20 integer bits, round to nearest, saturate):
 * every value is an integer multiple of 2^-30 in [-2^19, 2^19 - 2^-30].  b and
 * x0 are rounded to it on entry (ties towards +infinity, out-of-range values
 * saturate, NaN reads as 0); every statement of Algorithm 1 or 2 rounds its
 * exact result once (y +- a x formed exactly; a dot product sums its rounded
 * products exactly and saturates once; each division rounds once); the stop
 * test compares (r, r) with tol^2 (b, b) rounded to the format; x returns as
 * the exact FP64 value of the fixed-point result, and the result's relative
 * residuals are sqrt of ratios of fixed-point dot products.  Integer
 * arithmetic: the result does not depend on summation order, and every path
 * returns the same bits.  One work-group per solve (cg_plan_info.path 3)
 * holding two vectors in its 160 KiB of LDS: the grid must satisfy
 * (nx + 1)(ny + 2) + nx ny <= 20352 (100 x 100 fits; the paper's grids reach
 * 100 x 100; a single row or column up to 5087 or 6782 unknowns); larger
 * grids are CG_E_INVALID.  inner_tol is ignored. */
/* CG_PREC_AUTO: a size-based precision policy for batches and serving.
 * Grids of fewer than 20480 unknowns are solved in FP64 (the on-chip solver
 * and the shortest tile solves, where FP32 vectors buy nothing), larger ones
 * FP32-refined (CG_PREC_FP32_REFINED: half the bytes per inner iteration);
 * the result is bitwise that of the precision chosen (outer_iterations > 0
 * tells a refined one).  2D constant-coefficient problems without residual
 * replacement only; with precond > 0 the refined ones precondition their
 * FP32 inner solves. */
typedef enum {
  CG_PREC_FP64 = 0,
  CG_PREC_FP32_REFINED = 1,
  CG_PREC_FIXED = 2,
  CG_PREC_AUTO = 3
} cg_precision;
typedef enum { CG_MEM_HOST = 0, CG_MEM_DEVICE = 1 } cg_memspace;

enum {
  CG_OK = 0,             /* converged: ||r|| <= tol*||b|| (or tol == 0 and maxit done) */
  CG_PENDING = 1,        /* cg_poll: not finished yet                                 */
  CG_NOT_CONVERGED = 2,  /* maxit reached; x holds the last iterate                   */
  CG_BREAKDOWN = 3,      /* non-positive or non-finite curvature / scalar; x = last   */
  CG_E_INVALID = -1,     /* bad argument                                              */
  CG_E_NOMEM = -2,       /* footprint larger than the arena (or arena exhausted)      */
  CG_E_DEVICE = -3,      /* HIP error, no device, or the GPU library could not run    */
  CG_E_BUSY = -4,        /* context is shutting down                                  */
  CG_E_TICKET = -5       /* unknown or already-released ticket                        */
};

typedef struct {
  int32_t device;         /* HIP device ordinal                                         */
  void* stream;           /* hipStream_t the caller orders work on (may be NULL = the
                             null stream); the library runs on its own stream and
                             orders itself after this one at every call               */
  void* arena;            /* device memory the library may use for all workspace, or
                             NULL: then the library allocates arena_bytes itself      */
  size_t arena_bytes;     /* size of arena; admission budget (0 with arena == NULL
                             means 4 GiB)                                              */
  int32_t max_slots;      /* max solves resident at once (batch / serving); 0 = 256   */
  const char* tune_cache; /* path of the autotuner's JSON cache, or NULL              */
} cg_config;

typedef struct {
  int32_t nx, ny;          /* interior grid; zero Dirichlet ring implied (Section II) */
  cg_memspace mem;         /* where b, x0 and x live                                  */
  const double* b;         /* right-hand side, nx*ny, row-major; read until the final
                              status is returned                                      */
  const double* x0;        /* starting vector or NULL (= zeros); may alias x          */
  double* x;               /* out: solution, nx*ny                                    */
  double tol;              /* stop when ||r||_2 <= tol ||b||_2, 0 <= tol < 1; tol == 0
                              runs exactly maxit iterations (throughput mode)         */
  int32_t maxit;           /* >= 1; FP32-refined: cap on the total inner iterations   */
  cg_variant variant;      /* Algorithm 1 or Algorithm 2                              */
  cg_precision precision;  /* FP64, FP32 inner CG inside FP64 refinement, or fixed    */
  double inner_tol;        /* refined only: the inner solve stops at the relative
                              residual max(inner_tol, tol ||b|| / (2 ||b - A x||)),
                              i.e. no further than the outer tolerance needs;
                              0 = 1e-4                                            */
  int32_t precond;         /* 0: none; s = 1..8: FP64 CG preconditioned by
                              M^-1 = p_s(A), s steps of Chebyshev semi-iteration on
                              A y = r from y = 0 over [lmax / (2 s^2), lmax], lmax =
                              4 + 2cos(pi/(nx+1)) + 2cos(pi/(ny+1)) the largest
                              eigenvalue of A (the M^-1 of the pipelined-CG
                              literature Section I builds on): classic CG with
                              z = M^-1 r, or the preconditioned pipelined CG of
                              Ghysels and Vanroose (variant PIPELINED); the stop
                              test stays on ||r||; FP64 alone, in batches and
                              served.  With CG_PREC_FP32_REFINED (alone, in batches
                              and served): the inner solve of the refinement
                              becomes classic CG preconditioned
                              by the same M^-1 in binary32 (coefficients rounded
                              once; (r,z) and (p,Ap) summed in binary64, alpha and
                              beta rounded to binary32 once; the inner stop test on
                              (r,r)), for either variant                           */
  int32_t nz;              /* 0 or 1: the 2D problem above.  nz > 1: the 3D 7-point
                              Laplacian (centre 6, the six face neighbours -1) on an
                              nx x ny x nz interior grid with zero Dirichlet
                              boundary, the next structured-grid case the paper's
                              Section I names; unknown (i, j, l) at (l ny + j) nx + i,
                              so b, x0 and x hold nx * ny * nz values; FP64, either
                              variant, precond 0; alone, in batches and served      */
  int32_t rr_period;       /* 0: none.  k > 0 (even): residual replacement in the
                              pipelined variant (Algorithm 2) every k iterations:
                              q = A p, z = A q, r = b - A x and w = A r recomputed
                              from their definitions, after which the iteration
                              continues (the remedy of Cools et al. for the
                              accuracy Algorithm 2's recurrences lose); FP64, 2D
                              (either operator), precond 0; alone, in batches and
                              served (bitwise as alone); the solve runs on the
                              multi-work-group passes                          */
  const double* kx;        /* NULL (with ky NULL): the constant-coefficient operators
                              above.  Else the variable-coefficient 5-point operator,
                              the other structured-grid case Section I names beside
                              3D: the finite-volume form of -div(k grad u) with zero
                              Dirichlet boundary, (A u)_ij = d u_ij - kW u_W - kE u_E
                              - kS u_S - kN u_N (out-of-grid neighbours 0), d = ((kW
                              + kE) + kS) + kN; kx holds the conductivities of the
                              faces between columns, ny x (nx + 1) row-major (kW =
                              kx[j][i], kE = kx[j][i+1]; columns 0 and nx are the
                              boundary faces), in the memory space of b; read until
                              the final status is returned.  All ones give the
                              Section II-B operator.  Values must be positive and
                              finite (A is then symmetric positive definite); other
                              values are not checked and make the result undefined
                              (typically CG_BREAKDOWN).  FP64, 2D (nz <= 1), either
                              variant, precond 0; alone, in batches and served (a
                              served request's kx and ky are read when it is
                              admitted, like its b)                                 */
  const double* ky;        /* with kx: the conductivities of the faces between rows,
                              (ny + 1) x nx row-major (kS = ky[j][i], kN = ky[j+1][i];
                              rows 0 and ny are the boundary faces)                */
} cg_problem;

typedef struct {
  int32_t status;           /* CG_OK / CG_NOT_CONVERGED / CG_BREAKDOWN                */
  int32_t iterations;       /* x-updates (refined: total inner iterations)           */
  int32_t outer_iterations; /* refined: refinement steps; else 0                     */
  int32_t pad_;
  double rel_res_recursive; /* sqrt((r,r)/(b,b)) of the iteration's own residual     */
  double rel_res_true;      /* ||b - A x|| / ||b|| recomputed on the device (FP64;
                               fixed point: in the fixed-point arithmetic)           */
  double device_seconds;    /* wall time the solve held the device                   */
  double latency_seconds;   /* serving: submit -> completion; else = device_seconds  */
} cg_result;

/* Work layout a problem will use.  Its reduction order is the documented
 * arithmetic contract.  Tile order (paths 0 and 1; cg_dot; an FP64 problem of
 * path 0 or 1 in a batch): tile = 64 lanes x cols_per_lane columns by waves x
 * rows rows; lanes accumulate with fma in row order (walk_alt = 1: the odd
 * wavefronts of a tile from their strip's last row up); xor butterfly; waves
 * in order; tiles in index order through threads2 strided threads.  Column-
 * segment order (path 2, alone and in a batch): thread t of seg_waves*64
 * owns column t mod seg_cols and seg_rows rows of segment t div seg_cols
 * (threads of columns >= nx own nothing); fma in row order; xor butterfly;
 * waves in order.  Preconditioned CG (precond > 0) sums (r, z) in the tile
 * order of tiles 128 columns wide (2 per lane) and cheb_rows rows tall with
 * one wavefront each, through threads2 strided threads; its other sums follow
 * the tile fields.  Path 3 (fixed point) is exact integer arithmetic: no order
 * to describe.  The tile fields always describe the
 * tile geometry of the shape (cg_dot and cg_apply use it on every path). */
typedef struct {
  int32_t path;             /* 0 = multi-work-group passes, 1 = single work-group,
                               2 = single work-group with the vectors on chip,
                               3 = fixed point, single work-group                   */
  int32_t cols_per_lane, lanes, waves, rows, threads2;
  int32_t tiles;            /* tiles per pass                                        */
  int32_t grid;             /* work-groups per pass launch                           */
  int32_t pitch;            /* padded row length of one vector, in elements          */
  int32_t seg_rows;         /* path 2: rows per thread; else 0                       */
  int32_t seg_waves;        /* path 2: wavefronts of the work-group; else 0          */
  int32_t seg_cols;         /* path 2: threads per row of segments (nx + 1); else 0  */
  int32_t cheb_rows;        /* precond > 0: rows of a Chebyshev tile; else 0         */
  int32_t cheb_tiles;       /* precond > 0: Chebyshev tiles (partials of (r,z))      */
  int32_t cheb_grid;        /* precond > 0: work-groups of the Chebyshev pass        */
  int32_t row_stride;       /* elements from a row of a device vector to its next:
                               pitch, or pitch times the number of FP64 vectors
                               whose rows the workspace interleaves (pipelined
                               FP64 on path 0)                                     */
  int32_t walk_alt;         /* tile order: 1 = the odd wavefronts of a tile walk and
                               sum their strip from its last row up (the classic
                               variant's 5-point passes: a strip's halo row is then
                               read by both of its wavefronts at about the same
                               time); 0 = every wavefront top down                 */
  int32_t walk_z;           /* 1 = the 3D z-march tile order (nz > 1): a tile is 4
                               consecutive in-plane rows (waves, one per wavefront)
                               by `rows` planes, tile t = (tz * ceil(ny / 4) + ty) *
                               tiles across + tx, and each lane sums its row over
                               the planes in ascending z; 0 = the 2D tile order    */
  size_t footprint;         /* device bytes the solve occupies                       */
} cg_plan_info;

/* Per-kernel timing gathered while profiling is on (cg_set_profiling). */
typedef struct {
  char name[32];
  int64_t launches;
  double seconds;           /* summed HIP-event time of the launches                 */
  double bytes;             /* summed algorithmic HBM bytes of the launches          */
} cg_kstat;

/* Creates a context on cfg->device.  CG_E_DEVICE when no usable GPU. */
int cg_create(const cg_config* cfg, cg_ctx** out);
/* Cancels queued requests (they complete as CG_E_BUSY), waits for running
 * work, frees everything the library allocated. */
int cg_destroy(cg_ctx* ctx);

/* One blocking solve of A x = b (Algorithm 1 or 2; Section II problem). */
int cg_solve(cg_ctx* ctx, const cg_problem* prob, cg_result* res);

/* n independent solves on the device at once.  Every resident solve advances
 * by one CG pass per launch of a multi-solve step kernel (chunks of launches
 * replayed from a HIP graph); problems small enough for the on-chip solver
 * (cg_plan_info.path 2) and fixed-point problems (path 3) run whole, one
 * work-group each, beside the steps.
 * Solves are admitted in order while their footprint fits the arena and a
 * slot is free.  Each result is bitwise the one cg_solve gives.  Returns the
 * worst per-solve status; results[i] holds each outcome.  A breakdown of one
 * solve does not disturb the others.  Residual-replacement problems step
 * through the replacement's four passes on the same engine. */
int cg_solve_batch(cg_ctx* ctx, const cg_problem* probs, int32_t n, cg_result* results);

/* Serving: queue one request (non-blocking).  A scheduler thread admits
 * queued requests in order when the device footprint fits the free arena and
 * a slot is free; admitted requests join the resident set at the next chunk
 * of steps (or run whole on the on-chip solver) and are retired when final.
 * The request's b and x0 are read only once the caller's stream
 * (cg_config.stream) has passed the point of this call; x is written before
 * cg_poll returns the final status.  CG_E_NOMEM if its footprint exceeds
 * arena_bytes; CG_E_DEVICE if the ordering event cannot be recorded;
 * CG_E_INVALID for the problems cg_solve rejects. */
int cg_submit(cg_ctx* ctx, const cg_problem* prob, uint64_t* ticket);
/* CG_PENDING, or the final status (then *res is filled and the ticket is
 * released). */
int cg_poll(cg_ctx* ctx, uint64_t ticket, cg_result* res);

const char* cg_status_str(int code);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): n small
 * solves, each bitwise the one cg_solve and cg_solve_batch give, with no
 * context and no device or pinned-host allocation.  The solves run on the
 * on-chip solver (one work-group per solve, cg_plan_info.path 2) directly on
 * the caller's device vectors (mem must be CG_MEM_DEVICE; b, x0 and x hold
 * nx*ny doubles, row-major, unpadded), on the current HIP device, in `stream`
 * (hipStream_t, NULL = the null stream); the call returns when they are done.
 * Every problem must be FP64, 2D, unpreconditioned, constant-coefficient and
 * fit the on-chip solver: (nx + 1) * ceil(ny / 20) <= 512 (e.g. up to
 * 100 x 100, or 511 x 20); 1 <= n <= 64.  Anything else is CG_E_INVALID
 * before any device work.  The library keeps the solves' descriptors and
 * scalar states in a fixed 64 KiB device array of its own (one per device,
 * held until the process ends), rewritten whole by every call: calls are
 * serialised per device within the process, and calls from several processes
 * each use their own copy.  Returns the worst status, as cg_solve_batch;
 * results[i] holds each outcome (device_seconds: the call's wall time). */
int cg_solve_batch_small_noalloc(const cg_problem* probs, int32_t n, void* stream,
                                 cg_result* results);

/* ---- building blocks, exposed for verification and measurement ---------- */

/* y = A u on the nx-by-ny grid, matrix-free (Section II-B stencil). */
int cg_apply(cg_ctx* ctx, int32_t nx, int32_t ny, cg_memspace mem, const double* u, double* y);
/* *out = (a, b) with the library's deterministic two-stage reduction (the
 * order of cg_plan_info for an FP64 problem of this shape). */
int cg_dot(cg_ctx* ctx, int32_t nx, int32_t ny, cg_memspace mem, const double* a,
           const double* b, double* out);
/* Fills *info for prob (host-side; no device work).  CG_E_INVALID for a
 * fixed-point problem larger than the fixed-point solver takes. */
int cg_plan(cg_ctx* ctx, const cg_problem* prob, cg_plan_info* info);
/* Device bytes prob needs while resident (host-only; no context needed). */
int cg_footprint(const cg_problem* prob, size_t* bytes);
/* CG_OK or CG_E_INVALID (host-only; no context needed). */
int cg_validate(const cg_problem* prob);
/* Autotuner: times candidate tile shapes for (nx, ny, variant, precision) on
 * the device, the shape an unpinned solve would take first, and pins the
 * fastest for that grid shape, precision and variant (refined solves: one pin
 * for both variants).  With cfg->tune_cache the pins are saved as JSON lines
 * that name the device architecture and the HIP runtime version; a new
 * context loads only the lines of its own architecture and runtime.  Returns
 * CG_OK (fixed point: nothing to tune). */
int cg_tune(cg_ctx* ctx, int32_t nx, int32_t ny, cg_variant variant, cg_precision precision);
/* Pins the tile shape for a grid shape and precision, for both variants: tile
 * height (rows per wavefront strip), grid size (0 = occupancy-derived) and
 * columns per lane (0 = default: 2 for FP64, 4 for FP32-refined; classic FP64
 * may also use 4).  The reduction order follows the pinned shape (cg_plan
 * reports it).  For the autotuner, experiments and tests. */
int cg_pin_tile(cg_ctx* ctx, int32_t nx, int32_t ny, cg_precision precision, int32_t rows,
                int32_t grid, int32_t cols_per_lane);
/* HBM probe, for measurement only: runs a plain streaming kernel over
 * device buffers carved from the arena, `elems` doubles per vector, reps + 1
 * times (the first warms up) for each of the grids of 1, 2, 4 and 8
 * work-groups per CU, and returns the best time and the bytes it moves.
 * pattern 0: read one vector; 1: copy one vector to another (the known-size
 * copy that calibrates hardware traffic counters); 2: two reads, one write;
 * 3: three reads, two writes; 4: six vectors read and written in place (the
 * traffic mix of a pipelined CG pass); 5: six vectors read, six others
 * written; 6: as 4 with non-temporal stores; 7: as 4 with the six vectors'
 * rows (4096 doubles each) interleaved in one block, the layout of the
 * pipelined solve (elems rounded down to a multiple of 4096; CG_E_INVALID if
 * that leaves none).  CG_E_NOMEM if the arena is too small. */
int cg_stream_probe(cg_ctx* ctx, int32_t pattern, size_t elems, int32_t reps, double* seconds,
                    double* bytes);
/* Integer multiply probe, for measurement only (the ALU peak the fixed-point
 * path is measured against): 8 work-groups per CU of 256 threads, each thread
 * running 8 independent chains of `rounds` 32 x 32 -> 64-bit multiply-adds,
 * reps + 1 times (the first warms up); returns the best time and the number
 * of multiply-adds of one launch.  CG_E_INVALID for rounds or reps < 1. */
int cg_mul_probe(cg_ctx* ctx, int32_t rounds, int32_t reps, double* seconds, double* ops);
/* Profiling on/off; while on, every kernel launch is bracketed by HIP events
 * on the library's stream. */
int cg_set_profiling(cg_ctx* ctx, int32_t on);
/* Copies up to max entries of the per-kernel statistics; *count = entries
 * available.  reset != 0 clears them afterwards. */
int cg_kernel_stats(cg_ctx* ctx, cg_kstat* out, int32_t max, int32_t* count, int32_t reset);
/* Library build identifier. */
const char* cg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CG_H */
