/*
 * cg_oracle.c - CPU oracle for conjugate gradients on the 2D Laplace problem.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links, loads or calls this
 * file; only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or table with the GPU library.
 *
 * What it computes (paper: "Efficient FPGA Implementation of Conjugate Gradient
 * Methods for Laplacian System using HLS", arXiv 1803.03797):
 *   - the system A x = b of Section II: the Laplacian on an nx-by-ny interior
 *     grid with zero Dirichlet boundary, discretised by the 5-point stencil
 *     whose 3x3 form the paper prints in Section II-B (centre 4, the four
 *     compass neighbours -1, corners 0).  A is used unscaled (no 1/h^2).
 *   - A is ASSEMBLED EXPLICITLY as a CSR matrix (the paper applies it
 *     matrix-free; the oracle deliberately does not).
 *   - classic CG = Algorithm 1 (stdCG), with a general starting vector x0;
 *   - the modified CG = Algorithm 2 (newCG, the pipelined CG of Ghysels and
 *     Vanroose, unpreconditioned), with the sign/parenthesis readings listed
 *     in the design notes: r <- r - alpha*q, w <- w - alpha*z,
 *     alpha_i = 1 / (delta_i/gamma_i - beta_i/alpha_{i-1});
 *   - FP32-inner / FP64-outer iterative refinement around classic CG;
 *   - classic CG preconditioned by a Chebyshev polynomial in A (the M^-1 that
 *     the pipelined-CG literature the paper builds on carries);
 *   - both CG variants on the 3D 7-point Laplacian (oracle_cg3), the next
 *     structured-grid finite-difference system after the paper's 2D one;
 *   - both CG variants on the variable-coefficient 5-point operator
 *     (oracle_cg_vc): the finite-volume form of -div(k grad u) with face
 *     conductivities, equal to the paper's operator when k = 1.
 *
 * Unknown (i, j), 0 <= i < nx, 0 <= j < ny, has index k = j*nx + i.
 * Build with -O2 -ffp-contract=off (no fast-math): every operation below is
 * one correctly rounded IEEE binary64 (or binary32) operation, and fma() is
 * the correctly rounded fused multiply-add of C99.
 *
 * Two summation/rounding "modes", both valid FP64 CG runs:
 *   MODE_SEQUENTIAL  textbook: dot = sum over k ascending of a[k]*b[k]
 *                    (product rounded, then added); axpy y + a*x rounded
 *                    twice; CSR rows sorted by column.
 *   MODE_CANONICAL   the documented arithmetic contract of the GPU library
 *                    (written out again here from that contract, not shared):
 *                    axpys are fma(a, x, y); CSR row entries are stored in the
 *                    order centre, west, east, south, north so that the plain
 *                    CSR loop evaluates (((4uC - uW) - uE) - uS) - uN;
 *                    dots follow the tile / lane / butterfly order described
 *                    at dot_canonical() below, or, for the column-segment
 *                    layout of the small-grid solver, dot_segments().
 */
#define _POSIX_C_SOURCE 200809L
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Planted mistakes, for the tests that show the pins catch them (a test
 * builds a copy of this file with one of them; every real build has
 * ORACLE_MUTANT 0).  Refinement's inner solve:
 *   1: the inner vectors kept in binary64;
 *   2: the inner dot products summed in binary32;
 *   3: alpha and beta of the inner solve left in binary64.
 * Residual replacement of the pipelined variant:
 *   4: w = A r not recomputed;
 *   5: z = A q not recomputed. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

/* All-core timing build.  Built with -fopenmp (the benchmark's CPU baseline
 * only; the tests use the plain build, in which the pragmas below are inert),
 * the matrix-vector product and the vector updates split their rows over the
 * threads (each row's arithmetic unchanged), and the sequential-mode dot
 * product sums one contiguous block per thread in order and then adds the
 * per-thread partials in thread order: deterministic for a given number of
 * threads, and not the sequential order. */
int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Seconds the last solve of the calling thread spent after assembling its
 * matrix (the iterations, without the CSR assembly). */
static _Thread_local double g_solve_seconds = 0.0;
double oracle_last_solve_seconds(void) { return g_solve_seconds; }
static double wall_now(void) {
  struct timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

enum { OR_OK = 0, OR_NOT_CONVERGED = 2, OR_BREAKDOWN = 3,
       OR_E_INVALID = -1, OR_E_NOMEM = -2 };
enum { MODE_SEQUENTIAL = 0, MODE_CANONICAL = 1 };
enum { VARIANT_CLASSIC = 0, VARIANT_PIPELINED = 1 };

/* Reduction order of the canonical mode (see dot_canonical). */
typedef struct {
  int32_t cols_per_lane; /* consecutive columns owned by one lane            */
  int32_t lanes;         /* lanes per wavefront                              */
  int32_t waves;         /* wavefronts stacked vertically in one tile        */
  int32_t rows;          /* rows per wavefront strip                         */
  int32_t threads2;      /* threads of the cross-tile sum (multiple of lanes) */
  int32_t layout;        /* 0: tiles (dot_canonical); 1: column segments
                            (dot_segments: rows, lanes, waves, seg_cols)      */
  int32_t seg_cols;      /* layout 1: threads per row of segments (>= nx; the
                            threads of columns >= nx own nothing)             */
  int32_t alt;           /* layout 0: 1 = the odd wavefronts of a tile (w = 1,
                            3, ...) take their strip's rows from the last up */
  int32_t plane;         /* layout 2: rows per plane (the 3D grid's ny; the
                            vectors hold plane * nz rows)                    */
} oracle_order;

typedef struct {
  int32_t status;
  int32_t iterations;        /* x-updates (inner iterations for refinement) */
  int32_t outer_iterations;  /* refinement only                             */
  int32_t pad_;
  double rel_res_recursive;  /* sqrt(gamma / (b,b)) at exit                  */
  double rel_res_true;       /* ||b - A x|| / ||b|| recomputed at exit       */
} oracle_result;

/* Optional per-iteration records for the invariant tests.  Any pointer may be
 * NULL.  gamma has room for max_hist entries; r, p, x have room for max_hist
 * vectors of n entries each, entry m holding the vector after m updates. */
typedef struct {
  int32_t max_hist;
  int32_t count;   /* out: entries written */
  double* gamma;
  double* r;
  double* p;
  double* x;
} oracle_history;

/* ------------------------------------------------------------------ CSR -- */

int64_t oracle_csr_nnz(int32_t nx, int32_t ny) {
  if (nx < 1 || ny < 1) return -1;
  int64_t n = (int64_t)nx * ny;
  /* every unknown has itself plus the in-range compass neighbours */
  return n + 2 * (int64_t)(nx - 1) * ny + 2 * (int64_t)nx * (ny - 1);
}

/* Assemble A.  order 0: entries of a row sorted by column.  order 1: centre,
 * west (i-1), east (i+1), south (j-1), north (j+1).  Returns nnz or <0. */
int64_t oracle_csr_assemble(int32_t nx, int32_t ny, int32_t order,
                            int64_t* row_ptr, int32_t* col, double* val) {
  if (nx < 1 || ny < 1) return OR_E_INVALID;
  int64_t e = 0;
  for (int32_t j = 0; j < ny; ++j) {
    for (int32_t i = 0; i < nx; ++i) {
      int64_t k = (int64_t)j * nx + i;
      row_ptr[k] = e;
      if (order == 0) {
        if (j > 0)      { col[e] = (int32_t)(k - nx); val[e++] = -1.0; }
        if (i > 0)      { col[e] = (int32_t)(k - 1);  val[e++] = -1.0; }
        col[e] = (int32_t)k; val[e++] = 4.0;
        if (i < nx - 1) { col[e] = (int32_t)(k + 1);  val[e++] = -1.0; }
        if (j < ny - 1) { col[e] = (int32_t)(k + nx); val[e++] = -1.0; }
      } else {
        col[e] = (int32_t)k; val[e++] = 4.0;
        if (i > 0)      { col[e] = (int32_t)(k - 1);  val[e++] = -1.0; }
        if (i < nx - 1) { col[e] = (int32_t)(k + 1);  val[e++] = -1.0; }
        if (j > 0)      { col[e] = (int32_t)(k - nx); val[e++] = -1.0; }
        if (j < ny - 1) { col[e] = (int32_t)(k + nx); val[e++] = -1.0; }
      }
    }
  }
  row_ptr[(int64_t)nx * ny] = e;
  return e;
}

typedef struct {
  int32_t nx, ny;
  int64_t n;
  int64_t* row_ptr;
  int32_t* col;
  double* val;
  float* valf;
} csr_t;

static void csr_free(csr_t* A) {
  free(A->row_ptr); free(A->col); free(A->val); free(A->valf);
  memset(A, 0, sizeof(*A));
}

static int csr_build(csr_t* A, int32_t nx, int32_t ny, int32_t order, int want_float) {
  memset(A, 0, sizeof(*A));
  int64_t nnz = oracle_csr_nnz(nx, ny);
  if (nnz < 0) return OR_E_INVALID;
  A->nx = nx; A->ny = ny; A->n = (int64_t)nx * ny;
  A->row_ptr = (int64_t*)malloc((size_t)(A->n + 1) * sizeof(int64_t));
  A->col = (int32_t*)malloc((size_t)nnz * sizeof(int32_t));
  A->val = (double*)malloc((size_t)nnz * sizeof(double));
  if (want_float) A->valf = (float*)malloc((size_t)nnz * sizeof(float));
  if (!A->row_ptr || !A->col || !A->val || (want_float && !A->valf)) {
    csr_free(A); return OR_E_NOMEM;
  }
  oracle_csr_assemble(nx, ny, order, A->row_ptr, A->col, A->val);
  if (want_float)
    for (int64_t e = 0; e < nnz; ++e) A->valf[e] = (float)A->val[e];
  return OR_OK;
}

/* y = A u, each row summed in the stored entry order, starting from +0. */
static void spmv(const csr_t* A, const double* u, double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < A->n; ++k) {
    double acc = 0.0;
    for (int64_t e = A->row_ptr[k]; e < A->row_ptr[k + 1]; ++e)
      acc = acc + A->val[e] * u[A->col[e]];
    y[k] = acc;
  }
}

static void spmv_f32(const csr_t* A, const float* u, float* y) {
  for (int64_t k = 0; k < A->n; ++k) {
    float acc = 0.0f;
    for (int64_t e = A->row_ptr[k]; e < A->row_ptr[k + 1]; ++e)
      acc = acc + A->valf[e] * u[A->col[e]];
    y[k] = acc;
  }
}

/* Exported y = A u for the tests. */
int oracle_spmv(int32_t nx, int32_t ny, int32_t order, const double* u, double* y) {
  csr_t A;
  int rc = csr_build(&A, nx, ny, order, 0);
  if (rc) return rc;
  spmv(&A, u, y);
  csr_free(&A);
  return OR_OK;
}

/* ----------------------------------------------------------------- dots -- */

static double dot_sequential(int64_t n, const double* a, const double* b) {
#ifdef _OPENMP
  const int nt = omp_get_max_threads();
  if (nt > 1 && n >= 65536) {
    double part[1024];
    const int T = nt < 1024 ? nt : 1024;
#pragma omp parallel num_threads(T)
    {
      const int t = omp_get_thread_num(), tt = omp_get_num_threads();
      const int64_t k0 = n * t / tt, k1 = n * (t + 1) / tt;
      double s = 0.0;
      for (int64_t k = k0; k < k1; ++k) s = s + a[k] * b[k];
      part[t] = s;
      if (t == 0)
        for (int u = tt; u < T; ++u) part[u] = 0.0;
    }
    double s = 0.0;
    for (int t = 0; t < T; ++t) s = s + part[t];
    return s;
  }
#endif
  double s = 0.0;
  for (int64_t k = 0; k < n; ++k) s = s + a[k] * b[k];
  return s;
}

/* In-place xor butterfly over one wavefront: for m = lanes/2, ..., 1 every
 * lane l takes v[l] + v[l ^ m] (both partners form the same sum, since IEEE
 * addition is commutative).  Returns lane 0. */
static double butterfly(double* v, int32_t lanes) {
  double tmp[256];
  for (int32_t m = lanes / 2; m >= 1; m /= 2) {
    for (int32_t l = 0; l < lanes; ++l) tmp[l] = v[l] + v[l ^ m];
    for (int32_t l = 0; l < lanes; ++l) v[l] = tmp[l];
  }
  return v[0];
}

/* Canonical order of the GPU library's deterministic dot product over the
 * nx-by-ny grid (vectors here are dense, k = j*nx + i):
 *   tile width  TW = cols_per_lane * lanes   columns,
 *   tile height TH = waves * rows            rows,
 *   tiles numbered t = ty * ceil(nx/TW) + tx (row-major).
 *   In tile (tx, ty), wavefront w covers rows ty*TH + w*rows + [0, rows) and
 *   lane l covers columns tx*TW + l*cols_per_lane + e, e < cols_per_lane.
 *   Lane: one accumulator per owned column, starting at +0, updated as
 *     acc_e = fma(a, b, acc_e) over its in-range rows in ascending order
 *     (descending for the odd wavefronts w = 1, 3, ... when alt is set;
 *     out-of-range rows/columns are skipped); lane value
 *     ((acc_0 + acc_1) + acc_2) + ...
 *   Wavefront: xor butterfly (see butterfly()).
 *   Tile partial: ((wave_0 + wave_1) + wave_2) + ...
 *   Cross-tile: thread t of threads2 sums partial[t], partial[t+threads2], ...
 *     in that order starting at +0; then each group of `lanes` threads is
 *     butterflied and the group values are added in group order.
 */
static double dot_canonical(int32_t nx, int32_t ny, const double* a, const double* b,
                            const oracle_order* o) {
  const int32_t cpl = o->cols_per_lane, L = o->lanes, W = o->waves, R = o->rows;
  const int32_t TW = cpl * L, TH = W * R;
  const int64_t ntx = (nx + TW - 1) / TW, nty = (ny + TH - 1) / TH;
  const int64_t T = ntx * nty;
  double* part = (double*)malloc((size_t)T * sizeof(double));
  /* tiles are independent (each partial is formed alone, then summed in tile
     order below): the OpenMP build splits them over threads, same bits */
#pragma omp parallel for schedule(static) collapse(2)
  for (int64_t ty = 0; ty < nty; ++ty) {
    for (int64_t tx = 0; tx < ntx; ++tx) {
      double lane[256], accs[4096];  /* accs[l * cpl + e]: lane l, column e */
      double tile = 0.0;
      for (int32_t w = 0; w < W; ++w) {
        int64_t j0 = ty * TH + (int64_t)w * R;
        const int64_t j1 = (j0 + R < ny) ? j0 + R : ny;
        const int up = o->alt && (w & 1);
        for (int32_t k = 0; k < TW; ++k) accs[k] = 0.0;
        /* every lane's accumulators take the wavefront's rows in the same
           order (the row loop outside the lane loop only makes the memory
           walk contiguous) */
        for (int64_t i = j0; i < j1; ++i) {
          const int64_t j = up ? j1 - 1 - (i - j0) : i;
          for (int32_t k = 0; k < TW; ++k) {
            const int64_t c = tx * TW + k;
            if (c < nx) accs[k] = fma(a[j * nx + c], b[j * nx + c], accs[k]);
          }
        }
        for (int32_t l = 0; l < L; ++l) {
          double v = accs[l * cpl];
          for (int32_t e = 1; e < cpl; ++e) v = v + accs[l * cpl + e];
          lane[l] = v;
        }
        double wv = butterfly(lane, L);
        tile = (w == 0) ? wv : tile + wv;
      }
      part[ty * ntx + tx] = tile;
    }
  }
  const int32_t T2 = o->threads2;
  double* th = (double*)malloc((size_t)T2 * sizeof(double));
  for (int32_t t = 0; t < T2; ++t) {
    double s = 0.0;
    for (int64_t k = t; k < T; k += T2) s = s + part[k];
    th[t] = s;
  }
  double total = 0.0;
  for (int32_t g = 0; g < T2 / L; ++g) {
    double gv = butterfly(th + (int64_t)g * L, L);
    total = (g == 0) ? gv : total + gv;
  }
  free(th);
  free(part);
  return total;
}

/* Canonical order of the column-segment layout, used by a solver that keeps
 * one small grid in a single work-group of waves*lanes threads, each thread
 * owning a short piece of one grid column:
 *   E = rows;  segments per column S = ceil(ny / E);  C = seg_cols >= nx;
 *   thread t = w*lanes + l (wavefront w, lane l) owns column c = t mod C and
 *   rows s*E .. s*E + E - 1 (those < ny) of segment s = t div C; threads with
 *   c >= nx or s >= S own nothing (their lane value is +0).
 *   Lane: one accumulator from +0, acc = fma(a, b, acc) over its rows in
 *     ascending order.
 *   Wavefront: xor butterfly (see butterfly()).
 *   Total: ((wave_0 + wave_1) + wave_2) + ...
 * The layout must cover the grid: seg_cols >= nx and waves*lanes >= C*S
 * (else NaN). */
static double dot_segments(int32_t nx, int32_t ny, const double* a, const double* b,
                           const oracle_order* o) {
  const int32_t E = o->rows, L = o->lanes, W = o->waves, C = o->seg_cols;
  const int64_t S = (ny + E - 1) / E;
  if (C < nx || (int64_t)W * L < (int64_t)C * S) return NAN;
  double lane[256];
  double total = 0.0;
  for (int32_t w = 0; w < W; ++w) {
    for (int32_t l = 0; l < L; ++l) {
      const int64_t t = (int64_t)w * L + l;
      const int64_t c = t % C, s = t / C;
      double acc = 0.0;
      if (s < S && c < nx)
        for (int64_t j = s * E; j < s * E + E && j < ny; ++j)
          acc = fma(a[j * nx + c], b[j * nx + c], acc);
      lane[l] = acc;
    }
    const double wv = butterfly(lane, L);
    total = (w == 0) ? wv : total + wv;
  }
  return total;
}

/* Canonical order of the z-march layout of the 3D operator (layout 2): the
 * grid is nx x plane x nz, stored as ny = plane * nz rows of nx (row
 * z * plane + y).  A tile is TW = cols_per_lane * lanes columns by `waves`
 * consecutive in-plane rows y by `rows` planes z:
 *   ntx = ceil(nx / TW); nty = ceil(plane / waves); ntz = ceil(nz / rows);
 *   tile t = (tz * nty + ty) * ntx + tx.
 *   Wavefront w of tile (tx, ty, tz) owns in-plane row y = ty * waves + w
 *   (nothing when y >= plane) and planes tz * rows .. tz * rows + rows - 1
 *   (those < nz); lane l owns columns tx * TW + l * cols_per_lane + e.
 *   Lane: one accumulator per owned column from +0, acc = fma(a, b, acc)
 *     over the wavefront's planes in ascending z; lane value
 *     ((acc_0 + acc_1) + ...); wavefront: xor butterfly; tile partial:
 *     waves in order; cross-tile: as in dot_canonical. */
static double dot_zmarch(int32_t nx, int32_t ny, const double* a, const double* b,
                         const oracle_order* o) {
  const int32_t cpl = o->cols_per_lane, L = o->lanes, W = o->waves, R = o->rows;
  const int32_t pl = o->plane, nz = ny / pl;
  const int32_t TW = cpl * L;
  const int64_t ntx = (nx + TW - 1) / TW, nty = (pl + W - 1) / W, ntz = (nz + R - 1) / R;
  const int64_t T = ntx * nty * ntz;
  double* part = (double*)malloc((size_t)T * sizeof(double));
#pragma omp parallel for schedule(static) collapse(3)
  for (int64_t tz = 0; tz < ntz; ++tz)
    for (int64_t ty = 0; ty < nty; ++ty)
      for (int64_t tx = 0; tx < ntx; ++tx) {
        double lane[256], accs[4096];  /* accs[l * cpl + e]: lane l, column e */
        double tile = 0.0;
        for (int32_t w = 0; w < W; ++w) {
          const int64_t y = ty * W + w;
          for (int32_t k = 0; k < TW; ++k) accs[k] = 0.0;
          for (int64_t z = tz * R; y < pl && z < tz * R + R && z < nz; ++z) {
            const int64_t j = z * pl + y;
            for (int32_t k = 0; k < TW; ++k) {
              const int64_t c = tx * TW + k;
              if (c < nx) accs[k] = fma(a[j * nx + c], b[j * nx + c], accs[k]);
            }
          }
          for (int32_t l = 0; l < L; ++l) {
            double v = accs[l * cpl];
            for (int32_t e = 1; e < cpl; ++e) v = v + accs[l * cpl + e];
            lane[l] = v;
          }
          const double wv = butterfly(lane, L);
          tile = (w == 0) ? wv : tile + wv;
        }
        part[(tz * nty + ty) * ntx + tx] = tile;
      }
  const int32_t T2 = o->threads2;
  double* th = (double*)malloc((size_t)T2 * sizeof(double));
  for (int32_t t = 0; t < T2; ++t) {
    double sacc = 0.0;
    for (int64_t k = t; k < T; k += T2) sacc = sacc + part[k];
    th[t] = sacc;
  }
  double total = 0.0;
  for (int32_t g = 0; g < T2 / L; ++g) {
    const double gv = butterfly(th + (int64_t)g * L, L);
    total = (g == 0) ? gv : total + gv;
  }
  free(th);
  free(part);
  return total;
}

/* Exported dot for the tests. */
double oracle_dot(int32_t nx, int32_t ny, int32_t mode, const oracle_order* o,
                  const double* a, const double* b) {
  if (mode == MODE_CANONICAL)
    return o->layout == 1   ? dot_segments(nx, ny, a, b, o)
           : o->layout == 2 ? dot_zmarch(nx, ny, a, b, o)
                            : dot_canonical(nx, ny, a, b, o);
  return dot_sequential((int64_t)nx * ny, a, b);
}

/* --------------------------------------------------------- CG context -- */

typedef struct {
  int32_t nx, ny, mode;
  const oracle_order* ord;
  int32_t rr_period; /* pipelined: residual replacement every rr_period
                        iterations (0: never) */
} ctx_t;

static double dot(const ctx_t* c, const double* a, const double* b) {
  return oracle_dot(c->nx, c->ny, c->mode, c->ord, a, b);
}

/* y <- y + a*x */
static void axpy(const ctx_t* c, int64_t n, double a, const double* x, double* y) {
  const int fused = c->mode == MODE_CANONICAL;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) y[k] = fused ? fma(a, x[k], y[k]) : y[k] + a * x[k];
}

/* y <- x + a*y */
static void xpay(const ctx_t* c, int64_t n, const double* x, double a, double* y) {
  const int fused = c->mode == MODE_CANONICAL;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) y[k] = fused ? fma(a, y[k], x[k]) : x[k] + a * y[k];
}

static void record(oracle_history* h, int64_t n, double gamma, const double* r,
                   const double* p, const double* x) {
  if (!h || h->count >= h->max_hist) return;
  int64_t m = h->count;
  if (h->gamma) h->gamma[m] = gamma;
  if (h->r) memcpy(h->r + m * n, r, (size_t)n * sizeof(double));
  if (h->p) memcpy(h->p + m * n, p, (size_t)n * sizeof(double));
  if (h->x) memcpy(h->x + m * n, x, (size_t)n * sizeof(double));
  h->count++;
}

/* Stopping and failure rules shared by both variants (readings of "until
 * convergence", which the paper leaves open):
 *   ||r||_2 <= tol ||b||_2 is evaluated as gamma <= (tol*tol)*(b,b);
 *   a non-finite gamma, or a non-positive / non-finite curvature term, is a
 *   breakdown; reaching maxit is NOT_CONVERGED, except that tol == 0 asks for
 *   exactly maxit iterations and then reports OK. */
static int stop_rule(double gamma, double thr, int32_t k, int32_t maxit, double tol) {
  if (!isfinite(gamma)) return OR_BREAKDOWN;
  if (gamma <= thr) return OR_OK;
  if (k >= maxit) return tol == 0.0 ? OR_OK : OR_NOT_CONVERGED;
  return -100; /* keep iterating */
}

static void finish(const csr_t* A, const ctx_t* c, const double* b, const double* x,
                   double bb, double gamma, oracle_result* res) {
  int64_t n = A->n;
  double* t = (double*)malloc((size_t)n * sizeof(double));
  spmv(A, x, t);
  for (int64_t k = 0; k < n; ++k) t[k] = b[k] - t[k];
  double rr = dot(c, t, t);
  free(t);
  res->rel_res_recursive = sqrt(gamma / bb);
  res->rel_res_true = sqrt(rr / bb);
}

/* Classic CG (Algorithm 1, stdCG) with starting vector x0 (NULL = zeros):
 *   r = b - A x0; p = r; gamma = (r,r)
 *   repeat: s = A p; pi = (p,s); alpha = gamma/pi; x += alpha p;
 *           r -= alpha s; gamma' = (r,r); beta = gamma'/gamma; p = r + beta p */
static int cg_classic(const csr_t* A, const ctx_t* c, const double* b, const double* x0,
                      double* x, double tol, int32_t maxit, oracle_result* res,
                      oracle_history* h) {
  const int64_t n = A->n;
  double* r = (double*)malloc((size_t)n * sizeof(double));
  double* p = (double*)malloc((size_t)n * sizeof(double));
  double* s = (double*)malloc((size_t)n * sizeof(double));
  if (!r || !p || !s) { free(r); free(p); free(s); return OR_E_NOMEM; }

  const double bb = dot(c, b, b);
  int32_t k = 0;
  int st;
  if (bb == 0.0) {  /* zero right-hand side: x = 0 solves it exactly */
    memset(x, 0, (size_t)n * sizeof(double));
    res->rel_res_recursive = res->rel_res_true = 0.0;
    st = OR_OK;
    goto done;
  }
  if (x0) memcpy(x, x0, (size_t)n * sizeof(double));
  else    memset(x, 0, (size_t)n * sizeof(double));
  spmv(A, x, s);
  for (int64_t i = 0; i < n; ++i) r[i] = b[i] - s[i];
  memcpy(p, r, (size_t)n * sizeof(double));
  const double thr = (tol * tol) * bb;
  double gamma = dot(c, r, r);
  record(h, n, gamma, r, p, x);
  for (;;) {
    st = stop_rule(gamma, thr, k, maxit, tol);
    if (st != -100) break;
    spmv(A, p, s);
    double pi = dot(c, p, s);
    if (!(pi > 0.0) || !isfinite(pi)) { st = OR_BREAKDOWN; break; }
    double alpha = gamma / pi;
    axpy(c, n, alpha, p, x);
    axpy(c, n, -alpha, s, r);
    double gnew = dot(c, r, r);
    double beta = gnew / gamma;
    xpay(c, n, r, beta, p);
    gamma = gnew;
    ++k;
    record(h, n, gamma, r, p, x);
  }
  finish(A, c, b, x, bb, gamma, res);
done:
  res->status = st;
  res->iterations = k;
  res->outer_iterations = 0;
  free(r); free(p); free(s);
  return st;
}

/* Modified CG (Algorithm 2, newCG), readings as in the file header:
 *   r = b - A x0; w = A r; gamma = (r,r); delta = (w,r)
 *   nvec = A w; beta = 0; alpha = gamma/delta; z = nvec; q = w; p = r
 *   x += alpha p; r -= alpha q; w -= alpha z                      (k = 1)
 *   repeat: gamma_old = gamma; gamma = (r,r); delta = (w,r); nvec = A w;
 *           beta = gamma/gamma_old; alpha = 1/(delta/gamma - beta/alpha);
 *           z = nvec + beta z; q = w + beta q; p = r + beta p;
 *           x += alpha p; r -= alpha q; w -= alpha z
 * The vector called n in the paper is nvec here (n is also the size). */
static int cg_pipelined(const csr_t* A, const ctx_t* c, const double* b, const double* x0,
                        double* x, double tol, int32_t maxit, oracle_result* res,
                        oracle_history* h) {
  const int64_t n = A->n;
  double* r = (double*)malloc((size_t)n * sizeof(double));
  double* w = (double*)malloc((size_t)n * sizeof(double));
  double* nv = (double*)malloc((size_t)n * sizeof(double));
  double* z = (double*)malloc((size_t)n * sizeof(double));
  double* q = (double*)malloc((size_t)n * sizeof(double));
  double* p = (double*)malloc((size_t)n * sizeof(double));
  if (!r || !w || !nv || !z || !q || !p) {
    free(r); free(w); free(nv); free(z); free(q); free(p); return OR_E_NOMEM;
  }
  const double bb = dot(c, b, b);
  int32_t k = 0;
  int st;
  double gamma = 0.0;
  if (bb == 0.0) {
    memset(x, 0, (size_t)n * sizeof(double));
    res->rel_res_recursive = res->rel_res_true = 0.0;
    st = OR_OK;
    goto done;
  }
  if (x0) memcpy(x, x0, (size_t)n * sizeof(double));
  else    memset(x, 0, (size_t)n * sizeof(double));
  spmv(A, x, nv);
  for (int64_t i = 0; i < n; ++i) r[i] = b[i] - nv[i];
  spmv(A, r, w);
  const double thr = (tol * tol) * bb;
  gamma = dot(c, r, r);
  double delta = dot(c, w, r);
  record(h, n, gamma, r, r, x);
  st = stop_rule(gamma, thr, k, maxit, tol);
  if (st != -100) goto fin;
  if (!(delta > 0.0) || !isfinite(delta)) { st = OR_BREAKDOWN; goto fin; }
  spmv(A, w, nv);
  double alpha = gamma / delta;
  memcpy(z, nv, (size_t)n * sizeof(double));
  memcpy(q, w, (size_t)n * sizeof(double));
  memcpy(p, r, (size_t)n * sizeof(double));
  axpy(c, n, alpha, p, x);
  axpy(c, n, -alpha, q, r);
  axpy(c, n, -alpha, z, w);
  k = 1;
  for (;;) {
    double gamma_old = gamma;
    gamma = dot(c, r, r);
    delta = dot(c, w, r);
    record(h, n, gamma, r, p, x);
    st = stop_rule(gamma, thr, k, maxit, tol);
    if (st != -100) break;
    spmv(A, w, nv);
    double beta = gamma / gamma_old;
    double den = delta / gamma - beta / alpha;
    if (!(den > 0.0) || !isfinite(den)) { st = OR_BREAKDOWN; break; }
    alpha = 1.0 / den;
    xpay(c, n, nv, beta, z);
    xpay(c, n, w, beta, q);
    xpay(c, n, r, beta, p);
    axpy(c, n, alpha, p, x);
    axpy(c, n, -alpha, q, r);
    axpy(c, n, -alpha, z, w);
    ++k;
    if (c->rr_period > 0 && k % c->rr_period == 0) {
      /* Residual replacement (the attainable-accuracy remedy for pipelined
       * CG of Cools, Yetkin, Agullo, Giraud and Vanroose): the recurrence
       * vectors are recomputed from their definitions, q = A p, z = A q,
       * r = b - A x, w = A r; gamma and delta are then formed from them at
       * the loop head as always, and the scalar recurrences continue. */
      spmv(A, p, q);
#if ORACLE_MUTANT != 5
      spmv(A, q, z);
#endif
      spmv(A, x, nv);
      for (int64_t i = 0; i < n; ++i) r[i] = b[i] - nv[i];
#if ORACLE_MUTANT != 4
      spmv(A, r, w);
#endif
    }
  }
fin:
  finish(A, c, b, x, bb, gamma, res);
done:
  res->status = st;
  res->iterations = k;
  res->outer_iterations = 0;
  free(r); free(w); free(nv); free(z); free(q); free(p);
  return st;
}

static int order_valid(const oracle_order* o, int32_t nx, int32_t ny) {
  if (!o || o->lanes < 1 || o->lanes > 256 || (o->lanes & (o->lanes - 1)) || o->waves < 1 ||
      o->rows < 1)
    return 0;
  if (o->layout == 1)
    return o->seg_cols >= nx &&
           (int64_t)o->waves * o->lanes >= (int64_t)o->seg_cols * ((ny + o->rows - 1) / o->rows);
  if (o->layout == 2 && !(o->plane >= 1 && ny % o->plane == 0)) return 0;
  return (o->layout == 0 || o->layout == 2) && o->cols_per_lane >= 1 &&
         o->cols_per_lane <= 16 && o->threads2 >= o->lanes && o->threads2 % o->lanes == 0;
}

/* Solve A x = b.  variant: 0 classic, 1 pipelined.  mode: 0 sequential,
 * 1 canonical (then ord must describe the order).  x0 may be NULL.
 * Returns the status (also in res). */
static int cg_any(int32_t variant, int32_t mode, const oracle_order* ord, int32_t nx,
                  int32_t ny, const double* b, const double* x0, double* x, double tol,
                  int32_t maxit, int32_t rr_period, oracle_result* res, oracle_history* hist);

int oracle_cg(int32_t variant, int32_t mode, const oracle_order* ord, int32_t nx,
              int32_t ny, const double* b, const double* x0, double* x, double tol,
              int32_t maxit, oracle_result* res, oracle_history* hist) {
  return cg_any(variant, mode, ord, nx, ny, b, x0, x, tol, maxit, 0, res, hist);
}

/* oracle_cg with residual replacement every rr_period iterations of the
 * pipelined variant (rr_period >= 1; classic CG ignores it). */
int oracle_cg_rr(int32_t variant, int32_t mode, const oracle_order* ord, int32_t nx,
                 int32_t ny, const double* b, const double* x0, double* x, double tol,
                 int32_t maxit, int32_t rr_period, oracle_result* res) {
  if (rr_period < 1) return OR_E_INVALID;
  return cg_any(variant, mode, ord, nx, ny, b, x0, x, tol, maxit, rr_period, res, NULL);
}

static int cg_any(int32_t variant, int32_t mode, const oracle_order* ord, int32_t nx,
                  int32_t ny, const double* b, const double* x0, double* x, double tol,
                  int32_t maxit, int32_t rr_period, oracle_result* res, oracle_history* hist) {
  if (nx < 1 || ny < 1 || !b || !x || !res || maxit < 1 || !(tol >= 0.0) || tol >= 1.0)
    return OR_E_INVALID;
  if (mode == MODE_CANONICAL && !order_valid(ord, nx, ny)) return OR_E_INVALID;
  if (hist) hist->count = 0;
  csr_t A;
  int rc = csr_build(&A, nx, ny, mode == MODE_CANONICAL ? 1 : 0, 0);
  if (rc) return rc;
  ctx_t c = {nx, ny, mode, ord, rr_period};
  memset(res, 0, sizeof(*res));
  const double t0 = wall_now();
  rc = (variant == VARIANT_PIPELINED) ? cg_pipelined(&A, &c, b, x0, x, tol, maxit, res, hist)
                                      : cg_classic(&A, &c, b, x0, x, tol, maxit, res, hist);
  g_solve_seconds = wall_now() - t0;
  csr_free(&A);
  return rc;
}

/* ------------------------------------------------ 3D 7-point Laplacian -- */

/* The unscaled 7-point Laplacian on an nx-by-ny-by-nz interior grid with zero
 * Dirichlet boundary: centre 6, the six face neighbours -1.  Unknown (i, j, l),
 * 0 <= i < nx, 0 <= j < ny, 0 <= l < nz, has index k = (l*ny + j)*nx + i: nz
 * planes of ny rows, i.e. ny*nz rows of nx, on which every dot product of the
 * 2D case (and its canonical orders) applies unchanged. */
int64_t oracle_csr3_nnz(int32_t nx, int32_t ny, int32_t nz) {
  if (nx < 1 || ny < 1 || nz < 1) return -1;
  const int64_t n = (int64_t)nx * ny * nz;
  return n + 2 * (int64_t)(nx - 1) * ny * nz + 2 * (int64_t)nx * (ny - 1) * nz +
         2 * (int64_t)nx * ny * (nz - 1);
}

/* order 0: entries of a row sorted by column.  order 1: centre, west (i-1),
 * east (i+1), south (j-1), north (j+1), below (l-1), above (l+1), so that the
 * CSR loop evaluates (((((6uC - uW) - uE) - uS) - uN) - uB) - uT. */
int64_t oracle_csr3_assemble(int32_t nx, int32_t ny, int32_t nz, int32_t order,
                             int64_t* row_ptr, int32_t* col, double* val) {
  if (nx < 1 || ny < 1 || nz < 1) return OR_E_INVALID;
  const int64_t plane = (int64_t)nx * ny;
  int64_t e = 0;
  for (int32_t l = 0; l < nz; ++l) {
    for (int32_t j = 0; j < ny; ++j) {
      for (int32_t i = 0; i < nx; ++i) {
        const int64_t k = l * plane + (int64_t)j * nx + i;
        row_ptr[k] = e;
        if (order == 0) {
          if (l > 0)      { col[e] = (int32_t)(k - plane); val[e++] = -1.0; }
          if (j > 0)      { col[e] = (int32_t)(k - nx);    val[e++] = -1.0; }
          if (i > 0)      { col[e] = (int32_t)(k - 1);     val[e++] = -1.0; }
          col[e] = (int32_t)k; val[e++] = 6.0;
          if (i < nx - 1) { col[e] = (int32_t)(k + 1);     val[e++] = -1.0; }
          if (j < ny - 1) { col[e] = (int32_t)(k + nx);    val[e++] = -1.0; }
          if (l < nz - 1) { col[e] = (int32_t)(k + plane); val[e++] = -1.0; }
        } else {
          col[e] = (int32_t)k; val[e++] = 6.0;
          if (i > 0)      { col[e] = (int32_t)(k - 1);     val[e++] = -1.0; }
          if (i < nx - 1) { col[e] = (int32_t)(k + 1);     val[e++] = -1.0; }
          if (j > 0)      { col[e] = (int32_t)(k - nx);    val[e++] = -1.0; }
          if (j < ny - 1) { col[e] = (int32_t)(k + nx);    val[e++] = -1.0; }
          if (l > 0)      { col[e] = (int32_t)(k - plane); val[e++] = -1.0; }
          if (l < nz - 1) { col[e] = (int32_t)(k + plane); val[e++] = -1.0; }
        }
      }
    }
  }
  row_ptr[plane * nz] = e;
  return e;
}

static int csr3_build(csr_t* A, int32_t nx, int32_t ny, int32_t nz, int32_t order) {
  memset(A, 0, sizeof(*A));
  const int64_t nnz = oracle_csr3_nnz(nx, ny, nz);
  if (nnz < 0 || (int64_t)nx * ny * nz >= ((int64_t)1 << 31)) return OR_E_INVALID;
  A->nx = nx; A->ny = ny * nz; A->n = (int64_t)nx * ny * nz;
  A->row_ptr = (int64_t*)malloc((size_t)(A->n + 1) * sizeof(int64_t));
  A->col = (int32_t*)malloc((size_t)nnz * sizeof(int32_t));
  A->val = (double*)malloc((size_t)nnz * sizeof(double));
  if (!A->row_ptr || !A->col || !A->val) { csr_free(A); return OR_E_NOMEM; }
  oracle_csr3_assemble(nx, ny, nz, order, A->row_ptr, A->col, A->val);
  return OR_OK;
}

int oracle_spmv3(int32_t nx, int32_t ny, int32_t nz, int32_t order, const double* u,
                 double* y) {
  csr_t A;
  int rc = csr3_build(&A, nx, ny, nz, order);
  if (rc) return rc;
  spmv(&A, u, y);
  csr_free(&A);
  return OR_OK;
}

/* Algorithms 1 and 2 on the 7-point operator (the same loops as oracle_cg;
 * canonical dots over the ny*nz rows of nx). */
int oracle_cg3(int32_t variant, int32_t mode, const oracle_order* ord, int32_t nx, int32_t ny,
               int32_t nz, const double* b, const double* x0, double* x, double tol,
               int32_t maxit, oracle_result* res) {
  if (nx < 1 || ny < 1 || nz < 1 || !b || !x || !res || maxit < 1 || !(tol >= 0.0) ||
      tol >= 1.0 || (variant != VARIANT_CLASSIC && variant != VARIANT_PIPELINED))
    return OR_E_INVALID;
  if ((int64_t)ny * nz >= ((int64_t)1 << 31)) return OR_E_INVALID;
  const int32_t rows = ny * nz;
  if (mode == MODE_CANONICAL && !order_valid(ord, nx, rows)) return OR_E_INVALID;
  csr_t A;
  int rc = csr3_build(&A, nx, ny, nz, mode == MODE_CANONICAL ? 1 : 0);
  if (rc) return rc;
  ctx_t c = {nx, rows, mode, ord, 0};
  memset(res, 0, sizeof(*res));
  const double t0 = wall_now();
  rc = (variant == VARIANT_PIPELINED) ? cg_pipelined(&A, &c, b, x0, x, tol, maxit, res, NULL)
                                      : cg_classic(&A, &c, b, x0, x, tol, maxit, res, NULL);
  g_solve_seconds = wall_now() - t0;
  csr_free(&A);
  return rc;
}

/* ------------------------------------- variable-coefficient 5-point -- */

/* The finite-volume operator of -div(k grad u) on the nx-by-ny grid with zero
 * Dirichlet boundary and face conductivities: kx holds ny rows of nx + 1 faces
 * (kx[j][i] between cells i-1 and i of row j; i = 0 and i = nx are boundary
 * faces), ky holds ny + 1 rows of nx faces (ky[j][i] between rows j-1 and j).
 * With kW = kx[j][i], kE = kx[j][i+1], kS = ky[j][i], kN = ky[j+1][i]:
 *   A[k][k] = ((kW + kE) + kS) + kN,  A[k][k-1] = -kW,  A[k][k+1] = -kE,
 *   A[k][k-nx] = -kS,  A[k][k+nx] = -kN   (neighbours inside the grid only).
 * Every k = 1 gives the 5-point operator of Section II-B.  Entry orders as for
 * oracle_csr_assemble (order 1: centre, west, east, south, north, so that the
 * CSR loop evaluates (((d uC - kW uW) - kE uE) - kS uS) - kN uN, each product
 * rounded before its subtraction). */
int64_t oracle_csr_vc_assemble(int32_t nx, int32_t ny, const double* kx, const double* ky,
                               int32_t order, int64_t* row_ptr, int32_t* col, double* val) {
  if (nx < 1 || ny < 1 || !kx || !ky) return OR_E_INVALID;
  int64_t e = 0;
  for (int32_t j = 0; j < ny; ++j) {
    for (int32_t i = 0; i < nx; ++i) {
      const int64_t k = (int64_t)j * nx + i;
      const double kw = kx[(int64_t)j * (nx + 1) + i], ke = kx[(int64_t)j * (nx + 1) + i + 1];
      const double ks = ky[(int64_t)j * nx + i], kn = ky[(int64_t)(j + 1) * nx + i];
      const double d = ((kw + ke) + ks) + kn;
      row_ptr[k] = e;
      if (order == 0) {
        if (j > 0)      { col[e] = (int32_t)(k - nx); val[e++] = -ks; }
        if (i > 0)      { col[e] = (int32_t)(k - 1);  val[e++] = -kw; }
        col[e] = (int32_t)k; val[e++] = d;
        if (i < nx - 1) { col[e] = (int32_t)(k + 1);  val[e++] = -ke; }
        if (j < ny - 1) { col[e] = (int32_t)(k + nx); val[e++] = -kn; }
      } else {
        col[e] = (int32_t)k; val[e++] = d;
        if (i > 0)      { col[e] = (int32_t)(k - 1);  val[e++] = -kw; }
        if (i < nx - 1) { col[e] = (int32_t)(k + 1);  val[e++] = -ke; }
        if (j > 0)      { col[e] = (int32_t)(k - nx); val[e++] = -ks; }
        if (j < ny - 1) { col[e] = (int32_t)(k + nx); val[e++] = -kn; }
      }
    }
  }
  row_ptr[(int64_t)nx * ny] = e;
  return e;
}

static int csr_vc_build(csr_t* A, int32_t nx, int32_t ny, const double* kx, const double* ky,
                        int32_t order) {
  memset(A, 0, sizeof(*A));
  const int64_t nnz = oracle_csr_nnz(nx, ny);
  if (nnz < 0 || !kx || !ky) return OR_E_INVALID;
  A->nx = nx; A->ny = ny; A->n = (int64_t)nx * ny;
  A->row_ptr = (int64_t*)malloc((size_t)(A->n + 1) * sizeof(int64_t));
  A->col = (int32_t*)malloc((size_t)nnz * sizeof(int32_t));
  A->val = (double*)malloc((size_t)nnz * sizeof(double));
  if (!A->row_ptr || !A->col || !A->val) { csr_free(A); return OR_E_NOMEM; }
  oracle_csr_vc_assemble(nx, ny, kx, ky, order, A->row_ptr, A->col, A->val);
  return OR_OK;
}

int oracle_spmv_vc(int32_t nx, int32_t ny, const double* kx, const double* ky, int32_t order,
                   const double* u, double* y) {
  csr_t A;
  int rc = csr_vc_build(&A, nx, ny, kx, ky, order);
  if (rc) return rc;
  spmv(&A, u, y);
  csr_free(&A);
  return OR_OK;
}

/* Algorithms 1 and 2 on the variable-coefficient operator (the same loops as
 * oracle_cg); rr_period > 0: residual replacement every rr_period iterations
 * of the pipelined variant, as in oracle_cg_rr. */
int oracle_cg_vc_rr(int32_t variant, int32_t mode, const oracle_order* ord, int32_t nx,
                    int32_t ny, const double* kx, const double* ky, const double* b,
                    const double* x0, double* x, double tol, int32_t maxit, int32_t rr_period,
                    oracle_result* res) {
  if (nx < 1 || ny < 1 || !b || !x || !res || maxit < 1 || !(tol >= 0.0) || tol >= 1.0 ||
      (variant != VARIANT_CLASSIC && variant != VARIANT_PIPELINED) || rr_period < 0)
    return OR_E_INVALID;
  if (mode == MODE_CANONICAL && !order_valid(ord, nx, ny)) return OR_E_INVALID;
  csr_t A;
  int rc = csr_vc_build(&A, nx, ny, kx, ky, mode == MODE_CANONICAL ? 1 : 0);
  if (rc) return rc;
  ctx_t c = {nx, ny, mode, ord, rr_period};
  memset(res, 0, sizeof(*res));
  const double t0 = wall_now();
  rc = (variant == VARIANT_PIPELINED) ? cg_pipelined(&A, &c, b, x0, x, tol, maxit, res, NULL)
                                      : cg_classic(&A, &c, b, x0, x, tol, maxit, res, NULL);
  g_solve_seconds = wall_now() - t0;
  csr_free(&A);
  return rc;
}

int oracle_cg_vc(int32_t variant, int32_t mode, const oracle_order* ord, int32_t nx, int32_t ny,
                 const double* kx, const double* ky, const double* b, const double* x0,
                 double* x, double tol, int32_t maxit, oracle_result* res) {
  return oracle_cg_vc_rr(variant, mode, ord, nx, ny, kx, ky, b, x0, x, tol, maxit, 0, res);
}

/* ------------------------------------------ Chebyshev-preconditioned CG -- */

/* The preconditioner M^-1 = p_s(A): s steps of Chebyshev semi-iteration on
 * A y = r from y = 0, over the interval [lo, hi] = [lmax / (2 s^2), lmax],
 * where lmax = 4 + 2cos(pi/(nx+1)) + 2cos(pi/(ny+1)) is the largest eigenvalue
 * of A (closed form for this operator).  With theta = (hi + lo)/2,
 * delta = (hi - lo)/2, sigma = theta/delta, rho_0 = 1/sigma:
 *   d_0 = r * (1/theta);  y_1 = d_0;
 *   for k = 1 .. s-1:  r_k = r_(k-1) - A d_(k-1);
 *                      rho_k = 1 / (2 sigma - rho_(k-1));
 *                      d_k = (rho_k rho_(k-1)) d_(k-1) + (2 rho_k / delta) r_k;
 *                      y_(k+1) = y_k + d_k;
 *   z = y_s.
 * (the Chebyshev iteration of Saad, Iterative Methods for Sparse Linear
 * Systems, Section 12.3.)  Its residual polynomial R(l) = T_s((theta - l)/delta)
 * / T_s(sigma) lies in [-1/T_s(sigma), 1/T_s(sigma)] on [lo, hi] and in
 * [1/T_s(sigma), 1) on (0, lo), so p_s(l) = (1 - R(l))/l > 0 on the whole
 * spectrum and M is SPD.  The upper end sits at lmax itself and not below it:
 * for even s, R(lmax) would otherwise be near 1 and p_s(A) A would nearly
 * vanish on the highest modes.  The lower end lmax/(2 s^2) leaves the lowest
 * modes to the outer CG, which handles a few small outlying eigenvalues well,
 * and makes the bulk of the spectrum of p_s(A) A lie within 1 -+ 1/T_s(sigma).
 * c0 = 1/theta, c1[k-1] = rho_k rho_(k-1), c2[k-1] = 2 rho_k / delta. */
int oracle_cheb_coeffs(int32_t nx, int32_t ny, int32_t s, double* c0, double* c1,
                       double* c2) {
  if (nx < 1 || ny < 1 || s < 1 || !c0 || (s > 1 && (!c1 || !c2))) return OR_E_INVALID;
  const double pi = 3.14159265358979323846;
  const double hi = 4.0 + 2.0 * cos(pi / (double)(nx + 1)) + 2.0 * cos(pi / (double)(ny + 1));
  const double lo = hi / (2.0 * (double)s * (double)s);
  const double theta = (hi + lo) / 2.0, delta = (hi - lo) / 2.0;
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  *c0 = 1.0 / theta;
  for (int32_t k = 1; k < s; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    c1[k - 1] = rn * rho;
    c2[k - 1] = 2.0 * rn / delta;
    rho = rn;
  }
  return OR_OK;
}

/* z = M^-1 r.  Canonical mode: d_0 = r * c0; d_k = fma(c1, d_(k-1), c2 * r_k);
 * r_k = r_(k-1) - (A d_(k-1)) with the canonical stencil order; y adds d in
 * order.  Sequential mode: d_k = c1 * d_(k-1) + c2 * r_k with both products
 * rounded. */
static int cheb_apply(const csr_t* A, int32_t mode, int32_t s, const double* cc0,
                      const double* c1, const double* c2, const double* r, double* z) {
  const int64_t n = A->n;
  double* d = (double*)malloc((size_t)n * sizeof(double));
  double* rk = (double*)malloc((size_t)n * sizeof(double));
  double* t = (double*)malloc((size_t)n * sizeof(double));
  if (!d || !rk || !t) { free(d); free(rk); free(t); return OR_E_NOMEM; }
  const double c0 = *cc0;
  for (int64_t i = 0; i < n; ++i) {
    d[i] = r[i] * c0;
    z[i] = d[i];
    rk[i] = r[i];
  }
  for (int32_t k = 1; k < s; ++k) {
    spmv(A, d, t);
    for (int64_t i = 0; i < n; ++i) {
      rk[i] = rk[i] - t[i];
      d[i] = mode == MODE_CANONICAL ? fma(c1[k - 1], d[i], c2[k - 1] * rk[i])
                                    : c1[k - 1] * d[i] + c2[k - 1] * rk[i];
      z[i] = z[i] + d[i];
    }
  }
  free(d); free(rk); free(t);
  return OR_OK;
}

int oracle_cheb_apply(int32_t nx, int32_t ny, int32_t mode, int32_t s, const double* r,
                      double* z) {
  if (nx < 1 || ny < 1 || s < 1 || s > 64 || !r || !z) return OR_E_INVALID;
  double c0, c1[64], c2[64];
  oracle_cheb_coeffs(nx, ny, s, &c0, c1, c2);
  csr_t A;
  int rc = csr_build(&A, nx, ny, mode == MODE_CANONICAL ? 1 : 0, 0);
  if (rc) return rc;
  rc = cheb_apply(&A, mode, s, &c0, c1, c2, r, z);
  csr_free(&A);
  return rc;
}

/* Preconditioned pipelined CG (Ghysels and Vanroose's preconditioned form of
 * Algorithm 2, M^-1 = p_s(A)) from x0, with Algorithm 2's first block
 * unrolled and the stop test on the unpreconditioned (r,r):
 *   r = b - A x0; u = M^-1 r; w = A u
 *   gamma = (r,u); delta = (w,u); stop test on (r,r)
 *   breakdown unless delta > 0; m = M^-1 w; n = A m; alpha = gamma/delta
 *   z = n; q = m; s = w; p = u
 *   x += alpha p; r -= alpha s; u -= alpha q; w -= alpha z      (k = 1)
 *   repeat: gamma_old = gamma; gamma = (r,u); delta = (w,u); stop test on (r,r)
 *           m = M^-1 w; n = A m; beta = gamma/gamma_old;
 *           alpha = 1/(delta/gamma - beta/alpha) (breakdown unless the
 *           denominator is > 0); z = n + beta z; q = m + beta q;
 *           s = w + beta s; p = u + beta p;
 *           x += alpha p; r -= alpha s; u -= alpha q; w -= alpha z
 * In exact arithmetic its iterates are preconditioned classic CG's.  Every dot
 * follows ord in canonical mode. */
static int ppcg_run(const csr_t* A, const ctx_t* c, int32_t sdeg, const double* cc0,
                    const double* c1, const double* c2, const double* b, const double* x0,
                    double* x, double tol, int32_t maxit, oracle_result* res) {
  const int64_t n = A->n;
  double* v[9];
  for (int i = 0; i < 9; ++i) v[i] = (double*)malloc((size_t)n * sizeof(double));
  double *r = v[0], *u = v[1], *w = v[2], *m = v[3], *nv = v[4], *z = v[5], *q = v[6],
         *sv = v[7], *p = v[8];
  int st = OR_OK, rc;
  int32_t k = 0;
  double rr = 0.0;
  const double bb = dot(c, b, b);
  for (int i = 0; i < 9; ++i)
    if (!v[i]) { st = OR_E_NOMEM; goto done; }
  if (bb == 0.0) {
    memset(x, 0, (size_t)n * sizeof(double));
    res->rel_res_recursive = res->rel_res_true = 0.0;
    goto done;
  }
  if (x0) memcpy(x, x0, (size_t)n * sizeof(double));
  else    memset(x, 0, (size_t)n * sizeof(double));
  spmv(A, x, nv);
  for (int64_t i = 0; i < n; ++i) r[i] = b[i] - nv[i];
  if ((rc = cheb_apply(A, c->mode, sdeg, cc0, c1, c2, r, u))) { st = rc; goto done; }
  spmv(A, u, w);
  const double thr = (tol * tol) * bb;
  double gamma = dot(c, r, u), delta = dot(c, w, u);
  rr = dot(c, r, r);
  st = stop_rule(rr, thr, k, maxit, tol);
  if (st != -100) goto fin;
  if (!(delta > 0.0) || !isfinite(delta)) { st = OR_BREAKDOWN; goto fin; }
  if ((rc = cheb_apply(A, c->mode, sdeg, cc0, c1, c2, w, m))) { st = rc; goto done; }
  spmv(A, m, nv);
  double alpha = gamma / delta;
  memcpy(z, nv, (size_t)n * sizeof(double));
  memcpy(q, m, (size_t)n * sizeof(double));
  memcpy(sv, w, (size_t)n * sizeof(double));
  memcpy(p, u, (size_t)n * sizeof(double));
  axpy(c, n, alpha, p, x);
  axpy(c, n, -alpha, sv, r);
  axpy(c, n, -alpha, q, u);
  axpy(c, n, -alpha, z, w);
  k = 1;
  for (;;) {
    const double gamma_old = gamma;
    gamma = dot(c, r, u);
    delta = dot(c, w, u);
    rr = dot(c, r, r);
    st = stop_rule(rr, thr, k, maxit, tol);
    if (st != -100) break;
    if ((rc = cheb_apply(A, c->mode, sdeg, cc0, c1, c2, w, m))) { st = rc; goto done; }
    spmv(A, m, nv);
    const double beta = gamma / gamma_old;
    const double den = delta / gamma - beta / alpha;
    if (!(den > 0.0) || !isfinite(den)) { st = OR_BREAKDOWN; break; }
    alpha = 1.0 / den;
    xpay(c, n, nv, beta, z);
    xpay(c, n, m, beta, q);
    xpay(c, n, w, beta, sv);
    xpay(c, n, u, beta, p);
    axpy(c, n, alpha, p, x);
    axpy(c, n, -alpha, sv, r);
    axpy(c, n, -alpha, q, u);
    axpy(c, n, -alpha, z, w);
    ++k;
  }
fin:
  finish(A, c, b, x, bb, rr, res);
done:
  res->status = st;
  res->iterations = k;
  res->outer_iterations = 0;
  for (int i = 0; i < 9; ++i) free(v[i]);
  return st;
}

/* Preconditioned classic CG (Algorithm 1 with M^-1 = p_s(A)) from x0:
 *   r = b - A x0; gamma = (r,r)
 *   repeat: stop test on gamma (as for CG); z = M^-1 r; rho = (r,z)
 *           (breakdown unless 0 < rho < inf); p = z (first) or
 *           z + (rho/rho_old) p; s = A p; pi = (p,s); alpha = rho/pi;
 *           x += alpha p; r -= alpha s; gamma = (r,r); rho_old = rho
 * Canonical mode: rho follows ord_rho (NULL: ord), every other dot ord.
 * variant 1 runs the preconditioned pipelined CG above (ord_rho unused). */
int oracle_pcg(int32_t variant, int32_t mode, const oracle_order* ord,
               const oracle_order* ord_rho, int32_t nx, int32_t ny, int32_t sdeg,
               const double* b, const double* x0, double* x, double tol, int32_t maxit,
               oracle_result* res) {
  if (nx < 1 || ny < 1 || !b || !x || !res || maxit < 1 || !(tol >= 0.0) || tol >= 1.0 ||
      sdeg < 1 || sdeg > 64 || (variant != VARIANT_CLASSIC && variant != VARIANT_PIPELINED))
    return OR_E_INVALID;
  if (!ord_rho) ord_rho = ord;
  if (mode == MODE_CANONICAL && (!order_valid(ord, nx, ny) || !order_valid(ord_rho, nx, ny)))
    return OR_E_INVALID;
  double c0, c1[64], c2[64];
  oracle_cheb_coeffs(nx, ny, sdeg, &c0, c1, c2);
  csr_t A;
  int rc = csr_build(&A, nx, ny, mode == MODE_CANONICAL ? 1 : 0, 0);
  if (rc) return rc;
  ctx_t c = {nx, ny, mode, ord, 0};
  ctx_t c_rho = {nx, ny, mode, ord_rho, 0};
  memset(res, 0, sizeof(*res));
  if (variant == VARIANT_PIPELINED) {
    rc = ppcg_run(&A, &c, sdeg, &c0, c1, c2, b, x0, x, tol, maxit, res);
    csr_free(&A);
    return rc;
  }
  const int64_t n = A.n;
  double* r = (double*)malloc((size_t)n * sizeof(double));
  double* z = (double*)malloc((size_t)n * sizeof(double));
  double* p = (double*)malloc((size_t)n * sizeof(double));
  double* s = (double*)malloc((size_t)n * sizeof(double));
  int st = OR_OK;
  int32_t k = 0;
  double gamma = 0.0, rho_old = 0.0;
  const double bb = dot(&c, b, b);
  if (!r || !z || !p || !s) { st = OR_E_NOMEM; goto done; }
  if (bb == 0.0) {
    memset(x, 0, (size_t)n * sizeof(double));
    goto done;
  }
  if (x0) memcpy(x, x0, (size_t)n * sizeof(double));
  else    memset(x, 0, (size_t)n * sizeof(double));
  spmv(&A, x, s);
  for (int64_t i = 0; i < n; ++i) r[i] = b[i] - s[i];
  const double thr = (tol * tol) * bb;
  gamma = dot(&c, r, r);
  for (;;) {
    st = stop_rule(gamma, thr, k, maxit, tol);
    if (st != -100) break;
    if ((rc = cheb_apply(&A, mode, sdeg, &c0, c1, c2, r, z))) { st = rc; break; }
    const double rho = dot(&c_rho, r, z);
    if (!(rho > 0.0) || !isfinite(rho)) { st = OR_BREAKDOWN; break; }
    if (k == 0) memcpy(p, z, (size_t)n * sizeof(double));
    else        xpay(&c, n, z, rho / rho_old, p);
    spmv(&A, p, s);
    const double pi = dot(&c, p, s);
    if (!(pi > 0.0) || !isfinite(pi)) { st = OR_BREAKDOWN; break; }
    const double alpha = rho / pi;
    axpy(&c, n, alpha, p, x);
    axpy(&c, n, -alpha, s, r);
    gamma = dot(&c, r, r);
    rho_old = rho;
    ++k;
  }
  finish(&A, &c, b, x, bb, gamma, res);
done:
  res->status = st;
  res->iterations = k;
  free(r); free(z); free(p); free(s);
  csr_free(&A);
  return st;
}

/* ---------------------------------------------------------- refinement -- */

#if ORACLE_MUTANT == 1
typedef double inner_t;
#define spmv_inner spmv
#else
typedef float inner_t;
#define spmv_inner spmv_f32
#endif
#if ORACLE_MUTANT == 3
typedef double inner_scalar_t;
#else
typedef inner_t inner_scalar_t;
#endif

static double dot_f32_in_f64(int64_t n, const inner_t* a, const inner_t* b) {
  /* each product of two binary32 values is exact in binary64 */
#if ORACLE_MUTANT == 2
  float s = 0.0f;
  for (int64_t k = 0; k < n; ++k) s = s + (float)((double)a[k] * (double)b[k]);
  return s;
#else
  double s = 0.0;
  for (int64_t k = 0; k < n; ++k) s = s + (double)a[k] * (double)b[k];
  return s;
#endif
}

/* FP32-inner / FP64-outer iterative refinement around classic CG:
 *   outer: r = b - A x (FP64); stop when (r,r) <= tol^2 (b,b);
 *          s = ||r||; rho = fp32(r * (1/s));
 *   inner: classic CG on A d = rho with FP32 vectors and FP32 stencil/axpy
 *          arithmetic, FP64 dot products, scalars alpha/beta computed in FP64
 *          and rounded to FP32 once; stop when (ri,ri) <= e^2 (rho,rho) with
 *          e = max(inner_tol, (tol/2) ||b|| / s) (adaptive: no further than
 *          the outer tolerance needs);
 *          a breakdown of the inner solve ends it early;
 *   update: x += s * fp64(d).
 * maxit caps the total number of inner iterations; an outer step whose inner
 * solve made no iteration is a breakdown. */
/* z = M^-1 r in binary32: the Chebyshev recurrence of cheb_apply with the
 * coefficients rounded to binary32 once and every operation a binary32 one
 * (d_k = c1 d_(k-1) + c2 r_k with both products rounded). */
static void cheb_apply_f32(const csr_t* A, int32_t s, float c0, const float* c1,
                           const float* c2, const float* r, float* z, float* d, float* rk,
                           float* t) {
  const int64_t n = A->n;
  for (int64_t i = 0; i < n; ++i) {
    d[i] = r[i] * c0;
    z[i] = d[i];
    rk[i] = r[i];
  }
  for (int32_t k = 1; k < s; ++k) {
    spmv_f32(A, d, t);
    for (int64_t i = 0; i < n; ++i) {
      rk[i] = rk[i] - t[i];
      d[i] = c1[k - 1] * d[i] + c2[k - 1] * rk[i];
      z[i] = z[i] + d[i];
    }
  }
}

static int refine_any(int32_t nx, int32_t ny, const double* b, const double* x0, double* x,
                      double tol, double inner_tol, int32_t maxit, int32_t sdeg,
                      oracle_result* res);

/* Exported z = M^-1 r in binary32 (cheb_apply_f32) for the tests. */
int oracle_cheb_apply_f32(int32_t nx, int32_t ny, int32_t sdeg, const float* r, float* z) {
  if (nx < 1 || ny < 1 || sdeg < 1 || sdeg > 64 || !r || !z) return OR_E_INVALID;
  double c0, c1[64], c2[64];
  float c1f[64], c2f[64];
  oracle_cheb_coeffs(nx, ny, sdeg, &c0, c1, c2);
  for (int32_t k = 0; k + 1 < sdeg; ++k) {
    c1f[k] = (float)c1[k];
    c2f[k] = (float)c2[k];
  }
  csr_t A;
  int rc = csr_build(&A, nx, ny, 0, 1);
  if (rc) return rc;
  const int64_t n = A.n;
  float* w = (float*)malloc((size_t)n * 3 * sizeof(float));
  if (!w) {
    csr_free(&A);
    return OR_E_NOMEM;
  }
  cheb_apply_f32(&A, sdeg, (float)c0, c1f, c2f, r, z, w, w + n, w + 2 * n);
  free(w);
  csr_free(&A);
  return OR_OK;
}

int oracle_refine(int32_t nx, int32_t ny, const double* b, const double* x0, double* x,
                  double tol, double inner_tol, int32_t maxit, oracle_result* res) {
  return refine_any(nx, ny, b, x0, x, tol, inner_tol, maxit, 0, res);
}

/* Refinement whose inner solve is preconditioned classic CG in binary32 with
 * M^-1 = p_s(A) (the Chebyshev preconditioner of oracle_pcg, its recurrence in
 * binary32): z = M^-1 ri, rho = (ri, z) in binary64, p = z + beta p, alpha =
 * rho / (p, A p) and beta = rho / rho_old computed in binary64 and rounded to
 * binary32 once; the inner stop test stays on (ri, ri). */
int oracle_refine_pc(int32_t nx, int32_t ny, const double* b, const double* x0, double* x,
                     double tol, double inner_tol, int32_t maxit, int32_t sdeg,
                     oracle_result* res) {
  if (sdeg < 1 || sdeg > 64) return OR_E_INVALID;
  return refine_any(nx, ny, b, x0, x, tol, inner_tol, maxit, sdeg, res);
}

static int refine_any(int32_t nx, int32_t ny, const double* b, const double* x0, double* x,
                      double tol, double inner_tol, int32_t maxit, int32_t sdeg,
                      oracle_result* res) {
  if (nx < 1 || ny < 1 || !b || !x || !res || maxit < 1 || !(tol >= 0.0) || tol >= 1.0 ||
      !(inner_tol > 0.0) || inner_tol >= 1.0)
    return OR_E_INVALID;
  csr_t A;
  int rc = csr_build(&A, nx, ny, 0, 1);
  if (rc) return rc;
  const int64_t n = A.n;
  double* r = (double*)malloc((size_t)n * sizeof(double));
  inner_t* ri = (inner_t*)malloc((size_t)n * sizeof(inner_t));
  inner_t* d = (inner_t*)malloc((size_t)n * sizeof(inner_t));
  inner_t* p = (inner_t*)malloc((size_t)n * sizeof(inner_t));
  inner_t* s = (inner_t*)malloc((size_t)n * sizeof(inner_t));
  /* preconditioned: z and the Chebyshev recurrence's work vectors */
  float* zc = sdeg ? (float*)malloc((size_t)n * 4 * sizeof(float)) : NULL;
  float c0f = 0.0f, c1f[64], c2f[64];
  if (sdeg) {
    double c0, c1[64], c2[64];
    oracle_cheb_coeffs(nx, ny, sdeg, &c0, c1, c2);
    c0f = (float)c0;
    for (int32_t k = 0; k + 1 < sdeg; ++k) {
      c1f[k] = (float)c1[k];
      c2f[k] = (float)c2[k];
    }
  }
  memset(res, 0, sizeof(*res));
  int st = OR_OK;
  int32_t total = 0, outer = 0;
  const double bb = dot_sequential(n, b, b);
  double g = 0.0;
  if (!r || !ri || !d || !p || !s || (sdeg && !zc)) { st = OR_E_NOMEM; goto out; }
  if (bb == 0.0) {
    memset(x, 0, (size_t)n * sizeof(double));
    goto out;
  }
  if (x0) memcpy(x, x0, (size_t)n * sizeof(double));
  else    memset(x, 0, (size_t)n * sizeof(double));
  const double thr = (tol * tol) * bb;
  for (;;) {
    spmv(&A, x, r);
    for (int64_t k = 0; k < n; ++k) r[k] = b[k] - r[k];
    g = dot_sequential(n, r, r);
    if (!isfinite(g)) { st = OR_BREAKDOWN; break; }
    if (g <= thr) { st = OR_OK; break; }
    if (total >= maxit) { st = OR_NOT_CONVERGED; break; }
    const double sc = sqrt(g), inv = 1.0 / sc;
    for (int64_t k = 0; k < n; ++k) {
      ri[k] = (inner_t)(r[k] * inv);
      d[k] = 0;
      p[k] = ri[k];
    }
    double gamma = dot_f32_in_f64(n, ri, ri);
    /* the inner solve needs to reduce its residual by no more than what is
     * left to the outer tolerance, (tol ||b||) / ||r||, with a margin of two
     * for the FP32 arithmetic: the last outer step stops early */
    const double eff = fmax(inner_tol, (0.5 * tol) * (sqrt(bb) / sc));
    const double thr_in = (eff * eff) * gamma;
    int32_t kin = 0;
#if ORACLE_MUTANT != 1
    if (sdeg) {
      /* preconditioned classic CG in binary32, the loop of oracle_pcg */
      float* z = zc;
      double rho = 0.0, rho_old = 0.0;
      while (!(gamma <= thr_in) && total < maxit) {
        cheb_apply_f32(&A, sdeg, c0f, c1f, c2f, ri, z, zc + n, zc + 2 * n, zc + 3 * n);
        rho = dot_f32_in_f64(n, ri, z);
        if (!(rho > 0.0) || !isfinite(rho)) break;
        if (kin == 0) {
          for (int64_t k = 0; k < n; ++k) p[k] = z[k];
        } else {
          const float bf = (float)(rho / rho_old);
          for (int64_t k = 0; k < n; ++k) p[k] = z[k] + bf * p[k];
        }
        spmv_f32(&A, p, s);
        const double pi = dot_f32_in_f64(n, p, s);
        if (!(pi > 0.0) || !isfinite(pi)) break;
        const float af = (float)(rho / pi);
        for (int64_t k = 0; k < n; ++k) {
          d[k] = d[k] + af * p[k];
          ri[k] = ri[k] - af * s[k];
        }
        gamma = dot_f32_in_f64(n, ri, ri);
        rho_old = rho;
        ++kin; ++total;
      }
    }
#endif
    while (!sdeg && !(gamma <= thr_in) && total < maxit) {
      spmv_inner(&A, p, s);
      double pi = dot_f32_in_f64(n, p, s);
      if (!(pi > 0.0) || !isfinite(pi)) break;
      double alpha = gamma / pi;
      inner_scalar_t af = (inner_scalar_t)alpha;
      for (int64_t k = 0; k < n; ++k) {
        d[k] = (inner_t)(d[k] + af * p[k]);
        ri[k] = (inner_t)(ri[k] - af * s[k]);
      }
      double gnew = dot_f32_in_f64(n, ri, ri);
      inner_scalar_t bf = (inner_scalar_t)(gnew / gamma);
      for (int64_t k = 0; k < n; ++k) p[k] = (inner_t)(ri[k] + bf * p[k]);
      gamma = gnew;
      ++kin; ++total;
    }
    if (kin == 0) { st = OR_BREAKDOWN; break; }
    for (int64_t k = 0; k < n; ++k) x[k] = x[k] + sc * (double)d[k];
    ++outer;
  }
  res->rel_res_recursive = res->rel_res_true = sqrt(g / bb);
out:
  res->status = st;
  res->iterations = total;
  res->outer_iterations = outer;
  free(r); free(ri); free(d); free(p); free(s); free(zc);
  csr_free(&A);
  return st;
}
