/*
 * cg_oracle_fixed.c - CPU oracle for conjugate gradients on the 2D Laplace
 * problem in the fixed-point format of the paper's hardware.
 *
 * TEST INFRASTRUCTURE ONLY, like cg_oracle.c (same rules: nothing in the GPU
 * library links, loads or calls it).
 *
 * The paper's design computes in ap_fixed<50,20,AP_RND,AP_SAT> (Section II-B,
 * the HLS listing, and the fixed versus floating convergence discussion of
 * Section III).  This file runs Algorithms 1 and 2 in that format, written
 * from the definition of the format, with these readings:
 *
 *   - a value is an integer k times 2^-30 with -2^49 <= k <= 2^49 - 1
 *     (50 bits in two's complement, 20 of them above the binary point);
 *   - AP_RND rounds an exact value to the nearest multiple of 2^-30, ties
 *     towards plus infinity; AP_SAT replaces a value outside the range by the
 *     nearest extreme;
 *   - every assignment of the algorithm rounds and saturates its exact
 *     right-hand side once: y + a*x, y - a*x and a*x are formed exactly (a
 *     product of two values is an exact multiple of 2^-60) and then quantized;
 *     the stencil (((4uC - uW) - uE) - uS) - uN is exact and only saturates;
 *   - a dot product quantizes each product and sums the quantized products
 *     exactly, saturating the sum once (so its value does not depend on the
 *     summation order);
 *   - a quotient n / d (d > 0) is the exact quotient quantized once; the
 *     alpha recurrence of Algorithm 2 quantizes each division and the
 *     difference separately: t1 = Q(delta/gamma), t2 = Q(beta/alpha_old),
 *     alpha = Q(1 / Q(t1 - t2));
 *   - b and x0 enter as FP64 values quantized once (NaN as 0), and the stop
 *     threshold is Q(tol^2 (b,b)) from the quantized (b,b);
 *   - breakdown: (p, A p) <= 0 (classic); delta <= 0 in the first block, and
 *     alpha_old <= 0 or the quantized denominator <= 0 later (pipelined).
 *
 * gcc's __int128 holds every exact intermediate (at most 2^101 in magnitude).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

enum { FX_OK = 0, FX_NOT_CONVERGED = 2, FX_BREAKDOWN = 3, FX_E_INVALID = -1, FX_E_NOMEM = -2 };

#define FX_FRAC 30
static const int64_t FX_MAX = ((int64_t)1 << 49) - 1;
static const int64_t FX_MIN = -((int64_t)1 << 49);
static const int64_t FX_ONE = (int64_t)1 << FX_FRAC;

/* Same layout as oracle_result in cg_oracle.c (the Python side shares it). */
typedef struct {
  int32_t status;
  int32_t iterations;
  int32_t outer_iterations;
  int32_t pad_;
  double rel_res_recursive;
  double rel_res_true;
} fx_result;

static int64_t sat(i128 k) {
  if (k > FX_MAX) return FX_MAX;
  if (k < FX_MIN) return FX_MIN;
  return (int64_t)k;
}

/* floor(z / 2^s) of an exact integer (arithmetic shift, floor for negatives) */
static i128 floor_pow2(i128 z, int s) { return z >> s; }

/* Round half up of z * 2^-60 to a multiple of 2^-30, as an integer count. */
static i128 rnd60(i128 z) { return floor_pow2(z + ((i128)1 << (FX_FRAC - 1)), FX_FRAC); }

/* floor(num / den), den > 0 */
static i128 floor_div(i128 num, i128 den) {
  i128 q = num / den;
  if (num % den != 0 && num < 0) q -= 1;
  return q;
}

int64_t oracle_fx_quantize(double v) {
  if (v != v) return 0;
  if (v >= 524288.0) return FX_MAX;   /* 2^19 */
  if (v < -524288.0) return FX_MIN;
  const double s = ldexp(v, FX_FRAC); /* exact */
  return sat((i128)floor(s + 0.5));   /* s + 0.5 is exact for |s| < 2^52 */
}

double oracle_fx_value(int64_t k) { return ldexp((double)k, -FX_FRAC); }

/* Q(a b) */
int64_t oracle_fx_mul(int64_t a, int64_t b) { return sat(rnd60((i128)a * b)); }

/* Q(y + a x) and Q(y - a x) */
static int64_t axpy(int64_t a, int64_t x, int64_t y) { return sat((i128)y + rnd60((i128)a * x)); }
static int64_t axmy(int64_t a, int64_t x, int64_t y) { return sat((i128)y + rnd60(-((i128)a * x))); }

int64_t oracle_fx_axpy(int64_t a, int64_t x, int64_t y) { return axpy(a, x, y); }
int64_t oracle_fx_axmy(int64_t a, int64_t x, int64_t y) { return axmy(a, x, y); }

/* Q(n / d), d > 0: floor(n 2^30 / d + 1/2) = floor((2 n 2^30 + d) / (2 d)) */
int64_t oracle_fx_div(int64_t n, int64_t d) {
  const i128 num = (i128)n * ((i128)2 << FX_FRAC) + d;
  return sat(floor_div(num, (i128)2 * d));
}

/* sum of Q(a_k b_k), exact, saturated once */
int64_t oracle_fx_dot(int64_t n, const int64_t* a, const int64_t* b) {
  i128 s = 0;
  for (int64_t k = 0; k < n; ++k) s += rnd60((i128)a[k] * b[k]);
  return sat(s);
}

/* y = sat(A u): the 5-point stencil on the nx-by-ny grid, zero outside
 * (Section II-B), evaluated as (((4uC - uW) - uE) - uS) - uN exactly. */
int oracle_fx_spmv(int32_t nx, int32_t ny, const int64_t* u, int64_t* y) {
  if (nx < 1 || ny < 1 || !u || !y) return FX_E_INVALID;
  for (int64_t j = 0; j < ny; ++j) {
    for (int64_t i = 0; i < nx; ++i) {
      const int64_t k = j * nx + i;
      const i128 c = u[k];
      const i128 w = i > 0 ? u[k - 1] : 0, e = i + 1 < nx ? u[k + 1] : 0;
      const i128 s = j > 0 ? u[k - nx] : 0, nn = j + 1 < ny ? u[k + nx] : 0;
      y[k] = sat((((4 * c - w) - e) - s) - nn);
    }
  }
  return FX_OK;
}

/* r = sat(b - A x) */
static void residual(int32_t nx, int32_t ny, const int64_t* b, const int64_t* x, int64_t* ax,
                     int64_t* r) {
  const int64_t n = (int64_t)nx * ny;
  oracle_fx_spmv(nx, ny, x, ax);
  for (int64_t k = 0; k < n; ++k) r[k] = sat((i128)b[k] - ax[k]);
}

static int stop_code(int64_t gamma, int64_t thr, int32_t k, int32_t maxit, double tol) {
  if (gamma <= thr) return FX_OK;
  if (k >= maxit) return tol == 0.0 ? FX_OK : FX_NOT_CONVERGED;
  return -100;  /* keep going */
}

static void finish(int32_t nx, int32_t ny, const int64_t* b, const int64_t* x, int64_t* t1,
                   int64_t* t2, int64_t gamma, int64_t bb, fx_result* res) {
  const int64_t n = (int64_t)nx * ny;
  residual(nx, ny, b, x, t1, t2);
  const int64_t tt = oracle_fx_dot(n, t2, t2);
  res->rel_res_recursive = sqrt((double)gamma / (double)bb);
  res->rel_res_true = sqrt((double)tt / (double)bb);
}

/* Solve A x = b in the fixed-point format.  variant 0: Algorithm 1,
 * 1: Algorithm 2.  b, x0 (NULL = zeros) are FP64 and quantized on entry;
 * xq receives the solution's integer counts and x (may be NULL) its values.
 * Returns the status (also in res). */
int oracle_cg_fixed(int32_t variant, int32_t nx, int32_t ny, const double* b, const double* x0,
                    int64_t* xq, double* x, double tol, int32_t maxit, fx_result* res) {
  if (nx < 1 || ny < 1 || !b || !xq || !res || maxit < 1 || !(tol >= 0.0) || tol >= 1.0)
    return FX_E_INVALID;
  const int64_t n = (int64_t)nx * ny;
  memset(res, 0, sizeof(*res));
  int64_t* v = (int64_t*)calloc((size_t)n * 9, sizeof(int64_t));
  if (!v) return FX_E_NOMEM;
  int64_t *bq = v, *r = v + n, *p = v + 2 * n, *s = v + 3 * n, *w = v + 4 * n, *z = v + 5 * n,
          *q = v + 6 * n, *nv = v + 7 * n, *t = v + 8 * n;
  for (int64_t k = 0; k < n; ++k) {
    bq[k] = oracle_fx_quantize(b[k]);
    xq[k] = x0 ? oracle_fx_quantize(x0[k]) : 0;
  }
  int st = FX_OK;
  int32_t it = 0;
  const int64_t bb = oracle_fx_dot(n, bq, bq);
  int64_t gamma = 0;
  if (bb == 0) {
    memset(xq, 0, (size_t)n * sizeof(int64_t));
    goto out;
  }
  const int64_t thr = oracle_fx_quantize(tol * tol * oracle_fx_value(bb));
  residual(nx, ny, bq, xq, t, r);
  gamma = oracle_fx_dot(n, r, r);
  if (variant == 0) {
    /* Algorithm 1 */
    int64_t beta = 0;
    for (;;) {
      const int sc = stop_code(gamma, thr, it, maxit, tol);
      if (sc != -100) { st = sc; break; }
      for (int64_t k = 0; k < n; ++k) p[k] = it == 0 ? r[k] : axpy(beta, p[k], r[k]);
      oracle_fx_spmv(nx, ny, p, s);
      const int64_t pi = oracle_fx_dot(n, p, s);
      if (pi <= 0) { st = FX_BREAKDOWN; break; }
      const int64_t alpha = oracle_fx_div(gamma, pi);
      for (int64_t k = 0; k < n; ++k) {
        xq[k] = axpy(alpha, p[k], xq[k]);
        r[k] = axmy(alpha, s[k], r[k]);
      }
      const int64_t g2 = oracle_fx_dot(n, r, r);
      beta = oracle_fx_div(g2, gamma);
      gamma = g2;
      ++it;
    }
  } else {
    /* Algorithm 2 (first block, then the loop) */
    oracle_fx_spmv(nx, ny, r, w);
    int64_t delta = oracle_fx_dot(n, w, r);
    int64_t alpha = 0;
    int sc = stop_code(gamma, thr, it, maxit, tol);
    if (sc != -100) {
      st = sc;
    } else if (delta <= 0) {
      st = FX_BREAKDOWN;
    } else {
      oracle_fx_spmv(nx, ny, w, nv);
      alpha = oracle_fx_div(gamma, delta);
      for (int64_t k = 0; k < n; ++k) {
        z[k] = nv[k];
        q[k] = w[k];
        p[k] = r[k];
        xq[k] = axpy(alpha, p[k], xq[k]);
        r[k] = axmy(alpha, q[k], r[k]);
        w[k] = axmy(alpha, z[k], w[k]);
      }
      it = 1;
      for (;;) {
        const int64_t gamma_old = gamma;
        gamma = oracle_fx_dot(n, r, r);
        delta = oracle_fx_dot(n, w, r);
        sc = stop_code(gamma, thr, it, maxit, tol);
        if (sc != -100) { st = sc; break; }
        oracle_fx_spmv(nx, ny, w, nv);
        const int64_t beta = oracle_fx_div(gamma, gamma_old);
        if (alpha <= 0) { st = FX_BREAKDOWN; break; }
        const int64_t t1 = oracle_fx_div(delta, gamma);
        const int64_t t2 = oracle_fx_div(beta, alpha);
        const int64_t den = sat((i128)t1 - t2);
        if (den <= 0) { st = FX_BREAKDOWN; break; }
        alpha = oracle_fx_div(FX_ONE, den);
        for (int64_t k = 0; k < n; ++k) {
          z[k] = axpy(beta, z[k], nv[k]);
          q[k] = axpy(beta, q[k], w[k]);
          p[k] = axpy(beta, p[k], r[k]);
          xq[k] = axpy(alpha, p[k], xq[k]);
          r[k] = axmy(alpha, q[k], r[k]);
          w[k] = axmy(alpha, z[k], w[k]);
        }
        ++it;
      }
    }
  }
  finish(nx, ny, bq, xq, t, s, gamma, bb, res);
out:
  if (x)
    for (int64_t k = 0; k < n; ++k) x[k] = oracle_fx_value(xq[k]);
  res->status = st;
  res->iterations = it;
  free(v);
  return st;
}
