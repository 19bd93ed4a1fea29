// cg_fixed.hip - conjugate gradients in the paper's fixed-point format on gfx950.
//
// The FPGA design of the paper computes in a 50-bit fixed-point type with 20
// integer bits, rounding to nearest and saturating (Section II-B, the stencil
// listing; the fixed versus floating comparison of Section III).  Here a value
// is an int64 count k of 2^-30 with -2^49 <= k <= 2^49 - 1, and every
// statement of Algorithm 1 or 2 rounds its exact right-hand side once:
//
//   y +- a x   the product is exact (a multiple of 2^-60), the sum with y is
//              rounded to a multiple of 2^-30, ties towards +infinity, then
//              saturated (y - a x rounds its own tie: it is not -(a x - y));
//   A u        the 5-point stencil is exact in int64, then saturated;
//   (u, v)     each product rounded as above, the rounded products summed
//              exactly, the sum saturated once; integer sums are associative,
//              so any summation order gives the same bits;
//   n / d      the exact quotient rounded once, then saturated; Algorithm 2's
//              alpha recurrence rounds each division and the difference;
//   input      b and x0 arrive in FP64 and are rounded once (NaN as 0);
//   stop       (r, r) <= Q(tol^2 (b, b)), compared in counts.
//
// Exact products without 128-bit multiplies: a value v splits as
// v = vh 2^30 + vl with vh = v >> 30 (|vh| <= 2^19) and 0 <= vl < 2^30, so
//   Q(a x) = ah xh 2^30 + ah xl + al xh + floor((al xl + 2^29) / 2^30)
// with every term a 32 x 32 -> 64-bit product.  A dot product accumulates
// the two parts (sum of ah xh, and the rest) separately and recombines them
// after the work-group sum.
//
// One work-group runs a whole solve (the paper's grids reach 100 x 100):
// thread t owns unknowns k = t + e T, e < E, the kernel being compiled for
// E = 1, 2, 3, 4, 6, 8 or 10 (the launch takes the smallest that covers the
// grid: small grids get small code and few registers).  LDS holds two full
// vectors, the operand of the stencil (neighbours outside the grid read as
// zero by predicate) and one more vector; the rest of the per-unknown state
// lives in registers, Algorithm 2's x (and q from E = 8) in global memory.
// The scalars of a converging solve take update forms without 64-bit
// products (fx_upd); a uniform branch falls back to the general form.  Scalars are summed
// by a wave butterfly, one LDS slot per wave and a second butterfly over the
// slots; each thread then computes the same quotients, so no broadcast is
// needed.  Barriers per iteration: classic 3 (direction published, (p, s)
// summed, (r, r) summed), pipelined 2 (all stencil reads of w done, (r, r)
// and (w, r) summed).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "cg_internal.h"

namespace cgk {
namespace {

constexpr int64_t kFxMax = (int64_t(1) << 49) - 1;
constexpr int64_t kFxMin = -(int64_t(1) << 49);
constexpr int64_t kFxLow = (int64_t(1) << 30) - 1;
constexpr int64_t kFxOne = int64_t(1) << 30;
constexpr int kFxWaves = kFxThreads / kWave;
constexpr int kFxRedHalf = kFxWaves * 2 * 2;  // [wave][value < 2][h, m]
constexpr int kFxRed = 2 * kFxRedHalf;          // by call parity
static_assert(kFxRed == kFxSumWords, "sum slots as the host budgets them");

__device__ __forceinline__ int64_t fx_clamp(int64_t v) {
  return v > kFxMax ? kFxMax : (v < kFxMin ? kFxMin : v);
}

// v = h 2^30 + l, 0 <= l < 2^30; |h| <= 2^19 for |v| <= 2^49
struct FxSplit {
  int32_t h, l;
};

__device__ __forceinline__ FxSplit fx_split(int64_t v) {
  return {(int32_t)(v >> 30), (int32_t)(v & kFxLow)};
}

// floor((al xl + 2^29) / 2^30): the rounded low product, in [0, 2^30]
__device__ __forceinline__ int64_t fx_low(int32_t al, int32_t xl) {
  const uint64_t p = (uint64_t)(uint32_t)al * (uint32_t)xl + (uint64_t(1) << 29);
  return (int64_t)(p >> 30);
}

// Q(y + a x), a given split.  hh = ah xh decides saturation on its own once
// |hh| >= 2^22: the other terms stay below 2^51 in magnitude.
__device__ __forceinline__ int64_t fx_axpy(FxSplit a, int64_t x, int64_t y) {
  const FxSplit s = fx_split(x);
  const int64_t hh = (int64_t)a.h * s.h;
  const int64_t rest = (int64_t)a.h * s.l + (int64_t)a.l * s.h + fx_low(a.l, s.l) + y;
  if (hh >= (int64_t(1) << 22)) return kFxMax;
  if (hh <= -(int64_t(1) << 22)) return kFxMin;
  return fx_clamp(hh * kFxOne + rest);
}

// A cheaper exact form of Q(y + a x) for the scalars of a converging solve:
// Q(a x) = ah x + al xh + floor((al xl + 2^29) / 2^30), as ah 2^30 x / 2^30
// is an integer.  ZERO (ah = 0: 0 <= a < 1, every alpha and beta in practice)
// and NEG (ah = -1: -1 <= a < 0, -alpha) need no 64-bit product and no
// saturation test of the product: the int64 sum is exact, one clamp
// saturates it.  GENERAL is fx_axpy.
enum { FX_GENERAL = 0, FX_ZERO = 2, FX_NEG = 3 };

template <int M>
__device__ __forceinline__ int64_t fx_upd(FxSplit a, int64_t x, int64_t y) {
  if constexpr (M == FX_GENERAL) {
    return fx_axpy(a, x, y);
  } else {
    const FxSplit s = fx_split(x);
    const int64_t part = (int64_t)a.l * s.h + fx_low(a.l, s.l) + y;
    if constexpr (M == FX_ZERO) return fx_clamp(part);
    else return fx_clamp(part - x);
  }
}

// Runs f with std::true_type when `common` (a work-group-uniform flag: the
// update phase's scalars take the ZERO / NEG forms), std::false_type
// otherwise (GENERAL throughout).
template <class F>
__device__ __forceinline__ void fx_with(bool common, F&& f) {
  if (common) f(std::true_type{});
  else f(std::false_type{});
}

template <bool COMMON, int M>
constexpr int fx_form() {
  return COMMON ? M : FX_GENERAL;
}

// Exact running sum of Q(u v): u v rounded = h 2^30 + m.
struct FxAcc {
  int64_t h, m;
};

__device__ __forceinline__ void fx_acc(FxAcc& a, int64_t u, int64_t v) {
  const FxSplit su = fx_split(u), sv = fx_split(v);
  a.h += (int64_t)su.h * sv.h;
  a.m += (int64_t)su.h * sv.l + (int64_t)su.l * sv.h + fx_low(su.l, sv.l);
}

// the same for Q(u u): the two cross products are equal
__device__ __forceinline__ void fx_acc_sq(FxAcc& a, int64_t u) {
  const FxSplit su = fx_split(u);
  a.h += (int64_t)su.h * su.h;
  a.m += ((int64_t)su.h * su.l) * 2 + fx_low(su.l, su.l);
}

// moves the multiples of 2^30 of m into h, leaving 0 <= m < 2^30
__device__ __forceinline__ void fx_norm(FxAcc& a) {
  a.h += a.m >> 30;
  a.m &= kFxLow;
}

// saturated value of h 2^30 + m
__device__ __forceinline__ int64_t fx_finish(FxAcc a) {
  fx_norm(a);
  if (a.h >= (int64_t(1) << 19)) return kFxMax;
  if (a.h < -(int64_t(1) << 19)) return kFxMin;
  return a.h * kFxOne + a.m;
}

// Q(n / d) for d > 0: floor(n 2^30 / d + 1/2), saturated.  An FP64 estimate
// is within 1/4 of n 2^30 / d + 1/2 when that is below 2^50 in magnitude, so
// the floor of the estimate is off by at most one; the exact 128-bit
// remainder of (n 2^31 + d) / (2 d) corrects it.
__device__ __forceinline__ int64_t fx_div(int64_t n, int64_t d) {
  const double e = ldexp((double)n, 30) / (double)d + 0.5;
  if (e >= 0x1p50) return kFxMax;
  if (e <= -0x1p50) return kFxMin;
  int64_t q = (int64_t)floor(e);
  const __int128 num = (__int128)n * ((__int128)1 << 31) + d;
  const __int128 den = (__int128)d * 2;
  __int128 rem = num - (__int128)q * den;
  for (int i = 0; i < 2 && rem < 0; ++i) {
    --q;
    rem += den;
  }
  for (int i = 0; i < 2 && rem >= den; ++i) {
    ++q;
    rem -= den;
  }
  return fx_clamp(q);
}

// round-half-up, saturating quantization of an FP64 input
__device__ __forceinline__ int64_t fx_from(double v) {
  if (!(v == v)) return 0;
  if (v >= 524288.0) return kFxMax;
  if (v < -524288.0) return kFxMin;
  return fx_clamp((int64_t)floor(ldexp(v, 30) + 0.5));  // |ldexp| < 2^49: + 0.5 is exact
}

__device__ __forceinline__ int64_t fx_uniform(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// An opaque copy: addresses derived from it are formed where they are used,
// not hoisted out of the iteration loop into registers of their own.
__device__ __forceinline__ int fx_opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// y = sat(A u) at position c of the operand O stored with a zero ring: row
// length W = nx + 1 (one zero column between consecutive rows serves as the
// east ring of one row and the west ring of the next), a zero row above and
// below.  No predicates: the five reads are plain LDS reads.
__device__ __forceinline__ int64_t fx_stencil(const int64_t* O, int c, int W) {
  return fx_clamp((((4 * O[c] - O[c - 1]) - O[c + 1]) - O[c - W]) - O[c + W]);
}

// Work-group sums of NV <= 2 accumulators; every thread gets all NV results
// (sums of per-thread partials below 2^30 in m: no overflow in any order).
// Double-buffered slots: the slots of one call are rewritten two calls
// later, after a barrier every reader of this call has passed.
template <int NV>
__device__ __forceinline__ void fx_sum(FxAcc (&a)[NV], int64_t* red, int& par,
                                       int64_t (&out)[NV]) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    fx_norm(a[v]);
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1) {
      a[v].h += __shfl_xor((long long)a[v].h, m, kWave);
      a[v].m += __shfl_xor((long long)a[v].m, m, kWave);
    }
  }
  static_assert(NV >= 1 && NV <= 2, "two sums at most");
  int64_t* buf = red + par * kFxRedHalf;
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      buf[(wave * NV + v) * 2] = a[v].h;
      buf[(wave * NV + v) * 2 + 1] = a[v].m;
    }
  }
  __syncthreads();
  // lane l < nw of every wave takes wave l's partial; a 16-lane butterfly
  // leaves the total in lanes 0..15
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    FxAcc s = {0, 0};
    if (lane < nw) {
      s.h = buf[(lane * NV + v) * 2];
      s.m = buf[(lane * NV + v) * 2 + 1];
    }
#pragma unroll
    for (int m = kFxWaves / 2; m >= 1; m >>= 1) {
      s.h += __shfl_xor((long long)s.h, m, kWave);
      s.m += __shfl_xor((long long)s.m, m, kWave);
    }
    out[v] = fx_uniform(fx_finish(s));
  }
  par ^= 1;
}

// The final state, in counts (below 2^53, so the FP64 copies are exact): the
// host forms the relative residuals sqrt(gamma / bb) and sqrt(res2 / bb).
__device__ void fx_publish(const FxArgs& a, int status, int it, int64_t gamma, int64_t bb,
                           int64_t res2) {
  State st = *a.S[0];
  st.kind = K_DONE;
  st.status = status;
  st.k = it;
  st.gamma = (double)gamma;
  st.bb = (double)bb;
  st.res2 = (double)res2;
  *a.S[0] = st;
  *a.S[1] = st;
}

// LDS: O = the stencil operand (x, then p in Algorithm 1; x, r, then w in
// Algorithm 2), V = a second vector (s = A p in Algorithm 1, p in Algorithm 2),
// both nx * ny entries, then the sum slots.  Registers hold r and x
// (Algorithm 1) or z, q and r (Algorithm 2); Algorithm 2's x stays in global
// memory (xq), read and written once per iteration by its owner.
template <int VARIANT, int E>
__device__ __forceinline__ void fx_solve(const FxArgs& a, int64_t* lds) {
  // Algorithm 2 with 8 or more unknowns per thread keeps q in global memory
  // too (qg): three register vectors of that many unknowns spill (measured:
  // 100 x 100 runs 16% slower with q in registers).
  constexpr bool QG = VARIANT == 1 && E >= 8;
  const int T = blockDim.x, t = threadIdx.x;
  const int nx = a.g.nx, ny = a.g.ny, pitch = a.g.pitch, n = nx * ny;
  // unknown k = t + e T (row j = k / nx, column i) sits at c = (j + 1) W + i
  // = k + j + W of the zero-ringed operand O; V follows O; sum slots last
  const int W = nx + 1, L = (ny + 2) * W;
  int64_t* O = lds;
  int64_t* V = lds + L;
  int64_t* red = lds + kFxLdsWords - kFxRed;
  int par = 0;
  const double tol = a.S[0]->tol;
  const int maxit = a.S[0]->maxit;

  int c[E];  // -1: unowned
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = t + e * T;
    c[e] = k < n ? k + k / nx + W : -1;
  }
  for (int q = t; q < L; q += T) O[q] = 0;
  __syncthreads();

  // quantized inputs; x0 is the first operand (r = b - A x).  b goes to bq
  // and is read back by its owner (no register copy to hold meanwhile).
  int64_t xv[E];
  FxAcc acc[2] = {{0, 0}, {0, 0}};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    xv[e] = 0;
    if (c[e] >= 0) {
      const int k = t + e * T, j = c[e] - k - W, gk = j * pitch + (k - j * nx);
      const int64_t bv = fx_from(a.b[gk]);
      xv[e] = fx_from(a.x[gk]);
      a.bq[k] = bv;
      if constexpr (VARIANT == 1) {
        a.xq[k] = xv[e];
        V[k] = 0;  // p
        if constexpr (QG) a.qg[k] = 0;
      }
      O[c[e]] = xv[e];
      fx_acc_sq(acc[0], bv);
    }
  }
  __syncthreads();
  int64_t r[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    r[e] = 0;
    if (c[e] >= 0) {
      const int k = t + e * T;
      r[e] = fx_clamp(a.bq[k] - fx_stencil(O, c[e], W));
      fx_acc_sq(acc[1], r[e]);
    }
  }
  int64_t s2[2];
  fx_sum<2>(acc, red, par, s2);
  const int64_t bb = s2[0];
  int64_t gamma = s2[1];
  if (bb == 0) {
    if (t == 0) fx_publish(a, ST_ZERO_RHS, 0, 0, 0, 0);
    return;
  }
  const int64_t thr = fx_from(tol * tol * ldexp((double)bb, -30));
  auto stop = [&](int64_t g, int it) -> int {
    if (g <= thr) return ST_OK;
    if (it >= maxit) return tol == 0.0 ? ST_OK : ST_NOT_CONVERGED;
    return ST_RUNNING;
  };
  int it = 0, status = ST_RUNNING;

  // Every stencil read of an operand precedes the next sum's barrier, and
  // the operand is rewritten only after that sum: no extra barrier before a
  // rewrite.
  if constexpr (VARIANT == 0) {
    // Algorithm 1: p in O, s in V
    int64_t beta = 0;
    for (;;) {
      if ((status = stop(gamma, it)) != ST_RUNNING) break;
      const FxSplit sb = fx_split(beta);
      fx_with(sb.h == 0, [&](auto common) {
        constexpr int MB = fx_form<common(), FX_ZERO>();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (c[e] >= 0) {
            const int ce = fx_opaque(c[e]);
            O[ce] = it == 0 ? r[e] : fx_upd<MB>(sb, O[ce], r[e]);
          }
        }
      });
      __syncthreads();
      FxAcc api[1] = {{0, 0}};
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (c[e] >= 0) {
          const int k = fx_opaque(t) + e * T, ce = fx_opaque(c[e]);
          const int64_t sv = fx_stencil(O, ce, W);
          V[k] = sv;
          fx_acc(api[0], O[ce], sv);
        }
      }
      int64_t pi[1];
      fx_sum<1>(api, red, par, pi);
      if (pi[0] <= 0) {
        status = ST_BREAKDOWN;
        break;
      }
      const int64_t alpha = fx_div(gamma, pi[0]);
      const FxSplit sa = fx_split(alpha), sna = fx_split(-alpha);
      FxAcc ag[1] = {{0, 0}};
      fx_with(sa.h == 0 && sna.h == -1, [&](auto common) {
        constexpr int MA = fx_form<common(), FX_ZERO>(), MNA = fx_form<common(), FX_NEG>();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (c[e] >= 0) {
            const int k = fx_opaque(t) + e * T, ce = fx_opaque(c[e]);
            xv[e] = fx_upd<MA>(sa, O[ce], xv[e]);
            r[e] = fx_upd<MNA>(sna, V[k], r[e]);
            fx_acc_sq(ag[0], r[e]);
          }
        }
      });
      int64_t g2[1];
      fx_sum<1>(ag, red, par, g2);
      beta = fx_div(g2[0], gamma);
      gamma = g2[0];
      ++it;
    }
  } else {
    // Algorithm 2: w = A r and delta = (w, r) first; then w in O, p in V
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (c[e] >= 0) O[c[e]] = r[e];
    __syncthreads();
    int64_t delta;
    {
      int64_t w0[E];
      FxAcc ad[1] = {{0, 0}};
#pragma unroll
      for (int e = 0; e < E; ++e) {
        w0[e] = 0;
        if (c[e] >= 0) {
          w0[e] = fx_stencil(O, c[e], W);
          fx_acc(ad[0], w0[e], r[e]);
        }
      }
      int64_t d1[1];
      fx_sum<1>(ad, red, par, d1);
      delta = d1[0];
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (c[e] >= 0) O[c[e]] = w0[e];
    }
    __syncthreads();
    int64_t z[E];
#pragma unroll
    for (int e = 0; e < E; ++e) z[e] = 0;
    int64_t q[QG ? 1 : E];
#pragma unroll
    for (int e = 0; e < (QG ? 1 : E); ++e) q[e] = 0;
    int64_t alpha = 0, gamma_old = 0;
    for (;;) {
      if ((status = stop(gamma, it)) != ST_RUNNING) break;
      int64_t beta = 0;
      if (it == 0) {
        if (delta <= 0) {
          status = ST_BREAKDOWN;
          break;
        }
        alpha = fx_div(gamma, delta);
      } else {
        beta = fx_div(gamma, gamma_old);
        if (alpha <= 0) {
          status = ST_BREAKDOWN;
          break;
        }
        const int64_t den = fx_clamp(fx_div(delta, gamma) - fx_div(beta, alpha));
        if (den <= 0) {
          status = ST_BREAKDOWN;
          break;
        }
        alpha = fx_div(kFxOne, den);
      }
      const FxSplit sb = fx_split(beta), sa = fx_split(alpha), sna = fx_split(-alpha);
      const bool common = sb.h == 0 && sa.h == 0 && sna.h == -1;
      // n = A w and z = n + beta z (first iteration: beta = 0, z = q = p = 0)
      fx_with(common, [&](auto cm) {
        constexpr int MB = fx_form<cm(), FX_ZERO>();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (c[e] >= 0) z[e] = fx_upd<MB>(sb, z[e], fx_stencil(O, fx_opaque(c[e]), W));
        }
      });
      __syncthreads();  // w is overwritten below
      FxAcc gd[2] = {{0, 0}, {0, 0}};
      fx_with(common, [&](auto cm) {
        constexpr int MB = fx_form<cm(), FX_ZERO>(), MA = fx_form<cm(), FX_ZERO>();
        constexpr int MNA = fx_form<cm(), FX_NEG>();
        // x (and q) of the next unknown are loaded before this one's stores:
        // the global latency overlaps a whole unknown's arithmetic
        int64_t xn = 0, qn = 0;
        if (c[0] >= 0) {
          const int k0 = fx_opaque(t);
          xn = a.xq[k0];
          if constexpr (QG) qn = a.qg[k0];
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int64_t xc = xn, qc = qn;
          if (e + 1 < E && c[e + 1 < E ? e + 1 : e] >= 0) {
            const int kn = fx_opaque(t) + (e + 1) * T;
            xn = a.xq[kn];
            if constexpr (QG) qn = a.qg[kn];
          }
          if (c[e] >= 0) {
            const int k = fx_opaque(t) + e * T, ce = fx_opaque(c[e]);
            const int64_t w = O[ce];
            int64_t qe;
            if constexpr (QG) {
              qe = fx_upd<MB>(sb, qc, w);
              a.qg[k] = qe;
            } else {
              qe = q[e] = fx_upd<MB>(sb, q[e], w);
            }
            const int64_t p = fx_upd<MB>(sb, V[k], r[e]);
            V[k] = p;
            a.xq[k] = fx_upd<MA>(sa, p, xc);
            r[e] = fx_upd<MNA>(sna, qe, r[e]);
            const int64_t wn = fx_upd<MNA>(sna, z[e], w);
            O[ce] = wn;
            fx_acc_sq(gd[0], r[e]);
            fx_acc(gd[1], wn, r[e]);
          }
        }
      });
      int64_t sums[2];
      fx_sum<2>(gd, red, par, sums);
      gamma_old = gamma;
      gamma = sums[0];
      delta = sums[1];
      ++it;
    }
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (c[e] >= 0) xv[e] = a.xq[t + e * T];
  }

  // true residual b - A x in the same arithmetic, then x back to FP64
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e)
    if (c[e] >= 0) O[c[e]] = xv[e];
  __syncthreads();
  FxAcc at[1] = {{0, 0}};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (c[e] >= 0) {
      const int k = t + e * T, j = c[e] - k - W;
      const int64_t tv = fx_clamp(a.bq[k] - fx_stencil(O, c[e], W));
      fx_acc_sq(at[0], tv);
      a.x[j * pitch + (k - j * nx)] = ldexp((double)xv[e], -30);
    }
  }
  int64_t tt[1];
  fx_sum<1>(at, red, par, tt);
  if (t == 0) fx_publish(a, status, it, gamma, bb, tt[0]);
}

template <int VARIANT, int E>
__global__ __launch_bounds__(kFxThreads) void k_solve_fixed(FxArgs a) {
  __shared__ int64_t lds[kFxLdsWords];
  fx_solve<VARIANT, E>(a, lds);
}

// One work-group per listed slot; every listed slot runs VARIANT and has at
// most kFxThreads * E unknowns.
template <int VARIANT, int E>
__global__ __launch_bounds__(kFxThreads) void k_solve_fixed_many(const Slot* slots,
                                                                 const int* idx) {
  __shared__ int64_t lds[kFxLdsWords];
  const Slot& S = slots[__builtin_amdgcn_readfirstlane(idx[blockIdx.x])];
  FxArgs a;
  a.g = S.g;
  a.b = S.b;
  a.x = S.x;
  a.bq = reinterpret_cast<int64_t*>(S.r);
  a.xq = reinterpret_cast<int64_t*>(VARIANT == 1 ? S.z : S.PC[0]);
  a.qg = reinterpret_cast<int64_t*>(S.q);
  a.S[0] = S.S[0];
  a.S[1] = S.S[1];
  fx_solve<VARIANT, E>(a, lds);
}

template <int VARIANT>
static hipError_t launch_one(int e, const FxArgs& a, int threads, hipStream_t st) {
  switch (e) {
    case 1: hipLaunchKernelGGL((k_solve_fixed<VARIANT, 1>), 1, threads, 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_solve_fixed<VARIANT, 2>), 1, threads, 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_solve_fixed<VARIANT, 3>), 1, threads, 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_solve_fixed<VARIANT, 4>), 1, threads, 0, st, a); break;
    case 6: hipLaunchKernelGGL((k_solve_fixed<VARIANT, 6>), 1, threads, 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_solve_fixed<VARIANT, 8>), 1, threads, 0, st, a); break;
    case 10: hipLaunchKernelGGL((k_solve_fixed<VARIANT, 10>), 1, threads, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int VARIANT>
static hipError_t launch_many(int e, const Slot* slots, const int* idx, int n, hipStream_t st) {
  const dim3 g(n), b(kFxThreads);
  switch (e) {
    case 1: hipLaunchKernelGGL((k_solve_fixed_many<VARIANT, 1>), g, b, 0, st, slots, idx); break;
    case 2: hipLaunchKernelGGL((k_solve_fixed_many<VARIANT, 2>), g, b, 0, st, slots, idx); break;
    case 3: hipLaunchKernelGGL((k_solve_fixed_many<VARIANT, 3>), g, b, 0, st, slots, idx); break;
    case 4: hipLaunchKernelGGL((k_solve_fixed_many<VARIANT, 4>), g, b, 0, st, slots, idx); break;
    case 6: hipLaunchKernelGGL((k_solve_fixed_many<VARIANT, 6>), g, b, 0, st, slots, idx); break;
    case 8: hipLaunchKernelGGL((k_solve_fixed_many<VARIANT, 8>), g, b, 0, st, slots, idx); break;
    case 10: hipLaunchKernelGGL((k_solve_fixed_many<VARIANT, 10>), g, b, 0, st, slots, idx);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Measurement only: independent chains of 32 x 32 -> 64-bit multiply-adds
// (v_mad_u64_u32, the product the fixed-point updates are built from), 8 per
// thread, `rounds` rounds; one value per thread is written so that the work
// is kept.
__global__ __launch_bounds__(256) void k_mul_probe(uint64_t* sink, int rounds, uint32_t seed) {
  const uint32_t a = (threadIdx.x * 2654435761u + seed + blockIdx.x) | 1u;
  uint64_t v[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) v[c] = a + c * 977u;
  for (int i = 0; i < rounds; ++i) {
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = (uint64_t)(uint32_t)v[c] * a + v[c];
  }
  uint64_t x = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) x ^= v[c];
  sink[(size_t)blockIdx.x * 256 + threadIdx.x] = x;
}

}  // namespace

hipError_t launch_mul_probe(uint64_t* sink, int grid, int rounds, hipStream_t st) {
  if (grid < 1 || rounds < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mul_probe, dim3(grid), dim3(256), 0, st, sink, rounds, 12345u);
  return hipGetLastError();
}

hipError_t launch_solve_fixed(int variant, const FxArgs& a, int threads, hipStream_t st) {
  if (!fixed_fits(a.g.nx, a.g.ny) || threads < kWave || threads > kFxThreads ||
      threads % kWave || a.g.pitch < a.g.nx || !a.b || !a.x || !a.bq ||
      (variant == 1 && (!a.xq || !a.qg)) || !a.S[0] || !a.S[1])
    return hipErrorInvalidValue;
  const int e = fixed_elems((int64_t)a.g.nx * a.g.ny, threads);
  return variant == 1 ? launch_one<1>(e, a, threads, st) : launch_one<0>(e, a, threads, st);
}

hipError_t launch_solve_fixed_many(const Slot* slots, const int* idx, int n, int variant, int e,
                                   hipStream_t st) {
  if (n < 1) return hipErrorInvalidValue;
  return variant == 1 ? launch_many<1>(e, slots, idx, n, st)
                      : launch_many<0>(e, slots, idx, n, st);
}

}  // namespace cgk
