// cg_internal.h - structures shared by the host runtime and the gfx950 kernels.
//
// Layout in HBM.  Every grid vector is stored row-major with a padded pitch P
// (a multiple of the tile width, so each wavefront row access is a full
// aligned 1-2 KiB segment); columns [nx, P) are kept zero and are never
// written.  The Dirichlet ring is not stored: out-of-grid neighbours read as
// zero by predicate.
//
// Work decomposition (the arithmetic contract every pass obeys).  A tile is
// 64 lanes x CPL columns wide and 4 wavefronts x `rows` rows tall; wavefront w
// marches down its own `rows`-row strip.  Tiles are numbered row-major.  Each
// pass writes one FP64 partial per dot product per tile; the next pass sums
// them in tile order (cross-tile stage) before it starts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cgk {

constexpr int kWave = 64;
constexpr int kGroup = 256;       // threads that process one tile (4 wavefronts)
constexpr int kWavesPerTile = 4;
constexpr int kWgGroups = 2;     // tile groups of the single-work-group solver
constexpr int kRrRows = 20;       // rows per thread of the register-resident solver
constexpr int kRrThreads = 512;   // its largest work-group
constexpr int kChebMaxSteps = 8;  // Chebyshev preconditioner steps (halo s - 1)

// Device-side solve status (host maps it to the ABI codes).
enum : int32_t {
  ST_RUNNING = 0,
  ST_OK = 1,             // converged, or tol == 0 and maxit iterations done
  ST_NOT_CONVERGED = 2,
  ST_BREAKDOWN = 3,
  ST_ZERO_RHS = 4,       // (b,b) == 0: x = 0 is the answer
  ST_INNER_DONE = 5,     // refinement: inner solve finished, outer step pending
};

enum : int32_t {
  F_BB_PENDING = 1,      // the next prologue takes (b,b) from partial slot 1
  F_PRECOND = 2,         // classic CG preconditioned by the Chebyshev pass:
                         // K_CHEB makes the stop test on (r,r) of the pass
                         // before it, K_CG1 takes rho = (r,z) from the K_CHEB
                         // partials and keeps it in State::delta, and K_CG2
                         // forms alpha = rho / (p, A p)
};

// Scalar state of one solve.  Kept in device memory, double-buffered by pass
// parity: a pass reads state[m & 1] and its first work-group writes
// state[(m + 1) & 1], so no work-group overwrites what another still reads.
struct alignas(16) State {
  double gamma;      // (r, r) of the current iterate
  double gamma0;     // refinement: (rho, rho) at the start of the inner solve;
                     // preconditioned pipelined: (r, u)
  double delta;      // pipelined: (w, r); classic: alpha's numerator ((r, r), or
                     // rho = (r, z) when preconditioned)
  double alpha, beta;
  double bb;         // (b, b)
  double thr;        // stop when gamma <= thr = tol^2 (b, b)
  double thr_in;     // refinement inner stop threshold
  double scale;      // refinement: ||b - A x|| of the current outer step
  double res2;       // ||b - A x||^2 recomputed at exit (or last outer step)
  double tol, inner_tol;
  int32_t k;         // x-updates done (refinement: total inner iterations)
  int32_t status;
  int32_t flags;
  int32_t kin;       // refinement: iterations of the current inner solve
  int32_t outer;     // refinement: outer steps done
  int32_t maxit;
  int32_t kind;      // step engine: pass kind the solve runs at its next step
  int32_t pad_;
};

constexpr int32_t K_FINAL = 100;  // step engine: sum the true residual, then done
constexpr int32_t K_DONE = -1;    // step engine: nothing left to run

struct Geo {
  int32_t nx, ny;
  int32_t pitch;     // row stride of every vector of the solve, in elements: the
                     // padded row length ntx * 64 * cols_per_lane, times the
                     // number of FP64 vectors whose rows are interleaved (one
                     // row of each vector after the other) on the tile passes
  int32_t ntx, nty, tiles;
  int32_t rows;      // rows per wavefront strip
  int32_t th;        // rows per tile = 4 * rows
  int32_t plane;     // 3D (7-point operator): rows per plane, ny = plane * nz; 2D: 0
  int32_t alt;       // 1: the odd wavefronts of a tile walk their strip from its last
                     // row up (the 5-point operator only); 0: every wavefront top down
  // variable-coefficient 5-point operator: the west, east, south and north
  // face conductivities of every cell, four arrays laid out like a vector
  // (zero in the padding), kcs elements apart; null otherwise
  const double* kc;
  int64_t kcs;
};

// Pass kinds.
enum : int32_t {
  K_INIT_R = 0,   // r = b - A x;               slots (r,r), (b,b)
  K_INIT_W,       // w = A r;                   slots (r,r), (w,r)    [pipelined]
  K_PCG,          // fused pipelined iteration; slots (r,r), (w,r)
  K_CG1,          // p = r + beta p; s = A p;   slot  (p,s)          [classic]
  K_CG2,          // x += a p; r -= a A p;      slot  (r,r)          [classic]
  K_RESID,        // t = b - A x;               slots (t,t), (b,b)
  K_REF_SCALE,    // rho = fp32((b - A x)/s); d = 0; slot (rho,rho)  [refinement]
  K_CG1F,         // FP32 classic pass 1
  K_CG2F,         // FP32 classic pass 2
  K_REF_UPDATE,   // x += s * d
  K_APPLY,        // y = A u
  K_DOT,          // slot (u, y)
  K_PCGX,         // K_PCG of an even iteration: also applies both x updates
  K_CG2X,         // K_CG2 of an even iteration: also applies both x updates
  K_CG2FX,        // K_CG2F of an even inner iteration: both d updates
  K_CHEB,         // z = p_s(A) r (Chebyshev preconditioner); slot (r,z) in its own
                  // tiles: 128 columns x cheb_rows rows, one wavefront per tile
  K_INIT_WU,      // preconditioned pipelined: w = A u; slots (r,u), (w,u), (r,r)
  K_CHEBW,        // preconditioned pipelined: m = p_s(A) w after the scalar step
                  // (stop test, alpha, beta from the three slots); no slots
  K_PPCG,         // preconditioned pipelined fused iteration (n = A m and the eight
                  // updates); slots (r,u), (w,u), (r,r)
  K_CHEBF,        // refinement, preconditioned inner solve: z = p_s(A) r in FP32
                  // after the inner stop test on (r,r); slot (r,z) in the tiles
                  // of K_CHEB
  K_RRQ,          // residual replacement on the step engine: q = A p; no slots
  K_RRZ,          // residual replacement on the step engine: z = A q; no slots
  K_NKINDS
};

// Deferred x (FP64 classic and pipelined; the inner solution d of the FP32
// inner solve likewise, counted by inner iterations).  x is read and written
// only by the passes that end an even iteration: such a pass applies the
// previous (odd) iteration's update and then its own, x = fma(a_i, p_i,
// fma(a_(i-1), p_(i-1), x)), the same operations in the same order as one
// update per iteration.  A solve that stops after an odd iteration gets the
// pending update from the pass that stops it.

// Everything a pass may touch.  Unused pointers are null.
struct PassArgs {
  Geo g;
  const State* st_in;
  State* st_out;
  const double* part_in;   // [2][tiles] partials of the previous pass
  double* part_out;        // [2][tiles] partials of this pass
  const double* b;
  double* x;
  double* r;
  const double* w_in;      // pipelined: w of this iteration (read with halo)
  double* w_out;           //            w of the next iteration
  double* z;
  double* q;
  double* p;               // pipelined p
  const double* pc_in;     // classic: previous direction (read with halo)
  double* pc_out;          //          new direction
  const double* pc_prev;   //          pass 2: the direction before pc_in
  float* rf;               // refinement: inner residual rho / r_in
  float* df;               //             inner solution d
  float* zf;               //             preconditioned: z = M^-1 r_in
  const float* pf_in;      //             inner direction ping-pong
  float* pf_out;
  const float* pf_prev;    //             pass 2: the direction before pf_in
  const double* u;         // apply / dot inputs
  double* y;
  int32_t rev;             // walk the tiles in reverse order (alternate passes)
  int32_t cheb_s;          // K_CHEB: Chebyshev steps s (1..kChebMaxSteps)
  int32_t cheb_rows;       // K_CHEB: rows of one Chebyshev item / partial tile
  int32_t cheb_tiles;      // K_CG1 preconditioned: partials of the Chebyshev pass
  const double* cheb;      // K_CHEB: c0, then c1[s-1], then c2[s-1]
  double* uu;              // preconditioned pipelined: u = M^-1 r
  double* sv;              //                           s (the direction of r)
  const double* mv;        //                           m = M^-1 w (read with halo)
  double* wv;              //                           w (updated in place)
};

// Scalars a pass body needs, chosen by the preceding transition.
struct Sc {
  double al, be;
  int32_t first;   // first iteration: previous direction vectors are zero
  int32_t xu;      // this pass ends an even iteration: apply both x updates
  double inv;      // refinement: 1 / scale
  double alp;      // alpha of the pending x update (previous iteration)
};

// One resident solve of the multi-solve step kernel (batch and serving),
// written by the host at admission.  The solve's progress lives in its
// double-buffered State (which holds the kind of the next pass); a solve
// admitted at step a runs its pass number (step - a) at every step.
struct alignas(64) Slot {
  Geo g;
  int32_t variant, refined;
  int32_t cpl4;      // 4 columns per lane (refined, or pinned classic FP64)
  int32_t admit_step;
  int32_t precond;     // Chebyshev steps s of the preconditioner; 0 = none
  int32_t cheb_rows;   // rows of a Chebyshev item / partial tile
  int32_t cheb_tiles;  // partials of the Chebyshev pass
  int32_t cheb_items;  // Chebyshev items of one pass (the step's items number them)
  int32_t rr_period;   // pipelined: residual replacement every rr_period iterations; 0 none
  const double* cheb;  // c0, c1[s-1], c2[s-1]
  double* u;           // preconditioned pipelined: u = M^-1 r
  double* sv;          //                           s
  double* mv;          //                           m = M^-1 w
  double* b;
  double* x;
  double* r;
  double* z;
  double* q;
  double* p;
  double* W[2];      // pipelined w ping-pong
  double* PC[2];     // classic direction ping-pong
  float* rf;
  float* df;
  float* PF[2];      // refinement inner direction ping-pong
  float* zf;         // refinement, preconditioned: z = M^-1 r_in
  double* part[2];   // per-tile partials, by pass parity
  State* S[2];       // state, by pass parity
};

// A unit of work of one step: tiles [t0, t1) of one resident solve (for the
// Chebyshev step kernel: its Chebyshev items [t0, t1)).
struct Item {
  int32_t slot, t0, t1, pad_;
};

// Fixed-point variant (cg_fixed.hip): values are Q20.30 held as int64 counts
// of 2^-30 in [-2^49, 2^49 - 1] (the paper's 50-bit format with 20 integer
// bits, round to nearest with ties up, saturation).  One work-group of up to
// kFxThreads threads runs a whole solve: thread t owns unknowns t + e*T
// (e < kFxMaxE).  LDS (160 KiB, kFxLdsWords int64) holds the stencil operand
// with a zero ring ((ny + 2) rows of nx + 1), one more full vector and the
// kFxSumWords sum slots.
constexpr int kFxThreads = 1024;
constexpr int kFxMaxE = 10;
constexpr int kFxLdsWords = 20480;
constexpr int kFxSumWords = 128;

inline bool fixed_fits(int nx, int ny) {
  return nx >= 1 && ny >= 1 &&
         (int64_t)(ny + 2) * (nx + 1) + (int64_t)nx * ny <= kFxLdsWords - kFxSumWords &&
         (int64_t)nx * ny <= (int64_t)kFxThreads * kFxMaxE;
}

// Unknowns per thread the solver is compiled for (1, 2, 3, 4, 6, 8, 10): the
// smallest that covers dof unknowns with `threads` threads.
inline int fixed_elems(int64_t dof, int threads) {
  const int64_t e = (dof + threads - 1) / threads;
  return e <= 4 ? (int)(e < 1 ? 1 : e) : e <= 6 ? 6 : e <= 8 ? 8 : 10;
}

struct FxArgs {
  Geo g;
  const double* b;  // staged right-hand side (pitched FP64)
  double* x;        // staged x0 in, solution out (pitched FP64)
  int64_t* bq;      // quantized b, compact nx*ny
  int64_t* xq;      // pipelined: quantized x, compact nx*ny
  int64_t* qg;      // pipelined: q, compact nx*ny (used with 8+ unknowns per thread)
  State* S[2];      // tol and maxit in S[0]; the final state lands in both
};

// Host-side launchers (cg_kernels.hip, cg_fixed.hip).
hipError_t launch_pass(int kind, int fp32_geometry, const PassArgs& a, int grid, hipStream_t s);
hipError_t launch_final(const PassArgs& a, hipStream_t s);  // res2 = sum of slot 0
hipError_t launch_fill(void* p, size_t bytes, hipStream_t s);
hipError_t launch_solve_wg(int variant, const PassArgs& a, hipStream_t s);
// Whole solve in one work-group of `threads` threads with the vectors on chip;
// needs (nx + 1) * ceil(ny / kRrRows) <= threads <= kRrThreads.
hipError_t launch_solve_rr(int variant, const PassArgs& a, int threads, hipStream_t s);
// One register-resident solve per listed slot (slots[idx[i]], i < n), each
// fitting the solver; final states land in both state buffers, kind K_DONE.
hipError_t launch_solve_rr_many(const Slot* slots, const int* idx, int n, hipStream_t s);
// Whole fixed-point solve in one work-group of `threads` threads:
// fixed_fits(nx, ny), nx * ny <= threads * kFxMaxE, threads a multiple of 64
// no larger than kFxThreads.
hipError_t launch_solve_fixed(int variant, const FxArgs& a, int threads, hipStream_t s);
// One fixed-point solve per listed slot (slots[idx[i]], i < n), all of the
// given variant and each with at most kFxThreads * e unknowns, e =
// fixed_elems(dof, kFxThreads) of the largest; the slot's r holds the
// quantized b, its z (pipelined) or PC[0] (classic) the quantized x, and its
// q (pipelined) the vector q when it does not stay in registers.
// Final states land in both state buffers, kind K_DONE.
hipError_t launch_solve_fixed_many(const Slot* slots, const int* idx, int n, int variant, int e,
                                   hipStream_t s);
// Measurement only: grid work-groups of 256 threads, each thread 8 chains of
// `rounds` 32 x 32 -> 64-bit multiply-adds; writes grid * 256 words to sink.
hipError_t launch_mul_probe(uint64_t* sink, int grid, int rounds, hipStream_t s);
int pass_max_blocks_per_cu(int kind, int fp32_geometry);
// Work-groups of the Chebyshev pass with s steps that fit one CU (f32: the
// binary32 pass of the refinement); the pass runs 512-thread work-groups,
// grid a multiple of 8.
int cheb_max_blocks_per_cu(int s, bool f32 = false);
constexpr int kChebGroupCols = 896;  // columns of one Chebyshev item (7 tiles)
// Step *step_base + k of every resident solve: work-groups stride over the
// *n_items items; grid is any positive size.  The base step is read on the
// device so that a captured chunk of launches can be replayed.
hipError_t launch_step(const Slot* slots, const Item* items, const int* n_items,
                       const int* step_base, int k, int grid, hipStream_t s);
// Copies each listed slot's current state (pass parity of `step`) to out[i].
hipError_t launch_gather(const Slot* slots, const int* idx, int n, int step, State* out,
                         hipStream_t s);
int step_max_blocks_per_cu();
// The tile passes of preconditioned pipelined CG (K_INIT_WU, K_PPCG) of step
// *step_base + k, over launch_step's items; other kinds are skipped.
hipError_t launch_step_ppcg(const Slot* slots, const Item* items, const int* n_items,
                            const int* step_base, int k, int grid, hipStream_t st);
int step_ppcg_max_blocks_per_cu();
// Step *step_base + k of the resident solves on the 3D (op 1) or the
// variable-coefficient (op 2) operator, over the items of launch_step (which
// skips those solves); grid is any positive size.
hipError_t launch_step_op(int op, const Slot* slots, const Item* items, const int* n_items,
                          const int* step_base, int k, int grid, hipStream_t s);
int step_op_max_blocks_per_cu(int op);
// The Chebyshev passes (K_CHEB, K_CHEBW; f32: the refinement's K_CHEBF) of
// step *step_base + k of the resident preconditioned solves with s Chebyshev
// steps (1 <= s <= 8): work-groups of 512 threads stride over cinfo[2 s]
// items (Chebyshev item ranges) that start at items + cinfo[2 s + 1] (both
// read on the device); every other solve and pass kind is left to
// launch_step and the other form.
hipError_t launch_step_cheb(int s, bool f32, const Slot* slots, const Item* items,
                            const int* cinfo, const int* step_base, int k, int grid,
                            hipStream_t st);
hipError_t launch_stream(int pattern, double* const* v, size_t n, double* sink, int grid,
                         hipStream_t s);
size_t pass_algorithmic_bytes(int kind, int64_t dof);

}  // namespace cgk
