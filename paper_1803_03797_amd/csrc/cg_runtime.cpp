// cg_runtime.cpp - host runtime of the stencil CG library: context, device
// arena, planning, pass sequencing (with hipGraph-captured iteration chunks),
// profiling, and the C ABI of include/cg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/cg.h"
#include "cg_internal.h"
#include "cg_runtime.h"

namespace cgr {

using namespace cgk;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

static size_t round_up(size_t v, size_t m) { return (v + m - 1) / m * m; }

// ------------------------------------------------------------- planning --

static int32_t map_status(int32_t st) {
  switch (st) {
    case ST_OK:
    case ST_ZERO_RHS: return CG_OK;
    case ST_NOT_CONVERGED: return CG_NOT_CONVERGED;
    case ST_BREAKDOWN: return CG_BREAKDOWN;
    default: return CG_PENDING;
  }
}

cg_problem resolve_precision(const cg_problem& p) {
  cg_problem q = p;
  if (q.precision == CG_PREC_AUTO)
    q.precision = (int64_t)q.nx * q.ny < kAutoRefineDof ? CG_PREC_FP64 : CG_PREC_FP32_REFINED;
  return q;
}

int validate(const cg_problem* p) {
  if (!p) return CG_E_INVALID;
  if (p->precision == CG_PREC_AUTO) {
    // the policy picks FP64 or FP32 refinement: problems both can take (with
    // or without the preconditioner)
    if (p->nz > 1 || p->kx || p->ky || p->rr_period != 0) return CG_E_INVALID;
    const cg_problem q = resolve_precision(*p);
    return validate(&q);
  }
  if (p->nx < 1 || p->ny < 1 || p->nz < 0) return CG_E_INVALID;
  if ((int64_t)p->ny * std::max(p->nz, 1) >= (int64_t)1 << 31) return CG_E_INVALID;
  if ((int64_t)p->nx * p->ny * std::max(p->nz, 1) > (int64_t)1 << 31) return CG_E_INVALID;
  // the row stride (Geo::pitch, int32) is the padded width (at most nx
  // rounded up to 256 columns) times up to 14 interleaved vectors
  if (((int64_t)p->nx + 255) / 256 * 256 * 14 > (int64_t)INT32_MAX) return CG_E_INVALID;
  // 3D (7-point operator): FP64 CG of either variant, no preconditioner
  if (p->nz > 1 && (p->precision != CG_PREC_FP64 || p->precond != 0)) return CG_E_INVALID;
  // variable coefficients: both arrays, 2D FP64 CG of either variant, no
  // preconditioner
  if ((p->kx == nullptr) != (p->ky == nullptr)) return CG_E_INVALID;
  if (p->kx && (p->nz > 1 || p->precision != CG_PREC_FP64 || p->precond != 0))
    return CG_E_INVALID;
  if (!(p->tol >= 0.0) || !(p->tol < 1.0)) return CG_E_INVALID;
  if (p->maxit < 1) return CG_E_INVALID;
  if (!p->b || !p->x) return CG_E_INVALID;
  if (p->mem != CG_MEM_HOST && p->mem != CG_MEM_DEVICE) return CG_E_INVALID;
  if (p->variant != CG_VARIANT_CLASSIC && p->variant != CG_VARIANT_PIPELINED) return CG_E_INVALID;
  if (p->precision != CG_PREC_FP64 && p->precision != CG_PREC_FP32_REFINED &&
      p->precision != CG_PREC_FIXED)
    return CG_E_INVALID;
  if (p->precision == CG_PREC_FIXED && !fixed_fits(p->nx, p->ny)) return CG_E_INVALID;
  if (p->precond < 0 || p->precond > kChebMaxSteps) return CG_E_INVALID;
  // the preconditioner: FP64 CG of either variant, or the FP32 inner solve
  // of the refinement (preconditioned classic CG in binary32)
  if (p->precond > 0 && p->precision != CG_PREC_FP64 && p->precision != CG_PREC_FP32_REFINED)
    return CG_E_INVALID;
  if (p->precision == CG_PREC_FP32_REFINED && (!(p->inner_tol >= 0.0) || !(p->inner_tol < 1.0)))
    return CG_E_INVALID;
  // residual replacement: the pipelined FP64 2D solve, an even period (x is
  // brought up to date at even iterations)
  if (p->rr_period < 0 || (p->rr_period & 1)) return CG_E_INVALID;
  if (p->rr_period > 0 && (p->variant != CG_VARIANT_PIPELINED || p->precision != CG_PREC_FP64 ||
                           p->precond != 0 || p->nz > 1))
    return CG_E_INVALID;
  return CG_OK;
}

// Rows of the stored grid: ny, or ny * nz planes of the 3D operator.
int rows_of(const cg_problem* p) { return p->nz > 1 ? p->ny * p->nz : p->ny; }

// Partial slots per tile the passes of a solve write at most.
static int ndots_max(const cg_problem* p) {
  return p->precond > 0 && p->variant == CG_VARIANT_PIPELINED ? 3 : 2;
}

Geo make_geo(int nx, int ny, int fp32g, int rows) {
  Geo g{};
  const int cpl = fp32g ? 4 : 2, tw = kWave * cpl;
  g.nx = nx;
  g.ny = ny;
  g.pitch = (int)round_up((size_t)nx, (size_t)tw);
  g.ntx = g.pitch / tw;
  g.rows = std::max(1, rows);
  g.th = kWavesPerTile * g.rows;
  g.nty = (ny + g.th - 1) / g.th;
  g.tiles = g.ntx * g.nty;
  return g;
}

// 3D z-march tiles (the 7-point operator): 4 in-plane rows, one per
// wavefront, by zc planes; the stored grid is plane * nz rows.
Geo make_geo3(int nx, int plane, int nz, int zc) {
  Geo g = make_geo(nx, plane * nz, 0, 1);
  g.plane = plane;
  g.rows = std::max(1, zc);
  g.th = kWavesPerTile;
  g.nty = (plane + kWavesPerTile - 1) / kWavesPerTile;
  g.tiles = g.ntx * g.nty * ((nz + g.rows - 1) / g.rows);
  return g;
}

// Planes per z-march strip: about 1024 tiles (4 per CU), at least 8 planes
// (a strip loads the planes before and after it again, so short strips
// re-read) and at most 64.
static int default_planes(int nx, int plane, int nz) {
  const int ntx = (nx + 2 * kWave - 1) / (2 * kWave);
  const int nty = (plane + kWavesPerTile - 1) / kWavesPerTile;
  const int want_ntz = std::max(1, 1024 / std::max(1, ntx * nty));
  const int zc = (nz + want_ntz - 1) / want_ntz;
  return std::min(64, std::max(std::min(nz, 8), zc));
}

int default_rows(int nx, int ny, int fp32g) {
  const int cpl = fp32g ? 4 : 2, tw = kWave * cpl;
  const int ntx = (nx + tw - 1) / tw;
  // aim for about 1024 tiles (4 per CU) with strips of up to 32 rows: long
  // strips amortise the halo rows, enough tiles keep every CU busy
  const int want_nty = std::max(1, (1024 + ntx - 1) / ntx);
  int rows = ny / (kWavesPerTile * want_nty);
  return std::min(32, std::max(2, rows));
}

static int wg_rows(int nx, int ny) {
  // one tile per group of the single work-group when the width allows
  const int ntx = (nx + 2 * kWave - 1) / (2 * kWave);
  const int nty = std::max(1, (kWgGroups + ntx - 1) / ntx);
  return std::max(1, (ny + kWavesPerTile * nty - 1) / (kWavesPerTile * nty));
}

int Ctx::unpinned_rows(const cg_problem* p, int fp32g) const {
  const int ny = rows_of(p);
  if (p->nz > 1) return default_planes(p->nx, p->ny, p->nz);
  // pipelined FP64 5-point solves of 16M unknowns and more: about 4096
  // tiles, so that each of the one-per-CU work-groups walks some 16 short
  // ones (pcg_pass at 4096^2 with interleaved rows: 288 us with 8 rows per
  // strip against 296 us with 32; 8192^2 gets 32 either way)
  if (!fp32g && !p->precond && !p->kx && p->nz <= 1 && p->variant == CG_VARIANT_PIPELINED &&
      (int64_t)p->nx * ny >= 16 * 1024 * 1024) {
    const int ntx = (p->nx + 2 * kWave - 1) / (2 * kWave);
    const int want_nty = std::max(1, (4096 + ntx - 1) / ntx);
    return std::min(32, std::max(2, ny / (kWavesPerTile * want_nty)));
  }
  return default_rows(p->nx, ny, fp32g);
}

bool Ctx::use_wg(const cg_problem* p) const {
  return p->precision == CG_PREC_FP64 && p->precond == 0 && p->nz <= 1 && !p->kx &&
         p->rr_period == 0 && (int64_t)p->nx * p->ny <= wg_max_dof;
}

// threads of the register-resident solver: rows of nx + 1 (one idle thread
// per row of segments) times the segments per column
static int64_t rr_threads_needed(int nx, int ny) {
  return (int64_t)(nx + 1) * ((ny + kRrRows - 1) / kRrRows);
}

bool Ctx::use_rr(const cg_problem* p) const {
  return rr_enabled && p->precision == CG_PREC_FP64 && p->precond == 0 && p->nz <= 1 &&
         !p->kx && p->rr_period == 0 && rr_threads_needed(p->nx, p->ny) <= kRrThreads;
}

Plan Ctx::plan(const cg_problem* p, bool allow_rr, bool interleave) {
  Plan pl;
  const int ny = rows_of(p);
  pl.variant = p->variant;
  pl.refined = p->precision == CG_PREC_FP32_REFINED;
  pl.fp32g = pl.refined ? 1 : 0;
  pl.wg = use_wg(p);
  pl.rr = allow_rr && use_rr(p);
  pl.fixed = p->precision == CG_PREC_FIXED;
  pl.precond = p->precond;
  pl.rr_period = p->rr_period;
  pl.vc = p->kx != nullptr;
  if (pl.fixed) {
    // one unknown per thread up to 1024 unknowns, then 1024 threads
    const int64_t dof = (int64_t)p->nx * p->ny;
    pl.wg = true;
    pl.fx_threads = (int)std::min<int64_t>(kFxThreads, round_up((size_t)dof, (size_t)kWave));
  }
  if (pl.rr) {
    pl.wg = true;
    pl.rr_threads = (int)round_up((size_t)rr_threads_needed(p->nx, p->ny), (size_t)kWave);
  }
  int rows, grid = 0;
  if (pl.wg) {
    rows = wg_rows(p->nx, p->ny);
  } else {
    auto it = pins.find(key(p->nx, ny, pl.fp32g, p->variant));
    if (it != pins.end()) {
      rows = it->second.rows;
      grid = it->second.grid;
      // classic FP64 may run with 4 columns (32 B) per lane (the 5-point
      // operator without the preconditioner: the other passes are written
      // for 2)
      if (!pl.refined && p->variant == CG_VARIANT_CLASSIC && it->second.cpl == 4 && !pl.precond &&
          !pl.vc && p->nz <= 1)
        pl.fp32g = 1;
    } else {
      rows = unpinned_rows(p, pl.fp32g);
    }
  }
  // 3D: the z-march tiles, `rows` planes per strip
  pl.g = p->nz > 1 ? make_geo3(p->nx, p->ny, p->nz, rows) : make_geo(p->nx, ny, pl.fp32g, rows);
  // The classic passes (32-row strips of separate vectors) walk the odd
  // wavefronts of a tile upward: the row between two wavefronts' strips is
  // then read by both at about the same time (a cache hit for the second),
  // not 32 rows apart (measured at 4096^2: stencil_dot 84.1 -> 81.8 us,
  // update_norm 148.0 -> 141.4 us).  The pipelined pass (8-row strips,
  // interleaved rows) measured 0.8 % slower so and keeps one direction, as
  // does the 7-point operator's walker.
  pl.g.alt = (p->variant == CG_VARIANT_CLASSIC || pl.refined) && p->nz <= 1 ? 1 : 0;
  const int T = pl.g.tiles;
  if (pl.wg) {
    pl.grid = 1;
  } else if (grid > 0) {
    pl.grid = std::max(8, (int)round_up((size_t)grid, 8));
  } else {
    const int kind = pl.refined ? K_CG2F
                     : p->variant == CG_VARIANT_PIPELINED ? (pl.precond ? K_PPCG : K_PCG)
                                                          : K_CG2;
    int cap = std::max(8, pass_max_blocks_per_cu(kind, pl.fp32g) * num_cu);
    // The pipelined pass streams best with few work-groups walking several
    // tiles each once its vectors outgrow the caches: measured per-iteration
    // times, one / two / four work-groups per CU: 1024^2 22.8 / 20.7 / 20.0 us,
    // 2048^2 60.4 / 62.3 / 62.3 us, 4096^2 286 / 289 / 297 us, 8192^2
    // 1215 / 1193 / 1203 us.  The classic passes run as many as fit.
    if (!pl.refined && p->variant == CG_VARIANT_PIPELINED) {
      const int64_t dof = (int64_t)p->nx * ny;
      if (dof > 2 * 1024 * 1024) {
        const int per_cu = dof > 24 * 1024 * 1024 ? 2 : 1;
        cap = std::max(8, std::min(cap, per_cu * num_cu));
      }
    }
    const int tpb = (T + cap - 1) / cap;          // tiles per work-group
    pl.grid = (int)round_up((size_t)((T + tpb - 1) / tpb), 8);
  }
  pl.width = pl.g.pitch;
  const size_t elems = (size_t)pl.width * ny;
  pl.v64 = round_up(elems * 8, Arena::kAlign);
  pl.v32 = round_up(elems * 4, Arena::kAlign);
  int n64, n32 = 0;
  if (pl.refined) {
    n64 = 2;                   // b, x
    n32 = pl.precond ? 5 : 4;  // rho, d, p, p' (and z)
  } else if (p->variant == CG_VARIANT_PIPELINED) {
    // b, x, r, w, w', z, q, p; preconditioned: b, x, r, u, w, m, z, q, s, p
    n64 = pl.precond ? 10 : 8;
  } else {
    n64 = pl.precond ? 6 : 5;  // b, x, r, p, p' (and z)
  }
  if (pl.precond) {
    // Chebyshev items: groups of 7 tiles across, cheb_rows rows tall, about
    // one item per resident work-group (long items amortise the s - 1 halo
    // rows each item recomputes; at least 16 rows)
    const int ngx = (pl.g.pitch + kChebGroupCols - 1) / kChebGroupCols;
    const int slots = std::max(1, cheb_max_blocks_per_cu(pl.precond, pl.refined) * num_cu /
                                      std::max(1, cheb_item_div));
    const int nty = std::max(1, slots / ngx);
    int crows = (p->ny + nty - 1) / nty;
    crows = std::max(crows, std::min(p->ny, 16));
    const int ntyc = (p->ny + crows - 1) / crows;
    pl.cheb_rows = crows;
    // partials per 128-column tile (the FP32 geometry's tiles are 256 wide)
    pl.cheb_tiles = (pl.refined ? 2 : 1) * pl.g.ntx * ntyc;
    pl.cheb_grid = (int)round_up((size_t)std::min(ngx * ntyc, slots), 8);
  }
  pl.part = round_up((size_t)ndots_max(p) * std::max(T, pl.cheb_tiles) * 8, Arena::kAlign);
  // Pipelined FP64 tile passes: the rows of all vectors interleaved, row j
  // of every vector after the other, so that a pass streams one region
  // instead of seven (the six-vector read-modify-write of cg_stream_probe:
  // 6.08 TB/s with interleaved rows, pattern 7, against 5.29 TB/s with
  // separate vectors, pattern 4; pcg_pass at 4096^2 312 -> 295 us).  The classic passes touch three or four of their
  // five vectors and measured slower interleaved (update_norm 143 -> 155 us),
  // so they keep separate vectors.
  size_t vec_bytes = n64 * pl.v64 + (pl.vc ? round_up(4 * elems * 8, Arena::kAlign) : 0);
  pl.g.kcs = (int64_t)elems;
  if (interleave && !pl.wg && !pl.refined && !pl.fixed && p->variant == CG_VARIANT_PIPELINED) {
    pl.il = n64 + (pl.vc ? 4 : 0);
    pl.g.pitch = pl.width * pl.il;
    pl.g.kcs = pl.width;
    vec_bytes = round_up((size_t)pl.il * elems * 8, Arena::kAlign);
  }
  pl.footprint = vec_bytes + n32 * pl.v32 + 2 * pl.part + 2 * round_up(sizeof(State), 256) +
                 (pl.precond ? 256 : 0);
  return pl;
}

size_t footprint_of(const cg_problem* p) {
  // same arithmetic as Ctx::plan, without a device (tiling affects only the
  // partial buffers, bounded here by one tile per 2 rows)
  const int fp32g = p->precision == CG_PREC_FP32_REFINED;
  Geo g = p->nz > 1 ? make_geo3(p->nx, p->ny, p->nz, 1) : make_geo(p->nx, rows_of(p), fp32g, 1);
  const size_t elems = (size_t)g.pitch * rows_of(p);
  const size_t v64 = round_up(elems * 8, Arena::kAlign), v32 = round_up(elems * 4, Arena::kAlign);
  size_t n64 = fp32g ? 2
               : p->variant == CG_VARIANT_PIPELINED ? (p->precond ? 10 : 8)
                                                    : (p->precond ? 6 : 5);
  size_t n32 = fp32g ? (p->precond ? 5 : 4) : 0;
  const size_t part = round_up((size_t)ndots_max(p) * g.tiles * 8, Arena::kAlign);
  return n64 * v64 + n32 * v32 + 2 * part + 2 * round_up(sizeof(State), 256) +
         (p->precond ? 256 : 0) + (p->kx ? round_up(4 * elems * 8, Arena::kAlign) : 0);
}

// --------------------------------------------------------- profiling --

void Ctx::prof_add(const char* name, double seconds, double bytes, int64_t launches) {
  auto& s = stats[name];
  s.launches += launches;
  s.seconds += seconds;
  s.bytes += bytes;
}

hipEvent_t Ctx::event() {
  if (!ev_free.empty()) {
    hipEvent_t e = ev_free.back();
    ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Ctx::prof_collect() {
  for (auto& pr : pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pr.a, pr.b) == hipSuccess)
      prof_add(pr.name, ms * 1e-3, pr.bytes, 1);
    ev_free.push_back(pr.a);
    ev_free.push_back(pr.b);
  }
  pending.clear();
}

static const char* kind_name(int kind, int fp32g) {
  switch (kind) {
    case K_INIT_R: return fp32g ? "init_r_f32geo" : "init_r";
    case K_INIT_W: return "init_w";
    case K_PCG: return "pcg_pass_nx";
    case K_PCGX: return "pcg_pass";
    case K_CG1: return "stencil_dot";
    case K_CG2: return "update_norm_nx";
    case K_CG2X: return "update_norm";
    case K_RESID: return fp32g ? "resid_f32geo" : "resid";
    case K_REF_SCALE: return "ref_scale";
    case K_CG1F: return "stencil_dot_f32";
    case K_CG2F: return "update_norm_f32_nx";
    case K_CG2FX: return "update_norm_f32";
    case K_REF_UPDATE: return "ref_update";
    case K_CHEB: return "cheb_precond";
    case K_CHEBW: return "cheb_precond_w";
    case K_CHEBF: return "cheb_precond_f32";
    case K_INIT_WU: return "init_wu";
    case K_PPCG: return "ppcg_pass";
    case K_APPLY: return "apply";
    case K_DOT: return "dot";
    case K_RRQ: return "rr_q";
    case K_RRZ: return "rr_z";
  }
  return "?";
}

// Launches one pass; with profiling on, brackets it by events.
// A `check` pass only classifies the state reached by the previous pass (its
// body never runs); it is recorded under "final_check" with no bytes.
hipError_t Ctx::pass(int kind, int fp32g, const PassArgs& a, int grid, bool check) {
  if (!prof || capturing) return launch_pass(kind, fp32g, a, grid, st);
  hipEvent_t e0 = event(), e1 = event();
  (void)hipEventRecord(e0, st);
  hipError_t rc = launch_pass(kind, fp32g, a, grid, st);
  (void)hipEventRecord(e1, st);
  // the variable-coefficient operator also reads its four coefficients per
  // unknown in every pass that applies it
  const int64_t dof = (int64_t)a.g.nx * a.g.ny;
  const double kc_bytes = a.g.kc && kind != K_DOT ? 32.0 * (double)dof : 0.0;
  pending.push_back({e0, e1, check ? "final_check" : kind_name(kind, fp32g),
                     check ? 0.0 : (double)pass_algorithmic_bytes(kind, dof) + kc_bytes});
  return rc;
}

// ---------------------------------------------------------------- solve --

bool carve(Ctx& c, Work& w) {
  // an interleaved block holds exactly the vectors carved from it below
  if (w.pl.il > 1 && (w.pl.variant != CG_VARIANT_PIPELINED ||
                      w.pl.il != (w.pl.precond ? 10 : 8) + (w.pl.vc ? 4 : 0)))
    return false;
  w.mem = (char*)c.arena.alloc(w.pl.footprint);
  if (!w.mem) return false;
  char* q = w.mem;
  auto take = [&](size_t n) {
    char* r = q;
    q += n;
    return r;
  };
  const Plan& pl = w.pl;
  if (pl.il > 1) {
    // one block, the vectors' rows interleaved: vector k starts k rows of
    // one vector in
    double* blk = (double*)take(round_up((size_t)pl.il * pl.width * pl.g.ny * 8, Arena::kAlign));
    int k = 0;
    auto vec = [&]() { return blk + (size_t)(k++) * pl.width; };
    w.b = vec();
    w.x = vec();
    w.r = vec();
    w.w[0] = vec();
    if (pl.precond) {
      w.u = vec();
      w.mv = vec();
      w.sv = vec();
    } else {
      w.w[1] = vec();
    }
    w.z = vec();
    w.q = vec();
    w.p = vec();
    if (pl.vc) {
      w.kc = vec();  // west; east, south and north follow, width apart
      k += 3;
    }
    if (pl.precond) w.cheb = (double*)take(256);
    w.part[0] = (double*)take(pl.part);
    w.part[1] = (double*)take(pl.part);
    w.S[0] = (State*)take(round_up(sizeof(State), 256));
    w.S[1] = (State*)take(round_up(sizeof(State), 256));
    return true;
  }
  w.b = (double*)take(pl.v64);
  w.x = (double*)take(pl.v64);
  if (pl.refined) {
    w.rf = (float*)take(pl.v32);
    w.df = (float*)take(pl.v32);
    w.pf[0] = (float*)take(pl.v32);
    w.pf[1] = (float*)take(pl.v32);
    if (pl.precond) {
      w.zf = (float*)take(pl.v32);
      w.cheb = (double*)take(256);
    }
  } else if (pl.variant == CG_VARIANT_PIPELINED) {
    w.r = (double*)take(pl.v64);
    w.w[0] = (double*)take(pl.v64);
    if (pl.precond) {
      w.u = (double*)take(pl.v64);
      w.mv = (double*)take(pl.v64);
      w.sv = (double*)take(pl.v64);
      w.cheb = (double*)take(256);
    } else {
      w.w[1] = (double*)take(pl.v64);
    }
    w.z = (double*)take(pl.v64);
    w.q = (double*)take(pl.v64);
    w.p = (double*)take(pl.v64);
  } else {
    w.r = (double*)take(pl.v64);
    if (pl.precond) {
      w.z = (double*)take(pl.v64);
      w.cheb = (double*)take(256);
    }
    w.pc[0] = (double*)take(pl.v64);
    w.pc[1] = (double*)take(pl.v64);
  }
  w.part[0] = (double*)take(pl.part);
  w.part[1] = (double*)take(pl.part);
  w.S[0] = (State*)take(round_up(sizeof(State), 256));
  w.S[1] = (State*)take(round_up(sizeof(State), 256));
  if (pl.vc) w.kc = (double*)take(round_up(4 * (size_t)pl.g.pitch * pl.g.ny * 8, Arena::kAlign));
  return true;
}

static PassArgs base_args(const Work& w) {
  PassArgs a;
  memset(&a, 0, sizeof(a));
  a.g = w.pl.g;
  a.g.kc = w.kc;
  a.b = w.b;
  a.x = w.x;
  a.r = w.r;
  a.z = w.z;
  a.q = w.q;
  a.p = w.p;
  a.rf = w.rf;
  a.df = w.df;
  a.zf = w.zf;
  a.uu = w.u;
  a.sv = w.sv;
  a.mv = w.mv;
  a.wv = w.w[0];
  return a;
}

// Issues one pass of the solve with the state/partial double buffers of pass
// number w.m; `mod` sets the vector ping-pong pointers.
template <class F>
static hipError_t issue(Ctx& c, Work& w, int kind, F mod) {
  PassArgs a = base_args(w);
  a.st_in = w.S[w.m & 1];
  a.st_out = w.S[(w.m + 1) & 1];
  a.part_in = w.part[w.m & 1];
  a.part_out = w.part[(w.m + 1) & 1];
  a.rev = w.m & 1;
  mod(a);
  w.m++;
  const int grid =
      (kind == K_CHEB || kind == K_CHEBW || kind == K_CHEBF) ? w.pl.cheb_grid : w.pl.grid;
  return c.pass(kind, w.pl.fp32g, a, grid, w.check);
}

static hipError_t issue_iteration(Ctx& c, Work& w) {
  hipError_t e;
  const int i = w.i;
  if (w.pl.refined) {
    // preconditioned: the inner stop test and z = M^-1 r first (FP32), and
    // the direction is p = z + beta p
    e = hipSuccess;
    if (w.pl.precond)
      e = issue(c, w, K_CHEBF, [&](PassArgs& a) {
        a.cheb = w.cheb;
        a.cheb_s = w.pl.precond;
        a.cheb_rows = w.pl.cheb_rows;
        a.pf_in = w.pf[i & 1];  // direction of a pending d update, if the test stops
      });
    if (e == hipSuccess)
      e = issue(c, w, K_CG1F, [&](PassArgs& a) {
        if (w.pl.precond) {
          a.rf = w.zf;
          a.cheb_tiles = w.pl.cheb_tiles;
        }
        a.pf_in = w.pf[i & 1];
        a.pf_out = w.pf[(i + 1) & 1];
      });
    if (e == hipSuccess)
      e = issue(c, w, (i & 1) ? K_CG2FX : K_CG2F, [&](PassArgs& a) {
        a.pf_in = w.pf[(i + 1) & 1];
        a.pf_prev = w.pf[i & 1];
      });
  } else if (w.pl.variant == CG_VARIANT_PIPELINED && w.pl.precond) {
    // preconditioned: the scalar step and m = M^-1 w, then the fused pass
    e = issue(c, w, K_CHEBW, [&](PassArgs& a) {
      a.r = w.w[0];  // input of the Chebyshev pass
      a.z = w.mv;    // its output
      a.cheb = w.cheb;
      a.cheb_s = w.pl.precond;
      a.cheb_rows = w.pl.cheb_rows;
    });
    if (e == hipSuccess) e = issue(c, w, K_PPCG, [](PassArgs&) {});
  } else if (w.pl.variant == CG_VARIANT_PIPELINED) {
    // iteration i + 1 of the solve: an even one also brings x up to date
    e = issue(c, w, (i & 1) ? K_PCGX : K_PCG, [&](PassArgs& a) {
      a.w_in = w.w[i & 1];
      a.w_out = w.w[(i + 1) & 1];
    });
    // residual replacement after iteration i + 1 (even: x is current): q = A p
    // and z = A q (plain stencil passes, no state), then r = b - A x with its
    // sums and w = A r with (r,r), (w,r), the sums the next iteration takes
    if (e == hipSuccess && w.pl.rr_period > 0 && (i + 1) % w.pl.rr_period == 0) {
      PassArgs a = base_args(w);
      a.u = w.p;
      a.y = w.q;
      e = c.pass(K_APPLY, w.pl.fp32g, a, w.pl.grid, w.check);
      if (e == hipSuccess) {
        a.u = w.q;
        a.y = w.z;
        e = c.pass(K_APPLY, w.pl.fp32g, a, w.pl.grid, w.check);
      }
      if (e == hipSuccess) e = issue(c, w, K_INIT_R, [](PassArgs&) {});
      if (e == hipSuccess)
        e = issue(c, w, K_INIT_W, [&](PassArgs& a2) { a2.w_out = w.w[(i + 1) & 1]; });
    }
  } else {
    // preconditioned: z = M^-1 r first, and the direction is p = z + beta p
    e = hipSuccess;
    if (w.pl.precond)
      e = issue(c, w, K_CHEB, [&](PassArgs& a) {
        a.z = w.z;
        a.cheb = w.cheb;
        a.cheb_s = w.pl.precond;
        a.cheb_rows = w.pl.cheb_rows;
        a.pc_in = w.pc[i & 1];  // direction of a pending x update, if the test stops
      });
    if (e == hipSuccess)
      e = issue(c, w, K_CG1, [&](PassArgs& a) {
        if (w.pl.precond) {
          a.r = w.z;
          a.cheb_tiles = w.pl.cheb_tiles;
        }
        a.pc_in = w.pc[i & 1];
        a.pc_out = w.pc[(i + 1) & 1];
      });
    if (e == hipSuccess)
      e = issue(c, w, (i & 1) ? K_CG2X : K_CG2, [&](PassArgs& a) {
        a.pc_in = w.pc[(i + 1) & 1];
        a.pc_prev = w.pc[i & 1];
      });
  }
  w.i++;
  return e;
}

#define HIPCHK(x)                                     \
  do {                                                \
    hipError_t e_ = (x);                              \
    if (e_ != hipSuccess) {                           \
      c.last_error = hipGetErrorString(e_);           \
      return CG_E_DEVICE;                             \
    }                                                 \
  } while (0)

// Reads the state the next pass would read (after w.m passes).
static int read_state(Ctx& c, Work& w, State& out) {
  HIPCHK(hipMemcpyAsync(c.host_state, w.S[w.m & 1], sizeof(State), hipMemcpyDeviceToHost, c.st));
  HIPCHK(hipStreamSynchronize(c.st));
  if (c.prof) c.prof_collect();
  memcpy(&out, c.host_state, sizeof(State));
  return CG_OK;
}

// Runs `iters` iterations as one hipGraph replay; the graph is cached per
// workspace layout, chunk length and buffer parity.
static int run_chunk(Ctx& c, Work& w, int iters) {
  const bool graphs = c.graph_chunk > 0 && !c.prof;
  if (!graphs) {
    for (int k = 0; k < iters; ++k) HIPCHK(issue_iteration(c, w));
    return CG_OK;
  }
  const Plan& pl = w.pl;
  // with residual replacement the chunk's passes depend on where in the
  // replacement period it starts
  const int rph = pl.rr_period > 0 ? w.i % pl.rr_period : 0;
  GraphKey key{w.mem,
               {pl.g.nx, pl.g.ny, pl.g.rows, pl.grid, pl.variant, pl.refined, iters, w.m & 1,
                w.i & 1, pl.precond, pl.fp32g, pl.g.plane, pl.vc, pl.cheb_rows, pl.rr_period,
                rph}};
  auto it = c.graphs.find(key);
  if (it == c.graphs.end()) {
    hipGraph_t g;
    HIPCHK(hipStreamBeginCapture(c.st, hipStreamCaptureModeThreadLocal));
    c.capturing = true;
    const int m0 = w.m, i0 = w.i;
    hipError_t e = hipSuccess;
    for (int k = 0; k < iters && e == hipSuccess; ++k) e = issue_iteration(c, w);
    c.capturing = false;
    hipError_t e2 = hipStreamEndCapture(c.st, &g);
    w.m = m0;
    w.i = i0;
    HIPCHK(e);
    HIPCHK(e2);
    hipGraphExec_t ge;
    hipError_t e3 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e3);
    if (c.graphs.size() > 64) {
      for (auto& kv : c.graphs) (void)hipGraphExecDestroy(kv.second);
      c.graphs.clear();
    }
    it = c.graphs.emplace(key, ge).first;
  }
  HIPCHK(hipGraphLaunch(it->second, c.st));
  w.m += iters * (w.pl.variant == CG_VARIANT_PIPELINED && !w.pl.refined
                      ? (w.pl.precond ? 2 : 1)
                  : w.pl.precond ? 3
                                 : 2);
  // two state passes (K_INIT_R, K_INIT_W) per replacement in the chunk
  if (pl.rr_period > 0) w.m += 2 * ((w.i + iters) / pl.rr_period - w.i / pl.rr_period);
  w.i += iters;
  return CG_OK;
}

void Ctx::forget_graphs(const void* mem) {
  for (auto it = graphs.begin(); it != graphs.end();) {
    if (it->first.mem == mem) {
      (void)hipGraphExecDestroy(it->second);
      it = graphs.erase(it);
    } else {
      ++it;
    }
  }
}

// The Chebyshev preconditioner's coefficients (the same closed-form spectrum
// interval and recurrence as the oracle; both run on the host, so both get
// the host's cos()).
void cheb_coeffs(int nx, int ny, int s, double* out) {
  const double pi = 3.14159265358979323846;
  const double hi = 4.0 + 2.0 * std::cos(pi / (double)(nx + 1)) +
                    2.0 * std::cos(pi / (double)(ny + 1));
  const double lo = hi / (2.0 * (double)s * (double)s);
  const double theta = (hi + lo) / 2.0, delta = (hi - lo) / 2.0;
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  out[0] = 1.0 / theta;
  for (int k = 1; k < s; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    out[k] = rn * rho;                   // c1
    out[s - 1 + k] = 2.0 * rn / delta;   // c2
    rho = rn;
  }
}

State initial_state(const cg_problem* p) {
  State s;
  memset(&s, 0, sizeof(s));
  s.status = ST_RUNNING;
  s.flags = F_BB_PENDING | (p->precond > 0 ? F_PRECOND : 0);
  s.tol = p->tol;
  s.inner_tol = p->inner_tol > 0.0 ? p->inner_tol : 1e-4;
  s.maxit = p->maxit;
  return s;
}

int stage_in_async(Ctx& c, Work& w, const cg_problem* p, const State* pinned) {
  const Plan& pl = w.pl;
  HIPCHK(launch_fill(w.mem, pl.footprint, c.st));
  const hipMemcpyKind kind = p->mem == CG_MEM_HOST ? hipMemcpyHostToDevice
                                                   : hipMemcpyDeviceToDevice;
  const size_t row = (size_t)p->nx * 8, pitch = (size_t)pl.g.pitch * 8;
  HIPCHK(hipMemcpy2DAsync(w.b, pitch, p->b, row, row, rows_of(p), kind, c.st));
  if (p->x0) HIPCHK(hipMemcpy2DAsync(w.x, pitch, p->x0, row, row, rows_of(p), kind, c.st));
  if (pl.vc) {
    // cell arrays of the face conductivities: west kx[j][i], east kx[j][i+1],
    // south ky[j][i], north ky[j+1][i] (padding stays zero from the fill)
    const size_t one = (size_t)pl.g.kcs, rx = (size_t)(p->nx + 1) * 8;
    HIPCHK(hipMemcpy2DAsync(w.kc, pitch, p->kx, rx, row, p->ny, kind, c.st));
    HIPCHK(hipMemcpy2DAsync(w.kc + one, pitch, p->kx + 1, rx, row, p->ny, kind, c.st));
    HIPCHK(hipMemcpy2DAsync(w.kc + 2 * one, pitch, p->ky, row, row, p->ny, kind, c.st));
    HIPCHK(hipMemcpy2DAsync(w.kc + 3 * one, pitch, p->ky + p->nx, row, row, p->ny, kind, c.st));
  }
  HIPCHK(hipMemcpyAsync(w.S[0], pinned, sizeof(State), hipMemcpyHostToDevice, c.st));
  w.m = 0;
  w.i = 0;
  w.maxit = p->maxit;
  w.check = false;
  return CG_OK;
}

int stage_in(Ctx& c, Work& w, const cg_problem* p) {
  const State s = initial_state(p);
  memcpy(c.host_state, &s, sizeof(s));
  int rc = stage_in_async(c, w, p, (const State*)c.host_state);
  if (rc) return rc;
  if (w.pl.precond) {
    double* coef = (double*)(c.host_state + 1024);  // past the state, same pinned page
    cheb_coeffs(p->nx, p->ny, w.pl.precond, coef);
    HIPCHK(hipMemcpyAsync(w.cheb, coef, (size_t)(2 * w.pl.precond - 1) * sizeof(double),
                          hipMemcpyHostToDevice, c.st));
  }
  // the pinned staging buffer is reused by the next call: wait for the copy
  HIPCHK(hipStreamSynchronize(c.st));
  return CG_OK;
}

int stage_out(Ctx& c, Work& w, const cg_problem* p, const State& s) {
  const hipMemcpyKind kind = p->mem == CG_MEM_HOST ? hipMemcpyDeviceToHost
                                                   : hipMemcpyDeviceToDevice;
  const size_t row = (size_t)p->nx * 8, pitch = (size_t)w.pl.g.pitch * 8;
  if (s.status == ST_ZERO_RHS) {
    if (p->mem == CG_MEM_HOST) memset(p->x, 0, row * rows_of(p));
    else HIPCHK(hipMemsetAsync(p->x, 0, row * rows_of(p), c.st));
  } else {
    HIPCHK(hipMemcpy2DAsync(p->x, row, w.x, pitch, row, rows_of(p), kind, c.st));
  }
  HIPCHK(hipStreamSynchronize(c.st));
  return CG_OK;
}

void fill_result(const State& s, cg_result* res, double secs, bool refined) {
  memset(res, 0, sizeof(*res));
  res->status = map_status(s.status);
  res->iterations = s.k;
  res->outer_iterations = s.outer;
  if (s.status == ST_ZERO_RHS) {
    res->iterations = 0;
    res->rel_res_recursive = res->rel_res_true = 0.0;
  } else {
    // refinement: the outer residual is the true FP64 residual itself
    res->rel_res_recursive = std::sqrt((refined ? s.res2 : s.gamma) / s.bb);
    res->rel_res_true = std::sqrt(s.res2 / s.bb);
  }
  res->device_seconds = secs;
  res->latency_seconds = secs;
}

static int chunk_iters(Ctx& c, const Work& w) {
  int k = c.graph_chunk > 0 ? c.graph_chunk : 32;
  // small grids: longer chunks (launch-bound); keep it even
  const int64_t dof = (int64_t)w.pl.g.nx * w.pl.g.ny;
  if (dof < 512 * 512) k *= 4;
  else if (dof < 2048 * 2048) k *= 2;
  return std::max(2, k & ~1);
}

static int solve_tiled(Ctx& c, Work& w, const cg_problem* p, State& s) {
  int rc;
  if (w.pl.refined) {
    // outer loop: resid -> scale -> inner chunks -> update
    HIPCHK(issue(c, w, K_RESID, [](PassArgs&) {}));
    HIPCHK(issue(c, w, K_REF_SCALE, [](PassArgs&) {}));
    for (;;) {
      if ((rc = read_state(c, w, s))) return rc;
      if (s.status != ST_RUNNING) break;
      w.i = 0;  // inner direction ping-pong restarts every inner solve
      for (;;) {
        // while profiling, one iteration per chunk so that at most one no-op
        // pass pair per inner solve enters the statistics
        if ((rc = run_chunk(c, w, c.prof ? 1 : chunk_iters(c, w)))) return rc;
        if ((rc = read_state(c, w, s))) return rc;
        if (s.status != ST_RUNNING) break;
      }
      if (s.status != ST_INNER_DONE) break;
      HIPCHK(issue(c, w, K_REF_UPDATE, [](PassArgs&) {}));
      HIPCHK(issue(c, w, K_RESID, [](PassArgs&) {}));
      HIPCHK(issue(c, w, K_REF_SCALE, [](PassArgs&) {}));
    }
    return CG_OK;
  }
  HIPCHK(issue(c, w, K_INIT_R, [](PassArgs&) {}));
  if (w.pl.variant == CG_VARIANT_PIPELINED && w.pl.precond) {
    // u = M^-1 r (with the first stop test), then w = A u and the three sums
    HIPCHK(issue(c, w, K_CHEB, [&](PassArgs& a) {
      a.z = w.u;
      a.cheb = w.cheb;
      a.cheb_s = w.pl.precond;
      a.cheb_rows = w.pl.cheb_rows;
    }));
    HIPCHK(issue(c, w, K_INIT_WU, [](PassArgs&) {}));
  } else if (w.pl.variant == CG_VARIANT_PIPELINED) {
    HIPCHK(issue(c, w, K_INIT_W, [&](PassArgs& a) { a.w_out = w.w[0]; }));
  }
  const int K = chunk_iters(c, w);
  for (;;) {
    // never issue iterations past maxit: after maxit iterations one more
    // pass only classifies the final state
    const int left = p->maxit - w.i;
    w.check = left <= 0;
    if ((rc = run_chunk(c, w, left > 0 ? std::min(K, left) : 1))) return rc;
    w.check = false;
    if ((rc = read_state(c, w, s))) return rc;
    if (s.status != ST_RUNNING) break;
  }
  if (s.status != ST_ZERO_RHS) {
    HIPCHK(issue(c, w, K_RESID, [](PassArgs&) {}));
    PassArgs a = base_args(w);
    a.st_in = w.S[w.m & 1];
    a.st_out = w.S[(w.m + 1) & 1];
    a.part_in = w.part[w.m & 1];
    w.m++;
    HIPCHK(launch_final(a, c.st));
    if ((rc = read_state(c, w, s))) return rc;
  }
  return CG_OK;
}

static int solve_wg(Ctx& c, Work& w, const cg_problem* p, State& s) {
  PassArgs a = base_args(w);
  a.st_in = w.S[0];
  a.st_out = w.S[1];
  a.part_in = w.part[0];
  a.part_out = w.part[1];
  if (p->variant == CG_VARIANT_PIPELINED) {
    a.w_in = w.w[0];
    a.w_out = w.w[1];
  } else {
    a.pc_in = w.pc[0];
    a.pc_out = w.pc[1];
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c.prof) {
    e0 = c.event();
    e1 = c.event();
    (void)hipEventRecord(e0, c.st);
  }
  HIPCHK(launch_solve_wg(p->variant, a, c.st));
  if (c.prof) {
    (void)hipEventRecord(e1, c.st);
    c.pending.push_back({e0, e1, "solve_wg", 0.0});
  }
  w.m = 1;
  return read_state(c, w, s);
}

static int solve_fixed(Ctx& c, Work& w, const cg_problem* p, State& s) {
  FxArgs a;
  memset(&a, 0, sizeof(a));
  a.g = w.pl.g;
  a.b = w.b;
  a.x = w.x;
  a.bq = reinterpret_cast<int64_t*>(w.r);
  a.xq = reinterpret_cast<int64_t*>(p->variant == CG_VARIANT_PIPELINED ? w.z : w.pc[0]);
  a.qg = reinterpret_cast<int64_t*>(w.q);
  a.S[0] = w.S[0];
  a.S[1] = w.S[1];
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c.prof) {
    e0 = c.event();
    e1 = c.event();
    (void)hipEventRecord(e0, c.st);
  }
  HIPCHK(launch_solve_fixed(p->variant, a, w.pl.fx_threads, c.st));
  if (c.prof) {
    (void)hipEventRecord(e1, c.st);
    c.pending.push_back({e0, e1, "solve_fixed", 0.0});
  }
  w.m = 1;
  return read_state(c, w, s);
}

static int solve_rr(Ctx& c, Work& w, const cg_problem* p, State& s) {
  PassArgs a = base_args(w);
  a.st_in = w.S[0];
  a.st_out = w.S[1];
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c.prof) {
    e0 = c.event();
    e1 = c.event();
    (void)hipEventRecord(e0, c.st);
  }
  HIPCHK(launch_solve_rr(p->variant, a, w.pl.rr_threads, c.st));
  if (c.prof) {
    (void)hipEventRecord(e1, c.st);
    c.pending.push_back({e0, e1, "solve_rr", 0.0});
  }
  w.m = 1;
  return read_state(c, w, s);
}

int Ctx::solve(const cg_problem* p, cg_result* res) {
  Ctx& c = *this;
  const double t0 = now_s();
  Work w;
  w.pl = plan(p);
  if (w.pl.footprint > arena.size()) return CG_E_NOMEM;
  if (!carve(c, w)) return CG_E_NOMEM;
  struct Release {
    Ctx& c;
    Work& w;
    ~Release() { c.arena.release(w.mem); }
  } rel{c, w};
  int rc = order_after_user();
  if (rc) return rc;
  if ((rc = stage_in(c, w, p))) return rc;
  State s;
  rc = w.pl.fixed ? solve_fixed(c, w, p, s)
       : w.pl.rr  ? solve_rr(c, w, p, s)
       : w.pl.wg  ? solve_wg(c, w, p, s)
                  : solve_tiled(c, w, p, s);
  if (rc) return rc;
  if ((rc = stage_out(c, w, p, s))) return rc;
  fill_result(s, res, now_s() - t0, w.pl.refined);
  return res->status;
}

// The caller's stream (the null stream when none was given) must reach this
// point before the library reads any input: the library's own streams are
// non-blocking, so nothing orders them after the null stream implicitly.
int Ctx::order_after_user() {
  Ctx& c = *this;
  HIPCHK(hipEventRecord(user_ev, user_stream));
  HIPCHK(hipStreamWaitEvent(st, user_ev, 0));
  return CG_OK;
}

// ------------------------------------------------------- building blocks --

int Ctx::apply_or_dot(int kind, int nx, int ny, cg_memspace mem, const double* u,
                      const double* y_in, double* y_out, double* dot_out) {
  Ctx& c = *this;
  cg_problem p;
  memset(&p, 0, sizeof(p));
  p.nx = nx;
  p.ny = ny;
  p.maxit = 1;
  p.variant = CG_VARIANT_CLASSIC;
  p.precision = CG_PREC_FP64;
  // the tile geometry (hence reduction order) of this shape; always run by
  // the multi-work-group pass kernels
  Plan pl = plan(&p, false, false);
  if (pl.wg) {
    const int cap = std::max(8, pass_max_blocks_per_cu(kind, 0) * num_cu);
    pl.grid = (int)round_up((size_t)std::min(pl.g.tiles, cap), 8);
  }
  const size_t need = 2 * pl.v64 + pl.part + round_up(sizeof(State), 256);
  char* m = (char*)arena.alloc(need);
  if (!m) return CG_E_NOMEM;
  struct Rel {
    Arena& a;
    char* m;
    ~Rel() { a.release(m); }
  } rel{arena, m};
  double* U = (double*)m;
  double* Y = (double*)(m + pl.v64);
  double* part = (double*)(m + 2 * pl.v64);
  State* S = (State*)(m + 2 * pl.v64 + pl.part);
  int rc = order_after_user();
  if (rc) return rc;
  HIPCHK(launch_fill(m, need, st));
  const hipMemcpyKind kin = mem == CG_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  const size_t row = (size_t)nx * 8, pitch = (size_t)pl.g.pitch * 8;
  HIPCHK(hipMemcpy2DAsync(U, pitch, u, row, row, ny, kin, st));
  if (kind == K_DOT) HIPCHK(hipMemcpy2DAsync(Y, pitch, y_in, row, row, ny, kin, st));
  PassArgs a;
  memset(&a, 0, sizeof(a));
  a.g = pl.g;
  a.u = U;
  a.y = Y;
  a.part_out = part;
  HIPCHK(pass(kind, 0, a, pl.grid));
  if (kind == K_APPLY) {
    const hipMemcpyKind kout =
        mem == CG_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    HIPCHK(hipMemcpy2DAsync(y_out, row, Y, pitch, row, ny, kout, st));
  } else {
    PassArgs f;
    memset(&f, 0, sizeof(f));
    f.g = pl.g;
    f.part_in = part;
    f.st_in = S;  // zero-filled state; res2 receives the sum
    f.st_out = S;
    HIPCHK(launch_final(f, st));
    HIPCHK(hipMemcpyAsync(host_state, S, sizeof(State), hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  if (prof) prof_collect();
  if (kind == K_DOT) {
    State s;
    memcpy(&s, host_state, sizeof(s));
    *dot_out = s.res2;
  }
  return CG_OK;
}

// ------------------------------------------------------------ HBM probe --

int Ctx::stream_probe(int pattern, size_t elems, int reps, double* seconds, double* bytes) {
  Ctx& c = *this;
  static const int nv[] = {1, 2, 3, 5, 6, 12, 6, 6};
  static const int moved[] = {1, 2, 3, 5, 12, 12, 12, 12};
  if (pattern < 0 || pattern > 7 || elems < 2 || reps < 1) return CG_E_INVALID;
  elems &= ~(size_t)1;
  if (pattern == 7) {
    // whole rows of 4096 doubles; the six vectors form one contiguous block
    elems &= ~(size_t)4095;
    if (elems == 0) return CG_E_INVALID;
  }
  const size_t vb = round_up(elems * 8, Arena::kAlign);
  char* m = (char*)arena.alloc(nv[pattern] * vb + 256);
  if (!m) return CG_E_NOMEM;
  struct Rel {
    Arena& a;
    char* m;
    ~Rel() { a.release(m); }
  } rel{arena, m};
  double* v[12];
  for (int k = 0; k < 12; ++k) v[k] = (double*)(m + (k < nv[pattern] ? k : 0) * vb);
  double* sink = (double*)(m + nv[pattern] * vb);
  HIPCHK(launch_fill(m, nv[pattern] * vb + 256, st));
  hipEvent_t e0 = event(), e1 = event();
  double best = 1e30;
  // best over grids of 1, 2, 4 and 8 work-groups per CU
  for (int gpc = 1; gpc <= 8; gpc *= 2) {
    const int grid = gpc * num_cu;
    for (int r = 0; r < reps + 1; ++r) {
      HIPCHK(hipEventRecord(e0, st));
      HIPCHK(launch_stream(pattern, v, elems, sink, grid, st));
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (r > 0) best = std::min(best, ms * 1e-3);  // the first launch warms up
    }
  }
  ev_free.push_back(e0);
  ev_free.push_back(e1);
  *seconds = best;
  *bytes = (double)moved[pattern] * elems * 8.0;
  return CG_OK;
}

int Ctx::mul_probe(int rounds, int reps, double* seconds, double* ops) {
  Ctx& c = *this;
  if (rounds < 1 || reps < 1) return CG_E_INVALID;
  const int grid = 8 * num_cu;
  uint64_t* sink = (uint64_t*)arena.alloc((size_t)grid * 256 * sizeof(uint64_t));
  if (!sink) return CG_E_NOMEM;
  struct Rel {
    Arena& a;
    void* m;
    ~Rel() { a.release(m); }
  } rel{arena, sink};
  hipEvent_t e0 = event(), e1 = event();
  double best = 1e30;
  for (int r = 0; r < reps + 1; ++r) {
    HIPCHK(hipEventRecord(e0, st));
    HIPCHK(launch_mul_probe(sink, grid, rounds, st));
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    if (r > 0) best = std::min(best, ms * 1e-3);  // the first launch warms up
  }
  ev_free.push_back(e0);
  ev_free.push_back(e1);
  *seconds = best;
  *ops = (double)grid * 256 * 8 * rounds;
  return CG_OK;
}

// ---------------------------------------------------------- autotuner --

// Times candidate tile shapes for one grid shape on the device and pins the
// fastest.  Candidates: rows per wavefront strip x work-groups per pass (the
// occupancy limit and 1/2, 1/3, 1/4 of it, capped by the tile count) x
// columns per lane (2 or 4 for classic FP64).  Each candidate runs a short
// fixed-iteration solve (tol = 0) twice; the score is the HIP-event time of
// the iteration kernels of the second run per iteration.
int Ctx::tune(int nx, int ny, int variant, int precision) {
  Ctx& c = *this;
  cg_problem p;
  memset(&p, 0, sizeof(p));
  p.nx = nx;
  p.ny = ny;
  p.variant = (cg_variant)variant;
  p.precision = (cg_precision)precision;
  p.tol = 0.0;
  p.maxit = 24;
  p.mem = CG_MEM_DEVICE;
  if (use_wg(&p)) return CG_OK;  // single work-group path: nothing to tune
  const int fp32g = precision == CG_PREC_FP32_REFINED;
  const size_t n = (size_t)nx * ny;
  char* bx = (char*)arena.alloc(2 * n * 8);
  if (!bx) return CG_E_NOMEM;
  struct Rel {
    Arena& a;
    char* m;
    ~Rel() { a.release(m); }
  } rel{arena, bx};
  double* b = (double*)bx;
  double* x = b + n;
  HIPCHK(launch_fill(bx, 2 * n * 8, st));
  // b = 1 everywhere: the timing does not depend on the values
  std::vector<double> ones(std::min<size_t>(n, 1 << 20), 1.0);
  for (size_t o = 0; o < n; o += ones.size()) {
    const size_t k = std::min(ones.size(), n - o);
    HIPCHK(hipMemcpyAsync(b + o, ones.data(), k * 8, hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  p.b = b;
  p.x = x;
  const uint64_t k = key(nx, ny, fp32g, variant);
  std::vector<const char*> names;
  if (fp32g) names = {"stencil_dot_f32", "update_norm_f32", "update_norm_f32_nx"};
  else if (variant == CG_VARIANT_PIPELINED) names = {"pcg_pass", "pcg_pass_nx"};
  else names = {"stencil_dot", "update_norm", "update_norm_nx"};
  std::vector<int> cpls = {0};
  if (!fp32g && variant == CG_VARIANT_CLASSIC) cpls = {2, 4};
  const bool save_prof = prof;
  const auto save_stats = stats;
  prof = true;
  double best = 1e30;
  // the shape the solve takes unpinned is the fallback and the first
  // candidate, so the pick is never slower than it by the tuner's measure
  pins.erase(k);
  Pin bestp{unpinned_rows(&p, fp32g), plan(&p).grid, 0};
  auto score = [&](const Pin& pin, double& t) {
    pins[k] = pin;
    cg_result r;
    if (solve(&p, &r) < 0) return false;  // warms graphs and caches
    stats.clear();
    if (solve(&p, &r) < 0) return false;
    t = 0.0;
    int64_t launches = 0;
    for (const char* nm : names) {
      auto it = stats.find(nm);
      if (it != stats.end()) {
        t += it->second.seconds;
        launches += it->second.launches;
      }
    }
    t /= (double)p.maxit;  // per iteration (tol = 0: exactly maxit of them)
    return launches > 0;
  };
  {
    double t;
    if (score(bestp, t)) best = t;
  }
  for (int cpl : cpls) {
    const int geo4 = fp32g || cpl == 4;
    const int kind = fp32g ? K_CG2F : (variant == CG_VARIANT_PIPELINED ? K_PCG : K_CG2);
    const int cap = std::max(8, pass_max_blocks_per_cu(kind, geo4) * num_cu);
    for (int rows : {2, 4, 8, 16, 32, 64}) {
      const Geo g = make_geo(nx, ny, geo4, rows);
      if (rows > 4 * ((ny + 3) / 4)) continue;
      std::vector<int> grids;
      for (int div : {1, 2, 3, 4}) {
        int gsz = (int)round_up((size_t)std::max(8, cap / div), 8);
        gsz = std::min(gsz, (int)round_up((size_t)g.tiles, 8));
        if (std::find(grids.begin(), grids.end(), gsz) == grids.end()) grids.push_back(gsz);
      }
      for (int gsz : grids) {
        double t;
        if (!score(Pin{rows, gsz, cpl}, t)) continue;
        if (t < best) {
          best = t;
          bestp = Pin{rows, gsz, cpl};
        }
      }
    }
  }
  prof = save_prof;
  stats = save_stats;
  pins[k] = bestp;
  save_tune_cache();
  return CG_OK;
}

// The tune cache is one JSON object per line:
//   {"nx": 4096, "ny": 4096, "fp32": 0, "rows": 32, "grid": 1024, "cpl": 2}
void Ctx::load_tune_cache() {
  if (tune_path.empty()) return;
  FILE* f = fopen(tune_path.c_str(), "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof(line), f)) {
    // a pin measured on another architecture or HIP runtime is ignored
    int nx, ny, fp, var, rows, grid, cpl, hv;
    char ar[64];
    if (sscanf(line,
               " {\"arch\": \"%63[^\"]\", \"hip\": %d, \"nx\": %d, \"ny\": %d, \"fp32\": %d, "
               "\"variant\": %d, \"rows\": %d, \"grid\": %d, \"cpl\": %d}",
               ar, &hv, &nx, &ny, &fp, &var, &rows, &grid, &cpl) == 9 &&
        arch == ar && hv == hip_version && nx > 0 && ny > 0 && rows > 0 && rows <= 4096 &&
        grid >= 0 && (var == 0 || var == 1) && (cpl == 0 || cpl == 2 || cpl == 4))
      pins[key(nx, ny, fp, var)] = Pin{rows, grid, cpl};
  }
  fclose(f);
}

void Ctx::save_tune_cache() {
  if (tune_path.empty()) return;
  FILE* f = fopen(tune_path.c_str(), "w");
  if (!f) return;
  for (auto& kv : pins)
    fprintf(f,
            "{\"arch\": \"%s\", \"hip\": %d, \"nx\": %d, \"ny\": %d, \"fp32\": %d, "
            "\"variant\": %d, \"rows\": %d, \"grid\": %d, \"cpl\": %d}\n",
            arch.c_str(), hip_version, (int)(kv.first >> 34),
            (int)((kv.first >> 2) & 0xffffffff), (int)(kv.first & 1), (int)((kv.first >> 1) & 1),
            kv.second.rows, kv.second.grid, kv.second.cpl);
  fclose(f);
}

// --------------------------------------------------------------- create --

int Ctx::init(const cg_config* cfg) {
  Ctx& c = *this;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return CG_E_DEVICE;
  device = cfg ? cfg->device : 0;
  if (device < 0 || device >= ndev) return CG_E_DEVICE;
  HIPCHK(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  num_cu = prop.multiProcessorCount;
  {
    // "gfx950:sramecc+:xnack-": the architecture name before the features
    std::string a = prop.gcnArchName;
    arch = a.substr(0, a.find(':'));
    if (hipRuntimeGetVersion(&hip_version) != hipSuccess) hip_version = 0;
  }
  HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&user_ev, hipEventDisableTiming));
  HIPCHK(hipHostMalloc((void**)&host_state, 4096, hipHostMallocDefault));
  user_stream = cfg ? (hipStream_t)cfg->stream : nullptr;
  size_t bytes = cfg ? cfg->arena_bytes : 0;
  void* base = cfg ? cfg->arena : nullptr;
  if (!base) {
    if (bytes == 0) bytes = (size_t)4 << 30;
    HIPCHK(hipMalloc(&base, bytes));
    own_arena = base;
  } else if (bytes == 0) {
    return CG_E_INVALID;
  }
  arena.init((char*)base, bytes);
  max_slots = (cfg && cfg->max_slots > 0) ? cfg->max_slots : 256;
  if (cfg && cfg->tune_cache) tune_path = cfg->tune_cache;
  if (const char* e = getenv("CG_GRAPH_CHUNK")) graph_chunk = atoi(e);
  if (const char* e = getenv("CG_WG_MAX_DOF")) wg_max_dof = atoi(e);
  if (const char* e = getenv("CG_RR")) rr_enabled = atoi(e) != 0;
  if (const char* e = getenv("CG_STEP_CHUNK")) step_chunk = std::max(1, atoi(e));
  if (const char* e = getenv("CG_SERVE_CHUNK")) serve_chunk = std::max(1, atoi(e));
  if (const char* e = getenv("CG_CHEB_ITEM_DIV")) cheb_item_div = std::max(1, atoi(e));
  load_tune_cache();
  return CG_OK;
}

Ctx::~Ctx() {
  (void)hipSetDevice(device);
  if (st) (void)hipStreamSynchronize(st);
  if (side) (void)hipStreamSynchronize(side);
  for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& pr : pending) {
    (void)hipEventDestroy(pr.a);
    (void)hipEventDestroy(pr.b);
  }
  for (auto e : ev_free) (void)hipEventDestroy(e);
  if (user_ev) (void)hipEventDestroy(user_ev);
  if (host_state) (void)hipHostFree(host_state);
  if (own_arena) (void)hipFree(own_arena);
  if (side) (void)hipStreamDestroy(side);
  if (st) (void)hipStreamDestroy(st);
}

}  // namespace cgr
