// cg_abi.cpp - the extern "C" entry points of include/cg.h.
//
// Every call validates its arguments before touching the device, returns a
// negative CG_E_* code without side effects when it rejects, and serialises
// on the context's mutex.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/cg.h"
#include "cg_runtime.h"

using cgr::Ctx;

static Ctx* C(cg_ctx* c) { return reinterpret_cast<Ctx*>(c); }

extern "C" {

int cg_create(const cg_config* cfg, cg_ctx** out) {
  if (!out) return CG_E_INVALID;
  *out = nullptr;
  if (cfg && cfg->arena && cfg->arena_bytes == 0) return CG_E_INVALID;
  Ctx* c = new (std::nothrow) Ctx;
  if (!c) return CG_E_NOMEM;
  int rc = c->init(cfg);
  if (rc) {
    delete c;
    return rc;
  }
  *out = reinterpret_cast<cg_ctx*>(c);
  return CG_OK;
}

int cg_destroy(cg_ctx* ctx) {
  if (!ctx) return CG_E_INVALID;
  Ctx* c = C(ctx);
  cgr_server_stop(c);
  delete c;
  return CG_OK;
}

int cg_solve(cg_ctx* ctx, const cg_problem* prob, cg_result* res) {
  if (!ctx || !res) return CG_E_INVALID;
  int rc = cgr::validate(prob);
  if (rc) return rc;
  const cg_problem q = cgr::resolve_precision(*prob);
  Ctx* c = C(ctx);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  if (hipSetDevice(c->device) != hipSuccess) return CG_E_DEVICE;
  return c->solve(&q, res);
}

int cg_solve_batch(cg_ctx* ctx, const cg_problem* probs, int32_t n, cg_result* results) {
  if (!ctx || !probs || !results || n < 1) return CG_E_INVALID;
  std::vector<cg_problem> q;
  try {
    q.resize(n);
  } catch (const std::bad_alloc&) {
    return CG_E_NOMEM;
  }
  for (int32_t i = 0; i < n; ++i) {
    int rc = cgr::validate(&probs[i]);
    if (rc) return rc;
    q[i] = cgr::resolve_precision(probs[i]);
  }
  Ctx* c = C(ctx);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  if (hipSetDevice(c->device) != hipSuccess) return CG_E_DEVICE;
  return c->solve_batch(q.data(), n, results);
}

int cg_submit(cg_ctx* ctx, const cg_problem* prob, uint64_t* ticket) {
  if (!ctx || !ticket) return CG_E_INVALID;
  int rc = cgr::validate(prob);
  if (rc) return rc;
  const cg_problem q = cgr::resolve_precision(*prob);
  return cgr_server_submit(C(ctx), &q, ticket);
}

int cg_poll(cg_ctx* ctx, uint64_t ticket, cg_result* res) {
  if (!ctx || !res) return CG_E_INVALID;
  return cgr_server_poll(C(ctx), ticket, res);
}

const char* cg_status_str(int code) {
  switch (code) {
    case CG_OK: return "CG_OK";
    case CG_PENDING: return "CG_PENDING";
    case CG_NOT_CONVERGED: return "CG_NOT_CONVERGED";
    case CG_BREAKDOWN: return "CG_BREAKDOWN";
    case CG_E_INVALID: return "CG_E_INVALID";
    case CG_E_NOMEM: return "CG_E_NOMEM";
    case CG_E_DEVICE: return "CG_E_DEVICE";
    case CG_E_BUSY: return "CG_E_BUSY";
    case CG_E_TICKET: return "CG_E_TICKET";
  }
  return "CG_UNKNOWN";
}

int cg_apply(cg_ctx* ctx, int32_t nx, int32_t ny, cg_memspace mem, const double* u, double* y) {
  if (!ctx || nx < 1 || ny < 1 || !u || !y || (mem != CG_MEM_HOST && mem != CG_MEM_DEVICE))
    return CG_E_INVALID;
  Ctx* c = C(ctx);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  if (hipSetDevice(c->device) != hipSuccess) return CG_E_DEVICE;
  return c->apply_or_dot(cgk::K_APPLY, nx, ny, mem, u, nullptr, y, nullptr);
}

int cg_dot(cg_ctx* ctx, int32_t nx, int32_t ny, cg_memspace mem, const double* a,
           const double* b, double* out) {
  if (!ctx || nx < 1 || ny < 1 || !a || !b || !out ||
      (mem != CG_MEM_HOST && mem != CG_MEM_DEVICE))
    return CG_E_INVALID;
  Ctx* c = C(ctx);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  if (hipSetDevice(c->device) != hipSuccess) return CG_E_DEVICE;
  return c->apply_or_dot(cgk::K_DOT, nx, ny, mem, a, b, nullptr, out);
}

int cg_plan(cg_ctx* ctx, const cg_problem* prob, cg_plan_info* info) {
  if (!ctx || !info) return CG_E_INVALID;
  if (!prob || prob->nx < 1 || prob->ny < 1 || prob->nz < 0) return CG_E_INVALID;
  if (prob->precision == CG_PREC_FIXED && !cgk::fixed_fits(prob->nx, prob->ny))
    return CG_E_INVALID;
  Ctx* c = C(ctx);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  const cg_problem q = cgr::resolve_precision(*prob);
  cgr::Plan pl = c->plan(&q);
  memset(info, 0, sizeof(*info));
  info->path = pl.fixed ? 3 : pl.rr ? 2 : pl.wg ? 1 : 0;
  info->seg_rows = pl.rr ? cgk::kRrRows : 0;
  info->seg_waves = pl.rr ? pl.rr_threads / cgk::kWave : 0;
  info->seg_cols = pl.rr ? prob->nx + 1 : 0;
  info->cols_per_lane = pl.fp32g ? 4 : 2;
  info->lanes = cgk::kWave;
  info->waves = cgk::kWavesPerTile;
  info->rows = pl.g.rows;
  info->threads2 = cgk::kGroup;
  info->tiles = pl.g.tiles;
  info->grid = pl.grid;
  info->pitch = pl.width;
  info->row_stride = pl.g.pitch;
  info->walk_alt = pl.g.alt;
  info->walk_z = pl.g.plane > 0 ? 1 : 0;
  info->cheb_rows = pl.cheb_rows;
  info->cheb_tiles = pl.cheb_tiles;
  info->cheb_grid = pl.precond ? pl.cheb_grid : 0;
  info->footprint = pl.footprint;
  return CG_OK;
}

int cg_footprint(const cg_problem* prob, size_t* bytes) {
  if (!prob || !bytes || prob->nx < 1 || prob->ny < 1) return CG_E_INVALID;
  const cg_problem q = cgr::resolve_precision(*prob);
  *bytes = cgr::footprint_of(&q);
  return CG_OK;
}

int cg_validate(const cg_problem* prob) { return cgr::validate(prob); }

int cg_tune(cg_ctx* ctx, int32_t nx, int32_t ny, cg_variant variant, cg_precision precision) {
  if (!ctx || nx < 1 || ny < 1) return CG_E_INVALID;
  if (variant != CG_VARIANT_CLASSIC && variant != CG_VARIANT_PIPELINED) return CG_E_INVALID;
  if (precision == CG_PREC_FIXED) return CG_OK;  // one work-group, no tile shape
  if (precision != CG_PREC_FP64 && precision != CG_PREC_FP32_REFINED) return CG_E_INVALID;
  Ctx* c = C(ctx);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  if (hipSetDevice(c->device) != hipSuccess) return CG_E_DEVICE;
  return c->tune(nx, ny, variant, precision);
}

int cg_pin_tile(cg_ctx* ctx, int32_t nx, int32_t ny, cg_precision precision, int32_t rows,
                int32_t grid, int32_t cols_per_lane) {
  if (!ctx || nx < 1 || ny < 1 || rows < 1 || rows > 4096 || grid < 0) return CG_E_INVALID;
  if (precision != CG_PREC_FP64 && precision != CG_PREC_FP32_REFINED) return CG_E_INVALID;
  if (cols_per_lane != 0 && cols_per_lane != 2 && cols_per_lane != 4) return CG_E_INVALID;
  if (precision == CG_PREC_FP32_REFINED && cols_per_lane == 2) return CG_E_INVALID;
  Ctx* c = C(ctx);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  // the shape is pinned for both variants (refined solves have one key)
  const int fp = precision == CG_PREC_FP32_REFINED;
  for (int v = 0; v < 2; ++v)
    c->pins[Ctx::key(nx, ny, fp, v)] = cgr::Pin{rows, grid, cols_per_lane};
  return CG_OK;
}

int cg_stream_probe(cg_ctx* ctx, int32_t pattern, size_t elems, int32_t reps, double* seconds,
                    double* bytes) {
  if (!ctx || !seconds || !bytes || pattern < 0 || pattern > 7 || elems < 2 || reps < 1)
    return CG_E_INVALID;
  Ctx* c = C(ctx);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  if (hipSetDevice(c->device) != hipSuccess) return CG_E_DEVICE;
  return c->stream_probe(pattern, elems, reps, seconds, bytes);
}

int cg_mul_probe(cg_ctx* ctx, int32_t rounds, int32_t reps, double* seconds, double* ops) {
  if (!ctx || !seconds || !ops || rounds < 1 || reps < 1) return CG_E_INVALID;
  Ctx* c = C(ctx);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  if (hipSetDevice(c->device) != hipSuccess) return CG_E_DEVICE;
  return c->mul_probe(rounds, reps, seconds, ops);
}

int cg_set_profiling(cg_ctx* ctx, int32_t on) {
  if (!ctx) return CG_E_INVALID;
  Ctx* c = C(ctx);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  c->prof = on != 0;
  return CG_OK;
}

int cg_kernel_stats(cg_ctx* ctx, cg_kstat* out, int32_t max, int32_t* count, int32_t reset) {
  if (!ctx || !count || max < 0 || (max > 0 && !out)) return CG_E_INVALID;
  Ctx* c = C(ctx);
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  *count = (int32_t)c->stats.size();
  int32_t i = 0;
  for (auto& kv : c->stats) {
    if (i >= max) break;
    memset(&out[i], 0, sizeof(cg_kstat));
    strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
    out[i].launches = kv.second.launches;
    out[i].seconds = kv.second.seconds;
    out[i].bytes = kv.second.bytes;
    ++i;
  }
  if (reset) c->stats.clear();
  return CG_OK;
}

const char* cg_version(void) { return "mi355x-stencil-cg 0.1 (gfx950)"; }

}  // extern "C"
