// cg_noalloc.hip - cg_solve_batch_small_noalloc: small solves without any
// device allocation, for callers that cannot allocate (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The solves run on the on-chip solver of cg_solve_batch (one work-group per
// solve, every vector in registers or LDS) straight on the caller's device
// vectors (row-major, pitch nx).  The only device memory beyond the inputs and
// outputs is a file-scope array, `scratch`, that holds the solves' descriptors,
// their scalar states and the work-group -> solve index: kNoAllocMaxSolves
// of each.  Every call on a device shares that device's array and rewrites all
// of it that the call reads, so nothing carries over from one call to the next.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <mutex>

#include "../../include/cg.h"
#include "cg_runtime.h"

namespace {

using namespace cgk;

constexpr int kNoAllocMaxSolves = 64;
constexpr int kMaxDevices = 64;

struct ScratchLayout {
  Slot slots[kNoAllocMaxSolves];
  State states[2 * kNoAllocMaxSolves];
  int idx[kNoAllocMaxSolves];
};
constexpr size_t kScratchBytes = 64 * 1024;
static_assert(sizeof(ScratchLayout) <= kScratchBytes, "scratch too small");

}  // namespace

// One copy on each device the library runs on, held until the process ends.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of `scratch` on each device (host code uses only these: the
// array's name in host code is a host-side stand-in, not a device address).
void* g_scratch[kMaxDevices] = {};
std::mutex g_mu[kMaxDevices];

// Looks the array's address up on the current device, once per device.
int scratch_of(int dev, void** out) {
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CG_E_DEVICE;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return CG_OK;
}

bool fits_on_chip(const cg_problem& p) {
  return p.precision == CG_PREC_FP64 && p.precond == 0 && p.nz <= 1 && !p.kx &&
         (int64_t)(p.nx + 1) * ((p.ny + kRrRows - 1) / kRrRows) <= kRrThreads;
}

}  // namespace

extern "C" int cg_solve_batch_small_noalloc(const cg_problem* probs, int32_t n, void* stream,
                                            cg_result* results) {
  using clk = std::chrono::steady_clock;
  if (!probs || !results || n < 1 || n > kNoAllocMaxSolves) return CG_E_INVALID;
  for (int32_t i = 0; i < n; ++i) {
    const cg_problem& p = probs[i];
    if (cgr::validate(&p) || p.mem != CG_MEM_DEVICE || !fits_on_chip(p)) return CG_E_INVALID;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CG_E_DEVICE;
  std::lock_guard<std::mutex> lk(g_mu[dev]);
  void* base = nullptr;
  int rc = scratch_of(dev, &base);
  if (rc) return rc;
  const hipStream_t st = (hipStream_t)stream;
  const auto t0 = clk::now();
  ScratchLayout* d = reinterpret_cast<ScratchLayout*>(base);
  // descriptors, initial states and the index, written whole from the host
  ScratchLayout h;
  memset(&h, 0, sizeof(h));
  for (int32_t i = 0; i < n; ++i) {
    const cg_problem& p = probs[i];
    Slot& S = h.slots[i];
    S.g.nx = p.nx;
    S.g.ny = p.ny;
    S.g.pitch = p.nx;  // the caller's vectors, unpadded
    S.variant = p.variant;
    S.b = const_cast<double*>(p.b);
    S.x = p.x;
    S.S[0] = &d->states[2 * i];
    S.S[1] = &d->states[2 * i + 1];
    h.states[2 * i] = cgr::initial_state(&p);
    h.idx[i] = i;
  }
  // x0: zeros, or a copy into x (x itself when they alias)
  for (int32_t i = 0; i < n; ++i) {
    const cg_problem& p = probs[i];
    const size_t bytes = (size_t)p.nx * p.ny * sizeof(double);
    hipError_t e = hipSuccess;
    if (!p.x0) e = cgk::launch_fill(p.x, bytes, st);
    else if (p.x0 != p.x) e = hipMemcpyAsync(p.x, p.x0, bytes, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return CG_E_DEVICE;
  }
  if (hipMemcpyAsync(d, &h, sizeof(h), hipMemcpyHostToDevice, st) != hipSuccess ||
      cgk::launch_solve_rr_many(d->slots, d->idx, n, st) != hipSuccess ||
      hipMemcpyAsync(h.states, d->states, sizeof(h.states), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return CG_E_DEVICE;
  // a zero right-hand side has x = 0 as its answer
  bool zeroed = false;
  for (int32_t i = 0; i < n; ++i)
    if (h.states[2 * i].status == ST_ZERO_RHS) {
      const cg_problem& p = probs[i];
      if (cgk::launch_fill(p.x, (size_t)p.nx * p.ny * sizeof(double), st) != hipSuccess)
        return CG_E_DEVICE;
      zeroed = true;
    }
  if (zeroed && hipStreamSynchronize(st) != hipSuccess) return CG_E_DEVICE;
  const double secs = std::chrono::duration<double>(clk::now() - t0).count();
  int worst = CG_OK;
  for (int32_t i = 0; i < n; ++i) {
    cgr::fill_result(h.states[2 * i], &results[i], secs, false);
    if (results[i].status > worst) worst = results[i].status;
  }
  return worst;
}
