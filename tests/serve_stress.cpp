// Concurrency stress of the serving runtime, for a build whose host code runs
// under a sanitizer (the library's host sources and this driver instrumented,
// the kernels as usual).  Through the C ABI only:
//   - four threads submit mixed requests (2D classic and pipelined, FP32
//     refinement, the Chebyshev preconditioner, 3D, variable coefficients)
//     in host memory, polling their earlier tickets between submissions, and
//     check every result against a residual computed here on the host;
//   - one thread polls tickets that do not exist;
//   - the main thread runs blocking solves on the same context meanwhile;
//   - a last group of requests is still queued or running when the context
//     is destroyed (their buffers stay alive until cg_destroy returns).
// Exit status 0 when every check held.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "cg.h"

namespace {

struct Req {
  int nx = 0, ny = 0, nz = 0;
  int variant = 0, precision = CG_PREC_FP64, precond = 0;
  bool vc = false;
  double tol = 1e-8;
  std::vector<double> b, x, kx, ky;
  uint64_t ticket = 0;
  bool done = false;
};

// ||b - A x|| / ||b|| for the request's operator, in plain loops
double host_relres(const Req& q) {
  const int nx = q.nx, ny = q.ny, nz = q.nz > 1 ? q.nz : 1;
  auto X = [&](int i, int j, int l) -> double {
    if (i < 0 || i >= nx || j < 0 || j >= ny || l < 0 || l >= nz) return 0.0;
    return q.x[((size_t)l * ny + j) * nx + i];
  };
  double rr = 0.0, bb = 0.0;
  for (int l = 0; l < nz; ++l)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double ax;
        if (q.vc) {
          const double kw = q.kx[(size_t)j * (nx + 1) + i], ke = q.kx[(size_t)j * (nx + 1) + i + 1];
          const double ks = q.ky[(size_t)j * nx + i], kn = q.ky[(size_t)(j + 1) * nx + i];
          ax = (kw + ke + ks + kn) * X(i, j, 0) - kw * X(i - 1, j, 0) - ke * X(i + 1, j, 0) -
               ks * X(i, j - 1, 0) - kn * X(i, j + 1, 0);
        } else if (q.nz > 1) {
          ax = 6.0 * X(i, j, l) - X(i - 1, j, l) - X(i + 1, j, l) - X(i, j - 1, l) -
               X(i, j + 1, l) - X(i, j, l - 1) - X(i, j, l + 1);
        } else {
          ax = 4.0 * X(i, j, 0) - X(i - 1, j, 0) - X(i + 1, j, 0) - X(i, j - 1, 0) -
               X(i, j + 1, 0);
        }
        const double bv = q.b[((size_t)l * ny + j) * nx + i];
        rr += (bv - ax) * (bv - ax);
        bb += bv * bv;
      }
  return std::sqrt(rr / bb);
}

Req make_req(std::mt19937_64& g, int k) {
  static const int shapes[][3] = {{40, 30, 0},  {100, 100, 0}, {257, 129, 0}, {17, 3, 0},
                                  {64, 64, 0},  {300, 190, 0}, {37, 40, 23},  {130, 7, 5},
                                  {513, 257, 0}, {64, 1, 0}};
  std::uniform_real_distribution<double> u(-1.0, 1.0), kd(0.5, 2.0);
  Req q;
  const auto& s = shapes[k % 10];
  q.nx = s[0];
  q.ny = s[1];
  q.nz = s[2];
  q.variant = k & 1;
  const int kind = (k / 2) % 5;  // 0 FP64, 1 refined, 2 precond, 3 refined + precond, 4 vc
  if (q.nz <= 1) {
    if (kind == 1 || kind == 3) q.precision = CG_PREC_FP32_REFINED;
    if (kind == 2 || kind == 3) q.precond = 2 + (k % 3) * 2;
    q.vc = kind == 4;
  }
  q.tol = q.precision == CG_PREC_FP32_REFINED ? 1e-9 : 1e-8;
  const size_t n = (size_t)q.nx * q.ny * (q.nz > 1 ? q.nz : 1);
  q.b.resize(n);
  for (auto& v : q.b) v = u(g);
  q.x.assign(n, 0.0);
  if (q.vc) {
    q.kx.resize((size_t)q.ny * (q.nx + 1));
    q.ky.resize((size_t)(q.ny + 1) * q.nx);
    for (auto& v : q.kx) v = kd(g);
    for (auto& v : q.ky) v = kd(g);
  }
  return q;
}

cg_problem problem_of(Req& q, int maxit) {
  cg_problem p;
  std::memset(&p, 0, sizeof p);
  p.nx = q.nx;
  p.ny = q.ny;
  p.nz = q.nz;
  p.mem = CG_MEM_HOST;
  p.b = q.b.data();
  p.x = q.x.data();
  p.tol = q.tol;
  p.maxit = maxit;
  p.variant = (cg_variant)q.variant;
  p.precision = (cg_precision)q.precision;
  p.precond = q.precond;
  if (q.vc) {
    p.kx = q.kx.data();
    p.ky = q.ky.data();
  }
  return p;
}

std::atomic<int> g_fail{0};

void fail(const char* what, int id, int k, int rc, double v) {
  std::fprintf(stderr, "FAIL %s: thread %d request %d rc %d value %.3e\n", what, id, k, rc, v);
  g_fail.fetch_add(1);
}

// A result is right when the solve converged and the residual recomputed here
// is within a few times the tolerance (the library stops on its own
// residual, which rounding can leave slightly below the recomputed one).
void check(const Req& q, int rc, const cg_result& r, int id, int k) {
  if (rc != CG_OK || r.status != CG_OK) {
    fail("status", id, k, rc, (double)r.status);
    return;
  }
  const double rel = host_relres(q);
  if (!(rel <= 4.0 * q.tol)) fail("residual", id, k, rc, rel);
}

}  // namespace

int main() {
  cg_config cfg;
  std::memset(&cfg, 0, sizeof cfg);
  cfg.device = 0;
  cfg.arena_bytes = (size_t)1 << 30;
  cfg.max_slots = 16;
  cg_ctx* ctx = nullptr;
  const int crc = cg_create(&cfg, &ctx);
  if (crc != CG_OK) {
    int n = -1;
    const hipError_t e = hipGetDeviceCount(&n);
    std::fprintf(stderr, "FAIL cg_create: %s; hipGetDeviceCount: %s, %d devices\n",
                 cg_status_str(crc), hipGetErrorString(e), n);
    return 2;
  }
  const int kThreads = 4, kPer = 25;
  std::atomic<bool> stop_bogus{false};

  auto worker = [&](int id) {
    std::mt19937_64 g(1000 + id);
    std::vector<Req> reqs;
    reqs.reserve(kPer);
    int finished = 0;
    auto poll_some = [&](bool all) {
      const auto t0 = std::chrono::steady_clock::now();
      while (true) {
        for (int k = 0; k < (int)reqs.size(); ++k) {
          Req& q = reqs[k];
          if (q.done) continue;
          cg_result r;
          const int rc = cg_poll(ctx, q.ticket, &r);
          if (rc == CG_PENDING) continue;
          q.done = true;
          ++finished;
          check(q, rc, r, id, k);
          cg_result r2;
          if (cg_poll(ctx, q.ticket, &r2) != CG_E_TICKET) fail("released ticket", id, k, 0, 0);
        }
        if (!all || finished == (int)reqs.size()) return;
        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(180)) {
          fail("deadline", id, finished, 0, 0);
          return;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(200));
      }
    };
    for (int k = 0; k < kPer; ++k) {
      reqs.push_back(make_req(g, id * kPer + k));
      cg_problem p = problem_of(reqs.back(), 20000);
      const int rc = cg_submit(ctx, &p, &reqs.back().ticket);
      if (rc != CG_OK) {
        fail("submit", id, k, rc, 0);
        reqs.back().done = true;
        ++finished;
      }
      poll_some(false);
      std::this_thread::sleep_for(std::chrono::microseconds(300 * (k % 3)));
    }
    poll_some(true);
  };

  std::vector<std::thread> th;
  for (int i = 0; i < kThreads; ++i) th.emplace_back(worker, i);
  std::thread bogus([&] {
    uint64_t t = (uint64_t)1 << 40;
    while (!stop_bogus.load()) {
      cg_result r;
      if (cg_poll(ctx, t++, &r) != CG_E_TICKET) fail("unknown ticket", -1, 0, 0, 0);
      std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
  });
  // blocking solves on the same context while the server runs
  std::mt19937_64 g(7);
  for (int k = 0; k < 6; ++k) {
    Req q = make_req(g, 3 * k + 1);
    cg_problem p = problem_of(q, 20000);
    cg_result r;
    const int rc = cg_solve(ctx, &p, &r);
    check(q, rc, r, -2, k);
  }
  for (auto& t : th) t.join();
  stop_bogus.store(true);
  bogus.join();

  // requests still queued or running when the context goes away
  std::vector<Req> late;
  late.reserve(12);
  for (int k = 0; k < 12; ++k) {
    late.push_back(make_req(g, k));
    cg_problem p = problem_of(late.back(), 20000);
    if (cg_submit(ctx, &p, &late.back().ticket) != CG_OK) fail("late submit", -3, k, 0, 0);
  }
  if (cg_destroy(ctx) != CG_OK) fail("destroy", -3, 0, 0, 0);

  const int nf = g_fail.load();
  std::printf("serve_stress: %d threads x %d served requests, 6 blocking solves, 12 requests "
              "pending at destroy: %s\n",
              kThreads, kPer, nf ? "FAILED" : "ok");
  return nf ? 1 : 0;
}
