// cg_runtime.h - host runtime types of the stencil CG library.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cg.h"
#include "cg_arena.h"
#include "cg_internal.h"

namespace cgr {

struct Plan {
  int variant = 0;
  bool refined = false;
  int fp32g = 0;     // geometry of the FP32 lanes (4 columns per lane)
  bool wg = false;   // whole solve inside one work-group
  bool rr = false;   // ... with the vectors on chip (register-resident solver)
  int rr_threads = 0;
  bool fixed = false;  // fixed-point solve, one work-group (cg_fixed.hip)
  int precond = 0;     // Chebyshev preconditioner steps (classic FP64, tile passes)
  int cheb_rows = 0;   // ... rows of a Chebyshev item / partial tile
  int cheb_tiles = 0;  // ... partials of the Chebyshev pass
  int cheb_grid = 8;   // ... work-groups of the Chebyshev pass
  int fx_threads = 0;
  bool vc = false;     // variable-coefficient operator (four coefficient arrays)
  int width = 0;       // padded row length of one vector, in elements
  int il = 1;          // FP64 vectors with interleaved rows (g.pitch = il * width)
  int rr_period = 0;   // pipelined: residual replacement every rr_period iterations
  bool on_side() const { return rr || fixed; }  // batch: whole solve beside the steps
  cgk::Geo g{};
  int grid = 8;      // work-groups per pass
  size_t v64 = 0, v32 = 0, part = 0, footprint = 0;
};

struct Pin {
  int rows = 0;
  int grid = 0;
  int cpl = 0;  // columns per lane; 0 = default (2 for FP64, 4 for refined)
};

// A captured chunk of iterations holds every pass argument, so its key names
// everything that shapes them: the workspace, the geometry and operator, the
// iteration and the buffer parities.
struct GraphKey {
  const void* mem;
  int v[16];  // nx, ny, rows, grid, variant, refined, iters, mpar, ipar, precond,
              // fp32g, plane, vc, cheb_rows, rr_period, iteration within the period
  bool operator<(const GraphKey& o) const {
    if (mem != o.mem) return mem < o.mem;
    for (int i = 0; i < 16; ++i)
      if (v[i] != o.v[i]) return v[i] < o.v[i];
    return false;
  }
};

struct KStat {
  int64_t launches = 0;
  double seconds = 0.0, bytes = 0.0;
};

struct PendingEv {
  hipEvent_t a, b;
  const char* name;
  double bytes;
};

// Workspace of one resident solve, carved from the arena.
struct Work {
  Plan pl;
  char* mem = nullptr;
  double *b = nullptr, *x = nullptr, *r = nullptr, *w[2] = {}, *z = nullptr, *q = nullptr,
         *p = nullptr, *pc[2] = {};
  float *rf = nullptr, *df = nullptr, *pf[2] = {};
  float* zf = nullptr;  // refinement, preconditioned: z = M^-1 r_in
  double* cheb = nullptr;  // preconditioner coefficients (c0, c1[s-1], c2[s-1])
  double *u = nullptr, *sv = nullptr, *mv = nullptr;  // preconditioned pipelined
  double* kc = nullptr;  // variable coefficients: west, east, south, north arrays
  double* part[2] = {};
  cgk::State* S[2] = {};
  int m = 0;  // passes issued (state/partial parity)
  int i = 0;  // iterations issued (vector ping-pong parity)
  int maxit = 0;
  bool check = false;  // the passes being issued only classify the final state
};

struct Ctx;
double now_s();
bool carve(Ctx& c, Work& w);
int stage_in(Ctx& c, Work& w, const cg_problem* p);
cgk::State initial_state(const cg_problem* p);
// c0, c1[s-1], c2[s-1] of the Chebyshev preconditioner with s steps
void cheb_coeffs(int nx, int ny, int s, double* out);
// stage_in without waiting: the initial state is copied from `pinned` (host
// memory the caller keeps unchanged until the stream has passed the copy).
int stage_in_async(Ctx& c, Work& w, const cg_problem* p, const cgk::State* pinned);
int stage_out(Ctx& c, Work& w, const cg_problem* p, const cgk::State& s);
void fill_result(const cgk::State& s, cg_result* res, double secs, bool refined);

int validate(const cg_problem* p);
// CG_PREC_AUTO's choice: FP64 below kAutoRefineDof unknowns, FP32-refined from
// there (measured in batches of equal requests on the step engine: refinement
// 0.81x FP64's solves/s at 128^2, 1.17-1.39x from 181^2 to 2048^2); any other
// precision unchanged
constexpr int64_t kAutoRefineDof = 20480;
cg_problem resolve_precision(const cg_problem& p);
size_t footprint_of(const cg_problem* p);
cgk::Geo make_geo(int nx, int ny, int fp32g, int rows);
cgk::Geo make_geo3(int nx, int plane, int nz, int zc);
int default_rows(int nx, int ny, int fp32g);

class Server;  // serving scheduler (cg_serve.cpp)

struct Ctx {
  int device = 0;
  int num_cu = 256;
  hipStream_t st = nullptr;
  hipStream_t side = nullptr;  // register-resident solves of a batch, beside the steps
  hipStream_t user_stream = nullptr;
  hipEvent_t user_ev = nullptr;
  void* own_arena = nullptr;
  Arena arena;
  int max_slots = 256;
  std::string tune_path;
  std::recursive_mutex mu;
  char* host_state = nullptr;  // pinned staging for state words
  int graph_chunk = 32;        // iterations per captured chunk; 0 = plain launches
  int wg_max_dof = 16384;      // whole-solve-in-one-work-group threshold (FP64)
  bool rr_enabled = true;      // register-resident solver for grids that fit it
  int step_chunk = 32;         // batch: steps between harvests
  int serve_chunk = 8;         // serving: steps between admissions
  int cheb_item_div = 1;       // Chebyshev items per pass: resident work-groups / this
  int step_chunk_for(bool serving) const { return serving ? serve_chunk : step_chunk; }
  size_t engine_bytes() const {  // control block of the multi-solve engine
    return (size_t)max_slots * (sizeof(cgk::Slot) + 2 * 256 * sizeof(cgk::Item) +
                                2 * sizeof(int) + sizeof(cgk::State)) + 8192;
  }
  bool capturing = false;
  bool prof = false;
  std::string last_error;
  std::map<uint64_t, Pin> pins;  // tile shape pinned per grid shape
  std::map<GraphKey, hipGraphExec_t> graphs;
  std::map<std::string, KStat> stats;
  std::vector<PendingEv> pending;
  std::vector<hipEvent_t> ev_free;
  Server* server = nullptr;
  std::mutex server_mu;  // guards `server` only (submit/poll never wait for an epoch)

  // pins are kept per grid shape, precision and variant (the refined inner
  // solve is classic whatever the variant, so refined pins use variant 0)
  static uint64_t key(int nx, int ny, int fp32g, int variant) {
    const uint64_t v = fp32g ? 0 : (uint64_t)(variant & 1);
    return ((uint64_t)(uint32_t)nx << 34) | ((uint64_t)(uint32_t)ny << 2) | (v << 1) |
           (uint64_t)(fp32g & 1);
  }
  std::string arch;      // gcnArchName of the device (tune cache key)
  int hip_version = 0;   // hipRuntimeGetVersion (tune cache key)
  int init(const cg_config* cfg);
  ~Ctx();
  bool use_wg(const cg_problem* p) const;
  bool use_rr(const cg_problem* p) const;
  // allow_rr = false: the tile geometry even where the register-resident
  // solver would run the problem (building blocks use tiles)
  // interleave: lay the FP64 vectors of a tile-pass solve out with their rows
  // interleaved (off for the building blocks' scratch vectors)
  Plan plan(const cg_problem* p, bool allow_rr = true, bool interleave = true);
  // strip height of a tile-pass solve when no tile shape is pinned
  int unpinned_rows(const cg_problem* p, int fp32g) const;
  int solve(const cg_problem* p, cg_result* res);
  int solve_batch(const cg_problem* p, int n, cg_result* res);
  int apply_or_dot(int kind, int nx, int ny, cg_memspace mem, const double* u, const double* y_in,
                   double* y_out, double* dot_out);
  int tune(int nx, int ny, int variant, int precision);
  void load_tune_cache();
  void save_tune_cache();
  int order_after_user();
  hipError_t pass(int kind, int fp32g, const cgk::PassArgs& a, int grid, bool check = false);
  int stream_probe(int pattern, size_t elems, int reps, double* seconds, double* bytes);
  int mul_probe(int rounds, int reps, double* seconds, double* ops);
  hipEvent_t event();
  void prof_add(const char* name, double seconds, double bytes, int64_t launches);
  void prof_collect();
  void forget_graphs(const void* mem);
};

}  // namespace cgr

// Serving front end (cg_serve.cpp).
int cgr_server_submit(cgr::Ctx* c, const cg_problem* p, uint64_t* ticket);
int cgr_server_poll(cgr::Ctx* c, uint64_t ticket, cg_result* res);
void cgr_server_stop(cgr::Ctx* c);
