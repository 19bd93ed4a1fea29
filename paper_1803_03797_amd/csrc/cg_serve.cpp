// cg_serve.cpp - many solves on one GPU: the multi-solve step engine behind
// cg_solve_batch, and the continuous-batching request server behind
// cg_submit / cg_poll.
//
// Engine: a fixed array of device slots (cgk::Slot).  A solve is admitted
// into a free slot when its device footprint fits the arena (its workspace is
// carved from the arena, its inputs staged, its state initialised).  Every
// launch of the step kernel then advances all resident solves by one pass,
// over a table of (solve, tile range) items; chunks of steps run back to
// back, and between chunks finished solves are harvested (solution copied
// out, memory returned) and new ones admitted.  Each solve keeps its vectors
// and scalars resident on the device from admission to retirement.  Solves
// small enough for the register-resident solver take no step items: the
// chunk that follows their admission also launches them, one work-group
// each, on a side stream, and the next harvest waits for them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cg_runtime.h"

namespace cgr {

using namespace cgk;

struct Job {
  Job() = default;
  Job(const Job&) = delete;
  Job& operator=(const Job&) = delete;
  ~Job() {
    if (ready) (void)hipEventDestroy(ready);
  }
  cg_problem p;
  hipEvent_t ready = nullptr;  // served request: the caller's stream at submission
  uint64_t ticket = 0;
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
  Work w;
  int slot = -1;
  int64_t steps_cap = 0;
  bool finished = false;
  int rc = CG_PENDING;  // final status (or a negative error)
  cg_result res{};
};

class Engine {
 public:
  static constexpr int kMaxItemsPerSolve = 256;

  explicit Engine(Ctx& c, int nslots) : c_(c), n_(std::max(1, nslots)) {}
  ~Engine() {
    if (rr_pending_) (void)hipStreamSynchronize(c_.side);
    if (rr_ev_) (void)hipEventDestroy(rr_ev_);
    if (stage_ev_) (void)hipEventDestroy(stage_ev_);
    if (h_rr_idx_) (void)hipHostFree(h_rr_idx_);
    if (graph_) (void)hipGraphExecDestroy(graph_);
    for (Job* j : slot_job_)
      if (j) c_.arena.release(j->w.mem);
    if (ctrl_) c_.arena.release(ctrl_);
    if (h_slots_) (void)hipHostFree(h_slots_);
    if (h_items_) (void)hipHostFree(h_items_);
    if (h_idx_) (void)hipHostFree(h_idx_);
    if (h_states_) (void)hipHostFree(h_states_);
    if (h_admit_) (void)hipHostFree(h_admit_);
    if (h_coef_) (void)hipHostFree(h_coef_);
    if (h_citems_) (void)hipHostFree(h_citems_);
    if (h_step_) (void)hipHostFree(h_step_);
  }

  int init() {
    max_items_ = n_ * kMaxItemsPerSolve;
    const size_t b_slots = round256((size_t)n_ * sizeof(Slot));
    const size_t b_items = round256((size_t)max_items_ * sizeof(Item));
    const size_t b_idx = round256((size_t)n_ * sizeof(int) + sizeof(int));
    const size_t b_states = round256((size_t)n_ * sizeof(State));
    const size_t b_rr = round256((size_t)n_ * sizeof(int));
    // Chebyshev items (the same budget as the tile items) and, per s, their
    // count and offset
    const size_t b_citems = round256((size_t)max_items_ * sizeof(Item));
    const size_t b_cinfo = round256(2 * (kChebMaxSteps + 1) * sizeof(int));
    ctrl_ = (char*)c_.arena.alloc(b_slots + b_items + b_idx + b_states + b_rr + 256 + b_citems +
                                  b_cinfo);
    if (!ctrl_) return CG_E_NOMEM;
    d_citems_ = (Item*)(ctrl_ + b_slots + b_items + b_idx + b_states + b_rr + 256);
    d_cinfo_ = (int*)((char*)d_citems_ + b_citems);
    d_slots_ = (Slot*)ctrl_;
    d_items_ = (Item*)(ctrl_ + b_slots);
    d_idx_ = (int*)(ctrl_ + b_slots + b_items);
    d_nitems_ = d_idx_ + n_;
    d_states_ = (State*)(ctrl_ + b_slots + b_items + b_idx);
    d_rr_idx_ = (int*)(ctrl_ + b_slots + b_items + b_idx + b_states);
    d_step_ = (int*)(ctrl_ + b_slots + b_items + b_idx + b_states + b_rr);
    if (hipEventCreateWithFlags(&rr_ev_, hipEventDisableTiming) ||
        hipEventCreateWithFlags(&stage_ev_, hipEventDisableTiming) ||
        hipHostMalloc((void**)&h_rr_idx_, (size_t)n_ * sizeof(int), hipHostMallocDefault))
      return CG_E_DEVICE;
    if (hipHostMalloc((void**)&h_slots_, (size_t)n_ * sizeof(Slot), hipHostMallocDefault) ||
        hipHostMalloc((void**)&h_items_, (size_t)max_items_ * sizeof(Item) + 256,
                      hipHostMallocDefault) ||
        hipHostMalloc((void**)&h_idx_, (size_t)n_ * sizeof(int) + 256, hipHostMallocDefault) ||
        hipHostMalloc((void**)&h_states_, (size_t)n_ * sizeof(State), hipHostMallocDefault) ||
        hipHostMalloc((void**)&h_admit_, (size_t)n_ * sizeof(State), hipHostMallocDefault) ||
        hipHostMalloc((void**)&h_coef_, (size_t)n_ * kCoefPerSlot * sizeof(double),
                      hipHostMallocDefault) ||
        hipHostMalloc((void**)&h_citems_,
                      (size_t)max_items_ * sizeof(Item) + 2 * (kChebMaxSteps + 1) * sizeof(int),
                      hipHostMallocDefault) ||
        hipHostMalloc((void**)&h_step_, kStepRing * sizeof(int), hipHostMallocDefault))
      return CG_E_DEVICE;
    memset(h_slots_, 0, (size_t)n_ * sizeof(Slot));
    slot_job_.assign(n_, nullptr);
    grid_ = std::max(8, step_max_blocks_per_cu() * c_.num_cu);
    return upload_items();
  }

  int active() const { return active_; }
  bool has_free() const { return active_ < n_; }
  int step() const { return step_; }

  // CG_OK when admitted, CG_E_NOMEM when the arena has no room right now.
  int admit(Job* j) {
    int slot = -1;
    for (int i = 0; i < n_; ++i)
      if (!slot_job_[i]) {
        slot = i;
        break;
      }
    if (slot < 0) return CG_E_BUSY;
    j->w = Work();
    j->w.pl = c_.plan(&j->p);
    if (!carve(c_, j->w)) return CG_E_NOMEM;
    // the first pass: r = b - A x (FP64) or the first outer residual
    // (refined).  The slot's pinned records stay untouched until the slot is
    // freed again, which comes after a stream synchronisation: no wait here.
    State& s = h_admit_[slot];
    s = initial_state(&j->p);
    s.kind = j->w.pl.refined ? K_RESID : K_INIT_R;
    // a served request's inputs are complete once the caller's stream has
    // passed the point of submission
    int rc = j->ready && hipStreamWaitEvent(c_.st, j->ready, 0) != hipSuccess
                 ? CG_E_DEVICE
                 : stage_in_async(c_, j->w, &j->p, &s);
    if (!rc && j->w.pl.precond) {
      // the preconditioner's coefficients, from the slot's pinned records
      double* coef = h_coef_ + (size_t)slot * kCoefPerSlot;
      cheb_coeffs(j->p.nx, j->p.ny, j->w.pl.precond, coef);
      if (hipMemcpyAsync(j->w.cheb, coef, (size_t)(2 * j->w.pl.precond - 1) * sizeof(double),
                         hipMemcpyHostToDevice, c_.st))
        rc = CG_E_DEVICE;
    }
    if (rc) {
      (void)hipStreamSynchronize(c_.st);
      c_.arena.release(j->w.mem);
      return rc;
    }
    Slot& S = h_slots_[slot];
    memset(&S, 0, sizeof(S));
    const Work& w = j->w;
    S.g = w.pl.g;
    S.g.kc = w.kc;  // variable coefficients (null otherwise)
    S.variant = j->p.variant;
    S.refined = w.pl.refined ? 1 : 0;
    S.cpl4 = w.pl.fp32g;
    // pass m of this solve runs at step admit_step + m; its state is S[m & 1]
    S.admit_step = step_;
    S.b = w.b;
    S.x = w.x;
    S.r = w.r;
    S.z = w.z;
    S.q = w.q;
    S.p = w.p;
    S.W[0] = w.w[0];
    S.W[1] = w.w[1];
    S.PC[0] = w.pc[0];
    S.PC[1] = w.pc[1];
    S.rf = w.rf;
    S.df = w.df;
    S.PF[0] = w.pf[0];
    S.PF[1] = w.pf[1];
    S.zf = w.zf;
    S.part[0] = w.part[0];
    S.part[1] = w.part[1];
    S.S[0] = w.S[0];
    S.S[1] = w.S[1];
    S.precond = w.pl.precond;
    S.rr_period = w.pl.rr_period;
    if (w.pl.precond) {
      S.cheb_rows = w.pl.cheb_rows;
      S.cheb_tiles = w.pl.cheb_tiles;
      S.cheb_items = cheb_items_of(w.pl);
      S.cheb = w.cheb;
      S.u = w.u;
      S.sv = w.sv;
      S.mv = w.mv;
    }
    if (hipMemcpyAsync(d_slots_ + slot, &S, sizeof(Slot), hipMemcpyHostToDevice, c_.st)) {
      (void)hipStreamSynchronize(c_.st);
      c_.arena.release(j->w.mem);
      return CG_E_DEVICE;
    }
    slot_job_[slot] = j;
    j->slot = slot;
    j->t_admit = now_s();
    if (w.pl.rr) rr_new_.push_back(slot);
    else if (w.pl.fixed) fx_new_.push_back(slot);
    else ++step_jobs_;
    // a bound on the passes of the solve (a guard against a solve that never
    // reaches K_DONE; it cannot trigger for a correct pass sequence)
    j->steps_cap = (int64_t)step_ + step_bound(j->p, w.pl.refined, w.pl.precond);
    ++active_;
    dirty_ = true;
    return CG_OK;
  }

  // Launches `steps` steps of every resident solve: a replay of the captured
  // chunk when `steps` is the chunk length, plain launches otherwise.
  int run(int steps) {
    if (!active_) return CG_OK;
    if (dirty_ && upload_items()) return CG_E_DEVICE;
    if (!rr_new_.empty() || !fx_new_.empty()) {
      // newly admitted small and fixed-point solves: whole solves on the side
      // stream, after their staging on the main stream (slot lists of both
      // kinds side by side in one index buffer; each slot is listed once)
      const int nr = (int)rr_new_.size(), nf = (int)fx_new_.size();
      // fixed-point slots sorted by (unknowns per thread, variant)
      std::vector<std::pair<int, int>> fx(nf);
      for (int i = 0; i < nf; ++i) {
        const cg_problem& p = slot_job_[fx_new_[i]]->p;
        const int e = fixed_elems((int64_t)p.nx * p.ny, kFxThreads);
        fx[i] = {e * 2 + (p.variant == CG_VARIANT_PIPELINED ? 1 : 0), fx_new_[i]};
      }
      std::sort(fx.begin(), fx.end());
      fx_key_.resize(nf);
      for (int i = 0; i < nf; ++i) {
        fx_key_[i] = fx[i].first;
        fx_new_[i] = fx[i].second;
      }
      memcpy(h_rr_idx_, rr_new_.data(), (size_t)nr * sizeof(int));
      memcpy(h_rr_idx_ + nr, fx_new_.data(), (size_t)nf * sizeof(int));
      if (hipMemcpyAsync(d_rr_idx_, h_rr_idx_, (size_t)(nr + nf) * sizeof(int),
                         hipMemcpyHostToDevice, c_.st) ||
          hipEventRecord(stage_ev_, c_.st) || hipStreamWaitEvent(c_.side, stage_ev_, 0) ||
          (nr && launch_solve_rr_many(d_slots_, d_rr_idx_, nr, c_.side)))
        return CG_E_DEVICE;
      if (nf) {
        hipEvent_t f0 = nullptr, f1 = nullptr;
        if (c_.prof) {
          f0 = c_.event();
          f1 = c_.event();
          (void)hipEventRecord(f0, c_.side);
        }
        // one launch per run of equal (variant, unknowns per thread)
        for (int g0 = 0; g0 < nf;) {
          int g1 = g0 + 1;
          while (g1 < nf && fx_key_[g1] == fx_key_[g0]) ++g1;
          if (launch_solve_fixed_many(d_slots_, d_rr_idx_ + nr + g0, g1 - g0, fx_key_[g0] & 1,
                                      fx_key_[g0] >> 1, c_.side))
            return CG_E_DEVICE;
          g0 = g1;
        }
        if (c_.prof) {
          (void)hipEventRecord(f1, c_.side);
          c_.pending.push_back({f0, f1, "solve_fixed_many", 0.0});
        }
      }
      if (hipEventRecord(rr_ev_, c_.side)) return CG_E_DEVICE;
      rr_new_.clear();
      fx_new_.clear();
      rr_pending_ = true;
    }
    if (!step_jobs_) return CG_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c_.prof) {
      e0 = c_.event();
      e1 = c_.event();
      (void)hipEventRecord(e0, c_.st);
    }
    // the chunk's base step, read by every launch of the chunk on the device
    int* hs = h_step_ + (ring_++ % kStepRing);
    *hs = step_;
    if (hipMemcpyAsync(d_step_, hs, sizeof(int), hipMemcpyHostToDevice, c_.st)) return CG_E_DEVICE;
    const bool use_graph = c_.graph_chunk > 0 && steps == c_.step_chunk_for(this_is_serving_);
    if (use_graph && (!graph_ || graph_steps_ != steps || graph_mask_ != cheb_mask_)) {
      if (graph_) (void)hipGraphExecDestroy(graph_);
      graph_ = nullptr;
      hipGraph_t g;
      if (hipStreamBeginCapture(c_.st, hipStreamCaptureModeThreadLocal)) return CG_E_DEVICE;
      hipError_t e = hipSuccess;
      for (int k = 0; k < steps && e == hipSuccess; ++k) e = launch_one_step(k);
      hipError_t e2 = hipStreamEndCapture(c_.st, &g);
      if (e || e2) return CG_E_DEVICE;
      e = hipGraphInstantiate(&graph_, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e) {
        graph_ = nullptr;
        return CG_E_DEVICE;
      }
      graph_steps_ = steps;
      graph_mask_ = cheb_mask_;
    }
    if (use_graph) {
      if (hipGraphLaunch(graph_, c_.st)) return CG_E_DEVICE;
    } else {
      for (int k = 0; k < steps; ++k)
        if (launch_one_step(k) != hipSuccess) return CG_E_DEVICE;
    }
    if (c_.prof) {
      (void)hipEventRecord(e1, c_.st);
      c_.pending.push_back({e0, e1, "batch_steps", 0.0});
    }
    step_ += steps;
    return CG_OK;
  }

  // Moves finished solves out: copies x back, fills the result, frees memory.
  int harvest(std::vector<Job*>& done) {
    if (!active_) return CG_OK;
    if (rr_pending_) {
      if (hipStreamWaitEvent(c_.st, rr_ev_, 0)) return CG_E_DEVICE;
      rr_pending_ = false;
    }
    int n = 0;
    for (int i = 0; i < n_; ++i)
      if (slot_job_[i]) h_idx_[n++] = i;
    if (hipMemcpyAsync(d_idx_, h_idx_, (size_t)n * sizeof(int), hipMemcpyHostToDevice, c_.st) ||
        launch_gather(d_slots_, d_idx_, n, step_, d_states_, c_.st) ||
        hipMemcpyAsync(h_states_, d_states_, (size_t)n * sizeof(State), hipMemcpyDeviceToHost,
                       c_.st) ||
        hipStreamSynchronize(c_.st))
      return CG_E_DEVICE;
    if (c_.prof) c_.prof_collect();
    for (int k = 0; k < n; ++k) {
      const int i = h_idx_[k];
      Job* j = slot_job_[i];
      const State& s = h_states_[k];
      int rc;
      if (s.kind != K_DONE) {
        if (step_ <= j->steps_cap) continue;
        // past its pass bound: this solve alone fails; the others go on
        rc = CG_E_DEVICE;
      } else {
        rc = stage_out(c_, j->w, &j->p, s);
      }
      j->t_done = now_s();
      if (rc) {
        j->rc = rc;
      } else {
        fill_result(s, &j->res, j->t_done - j->t_admit, j->w.pl.refined);
        j->rc = j->res.status;
      }
      if (!j->w.pl.on_side()) --step_jobs_;
      c_.arena.release(j->w.mem);
      j->w.mem = nullptr;
      slot_job_[i] = nullptr;
      j->slot = -1;
      --active_;
      dirty_ = true;
      done.push_back(j);
    }
    return CG_OK;
  }

  // Fails every resident solve (used after a device error).
  void abandon(std::vector<Job*>& done, int rc) {
    if (rr_pending_) (void)hipStreamSynchronize(c_.side);
    rr_pending_ = false;
    rr_new_.clear();
    fx_new_.clear();
    step_jobs_ = 0;
    for (int i = 0; i < n_; ++i) {
      Job* j = slot_job_[i];
      if (!j) continue;
      c_.arena.release(j->w.mem);
      j->w.mem = nullptr;
      j->rc = rc;
      j->t_done = now_s();
      slot_job_[i] = nullptr;
      done.push_back(j);
    }
    active_ = 0;
    dirty_ = true;
  }

 private:
  static size_t round256(size_t v) { return (v + 255) / 256 * 256; }

  // Upper bound on the step-engine passes of one solve from admission to
  // K_DONE.  FP64: the initial passes, at most two per iteration (classic:
  // pass 1 and pass 2; pipelined: one), the pass that detects the stop, the
  // true residual and its sum.  Refined: each outer step runs RESID,
  // REF_SCALE, two passes per inner iteration, the pass 1 that ends the
  // inner solve and REF_UPDATE, i.e. 2 K + 4 passes for K inner iterations,
  // and every outer step but the last takes at least one of the maxit inner
  // iterations, so at most 2 maxit + 4 (maxit + 1) passes, plus the final
  // RESID and REF_SCALE.
  // Preconditioned: classic runs three passes per iteration (K_CHEB, K_CG1,
  // K_CG2), the pipelined variant two (K_CHEBW, K_PPCG); the refinement's
  // inner solve three (K_CHEBF, K_CG1F, K_CG2F), ended by K_CHEBF (or by the
  // K_CG1F after it), i.e. 3 K + 5 passes with the outer ones, at most
  // 3 maxit + 5 (maxit + 1) plus the final RESID and REF_SCALE.
  static int64_t step_bound(const cg_problem& p, bool refined, int precond) {
    const int64_t m = p.maxit;
    // residual replacement adds four passes per rr_period iterations
    const int64_t rr = p.rr_period > 0 ? 4 * (m / p.rr_period + 1) : 0;
    return (refined ? (precond ? 8 * m + 32 : 6 * m + 32) : precond ? 3 * m + 32 : 2 * m + 32) + rr;
  }

  // Chebyshev items of one pass of a preconditioned solve (as k_cheb and
  // k_chebf number them: groups of kChebGroupCols columns of the padded row
  // by cheb_rows rows)
  static int cheb_items_of(const Plan& pl) {
    const int ngx = (pl.width + kChebGroupCols - 1) / kChebGroupCols;
    const int nty = (pl.g.ny + pl.cheb_rows - 1) / pl.cheb_rows;
    return ngx * nty;
  }

  // Rebuilds the item table: each resident solve contributes up to
  // kMaxItemsPerSolve items of consecutive tiles.
  int upload_items() {
    int n = 0;
    for (int i = 0; i < n_; ++i) {
      Job* j = slot_job_[i];
      if (!j || j->w.pl.on_side()) continue;
      const int T = j->w.pl.g.tiles;
      const int per = (T + kMaxItemsPerSolve - 1) / kMaxItemsPerSolve;
      for (int t = 0; t < T; t += per) h_items_[n++] = Item{i, t, std::min(T, t + per), 0};
    }
    int* nn = (int*)(h_items_ + max_items_);
    *nn = n;
    // a preconditioned pipelined solve: its tile passes run in k_step_ppcg
    // (bit 0 of the mask); a 3D or variable-coefficient solve: its passes run
    // in k_step_op (bits kOpBit and kOpBit + 1)
    for (int i = 0; i < n_; ++i) {
      Job* j = slot_job_[i];
      if (!j || j->w.pl.on_side()) continue;
      if (j->w.pl.precond && !j->w.pl.refined && j->w.pl.variant == CG_VARIANT_PIPELINED)
        cheb_mask_ |= 1u;
      if (j->w.pl.g.plane > 0) cheb_mask_ |= 1u << kOpBit;
      if (j->w.pl.vc) cheb_mask_ |= 1u << (kOpBit + 1);
    }
    // Chebyshev items, grouped by s (each group's count and offset in cinfo)
    int nc = 0;
    int* cinfo = (int*)(h_citems_ + max_items_);
    for (int sd = 0; sd <= kChebMaxSteps; ++sd) {
      cinfo[2 * sd] = 0;
      cinfo[2 * sd + 1] = nc;
      if (sd == 0) continue;
      for (int i = 0; i < n_; ++i) {
        Job* j = slot_job_[i];
        if (!j || j->w.pl.on_side() || j->w.pl.precond != sd) continue;
        const int I = cheb_items_of(j->w.pl);
        const int per = (I + kMaxItemsPerSolve - 1) / kMaxItemsPerSolve;
        for (int t = 0; t < I; t += per) h_citems_[nc++] = Item{i, t, std::min(I, t + per), 0};
      }
      cinfo[2 * sd] = nc - cinfo[2 * sd + 1];
      // bit s: an FP64 solve with s steps, bit 8 + s: a refined one
      for (int i = 0; i < n_; ++i) {
        Job* j = slot_job_[i];
        if (!j || j->w.pl.on_side() || j->w.pl.precond != sd) continue;
        cheb_mask_ |= 1u << (j->w.pl.refined ? kChebMaxSteps + sd : sd);
      }
    }
    if (hipMemcpyAsync(d_items_, h_items_, (size_t)std::max(n, 1) * sizeof(Item),
                       hipMemcpyHostToDevice, c_.st) ||
        hipMemcpyAsync(d_nitems_, nn, sizeof(int), hipMemcpyHostToDevice, c_.st) ||
        (nc && hipMemcpyAsync(d_citems_, h_citems_, (size_t)nc * sizeof(Item),
                              hipMemcpyHostToDevice, c_.st)) ||
        hipMemcpyAsync(d_cinfo_, cinfo, 2 * (kChebMaxSteps + 1) * sizeof(int),
                       hipMemcpyHostToDevice, c_.st) ||
        hipStreamSynchronize(c_.st))
      return CG_E_DEVICE;
    dirty_ = false;
    return CG_OK;
  }

  // One step: the step kernel, the preconditioned pipelined passes' step
  // kernel once such a solve has been admitted, then the Chebyshev step
  // kernel of every s that a preconditioned solve of this engine has used
  // (each kernel skips the solves at passes of the others; an s with no solve
  // resident has no items).
  hipError_t launch_one_step(int k) {
    hipError_t e = launch_step(d_slots_, d_items_, d_nitems_, d_step_, k, grid_, c_.st);
    if (e == hipSuccess && (cheb_mask_ & 1u))
      e = launch_step_ppcg(d_slots_, d_items_, d_nitems_, d_step_, k,
                           std::max(8, step_ppcg_max_blocks_per_cu() * c_.num_cu), c_.st);
    for (int op = 1; op <= 2 && e == hipSuccess; ++op)
      if (cheb_mask_ & (1u << (kOpBit + op - 1)))
        e = launch_step_op(op, d_slots_, d_items_, d_nitems_, d_step_, k,
                           std::max(8, step_op_max_blocks_per_cu(op) * c_.num_cu), c_.st);
    for (int sd = 1; sd <= kChebMaxSteps && e == hipSuccess; ++sd)
      for (int f32 = 0; f32 < 2 && e == hipSuccess; ++f32)
        if (cheb_mask_ & (1u << (f32 ? kChebMaxSteps + sd : sd)))
          e = launch_step_cheb(sd, f32, d_slots_, d_citems_, d_cinfo_, d_step_, k,
                               std::max(8, cheb_max_blocks_per_cu(sd, f32) * c_.num_cu), c_.st);
    return e;
  }

  static constexpr int kStepRing = 64;
  Ctx& c_;
  int n_;
  int max_items_ = 0;
  int* d_step_ = nullptr;
  int* h_step_ = nullptr;
  unsigned ring_ = 0;
  hipGraphExec_t graph_ = nullptr;
  int graph_steps_ = 0;

 public:
  bool this_is_serving_ = false;

 private:
  char* ctrl_ = nullptr;
  Slot* d_slots_ = nullptr;
  Item* d_items_ = nullptr;
  int* d_idx_ = nullptr;
  int* d_nitems_ = nullptr;
  State* d_states_ = nullptr;
  Slot* h_slots_ = nullptr;
  State* h_admit_ = nullptr;  // initial state of each slot's solve (pinned)
  static constexpr int kCoefPerSlot = 16;
  double* h_coef_ = nullptr;  // Chebyshev coefficients of each slot's solve (pinned)
  Item* h_citems_ = nullptr;  // Chebyshev items, then cinfo (pinned)
  Item* d_citems_ = nullptr;
  int* d_cinfo_ = nullptr;
  unsigned cheb_mask_ = 0;    // bit s (8 + s): Chebyshev steps s that any admitted FP64
                              // (refined) solve has used; bit 0: a preconditioned
                              // pipelined solve was admitted; bits kOpBit, kOpBit + 1:
                              // a 3D, a variable-coefficient solve was admitted
  static constexpr int kOpBit = 2 * kChebMaxSteps + 1;
  unsigned graph_mask_ = 0;   // ... when the cached chunk was captured
  Item* h_items_ = nullptr;
  int* h_idx_ = nullptr;
  State* h_states_ = nullptr;
  std::vector<Job*> slot_job_;
  std::vector<int> rr_new_;  // slots of register-resident solves not yet launched
  std::vector<int> fx_new_;  // slots of fixed-point solves not yet launched
  std::vector<int> fx_key_;  // their launch keys: unknowns per thread * 2 + variant
  int* d_rr_idx_ = nullptr;
  int* h_rr_idx_ = nullptr;
  hipEvent_t rr_ev_ = nullptr, stage_ev_ = nullptr;
  bool rr_pending_ = false;  // launched, not yet joined by a harvest
  int step_jobs_ = 0;        // resident solves that take step items
  int active_ = 0;
  int grid_ = 8;
  int step_ = 0;
  bool dirty_ = true;
};

static int worse(int a, int b) {
  if (a < 0 || b < 0) return std::min(a, b);
  auto rank = [](int s) { return s == CG_BREAKDOWN ? 3 : s == CG_NOT_CONVERGED ? 2 : 0; };
  return rank(a) >= rank(b) ? a : b;
}

int Ctx::solve_batch(const cg_problem* probs, int n, cg_result* results) {
  for (int i = 0; i < n; ++i)
    if (plan(&probs[i]).footprint + engine_bytes() > arena.size())
      return CG_E_NOMEM;
  int rc = order_after_user();
  if (rc) return rc;
  Engine eng(*this, std::min(n, max_slots));
  const int chunk = step_chunk;
  if ((rc = eng.init())) return rc;
  std::vector<Job> jobs(n);
  std::deque<int> pending;
  for (int i = 0; i < n; ++i) {
    jobs[i].p = probs[i];
    jobs[i].t_submit = now_s();
    pending.push_back(i);
  }
  std::vector<Job*> done;
  int worst = CG_OK;
  while (!pending.empty() || eng.active() > 0) {
    while (!pending.empty() && eng.has_free()) {
      int a = eng.admit(&jobs[pending.front()]);
      if (a == CG_E_NOMEM && eng.active() > 0) break;  // wait for memory to free up
      if (a != CG_OK) {
        std::vector<Job*> tmp;
        eng.abandon(tmp, a);
        return a;
      }
      pending.pop_front();
    }
    if ((rc = eng.run(chunk)) || (rc = eng.harvest(done))) {
      eng.abandon(done, rc);
      return rc;
    }
  }
  for (int i = 0; i < n; ++i) {
    results[i] = jobs[i].res;
    results[i].latency_seconds = jobs[i].t_done - jobs[i].t_submit;
    worst = worse(worst, jobs[i].rc);
  }
  return worst;
}

// ---------------------------------------------------------------- server --

class Server {
 public:
  explicit Server(Ctx& c) : c_(c) {}
  ~Server() { stop(); }

  int submit(const cg_problem* p, uint64_t* ticket) {
    if (footprint_of(p) + c_.engine_bytes() > c_.arena.size())
      return CG_E_NOMEM;
    Job* j = new Job;
    j->p = *p;
    j->t_submit = now_s();
    // the inputs may still be in flight on the caller's stream (the null
    // stream when the context names none): remember where it stands now
    if (hipSetDevice(c_.device) != hipSuccess ||
        hipEventCreateWithFlags(&j->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(j->ready, c_.user_stream) != hipSuccess) {
      delete j;
      return CG_E_DEVICE;
    }
    {
      std::lock_guard<std::mutex> lk(m_);
      if (stopping_) {
        delete j;
        return CG_E_BUSY;
      }
      j->ticket = next_ticket_++;
      jobs_[j->ticket] = j;
      queue_.push_back(j);
      if (!th_.joinable()) th_ = std::thread([this] { loop(); });
    }
    cv_.notify_one();
    *ticket = j->ticket;
    return CG_OK;
  }

  int poll(uint64_t t, cg_result* r) {
    std::lock_guard<std::mutex> lk(m_);
    auto it = jobs_.find(t);
    if (it == jobs_.end()) return CG_E_TICKET;
    Job* j = it->second;
    if (!j->finished) return CG_PENDING;
    *r = j->res;
    r->latency_seconds = j->t_done - j->t_submit;
    const int rc = j->rc;
    jobs_.erase(it);
    delete j;
    return rc;
  }

  void stop() {
    {
      std::lock_guard<std::mutex> lk(m_);
      stopping_ = true;
    }
    cv_.notify_all();
    if (th_.joinable()) th_.join();
    std::lock_guard<std::mutex> lk(m_);
    for (auto& kv : jobs_) delete kv.second;
    jobs_.clear();
    queue_.clear();
  }

 private:
  void loop() {
    std::unique_ptr<Engine> eng;
    std::vector<Job*> done;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] {
          return stopping_ || !queue_.empty() || (eng && eng->active() > 0);
        });
        if (stopping_ && (!eng || eng->active() == 0)) {
          for (Job* j : queue_) {  // cancelled before admission
            j->rc = CG_E_BUSY;
            j->finished = true;
            j->t_done = now_s();
          }
          queue_.clear();
          break;
        }
      }
      done.clear();
      {
        std::lock_guard<std::recursive_mutex> ck(c_.mu);
        if (hipSetDevice(c_.device) != hipSuccess) break;
        int rc = CG_OK;
        if (!eng) {
          eng.reset(new Engine(c_, c_.max_slots));
          eng->this_is_serving_ = true;
          rc = eng->init();
        }
        // admission: FIFO while a slot is free and the footprint fits
        while (rc == CG_OK) {
          Job* j = nullptr;
          {
            std::lock_guard<std::mutex> lk(m_);
            if (stopping_ || queue_.empty() || !eng->has_free()) break;
            j = queue_.front();
          }
          const int a = eng->admit(j);
          if (a == CG_E_NOMEM && eng->active() > 0) break;
          std::lock_guard<std::mutex> lk(m_);
          queue_.pop_front();
          if (a != CG_OK) {
            j->rc = a;
            j->finished = true;
            j->t_done = now_s();
          }
        }
        if (rc == CG_OK) rc = eng->run(c_.serve_chunk);
        if (rc == CG_OK) rc = eng->harvest(done);
        if (rc != CG_OK) eng->abandon(done, rc);
      }
      {
        std::lock_guard<std::mutex> lk(m_);
        for (Job* j : done) j->finished = true;
      }
    }
    if (eng) {
      std::lock_guard<std::recursive_mutex> ck(c_.mu);
      eng.reset();
    }
  }

  Ctx& c_;
  std::thread th_;
  std::mutex m_;
  std::condition_variable cv_;
  std::deque<Job*> queue_;
  std::unordered_map<uint64_t, Job*> jobs_;
  bool stopping_ = false;
  uint64_t next_ticket_ = 1;
};

}  // namespace cgr

using cgr::Ctx;
using cgr::Server;

int cgr_server_submit(Ctx* c, const cg_problem* p, uint64_t* ticket) {
  Server* s;
  {
    std::lock_guard<std::mutex> lk(c->server_mu);
    if (!c->server) c->server = new Server(*c);
    s = c->server;
  }
  return s->submit(p, ticket);
}

int cgr_server_poll(Ctx* c, uint64_t ticket, cg_result* res) {
  Server* s;
  {
    std::lock_guard<std::mutex> lk(c->server_mu);
    s = c->server;
  }
  if (!s) return CG_E_TICKET;
  return s->poll(ticket, res);
}

void cgr_server_stop(Ctx* c) {
  Server* s;
  {
    std::lock_guard<std::mutex> lk(c->server_mu);
    s = c->server;
    c->server = nullptr;
  }
  delete s;
}
