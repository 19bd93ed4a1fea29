// cg_serve.cpp - batched persistent solves and the serving loop.
#include "cg_runtime.h"

namespace cgr {
int Ctx::solve_batch(const cg_problem*, int, cg_result*) { return CG_E_DEVICE; }
}  // namespace cgr

int cgr_server_submit(cgr::Ctx*, const cg_problem*, uint64_t*) { return CG_E_DEVICE; }
int cgr_server_poll(cgr::Ctx*, uint64_t, cg_result*) { return CG_E_TICKET; }
void cgr_server_stop(cgr::Ctx*) {}
