// Batched solves / serving engine - placeholder.
#include "krylov.h"

extern "C" {
rt_status rt_batch_create(int, int64_t, int, int, rt_batch* out) {
  if (out) *out = nullptr;
  return RT_E_INVALID;
}
rt_status rt_batch_submit(rt_batch, rt_problem, const rt_solver_opts*, double*, uint64_t*) {
  return RT_E_INVALID;
}
rt_status rt_batch_step(rt_batch, int*) { return RT_E_INVALID; }
rt_status rt_batch_poll(rt_batch, uint64_t, rt_solve_stats*) { return RT_E_INVALID; }
rt_status rt_batch_wait_all(rt_batch) { return RT_E_INVALID; }
rt_status rt_batch_destroy(rt_batch) { return RT_E_INVALID; }
}
