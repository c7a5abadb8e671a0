// Batched products (pm_poly_mul_batch).
#include "internal.h"

namespace pm {
bool plan_valid(const Plan& P, long lc, int pidx);
Plan choose_plan(long lc, int pidx);
size_t plan_workspace_bytes(const Plan& P);
pm_status run_product(DevCtx* c, const Plan& P, const void* a, long la, const void* b, long lb, int in_type, u32* out,
                      long lc, int pidx, void* ws, hipStream_t s);
}  // namespace pm

using namespace pm;

extern "C" pm_status pm_poly_mul_batch(const pm_problem* probs, size_t count, void* stream) {
  if (!probs && count) return PM_EINVAL;
  std::vector<Plan> plans(count);
  std::vector<int> pidx(count);
  size_t wsb = 0;
  for (size_t i = 0; i < count; ++i) {
    const pm_problem& q = probs[i];
    if (!q.a || !q.b || !q.c || q.len_a == 0 || q.len_b == 0) return PM_EINVAL;
    pidx[i] = prime_index(q.p);
    if (pidx[i] < 0) return PM_EUNSUPPORTED;
    const long lc = (long)(q.len_a + q.len_b - 1);
    plans[i] = choose_plan(lc, pidx[i]);
    if (!plan_valid(plans[i], lc, pidx[i])) return PM_ETOOLARGE;
    const size_t w = plan_workspace_bytes(plans[i]);
    if (w > wsb) wsb = w;
  }
  pm_status st;
  DevCtx* c = ctx_current(&st);
  if (!c) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  if (wsb) {
    st = ensure_workspace(c, wsb);
    if (st) return st;
  }
  for (size_t i = 0; i < count; ++i) {
    const pm_problem& q = probs[i];
    st = run_product(c, plans[i], q.a, (long)q.len_a, q.b, (long)q.len_b, 0, q.c, (long)(q.len_a + q.len_b - 1),
                     pidx[i], c->ws, (hipStream_t)stream);
    if (st) return st;
  }
  return PM_OK;
}
