// The empirical autotuner and the learned plan policy.
//
// The tuner times every candidate plan of an output length on the device
// (hipEvents, median of repeated runs) and records (length, prime, plan,
// time) rows in the timing database; the fastest plan goes to the plan
// cache.  This is the library's counterpart of the paper's search that
// measures the running time of candidate implementations and keeps the best
// (section 2.2; section 5, autotuned library).  The cost model is trained
// on those rows (mlp.hip) and predicts, for lengths never timed, the log
// running time of every candidate; the learned policy takes the argmin.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include <map>

#include "internal.h"
#include "mlp.h"

namespace pm {
bool plan_valid(const Plan& P, long lc, int pidx);
size_t plan_workspace_bytes(const Plan& P);
pm_status run_product(DevCtx* c, const Plan& P, const void* a, long la, const void* b, long lb, int in_type, u32* out,
                      long lc, int pidx, void* ws, hipStream_t s);
Plan default_plan(long lc, int pidx);
void plan_epoch_bump();

struct DbRow {
  long lc;
  u32 p;
  Plan plan;
  double us;
  int tctx = kCtxSingle;  // timed alone (latency) or in a batch (time per product)
};
static std::mutex g_db_mu;
static std::vector<DbRow> g_db;

// ---------------------------------------------------------------------------
// features of (length, prime, plan) for the cost model

void plan_features(long lc, int pidx, const Plan& P, int tctx, float* f) {
  const double nprime = P.kind == PLAN_DIRECT ? (double)lc : (double)plan_nprime(P);
  const double L = P.kind == PLAN_DIRECT ? (double)lc : (double)(1l << P.logL);
  const int rows = P.kind == PLAN_FOURSTEP ? (P.ma << P.logRB) : P.ma;
  f[0] = (float)(std::log2((double)lc) / 24.0);
  f[1] = (float)(std::log2(L) / 24.0);
  f[2] = (float)(nprime / L);
  f[3] = (float)((double)lc / nprime);
  f[4] = P.kind == PLAN_LDS ? 1.f : 0.f;
  f[5] = P.kind == PLAN_FOURSTEP ? 1.f : 0.f;
  f[6] = (float)P.logRA / 5.f;
  f[7] = (float)P.logRB / 5.f;
  f[8] = (float)P.logC / 14.f;
  f[9] = (float)P.lq / 4.f;
  f[10] = P.kind == PLAN_FOURSTEP ? (float)plan_row_lnt(P) / 10.f : 0.f;
  f[11] = prime_info(pidx).lazy ? 1.f : 0.f;
  f[12] = (float)(std::log2((double)std::max(rows, 1)) / 10.0);
  // values per row thread (log2): the row pass's register/occupancy trade-off
  f[13] = P.kind == PLAN_FOURSTEP ? (float)(P.logC - plan_row_lnt(P)) / 5.f : 0.f;
  f[14] = P.kind == PLAN_FOURSTEP ? (float)(P.logL - P.logC) / 10.f : 0.f;
  f[15] = P.kind == PLAN_DIRECT ? 0.f : (float)P.ma / (float)(1 << P.logRA);
  // the context: a product alone is bound by its own parallelism, one of a
  // batch by its work and traffic
  f[16] = tctx == kCtxBatch ? 1.f : 0.f;
}

static double plan_nprime_d(long lc, const Plan& P) {
  return P.kind == PLAN_DIRECT ? (double)lc : (double)plan_nprime(P);
}

// ---------------------------------------------------------------------------
// timing

// deterministic filler (input values do not change the running time)
__global__ void k_fill_mod(u32* x, long n, u32 p, u32 seed) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  u32 h = (u32)i * 0x9E3779B1u ^ seed;
  h ^= h >> 15;
  h *= 0x85EBCA77u;
  h ^= h >> 13;
  x[i] = h % p;
}

struct TuneBufs {
  u32 *a = nullptr, *b = nullptr, *c = nullptr;
  long la = 0, lb = 0;
  ~TuneBufs() {
    if (a) hipFree(a);
    if (b) hipFree(b);
    if (c) hipFree(c);
  }
};

static pm_status tune_inputs(long lc, u32 p, TuneBufs* T, hipStream_t s) {
  T->la = (lc + 2) / 2;
  T->lb = lc + 1 - T->la;
  if (hipMalloc(&T->a, T->la * 4) || hipMalloc(&T->b, T->lb * 4) || hipMalloc(&T->c, lc * 4)) return PM_ENOMEM;
  k_fill_mod<<<(unsigned)((T->la + 255) / 256), 256, 0, s>>>(T->a, T->la, p, 1);
  k_fill_mod<<<(unsigned)((T->lb + 255) / 256), 256, 0, s>>>(T->b, T->lb, p, 2);
  return hipGetLastError() == hipSuccess ? PM_OK : PM_EDEVICE;
}

// median time in microseconds of `reps` runs of plan P (after one warm-up)
static pm_status time_plan(DevCtx* c, const Plan& P, long lc, int pidx, const TuneBufs& B, int reps, hipStream_t s,
                           double* us) {
  const size_t wsb = plan_workspace_bytes(P);
  void* ws = nullptr;
  if (wsb) {
    pm_status st = stream_workspace(c, s, wsb, &ws);
    if (st) return st;
  }
  pm_status st = run_product(c, P, B.a, B.la, B.b, B.lb, 0, B.c, lc, pidx, ws, s);
  if (st) return st;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) || hipEventCreate(&e1)) return PM_EDEVICE;
  std::vector<float> t;
  for (int r = 0; r < reps && st == PM_OK; ++r) {
    hipEventRecord(e0, s);
    st = run_product(c, P, B.a, B.la, B.b, B.lb, 0, B.c, lc, pidx, ws, s);
    hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) st = PM_EDEVICE;
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    t.push_back(ms);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st) return st;
  std::sort(t.begin(), t.end());
  *us = 1e3 * (t.size() % 2 ? t[t.size() / 2] : 0.5 * (t[t.size() / 2 - 1] + t[t.size() / 2]));
  return PM_OK;
}

// Batch context: `count` independent products of length lc (distinct
// operands, outputs and workspaces), every pass one launch over all of them as
// the batch executor runs a class, with count * L about 2^24: enough products
// to keep the device full whatever the plan, as the other classes of a batch
// do, so that the time per product measures throughput, not latency.
struct BatchBufs {
  int count = 0;
  long la = 0, lb = 0, lc = 0;
  u32 *a = nullptr, *b = nullptr, *c = nullptr, *ws = nullptr;
  ConvJob* jobs = nullptr;
  ~BatchBufs() {
    for (void* q : {(void*)a, (void*)b, (void*)c, (void*)ws, (void*)jobs})
      if (q) hipFree(q);
  }
};

static int batch_count(long lc) {
  long L = 1;
  while (L < lc) L <<= 1;
  const long n = (1l << 24) / L;
  return (int)(n < 1 ? 1 : (n > 4096 ? 4096 : n));
}

static pm_status batch_inputs(long lc, u32 p, BatchBufs* T, hipStream_t s) {
  T->count = batch_count(lc);
  T->lc = lc;
  T->la = (lc + 2) / 2;
  T->lb = lc + 1 - T->la;
  long L = 1;
  while (L < lc) L <<= 1;
  const size_t n = (size_t)T->count;
  if (hipMalloc(&T->a, n * T->la * 4) || hipMalloc(&T->b, n * T->lb * 4) || hipMalloc(&T->c, n * lc * 4) ||
      hipMalloc(&T->ws, n * 2 * (size_t)L * 4) || hipMalloc(&T->jobs, n * sizeof(ConvJob)))
    return PM_ENOMEM;
  const long na = (long)n * T->la, nb = (long)n * T->lb;
  k_fill_mod<<<(unsigned)((na + 255) / 256), 256, 0, s>>>(T->a, na, p, 1);
  k_fill_mod<<<(unsigned)((nb + 255) / 256), 256, 0, s>>>(T->b, nb, p, 2);
  return hipGetLastError() == hipSuccess ? PM_OK : PM_EDEVICE;
}

pm_status launch_class(const Plan& P, bool lazy, int in_type, const JobRef& jr, int njobs, int max_rows,
                       hipStream_t s);

// median time per product in microseconds of `reps` batch runs of plan P
static pm_status time_plan_batch(DevCtx* c, const Plan& P, int pidx, const BatchBufs& B, int reps, hipStream_t s,
                                 double* us) {
  if (P.kind == PLAN_DIRECT) {  // the executor launches these one by one
    std::vector<float> t;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) || hipEventCreate(&e1)) return PM_EDEVICE;
    pm_status st = PM_OK;
    for (int r = 0; r <= reps && st == PM_OK; ++r) {
      hipEventRecord(e0, s);
      for (int k = 0; k < B.count && st == PM_OK; ++k)
        st = run_product(c, P, B.a + (long)k * B.la, B.la, B.b + (long)k * B.lb, B.lb, 0, B.c + (long)k * B.lc, B.lc,
                         pidx, nullptr, s);
      hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) st = PM_EDEVICE;
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      if (r) t.push_back(ms);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st) return st;
    std::sort(t.begin(), t.end());
    *us = 1e3 * t[t.size() / 2] / B.count;
    return PM_OK;
  }
  const long np = plan_nprime(P);
  std::vector<ConvJob> jobs(B.count);
  int max_rows = 0;
  for (int k = 0; k < B.count; ++k) {
    u32* Ta = P.kind == PLAN_FOURSTEP ? B.ws + (size_t)k * 2 * np : nullptr;
    u32* Tb = Ta ? Ta + np : nullptr;
    pm_status st = make_job(c, P, pidx, B.a + (long)k * B.la, B.la, B.b + (long)k * B.lb, B.lb, B.c + (long)k * B.lc,
                            B.lc, Ta, Tb, &jobs[k], 0);
    if (st) return st;
    max_rows = std::max(max_rows, jobs[k].rows);
  }
  if (hipMemcpyAsync(B.jobs, jobs.data(), jobs.size() * sizeof(ConvJob), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return PM_EDEVICE;
  JobRef jr;
  jr.one = jobs[0];
  jr.many = B.jobs;
  const bool lazy = prime_info(pidx).lazy;
  pm_status st = launch_class(P, lazy, 0, jr, B.count, max_rows, s);
  if (st) return st;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) || hipEventCreate(&e1)) return PM_EDEVICE;
  std::vector<float> t;
  for (int r = 0; r < reps && st == PM_OK; ++r) {
    hipEventRecord(e0, s);
    st = launch_class(P, lazy, 0, jr, B.count, max_rows, s);
    hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) st = PM_EDEVICE;
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    t.push_back(ms);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st) return st;
  std::sort(t.begin(), t.end());
  *us = 1e3 * (t.size() % 2 ? t[t.size() / 2] : 0.5 * (t[t.size() / 2 - 1] + t[t.size() / 2])) / B.count;
  return PM_OK;
}

// Time every candidate of one length in context tctx, record the rows, cache
// the best.  The caller holds the device lock.
pm_status tune_one(DevCtx* c, long lc, int pidx, int reps, hipStream_t s, Plan* best_out, int tctx) {
  const u32 p = prime_info(pidx).p;
  TuneBufs B;
  BatchBufs BB;
  pm_status st = tctx == kCtxBatch ? batch_inputs(lc, p, &BB, s) : tune_inputs(lc, p, &B, s);
  if (st) return st;
  // the general-radix plans for products alone (the batch executor does not run them)
  std::vector<Plan> cands = plan_candidates(lc, pidx, tctx == kCtxSingle);
  double best = 1e300;
  Plan bestP = default_plan(lc, pidx);
  for (const Plan& P : cands) {
    double us = 0;
    st = tctx == kCtxBatch ? time_plan_batch(c, P, pidx, BB, reps, s, &us) : time_plan(c, P, lc, pidx, B, reps, s, &us);
    if (st) return st;
    {
      std::lock_guard<std::mutex> lk(g_db_mu);
      g_db.push_back(DbRow{lc, p, P, us, tctx});
    }
    if (us < best) {
      best = us;
      bestP = P;
    }
  }
  plan_cache_set(lc, p, bestP, tctx);
  if (best_out) *best_out = bestP;
  return PM_OK;
}

// ---------------------------------------------------------------------------
// the trained model (host copy of the weights and the target normalisation)

struct Model {
  bool ok = false;
  std::vector<float> w;
  float mean = 0.f, std = 1.f;
  unsigned long ver = 0;  // changes with every new set of weights
};
static std::mutex g_model_mu;
static Model g_model;
static unsigned long g_model_ver = 0;  // guarded by g_model_mu

// the network on the current device's preallocated inference buffers
static pm_status infer_rows(const Model& M, const float* X, int B, float* y) {
  pm_status st;
  DevCtx* c = ctx_current(&st);
  if (!c) return st;
  return mlp_infer(&c->infer, M.w.data(), M.ver, X, B, y);
}

// predicted log(us) of each plan for (lc, pidx); the caller holds no locks
static pm_status model_predict(long lc, int pidx, const std::vector<Plan>& plans, int tctx, std::vector<double>* out) {
  Model M;
  {
    std::lock_guard<std::mutex> lk(g_model_mu);
    if (!g_model.ok) return PM_EINVAL;
    M = g_model;
  }
  const int B = (int)plans.size();
  std::vector<float> X((size_t)B * kMlpF), y(B);
  for (int i = 0; i < B; ++i) plan_features(lc, pidx, plans[i], tctx, &X[(size_t)i * kMlpF]);
  pm_status st = infer_rows(M, X.data(), B, y.data());
  if (st) return st;
  out->resize(B);
  for (int i = 0; i < B; ++i) (*out)[i] = (double)y[i] * M.std + M.mean + std::log(plan_nprime_d(lc, plans[i]));
  return PM_OK;
}

Plan learned_plan(long lc, int pidx, bool* ok, int tctx) {
  *ok = false;
  std::vector<Plan> cands = plan_candidates(lc, pidx);
  std::vector<double> pred;
  if (cands.empty() || model_predict(lc, pidx, cands, tctx, &pred) != PM_OK) return Plan();
  size_t bi = 0;
  for (size_t i = 1; i < cands.size(); ++i)
    if (pred[i] < pred[bi]) bi = i;
  *ok = true;
  return cands[bi];
}

// Plans for the products of one batch, chosen per size class: the items of
// one transform length L and prime share one plan family (every plan
// parameter but the kept blocks ma, which follow each item's length), the one
// whose predicted times, summed over the items, are least.  Chosen item by
// item, neighbouring lengths scatter over many plan variants, and the
// executor would launch each variant as a class of its own.
pm_status learned_batch_plans(const std::vector<long>& lcs, const std::vector<int>& pidx, std::vector<Plan>* out) {
  Model M;
  {
    std::lock_guard<std::mutex> lk(g_model_mu);
    if (!g_model.ok) return PM_EINVAL;
    M = g_model;
  }
  out->assign(lcs.size(), Plan());
  std::map<std::pair<int, int>, std::vector<size_t>> groups;  // (log L, prime) -> items
  for (size_t i = 0; i < lcs.size(); ++i) {
    if (lcs[i] <= 64) continue;
    int l = 0;
    while ((1l << l) < lcs[i]) ++l;
    groups[std::make_pair(l, pidx[i])].push_back(i);
  }
  for (auto& g : groups) {
    const std::vector<size_t>& items = g.second;
    const int pid = g.first.second;
    // families from the candidates of the longest item (its kept blocks are
    // the most, so every family valid for it is valid for the others); each
    // shape both untruncated and truncated to each item's own kept blocks,
    // also where the longest item keeps every block and so has no truncated
    // candidate of its own
    size_t rep = items[0];
    for (size_t i : items)
      if (lcs[i] > lcs[rep]) rep = i;
    std::vector<Plan> fams;
    for (const Plan& P : plan_candidates(lcs[rep], pid)) {
      for (int fm = 0; fm >= -1; --fm) {
        Plan F = P;
        F.ma = fm;  // 0: all blocks kept, -1: the item's own kept blocks
        bool dup = false;
        for (const Plan& Q : fams)
          dup |= Q.kind == F.kind && Q.logRA == F.logRA && Q.logRB == F.logRB && Q.logC == F.logC &&
                 Q.lq == F.lq && Q.lnt == F.lnt && Q.ma == F.ma;
        if (!dup) fams.push_back(F);
      }
    }
    auto item_plan = [&](const Plan& F, long lc) {
      Plan P = F;
      const long gran = 1l << (P.logL - P.logRA);
      P.ma = F.ma == 0 ? (1 << P.logRA) : (int)((lc + gran - 1) / gran);
      return P;
    };
    const size_t nf = fams.size(), B = items.size() * nf;
    std::vector<float> X(B * kMlpF), y(B);
    for (size_t k = 0; k < items.size(); ++k)
      for (size_t f = 0; f < nf; ++f)
        plan_features(lcs[items[k]], pid, item_plan(fams[f], lcs[items[k]]), kCtxBatch, &X[(k * nf + f) * kMlpF]);
    pm_status st = infer_rows(M, X.data(), (int)B, y.data());
    if (st) return st;
    std::vector<double> total(nf, 0.0);
    for (size_t k = 0; k < items.size(); ++k)
      for (size_t f = 0; f < nf; ++f) {
        const Plan P = item_plan(fams[f], lcs[items[k]]);
        total[f] += std::exp((double)y[k * nf + f] * M.std + M.mean) * plan_nprime_d(lcs[items[k]], P);
      }
    size_t bf = 0;
    for (size_t f = 1; f < nf; ++f)
      if (total[f] < total[bf]) bf = f;
    for (size_t i : items) (*out)[i] = item_plan(fams[bf], lcs[i]);
  }
  return PM_OK;
}

// SplitMix64 (Steele, Lea, Flood 2014): the initial weights when none are given
static u64 splitmix64(u64& s) {
  u64 z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace pm

using namespace pm;

extern "C" {

pm_status pm_tune(const size_t* lcs, size_t n, uint32_t p, int reps, void* stream) {
  return pm_tune_ctx(lcs, n, p, reps, PM_CTX_SINGLE, stream);
}

pm_status pm_tune_ctx(const size_t* lcs, size_t n, uint32_t p, int reps, int context, void* stream) {
  if (!lcs || reps < 1 || (context != PM_CTX_SINGLE && context != PM_CTX_BATCH)) return PM_EINVAL;
  const int pidx = prime_index(p);
  if (pidx < 0) return PM_EUNSUPPORTED;
  for (size_t i = 0; i < n; ++i) {
    if (lcs[i] == 0) return PM_EINVAL;
    int l = 0;
    while ((1ul << l) < lcs[i]) ++l;
    if (lcs[i] > 64 && (l > prime_info(pidx).two_adic || l > 24)) return PM_ETOOLARGE;
  }
  pm_status st;
  DevCtx* c = ctx_current(&st);
  if (!c) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  for (size_t i = 0; i < n; ++i) {
    st = tune_one(c, (long)lcs[i], pidx, reps, (hipStream_t)stream, nullptr, context);
    if (st) return st;
  }
  return PM_OK;
}

pm_status pm_time_plan(size_t lc, uint32_t p, const pm_plan* plan, int reps, double* us) {
  return pm_time_plan_ctx(lc, p, plan, reps, PM_CTX_SINGLE, us);
}

pm_status pm_time_plan_ctx(size_t lc, uint32_t p, const pm_plan* plan, int reps, int context, double* us) {
  if (!plan || !us || lc == 0 || reps < 1 || (context != PM_CTX_SINGLE && context != PM_CTX_BATCH))
    return PM_EINVAL;
  const int pidx = prime_index(p);
  if (pidx < 0) return PM_EUNSUPPORTED;
  Plan P = plan_from_pub(*plan);
  if (!plan_valid(P, (long)lc, pidx) || (P.kind == PLAN_MIXED && context == PM_CTX_BATCH)) return PM_EINVAL;
  pm_status st;
  DevCtx* c = ctx_current(&st);
  if (!c) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  if (context == PM_CTX_BATCH) {
    BatchBufs BB;
    st = batch_inputs((long)lc, p, &BB, 0);
    if (st) return st;
    return time_plan_batch(c, P, pidx, BB, reps, 0, us);
  }
  TuneBufs B;
  st = tune_inputs((long)lc, p, &B, 0);
  if (st) return st;
  return time_plan(c, P, (long)lc, pidx, B, reps, 0, us);
}

size_t pm_tune_db_size(void) {
  std::lock_guard<std::mutex> lk(g_db_mu);
  return g_db.size();
}

pm_status pm_tune_db_get(size_t i, size_t* lc, uint32_t* p, pm_plan* plan, double* us, int* context) {
  std::lock_guard<std::mutex> lk(g_db_mu);
  if (i >= g_db.size()) return PM_EINVAL;
  if (lc) *lc = (size_t)g_db[i].lc;
  if (p) *p = g_db[i].p;
  if (plan) *plan = plan_to_pub(g_db[i].plan);
  if (us) *us = g_db[i].us;
  if (context) *context = g_db[i].tctx;
  return PM_OK;
}

pm_status pm_tune_db_add(size_t lc, uint32_t p, const pm_plan* plan, double us, int context) {
  if (!plan || lc == 0 || (context != PM_CTX_SINGLE && context != PM_CTX_BATCH)) return PM_EINVAL;
  if (prime_index(p) < 0) return PM_EUNSUPPORTED;
  const Plan P = plan_from_pub(*plan);
  if (P.kind == PLAN_MIXED && context != PM_CTX_SINGLE) return PM_EINVAL;
  std::lock_guard<std::mutex> lk(g_db_mu);
  g_db.push_back(DbRow{(long)lc, p, P, us, context});
  return PM_OK;
}

void pm_tune_db_clear(void) {
  std::lock_guard<std::mutex> lk(g_db_mu);
  g_db.clear();
}

pm_status pm_tune_db_save(const char* path) {
  if (!path) return PM_EINVAL;
  FILE* f = fopen(path, "w");
  if (!f) return PM_EINVAL;
  std::lock_guard<std::mutex> lk(g_db_mu);
  fprintf(f, "# lc p kind log_l log_ra log_rb log_c ma lq lnt us context q\n");
  for (auto& r : g_db)
    fprintf(f, "%ld %u %d %d %d %d %d %d %d %d %.4f %d %d\n", r.lc, r.p, r.plan.kind, r.plan.logL, r.plan.logRA,
            r.plan.logRB, r.plan.logC, r.plan.ma, r.plan.lq, r.plan.lnt, r.us, r.tctx, r.plan.q);
  fclose(f);
  return PM_OK;
}

pm_status pm_tune_db_load(const char* path) {
  if (!path) return PM_EINVAL;
  FILE* f = fopen(path, "r");
  if (!f) return PM_EINVAL;
  char line[512];
  std::vector<DbRow> rows;
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    DbRow r;
    // 11 fields: a single-context row; 13: the odd factor of a general-radix plan last
    const int got = sscanf(line, "%ld %u %d %d %d %d %d %d %d %d %lf %d %d", &r.lc, &r.p, &r.plan.kind, &r.plan.logL,
                           &r.plan.logRA, &r.plan.logRB, &r.plan.logC, &r.plan.ma, &r.plan.lq, &r.plan.lnt, &r.us,
                           &r.tctx, &r.plan.q);
    if (got < 11 || (got >= 12 && r.tctx != kCtxSingle && r.tctx != kCtxBatch) ||
        (r.plan.kind == PLAN_MIXED && (got < 13 || r.tctx != kCtxSingle))) {
      fclose(f);
      return PM_EINVAL;
    }
    const int pidx = prime_index(r.p);
    if (pidx < 0 || !plan_valid(r.plan, r.lc, pidx)) {
      fclose(f);
      return PM_EINVAL;
    }
    rows.push_back(r);
  }
  fclose(f);
  std::lock_guard<std::mutex> lk(g_db_mu);
  g_db.insert(g_db.end(), rows.begin(), rows.end());
  return PM_OK;
}

pm_status pm_model_features(size_t lc, uint32_t p, const pm_plan* plan, int context, float* out) {
  if (!plan || !out || lc == 0 || (context != PM_CTX_SINGLE && context != PM_CTX_BATCH)) return PM_EINVAL;
  const int pidx = prime_index(p);
  if (pidx < 0) return PM_EUNSUPPORTED;
  const Plan P = plan_from_pub(*plan);
  if (P.kind == PLAN_MIXED) return PM_EINVAL;  // the cost model covers the power-of-two plans
  plan_features((long)lc, pidx, P, context, out);
  return PM_OK;
}

/* Train the model on the timing database with the device kernels. */
pm_status pm_model_train(const float* init, int steps, float lr, float* losses) {
  std::vector<DbRow> rows;
  {
    std::lock_guard<std::mutex> lk(g_db_mu);
    for (const DbRow& r : g_db)
      if (r.plan.kind != PLAN_MIXED) rows.push_back(r);  // the cost model covers the power-of-two plans
  }
  if (rows.empty() || steps < 1) return PM_EINVAL;
  const int B = (int)rows.size();
  std::vector<float> X((size_t)B * kMlpF), t(B);
  double mean = 0, var = 0;
  std::vector<double> raw(B);
  for (int i = 0; i < B; ++i) {
    const int pidx = prime_index(rows[i].p);
    plan_features(rows[i].lc, pidx, rows[i].plan, rows[i].tctx, &X[(size_t)i * kMlpF]);
    raw[i] = std::log(rows[i].us) - std::log(plan_nprime_d(rows[i].lc, rows[i].plan));
    mean += raw[i];
  }
  mean /= B;
  for (int i = 0; i < B; ++i) var += (raw[i] - mean) * (raw[i] - mean);
  const double sd = std::sqrt(var / B) + 1e-9;
  for (int i = 0; i < B; ++i) t[i] = (float)((raw[i] - mean) / sd);
  std::vector<float> w(kMlpParams);
  if (init) {
    memcpy(w.data(), init, kMlpParams * sizeof(float));
  } else {
    u64 s = 1609010101ull;
    auto uni = [&](float a) { return (float)(((splitmix64(s) >> 11) * (1.0 / 9007199254740992.0)) * 2 - 1) * a; };
    const float a1 = std::sqrt(6.f / (kMlpF + kMlpH)), a2 = std::sqrt(6.f / (2 * kMlpH)), a3 = std::sqrt(6.f / (kMlpH + 1));
    for (int i = kOffW1; i < kOffB1; ++i) w[i] = uni(a1);
    for (int i = kOffW2; i < kOffB2; ++i) w[i] = uni(a2);
    for (int i = kOffW3; i < kOffB3; ++i) w[i] = uni(a3);
  }
  pm_status st = pm_mlp_train(w.data(), X.data(), t.data(), B, steps, lr, losses);
  if (st) return st;
  std::lock_guard<std::mutex> lk(g_model_mu);
  g_model.w = w;
  g_model.mean = (float)mean;
  g_model.std = (float)sd;
  g_model.ok = true;
  g_model.ver = ++g_model_ver;
  plan_epoch_bump();
  return PM_OK;
}

pm_status pm_model_get(float* params, float* mean, float* sd) {
  std::lock_guard<std::mutex> lk(g_model_mu);
  if (!g_model.ok) return PM_EINVAL;
  if (params) memcpy(params, g_model.w.data(), kMlpParams * sizeof(float));
  if (mean) *mean = g_model.mean;
  if (sd) *sd = g_model.std;
  return PM_OK;
}

pm_status pm_model_set(const float* params, float mean, float sd) {
  if (!params || !(sd > 0)) return PM_EINVAL;
  std::lock_guard<std::mutex> lk(g_model_mu);
  g_model.w.assign(params, params + kMlpParams);
  g_model.mean = mean;
  g_model.std = sd;
  g_model.ok = true;
  g_model.ver = ++g_model_ver;
  plan_epoch_bump();
  return PM_OK;
}

pm_status pm_model_predict(size_t lc, uint32_t p, const pm_plan* plans, size_t n, int context, double* log_us) {
  if (!plans || !log_us || lc == 0 || n == 0 || (context != PM_CTX_SINGLE && context != PM_CTX_BATCH))
    return PM_EINVAL;
  const int pidx = prime_index(p);
  if (pidx < 0) return PM_EUNSUPPORTED;
  std::vector<Plan> v(n);
  for (size_t i = 0; i < n; ++i) {
    v[i] = plan_from_pub(plans[i]);
    if (v[i].kind == PLAN_MIXED) return PM_EINVAL;  // the cost model covers the power-of-two plans
  }
  std::vector<double> out;
  pm_status st = model_predict((long)lc, pidx, v, context, &out);
  if (st) return st;
  for (size_t i = 0; i < n; ++i) log_us[i] = out[i];
  return PM_OK;
}

pm_status pm_model_save(const char* path) {
  if (!path) return PM_EINVAL;
  std::lock_guard<std::mutex> lk(g_model_mu);
  if (!g_model.ok) return PM_EINVAL;
  FILE* f = fopen(path, "w");
  if (!f) return PM_EINVAL;
  fprintf(f, "polymul-cost-model v2 features=%d hidden=%d params=%d\n%.9g %.9g\n", kMlpF, kMlpH, kMlpParams,
          g_model.mean, g_model.std);
  for (float x : g_model.w) fprintf(f, "%.9g\n", x);
  fclose(f);
  return PM_OK;
}

pm_status pm_model_load(const char* path) {
  if (!path) return PM_EINVAL;
  FILE* f = fopen(path, "r");
  if (!f) return PM_EINVAL;
  int nf = 0, nh = 0, np = 0;
  Model M;
  if (fscanf(f, "polymul-cost-model v2 features=%d hidden=%d params=%d", &nf, &nh, &np) != 3 || nf != kMlpF ||
      nh != kMlpH || np != kMlpParams || fscanf(f, "%f %f", &M.mean, &M.std) != 2) {
    fclose(f);
    return PM_EINVAL;
  }
  M.w.resize(kMlpParams);
  for (int i = 0; i < kMlpParams; ++i)
    if (fscanf(f, "%f", &M.w[i]) != 1) {
      fclose(f);
      return PM_EINVAL;
    }
  fclose(f);
  M.ok = true;
  std::lock_guard<std::mutex> lk(g_model_mu);
  g_model = M;
  g_model.ver = ++g_model_ver;
  plan_epoch_bump();
  return PM_OK;
}

}  // extern "C"
