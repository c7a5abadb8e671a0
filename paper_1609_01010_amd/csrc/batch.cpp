// Batched products (pm_poly_mul_batch): thousands of independent products of
// uneven lengths and mixed primes in one hipGraph launch.
//
// Products are grouped into classes of equal plan and prime range; each
// class runs as one launch per pass over all its products (blockIdx.z picks
// the product's job descriptor).  The class launches are captured once per
// batch shape into a graph whose classes hang off a fork, so independent
// classes may run concurrently; later batches of the same shape reuse the
// graph and only upload their job descriptors.
#include <algorithm>
#include <cstring>
#include <tuple>

#include "internal.h"
#include "trace.h"

namespace pm {
bool plan_valid(const Plan& P, long lc, int pidx);
size_t plan_workspace_bytes(const Plan& P);
pm_status make_job(DevCtx* c, const Plan& P, int pidx, const void* a, long la, const void* b, long lb, u32* out,
                   long lc, u32* Ta, u32* Tb, ConvJob* J, int ring);
pm_status launch_class(const Plan& P, bool lazy, int in_type, const JobRef& jr, int njobs, int max_rows,
                       hipStream_t s);
void trace_suppress(bool on);
unsigned long plan_epoch();

namespace {

typedef std::tuple<int, int, int, int, int, int, int, int> ClassKey;  // kind, L, RA, RB, C, lq, lnt, lazy

ClassKey class_key(const Plan& P, bool lazy) {
  return ClassKey(P.kind, P.logL, P.logRA, P.logRB, P.logC, P.lq, P.kind == PLAN_FOURSTEP ? plan_row_lnt(P) : 0,
                  lazy ? 1 : 0);
}

struct ClassRun {
  ClassKey key;
  Plan plan;
  bool lazy;
  int first;  // offset in the job array
  int count;
  int max_rows;
  double work = 0;  // sum over the products of n' (3 log2 L + 10): the butterflies and multiplies
};

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  ConvJob* djobs = nullptr;  // device job array baked into the graph
  size_t njobs = 0;
};

// the batch shape: classes with their sizes (the graph depends on nothing else)
typedef std::vector<std::tuple<ClassKey, int, int>> Signature;

// The last batch shape: when the next call has the same lengths and primes
// (and no plan choice changed), its jobs differ only in the operand and
// output pointers, which are patched in place.
struct LastShape {
  std::vector<u64> key;     // (len_a, len_b, p) per problem
  unsigned long epoch = 0;  // plan epoch the jobs were built under
  void* ws = nullptr;       // workspace the jobs point into
  std::vector<ConvJob> jobs;
  std::vector<int> order;   // job index -> problem index
  std::vector<size_t> direct;
  std::vector<int> direct_pidx;
  GraphEntry* graph = nullptr;
};

struct BatchState {
  std::map<std::pair<int, Signature>, GraphEntry> graphs;  // (device, shape) -> graph
  LastShape last;
  hipStream_t cap = nullptr;                                // capture stream
  std::vector<hipStream_t> branches;                        // fork streams
  ConvJob* staging = nullptr;                               // pinned host copy of the jobs
  size_t staging_cap = 0;
  hipEvent_t staged = nullptr;  // the last upload from `staging` has completed
  // learned policy: per batch shape (hash of the lengths and primes), whether
  // the default plans ran the whole batch faster than the model's (1) or not (0)
  std::map<u64, int> plan_choice;
};
// one state per (device, stream): batches on different streams may overlap
std::map<std::pair<int, hipStream_t>, BatchState*> g_batch;

constexpr int kBranches = 4;

pm_status batch_state(DevCtx* c, hipStream_t s, BatchState** out) {
  auto it = g_batch.find({c->dev, s});
  if (it != g_batch.end()) {
    *out = it->second;
    return PM_OK;
  }
  BatchState* b = new BatchState();
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) return PM_EDEVICE;
  b->branches.resize(kBranches);
  for (auto& s : b->branches)
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return PM_EDEVICE;
  if (hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) return PM_EDEVICE;
  g_batch[{c->dev, s}] = b;
  *out = b;
  return PM_OK;
}

pm_status capture_graph(BatchState* B, const std::vector<ClassRun>& runs, ConvJob* djobs, hipGraphExec_t* exec) {
  hipStream_t cs = B->cap;
  trace_suppress(true);
  pm_status st = PM_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    trace_suppress(false);
    return PM_EDEVICE;
  }
  std::vector<hipEvent_t> evs;
  hipEvent_t fork;
  hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  hipEventRecord(fork, cs);
  // classes in decreasing work, each on the branch with the least work so far
  std::vector<bool> used(B->branches.size(), false);
  std::vector<double> load(B->branches.size(), 0.0);
  for (size_t k = 0; k < runs.size() && st == PM_OK; ++k) {
    const ClassRun& r = runs[k];
    const size_t bi = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
    load[bi] += r.work;
    hipStream_t bs = B->branches[bi];
    if (!used[bi]) {
      hipStreamWaitEvent(bs, fork, 0);
      used[bi] = true;
    }
    JobRef jr;
    memset(&jr.one, 0, sizeof(jr.one));
    jr.many = djobs + r.first;
    st = launch_class(r.plan, r.lazy, 0, jr, r.count, r.max_rows, bs);
  }
  for (size_t bi = 0; bi < B->branches.size(); ++bi) {
    if (!used[bi]) continue;
    hipEvent_t e;
    hipEventCreateWithFlags(&e, hipEventDisableTiming);
    hipEventRecord(e, B->branches[bi]);
    hipStreamWaitEvent(cs, e, 0);
    evs.push_back(e);
  }
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(cs, &g);
  trace_suppress(false);
  for (auto e : evs) hipEventDestroy(e);
  hipEventDestroy(fork);
  if (st) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (ec != hipSuccess || !g) return PM_EDEVICE;
  const hipError_t ei = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  return ei == hipSuccess ? PM_OK : PM_EDEVICE;
}

}  // namespace
}  // namespace pm

using namespace pm;

// validate the problems and pick their plans (cache, cost model or default)
static pm_status batch_plans(const pm_problem* probs, size_t count, std::vector<Plan>& plans, std::vector<int>& pidx) {
  plans.resize(count);
  pidx.resize(count);
  if (current_policy() == PM_POLICY_LEARNED) {
    // lengths not planned yet: one plan family per size class, from the cost
    // model, into the batch context's plan cache
    std::vector<long> lcs;
    std::vector<int> pix;
    for (size_t i = 0; i < count; ++i) {
      const pm_problem& q = probs[i];
      const int pi = prime_index(q.p);
      if (pi < 0 || q.len_a == 0 || q.len_b == 0 || q.len_a > (1ul << 24) || q.len_b > (1ul << 24)) continue;
      const long lc = (long)(q.len_a + q.len_b - 1);
      Plan P;
      if (lc > 64 && !plan_cache_get(lc, q.p, &P, kCtxBatch)) {
        lcs.push_back(lc);
        pix.push_back(pi);
      }
    }
    std::vector<Plan> picked;
    if (!lcs.empty() && learned_batch_plans(lcs, pix, &picked) == PM_OK)
      for (size_t k = 0; k < lcs.size(); ++k)
        if (plan_valid(picked[k], lcs[k], pix[k])) plan_cache_set(lcs[k], prime_info(pix[k]).p, picked[k], kCtxBatch);
  }
  for (size_t i = 0; i < count; ++i) {
    const pm_problem& q = probs[i];
    if (!q.a || !q.b || !q.c || q.len_a == 0 || q.len_b == 0) return PM_EINVAL;
    if (q.len_a > (1ul << 24) || q.len_b > (1ul << 24)) return PM_ETOOLARGE;
    pidx[i] = prime_index(q.p);
    if (pidx[i] < 0) return PM_EUNSUPPORTED;
    const long lc = (long)(q.len_a + q.len_b - 1);
    plans[i] = choose_plan(lc, pidx[i], nullptr, 0, kCtxBatch);
    if (!plan_valid(plans[i], lc, pidx[i])) return PM_ETOOLARGE;
  }
  return PM_OK;
}

// the batch's workspace: every four-step item's, each rounded up to 256 bytes
static size_t batch_workspace_bytes(const std::vector<Plan>& plans) {
  size_t wsb = 0;
  for (const Plan& P : plans)
    if (P.kind != PLAN_DIRECT) wsb += (plan_workspace_bytes(P) + 255) & ~(size_t)255;
  return wsb;
}

extern "C" pm_status pm_batch_workspace_query(const pm_problem* probs, size_t count, size_t* bytes) {
  if ((!probs && count) || !bytes || count > 65535) return PM_EINVAL;
  size_t wsb = 0;
  for (size_t i = 0; i < count; ++i) {
    const pm_problem& q = probs[i];
    if (!q.a || !q.b || !q.c || q.len_a == 0 || q.len_b == 0) return PM_EINVAL;
    if (q.len_a > (1ul << 24) || q.len_b > (1ul << 24)) return PM_ETOOLARGE;
    const int pi = prime_index(q.p);
    if (pi < 0) return PM_EUNSUPPORTED;
    const long lc = (long)(q.len_a + q.len_b - 1);
    if (!plan_valid(default_plan(lc, pi), lc, pi)) return PM_ETOOLARGE;
    // the same bound per product as pm_workspace_query, batched the way the executor lays it out
    Plan P;
    const size_t w = current_policy() == PM_POLICY_DEFAULT && !plan_cache_get(lc, q.p, &P, kCtxBatch)
                         ? plan_workspace_bytes(default_plan(lc, pi))
                         : product_workspace_bound(lc, pi);
    if (w) wsb += (w + 255) & ~(size_t)255;
  }
  *bytes = wsb;
  return PM_OK;
}

// Fast path: the same shape (lengths and primes, in order) as the previous
// batch on this stream, under the same plans and workspace: patch the
// operand and output pointers into the previous jobs, upload them, relaunch
// the graph.  Returns false, launching nothing, when the shape differs.
static bool batch_fast(DevCtx* c, BatchState* B, const pm_problem* probs, size_t count, hipStream_t s,
                       pm_status* st) {
  LastShape& L = B->last;
  bool same = L.graph && L.key.size() == 3 * count && L.epoch == plan_epoch() && L.ws == stream_workspace_current(c, s);
  for (size_t i = 0; same && i < count; ++i)
    same = L.key[3 * i] == probs[i].len_a && L.key[3 * i + 1] == probs[i].len_b && L.key[3 * i + 2] == probs[i].p;
  if (!same) return false;
  for (size_t i = 0; i < count; ++i)
    if (!probs[i].a || !probs[i].b || !probs[i].c) {
      *st = PM_EINVAL;
      return true;
    }
  *st = PM_EDEVICE;
  for (size_t k = 0; k < L.direct.size(); ++k) {
    const pm_problem& q = probs[L.direct[k]];
    if (launch_direct(q.a, (long)q.len_a, q.b, (long)q.len_b, q.c, L.direct_pidx[k], c->errflag, s) != hipSuccess)
      return true;
  }
  if (L.jobs.empty()) {
    *st = PM_OK;
    return true;
  }
  if (hipEventSynchronize(B->staged) != hipSuccess) return true;
  for (size_t k = 0; k < L.jobs.size(); ++k) {
    const pm_problem& q = probs[L.order[k]];
    ConvJob& J = B->staging[k];
    J = L.jobs[k];
    J.a = q.a;
    J.b = q.b;
    J.c = q.c;
  }
  const size_t bytes = L.jobs.size() * sizeof(ConvJob);
  if (hipMemcpyAsync(L.graph->djobs, B->staging, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return true;
  if (hipEventRecord(B->staged, s) != hipSuccess) return true;
  TraceScope ts(s, "batch_graph");
  *st = hipGraphLaunch(L.graph->exec, s) == hipSuccess ? PM_OK : PM_EDEVICE;
  return true;
}

// Run one batch with the given plans: the fast path when the shape repeats,
// else classes, jobs and (cached per class signature) the graph.  The caller
// holds the device lock.
static pm_status batch_run(DevCtx* c, BatchState* B, const pm_problem* probs, size_t count,
                           const std::vector<Plan>& plans, const std::vector<int>& pidx, hipStream_t s) {
  pm_status st = PM_OK;
  if (batch_fast(c, B, probs, count, s, &st)) return st;

  // classes, largest transforms first
  std::map<ClassKey, std::vector<size_t>> groups;
  std::vector<size_t> direct;
  const size_t wsb = batch_workspace_bytes(plans);
  for (size_t i = 0; i < count; ++i) {
    if (plans[i].kind == PLAN_DIRECT) {
      direct.push_back(i);
      continue;
    }
    groups[class_key(plans[i], prime_info(pidx[i]).lazy)].push_back(i);
  }
  void* wsp = nullptr;
  if (wsb) {
    st = stream_workspace(c, s, wsb, &wsp);
    if (st) return st;
  }
  std::vector<ClassRun> runs;
  std::vector<ConvJob> jobs;
  std::vector<int> order;
  jobs.reserve(count);
  char* ws = (char*)wsp;
  for (auto& kv : groups) {
    ClassRun r;
    r.key = kv.first;
    r.plan = plans[kv.second[0]];
    r.lazy = std::get<7>(kv.first) != 0;
    r.first = (int)jobs.size();
    r.count = (int)kv.second.size();
    r.max_rows = 0;
    for (size_t i : kv.second) {
      const pm_problem& q = probs[i];
      const long lc = (long)(q.len_a + q.len_b - 1);
      u32 *Ta = nullptr, *Tb = nullptr;
      const size_t w = plan_workspace_bytes(plans[i]);
      if (w) {
        Ta = (u32*)ws;
        Tb = Ta + plan_nprime(plans[i]);
        ws += (w + 255) & ~(size_t)255;
      }
      ConvJob J;
      st = make_job(c, plans[i], pidx[i], q.a, (long)q.len_a, q.b, (long)q.len_b, q.c, lc, Ta, Tb, &J, 0);
      if (st) return st;
      r.max_rows = std::max(r.max_rows, J.rows);
      r.work += (double)plan_nprime(plans[i]) * (3.0 * plans[i].logL + 10.0);
      jobs.push_back(J);
      order.push_back((int)i);
    }
    runs.push_back(r);
  }
  std::stable_sort(runs.begin(), runs.end(), [](const ClassRun& x, const ClassRun& y) { return x.work > y.work; });

  for (size_t i : direct) {
    const pm_problem& q = probs[i];
    if (launch_direct(q.a, (long)q.len_a, q.b, (long)q.len_b, q.c, pidx[i], c->errflag, s) != hipSuccess)
      return PM_EDEVICE;
  }
  if (jobs.empty()) return PM_OK;

  Signature sig;
  for (auto& r : runs) sig.emplace_back(r.key, r.count, r.max_rows);
  auto gkey = std::make_pair(c->dev, sig);
  GraphEntry* G = nullptr;
  auto git = B->graphs.find(gkey);
  if (git == B->graphs.end()) {
    GraphEntry ge;
    ge.njobs = jobs.size();
    if (hipMalloc(&ge.djobs, jobs.size() * sizeof(ConvJob)) != hipSuccess) return PM_ENOMEM;
    st = capture_graph(B, runs, ge.djobs, &ge.exec);
    if (st) {
      hipFree(ge.djobs);
      return st;
    }
    G = &(B->graphs[gkey] = ge);
  } else {
    G = &git->second;
  }
  // upload the job descriptors (the graph reads them from G->djobs)
  if (hipEventSynchronize(B->staged) != hipSuccess) return PM_EDEVICE;
  if (B->staging_cap < jobs.size()) {
    if (B->staging) hipHostFree(B->staging);
    B->staging = nullptr;
    if (hipHostMalloc((void**)&B->staging, jobs.size() * sizeof(ConvJob), hipHostMallocDefault) != hipSuccess) {
      B->staging_cap = 0;
      return PM_ENOMEM;
    }
    B->staging_cap = jobs.size();
  }
  // the device array keeps the class-by-class layout the graph was captured with
  memcpy(B->staging, jobs.data(), jobs.size() * sizeof(ConvJob));
  {
    LastShape& L = B->last;
    L.key.resize(3 * count);
    for (size_t i = 0; i < count; ++i) {
      L.key[3 * i] = probs[i].len_a;
      L.key[3 * i + 1] = probs[i].len_b;
      L.key[3 * i + 2] = probs[i].p;
    }
    L.epoch = plan_epoch();
    L.ws = wsp;
    L.jobs = jobs;
    L.order = order;
    L.direct = direct;
    L.direct_pidx.clear();
    for (size_t i : direct) L.direct_pidx.push_back(pidx[i]);
    L.graph = G;
  }
  if (hipMemcpyAsync(G->djobs, B->staging, jobs.size() * sizeof(ConvJob), hipMemcpyHostToDevice, s) != hipSuccess)
    return PM_EDEVICE;
  if (hipEventRecord(B->staged, s) != hipSuccess) return PM_EDEVICE;
  TraceScope ts(s, "batch_graph");
  if (hipGraphLaunch(G->exec, s) != hipSuccess) return PM_EDEVICE;
  return PM_OK;
}

// FNV-1a over the (len_a, len_b, p) of every problem
static u64 shape_hash(const pm_problem* probs, size_t count) {
  u64 h = 1469598103934665603ull;
  auto mix = [&h](u64 v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xFF;
      h *= 1099511628211ull;
    }
  };
  mix(count);
  for (size_t i = 0; i < count; ++i) {
    mix(probs[i].len_a);
    mix(probs[i].len_b);
    mix(probs[i].p);
  }
  return h;
}

// median milliseconds of three runs of the batch with these plans (after one)
static pm_status time_batch(DevCtx* c, BatchState* B, const pm_problem* probs, size_t count,
                            const std::vector<Plan>& plans, const std::vector<int>& pidx, hipStream_t s, float* ms) {
  pm_status st = batch_run(c, B, probs, count, plans, pidx, s);
  hipEvent_t e0, e1;
  if (st || hipEventCreate(&e0) || hipEventCreate(&e1)) return st ? st : PM_EDEVICE;
  std::vector<float> t;
  for (int r = 0; r < 3 && st == PM_OK; ++r) {
    hipEventRecord(e0, s);
    st = batch_run(c, B, probs, count, plans, pidx, s);
    hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) st = PM_EDEVICE;
    float x = 0;
    hipEventElapsedTime(&x, e0, e1);
    t.push_back(x);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st) return st;
  std::sort(t.begin(), t.end());
  *ms = t[1];
  return PM_OK;
}

extern "C" pm_status pm_poly_mul_batch(const pm_problem* probs, size_t count, void* stream) {
  if (!probs && count) return PM_EINVAL;
  if (count == 0) return PM_OK;
  if (count > 65535) return PM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  pm_status st;
  DevCtx* c = ctx_current(&st);
  if (!c) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  BatchState* B;
  st = batch_state(c, s, &B);
  if (st) return st;
  // a repeated shape needs no planning at all
  if (batch_fast(c, B, probs, count, s, &st)) return st;
  std::vector<Plan> plans;
  std::vector<int> pidx;
  st = batch_plans(probs, count, plans, pidx);
  if (st) return st;
  if (current_policy() != PM_POLICY_LEARNED) return batch_run(c, B, probs, count, plans, pidx, s);
  // Learned policy: the model's plans are chosen per transform length, but
  // the classes of a batch share the device, and how well they overlap
  // decides its time.  The first call of a batch shape therefore runs it
  // with the model's plans and with the default plans, waits, and keeps the
  // faster for that shape.
  std::vector<Plan> dplans(count);
  bool differ = false;
  for (size_t i = 0; i < count; ++i) {
    const long lc = (long)(probs[i].len_a + probs[i].len_b - 1);
    // a plan the caller put into the cache is kept in both
    dplans[i] = plan_pinned(lc, probs[i].p) ? plans[i] : default_plan(lc, pidx[i]);
    const Plan& P = plans[i];
    const Plan& D = dplans[i];
    differ |= P.kind != D.kind || P.logL != D.logL || P.logRA != D.logRA || P.logRB != D.logRB ||
              P.logC != D.logC || P.ma != D.ma || P.lq != D.lq || plan_row_lnt(P) != plan_row_lnt(D);
  }
  if (!differ) return batch_run(c, B, probs, count, plans, pidx, s);
  const u64 h = shape_hash(probs, count);
  auto v = B->plan_choice.find(h);
  if (v == B->plan_choice.end()) {
    float t_model = 0, t_default = 0;
    st = time_batch(c, B, probs, count, plans, pidx, s, &t_model);
    if (st == PM_OK) st = time_batch(c, B, probs, count, dplans, pidx, s, &t_default);
    if (st) return st;
    v = B->plan_choice.emplace(h, t_default < t_model ? 1 : 0).first;
  }
  return batch_run(c, B, probs, count, v->second ? dplans : plans, pidx, s);
}
