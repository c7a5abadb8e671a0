// Batched products (pm_poly_mul_batch): thousands of independent products of
// uneven lengths and mixed primes in one hipGraph launch.
//
// Products are grouped into classes of equal plan and prime range (the
// products of at most 64 outputs, computed by their defining sums, form one
// class); each class runs as one launch per pass over all its products
// (blockIdx.z picks the product's job descriptor).  The class launches are
// captured once per batch shape into a graph whose classes hang off a fork,
// so independent classes may run concurrently; later batches of the same
// shape reuse the graph and only upload their job descriptors.  While
// kernel tracing is on, the classes run one after the other on the caller's
// stream instead, so that each launch's recorded time is its own.
#include <algorithm>
#include <cstring>
#include <tuple>

#include "internal.h"
#include "trace.h"

namespace pm {
bool plan_valid(const Plan& P, long lc, int pidx);
size_t plan_workspace_bytes(const Plan& P);
pm_status launch_class(const Plan& P, bool lazy, int in_type, const JobRef& jr, int njobs, int max_rows,
                       hipStream_t s);
void trace_suppress(bool on);
unsigned long plan_epoch();

namespace {

typedef std::tuple<int, int, int, int, int, int, int, int> ClassKey;  // kind, L, RA, RB, C, lq, lnt, lazy

// The one-work-group products of the lengths the several-length kernel
// takes form one class per value range (L = 0 in the key): one launch for
// all of them instead of one per length and first radix.
ClassKey class_key(const Plan& P, bool lazy) {
  if (lds_multi_ok(P)) return ClassKey(P.kind, 0, 0, 0, 0, 0, 0, lazy ? 1 : 0);
  return ClassKey(P.kind, P.logL, P.logRA, P.logRB, P.logC, P.lq, P.kind == PLAN_FOURSTEP ? plan_row_lnt(P) : 0,
                  lazy ? 1 : 0);
}

bool multi_lds_class(const ClassKey& k) { return std::get<0>(k) == PLAN_LDS && std::get<1>(k) == 0; }

// the launches of one class (the several-length one-work-group class has
// its own kernel)
pm_status launch_run(const ClassKey& key, const Plan& P, bool lazy, const JobRef& jr, int njobs, int max_rows,
                     hipStream_t s) {
  if (multi_lds_class(key)) return launch_lds_conv_multi(lazy, jr, njobs, s) == hipSuccess ? PM_OK : PM_EDEVICE;
  return launch_class(P, lazy, 0, jr, njobs, max_rows, s);
}

struct ClassRun {
  ClassKey key;
  Plan plan;
  bool lazy;
  int first;  // offset in the job array
  int count;
  int max_rows;
  double work = 0;  // sum over the products of n' (3 log2 L + 10): the butterflies and multiplies
  long wgs = 0;     // work-groups of the class's widest launch
};

// A class whose launches have fewer work-groups than the device has compute
// units cannot fill it: its time is the latency of its rounds, and it runs
// beside the large classes rather than after them.
constexpr long kSmallClassWgs = 256;

// latency-bound classes, which start first on branch 0 beside the large
// ones: fewer work-groups than compute units, or the several-length class of
// one-work-group products (at most 2^11 points each)
bool small_class(const ClassRun& r) { return r.wgs < kSmallClassWgs || multi_lds_class(r.key); }

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  ConvJob* djobs = nullptr;      // device job array baked into the graph
  const void** dptrs = nullptr;  // (a, b, c) per job: the graph's first kernel patches them into djobs
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
  std::vector<ClassRun> runs;
  std::vector<Plan> plans;  // per problem
  GraphEntry* graph = nullptr;
};

struct BatchState {
  std::map<std::pair<int, Signature>, GraphEntry> graphs;  // (device, shape) -> graph
  LastShape last;
  hipStream_t cap = nullptr;                                // capture stream
  std::vector<hipStream_t> branches;                        // fork streams
  ConvJob* staging = nullptr;                               // pinned host copy of the jobs
  size_t staging_cap = 0;
  const void** pstaging = nullptr;                          // pinned host copy of the pointers
  size_t pstaging_cap = 0;
  hipEvent_t staged = nullptr;  // the last upload from the staging buffers has completed
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

pm_status capture_graph(BatchState* B, const std::vector<ClassRun>& runs, const GraphEntry& G,
                        hipGraphExec_t* exec) {
  hipStream_t cs = B->cap;
  ConvJob* djobs = G.djobs;
  trace_suppress(true);
  pm_status st = PM_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    trace_suppress(false);
    return PM_EDEVICE;
  }
  // this launch's operand and output pointers into the descriptors, before any class
  if (launch_patch_jobs(djobs, G.dptrs, (int)G.njobs, cs) != hipSuccess) st = PM_EDEVICE;
  std::vector<hipEvent_t> evs;
  hipEvent_t fork;
  hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  hipEventRecord(fork, cs);
  // The small classes first, all on branch 0, so that they start with the
  // large ones instead of trailing them; then the large classes in
  // decreasing work, each on the branch with the least work so far.
  std::vector<bool> used(B->branches.size(), false);
  std::vector<double> load(B->branches.size(), 0.0);
  std::vector<size_t> order;
  for (int pass = 0; pass < 2; ++pass)
    for (size_t k = 0; k < runs.size(); ++k)
      if (small_class(runs[k]) == (pass == 0)) order.push_back(k);
  for (size_t k : order) {
    if (st != PM_OK) break;
    const ClassRun& r = runs[k];
    const size_t bi = small_class(r)
                          ? 0
                          : (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
    load[bi] += r.work;
    hipStream_t bs = B->branches[bi];
    if (!used[bi]) {
      hipStreamWaitEvent(bs, fork, 0);
      used[bi] = true;
    }
    JobRef jr;
    memset(&jr.one, 0, sizeof(jr.one));
    jr.many = djobs + r.first;
    st = launch_run(r.key, r.plan, r.lazy, jr, r.count, r.max_rows, bs);
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

// The batch's classes: one graph launch, or (kernel tracing on) the class
// launches one after the other on s
static pm_status launch_batch(GraphEntry* G, const std::vector<ClassRun>& runs, hipStream_t s) {
  if (trace_on()) {
    if (launch_patch_jobs(G->djobs, G->dptrs, (int)G->njobs, s) != hipSuccess) return PM_EDEVICE;
    for (const ClassRun& r : runs) {
      JobRef jr;
      memset(&jr.one, 0, sizeof(jr.one));
      jr.many = G->djobs + r.first;
      const pm_status st = launch_run(r.key, r.plan, r.lazy, jr, r.count, r.max_rows, s);
      if (st) return st;
    }
    return PM_OK;
  }
  TraceScope ts(s, "batch_graph");
  return hipGraphLaunch(G->exec, s) == hipSuccess ? PM_OK : PM_EDEVICE;
}

// pinned staging of at least n entries
template <typename T>
static pm_status staging_room(T** buf, size_t* cap, size_t n) {
  if (*cap >= n) return PM_OK;
  if (*buf) hipHostFree((void*)*buf);
  *buf = nullptr;
  *cap = 0;
  if (hipHostMalloc((void**)buf, n * sizeof(T), hipHostMallocDefault) != hipSuccess) return PM_ENOMEM;
  *cap = n;
  return PM_OK;
}

// upload the (a, b, c) pointers of every job, in job order, to G->dptrs
static pm_status upload_ptrs(BatchState* B, GraphEntry* G, const pm_problem* probs, const std::vector<int>& order,
                             hipStream_t s) {
  const size_t n = order.size();
  for (size_t k = 0; k < n; ++k) {
    const pm_problem& q = probs[order[k]];
    B->pstaging[3 * k] = q.a;
    B->pstaging[3 * k + 1] = q.b;
    B->pstaging[3 * k + 2] = q.c;
  }
  if (hipMemcpyAsync(G->dptrs, B->pstaging, 3 * n * sizeof(void*), hipMemcpyHostToDevice, s) != hipSuccess)
    return PM_EDEVICE;
  return PM_OK;
}

// Fast path: the same shape (lengths and primes, in order) as the previous
// batch on this stream, under the same plan epoch and workspace: upload the
// new operand and output pointers (the graph's first kernel patches them
// into the descriptors) and relaunch the graph.  Returns false, launching
// nothing, when the shape differs.  A caller that holds plans of its own
// checks first that the last graph was built from them (same_plans).
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
  if (hipEventSynchronize(B->staged) != hipSuccess) return true;
  *st = upload_ptrs(B, L.graph, probs, L.order, s);
  if (*st) return true;
  *st = PM_EDEVICE;
  if (hipEventRecord(B->staged, s) != hipSuccess) return true;
  *st = launch_batch(L.graph, L.runs, s);
  return true;
}

static bool same_plans(const std::vector<Plan>& x, const std::vector<Plan>& y) {
  if (x.size() != y.size()) return false;
  for (size_t i = 0; i < x.size(); ++i)
    if (!same_plan(x[i], y[i])) return false;
  return true;
}

// Run one batch with the given plans: the fast path when the shape repeats
// under the same plans, else classes, jobs and (cached per class signature)
// the graph.  The caller holds the device lock.
static pm_status batch_run(DevCtx* c, BatchState* B, const pm_problem* probs, size_t count,
                           const std::vector<Plan>& plans, const std::vector<int>& pidx, hipStream_t s) {
  pm_status st = PM_OK;
  if (same_plans(B->last.plans, plans) && batch_fast(c, B, probs, count, s, &st)) return st;

  // classes, largest transforms first (the defining sums form one class)
  std::map<ClassKey, std::vector<size_t>> groups;
  const size_t wsb = batch_workspace_bytes(plans);
  for (size_t i = 0; i < count; ++i) {
    const bool lazy = plans[i].kind != PLAN_DIRECT && prime_info(pidx[i]).lazy;
    groups[class_key(plans[i], lazy)].push_back(i);
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
    if (multi_lds_class(kv.first))  // longest first: the tail is short
      std::stable_sort(kv.second.begin(), kv.second.end(),
                       [&](size_t x, size_t y) { return plans[x].logL > plans[y].logL; });
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
      r.work += plans[i].kind == PLAN_DIRECT ? (double)q.len_a * q.len_b
                                              : (double)plan_nprime(plans[i]) * (3.0 * plans[i].logL + 10.0);
      jobs.push_back(J);
      order.push_back((int)i);
    }
    r.wgs = r.plan.kind == PLAN_FOURSTEP ? (long)r.count * r.max_rows : (long)r.count;
    runs.push_back(r);
  }
  std::stable_sort(runs.begin(), runs.end(), [](const ClassRun& x, const ClassRun& y) { return x.work > y.work; });


  Signature sig;
  for (auto& r : runs) sig.emplace_back(r.key, r.count, r.max_rows);
  auto gkey = std::make_pair(c->dev, sig);
  GraphEntry* G = nullptr;
  auto git = B->graphs.find(gkey);
  if (git == B->graphs.end()) {
    GraphEntry ge;
    ge.njobs = jobs.size();
    if (hipMalloc(&ge.djobs, jobs.size() * sizeof(ConvJob)) != hipSuccess) return PM_ENOMEM;
    if (hipMalloc((void**)&ge.dptrs, 3 * jobs.size() * sizeof(void*)) != hipSuccess) {
      hipFree(ge.djobs);
      return PM_ENOMEM;
    }
    st = capture_graph(B, runs, ge, &ge.exec);
    if (st) {
      hipFree(ge.djobs);
      hipFree((void*)ge.dptrs);
      return st;
    }
    G = &(B->graphs[gkey] = ge);
  } else {
    G = &git->second;
  }
  // upload the job descriptors (the graph reads them from G->djobs) and
  // their pointers (which its first kernel writes into them again)
  if (hipEventSynchronize(B->staged) != hipSuccess) return PM_EDEVICE;
  st = staging_room(&B->staging, &B->staging_cap, jobs.size());
  if (st == PM_OK) st = staging_room(&B->pstaging, &B->pstaging_cap, 3 * jobs.size());
  if (st) return st;
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
    L.runs = runs;
    L.plans = plans;
    L.graph = G;
  }
  if (hipMemcpyAsync(G->djobs, B->staging, jobs.size() * sizeof(ConvJob), hipMemcpyHostToDevice, s) != hipSuccess)
    return PM_EDEVICE;
  st = upload_ptrs(B, G, probs, order, s);
  if (st) return st;
  if (hipEventRecord(B->staged, s) != hipSuccess) return PM_EDEVICE;
  return launch_batch(G, runs, s);
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

// three timed runs of the batch with these plans (after one that builds its
// jobs and graph), appended to *ms
static pm_status time_batch(DevCtx* c, BatchState* B, const pm_problem* probs, size_t count,
                            const std::vector<Plan>& plans, const std::vector<int>& pidx, hipStream_t s,
                            std::vector<float>* ms) {
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
  ms->insert(ms->end(), t.begin(), t.end());
  return PM_OK;
}

static float median_of(std::vector<float> v) {
  std::sort(v.begin(), v.end());
  return v[v.size() / 2];
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
  // with the model's plans and with the default plans, twice each in turn,
  // waits, and keeps the plans with the lower median time for that shape.
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
    std::vector<float> t_model, t_default;
    for (int r = 0; r < 2 && st == PM_OK; ++r) {
      st = time_batch(c, B, probs, count, plans, pidx, s, &t_model);
      if (st == PM_OK) st = time_batch(c, B, probs, count, dplans, pidx, s, &t_default);
    }
    if (st) return st;
    v = B->plan_choice.emplace(h, median_of(t_default) < median_of(t_model) ? 1 : 0).first;
  }
  return batch_run(c, B, probs, count, v->second ? dplans : plans, pidx, s);
}

extern "C" pm_status pm_batch_plans_used(void* stream, pm_plan* out, size_t count) {
  if (!out) return PM_EINVAL;
  pm_status st;
  DevCtx* c = ctx_current(&st);
  if (!c) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = g_batch.find({c->dev, (hipStream_t)stream});
  if (it == g_batch.end() || it->second->last.plans.size() != count) return PM_EINVAL;
  const std::vector<Plan>& v = it->second->last.plans;
  for (size_t i = 0; i < count; ++i) {
    out[i].kind = v[i].kind;
    out[i].log_l = v[i].logL;
    out[i].log_ra = v[i].logRA;
    out[i].log_rb = v[i].logRB;
    out[i].log_c = v[i].logC;
    out[i].ma = v[i].ma;
    out[i].lq = v[i].lq;
    out[i].lnt = v[i].lnt;
  }
  return PM_OK;
}
