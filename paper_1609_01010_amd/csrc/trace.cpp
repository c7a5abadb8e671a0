// Kernel tracing: when enabled, every library kernel launch carries a start
// and a stop event (graph launches are bracketed by two); pm_trace_query
// aggregates the durations by kernel name.  Off by default (one relaxed load
// per launch).
#include "trace.h"

#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/polymul.h"

namespace pm {

static std::atomic<bool> g_on{false};
static thread_local bool g_suppress = false;  // no event records while a graph is being captured

void trace_suppress(bool on) { g_suppress = on; }
static std::mutex g_mu;
struct Rec {
  std::string name;
  hipEvent_t a, b;
};
static std::vector<Rec> g_recs;
static std::vector<hipEvent_t> g_pool;

static hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

bool trace_on() { return g_on.load(std::memory_order_relaxed) && !g_suppress; }

bool trace_begin(const char* name, hipEvent_t* start, hipEvent_t* stop) {
  if (!trace_on()) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  Rec r;
  r.name = name;
  r.a = take_event();
  r.b = take_event();
  if (!r.a || !r.b) return false;
  g_recs.push_back(r);
  *start = r.a;
  *stop = r.b;
  return true;
}

TraceScope::TraceScope(hipStream_t s_, const char* name) : s(s_), slot(-1) {
  if (!trace_on()) return;
  std::lock_guard<std::mutex> lk(g_mu);
  Rec r;
  r.name = name;
  r.a = take_event();
  r.b = take_event();
  if (!r.a || !r.b) return;
  if (hipEventRecord(r.a, s) != hipSuccess) return;
  g_recs.push_back(r);
  slot = (int)g_recs.size() - 1;
}

TraceScope::~TraceScope() {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (slot < (int)g_recs.size()) hipEventRecord(g_recs[slot].b, s);
}

}  // namespace pm

using namespace pm;

extern "C" {

void pm_trace_enable(int on) { g_on.store(on != 0); }

void pm_trace_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& r : g_recs) {
    hipEventSynchronize(r.b);
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
}

pm_status pm_trace_query(const char* kernel, double* total_ms, int64_t* count) {
  if (!kernel || !total_ms || !count) return PM_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  double tot = 0;
  int64_t n = 0;
  for (auto& r : g_recs) {
    if (r.name != kernel) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return PM_EDEVICE;
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return PM_EDEVICE;
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *count = n;
  return PM_OK;
}

size_t pm_trace_names(char* buf, size_t cap) {
  std::lock_guard<std::mutex> lk(g_mu);
  std::vector<std::string> names;
  for (auto& r : g_recs) {
    bool seen = false;
    for (auto& n : names) seen |= n == r.name;
    if (!seen) names.push_back(r.name);
  }
  std::string all;
  for (auto& n : names) all += n + "\n";
  if (buf && cap) {
    size_t k = all.size() < cap - 1 ? all.size() : cap - 1;
    memcpy(buf, all.data(), k);
    buf[k] = 0;
  }
  return all.size() + 1;
}

}  // extern "C"
