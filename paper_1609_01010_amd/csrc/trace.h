// Per-kernel timing with HIP events recorded on the launch stream.
#pragma once
#include <hip/hip_runtime.h>

namespace pm {

bool trace_on();
// brackets one kernel launch: events are recorded on `s` before and after
struct TraceScope {
  hipStream_t s;
  int slot;
  TraceScope(hipStream_t s_, const char* name);
  ~TraceScope();
};

}  // namespace pm
