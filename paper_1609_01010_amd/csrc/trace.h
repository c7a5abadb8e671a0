// Per-kernel timing with HIP events.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace pm {

bool trace_on();
// Registers one traced launch of kernel `name` and returns its two events
// (false when tracing is off or events are unavailable).
bool trace_begin(const char* name, hipEvent_t* start, hipEvent_t* stop);

// brackets a graph launch: events are recorded on `s` before and after
struct TraceScope {
  hipStream_t s;
  int slot;
  TraceScope(hipStream_t s_, const char* name);
  ~TraceScope();
};

// Launch a library kernel.  While tracing is on the dispatch carries its own
// start and stop events, so the recorded time is that of the kernel alone
// (no marker packets between consecutive kernels).
template <typename... KArgs, typename... Args>
inline hipError_t launch(const char* name, void (*kern)(KArgs...), dim3 grid, dim3 block, size_t lds,
                         hipStream_t s, Args... args) {
  hipEvent_t e0, e1;
  if (trace_begin(name, &e0, &e1))
    hipExtLaunchKernelGGL(kern, grid, block, (uint32_t)lds, s, e0, e1, 0u, static_cast<KArgs>(args)...);
  else
    hipLaunchKernelGGL(kern, grid, block, (uint32_t)lds, s, static_cast<KArgs>(args)...);
  return hipGetLastError();
}

}  // namespace pm
