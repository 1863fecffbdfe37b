// Kernel launches of the library.  The per-kernel profiler sets the two
// events of the calling thread around one launch; the runtime then records
// them together with that kernel's dispatch instead of as separate markers
// (a few microseconds of dispatch overhead remain in each figure).  Outside
// the profiler both are null and the launch is an ordinary one.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

// The calling thread's pair of profiling events (both null when not timing).
__attribute__((visibility("hidden"))) hipEvent_t* mm_launch_events();

#define MM_LAUNCH(K, G, B, S, Q, ...)                                                           \
  do {                                                                                          \
    hipEvent_t* ev_ = mm_launch_events();                                                       \
    if (ev_[0])                                                                                 \
      hipExtLaunchKernelGGL(K, G, B, S, Q, ev_[0], ev_[1], 0u, __VA_ARGS__);                    \
    else                                                                                        \
      hipLaunchKernelGGL(K, G, B, S, Q, __VA_ARGS__);                                           \
  } while (0)
