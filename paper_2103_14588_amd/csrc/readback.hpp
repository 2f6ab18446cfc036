// readback.hpp -- page-locked host memory for the solvers' scalar readbacks.
#pragma once

#include <hip/hip_runtime.h>

namespace dst {

// A small page-locked host buffer per host thread, allocated on first use and
// kept for the life of the process.  The solvers copy their convergence
// scalars (norms, residual estimates, breakdown flags) into it before each
// host decision: a device-to-host copy into pageable memory is staged through
// a driver buffer and adds a round trip to every such decision.  Returns
// nullptr if the allocation failed; the caller then reads into its own memory.
constexpr int kReadbackDoubles = 64;
inline double *readback_buffer() {
  thread_local double *p = nullptr;
  thread_local bool tried = false;
  if (!tried) {
    tried = true;
    if (hipHostMalloc((void **)&p, kReadbackDoubles * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();  // the failure is handled here, not by the next call's check
    }
  }
  return p;
}

}  // namespace dst
