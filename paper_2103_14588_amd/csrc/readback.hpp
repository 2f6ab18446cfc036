// readback.hpp -- page-locked host memory for the solvers' scalar readbacks.
#pragma once

#include <cstddef>

#include <hip/hip_runtime.h>

namespace dst {

// A page-locked host buffer per host thread of at least `bytes`, allocated on
// first use, grown when a larger one is asked for and kept for the life of
// the process.  The solvers copy their convergence scalars (norms, residual
// estimates, breakdown flags) into it before each host decision: a
// device-to-host copy into pageable memory is staged through a driver buffer
// and adds a round trip to every such decision.  Every use waits for its
// copy before returning, so no copy is in flight when the buffer is replaced.
// Returns nullptr if the allocation failed; the caller then reads into its
// own memory.
inline void *readback_buffer(size_t bytes) {
  thread_local void *p = nullptr;
  thread_local size_t cap = 0;
  if (bytes > cap) {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    const size_t want = bytes < 4096 ? 4096 : bytes;
    if (hipHostMalloc(&p, want, hipHostMallocDefault) == hipSuccess) {
      cap = want;
    } else {
      p = nullptr;
      (void)hipGetLastError();  // handled here, not reported by the next call's check
    }
  }
  return p;
}

}  // namespace dst
