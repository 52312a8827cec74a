// Device memory of the library.  Every device allocation goes through
// dev_malloc / dev_free: hipMalloc / hipFree by default, or the caller's
// allocator installed with h2_set_allocator.  A block is always released by the
// allocator that made it, even after the hook has changed.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace h2 {

// hipSuccess with *p set (nullptr for bytes == 0), or hipErrorOutOfMemory when
// the installed allocator returned NULL (or hipMalloc's own error).
hipError_t dev_malloc_bytes(void** p, size_t bytes);

// Releases a block from dev_malloc (nullptr: no-op).  A block from the
// caller's allocator is handed back only after the device has finished all
// work queued so far, as hipFree does.
hipError_t dev_free(void* p);

template <class T>
inline hipError_t dev_malloc(T** p, size_t bytes) {
  return dev_malloc_bytes(reinterpret_cast<void**>(p), bytes);
}

}  // namespace h2
