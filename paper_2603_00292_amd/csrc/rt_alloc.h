// rt_alloc.h -- every device and pinned-host allocation of librtq goes
// through these calls (librtq internal).  They add one test hook: when the
// environment variable RT_FAULT_ALLOC = k (k >= 1) is set at
// rt_context_create, the k-th allocation after that call fails with
// hipErrorOutOfMemory without allocating (once; later ones succeed), so
// that tests can drive every out-of-memory path.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

// true for the one allocation the hook fails (defined in rt_api.cpp)
__attribute__((visibility("hidden"))) bool rt_alloc_fault();

inline hipError_t rt_malloc(void** p, size_t bytes) {
  if (rt_alloc_fault()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

template <typename T>
inline hipError_t rt_malloc(T** p, size_t bytes) {
  return rt_malloc(reinterpret_cast<void**>(p), bytes);
}

inline hipError_t rt_malloc_async(void** p, size_t bytes, hipStream_t s) {
  if (rt_alloc_fault()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMallocAsync(p, bytes, s);
}

template <typename T>
inline hipError_t rt_host_malloc(T** p, size_t bytes, unsigned flags) {
  if (rt_alloc_fault()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipHostMalloc(reinterpret_cast<void**>(p), bytes, flags);
}
