// accumulate.hip -- deterministic scatter-add (see accumulate.h).
#include "accumulate.h"

#include <hipcub/hipcub.hpp>

namespace rta {
namespace {

struct Add3 {
  __device__ __forceinline__ rta_f3 operator()(const rta_f3& a, const rta_f3& b) const {
    return rta_f3{a.x + b.x, a.y + b.y, a.z + b.z};
  }
};

// one thread per run: the keys of the runs are distinct, so plain += is safe
__global__ void add_runs_kernel(const uint32_t* keys, const rta_f3* sums, const uint32_t* count,
                                uint32_t bound, float* out) {
  uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= bound || i >= *count) return;
  uint32_t k = keys[i];
  if (k == 0xFFFFFFFFu) return;
  rta_f3 v = sums[i];
  out[3 * (size_t)k + 0] += v.x;
  out[3 * (size_t)k + 1] += v.y;
  out[3 * (size_t)k + 2] += v.z;
}

template <typename T>
hipError_t grow(T** p, size_t n) {
  if (*p) {
    hipError_t e = hipFree(*p);
    *p = nullptr;
    if (e != hipSuccess) return e;
  }
  return hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
}

}  // namespace

void release(Buffers& b) {
  void* ps[] = {b.keys, b.keys_sorted, b.vals, b.vals_sorted, b.run_keys, b.run_sums, b.run_count, b.temp};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  b = Buffers();
}

hipError_t reserve(Buffers& b, size_t m) {
  if (m <= b.cap && b.run_count) return hipSuccess;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return e;
  size_t cap = b.cap * 2 > m ? b.cap * 2 : m;
  if (cap < 1024) cap = 1024;
  release(b);
  if ((e = grow(&b.keys, cap)) != hipSuccess) return e;
  if ((e = grow(&b.keys_sorted, cap)) != hipSuccess) return e;
  if ((e = grow(&b.vals, cap)) != hipSuccess) return e;
  if ((e = grow(&b.vals_sorted, cap)) != hipSuccess) return e;
  if ((e = grow(&b.run_keys, cap)) != hipSuccess) return e;
  if ((e = grow(&b.run_sums, cap)) != hipSuccess) return e;
  if ((e = grow(&b.run_count, 1)) != hipSuccess) return e;
  size_t s1 = 0, s2 = 0;
  if ((e = hipcub::DeviceRadixSort::SortPairs(nullptr, s1, b.keys, b.keys_sorted, b.vals, b.vals_sorted,
                                              (int)cap, 0, 32)) != hipSuccess)
    return e;
  if ((e = hipcub::DeviceReduce::ReduceByKey(nullptr, s2, b.keys_sorted, b.run_keys, b.vals_sorted,
                                             b.run_sums, b.run_count, Add3(), (int)cap)) != hipSuccess)
    return e;
  b.temp_bytes = s1 > s2 ? s1 : s2;
  if ((e = hipMalloc(&b.temp, b.temp_bytes)) != hipSuccess) return e;
  b.cap = cap;
  return hipSuccess;
}

hipError_t scatter_add(Buffers& b, size_t m, int key_bits, float* out, hipStream_t s) {
  if (m == 0) return hipSuccess;
  if (m > b.cap || m > 0x7FFFFFFFull) return hipErrorInvalidValue;
  size_t bytes = b.temp_bytes;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(b.temp, bytes, b.keys, b.keys_sorted, b.vals, b.vals_sorted,
                                                    (int)m, 0, key_bits, s);
  if (e != hipSuccess) return e;
  bytes = b.temp_bytes;
  e = hipcub::DeviceReduce::ReduceByKey(b.temp, bytes, b.keys_sorted, b.run_keys, b.vals_sorted, b.run_sums,
                                        b.run_count, Add3(), (int)m, s);
  if (e != hipSuccess) return e;
  uint32_t bound = (uint32_t)m;
  hipLaunchKernelGGL(add_runs_kernel, dim3((bound + 255) / 256), dim3(256), 0, s, b.run_keys, b.run_sums,
                     b.run_count, bound, out);
  return hipGetLastError();
}

}  // namespace rta
