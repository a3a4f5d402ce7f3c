// accumulate.h -- deterministic scatter-add of per-ray gradient contributions
// (librtq internal).
//
// Each contribution is (key, three floats).  The contributions are sorted by
// key with a stable radix sort (equal keys keep their input order), runs of
// equal keys are summed in that order, and each sum is added to
// out[3 * key .. 3 * key + 2]: the result does not depend on how the GPU
// schedules the producing kernel.  Keys equal to 0xFFFFFFFF are dropped.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

struct rta_f3 {
  float x, y, z;
};

namespace rta {

// Device buffers of `cap` entries each, and hipCUB temporary storage.
struct Buffers {
  uint32_t* keys = nullptr;
  uint32_t* keys_sorted = nullptr;
  rta_f3* vals = nullptr;
  rta_f3* vals_sorted = nullptr;
  uint32_t* run_keys = nullptr;
  rta_f3* run_sums = nullptr;
  uint32_t* run_count = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0;
  size_t cap = 0;
};

// Grows `b` to hold m entries (synchronising the device before freeing).
hipError_t reserve(Buffers& b, size_t m);
void release(Buffers& b);

// Sorts b.keys / b.vals (m entries) on the low `key_bits` bits, where every
// valid key is < 2^key_bits - 1 and 0xFFFFFFFF sorts last, sums the runs and
// adds them to out.
hipError_t scatter_add(Buffers& b, size_t m, int key_bits, float* out, hipStream_t stream);

}  // namespace rta
