// Stable radix sort of (64-bit key, 32-bit value) pairs, used to order the
// invocations by affinity (Eq. 3 priority-based commit).  The sort itself is
// hipCUB's device radix sort (a library primitive); the keys are prepared by
// affinity_kernel.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "llama_internal.h"

namespace llama {

hipError_t sort_pairs_bytes(int n, size_t* bytes) {
  return hipcub::DeviceRadixSort::SortPairs(nullptr, *bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                            (const int32_t*)nullptr, (int32_t*)nullptr, n, 0, 64);
}

hipError_t sort_pairs(void* tmp, size_t tmp_bytes, const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                      int32_t* vout, int n, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, vin, vout, n, 0, 64, s);
}

}  // namespace llama
