// Sorting network for up to 1024 (key, value) pairs held one per thread by a
// workgroup of 1024 threads.
#pragma once

#include "common.hpp"

namespace hfcr {

__device__ inline uint64_t shfl_xor_u64(uint64_t x, int m) {
  const int lo = __shfl_xor((int)(uint32_t)x, m), hi = __shfl_xor((int)(uint32_t)(x >> 32), m);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Bitonic sort of P (a power of two, <= 1024) elements, element t in thread
// t's (k, v); threads t >= P hold padding and take part.  Pair (i, i +
// stride) swaps when (key_i > key_{i+stride}) equals the direction of i's
// block.  Exchanges less than a wavefront apart use lane shuffles, longer
// ones go through the LDS arrays sk, sv (1024 entries each).  Every thread
// of the workgroup must call it.
__device__ inline void wg_bitonic_1k(uint64_t &k, uint32_t &v, int P, uint64_t *sk, uint32_t *sv) {
  const int t = threadIdx.x;
  for (int size = 2; size <= P; size <<= 1) {
    const bool up = (t & size) == 0;
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      uint64_t k2;
      uint32_t v2;
      if (stride >= kWave) {
        __syncthreads();
        sk[t] = k;
        sv[t] = v;
        __syncthreads();
        k2 = sk[t ^ stride];
        v2 = sv[t ^ stride];
      } else {
        k2 = shfl_xor_u64(k, stride);
        v2 = (uint32_t)__shfl_xor((int)v, stride);
      }
      const bool lower = (t & stride) == 0;
      const bool swap = lower ? ((k > k2) == up) : ((k2 > k) == up);
      if (swap) {
        k = k2;
        v = v2;
      }
    }
  }
  __syncthreads();  // sk, sv free for the caller
}

}  // namespace hfcr
