// Block-wide helpers for radix selection (blockDim.x == BLOCK threads).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rift2 {

// Inclusive prefix sum of one value per thread across the block.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t v, uint32_t* scratch /* BLOCK */) {
  const int t = threadIdx.x;
  scratch[t] = v;
  __syncthreads();
#pragma unroll
  for (int off = 1; off < BLOCK; off <<= 1) {
    const uint32_t add = t >= off ? scratch[t - off] : 0u;
    __syncthreads();
    scratch[t] += add;
    __syncthreads();
  }
  const uint32_t r = scratch[t];
  __syncthreads();
  return r;
}

// Finds the bin of hist[0..NB) that holds the element of 0-based rank `r`,
// counting elements in ascending bin order (or descending when FROM_TOP).
// Writes the bin and the number of elements in bins scanned before it to
// *bin / *before (shared).  r must be below the histogram total.
template <int NB, int BLOCK, bool FROM_TOP>
__device__ void block_find_rank(const uint32_t* hist, uint32_t r, int* bin, uint32_t* before,
                                uint32_t* scratch /* BLOCK */) {
  static_assert(NB % BLOCK == 0, "bins per thread");
  constexpr int PER = NB / BLOCK;
  const int t = threadIdx.x;
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = t * PER + i;
    sum += hist[FROM_TOP ? NB - 1 - j : j];
  }
  const uint32_t incl = block_inclusive_scan<BLOCK>(sum, scratch);
  const uint32_t excl = incl - sum;
  if (excl <= r && r < incl) {
    uint32_t acc = excl;
    int j = t * PER;
    for (int i = 0; i < PER; ++i, ++j) {
      const uint32_t c = hist[FROM_TOP ? NB - 1 - j : j];
      if (acc + c > r) break;
      acc += c;
    }
    *bin = FROM_TOP ? NB - 1 - j : j;
    *before = acc;
  }
  __syncthreads();
}

}  // namespace rift2
