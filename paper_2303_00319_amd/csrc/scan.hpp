// Block-wide helpers for radix selection (blockDim.x == BLOCK threads).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rift2 {

// Inclusive prefix sum within one wave (64 lanes) by lane shuffles.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t n = __shfl_up(v, off, 64);
    if (lane >= off) v += n;
  }
  return v;
}

// Inclusive prefix sum of one value per thread across the block: a scan per
// wave, then the wave totals through `scratch` (one barrier before, one after
// so that scratch can be reused at once).
template <int BLOCK>
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t v, uint32_t* scratch /* >= BLOCK / 64 */) {
  static_assert(BLOCK % 64 == 0 && BLOCK <= 1024, "whole waves");
  constexpr int NW = BLOCK / 64;
  const int w = threadIdx.x >> 6;
  v = wave_inclusive_scan(v);
  if (NW == 1) return v;
  if ((threadIdx.x & 63) == 63) scratch[w] = v;
  __syncthreads();
  uint32_t base = 0;
#pragma unroll
  for (int i = 0; i < NW - 1; ++i) base += i < w ? scratch[i] : 0u;
  __syncthreads();
  return v + base;
}

// Finds the bin of hist[0..NB) that holds the element of 0-based rank `r`,
// counting elements in ascending bin order (or descending when FROM_TOP).
// Writes the bin and the number of elements in bins scanned before it to
// *bin / *before (shared).  r must be below the histogram total.  Each
// thread reads its PER bins once and keeps them in registers.
template <int NB, int BLOCK, bool FROM_TOP>
__device__ void block_find_rank(const uint32_t* hist, uint32_t r, int* bin, uint32_t* before,
                                uint32_t* scratch /* >= BLOCK / 64 */) {
  static_assert(NB % BLOCK == 0, "bins per thread");
  constexpr int PER = NB / BLOCK;
  const int t = threadIdx.x;
  uint32_t c[PER];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = t * PER + i;
    c[i] = hist[FROM_TOP ? NB - 1 - j : j];
    sum += c[i];
  }
  const uint32_t incl = block_inclusive_scan<BLOCK>(sum, scratch);
  const uint32_t excl = incl - sum;
  if (excl <= r && r < incl) {
    uint32_t acc = excl;
    int hit = PER - 1;
    uint32_t acc_hit = 0;
    bool found = false;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (!found && acc + c[i] > r) {
        found = true;
        hit = i;
        acc_hit = acc;
      }
      acc += c[i];
    }
    const int j = t * PER + hit;
    *bin = FROM_TOP ? NB - 1 - j : j;
    *before = acc_hit;
  }
  __syncthreads();
}

// The bins of ranks r and r + 1 (ascending) in one pass over hist[0..NB):
// one scan, and each rank resolved by the thread whose bins hold it.  Writes
// bin[q] / before[q] for rank r + q (shared); r + 1 must be below the total.
template <int NB, int BLOCK>
__device__ void block_find_two_ranks(const uint32_t* hist, uint32_t r, int* bin, uint32_t* before,
                                     uint32_t* scratch /* >= BLOCK / 64 */) {
  static_assert(NB % BLOCK == 0, "bins per thread");
  constexpr int PER = NB / BLOCK;
  const int t = threadIdx.x;
  uint32_t c[PER];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    c[i] = hist[t * PER + i];
    sum += c[i];
  }
  const uint32_t incl = block_inclusive_scan<BLOCK>(sum, scratch);
  const uint32_t excl = incl - sum;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const uint32_t rq = r + (uint32_t)q;
    if (excl <= rq && rq < incl) {
      uint32_t acc = excl;
      int hit = PER - 1;
      uint32_t acc_hit = 0;
      bool found = false;
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        if (!found && acc + c[i] > rq) {
          found = true;
          hit = i;
          acc_hit = acc;
        }
        acc += c[i];
      }
      bin[q] = t * PER + hit;
      before[q] = acc_hit;
    }
  }
  __syncthreads();
}

}  // namespace rift2
