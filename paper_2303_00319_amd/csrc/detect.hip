// FAST keypoint kernels (Section 2.1 of the paper; Table 1 settings).
//
//   k_det_init    clear counters / histogram, min-max identities
//   k_det_minmax  global min and max of the map (order-preserving uint keys)
//   k_det_fast    per 32x8 tile: normalise (correctly rounded FP32 division),
//                 FAST-9 score on the 16-pixel circle, 3x3 NMS with raster
//                 tie-break, patch-border mask; survivors appended as 64-bit
//                 keys (score bits << 32 | ~raster) plus a histogram of the
//                 top 16 score bits
//   k_det_select  threshold bin of rank K, candidates at or above it gathered;
//                 the last block radix-selects the exact K-th key on the
//                 boundary bin and compacts the K winners
//   k_det_sort    rank of every winner by counting larger keys -> output order
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rift2 {

constexpr int kDetHistBins = 1 << 14;  // score bits >> 16 for scores in (0, 1]
constexpr int kTileX = 32, kTileY = 8;
constexpr int kHalo = 4;  // FAST radius 3 + NMS 1

struct DetWs {
  // header (uint32 words), zeroed per call
  uint32_t* hdr;      // [0] n_cand, [1] done, [2] n_sel, [3] n_final, [4] min key, [5] max key, [6] done2
  uint32_t* hist;     // kDetHistBins
  uint64_t* cand;     // candidate keys
  uint64_t* sel;      // keys at or above the threshold bin
  uint64_t* fin;      // exactly min(K, n_cand) winners
};

__device__ __forceinline__ uint32_t float_order_key(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float float_from_order_key(uint32_t k) {
  const uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(b);
}

__global__ void k_det_init(uint32_t* __restrict__ hdr, uint32_t* __restrict__ hist) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kDetHistBins) hist[i] = 0u;
  if (i < 16) hdr[i] = (i == 4) ? 0xffffffffu : 0u;
}

__global__ void __launch_bounds__(256) k_det_minmax(const float* __restrict__ d, int n, uint32_t* __restrict__ hdr) {
  uint32_t lo = 0xffffffffu, hi = 0u;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t k = float_order_key(d[i]);
    lo = min(lo, k);
    hi = max(hi, k);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, off));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, off));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&hdr[4], lo);
    atomicMax(&hdr[5], hi);
  }
}

// Largest t such that 9 contiguous circle values all exceed p + t, or all fall below p - t.
__device__ __forceinline__ float fast_score(const float (&c)[16], float p) {
  float mn2[16], mx2[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    mn2[i] = fminf(c[i], c[(i + 1) & 15]);
    mx2[i] = fmaxf(c[i], c[(i + 1) & 15]);
  }
  float mn4[16], mx4[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    mn4[i] = fminf(mn2[i], mn2[(i + 2) & 15]);
    mx4[i] = fmaxf(mx2[i], mx2[(i + 2) & 15]);
  }
  float best_lo = -INFINITY, best_hi = INFINITY;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const float lo9 = fminf(fminf(mn4[i], mn4[(i + 4) & 15]), c[(i + 8) & 15]);
    const float hi9 = fmaxf(fmaxf(mx4[i], mx4[(i + 4) & 15]), c[(i + 8) & 15]);
    best_lo = fmaxf(best_lo, lo9);
    best_hi = fminf(best_hi, hi9);
  }
  const float bright = __fsub_rn(best_lo, p);
  const float dark = __fsub_rn(p, best_hi);
  return fmaxf(bright, dark);
}

__global__ void __launch_bounds__(kTileX * kTileY) k_det_fast(const float* __restrict__ d, int H, int W, float thr,
                                                              int half_patch, uint32_t* __restrict__ hdr,
                                                              uint32_t* __restrict__ hist, uint64_t* __restrict__ cand) {
  constexpr int LX = kTileX + 2 * kHalo, LY = kTileY + 2 * kHalo;
  constexpr int SX = kTileX + 2, SY = kTileY + 2;
  __shared__ float sd[LY][LX];
  __shared__ float ss[SY][SX];
  const float lo = float_from_order_key(hdr[4]);
  const float hi = float_from_order_key(hdr[5]);
  if (!(hi > lo)) return;  // flat map: no keypoints (uniform across the grid)
  const float rng = __fsub_rn(hi, lo);
  const int x0 = blockIdx.x * kTileX - kHalo, y0 = blockIdx.y * kTileY - kHalo;
  for (int i = threadIdx.x; i < LX * LY; i += blockDim.x) {
    const int ly = i / LX, lx = i % LX;
    const int gy = y0 + ly, gx = x0 + lx;
    float v = 0.0f;
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = __fdiv_rn(__fsub_rn(d[(size_t)gy * W + gx], lo), rng);
    sd[ly][lx] = v;
  }
  __syncthreads();
  // scores of the tile plus a one-pixel ring
  for (int i = threadIdx.x; i < SX * SY; i += blockDim.x) {
    const int sy = i / SX, sx = i % SX;
    const int gy = y0 + kHalo - 1 + sy, gx = x0 + kHalo - 1 + sx;
    float sc = 0.0f;
    if (gy >= 3 && gy <= H - 4 && gx >= 3 && gx <= W - 4) {
      const int cy = sy + kHalo - 1, cx = sx + kHalo - 1;
      const float c[16] = {sd[cy - 3][cx], sd[cy - 3][cx + 1], sd[cy - 2][cx + 2], sd[cy - 1][cx + 3],
                           sd[cy][cx + 3],     sd[cy + 1][cx + 3], sd[cy + 2][cx + 2], sd[cy + 3][cx + 1],
                           sd[cy + 3][cx],     sd[cy + 3][cx - 1], sd[cy + 2][cx - 2], sd[cy + 1][cx - 3],
                           sd[cy][cx - 3],     sd[cy - 1][cx - 3], sd[cy - 2][cx - 2], sd[cy - 3][cx - 1]};
      sc = fast_score(c, sd[cy][cx]);
    }
    ss[sy][sx] = sc;
  }
  __syncthreads();
  const int tx = threadIdx.x % kTileX, ty = threadIdx.x / kTileX;
  const int gx = blockIdx.x * kTileX + tx, gy = blockIdx.y * kTileY + ty;
  bool keep = false;
  float sc = 0.0f;
  if (gx < W && gy < H) {
    sc = ss[ty + 1][tx + 1];
    keep = sc > thr;
    if (keep) {
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (dx == 0 && dy == 0) continue;
          const float q = ss[ty + 1 + dy][tx + 1 + dx];
          if (!(q > thr)) continue;
          const bool earlier = (dy < 0) || (dy == 0 && dx < 0);
          if (earlier ? !(sc > q) : !(sc >= q)) keep = false;
        }
      }
    }
    keep = keep && gy >= half_patch && gy <= H - half_patch && gx >= half_patch && gx <= W - half_patch;
  }
  const uint64_t mask = __ballot(keep);
  if (mask) {
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&hdr[0], (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (keep) {
      const uint32_t raster = (uint32_t)gy * (uint32_t)W + (uint32_t)gx;
      const uint32_t sb = __float_as_uint(sc);
      cand[base + __popcll(mask & ((1ull << lane) - 1ull))] = ((uint64_t)sb << 32) | (uint64_t)(~raster);
      atomicAdd(&hist[min(sb >> 16, (uint32_t)(kDetHistBins - 1))], 1u);
    }
  }
}

// Find the score bin of rank K (counted from the top), gather candidates of
// that bin and above; the last block finishes the exact selection.
__global__ void __launch_bounds__(256) k_det_select(uint32_t* __restrict__ hdr, const uint32_t* __restrict__ hist,
                                                    const uint64_t* __restrict__ cand, uint64_t* __restrict__ sel,
                                                    uint64_t* __restrict__ fin, uint32_t kmax) {
  __shared__ uint32_t part[256];
  __shared__ uint32_t sh_bin, sh_above, sh_last;
  __shared__ uint32_t lh[4096];
  const uint32_t n = hdr[0];
  const uint32_t k = min(kmax, n);
  // Suffix search: thread t owns bins [PER t, PER t + PER).
  constexpr int PER = kDetHistBins / 256;
  uint32_t sum = 0;
  for (int i = 0; i < PER; ++i) sum += hist[threadIdx.x * PER + i];
  part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t bin = 0, above = 0;
    if (k > 0 && k < n) {
      int c = 255;
      while (c > 0 && above + part[c] < k) above += part[c--];
      int b = c * PER + PER - 1;
      while (b > c * PER && above + hist[b] < k) above += hist[b--];
      bin = (uint32_t)b;
    }
    sh_bin = bin;      // candidates with (score bits >> 16) >= bin are gathered
    sh_above = above;  // count strictly above bin
  }
  __syncthreads();
  const uint32_t bin = sh_bin;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint64_t key = cand[i];
    const bool take = (uint32_t)(key >> 48) >= bin;
    const uint64_t mask = __ballot(take);
    if (mask) {
      const int lane = threadIdx.x & 63;
      const int leader = __ffsll((unsigned long long)mask) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(&hdr[2], (uint32_t)__popcll(mask));
      base = __shfl(base, leader);
      if (take) sel[base + __popcll(mask & ((1ull << lane) - 1ull))] = key;
    }
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) sh_last = (atomicAdd(&hdr[1], 1u) == gridDim.x - 1);
  __syncthreads();
  if (!sh_last) return;
  __threadfence();
  const uint32_t ns = __atomic_load_n(&hdr[2], __ATOMIC_RELAXED);
  // Exact K-th largest key among sel: keys of bins above `bin` are all in;
  // within `bin` select rank (k - above - 1) from the top by 4 levels of 12 bits
  // over the low 48 bits (16 score bits + 32 inverted raster bits).
  uint64_t kth = 0;  // every key >= kth is a winner
  if (k > 0 && k < n) {
    uint32_t r = k - sh_above - 1;  // 0-based rank from the top inside the bin
    uint64_t prefix = bin;           // known high bits
    int known = 16;
    for (int lv = 0; lv < 4; ++lv) {
      const int shift = 64 - known - 12;
      for (int i = threadIdx.x; i < 4096; i += 256) lh[i] = 0u;
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < ns; i += 256) {
        const uint64_t key = __atomic_load_n(&sel[i], __ATOMIC_RELAXED);
        if ((key >> (64 - known)) == prefix) atomicAdd(&lh[(key >> shift) & 4095u], 1u);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t acc = 0;
        int b = 4095;
        while (b > 0 && acc + lh[b] <= r) acc += lh[b--];
        sh_bin = (uint32_t)b;
        sh_above = acc;
      }
      __syncthreads();
      r -= sh_above;
      prefix = (prefix << 12) | sh_bin;
      known += 12;
      __syncthreads();
    }
    kth = prefix;
  }
  // Compact the winners.
  for (uint32_t i0 = 0; i0 < ns; i0 += 256) {
    const uint32_t i = i0 + threadIdx.x;
    uint64_t key = 0;
    bool take = false;
    if (i < ns) {
      key = __atomic_load_n(&sel[i], __ATOMIC_RELAXED);
      take = key >= kth;
    }
    const uint64_t mask = __ballot(take);
    if (mask) {
      const int lane = threadIdx.x & 63;
      const int leader = __ffsll((unsigned long long)mask) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(&hdr[3], (uint32_t)__popcll(mask));
      base = __shfl(base, leader);
      if (take) fin[base + __popcll(mask & ((1ull << lane) - 1ull))] = key;
    }
  }
}

struct KeypointOut {
  int x, y;
  float score;
};

// Output position of each winner = number of winners with a larger key.
__global__ void __launch_bounds__(256) k_det_sort(const uint32_t* __restrict__ hdr, const uint64_t* __restrict__ fin,
                                                  int W, KeypointOut* __restrict__ out, int32_t* __restrict__ n_out) {
  __shared__ uint64_t tile[1024];
  const uint32_t n = hdr[3];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = (int32_t)n;
  if (blockIdx.x * blockDim.x >= n) return;
  const uint64_t mine = i < n ? fin[i] : 0;
  uint32_t rank = 0;
  for (uint32_t t0 = 0; t0 < n; t0 += 1024) {
    const uint32_t cnt = min(1024u, n - t0);
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < cnt; j += 256) tile[j] = fin[t0 + j];
    __syncthreads();
    for (uint32_t j = 0; j < cnt; ++j) rank += tile[j] > mine ? 1u : 0u;
  }
  if (i < n) {
    const uint32_t raster = ~(uint32_t)(mine & 0xffffffffu);
    KeypointOut kp;
    kp.x = (int)(raster % (uint32_t)W);
    kp.y = (int)(raster / (uint32_t)W);
    kp.score = __uint_as_float((uint32_t)(mine >> 32));
    out[rank] = kp;
  }
}

}  // namespace rift2
