// FAST keypoint kernels (Section 2.1 of the paper; Table 1 settings).
//
//   k_det_minmax  per-block min and max of the map (order-preserving uint keys,
//                 16-byte loads) into partials; clears the score histogram
//   k_det_fast    per 32x8 tile: global min / max from the partials,
//                 normalise (correctly rounded FP32 division), FAST-9 score on
//                 the 16-pixel circle, 3x3 NMS with raster tie-break,
//                 patch-border mask; survivors appended as 64-bit keys (score
//                 bits << 32 | ~raster) plus a histogram of the top 16 score bits
//   k_det_bin     one block: candidate total, score bin of rank K and the count
//                 above it (block-wide prefix search)
//   k_det_select1 candidates of that bin and above gathered, one wave per tile
//   k_det_select2 one block: exact K-th key inside the boundary bin (direct
//                 ranking of a small boundary set, else a 4 x 12-bit radix
//                 selection), winners compacted
//   k_det_rank    rank of every winner = number of larger keys, counted over
//                 key chunks in parallel
//   k_det_emit    output record at its rank
// Above kCountSortMin keypoints the all-pairs count is replaced by a counting
// sort over the score bins:
//   k_det_offsets one block: per bin, the number of candidates in the bins
//                 above it (every one a winner for bins at or above the
//                 boundary bin)
//   k_det_group   winners scattered into score-bin order
//   k_det_rank_bins  rank = the bin's offset + the larger keys of its own bin;
//                 output record at its rank
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scan.hpp"

namespace rift2 {

constexpr int kDetHistBins = 1 << 14;  // score bits >> 16 for scores in (0, 1]
constexpr int kTileX = 32, kTileY = 8;
constexpr int kHalo = 4;  // FAST radius 3 + NMS 1

// Header words (written per call): [0] candidates, [3] winners, [8] boundary
// bin, [9] candidates above it.
constexpr int kMinMaxBlocks = 256;  // == k_det_fast's block size: one partial per thread

__device__ __forceinline__ uint32_t float_order_key(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float float_from_order_key(uint32_t k) {
  const uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(b);
}

__global__ void __launch_bounds__(256) k_det_minmax(const float* __restrict__ d, int n, uint32_t* __restrict__ mm,
                                                    uint32_t* __restrict__ hist) {
  __shared__ uint32_t red[2][4];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < kDetHistBins; i += gridDim.x * 256) hist[i] = 0u;
  uint32_t lo = 0xffffffffu, hi = 0u;
  const int n4 = n / 4;  // the map is 16-byte aligned (checked on the host)
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n4; i += gridDim.x * 256) {
    const float4 v = ((const float4*)d)[i];
    const uint32_t k[4] = {float_order_key(v.x), float_order_key(v.y), float_order_key(v.z), float_order_key(v.w)};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      lo = min(lo, k[e]);
      hi = max(hi, k[e]);
    }
  }
  for (int i = 4 * n4 + blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const uint32_t k = float_order_key(d[i]);
    lo = min(lo, k);
    hi = max(hi, k);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, off));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, off));
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = lo;
    red[1][threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      lo = min(lo, red[0][w]);
      hi = max(hi, red[1][w]);
    }
    mm[2 * blockIdx.x] = lo;
    mm[2 * blockIdx.x + 1] = hi;
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

// A tile keeps at most (kTileX/2) (kTileY/2) points: survivors of the 3x3
// suppression are never 8-neighbours.
constexpr int kTileCap = (kTileX / 2) * (kTileY / 2);

static_assert(kTileX * kTileY == kMinMaxBlocks, "one min/max partial per k_det_fast thread");

constexpr int kLX = kTileX + 2 * kHalo, kLY = kTileY + 2 * kHalo;
constexpr int kSX = kTileX + 2, kSY = kTileY + 2;

// One map's FAST stage for this block's tile: global min / max from the
// kMinMaxBlocks partials `mm`, the normalised tile plus halo in `sd`, scores
// of the tile plus a one-pixel ring in `ss`, then 3x3 suppression and the
// patch-border mask.  Returns whether this thread's pixel survives, with its
// score in `sc`.  A flat map (max == min) has no keypoints.  Every thread of
// the block must call it (it holds barriers).
__device__ __forceinline__ bool tile_fast(const float* __restrict__ d, int H, int W, float thr, int half_patch,
                                          const uint32_t* __restrict__ mm, float (&sd)[kLY][kLX],
                                          float (&ss)[kSY][kSX], uint32_t (&s_red)[2][4], float& sc) {
  uint32_t klo = mm[2 * threadIdx.x], khi = mm[2 * threadIdx.x + 1];
  for (int off = 32; off > 0; off >>= 1) {
    klo = min(klo, (uint32_t)__shfl_xor((int)klo, off));
    khi = max(khi, (uint32_t)__shfl_xor((int)khi, off));
  }
  __syncthreads();  // s_red may still be read by a previous call
  if ((threadIdx.x & 63) == 0) {
    s_red[0][threadIdx.x >> 6] = klo;
    s_red[1][threadIdx.x >> 6] = khi;
  }
  __syncthreads();
  klo = min(min(s_red[0][0], s_red[0][1]), min(s_red[0][2], s_red[0][3]));
  khi = max(max(s_red[1][0], s_red[1][1]), max(s_red[1][2], s_red[1][3]));
  const float lo = float_from_order_key(klo);
  const float hi = float_from_order_key(khi);
  sc = 0.0f;
  if (!(hi > lo)) return false;  // uniform across the grid
  const float rng = __fsub_rn(hi, lo);
  const int x0 = blockIdx.x * kTileX - kHalo, y0 = blockIdx.y * kTileY - kHalo;
  for (int i = threadIdx.x; i < kLX * kLY; i += blockDim.x) {
    const int ly = i / kLX, lx = i % kLX;
    const int gy = y0 + ly, gx = x0 + lx;
    float v = 0.0f;
    if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = __fdiv_rn(__fsub_rn(d[(size_t)gy * W + gx], lo), rng);
    sd[ly][lx] = v;
  }
  __syncthreads();
  // scores of the tile plus a one-pixel ring
  for (int i = threadIdx.x; i < kSX * kSY; i += blockDim.x) {
    const int sy = i / kSX, sx = i % kSX;
    const int gy = y0 + kHalo - 1 + sy, gx = x0 + kHalo - 1 + sx;
    float v = 0.0f;
    if (gy >= 3 && gy <= H - 4 && gx >= 3 && gx <= W - 4) {
      const int cy = sy + kHalo - 1, cx = sx + kHalo - 1;
      const float c[16] = {sd[cy - 3][cx], sd[cy - 3][cx + 1], sd[cy - 2][cx + 2], sd[cy - 1][cx + 3],
                           sd[cy][cx + 3],     sd[cy + 1][cx + 3], sd[cy + 2][cx + 2], sd[cy + 3][cx + 1],
                           sd[cy + 3][cx],     sd[cy + 3][cx - 1], sd[cy + 2][cx - 2], sd[cy + 1][cx - 3],
                           sd[cy][cx - 3],     sd[cy - 1][cx - 3], sd[cy - 2][cx - 2], sd[cy - 3][cx - 1]};
      v = fast_score(c, sd[cy][cx]);
    }
    ss[sy][sx] = v;
  }
  __syncthreads();
  const int tx = threadIdx.x % kTileX, ty = threadIdx.x / kTileX;
  const int gx = blockIdx.x * kTileX + tx, gy = blockIdx.y * kTileY + ty;
  bool keep = false;
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
  return keep;
}

// Appends the block's surviving pixels (score sc) to the slots of list
// `tile`, counted in s_count, plus the score histogram.
__device__ __forceinline__ void tile_append(bool keep, float sc, int W, int tile, uint32_t* s_count,
                                            uint32_t* __restrict__ hist, uint64_t* __restrict__ cand) {
  const uint64_t mask = __ballot(keep);
  if (!mask) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(s_count, (uint32_t)__popcll(mask));
  base = __shfl(base, leader);
  if (keep) {
    const int gx = blockIdx.x * kTileX + (int)(threadIdx.x % kTileX);
    const int gy = blockIdx.y * kTileY + (int)(threadIdx.x / kTileX);
    const uint32_t raster = (uint32_t)gy * (uint32_t)W + (uint32_t)gx;
    const uint32_t sb = __float_as_uint(sc);
    cand[(size_t)tile * kTileCap + base + __popcll(mask & ((1ull << lane) - 1ull))] =
        ((uint64_t)sb << 32) | (uint64_t)(~raster);
    atomicAdd(&hist[min(sb >> 16, (uint32_t)(kDetHistBins - 1))], 1u);
  }
}

__global__ void __launch_bounds__(kTileX * kTileY) k_det_fast(const float* __restrict__ d, int H, int W, float thr,
                                                              int half_patch, const uint32_t* __restrict__ mm,
                                                              uint32_t* __restrict__ hist, uint32_t* __restrict__ tile_cnt,
                                                              uint64_t* __restrict__ cand) {
  __shared__ float sd[kLY][kLX];
  __shared__ float ss[kSY][kSX];
  __shared__ uint32_t s_count;
  __shared__ uint32_t s_red[2][4];
  const int tile = blockIdx.y * gridDim.x + blockIdx.x;
  if (threadIdx.x == 0) s_count = 0u;
  float sc;
  const bool keep = tile_fast(d, H, W, thr, half_patch, mm, sd, ss, s_red, sc);
  tile_append(keep, sc, W, tile, &s_count, hist, cand);
  __syncthreads();
  if (threadIdx.x == 0) tile_cnt[tile] = s_count;
}

// RIFT's detector (Section 2.1): FAST points on the maximum-moment map
// (edges) and on the minimum-moment map (corners), each map with its own
// normalisation, scores and suppression, then their union.  A pixel kept on
// both maps appears once, in the first map's list, with the larger score;
// the second map's other survivors go to list n_tiles + tile.  Each list is
// one map's suppression survivors, so kTileCap bounds both.
__global__ void __launch_bounds__(kTileX * kTileY) k_det_fast_union(const float* __restrict__ d_edge,
                                                                    const float* __restrict__ d_corner, int H, int W,
                                                                    float thr, int half_patch,
                                                                    const uint32_t* __restrict__ mm_edge,
                                                                    const uint32_t* __restrict__ mm_corner,
                                                                    uint32_t* __restrict__ hist,
                                                                    uint32_t* __restrict__ tile_cnt,
                                                                    uint64_t* __restrict__ cand) {
  __shared__ float sd[kLY][kLX];
  __shared__ float ss[kSY][kSX];
  __shared__ uint32_t s_count[2];
  __shared__ uint32_t s_red[2][4];
  const int tile = blockIdx.y * gridDim.x + blockIdx.x;
  const int n_tiles = gridDim.x * gridDim.y;
  if (threadIdx.x == 0) {
    s_count[0] = 0u;
    s_count[1] = 0u;
  }
  float sc_e, sc_c;
  const bool keep_e = tile_fast(d_edge, H, W, thr, half_patch, mm_edge, sd, ss, s_red, sc_e);
  const bool keep_c = tile_fast(d_corner, H, W, thr, half_patch, mm_corner, sd, ss, s_red, sc_c);
  const float sc_first = keep_c ? fmaxf(sc_e, sc_c) : sc_e;
  tile_append(keep_e, sc_first, W, tile, &s_count[0], hist, cand);
  tile_append(keep_c && !keep_e, sc_c, W, n_tiles + tile, &s_count[1], hist, cand);
  __syncthreads();
  if (threadIdx.x == 0) {
    tile_cnt[tile] = s_count[0];
    tile_cnt[n_tiles + tile] = s_count[1];
  }
}

// One block: candidate total n, the score bin holding the candidate of rank
// min(K, n) - 1 from the top, and the number of candidates above that bin,
// published in hdr[0], [8], [9] (bin 0 / above 0 when every candidate wins).
constexpr int kSelBlocks = 256;

__global__ void __launch_bounds__(1024) k_det_bin(uint32_t* __restrict__ hdr, const uint32_t* __restrict__ hist,
                                                  uint32_t kmax) {
  __shared__ uint32_t scratch[16];
  __shared__ int sh_bin;
  __shared__ uint32_t sh_above, sh_total;
  constexpr int PER = kDetHistBins / 1024;
  // one scan from the top bin down gives the total and, once the total fixes
  // K, the bin of the K-th strongest key (its thread holds the bins in registers)
  uint32_t c[PER];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    c[i] = hist[kDetHistBins - 1 - (threadIdx.x * PER + i)];
    sum += c[i];
  }
  const uint32_t incl = block_inclusive_scan<1024>(sum, scratch);
  const uint32_t excl = incl - sum;
  if (threadIdx.x == 1023) sh_total = incl;
  if (threadIdx.x == 0) {
    sh_bin = 0;
    sh_above = 0;
  }
  __syncthreads();
  const uint32_t n = sh_total;
  const uint32_t k = min(kmax, n);
  if (k > 0 && k < n) {
    const uint32_t r = k - 1;
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
      sh_bin = kDetHistBins - 1 - (int)(threadIdx.x * PER + hit);
      sh_above = acc_hit;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    hdr[0] = n;
    hdr[8] = (uint32_t)sh_bin;
    hdr[9] = sh_above;
  }
}

// Every candidate of the boundary bin and above is copied into this block's
// region of `sel` (region b holds the slots of the tiles block b scans, so it
// cannot overflow); one wave reads one tile's compacted candidates.
__global__ void __launch_bounds__(256) k_det_select1(const uint32_t* __restrict__ hdr,
                                                     const uint32_t* __restrict__ tile_cnt, int n_tiles,
                                                     const uint64_t* __restrict__ cand, uint64_t* __restrict__ sel,
                                                     uint32_t* __restrict__ sel_cnt) {
  __shared__ uint32_t s_count;
  if (threadIdx.x == 0) s_count = 0u;
  __syncthreads();
  const uint32_t bin = hdr[8];
  const int per = (n_tiles + (int)gridDim.x - 1) / (int)gridDim.x;
  const int t0 = blockIdx.x * per;
  const int t1 = min(n_tiles, t0 + per);
  uint64_t* region = sel + (size_t)t0 * kTileCap;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  static_assert(kTileCap == 64, "one lane per candidate slot of a tile");
  // four tiles per wave per round: the counts, then the keys, are loaded
  // together before any is used
  for (int tb = t0 + wave; tb < t1; tb += 16) {
    uint32_t cnt[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) cnt[u] = tb + 4 * u < t1 ? tile_cnt[tb + 4 * u] : 0u;
    uint64_t key[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) key[u] = (uint32_t)lane < cnt[u] ? cand[(size_t)(tb + 4 * u) * kTileCap + lane] : 0ull;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool take = (uint32_t)lane < cnt[u] && (uint32_t)(key[u] >> 48) >= bin;
      const uint64_t mask = __ballot(take);
      if (mask) {
        const int leader = __ffsll((unsigned long long)mask) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&s_count, (uint32_t)__popcll(mask));
        base = __shfl(base, leader);
        if (take) region[base + __popcll(mask & ((1ull << lane) - 1ull))] = key[u];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) sel_cnt[blockIdx.x] = s_count;
}

constexpr int kEdgeMax = 4096;
constexpr uint32_t kEdgeDirect = 512;  // boundary sets up to this size are ranked directly

// One block of 1024 threads: exact K-th key inside the boundary bin, then the
// winners (keys >= K-th key) compacted into `fin` (exactly min(K, n) keys,
// the keys being distinct).
// Key `i` of the concatenation of the select1 regions (sizes sel_cnt, prefix
// sums in `pre`, pre[kSelBlocks] = total).
__device__ __forceinline__ uint64_t sel_key(const uint64_t* __restrict__ sel, const uint32_t* pre, uint32_t region_size,
                                            uint32_t i) {
  int lo = 0, hi = kSelBlocks - 1;  // last region with pre[r] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return sel[(size_t)lo * region_size + (i - pre[lo])];
}

__global__ void __launch_bounds__(1024) k_det_select2(uint32_t* __restrict__ hdr, const uint64_t* __restrict__ sel,
                                                      const uint32_t* __restrict__ sel_cnt, uint32_t region_size,
                                                      uint64_t* __restrict__ fin, uint32_t kmax) {
  __shared__ uint32_t scratch[1024];
  __shared__ uint32_t lh[4096];
  __shared__ uint64_t edge[kEdgeMax];
  __shared__ uint32_t pre[kSelBlocks + 1];
  __shared__ uint32_t n_edge, s_final;
  __shared__ uint64_t s_kth;
  __shared__ int sh_b;
  __shared__ uint32_t sh_before;
  const uint32_t n = hdr[0];
  const uint32_t k = min(kmax, n);
  const uint64_t bin = hdr[8];
  static_assert(kSelBlocks <= 1024, "one region count per thread");
  if (threadIdx.x == 0) {
    n_edge = 0;
    s_final = 0;
  }
  {
    // region offsets: exclusive prefix sums of the region counts
    const uint32_t c = threadIdx.x < kSelBlocks ? sel_cnt[threadIdx.x] : 0u;
    const uint32_t incl = block_inclusive_scan<1024>(c, scratch);
    if (threadIdx.x < kSelBlocks) pre[threadIdx.x] = incl - c;
    if (threadIdx.x == kSelBlocks - 1) pre[kSelBlocks] = incl;
  }
  __syncthreads();
  const uint32_t ns = pre[kSelBlocks];
  uint64_t kth = 0;
  if (k > 0 && k < n) {
    // four keys per thread per round: their loads are in flight together
    for (uint32_t i0 = 0; i0 < ns; i0 += 4 * 1024) {
      uint64_t key[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t i = i0 + e * 1024 + threadIdx.x;
        key[e] = i < ns ? sel_key(sel, pre, region_size, i) : 0ull;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (i0 + e * 1024 + threadIdx.x < ns && (key[e] >> 48) == bin) {
          const uint32_t pos = atomicAdd(&n_edge, 1u);
          if (pos < kEdgeMax) edge[pos] = key[e];
        }
      }
    }
    __syncthreads();
    const uint32_t ne = n_edge;
    const bool staged = ne <= kEdgeMax;
    uint32_t r = k - hdr[9] - 1;  // rank from the top inside the bin
    uint64_t prefix = bin;
    int known = 16;
    if (ne <= kEdgeDirect) {
      // small boundary set: every key's rank among the others (the keys are distinct)
      if (threadIdx.x < ne) {
        const uint64_t mine = edge[threadIdx.x];
        uint32_t above = 0;
        for (uint32_t j = 0; j < ne; ++j) above += edge[j] > mine ? 1u : 0u;
        if (above == r) s_kth = mine;
      }
      __syncthreads();
      prefix = s_kth;
      known = 64;
    }
    for (int lv = 0; lv < 4 && known < 64; ++lv) {
      const int shift = 64 - known - 12;
      for (int i = threadIdx.x; i < 4096; i += 1024) lh[i] = 0u;
      __syncthreads();
      const uint32_t cnt = staged ? ne : ns;
      for (uint32_t i = threadIdx.x; i < cnt; i += 1024) {
        const uint64_t key = staged ? edge[i] : sel_key(sel, pre, region_size, i);
        if ((key >> (64 - known)) == prefix) atomicAdd(&lh[(key >> shift) & 4095u], 1u);
      }
      __syncthreads();
      block_find_rank<4096, 1024, true>(lh, r, &sh_b, &sh_before, scratch);
      r -= sh_before;
      prefix = (prefix << 12) | (uint64_t)sh_b;
      known += 12;
    }
    kth = prefix;
  }
  for (uint32_t i0 = 0; i0 < ns; i0 += 4 * 1024) {
    uint64_t key[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t i = i0 + e * 1024 + threadIdx.x;
      key[e] = i < ns ? sel_key(sel, pre, region_size, i) : 0ull;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const bool take = i0 + e * 1024 + threadIdx.x < ns && key[e] >= kth;
      const uint64_t mask = __ballot(take);
      if (mask) {
        const int lane = threadIdx.x & 63;
        const int leader = __ffsll((unsigned long long)mask) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&s_final, (uint32_t)__popcll(mask));
        base = __shfl(base, leader);
        if (take) fin[base + __popcll(mask & ((1ull << lane) - 1ull))] = key[e];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) hdr[3] = s_final;
}

struct KeypointOut {
  int x, y;
  float score;
};

// Partial ranks: grid = (ceil(kmax / 256), S); block y counts, for each of its
// 256 winners, the larger keys among winners [y n / S, (y + 1) n / S).
__global__ void __launch_bounds__(256) k_det_rank(const uint32_t* __restrict__ hdr, const uint64_t* __restrict__ fin,
                                                  uint32_t* __restrict__ part, uint32_t kmax) {
  __shared__ uint64_t tile[1024];
  const uint32_t n = hdr[3];
  if (blockIdx.x * 256 >= n) return;
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  const uint64_t mine = i < n ? fin[i] : 0;
  const uint32_t beg = (uint32_t)((uint64_t)n * blockIdx.y / gridDim.y);
  const uint32_t end = (uint32_t)((uint64_t)n * (blockIdx.y + 1) / gridDim.y);
  uint32_t rank = 0;
  for (uint32_t t0 = beg; t0 < end; t0 += 1024) {
    const uint32_t cnt = min(1024u, end - t0);
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < cnt; j += 256) tile[j] = fin[t0 + j];
    __syncthreads();
#pragma unroll 8
    for (uint32_t j = 0; j < cnt; ++j) rank += tile[j] > mine ? 1u : 0u;
  }
  if (i < n) part[(size_t)blockIdx.y * kmax + i] = rank;
}

__global__ void __launch_bounds__(256) k_det_emit(const uint32_t* __restrict__ hdr, const uint64_t* __restrict__ fin,
                                                  const uint32_t* __restrict__ part, int n_part, uint32_t kmax, int W,
                                                  KeypointOut* __restrict__ out, int32_t* __restrict__ n_out) {
  const uint32_t n = hdr[3];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = (int32_t)n;
  if (i >= n) return;
  // eight independent partial sums: the loads are issued together instead of
  // one latency after another
  uint32_t acc[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
  int s = 0;
  for (; s + 8 <= n_part; s += 8) {
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] += part[(size_t)(s + e) * kmax + i];
  }
  for (; s < n_part; ++s) acc[0] += part[(size_t)s * kmax + i];
  const uint32_t rank = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  const uint64_t key = fin[i];
  const uint32_t raster = ~(uint32_t)(key & 0xffffffffu);
  KeypointOut kp;
  kp.x = (int)(raster % (uint32_t)W);
  kp.y = (int)(raster / (uint32_t)W);
  kp.score = __uint_as_float((uint32_t)(key >> 32));
  out[rank] = kp;
}

// ---- counting sort of the winners by score bin (large K)

// The all-pairs ranking costs K^2 comparisons; from this many keypoints on,
// the winners are sorted by score bin instead (measured at 1024^2 with 5000
// keypoints the all-pairs form is faster, 58.7 against 68.3 us for the
// detection; at 2048^2 / 20000 and 4096^2 / 50000 the counting sort is faster,
// 162 against 176 us and 491 against 744 us).
constexpr uint32_t kCountSortMin = 12000;

// One block: above[b] = candidates in the score bins above b, and the
// scatter cursors, which start there.
__global__ void __launch_bounds__(1024) k_det_offsets(const uint32_t* __restrict__ hist, uint32_t* __restrict__ above,
                                                      uint32_t* __restrict__ cursor) {
  __shared__ uint32_t scratch[16];
  constexpr int PER = kDetHistBins / 1024;
  const int top = kDetHistBins - 1 - (int)threadIdx.x * PER;  // this thread's bins, descending
  uint32_t c[PER];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    c[i] = hist[top - i];
    sum += c[i];
  }
  uint32_t acc = block_inclusive_scan<1024>(sum, scratch) - sum;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    above[top - i] = acc;
    cursor[top - i] = acc;
    acc += c[i];
  }
}

// Each winner takes the next slot of its score bin (bins ordered from the top).
__global__ void __launch_bounds__(256) k_det_group(const uint32_t* __restrict__ hdr, const uint64_t* __restrict__ fin,
                                                   uint32_t* __restrict__ cursor, uint64_t* __restrict__ grouped) {
  const uint32_t n = hdr[3];
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t key = fin[i];
  grouped[atomicAdd(&cursor[(uint32_t)(key >> 48)], 1u)] = key;
}

// Rank of a winner = the winners in higher score bins (its bin's offset) +
// the larger keys of its own bin, which holds the winners between the bin's
// offset and the next bin's: all of the bin's candidates above the boundary
// bin, the rest of the winners in the boundary bin.  The record goes to its
// rank.
__global__ void __launch_bounds__(256) k_det_rank_bins(const uint32_t* __restrict__ hdr,
                                                       const uint64_t* __restrict__ grouped,
                                                       const uint32_t* __restrict__ above,
                                                       const uint32_t* __restrict__ hist, int W,
                                                       KeypointOut* __restrict__ out, int32_t* __restrict__ n_out) {
  const uint32_t n = hdr[3];
  const uint32_t bbin = hdr[8];
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = (int32_t)n;
  if (i >= n) return;
  const uint64_t key = grouped[i];
  const uint32_t b = (uint32_t)(key >> 48);
  const uint32_t lo = above[b];
  const uint32_t hi = b == bbin ? n : lo + hist[b];
  // eight independent counts, so the loads of a chunk are issued together
  uint32_t cnt[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
  uint32_t q = lo;
  for (; q + 8 <= hi; q += 8) {
#pragma unroll
    for (int e = 0; e < 8; ++e) cnt[e] += grouped[q + e] > key ? 1u : 0u;
  }
  for (; q < hi; ++q) cnt[0] += grouped[q] > key ? 1u : 0u;
  const uint32_t rank = lo + ((cnt[0] + cnt[1]) + (cnt[2] + cnt[3])) + ((cnt[4] + cnt[5]) + (cnt[6] + cnt[7]));
  const uint32_t raster = ~(uint32_t)(key & 0xffffffffu);
  KeypointOut kp;
  kp.x = (int)(raster % (uint32_t)W);
  kp.y = (int)(raster / (uint32_t)W);
  kp.score = __uint_as_float((uint32_t)(key >> 32));
  out[rank] = kp;
}

}  // namespace rift2
