// Brute-force descriptor matching (Section 4: nearest feature distance) with a
// second-neighbour ratio test.
//
//   k_match_prep   counts -> zero-padded GEMM tables (BF16 bits or FP32),
//                  per-keypoint best slots reset
//   k_match_gemm   MFMA distance tiles (32 candidates x 32 queries per wave
//                  step, candidate tiles shared by the block through LDS)
//                  with a fused per-query top-3 in registers; rows of B are
//                  split into slices across blocks
//   k_match_merge  per A row: merge the slice/half-wave top-3 lists, nearest
//                  row j1, nearest row of another B keypoint j2, ratio test,
//                  per-keypoint best by a 64-bit atomic min of (d2, row)
//   k_match_emit   accepted keypoints in ascending order -> output records
//
// All dot products are exact: counts <= 256 are exact in BF16, and FP32
// accumulation of integer products stays exact below 2^24.  The squared
// distance is then evaluated identically in both precisions:
// t = fl(fl(dot * ia) * ib), d2 = fl(2 - 2 t).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scan.hpp"

namespace rift2 {

constexpr int kTopK = 3;  // a keypoint owns <= 2 rows, so 3 rows hold j1 and j2

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx16_t __attribute__((ext_vector_type(16)));
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint16_t bf16_bits_of_count(uint32_t c) {
  // round to nearest even; exact for c <= 256
  const uint32_t f = __float_as_uint((float)c);
  return (uint16_t)((f + 0x7fffu + ((f >> 16) & 1u)) >> 16);
}

// Table layout: rows_pad x RS elements (BF16 bits as uint16, or float); RS is the
// MFMA depth plus a zero pad that staggers the rows over the LDS banks.  One
// work item = CH consecutive elements of a row (8 for BF16: 16-byte load and
// store; 4 for FP32: 8-byte load, 16-byte store; D and RS are multiples).
// One table of a match call: its counts, actual row count and capacity, the
// padded table it fills, and (table A only) the per-keypoint best slots.
struct PrepJob {
  const uint16_t* desc;
  const int32_t* n_dev;
  int cap, rows_pad;
  void* table;
  uint64_t* best;
  int n_best;
};

// Both tables of a match call in one launch: blockIdx.y picks the table.
template <bool BF16>
__global__ void __launch_bounds__(256) k_match_prep(PrepJob ja, PrepJob jb, int D, int RS) {
  const PrepJob j = blockIdx.y ? jb : ja;
  const uint16_t* __restrict__ desc = j.desc;
  constexpr int CH = BF16 ? 8 : 4;
  const int n = min(*j.n_dev, j.cap);
  const int chunks = RS / CH;
  const size_t total = (size_t)j.rows_pad * chunks;
  for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < total; w += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(w / chunks), k0 = CH * (int)(w % chunks);
    const bool in = r < n && k0 < D;
    if (BF16) {
      uint4 raw = make_uint4(0u, 0u, 0u, 0u);
      if (in) raw = *(const uint4*)(desc + (size_t)r * D + k0);
      const uint32_t word[4] = {raw.x, raw.y, raw.z, raw.w};
      uint32_t o[4];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        o[e] = (uint32_t)bf16_bits_of_count(word[e] & 0xffffu) | ((uint32_t)bf16_bits_of_count(word[e] >> 16) << 16);
      *(uint4*)((uint16_t*)j.table + (size_t)r * RS + k0) = make_uint4(o[0], o[1], o[2], o[3]);
    } else {
      uint2 raw = make_uint2(0u, 0u);
      if (in) raw = *(const uint2*)(desc + (size_t)r * D + k0);
      *(float4*)((float*)j.table + (size_t)r * RS + k0) =
          make_float4((float)(raw.x & 0xffffu), (float)(raw.x >> 16), (float)(raw.y & 0xffffu), (float)(raw.y >> 16));
    }
  }
  if (j.best) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < j.n_best; i += gridDim.x * blockDim.x) j.best[i] = ~0ull;
  }
}

struct Top3 {
  float d[kTopK];
  int j[kTopK];
};

__device__ __forceinline__ void top3_insert(Top3& t, float d, int j) {
  if (d < t.d[2]) {
    if (d < t.d[1]) {
      t.d[2] = t.d[1];
      t.j[2] = t.j[1];
      if (d < t.d[0]) {
        t.d[1] = t.d[0];
        t.j[1] = t.j[0];
        t.d[0] = d;
        t.j[0] = j;
      } else {
        t.d[1] = d;
        t.j[1] = j;
      }
    } else {
      t.d[2] = d;
      t.j[2] = j;
    }
  }
}

// Epilogue of one 32x32 tile: lane holds 16 candidate dots of its query.
// Accumulator register r of lane l is candidate row 8 (r/4) + 4 (l/32) + r%4;
// `ibt` holds the tile's 32 candidate inverse norms (LDS), so the four rows
// 8k + 4g .. 8k + 4g + 3 of register group k are one 16-byte read.  All 16
// distances are formed first; the insertion runs only where one of them can
// enter the lane's top 3.  CF (candidate first) multiplies by the candidate's
// inverse norm before the query's: the reverse pass of the mutual check (B rows
// as queries) then forms exactly the d2 of the forward pass, fl(fl(dot ia) ib)
// with ia the A row's and ib the B row's inverse norm.
template <bool CF = false>
__device__ __forceinline__ void tile_epilogue(const floatx16_t& acc, int lane, int j0, int j_end, float ia,
                                              const float* ibt, Top3& top) {
  const int g = lane >> 5;
  float d2[16];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float4 ib4 = *(const float4*)(ibt + 8 * k + 4 * g);
    const float ibv[4] = {ib4.x, ib4.y, ib4.z, ib4.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 4 * k + e;
      const float t2 = CF ? __fmul_rn(__fmul_rn(acc[r], ibv[e]), ia) : __fmul_rn(__fmul_rn(acc[r], ia), ibv[e]);
      // 2 t2 is exact, so one fused rounding equals fl(2 - fl(2 t2))
      d2[r] = __fmaf_rn(-2.0f, t2, 2.0f);
    }
  }
  const bool full = j0 + 32 <= j_end;  // uniform: only a slice's last tile is partial
  bool any = false;
  if (full) {
    float mn = d2[0];
#pragma unroll
    for (int r = 1; r < 16; ++r) mn = fminf(mn, d2[r]);
    any = mn < top.d[2];
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r) any |= (j0 + 8 * (r >> 2) + 4 * g + (r & 3) < j_end) && d2[r] < top.d[2];
  }
  if (!any) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int j = j0 + 8 * (r >> 2) + 4 * g + (r & 3);
    if (j < j_end && d2[r] < top.d[2]) top3_insert(top, d2[r], j);
  }
}

// Candidate tiles of 32 rows are copied from the table straight into LDS
// (global_load_lds, no staging registers; the BF16 kernel double buffers, so
// the next tile's copy is in flight while the current one is multiplied) and
// read by the block's 4 waves, each holding 32 queries in registers.  The
// table rows already carry the LDS row stride RS, so a tile is one contiguous
// block.  The FP32 and FP8 grids are (ceil(rows_a / 128), S); the BF16 grid
// is one-dimensional (gemm_cell).
template <typename TE, int RS>
struct TileCopy {
  static constexpr int BYTES = 32 * RS * (int)sizeof(TE);
  static constexpr int CHUNKS = BYTES / 16;          // 16-byte pieces per tile
  static constexpr int ROUNDS = (CHUNKS + 255) / 256;  // copies per thread
  static_assert(BYTES % 16 == 0, "16-byte rows");
};

template <typename TE, int RS>
__device__ __forceinline__ void tile_copy(const TE* __restrict__ tb, int j0, TE* tile) {
  using C = TileCopy<TE, RS>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const char* src = (const char*)(tb + (size_t)j0 * RS);
#pragma unroll
  for (int q = 0; q < C::ROUNDS; ++q) {
    const int first = (q * 4 + wave) * 64;  // this wave's first piece in round q
    if (first + lane < C::CHUNKS)
      __builtin_amdgcn_global_load_lds((const void*)(src + 16 * (first + lane)),
                                       (__attribute__((address_space(3))) void*)((char*)tile + 16 * first), 16, 0, 0);
  }
}

// Waits for this wave's tile copies to land in LDS (the block barrier that
// follows publishes them).
__device__ __forceinline__ void tile_copy_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// The tile's candidate inverse norms (zero past the last row) go to LDS with
// the tile itself.
__device__ __forceinline__ float tile_inv_load(const float* __restrict__ inv_b, int j0, int nb) {
  const int j = j0 + (int)threadIdx.x;
  return (threadIdx.x < 32 && j < nb) ? inv_b[j] : 0.0f;
}

template <int DP>
constexpr int bf16_stride() { return DP + 8; }  // rows start 16 bytes apart modulo 128
template <int DP>
constexpr int f32_stride() { return DP + 4; }

// Products of one 32-candidate tile with the wave's 32 queries.  Each
// candidate fragment is read from LDS PF MFMAs ahead of its use, so the LDS
// latency overlaps the dependent MFMA chain instead of preceding every MFMA.
template <int KS, int RS>
__device__ __forceinline__ floatx16_t bf16_tile_products(const uint16_t* tile, int lane, const bf16x8_t* qa) {
  constexpr int PF = KS < 4 ? KS : 4;
  const uint16_t* crow = tile + (lane & 31) * RS + 8 * (lane >> 5);
  uint4 fr[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) fr[p] = *(const uint4*)(crow + 16 * p);
  floatx16_t acc = {};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const uint4 cur = fr[ks % PF];
    if (ks + PF < KS) fr[ks % PF] = *(const uint4*)(crow + 16 * (ks + PF));
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, cur), qa[ks], acc, 0, 0, 0);
  }
  return acc;
}

// The two tile buffers are separate LDS objects and the loop body is written
// out once per buffer, so every read names a buffer that the copy in flight
// does not write: the compiler then lets the next tile's copy run under the
// current tile's products instead of waiting for it before the first read.
// Which (query block, slice) a block of the GEMM grid computes.  Blocks are
// dealt to the 8 XCDs round robin by their linear id, and each XCD has its
// own L2; so XCD x works only on half x / 4 of the actual query blocks
// against quarter x % 4 of the actual candidate slices (about 1.4 + 1.1 MB of
// BF16 tables at 1024^2 / 5000 keypoints), which its L2 holds, instead of
// streaming all of B past every L2.  The halves and quarters are cut from
// the device-side row counts, so every XCD gets the same share whatever the
// capacities; blocks beyond their XCD's share leave at once.  The grid is
// 8 * ceil(query blocks of the capacity / 2) * ceil(slices / 4).
struct GemmCell {
  int qb, slice, n_slices_act;
  bool ok;
};

__device__ __forceinline__ GemmCell gemm_cell(int na, int nb, int slice_rows, int slices) {
  GemmCell c;
  const int nqb = (na + 127) / 128;
  // a candidate count of zero still has one (empty) slice, which writes the lists
  c.n_slices_act = max(1, min(slices, (nb + slice_rows - 1) / slice_rows));
  const int xcd = (int)(blockIdx.x & 7u), w = (int)(blockIdx.x >> 3);
  const int ha = xcd >> 2, hb = xcd & 3;
  const int q_lo = ha * nqb / 2, q_n = (ha + 1) * nqb / 2 - q_lo;
  const int s_lo = hb * c.n_slices_act / 4, s_n = (hb + 1) * c.n_slices_act / 4 - s_lo;
  c.ok = q_n > 0 && w < q_n * s_n;
  c.qb = c.ok ? q_lo + w % q_n : 0;
  c.slice = c.ok ? s_lo + w / q_n : 0;
  return c;
}

template <int DP, bool CF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_match_gemm_bf16(const uint16_t* __restrict__ ta, const float* __restrict__ inv_a,
                                                         const int32_t* __restrict__ na_dev,
                                                         const uint16_t* __restrict__ tb, const float* __restrict__ inv_b,
                                                         const int32_t* __restrict__ nb_dev, int cap_a, int cap_b,
                                                         int slice_rows, int slices, int2* __restrict__ part) {
  static_assert(DP % 16 == 0, "padded depth");
  constexpr int KS = DP / 16;
  constexpr int RS = bf16_stride<DP>();
  __shared__ __attribute__((aligned(16))) uint16_t tile0[32 * RS];
  __shared__ __attribute__((aligned(16))) uint16_t tile1[32 * RS];
  __shared__ __attribute__((aligned(16))) float ibt0[32];
  __shared__ __attribute__((aligned(16))) float ibt1[32];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 5;
  const int na = min(*na_dev, cap_a), nb = min(*nb_dev, cap_b);
  // blocks without a cell leave at once (uniformly, before any barrier)
  const GemmCell cell = gemm_cell(na, nb, slice_rows, slices);
  if (!cell.ok) return;
  const int q0 = (cell.qb * 4 + wave) * 32;
  const bool active = q0 < na;
  const int qi = q0 + (lane & 31);
  bf16x8_t qa[KS];
  if (active) {
    const uint16_t* qrow = ta + (size_t)qi * RS + 8 * g;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) qa[ks] = __builtin_bit_cast(bf16x8_t, *(const uint4*)(qrow + 16 * ks));
  }
  const float ia = (active && qi < na) ? inv_a[qi] : 0.0f;
  const int j_beg = cell.slice * slice_rows;
  const int j_end = min(nb, j_beg + slice_rows);
  const int ntile = j_end > j_beg ? (j_end - j_beg + 31) / 32 : 0;
  Top3 top;
#pragma unroll
  for (int q = 0; q < kTopK; ++q) {
    top.d[q] = INFINITY;
    top.j[q] = -1;
  }
  if (ntile > 0) {
    tile_copy<uint16_t, RS>(tb, j_beg, tile0);
    const float ib0 = tile_inv_load(inv_b, j_beg, nb);
    if (threadIdx.x < 32) ibt0[threadIdx.x] = ib0;
    tile_copy_wait();
  }
  __syncthreads();
  // tile `it` is in (tc, ic); tile it + 1 goes to (tn, in) meanwhile
  auto step = [&](int it, const uint16_t* tc, uint16_t* tn, const float* ic, float* in) {
    const int j0 = j_beg + 32 * it;
    const bool more = it + 1 < ntile;
    float ib_next = 0.0f;
    if (more) {
      tile_copy<uint16_t, RS>(tb, j0 + 32, tn);
      ib_next = tile_inv_load(inv_b, j0 + 32, nb);
    }
    if (active) tile_epilogue<CF>(bf16_tile_products<KS, RS>(tc, lane, qa), lane, j0, j_end, ia, ic, top);
    if (more) {
      if (threadIdx.x < 32) in[threadIdx.x] = ib_next;
      tile_copy_wait();
    }
    __syncthreads();
  };
  for (int it = 0; it < ntile; it += 2) {
    step(it, tile0, tile1, ibt0, ibt1);
    if (it + 1 < ntile) step(it + 1, tile1, tile0, ibt1, ibt0);
  }
  if (active && qi < na) {
    int2* row = part + (size_t)qi * slices * (2 * kTopK) + g * kTopK;
    int2* dst = row + (size_t)cell.slice * (2 * kTopK);
#pragma unroll
    for (int q = 0; q < kTopK; ++q) dst[q] = make_int2(__float_as_int(top.d[q]), top.j[q]);
    // the last actual slice also writes the empty lists of the slices past nb
    if (cell.slice == cell.n_slices_act - 1)
      for (int sl = cell.n_slices_act; sl < slices; ++sl)
#pragma unroll
        for (int q = 0; q < kTopK; ++q) row[(size_t)sl * (2 * kTopK) + q] = make_int2(__float_as_int(INFINITY), -1);
  }
}

// FP32 MFMA (32x32x2).  The depth is split into chunks of 8: lane half g
// owns k = 8c + 4g + e, MFMA e of chunk c consumes element e, so both
// operands use the same k assignment.  The query counts are small integers
// (<= 256), held exactly as FP16 pairs and widened to FP32 for each MFMA,
// which halves their registers; with one tile buffer (28 KB of LDS) three
// blocks share a CU, and they cover each other's tile copies.
template <int DP, bool CF>
__global__ void __launch_bounds__(256) k_match_gemm_f32(const float* __restrict__ ta, const float* __restrict__ inv_a,
                                                        const int32_t* __restrict__ na_dev,
                                                        const float* __restrict__ tb, const float* __restrict__ inv_b,
                                                        const int32_t* __restrict__ nb_dev, int cap_a, int cap_b,
                                                        int slice_rows, int2* __restrict__ part) {
  static_assert(DP % 8 == 0, "padded depth");
  constexpr int KC = DP / 8;
  constexpr int RS = f32_stride<DP>();
  __shared__ __attribute__((aligned(16))) float tile[1][32 * RS];
  __shared__ __attribute__((aligned(16))) float ibt[1][32];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 5;
  const int na = min(*na_dev, cap_a), nb = min(*nb_dev, cap_b);
  if ((int)blockIdx.x * 128 >= na) return;
  const int q0 = (blockIdx.x * 4 + wave) * 32;
  const bool active = q0 < na;
  const int qi = q0 + (lane & 31);
  half2_t qh[KC][2];
  if (active) {
    const float* qrow = ta + (size_t)qi * RS + 4 * g;
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const float4 v = *(const float4*)(qrow + 8 * c);
      qh[c][0] = half2_t{(_Float16)v.x, (_Float16)v.y};
      qh[c][1] = half2_t{(_Float16)v.z, (_Float16)v.w};
    }
  }
  const float ia = (active && qi < na) ? inv_a[qi] : 0.0f;
  const int j_beg = blockIdx.y * slice_rows;
  const int j_end = min(nb, j_beg + slice_rows);
  const int ntile = j_end > j_beg ? (j_end - j_beg + 31) / 32 : 0;
  Top3 top;
#pragma unroll
  for (int q = 0; q < kTopK; ++q) {
    top.d[q] = INFINITY;
    top.j[q] = -1;
  }
  for (int it = 0; it < ntile; ++it) {
    const int j0 = j_beg + 32 * it;
    if (it > 0) __syncthreads();
    tile_copy<float, RS>(tb, j0, tile[0]);
    const float ibv = tile_inv_load(inv_b, j0, nb);
    if (threadIdx.x < 32) ibt[0][threadIdx.x] = ibv;
    tile_copy_wait();
    __syncthreads();
    if (active) {
      const float* crow = tile[0] + (lane & 31) * RS + 4 * g;
      floatx16_t acc = {};
      // the next chunk's candidate values are read before this chunk's
      // products, so the LDS latency hides behind four MFMAs
      float4 cb_next = *(const float4*)crow;
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        const float4 cb = cb_next;
        if (c + 1 < KC) cb_next = *(const float4*)(crow + 8 * (c + 1));
        asm volatile("" : "+v"(qh[c][0]), "+v"(qh[c][1]));
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(cb.x, (float)qh[c][0].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(cb.y, (float)qh[c][0].y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(cb.z, (float)qh[c][1].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(cb.w, (float)qh[c][1].y, acc, 0, 0, 0);
      }
      tile_epilogue<CF>(acc, lane, j0, j_end, ia, ibt[0], top);
    }
  }
  if (active && qi < na) {
    int2* dst = part + ((size_t)qi * gridDim.y + blockIdx.y) * (2 * kTopK) + g * kTopK;
#pragma unroll
    for (int q = 0; q < kTopK; ++q) dst[q] = make_int2(__float_as_int(top.d[q]), top.j[q]);
  }
}

__device__ __forceinline__ bool better(float d, int j, float bd, int bj) { return d < bd || (d == bd && j < bj); }

// Lexicographic (d, j) minimum over a wave.
__device__ __forceinline__ void wave_argmin(float& d, int& j) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float od = __shfl_xor(d, off);
    const int oj = __shfl_xor(j, off);
    if (oj >= 0 && (j < 0 || better(od, oj, d, j))) {
      d = od;
      j = oj;
    }
  }
}

// One wave per A row: merge the 2 x S top-3 lists, ratio test, keypoint best.
// With `a1` (the mutual check) an accepted row also needs the nearest A row of
// its j1 to belong to its own keypoint.
__global__ void __launch_bounds__(256) k_match_merge(const int2* __restrict__ part, int lists,
                                                     const int32_t* __restrict__ na_dev, const int32_t* __restrict__ kp_a,
                                                     const int32_t* __restrict__ kp_b, float ratio_sq, int cap_a,
                                                     const int32_t* __restrict__ a1, uint64_t* __restrict__ best,
                                                     int32_t* __restrict__ row_j1, float* __restrict__ row_d1) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int na = min(*na_dev, cap_a);
  if (i >= na) return;
  const int2* src = part + (size_t)i * lists * kTopK;
  const int total = lists * kTopK;
  float d1 = INFINITY;
  int j1 = -1;
  for (int q = lane; q < total; q += 64) {
    const int2 e = src[q];
    const float d = __int_as_float(e.x);
    if (e.y >= 0 && (j1 < 0 || better(d, e.y, d1, j1))) {
      d1 = d;
      j1 = e.y;
    }
  }
  wave_argmin(d1, j1);
  if (j1 < 0) return;
  const int k1 = kp_b[j1];
  float d2 = INFINITY;
  int j2 = -1;
  for (int q = lane; q < total; q += 64) {
    const int2 e = src[q];
    const float d = __int_as_float(e.x);
    if (e.y >= 0 && kp_b[e.y] != k1 && (j2 < 0 || better(d, e.y, d2, j2))) {
      d2 = d;
      j2 = e.y;
    }
  }
  wave_argmin(d2, j2);
  if (lane != 0) return;
  row_j1[i] = j1;
  row_d1[i] = d1;
  if (j2 < 0) return;
  if (!(d1 < __fmul_rn(ratio_sq, d2))) return;
  const int ka = kp_a[i];
  if (ka < 0 || ka >= cap_a) return;
  if (a1) {
    const int back = a1[j1];
    if (back < 0 || back >= na || kp_a[back] != ka) return;
  }
  // order-preserving key: rounding can make d1 slightly negative for identical rows
  const uint32_t b = __float_as_uint(d1);
  const uint32_t ok = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  const uint64_t key = ((uint64_t)ok << 32) | (uint32_t)i;
  atomicMin((unsigned long long*)&best[ka], (unsigned long long)key);
}

// Ring form (RIFT's convolution-sequence ring, the baseline variant): A holds
// R consecutive rows per keypoint, row g R + w being keypoint g's counts
// shifted by w, and B one plain row per keypoint.  The dot product of A row
// g R + w with B row r equals that of g's plain row with B keypoint r's ring
// row (R - w) mod R, so candidate (w, r) stands for reference ring row
// r R + (R - w) mod R, and the nearest / second-nearest choice runs over all R
// lists of the keypoint with that index order.  Each B row is a different
// keypoint, so every per-query top-3 list holds the best candidate of a
// keypoint other than j1's.  One wave per A keypoint; the decision goes
// straight into best[kp] with g standing for the row.
__global__ void __launch_bounds__(256) k_match_merge_ring(const int2* __restrict__ part, int lists, int R,
                                                          const int32_t* __restrict__ na_dev,
                                                          const int32_t* __restrict__ kp_a,
                                                          const int32_t* __restrict__ kp_b, float ratio_sq, int cap_a,
                                                          uint64_t* __restrict__ best, int32_t* __restrict__ row_j1,
                                                          float* __restrict__ row_d1) {
  const int lane = threadIdx.x & 63;
  const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int na = min(*na_dev, cap_a);
  if (g >= na / R) return;
  const int per = lists * kTopK;
  const int total = R * per;
  const int2* src = part + (size_t)g * R * per;  // the R query rows' lists are contiguous
  float d1 = INFINITY;
  int j1 = -1;
  for (int q = lane; q < total; q += 64) {
    const int2 e = src[q];
    if (e.y < 0) continue;
    const int w = q / per;
    const int jr = e.y * R + (w == 0 ? 0 : R - w);
    const float d = __int_as_float(e.x);
    if (j1 < 0 || better(d, jr, d1, j1)) {
      d1 = d;
      j1 = jr;
    }
  }
  wave_argmin(d1, j1);
  if (j1 < 0) return;
  const int r1 = j1 / R;
  const int k1 = kp_b[r1];
  float d2 = INFINITY;
  int j2 = -1;
  for (int q = lane; q < total; q += 64) {
    const int2 e = src[q];
    if (e.y < 0 || kp_b[e.y] == k1) continue;
    const int w = q / per;
    const int jr = e.y * R + (w == 0 ? 0 : R - w);
    const float d = __int_as_float(e.x);
    if (j2 < 0 || better(d, jr, d2, j2)) {
      d2 = d;
      j2 = jr;
    }
  }
  wave_argmin(d2, j2);
  if (lane != 0) return;
  row_j1[g] = r1;
  row_d1[g] = d1;
  if (j2 < 0) return;
  if (!(d1 < __fmul_rn(ratio_sq, d2))) return;
  const int ka = kp_a[g * R];
  if (ka < 0 || ka >= cap_a) return;
  const uint32_t b = __float_as_uint(d1);
  const uint32_t ok = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  const uint64_t key = ((uint64_t)ok << 32) | (uint32_t)g;
  atomicMin((unsigned long long*)&best[ka], (unsigned long long)key);
}

// Reverse pass of the mutual check: one wave per B row (the queries of the
// swapped GEMM) merges its lists into the nearest A row, ties to the lowest
// row; -1 when there is none.
__global__ void __launch_bounds__(256) k_match_rnn(const int2* __restrict__ part, int lists,
                                                   const int32_t* __restrict__ nb_dev, int cap_b,
                                                   int32_t* __restrict__ a1) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nb = min(*nb_dev, cap_b);
  if (j >= nb) return;
  const int2* src = part + (size_t)j * lists * kTopK;
  const int total = lists * kTopK;
  float d1 = INFINITY;
  int i1 = -1;
  for (int q = lane; q < total; q += 64) {
    const int2 e = src[q];
    const float d = __int_as_float(e.x);
    if (e.y >= 0 && (i1 < 0 || better(d, e.y, d1, i1))) {
      d1 = d;
      i1 = e.y;
    }
  }
  wave_argmin(d1, i1);
  if (lane == 0) a1[j] = i1;
}

struct MatchOut {
  int kp_a, kp_b;
  float dist2;
};

// Accepted keypoints in ascending order.  grid = ceil(cap_a / 256).
__global__ void __launch_bounds__(256) k_match_emit(const uint64_t* __restrict__ best, int cap_a,
                                                    const int32_t* __restrict__ row_j1, const float* __restrict__ row_d1,
                                                    const int32_t* __restrict__ kp_b, MatchOut* __restrict__ out,
                                                    int32_t* __restrict__ n_out) {
  __shared__ uint32_t scratch[4];
  __shared__ uint32_t sh_base;
  const int start = blockIdx.x * 256;
  uint32_t before = 0;
#pragma unroll 4
  for (int k = threadIdx.x; k < start; k += 256) before += best[k] != ~0ull;
  const uint32_t tot = block_inclusive_scan<256>(before, scratch);
  if (threadIdx.x == 255) sh_base = tot;
  const int k = start + threadIdx.x;
  const uint64_t bk = k < cap_a ? best[k] : ~0ull;
  const bool valid = bk != ~0ull;
  const uint32_t incl = block_inclusive_scan<256>(valid ? 1u : 0u, scratch);
  const uint32_t base = sh_base;  // published before the second scan's barriers
  if (valid) {
    const int row = (int)(bk & 0xffffffffu);
    MatchOut m;
    m.kp_a = k;
    m.kp_b = kp_b[row_j1[row]];
    m.dist2 = row_d1[row];
    out[base + incl - 1] = m;
  }
  if (start + 256 >= cap_a && threadIdx.x == 255) *n_out = (int32_t)(base + incl);
}

}  // namespace rift2
