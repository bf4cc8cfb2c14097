// FP8 form of the distance GEMM (the large 288-d case): E4M3 MFMA
// (32x32x64) with a power-of-two scale per descriptor row, FP32
// accumulation, a top-8 candidate list per query, then an exact re-rank of
// the 8 candidates from the integer counts before the nearest / second
// nearest selection and the ratio test (Section 4 matching rule, unchanged).
//
//   k_match_prep_fp8   one wave per row: e = largest power with
//                      max_count * 2^e <= 448, fp8(count * 2^e), row weight
//                      inv_norm * 2^-e (exact: a power of two)
//   k_match_gemm_fp8   approximate d2 = 2 - 2 acc w_a w_b per tile, top 8
//   k_match_merge8     global top 8 of the slice lists, exact dots, exact
//                      d2 = fl(2 - 2 fl(fl(dot ia) ib)), j1 / j2 / ratio test,
//                      per-keypoint best (same key as k_match_merge)
//
// With counts below 16 every scaled value is exact in E4M3 and the FP32
// accumulation is exact (all partial sums are multiples of 2^(e_a + e_b)
// below 2^24 of them), so the approximate scores equal the exact ones bit for
// bit; larger counts round to 4 significant bits and only the candidate
// choice is approximate.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "match.hip"

namespace rift2 {

constexpr int kTopK8 = 8;
typedef int intx8_t __attribute__((ext_vector_type(8)));

template <int DP>
constexpr int fp8_stride() { return DP + 16; }  // bytes; rows start 16 bytes apart modulo 128

__global__ void __launch_bounds__(256) k_match_prep_fp8(const uint16_t* __restrict__ desc, const float* __restrict__ inv,
                                                        const int32_t* __restrict__ n_dev, int cap, int D, int RS,
                                                        int rows_pad, uint8_t* __restrict__ table,
                                                        float* __restrict__ wrow, uint64_t* __restrict__ best,
                                                        int n_best) {
  const int lane = threadIdx.x & 63;
  const int n = min(*n_dev, cap);
  const int k0 = 8 * lane;  // this lane's 8 elements (D and RS are multiples of 8)
  for (int r = blockIdx.x * 4 + (threadIdx.x >> 6); r < rows_pad; r += gridDim.x * 4) {
    uint32_t c[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    if (r < n && k0 < D) {
      const uint4 raw = *(const uint4*)(desc + (size_t)r * D + k0);
      const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        c[2 * e] = w[e] & 0xffffu;
        c[2 * e + 1] = w[e] >> 16;
      }
    }
    uint32_t m = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) m = max(m, c[e]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    int ex = 0;
    if (m > 0) {
      while (ex < 30 && (m << (ex + 1)) <= 448u) ++ex;
    }
    const float s = (float)(1u << ex);
    if (k0 < RS) {
      int lo = __builtin_amdgcn_cvt_pk_fp8_f32((float)c[0] * s, (float)c[1] * s, 0, false);
      lo = __builtin_amdgcn_cvt_pk_fp8_f32((float)c[2] * s, (float)c[3] * s, lo, true);
      int hi = __builtin_amdgcn_cvt_pk_fp8_f32((float)c[4] * s, (float)c[5] * s, 0, false);
      hi = __builtin_amdgcn_cvt_pk_fp8_f32((float)c[6] * s, (float)c[7] * s, hi, true);
      *(uint2*)(table + (size_t)r * RS + k0) = make_uint2((uint32_t)lo, (uint32_t)hi);
    }
    if (lane == 0) wrow[r] = r < n ? inv[r] / s : 0.0f;
  }
  if (best) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_best; i += gridDim.x * blockDim.x) best[i] = ~0ull;
  }
}

struct Top8 {
  float d[kTopK8];
  int j[kTopK8];
};

__device__ __forceinline__ void top8_insert(Top8& t, float d, int j) {
  // t is sorted ascending; d < t.d[7] on entry
  float cd = d;
  int cj = j;
#pragma unroll
  for (int q = 0; q < kTopK8; ++q) {
    if (cd < t.d[q]) {
      const float td = t.d[q];
      const int tj = t.j[q];
      t.d[q] = cd;
      t.j[q] = cj;
      cd = td;
      cj = tj;
    }
  }
}

__device__ __forceinline__ void tile_epilogue8(const floatx16_t& acc, int lane, int j0, int j_end, float wa,
                                               const float* wbt, Top8& top) {
  const int g = lane >> 5;
  float d2[16];
  bool any = false;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float4 w4 = *(const float4*)(wbt + 8 * k + 4 * g);
    const float wv[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 4 * k + e;
      const float t1 = __fmul_rn(acc[r], wa);
      const float t2 = __fmul_rn(t1, wv[e]);
      d2[r] = __fsub_rn(2.0f, __fmul_rn(2.0f, t2));
      any |= (j0 + 8 * k + 4 * g + e < j_end) && d2[r] < top.d[kTopK8 - 1];
    }
  }
  if (!any) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int j = j0 + 8 * (r >> 2) + 4 * g + (r & 3);
    if (j < j_end && d2[r] < top.d[kTopK8 - 1]) top8_insert(top, d2[r], j);
  }
}

// Lane half g of lane l holds depth bytes [64 s + 32 g, 64 s + 32 g + 32) of
// row l % 32 for MFMA step s, for both operands (the same assignment on both
// sides, so the products pair up whatever order the instruction sums them).
template <int DP>
__global__ void __launch_bounds__(256) k_match_gemm_fp8(const uint8_t* __restrict__ ta, const float* __restrict__ wa_row,
                                                        const int32_t* __restrict__ na_dev,
                                                        const uint8_t* __restrict__ tb, const float* __restrict__ wb_row,
                                                        const int32_t* __restrict__ nb_dev, int cap_a, int cap_b,
                                                        int slice_rows, int2* __restrict__ part) {
  static_assert(DP % 64 == 0, "padded depth");
  constexpr int KS = DP / 64;
  constexpr int RS = fp8_stride<DP>();
  __shared__ __attribute__((aligned(16))) uint8_t tile[2][32 * RS];
  __shared__ __attribute__((aligned(16))) float wbt[2][32];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 5;
  const int na = min(*na_dev, cap_a), nb = min(*nb_dev, cap_b);
  if ((int)blockIdx.x * 128 >= na) return;
  const int q0 = (blockIdx.x * 4 + wave) * 32;
  const bool active = q0 < na;
  const int qi = q0 + (lane & 31);
  intx8_t qa[KS];
  if (active) {
    const uint8_t* qrow = ta + (size_t)qi * RS + 32 * g;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const uint4 lo = *(const uint4*)(qrow + 64 * ks);
      const uint4 hi = *(const uint4*)(qrow + 64 * ks + 16);
      qa[ks] = intx8_t{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
    }
  }
  const float wa = (active && qi < na) ? wa_row[qi] : 0.0f;
  const int j_beg = blockIdx.y * slice_rows;
  const int j_end = min(nb, j_beg + slice_rows);
  const int ntile = j_end > j_beg ? (j_end - j_beg + 31) / 32 : 0;
  Top8 top;
#pragma unroll
  for (int q = 0; q < kTopK8; ++q) {
    top.d[q] = INFINITY;
    top.j[q] = -1;
  }
  if (ntile > 0) {
    tile_copy<uint8_t, RS>(tb, j_beg, tile[0]);
    const float w0 = tile_inv_load(wb_row, j_beg, nb);
    if (threadIdx.x < 32) wbt[0][threadIdx.x] = w0;
    tile_copy_wait();
  }
  __syncthreads();
  for (int it = 0; it < ntile; ++it) {
    const int cur = it & 1;
    const int j0 = j_beg + 32 * it;
    float w_next = 0.0f;
    if (it + 1 < ntile) {
      tile_copy<uint8_t, RS>(tb, j0 + 32, tile[cur ^ 1]);
      w_next = tile_inv_load(wb_row, j0 + 32, nb);
    }
    if (active) {
      const uint8_t* crow = tile[cur] + (lane & 31) * RS + 32 * g;
      floatx16_t acc = {};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const uint4 lo = *(const uint4*)(crow + 64 * ks);
        const uint4 hi = *(const uint4*)(crow + 64 * ks + 16);
        const intx8_t cb = {(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        // formats 0/0: E4M3 for both operands; scales 127: 2^0
        acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(cb, qa[ks], acc, 0, 0, 0, 127, 0, 127);
      }
      tile_epilogue8(acc, lane, j0, j_end, wa, wbt[cur], top);
    }
    if (it + 1 < ntile) {
      if (threadIdx.x < 32) wbt[cur ^ 1][threadIdx.x] = w_next;
      tile_copy_wait();
    }
    __syncthreads();
  }
  if (active && qi < na) {
    int2* dst = part + ((size_t)qi * gridDim.y + blockIdx.y) * (2 * kTopK8) + g * kTopK8;
#pragma unroll
    for (int q = 0; q < kTopK8; ++q) dst[q] = make_int2(__float_as_int(top.d[q]), top.j[q]);
  }
}

// One wave per A row: the 8 best (approximate d2, row) of all slice lists,
// their exact d2 from the counts, then the same decision as k_match_merge.
__global__ void __launch_bounds__(256) k_match_merge8(const int2* __restrict__ part, int lists,
                                                      const int32_t* __restrict__ na_dev,
                                                      const uint16_t* __restrict__ desc_a, const float* __restrict__ inv_a,
                                                      const int32_t* __restrict__ kp_a,
                                                      const uint16_t* __restrict__ desc_b, const float* __restrict__ inv_b,
                                                      const int32_t* __restrict__ kp_b, int D, float ratio_sq, int cap_a,
                                                      const int32_t* __restrict__ a1, uint64_t* __restrict__ best,
                                                      int32_t* __restrict__ row_j1, float* __restrict__ row_d1) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int na = min(*na_dev, cap_a);
  if (i >= na) return;
  const int2* src = part + (size_t)i * lists * kTopK8;
  const int total = lists * kTopK8;
  // candidate selection: 8 rounds of a lexicographic (d, j) minimum above the last pick
  int cand[kTopK8];
  float last_d = -INFINITY;
  int last_j = -1;
#pragma unroll
  for (int q = 0; q < kTopK8; ++q) {
    float bd = INFINITY;
    int bj = -1;
    for (int e = lane; e < total; e += 64) {
      const int2 v = src[e];
      const float d = __int_as_float(v.x);
      if (v.y < 0) continue;
      const bool after = d > last_d || (d == last_d && v.y > last_j);
      if (after && (bj < 0 || better(d, v.y, bd, bj))) {
        bd = d;
        bj = v.y;
      }
    }
    wave_argmin(bd, bj);
    cand[q] = bj;
    if (bj >= 0) {
      last_d = bd;
      last_j = bj;
    }
  }
  // exact d2 of the candidates
  const float ia = inv_a[i];
  const uint16_t* ra = desc_a + (size_t)i * D;
  float d2[kTopK8];
#pragma unroll
  for (int q = 0; q < kTopK8; ++q) {
    d2[q] = INFINITY;
    const int j = cand[q];
    if (j < 0) continue;
    const uint16_t* rb = desc_b + (size_t)j * D;
    uint32_t dot = 0;
    for (int k = lane; k < D; k += 64) dot += (uint32_t)ra[k] * (uint32_t)rb[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dot += (uint32_t)__shfl_xor((int)dot, off);
    d2[q] = __fsub_rn(2.0f, __fmul_rn(2.0f, __fmul_rn(__fmul_rn((float)dot, ia), inv_b[j])));
  }
  if (lane != 0) return;
  float d1 = INFINITY;
  int j1 = -1;
#pragma unroll
  for (int q = 0; q < kTopK8; ++q)
    if (cand[q] >= 0 && (j1 < 0 || better(d2[q], cand[q], d1, j1))) {
      d1 = d2[q];
      j1 = cand[q];
    }
  if (j1 < 0) return;
  const int k1 = kp_b[j1];
  float dd2 = INFINITY;
  int j2 = -1;
#pragma unroll
  for (int q = 0; q < kTopK8; ++q)
    if (cand[q] >= 0 && kp_b[cand[q]] != k1 && (j2 < 0 || better(d2[q], cand[q], dd2, j2))) {
      dd2 = d2[q];
      j2 = cand[q];
    }
  row_j1[i] = j1;
  row_d1[i] = d1;
  if (j2 < 0) return;
  if (!(d1 < __fmul_rn(ratio_sq, dd2))) return;
  const int ka = kp_a[i];
  if (ka < 0 || ka >= cap_a) return;
  if (a1) {
    const int back = a1[j1];
    if (back < 0 || back >= na || kp_a[back] != ka) return;
  }
  const uint32_t b = __float_as_uint(d1);
  const uint32_t ok = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  const uint64_t key = ((uint64_t)ok << 32) | (uint32_t)i;
  atomicMin((unsigned long long*)&best[ka], (unsigned long long)key);
}

// Reverse pass of the mutual check in the FP8 form: one wave per B row (the
// queries of the swapped GEMM) takes the 8 best approximate candidates (A
// rows), re-ranks them with exact dots and d2 = fl(2 - 2 fl(fl(dot ia) ib)),
// the forward pass's rounding, and keeps the nearest (ties to the lowest row).
__global__ void __launch_bounds__(256) k_match_rnn8(const int2* __restrict__ part, int lists,
                                                    const int32_t* __restrict__ nb_dev, int cap_b,
                                                    const uint16_t* __restrict__ desc_a, const float* __restrict__ inv_a,
                                                    const uint16_t* __restrict__ desc_b, const float* __restrict__ inv_b,
                                                    int D, int32_t* __restrict__ a1) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nb = min(*nb_dev, cap_b);
  if (j >= nb) return;
  const int2* src = part + (size_t)j * lists * kTopK8;
  const int total = lists * kTopK8;
  int cand[kTopK8];
  float last_d = -INFINITY;
  int last_i = -1;
#pragma unroll
  for (int q = 0; q < kTopK8; ++q) {
    float bd = INFINITY;
    int bi = -1;
    for (int e = lane; e < total; e += 64) {
      const int2 v = src[e];
      const float d = __int_as_float(v.x);
      if (v.y < 0) continue;
      const bool after = d > last_d || (d == last_d && v.y > last_i);
      if (after && (bi < 0 || better(d, v.y, bd, bi))) {
        bd = d;
        bi = v.y;
      }
    }
    wave_argmin(bd, bi);
    cand[q] = bi;
    if (bi >= 0) {
      last_d = bd;
      last_i = bi;
    }
  }
  const float ib = inv_b[j];
  const uint16_t* rb = desc_b + (size_t)j * D;
  float d1 = INFINITY;
  int i1 = -1;
#pragma unroll
  for (int q = 0; q < kTopK8; ++q) {
    const int i = cand[q];
    if (i < 0) continue;
    const uint16_t* ra = desc_a + (size_t)i * D;
    uint32_t dot = 0;
    for (int k = lane; k < D; k += 64) dot += (uint32_t)ra[k] * (uint32_t)rb[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dot += (uint32_t)__shfl_xor((int)dot, off);
    const float d = __fsub_rn(2.0f, __fmul_rn(2.0f, __fmul_rn(__fmul_rn((float)dot, inv_a[i]), ib)));
    if (i1 < 0 || better(d, i, d1, i1)) {
      d1 = d;
      i1 = i;
    }
  }
  if (lane == 0) a1[j] = i1;
}

}  // namespace rift2
