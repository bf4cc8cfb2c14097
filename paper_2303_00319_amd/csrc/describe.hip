// Dominant-index MIM descriptor kernels (Section 2.2 histogram descriptor;
// Section 3, Eqs. 1-2 and the second-peak rule).
//
//   k_describe    KPB keypoints per block, one thread per patch column: each
//                 thread counts the MIM values of its column inside each cell
//                 band with 8-bit fields of one 64-bit word (one shift-add per
//                 pixel); the counts widen to 16-bit fields and are summed over
//                 the cell's columns with lane shuffles.  The patch histogram
//                 gives s (first argmax) and s2; the primary row is the cell
//                 histograms cyclically shifted by s.
//   k_describe2   secondary rows (shift s2) for keypoints whose second peak
//                 reaches num/den of the first, placed after all primary rows
//                 in keypoint order.
//
// Two more row forms serve RIFT's convolution-sequence ring (Section 2.3),
// the baseline RIFT2 replaces: kDescPlain writes the cell histograms as they
// are (no normalisation, one row per keypoint) and kDescRing writes N_o rows
// per keypoint, row i N_o + w being the histograms of the MIM rebuilt with
// layer w as the ring's first (bin b counts value (b + w) mod N_o).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scan.hpp"

namespace rift2 {

// fl32(1 / fl32(sqrt(n))) correctly rounded, for 0 < n < 2^24.  The hardware
// square root and reciprocal are only faithful, so both roundings are fixed
// by exact midpoint tests in FP64 (every product below is exact there).
__device__ __forceinline__ float inv_sqrt_rn(uint32_t n) {
  const double dn = (double)n;
  float s = sqrtf((float)n);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const float up = __uint_as_float(__float_as_uint(s) + 1u);
    const float dnx = __uint_as_float(__float_as_uint(s) - 1u);
    const double mu = 0.5 * ((double)s + (double)up);
    const double md = 0.5 * ((double)s + (double)dnx);
    if (dn > mu * mu) s = up;
    else if (dn < md * md) s = dnx;
  }
  float q = 1.0f / s;
  const double ds = (double)s;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const float up = __uint_as_float(__float_as_uint(q) + 1u);
    const float dnx = __uint_as_float(__float_as_uint(q) - 1u);
    const double mu = 0.5 * ((double)q + (double)up);
    const double md = 0.5 * ((double)q + (double)dnx);
    if (mu * ds < 1.0) q = up;        // 1/s lies above the upper midpoint
    else if (md * ds > 1.0) q = dnx;  // 1/s lies below the lower midpoint
  }
  return q;
}

constexpr int kDescDominant = 0, kDescPlain = 1, kDescRing = 2, kDescTurned = 3;

template <int P>
constexpr int desc_kpb() { return (P % 64 == 0) ? 1 : (P % 32 == 0 ? 2 : 4); }

template <int P, int G, int NO>
__global__ void __launch_bounds__(P * desc_kpb<P>()) k_describe(const uint8_t* __restrict__ mim, int H, int W,
                                                                const int* __restrict__ kpts /* x, y, score */,
                                                                const int32_t* __restrict__ n_kpts, int kpt_cap,
                                                                int dom_num, int dom_den, int mode,
                                                                uint16_t* __restrict__ desc,
                                                                float* __restrict__ inv_norm, int32_t* __restrict__ desc_kp,
                                                                uint32_t* __restrict__ info, int32_t* __restrict__ n_desc) {
  constexpr int KPB = desc_kpb<P>();
  constexpr int CS = P / G;  // cell side, a power of two dividing 64
  constexpr int D = G * G * NO;
  static_assert(CS == 8 || CS == 16 || CS == 32, "cell side");
  static_assert(NO >= 2 && NO <= 8, "orientations");
  __shared__ uint32_t h[KPB][G * G][NO];
  __shared__ uint32_t hist[KPB][NO];
  __shared__ int sh_s[KPB], sh_delta[KPB], sh_two[KPB], sh_ok[KPB];
  __shared__ uint32_t sh_n2[KPB];
  const int local = threadIdx.x / P, x = threadIdx.x % P;
  const int n = min(*n_kpts, kpt_cap);
  const int i = blockIdx.x * KPB + local;
  const bool active = i < n;
  // plain and ring forms have no secondary rows, so the row count is known here
  if (mode != kDescDominant && blockIdx.x == 0 && threadIdx.x == 0) *n_desc = (mode == kDescRing ? NO : 1) * n;
  int kx = 0, ky = 0;
  if (active) {
    kx = kpts[3 * i];
    ky = kpts[3 * i + 1];
  }
  const int px0 = kx - P / 2, py0 = ky - P / 2;
  const bool inside = active && px0 >= 0 && py0 >= 0 && px0 + P <= W && py0 + P <= H;
  if (x == 0) {
    sh_ok[local] = inside;
    sh_n2[local] = 0u;
  }
  for (int cy = 0; cy < G; ++cy) {
    uint64_t cnt = 0;
    if (inside) {
      const uint8_t* src = mim + (size_t)(py0 + cy * CS) * W + px0 + x;
#pragma unroll 8
      for (int r = 0; r < CS; ++r) cnt += 1ull << (8 * (src[(size_t)r * W] & 7));
    }
    const uint32_t lo = (uint32_t)cnt, hi = (uint32_t)(cnt >> 32);
    uint32_t w[4];
    w[0] = (lo & 0xffu) | ((lo << 8) & 0xff0000u);
    w[1] = ((lo >> 16) & 0xffu) | ((lo >> 8) & 0xff0000u);
    w[2] = (hi & 0xffu) | ((hi << 8) & 0xff0000u);
    w[3] = ((hi >> 16) & 0xffu) | ((hi >> 8) & 0xff0000u);
    constexpr int NW = (NO + 1) / 2;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
#pragma unroll
      for (int off = 1; off < CS; off <<= 1) w[q] += (uint32_t)__shfl_xor((int)w[q], off);
    }
    if ((x % CS) == 0) {
      const int cx = x / CS;
#pragma unroll
      for (int b = 0; b < NO; ++b) h[local][cy * G + cx][b] = (w[b >> 1] >> (16 * (b & 1))) & 0xffffu;
    }
  }
  __syncthreads();
  if (x < NO) {
    uint32_t s = 0;
    for (int c = 0; c < G * G; ++c) s += h[local][c][x];
    hist[local][x] = s;
  }
  __syncthreads();
  if (x == 0) {
    int s = 0;
    for (int b = 1; b < NO; ++b)
      if (hist[local][b] > hist[local][s]) s = b;
    int s2 = (s == 0) ? 1 : 0;
    for (int b = 0; b < NO; ++b)
      if (b != s && hist[local][b] > hist[local][s2]) s2 = b;
    const bool two = mode == kDescDominant && sh_ok[local] &&
                     (uint64_t)dom_den * hist[local][s2] >= (uint64_t)dom_num * hist[local][s];
    if (mode != kDescDominant) s = 0;
    sh_s[local] = s;
    sh_delta[local] = (s2 - s + NO) % NO;
    sh_two[local] = two;
  }
  __syncthreads();
  const int s = sh_s[local];
  uint32_t n2 = 0;
  const int rows_per_kp = mode == kDescRing ? NO : 1;
  if (active) {
    uint16_t* row = desc + (size_t)i * rows_per_kp * D;  // ring: row i NO + 0 (s = 0)
    for (int e = x; e < D; e += P) {
      const int c = e / NO, b = e % NO;
      int bb = b + s;
      if (bb >= NO) bb -= NO;
      const uint32_t v = h[local][c][bb];
      row[e] = (uint16_t)v;
      n2 += v * v;
    }
  }
  atomicAdd(&sh_n2[local], n2);
  if (mode == kDescRing && active) {
    // rows i NO + w for w >= 1; the norm is shared (each row permutes the same counts)
    uint16_t* rows = desc + (size_t)i * NO * D;
    for (int e = D + x; e < NO * D; e += P) {
      const int w = e / D, r = e - w * D;
      const int c = r / NO, b = r - c * NO;
      int bb = b + w;
      if (bb >= NO) bb -= NO;
      rows[e] = (uint16_t)h[local][c][bb];
    }
  }
  __syncthreads();
  if (active && x == 0) {
    const uint32_t nn = sh_n2[local];
    const float inv = nn ? inv_sqrt_rn(nn) : 0.0f;
    if (mode == kDescRing) {
      for (int w = 0; w < NO; ++w) {
        inv_norm[i * NO + w] = inv;
        desc_kp[i * NO + w] = i;
      }
    } else {
      inv_norm[i] = inv;
      desc_kp[i] = i;
    }
    info[i] = sh_two[local] ? (0x100u | (uint32_t)sh_delta[local]) : 0u;
  }
}

// ---------------------------------------------------------------- grid turned by the dominant index
//
// SIFT-style variant of the descriptor: the dominant index s stands for the
// filter direction s pi / N_o, so the sampling grid is turned by that angle
// (counter-clockwise on screen, y down) before the cells are counted.
//   * s and s2 come from the MIM values inside the disc of diameter P;
//   * sample (i, j) sits at offset ((2i - P + 1) / 2, (2j - P + 1) / 2) from
//     the keypoint pixel's upper-left corner, turned with 16-bit fixed-point
//     cos / sin, nearest pixel X = x + ((c U + s V) >> 17),
//     Y = y + ((-s U + c V) >> 17), U = 2i - P + 1, V = 2j - P + 1;
//   * samples outside the image are not counted; values recode by the row's
//     own index (Eq. 2).
// The primary row goes to row i; a second row (80 % rule) is built on its own
// turned grid into the staging rows and placed after the primary rows by
// k_describe2.
struct TurnTable {
  int c[8], s[8];  // round(2^16 cos(k pi / N_o)), round(2^16 sin(k pi / N_o))
};

// Every sample a keypoint needs -- the disc and both turned grids -- lies in
// the square of offsets [-R, R) around it: |c U + s V| <= |(c, s)| |(U, V)|
// < 2^16 (1 + 2^-15) (P - 1) sqrt 2, so (c U + s V) >> 17 lies in
// [-(R - 1) - 1, R - 1].  The block first copies that window of the MIM into
// LDS with whole-row (coalesced) loads, values masked to 3 bits and pixels
// outside the image marked by bit 7; the turned samples are then gathered
// from LDS instead of each touching its own cache line in global memory.
template <int P>
constexpr int turn_reach() { return ((P - 1) * 70712 + 99999) / 100000 + 1; }

template <int P, int G, int NO>
__global__ void __launch_bounds__(P * desc_kpb<P>()) k_describe_turn(const uint8_t* __restrict__ mim, int H, int W,
                                                                     const int* __restrict__ kpts,
                                                                     const int32_t* __restrict__ n_kpts, int kpt_cap,
                                                                     int dom_num, int dom_den, TurnTable tt,
                                                                     uint16_t* __restrict__ desc,
                                                                     float* __restrict__ inv_norm,
                                                                     int32_t* __restrict__ desc_kp,
                                                                     uint32_t* __restrict__ info,
                                                                     uint16_t* __restrict__ stage,
                                                                     float* __restrict__ stage_inv) {
  constexpr int KPB = desc_kpb<P>();
  constexpr int CS = P / G;
  constexpr int D = G * G * NO;
  constexpr int R = turn_reach<P>();
  static_assert((R - 1) * 100000 >= (P - 1) * 70712, "window reach");
  constexpr int WR = 2 * R;                // window rows and columns
  constexpr int NWD = (WR + 3 + 3) / 4;    // dwords loaded per window row (start aligned down to 4)
  constexpr int WS = 4 * (NWD | 1);        // LDS row stride in bytes: an odd number of dwords
  static_assert(CS == 8 || CS == 16 || CS == 32, "cell side");
  static_assert(NO >= 2 && NO <= 8, "orientations");
  __shared__ uint32_t win[KPB][WR * WS / 4];
  __shared__ uint32_t h[KPB][G * G][NO];
  __shared__ uint32_t hist[KPB][NO];
  __shared__ int sh_s[KPB], sh_s2[KPB], sh_two[KPB];
  __shared__ uint32_t sh_n2[KPB][2];
  const int local = threadIdx.x / P, x = threadIdx.x % P;
  const int n = min(*n_kpts, kpt_cap);
  const int i = blockIdx.x * KPB + local;
  const bool active = i < n;
  int kx = 0, ky = 0;
  if (active) {
    kx = kpts[3 * i];
    ky = kpts[3 * i + 1];
  }
  if (x < NO) hist[local][x] = 0u;
  if (x < 2) sh_n2[local][x] = 0u;
  // window of the MIM: rows ky - R .., columns from x0a (x0 = kx - R aligned down to 4)
  const int x0 = kx - R;
  const int xo = x0 & 3;  // two's complement: x0 - xo is the multiple of 4 at or below x0
  const int x0a = x0 - xo;
  const uint8_t* wb = (const uint8_t*)win[local];
  if (active) {
    // whole dwords when every row start is 4-byte aligned (then a dword is
    // either inside [0, W) or outside it), single bytes otherwise
    const bool words = ((reinterpret_cast<uintptr_t>(mim) | (uintptr_t)W) & 3u) == 0;
    if (words) {
      // branch-free body (the load address is clamped into the image and the
      // result masked), so the unrolled loads are all in flight together
#pragma unroll 8
      for (int d = x; d < WR * NWD; d += P) {
        const int row = d / NWD, c = d - row * NWD;
        const int gy = ky - R + row, gx = x0a + 4 * c;
        const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
        const int cy = min(max(gy, 0), H - 1), cx = min(max(gx, 0), W - 4);
        const uint32_t raw = *(const uint32_t*)(mim + (size_t)cy * W + cx);
        win[local][row * (WS / 4) + c] = in ? (raw & 0x07070707u) : 0x80808080u;
      }
    } else {
      for (int d = x; d < WR * NWD; d += P) {
        const int row = d / NWD, c = d - row * NWD;
        const int gy = ky - R + row, gx = x0a + 4 * c;
        uint32_t v = 0x80808080u;
        if (gy >= 0 && gy < H) {
          const uint8_t* src = mim + (size_t)gy * W;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int xx = gx + e;
            const uint32_t byte = (xx >= 0 && xx < W) ? (uint32_t)(src[xx] & 7) : 0x80u;
            v = (v & ~(0xffu << (8 * e))) | (byte << (8 * e));
          }
        }
        win[local][row * (WS / 4) + c] = v;
      }
    }
  }
  __syncthreads();
  // disc histogram: this thread's column, offsets U = 2x - P + 1
  {
    const int U = 2 * x - P + 1;
    const int lx = x - P / 2 + R + xo;
    uint64_t cnt = 0;  // 8-bit field per value; a column holds at most P < 256 pixels
    if (active) {
      // batches of 16 reads in flight, then branch-free counting
      for (int j0 = 0; j0 < P; j0 += 16) {
        uint32_t vv[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) vv[e] = j0 + e < P ? wb[(j0 + e - P / 2 + R) * WS + lx] : 0x80u;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int V = 2 * (j0 + e) - P + 1;
          const bool in = U * U + V * V <= P * P && vv[e] < 0x80u;
          cnt += (uint64_t)(in ? 1u : 0u) << (8 * (vv[e] & 7u));
        }
      }
    }
#pragma unroll
    for (int b = 0; b < NO; ++b) {
      const uint32_t v = (uint32_t)(cnt >> (8 * b)) & 0xffu;
      if (v) atomicAdd(&hist[local][b], v);
    }
  }
  __syncthreads();
  if (x == 0) {
    int s = 0;
    for (int b = 1; b < NO; ++b)
      if (hist[local][b] > hist[local][s]) s = b;
    int s2 = (s == 0) ? 1 : 0;
    for (int b = 0; b < NO; ++b)
      if (b != s && hist[local][b] > hist[local][s2]) s2 = b;
    sh_s[local] = s;
    sh_s2[local] = s2;
    sh_two[local] = active && (uint64_t)dom_den * hist[local][s2] >= (uint64_t)dom_num * hist[local][s];
  }
  __syncthreads();
  const int rows = sh_two[local] ? 2 : 1;  // uniform over the keypoint's threads
  int rows_blk = 1;                         // uniform over the block (the loop below holds barriers)
  for (int q = 0; q < KPB; ++q) rows_blk = max(rows_blk, sh_two[q] ? 2 : 1);
  for (int form = 0; form < rows_blk; ++form) {
    const int r = form == 0 ? sh_s[local] : sh_s2[local];
    const int cq = tt.c[r], sq = tt.s[r];
    const int U = 2 * x - P + 1;
    const bool live = active && form < rows;
    for (int cy = 0; cy < G; ++cy) {
      uint64_t cnt = 0;
      if (live) {
        // all CS reads of the band in flight, then branch-free counting
        uint32_t vv[CS];
        // the turned offsets advance by (2 s, 2 c) per grid row: products once
        // per band (24-bit operands: |c|, |s| <= 2^16, |U|, |V| < P), sums after
        const int V0 = 2 * cy * CS - P + 1;
        int tx = __mul24(cq, U) + __mul24(sq, V0), ty = __mul24(cq, V0) - __mul24(sq, U);
#pragma unroll
        for (int rr = 0; rr < CS; ++rr) {
          const int lx = (tx >> 17) + R + xo;
          const int ly = (ty >> 17) + R;
          vv[rr] = wb[ly * WS + lx];
          tx += 2 * sq;
          ty += 2 * cq;
        }
#pragma unroll
        for (int rr = 0; rr < CS; ++rr) {
          int b = (int)(vv[rr] & 7u) - r;
          b += b < 0 ? NO : 0;
          cnt += (uint64_t)(vv[rr] < 0x80u ? 1u : 0u) << (8 * b);
        }
      }
      const uint32_t lo = (uint32_t)cnt, hi = (uint32_t)(cnt >> 32);
      uint32_t w[4];
      w[0] = (lo & 0xffu) | ((lo << 8) & 0xff0000u);
      w[1] = ((lo >> 16) & 0xffu) | ((lo >> 8) & 0xff0000u);
      w[2] = (hi & 0xffu) | ((hi << 8) & 0xff0000u);
      w[3] = ((hi >> 16) & 0xffu) | ((hi >> 8) & 0xff0000u);
      constexpr int NW = (NO + 1) / 2;
#pragma unroll
      for (int q = 0; q < NW; ++q) {
#pragma unroll
        for (int off = 1; off < CS; off <<= 1) w[q] += (uint32_t)__shfl_xor((int)w[q], off);
      }
      if ((x % CS) == 0) {
        const int cx = x / CS;
#pragma unroll
        for (int b = 0; b < NO; ++b) h[local][cy * G + cx][b] = (w[b >> 1] >> (16 * (b & 1))) & 0xffffu;
      }
    }
    __syncthreads();
    uint32_t n2 = 0;
    if (live) {
      uint16_t* row = (form == 0 ? desc : stage) + (size_t)i * D;
      for (int e = x; e < D; e += P) {
        const uint32_t v = h[local][e / NO][e % NO];
        row[e] = (uint16_t)v;
        n2 += v * v;
      }
      atomicAdd(&sh_n2[local][form], n2);
    }
    __syncthreads();  // h is rewritten by the next form
  }
  if (active && x == 0) {
    const uint32_t nn = sh_n2[local][0];
    inv_norm[i] = nn ? inv_sqrt_rn(nn) : 0.0f;
    desc_kp[i] = i;
    if (rows == 2) {
      const uint32_t n2 = sh_n2[local][1];
      stage_inv[i] = n2 ? inv_sqrt_rn(n2) : 0.0f;
    }
    info[i] = rows == 2 ? 0x100u : 0u;  // second row staged, no further rotation
  }
}

// Secondary rows: row n + (number of flagged keypoints before i).  A block
// covers kDesc2Kpts keypoints; its flagged keypoints are compacted by one
// wave ballot, and every (flagged keypoint, cell) pair is one work item that
// gathers the cell's counts from the primary row, rotated by s2 - s.
// Keypoint index and rotation are kept in separate words: this compiler
// drops a 24-bit mask (x & 0xffffff) in front of a 64-bit multiply-add, so a
// packed (index | rotation << 24) word would address far outside the rows.
constexpr int kDesc2Kpts = 64;

// src_rows / src_inv: where keypoint k's second row is built from -- the
// primary rows and their norms (rotated by the stored delta), or a staging
// area that already holds finished second rows (delta 0).
//
// WIDE (info 16-byte aligned, rows 4-byte aligned, N_o even): the flags
// before the block are counted four info words per load, and a cell's N_o
// counts move as N_o / 2 words, rotated by whole words and then, for an odd
// delta, by one 16-bit half.
template <int NW>
__device__ __forceinline__ void rotate_halves(const uint32_t (&x)[NW], int delta, uint32_t (&z)[NW]) {
  // out element b = in element (b + delta) mod 2 NW; element 2k is the low half of word k
  const int q = delta >> 1;
  uint32_t y[NW];
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    uint32_t v = x[k];
#pragma unroll
    for (int r = 1; r < NW; ++r)
      if (q == r) v = x[(k + r) % NW];
    y[k] = v;
  }
#pragma unroll
  for (int k = 0; k < NW; ++k) z[k] = (delta & 1) ? (y[k] >> 16) | (y[(k + 1) % NW] << 16) : y[k];
}

template <int G, int NO, bool WIDE>
__global__ void __launch_bounds__(256) k_describe2(const int32_t* __restrict__ n_kpts, int kpt_cap,
                                                   const uint32_t* __restrict__ info, const uint16_t* src_rows,
                                                   const float* src_inv, uint16_t* desc, float* inv_norm,
                                                   int32_t* __restrict__ desc_kp, int32_t* __restrict__ n_desc) {
  constexpr int CELLS = G * G;
  constexpr int D = CELLS * NO;
  __shared__ uint32_t scratch[4];
  __shared__ int flagged_kp[kDesc2Kpts];
  __shared__ int flagged_delta[kDesc2Kpts];
  __shared__ uint32_t sh_base, sh_nflag;
  const int n = min(*n_kpts, kpt_cap);
  const int start = blockIdx.x * kDesc2Kpts;
  if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) *n_desc = 0;
  if (start >= n) return;
  uint32_t before = 0;
  if constexpr (WIDE) {
    // start is a multiple of kDesc2Kpts: whole 16-byte groups
    const uint4* info4 = reinterpret_cast<const uint4*>(info);
#pragma unroll 8
    for (int j = threadIdx.x; j < start / 4; j += 256) {
      const uint4 g = info4[j];
      before += ((g.x >> 8) & 1u) + ((g.y >> 8) & 1u) + ((g.z >> 8) & 1u) + ((g.w >> 8) & 1u);
    }
  } else {
#pragma unroll 4
    for (int j = threadIdx.x; j < start; j += 256) before += (info[j] >> 8) & 1u;
  }
  const uint32_t tot = block_inclusive_scan<256>(before, scratch);
  if (threadIdx.x == 255) sh_base = tot;
  if (threadIdx.x < kDesc2Kpts) {  // wave 0
    const int i = start + threadIdx.x;
    const uint32_t word = (i < n) ? info[i] : 0u;
    const bool f = (word >> 8) & 1u;
    const uint64_t mask = __ballot(f);
    if (f) {
      const int pos = __popcll(mask & ((1ull << threadIdx.x) - 1ull));
      flagged_kp[pos] = i;
      flagged_delta[pos] = (int)(word & 0xffu);
    }
    if (threadIdx.x == 0) sh_nflag = (uint32_t)__popcll(mask);
  }
  __syncthreads();
  const int base = (int)sh_base;
  const int nflag = (int)sh_nflag;
  if (threadIdx.x == 0 && min(n, start + kDesc2Kpts) == n) *n_desc = n + base + nflag;
  for (int w = threadIdx.x; w < nflag * CELLS; w += 256) {
    const int fi = w / CELLS, c = w - fi * CELLS;
    const int src_kp = flagged_kp[fi], delta = flagged_delta[fi];
    const uint16_t* src = src_rows + (size_t)src_kp * D + c * NO;
    uint16_t* dst = desc + (size_t)(n + base + fi) * D + c * NO;
    if constexpr (WIDE) {
      static_assert(NO % 2 == 0, "whole words per cell");
      constexpr int NW = NO / 2;
      uint32_t x[NW], z[NW];
#pragma unroll
      for (int k = 0; k < NW; ++k) x[k] = reinterpret_cast<const uint32_t*>(src)[k];
      rotate_halves<NW>(x, delta, z);
#pragma unroll
      for (int k = 0; k < NW; ++k) reinterpret_cast<uint32_t*>(dst)[k] = z[k];
    } else {
#pragma unroll
      for (int b = 0; b < NO; ++b) {
        int bb = b + delta;
        if (bb >= NO) bb -= NO;
        dst[b] = src[bb];
      }
    }
  }
  for (int fi = threadIdx.x; fi < nflag; fi += 256) {
    const int row = n + base + fi;
    const int src_kp = flagged_kp[fi];
    inv_norm[row] = src_inv[src_kp];
    desc_kp[row] = src_kp;
  }
}

// FP32 view of descriptor rows: fl(count * inv_norm) for the first n rows
// (grid-stride over row-major elements).
__global__ void __launch_bounds__(256) k_desc_normalize(const uint16_t* __restrict__ desc,
                                                        const float* __restrict__ inv_norm,
                                                        const int32_t* __restrict__ n_dev, int cap, int D,
                                                        float* __restrict__ out) {
  const int n = min(*n_dev, cap);
  const int64_t total = (int64_t)n * D;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = __fmul_rn((float)desc[e], inv_norm[e / D]);
}

}  // namespace rift2

