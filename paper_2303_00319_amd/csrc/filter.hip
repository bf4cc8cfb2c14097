// Filter-bank / MIM / moment kernels (Sections 2.1 and 2.2 of the paper).
//
// Data flow for one H x W image, F = N_s * N_o filters:
//   k_fwd_rows   image -> Rrow = row DFTs                          (row-major complex)
//   k_pass_a     per block of C columns (each wave spans C columns, so every
//                global access is a C-point row segment): column DFT of Rrow
//                -> spectrum S in registers; for every filter of the block's
//                orientation group: S * G_{s,o} / (HW), inverse column DFT
//                -> Y_{s,o}                                        (row-major complex)
//   k_noise_pre  row IDFT of the s = 0 planes, written back in place as
//                EO_{0,o}, -> A0_o = |EO_{0,o}| and a 12-bit radix histogram
//                of its float bits per orientation
//   k_noise_sel1/2, k_noise_threshold  exact median of A0_o (radix select
//                over the candidates of the level-1 and level-2 bins) and the
//                noise threshold T_o, evaluated in FP64
//   k_pass_b_orient  per row and orientation: row IDFTs of the other scales;
//                per-pixel amplitude sum and phase congruency
//   k_pass_b_reduce  per pixel over orientations: MIM argmax and moments
//   k_pass_b_fused   both of the above in one launch, for rows that one wave
//                transforms (N_o = 6)
#pragma once

#include "fft.hpp"
#include "scan.hpp"

namespace rift2 {

constexpr int kMaxOrient = 8;
constexpr int kMaxScales = 8;
constexpr int kHistBits1 = 12;  // level-1 key: float bits >> 19 (sign 0, 8 exponent, 3 mantissa)
constexpr int kHist1 = 1 << kHistBits1;

// Threads per block for row kernels: whole lines, at least 256 threads.
template <int N, int P>
constexpr int row_block() { return (N / P) >= 256 ? (N / P) : 256; }

struct FilterConsts {
  int H, W, n_scales, n_orient;
  float log_f0[kMaxScales];    // ln(f0_s)
  float inv_2ln2_sigma;        // 1 / (2 ln^2 sigma_onf)
  float log_lp_cutoff;         // ln(lp_cutoff)
  float two_n;                 // 2 * lp_order
  float theta_o[kMaxOrient];   // o pi / N_o
  float inv_2sig_theta2;       // 1 / (2 sigma_theta^2)
  float inv_hw;                // 1 / (H W), folded into the filter
};

// Hardware square root and reciprocal (v_sqrt_f32 / v_rcp_f32, about 1 ulp).
// The filter path's results carry the FP32 FFT's rounding (~1e-6 relative),
// so the correctly rounded library forms (a dozen instructions each) buy no
// accuracy there.
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

struct PCConsts {
  float eps, g, cutoff;
  float cos_o[kMaxOrient], sin_o[kMaxOrient];
};

// Batched launches: the images of one filter-bank call (same size and bank)
// share every kernel launch, blockIdx.z picking the image.  Each image brings
// its input, its workspace regions and its outputs.
constexpr int kMaxFilterBatch = 8;
struct FilterImage {
  const void* img;
  float2* rrow;
  float2* yplanes;
  float* a0;
  uint32_t* cand;
  uint32_t* zero;
  float* t32;
  double* t64;
  float* ostat;
  float2* spc;
  uint8_t* mim;
  float* mmax;
  float* mmin;
  float* amp;
};
struct FilterBatch {
  FilterImage im[kMaxFilterBatch];
};

// ---------------------------------------------------------------- forward rows

template <int W, int P, typename Tin>
__global__ void __launch_bounds__(256) k_fwd_rows(FilterBatch B, int64_t pitch, int n_zero) {
  const FilterImage& I = B.im[blockIdx.z];
  const Tin* __restrict__ img = (const Tin*)I.img;
  float2* __restrict__ rrow = I.rrow;
  uint32_t* __restrict__ zero = I.zero;
  using PL = FftPlan<W, P>;
  constexpr int T = PL::T;
  constexpr int LINES = 256 / T;
  __shared__ float2 lines[LINES][lds_line<W, T>()];
  // clear the noise-selection counters and histograms (spread over the grid)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_zero; i += gridDim.x * blockDim.x) zero[i] = 0u;
  const int team = threadIdx.x / T, t = threadIdx.x % T;
  const int y = blockIdx.x * LINES + team;  // H % LINES == 0 (checked on the host)
  const Tin* row = img + (int64_t)y * pitch;
  float2 v[P];
#pragma unroll
  for (int m = 0; m < P; ++m) v[m] = make_float2((float)row[t + T * m], 0.0f);
  // a team that is exactly one wave exchanges with wave barriers only
  fft_line<-1, W, P, T == 64>(v, t, lines[team]);
  float2* out = rrow + (size_t)y * W;
#pragma unroll
  for (int m = 0; m < P; ++m) out[t + T * m] = v[m];
}

// ---------------------------------------------------------------- pass A

// Polar coordinates of DFT bin (k, l): ln r and theta = atan2(-v, u).  DC and
// the Nyquist row/column carry no filter response (dead).
struct BinPolar {
  float lr, th;
  bool dead;
};

__device__ __forceinline__ BinPolar bin_polar(int k, int l, const FilterConsts& fc) {
  BinPolar b;
  const int kt = (k >= (fc.H + 1) / 2) ? k - fc.H : k;
  const int lt = (l >= (fc.W + 1) / 2) ? l - fc.W : l;
  const float v = (float)kt / (float)fc.H;
  const float u = (float)lt / (float)fc.W;
  b.dead = (kt == 0 && lt == 0) || ((fc.H & 1) == 0 && kt == -fc.H / 2) || ((fc.W & 1) == 0 && lt == -fc.W / 2);
  b.lr = b.dead ? 0.0f : 0.5f * __logf(u * u + v * v);
  b.th = atan2f(-v, u);
  return b;
}

// angular(o) * lowpass * 1/(HW) of one bin; the angular distance is theta -
// theta_o wrapped to [-pi, pi].
__device__ __forceinline__ float ang_lowpass(float lr, float th, bool dead, int o, const FilterConsts& fc) {
  constexpr float kPi = 3.14159265358979323846f;
  float d = th - fc.theta_o[o];
  d = d > kPi ? d - 2.0f * kPi : (d < -kPi ? d + 2.0f * kPi : d);
  const float ang = __expf(-d * d * fc.inv_2sig_theta2);
  const float lp = hw_rcp(1.0f + __expf(fc.two_n * (lr - fc.log_lp_cutoff)));
  return dead ? 0.0f : ang * lp * fc.inv_hw;
}

// One block = C adjacent columns.  Lane l of wave w works on column l % C at
// FFT team position t = l / C + (64 / C) w, so a wave's global accesses are
// 64/C rows x C contiguous points.  Column lines in LDS are 4 points apart
// modulo 32, which measured fastest for this interleaving.
template <int H, int P, int C>
__global__ void __launch_bounds__(C * (H / P)) k_pass_a(FilterBatch B, FilterConsts fc) {
  const float2* __restrict__ rrow = B.im[blockIdx.z].rrow;
  float2* __restrict__ y_out = B.im[blockIdx.z].yplanes;
  using PL = FftPlan<H, P>;
  constexpr int T = PL::T;
  constexpr int L = 64 / C;
  static_assert(64 % C == 0 && (C * T) % 64 == 0, "column mapping");
  __shared__ float2 lines[C][lds_line<H, 4>()];
  const int W = fc.W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane % C;
  const int t = lane / C + L * wave;
  // Consecutive block ids run on different XCDs (round robin over 8), each
  // with its own L2: hand every XCD a contiguous run of column blocks so that
  // neighbouring C-point row segments of the planes are written through one
  // L2 and leave it as whole lines.
  const int nbx = gridDim.x;
  const int cb = (nbx % 8 == 0) ? (int)(blockIdx.x % 8) * (nbx / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  const int l = cb * C + c;
  float2 spec[P];
#pragma unroll
  for (int m = 0; m < P; ++m) spec[m] = rrow[(size_t)(t + T * m) * W + l];
  fft_line<-1, H, P>(spec, t, lines[c]);  // spec[m] = S[k = t + T m][l]

  float lr[P], th[P];
  unsigned dead = 0u;
#pragma unroll
  for (int m = 0; m < P; ++m) {
    const BinPolar b = bin_polar(t + T * m, l, fc);
    lr[m] = b.lr;
    th[m] = b.th;
    dead |= (unsigned)b.dead << m;
  }
  const size_t plane = (size_t)H * W;
  // orientation group of this block (grid.y splits the bank for parallelism)
  const int o_beg = (int)(blockIdx.y * fc.n_orient / gridDim.y);
  const int o_end = (int)((blockIdx.y + 1) * fc.n_orient / gridDim.y);
  for (int o = o_beg; o < o_end; ++o) {
    float ang[P];
#pragma unroll
    for (int m = 0; m < P; ++m) ang[m] = ang_lowpass(lr[m], th[m], (dead >> m) & 1u, o, fc);
    for (int s = 0; s < fc.n_scales; ++s) {
      const float lf0 = fc.log_f0[s];
      float2 v[P];
#pragma unroll
      for (int m = 0; m < P; ++m) {
        const float d = lr[m] - lf0;
        v[m] = cscale(spec[m], __expf(-d * d * fc.inv_2ln2_sigma) * ang[m]);
      }
      fft_line<+1, H, P>(v, t, lines[c]);
      float2* dst = y_out + (size_t)(o * fc.n_scales + s) * plane + l;
#pragma unroll
      for (int m = 0; m < P; ++m) dst[(size_t)(t + T * m) * W] = v[m];
    }
  }
}

// ---------------------------------------------------------------- noise threshold

// Exact median of A0_o (mean of the order statistics of rank HW/2-1 and HW/2)
// by a three-level radix selection on the float bit patterns (values are
// non-negative, so the bits order like the values): 13 bits (histogram built
// by k_noise_pre), 10 bits (k_noise_sel1), 9 bits (k_noise_sel2).  Each level
// is resolved at the start of the next kernel by every block that needs it
// (the kernel boundary orders the histogram merges before the search, with no
// device-wide fence, which would write back every XCD's L2 full of freshly
// written planes); block 0 of each orientation publishes the level's bins in
// state[o] for the kernels after it.  One block per orientation resolves the
// last level and evaluates the threshold T_o in FP64 (k_noise_threshold):
// done by every row-pass block instead, it measured 8 us slower at 1024^2.
constexpr int kHist2 = 1024, kHist3 = 512;

struct NoiseConsts {
  double mult, k;
  int n_scales;
};

struct NoiseWs {
  uint32_t* hist1;  // [N_o][kHist1]
  uint32_t* hist2;  // [N_o][2][kHist2]
  uint32_t* hist3;  // [N_o][2][kHist3]
  uint32_t* state;  // [N_o][8] level-1 bins, counts below them, level-2 bins, counts below (two ranks each)
  uint32_t* cnt;    // [N_o][regions] candidate counts of each k_noise_sel1 block
  int regions;      // k_noise_sel1 / k_noise_sel2 blocks per orientation
  uint32_t* cand;   // [N_o][HW] candidate bit patterns
};

// The selection's histograms, state and counters live in the image's
// zeroed region, in this order; the candidate lists in its own region.
__host__ __device__ __forceinline__ NoiseWs noise_ws(const FilterImage& I, int n_orient, int regions) {
  NoiseWs w;
  w.hist1 = I.zero;
  w.hist2 = w.hist1 + n_orient * kHist1;
  w.hist3 = w.hist2 + n_orient * 2 * kHist2;
  w.state = w.hist3 + n_orient * 2 * kHist3;
  w.cnt = w.state + 8 * n_orient;
  w.regions = regions;
  w.cand = I.cand;
  return w;
}

// Ranks of the two middle order statistics.
__device__ __forceinline__ uint32_t noise_rank(int hw, int q) { return (uint32_t)(hw / 2 - 1 + q); }

// T_o from the median of A0_o in FP64: tau = median / sqrt(ln 4), the
// expected total amplitude over the geometric series of scales, then mean +
// k sigma of the Rayleigh-distributed noise energy.
__device__ __forceinline__ double noise_threshold(float v0, float v1, const NoiseConsts& nc) {
  const double med = 0.5 * ((double)v0 + (double)v1);
  const double tau = med / sqrt(log(4.0));
  const double total = tau * (1.0 - pow(1.0 / nc.mult, (double)nc.n_scales)) / (1.0 - 1.0 / nc.mult);
  const double pi = 3.14159265358979323846;
  return total * sqrt(pi / 2.0) + nc.k * total * sqrt((4.0 - pi) / 2.0);
}

// Block = LINES rows of one orientation.  A0 = |EO_{0,o}| written as float,
// level-1 histogram of its bit pattern (bits >> 19) merged into hist1[o].
template <int W, int P>
__global__ void __launch_bounds__(256) k_noise_pre(FilterBatch B, int H, int n_scales, int n_orient, int regions) {
  const FilterImage& I = B.im[blockIdx.z];
  float2* __restrict__ y_in = I.yplanes;
  float* __restrict__ a0 = I.a0;
  const NoiseWs ws = noise_ws(I, n_orient, regions);
  using PL = FftPlan<W, P>;
  constexpr int T = PL::T;
  constexpr int LINES = 256 / T;
  __shared__ float2 lines[LINES][lds_line<W, T>()];
  // the block histogram reuses the lines once every team has transformed its
  // row, so the kernel's LDS is the lines alone (4 blocks per CU at 1024)
  static_assert(sizeof(lines) >= kHist1 * sizeof(uint32_t), "histogram fits the lines");
  uint32_t* hist = reinterpret_cast<uint32_t*>(&lines[0][0]);
  const int o = blockIdx.y;
  const int team = threadIdx.x / T, t = threadIdx.x % T;
  const int y = blockIdx.x * LINES + team;
  const size_t plane = (size_t)H * W;
  float2* src = y_in + (size_t)(o * n_scales) * plane + (size_t)y * W;
  float2 v[P];
#pragma unroll
  for (int m = 0; m < P; ++m) v[m] = src[t + T * m];
  fft_line<+1, W, P, T == 64>(v, t, lines[team]);  // one-wave teams: wave barriers only
  float* dst = a0 + (size_t)o * plane + (size_t)y * W;
  // the transformed row replaces its input: pass B takes EO_{0,o} as is
  float2* eo = src;
  uint32_t key[P];
#pragma unroll
  for (int m = 0; m < P; ++m) {
    eo[t + T * m] = v[m];
    const float a = hw_sqrt(v[m].x * v[m].x + v[m].y * v[m].y);
    dst[t + T * m] = a;
    key[m] = min(__float_as_uint(a) >> (32 - kHistBits1 - 1), (uint32_t)(kHist1 - 1));
  }
  __syncthreads();  // every team is done with its line
  for (int i = threadIdx.x; i < kHist1; i += 256) hist[i] = 0u;
  __syncthreads();
#pragma unroll
  for (int m = 0; m < P; ++m) atomicAdd(&hist[key[m]], 1u);
  __syncthreads();
  uint32_t* gh = ws.hist1 + (size_t)o * kHist1;
  for (int i = threadIdx.x; i < kHist1; i += 256) {
    const uint32_t c = hist[i];
    if (c) atomicAdd(&gh[i], c);
  }
}

// Appends the taking lanes' values to this block's own list region; the
// position comes from a block-local LDS counter (no global atomics).
__device__ __forceinline__ void block_append(bool take, uint32_t value, uint32_t* lds_count, uint32_t* region) {
  const uint64_t mask = __ballot(take);
  if (!mask) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(lds_count, (uint32_t)__popcll(mask));
  base = __shfl(base, leader);
  if (take) region[base + __popcll(mask & ((1ull << lane) - 1ull))] = value;
}

// Level 2: every block copies the values of the two level-1 bins from its
// chunk of A0 into its own region of the candidate list (region b = chunk
// b, so it cannot overflow) and histograms their next 10 bits.
__global__ void __launch_bounds__(256) k_noise_sel1(FilterBatch B, int hw, int n_orient, int regions) {
  const FilterImage& I = B.im[blockIdx.z];
  const float* __restrict__ a0 = I.a0;
  const NoiseWs ws = noise_ws(I, n_orient, regions);
  __shared__ uint32_t h2[2][kHist2];
  __shared__ uint32_t s_count;
  __shared__ uint32_t scratch[4];
  __shared__ int s_bin[2];
  __shared__ uint32_t s_below[2];
  const int o = blockIdx.y;
  for (int i = threadIdx.x; i < 2 * kHist2; i += 256) (&h2[0][0])[i] = 0u;
  if (threadIdx.x == 0) s_count = 0u;
  // level 1: the bins of both ranks in the histogram k_noise_pre completed
  const uint32_t* h1 = ws.hist1 + (size_t)o * kHist1;
  block_find_two_ranks<kHist1, 256>(h1, noise_rank(hw, 0), s_bin, s_below, scratch);
  const uint32_t b0 = (uint32_t)s_bin[0], b1 = (uint32_t)s_bin[1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    uint32_t* st = ws.state + 8 * o;
    st[0] = b0;
    st[1] = b1;
    st[2] = s_below[0];
    st[3] = s_below[1];
  }
  __syncthreads();
  const float* src = a0 + (size_t)o * hw;
  const int per_block = (hw + gridDim.x - 1) / gridDim.x;
  const int beg = blockIdx.x * per_block;
  const int end = min(hw, beg + per_block);
  uint32_t* region = ws.cand + (size_t)o * hw + beg;
  // chunk bounds are multiples of 4 (both sides are multiples of 256, HW / regions is): 16-byte loads
  for (int i0 = beg; i0 < end; i0 += 1024) {
    const int i = i0 + 4 * threadIdx.x;
    const bool in = i < end;
    const float4 q4 = in ? *(const float4*)(src + i) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float qv[4] = {q4.x, q4.y, q4.z, q4.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t bits = __float_as_uint(qv[e]);
      const uint32_t key = bits >> 19;
      const uint32_t sub = (bits >> 9) & (kHist2 - 1);
      const bool t0 = in && key == b0, t1 = in && key == b1;
      if (t0) atomicAdd(&h2[0][sub], 1u);
      if (t1) atomicAdd(&h2[1][sub], 1u);
      block_append(t0 || t1, bits, &s_count, region);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) ws.cnt[(size_t)o * gridDim.x + blockIdx.x] = s_count;
  uint32_t* gh2 = ws.hist2 + (size_t)o * 2 * kHist2;
  for (int i = threadIdx.x; i < 2 * kHist2; i += 256) {
    const uint32_t c = (&h2[0][0])[i];
    if (c) atomicAdd(&gh2[i], c);
  }
}

// Level 3: one block per candidate region histograms the last 9 bits of the
// candidates that share both upper levels of a rank.
__global__ void __launch_bounds__(256) k_noise_sel2(FilterBatch B, int hw, int n_orient, int regions) {
  const NoiseWs ws = noise_ws(B.im[blockIdx.z], n_orient, regions);
  __shared__ uint32_t h3[2][kHist3];
  __shared__ uint32_t scratch[4];
  __shared__ int s_bin[2];
  __shared__ uint32_t s_below[2];
  const int o = blockIdx.y;
  for (int i = threadIdx.x; i < 2 * kHist3; i += 256) (&h3[0][0])[i] = 0u;
  uint32_t* st = ws.state + 8 * o;
  // level 2: the sub-bins of both ranks inside their level-1 bins
  const uint32_t* h2 = ws.hist2 + (size_t)o * 2 * kHist2;
  // both ranks in one level-1 bin (the usual case): their histograms are the
  // same and their ranks in it consecutive
  if (st[0] == st[1]) {
    block_find_two_ranks<kHist2, 256>(h2, noise_rank(hw, 0) - st[2], s_bin, s_below, scratch);
  } else {
    for (int q = 0; q < 2; ++q)
      block_find_rank<kHist2, 256, false>(h2 + q * kHist2, noise_rank(hw, q) - st[2 + q], &s_bin[q], &s_below[q],
                                          scratch);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st[4] = (uint32_t)s_bin[0];
    st[5] = (uint32_t)s_bin[1];
    st[6] = s_below[0];
    st[7] = s_below[1];
  }
  const uint32_t p0 = (st[0] << 10) | (uint32_t)s_bin[0];
  const uint32_t p1 = (st[1] << 10) | (uint32_t)s_bin[1];
  const int per_region = (hw + ws.regions - 1) / ws.regions;
  const int rg = blockIdx.x;
  const uint32_t n = ws.cnt[(size_t)o * ws.regions + rg];
  const uint32_t* list = ws.cand + (size_t)o * hw + (size_t)rg * per_region;  // 16-byte aligned
  __syncthreads();
  for (uint32_t i = 4 * threadIdx.x; i < n; i += 1024) {
    uint32_t qv[4];
    if (i + 4 <= n) {
      const uint4 q4 = *(const uint4*)(list + i);
      qv[0] = q4.x;
      qv[1] = q4.y;
      qv[2] = q4.z;
      qv[3] = q4.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) qv[e] = i + e < n ? list[i + e] : 0u;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (i + e >= n) break;
      const uint32_t bits = qv[e];
      const uint32_t pre = bits >> 9;
      if (pre == p0) atomicAdd(&h3[0][bits & (kHist3 - 1)], 1u);
      if (pre == p1) atomicAdd(&h3[1][bits & (kHist3 - 1)], 1u);
    }
  }
  __syncthreads();
  uint32_t* gh3 = ws.hist3 + (size_t)o * 2 * kHist3;
  for (int i = threadIdx.x; i < 2 * kHist3; i += 256) {
    const uint32_t c = (&h3[0][0])[i];
    if (c) atomicAdd(&gh3[i], c);
  }
}

// One block per orientation: the last selection level, the two middle order
// statistics (kept for diagnostics) and the threshold T_o (FP64; FP32 copy
// for the row pass).
__global__ void __launch_bounds__(256) k_noise_threshold(FilterBatch B, int hw, int n_orient, int regions,
                                                         NoiseConsts nc) {
  const FilterImage& I = B.im[blockIdx.z];
  const NoiseWs ws = noise_ws(I, n_orient, regions);
  __shared__ uint32_t scratch[4];
  __shared__ int s_bin[2];
  __shared__ uint32_t s_below[2];
  const int o = blockIdx.x;
  const uint32_t* st = ws.state + 8 * o;
  const uint32_t* h3 = ws.hist3 + (size_t)o * 2 * kHist3;
  float vals[2];
  if (st[0] == st[1] && st[4] == st[5]) {
    block_find_two_ranks<kHist3, 256>(h3, noise_rank(hw, 0) - st[2] - st[6], s_bin, s_below, scratch);
  } else {
    for (int q = 0; q < 2; ++q)
      block_find_rank<kHist3, 256, false>(h3 + q * kHist3, noise_rank(hw, q) - st[2 + q] - st[6 + q], &s_bin[q],
                                          &s_below[q], scratch);
  }
  for (int q = 0; q < 2; ++q) vals[q] = __uint_as_float((((st[q] << 10) | st[4 + q]) << 9) | (uint32_t)s_bin[q]);
  if (threadIdx.x == 0) {
    const double tt = noise_threshold(vals[0], vals[1], nc);
    I.ostat[2 * o] = vals[0];
    I.ostat[2 * o + 1] = vals[1];
    I.t32[o] = (float)tt;
    I.t64[o] = tt;
  }
}

// Row IDFT of one column-inverted plane into `out` (the complex response
// EO_{s,o} itself, for diagnostics).  Block = LINES rows.
template <int W, int P>
__global__ void __launch_bounds__(256) k_rows_inverse(const float2* __restrict__ y_in, float2* __restrict__ out) {
  using PL = FftPlan<W, P>;
  constexpr int T = PL::T;
  constexpr int LINES = 256 / T;
  __shared__ float2 lines[LINES][lds_line<W, T>()];
  const int team = threadIdx.x / T, t = threadIdx.x % T;
  const size_t row = (size_t)(blockIdx.x * LINES + team) * W;
  float2 v[P];
#pragma unroll
  for (int m = 0; m < P; ++m) v[m] = y_in[row + t + T * m];
  fft_line<+1, W, P, T == 64>(v, t, lines[team]);
#pragma unroll
  for (int m = 0; m < P; ++m) out[row + t + T * m] = v[m];
}

// ---------------------------------------------------------------- pass B

// One block per (row, orientation): the row IDFT z_s of every scale stays in
// registers (z_0 was transformed in place by k_noise_pre); Z = E + iO = sum_s z_s, and the energy along the mean phase is
// En = (|Z|^2 - sum_s |Im(z_s conj Z)|) / X with X = |Z| + eps -- the same
// quantity as sum_s (e_s phi_e + o_s phi_o - |e_s phi_o - o_s phi_e|).  The
// pixel's (A_o, PC_o) pair goes to `spc` (orientation-major) for
// k_pass_b_reduce.
template <int W, int P, int NS>
__global__ void __launch_bounds__(W / P) k_pass_b_orient(FilterBatch B, int H, PCConsts pcc) {
  const FilterImage& I = B.im[blockIdx.z];
  const float2* __restrict__ y_in = I.yplanes;
  const float* __restrict__ t_o = I.t32;
  float2* __restrict__ spc = I.spc;
  float* __restrict__ amp = I.amp;
  constexpr int T = W / P;
  // scales past the first are transformed two at a time (shared exchanges)
  // where the second LDS line leaves the occupancy alone; a row team of one
  // wave (T = 64) exchanges with wave barriers only
  constexpr bool PAIR = W <= 2048;
  __shared__ float2 line[PAIR ? 2 : 1][lds_line<W, T>()];
  const int t = threadIdx.x;
  const int y = blockIdx.x, o = blockIdx.y;
  const size_t plane = (size_t)H * W;
  const size_t rowo = (size_t)y * W;
  const float2* base = y_in + (size_t)(o * NS) * plane + rowo + t;
  float2 zs[NS][P];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
#pragma unroll
    for (int m = 0; m < P; ++m) zs[s][m] = base[(size_t)s * plane + T * m];
  }
#pragma unroll
  for (int s = 1; s < NS; s += PAIR ? 2 : 1) {
    if constexpr (PAIR) {
      if (s + 1 < NS) {
        fft_line2<+1, W, P, T == 64>(zs[s], zs[s + 1], t, line[0], line[PAIR ? 1 : 0]);
        continue;
      }
    }
    fft_line<+1, W, P, T == 64>(zs[s], t, line[0]);
  }
  float sa[P], mx[P];
#pragma unroll
  for (int m = 0; m < P; ++m) sa[m] = mx[m] = 0.0f;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
#pragma unroll
    for (int m = 0; m < P; ++m) {
      const float a = hw_sqrt(zs[s][m].x * zs[s][m].x + zs[s][m].y * zs[s][m].y);
      sa[m] += a;
      mx[m] = __uint_as_float(max(__float_as_uint(mx[m]), __float_as_uint(a)));
    }
  }
  const float thr = t_o[o];
  float2* out = spc + (size_t)o * plane + rowo + t;
#pragma unroll
  for (int m = 0; m < P; ++m) {
    float2 z = zs[0][m];
#pragma unroll
    for (int s = 1; s < NS; ++s) z = cadd(z, zs[s][m]);
    float si = 0.0f;
#pragma unroll
    for (int s = 0; s < NS; ++s) si += fabsf(zs[s][m].y * z.x - zs[s][m].x * z.y);
    const float z2 = z.x * z.x + z.y * z.y;
    const float xe = hw_sqrt(z2) + pcc.eps;
    const float en = (z2 - si) * hw_rcp(xe);
    const float spread = (sa[m] * hw_rcp(mx[m] + pcc.eps) - 1.0f) * (1.0f / (float)(NS - 1));
    const float wgt = hw_rcp(1.0f + __expf(pcc.g * (pcc.cutoff - spread)));
    const float pc = wgt * fmaxf(en - thr, 0.0f) * hw_rcp(sa[m] + pcc.eps);
    out[T * m] = make_float2(sa[m], pc);
  }
  if (amp) {
#pragma unroll
    for (int m = 0; m < P; ++m) amp[(size_t)o * plane + rowo + t + T * m] = sa[m];
  }
}

// The row pass with the orientation reduction fused in, for rows that one
// wave transforms (W / P = 64).  One block per row: wave w computes
// orientations w, w + NW, ... exactly as k_pass_b_orient does (its own LDS
// line) and leaves (A_o, PC_o) in LDS instead of `spc`; after one block
// barrier the block reduces each pixel over the orientations in ascending
// order exactly as k_pass_b_reduce does, so the results are bit-identical to
// the split form and the N_o x HW hand-off never reaches memory.  With two
// orientations per wave a block holds 3 waves and about 75 KB of LDS at
// W = 1024, so two blocks share a CU and one's tail overlaps the other's work.
template <int W, int P, int NS, int NO, int G>
__global__ void __launch_bounds__(64 * NO / G) k_pass_b_fused(FilterBatch B, int H, PCConsts pcc) {
  static_assert(W / P == 64 && NO % G == 0, "one wave per row and orientation");
  constexpr int T = 64;
  constexpr int NW = NO / G;
  const FilterImage& I = B.im[blockIdx.z];
  const float2* __restrict__ y_in = I.yplanes;
  __shared__ float2 line[NW][lds_line<W, T>()];
  __shared__ __align__(16) float res_a[NO][W];
  __shared__ __align__(16) float res_p[NO][W];
  const int t = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const size_t plane = (size_t)H * W;
  const size_t rowo = (size_t)blockIdx.x * W;
  for (int j = 0; j < G; ++j) {
    const int o = w + j * NW;
    const float2* base = y_in + (size_t)(o * NS) * plane + rowo + t;
    float2 zs[NS][P];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
      for (int m = 0; m < P; ++m) zs[s][m] = base[(size_t)s * plane + T * m];
    }
#pragma unroll
    for (int s = 1; s < NS; ++s) fft_line<+1, W, P, true>(zs[s], t, line[w]);
    float sa[P], mx[P];
#pragma unroll
    for (int m = 0; m < P; ++m) sa[m] = mx[m] = 0.0f;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
      for (int m = 0; m < P; ++m) {
        const float a = hw_sqrt(zs[s][m].x * zs[s][m].x + zs[s][m].y * zs[s][m].y);
        sa[m] += a;
        mx[m] = __uint_as_float(max(__float_as_uint(mx[m]), __float_as_uint(a)));
      }
    }
    const float thr = I.t32[o];
#pragma unroll
    for (int m = 0; m < P; ++m) {
      float2 z = zs[0][m];
#pragma unroll
      for (int s = 1; s < NS; ++s) z = cadd(z, zs[s][m]);
      float si = 0.0f;
#pragma unroll
      for (int s = 0; s < NS; ++s) si += fabsf(zs[s][m].y * z.x - zs[s][m].x * z.y);
      const float z2 = z.x * z.x + z.y * z.y;
      const float xe = hw_sqrt(z2) + pcc.eps;
      const float en = (z2 - si) * hw_rcp(xe);
      const float spread = (sa[m] * hw_rcp(mx[m] + pcc.eps) - 1.0f) * (1.0f / (float)(NS - 1));
      const float wgt = hw_rcp(1.0f + __expf(pcc.g * (pcc.cutoff - spread)));
      res_a[o][t + T * m] = sa[m];
      res_p[o][t + T * m] = wgt * fmaxf(en - thr, 0.0f) * hw_rcp(sa[m] + pcc.eps);
    }
    if (I.amp) {
#pragma unroll
      for (int m = 0; m < P; ++m) I.amp[(size_t)o * plane + rowo + t + T * m] = sa[m];
    }
  }
  __syncthreads();
  for (int i = 4 * threadIdx.x; i < W; i += 4 * 64 * NW) {
    float best[4], ma[4], mb[4], mc[4];
    int idx[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      best[e] = -1.0f;
      idx[e] = 0;
      ma[e] = mb[e] = mc[e] = 0.0f;
    }
#pragma unroll
    for (int q = 0; q < NO; ++q) {
      const float4 a4 = *(const float4*)&res_a[q][i];
      const float4 p4 = *(const float4*)&res_p[q][i];
      const float av[4] = {a4.x, a4.y, a4.z, a4.w};
      const float pv[4] = {p4.x, p4.y, p4.z, p4.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (av[e] > best[e]) {
          best[e] = av[e];
          idx[e] = q;
        }
        const float pcc_ = pv[e] * pcc.cos_o[q], pcs_ = pv[e] * pcc.sin_o[q];
        ma[e] += pcc_ * pcc_;
        mb[e] += 2.0f * pcc_ * pcs_;
        mc[e] += pcs_ * pcs_;
      }
    }
    float4 mxv, mnv;
    float* mxp = &mxv.x;
    float* mnp = &mnv.x;
    uint32_t packed = 0u;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float root = sqrtf(mb[e] * mb[e] + (ma[e] - mc[e]) * (ma[e] - mc[e]));
      mxp[e] = 0.5f * (ma[e] + mc[e] + root);
      mnp[e] = 0.5f * (ma[e] + mc[e] - root);
      packed |= (uint32_t)idx[e] << (8 * e);
    }
    *(float4*)(I.mmax + rowo + i) = mxv;
    if (I.mmin) *(float4*)(I.mmin + rowo + i) = mnv;
    *(uint32_t*)(I.mim + rowo + i) = packed;
  }
}

// Per pixel over orientations (ascending): MIM = first argmax of A_o,
// moments of PC_o.  Four pixels per thread, 16-byte accesses.
template <int NO>
__global__ void __launch_bounds__(256) k_pass_b_reduce(FilterBatch B, int hw, PCConsts pcc) {
  const FilterImage& I = B.im[blockIdx.z];
  const float2* __restrict__ spc = I.spc;
  uint8_t* __restrict__ mim = I.mim;
  float* __restrict__ mmax = I.mmax;
  float* __restrict__ mmin = I.mmin;
  const int i = 4 * (blockIdx.x * 256 + threadIdx.x);
  if (i >= hw) return;  // hw is a multiple of 4
  float best[4], ma[4], mb[4], mc[4];
  int idx[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    best[e] = -1.0f;
    idx[e] = 0;
    ma[e] = mb[e] = mc[e] = 0.0f;
  }
#pragma unroll
  for (int q = 0; q < NO; ++q) {
    const float4* src = (const float4*)(spc + (size_t)q * hw + i);
    const float4 r01 = src[0], r23 = src[1];
    const float av[4] = {r01.x, r01.z, r23.x, r23.z};
    const float pv[4] = {r01.y, r01.w, r23.y, r23.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (av[e] > best[e]) {
        best[e] = av[e];
        idx[e] = q;
      }
      const float pcc_ = pv[e] * pcc.cos_o[q], pcs_ = pv[e] * pcc.sin_o[q];
      ma[e] += pcc_ * pcc_;
      mb[e] += 2.0f * pcc_ * pcs_;
      mc[e] += pcs_ * pcs_;
    }
  }
  float4 mxv, mnv;
  float* mxp = &mxv.x;
  float* mnp = &mnv.x;
  uint32_t packed = 0u;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float root = sqrtf(mb[e] * mb[e] + (ma[e] - mc[e]) * (ma[e] - mc[e]));
    mxp[e] = 0.5f * (ma[e] + mc[e] + root);
    mnp[e] = 0.5f * (ma[e] + mc[e] - root);
    packed |= (uint32_t)idx[e] << (8 * e);
  }
  *(float4*)(mmax + i) = mxv;
  if (mmin) *(float4*)(mmin + i) = mnv;
  *(uint32_t*)(mim + i) = packed;
}

}  // namespace rift2
