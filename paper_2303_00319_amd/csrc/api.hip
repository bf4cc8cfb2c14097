// C ABI of librift2.so: argument validation, workspace layout, kernel launches.
// The declarations and their documentation live in include/rift2.h.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "rift2.h"
#include "describe.hip"
#include "detect.hip"
#include "fft.hpp"
#include "filter.hip"
#include "match.hip"
#include "match_fp8.hip"
#include "ransac.hip"
#include "engine.hip"
#include "calib.hip"

using namespace rift2;

// Detection scratch of rift2_detect_noalloc: the library holds it on every
// device it runs on until the process ends.  In host code `scratch` names a
// host-side stand-in, never the device memory; rift2_init looks up each
// device's own address of it with hipGetSymbolAddress, and only that address
// is passed to kernels.
constexpr size_t kNoAllocScratchBytes = (size_t)20 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Sequential carve of a workspace into aligned regions.
struct Carver {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  }
};

constexpr int kNoiseRegions = 256;  // k_noise_sel1 / k_noise_sel2 blocks (candidate list regions) per orientation

bool size_ok(int n) {
  switch (n) {
    case 256: case 512: case 768: case 1024: case 1536: case 2048: case 4096: return true;
    default: return false;
  }
}

bool pc_ok(const rift2_pc_params* p) {
  return p && p->n_scales >= 2 && p->n_scales <= kMaxScales && p->n_orient >= 2 && p->n_orient <= kMaxOrient &&
         p->min_wavelength > 0.f && p->mult > 1.f && p->sigma_onf > 0.f && p->sigma_onf < 1.f &&
         p->dtheta_on_sigma > 0.f && p->lp_cutoff > 0.f && p->lp_order >= 1 && p->lp_order <= 64 && p->eps > 0.f &&
         std::isfinite(p->k) && std::isfinite(p->cutoff) && std::isfinite(p->g);
}

// Only the (N_s, N_o) combinations instantiated for pass B.
bool pc_built(const rift2_pc_params* p) {
  return (p->n_scales == 4 && p->n_orient == 6) || (p->n_scales == 5 && p->n_orient == 8) ||
         (p->n_scales == 4 && p->n_orient == 8) || (p->n_scales == 5 && p->n_orient == 6);
}

struct FilterLayout {
  size_t rrow, yplanes, a0, cand, spc, zero, t32, t64, ostat, total;
  int zero_words;
};

FilterLayout filter_layout(int H, int W, const rift2_pc_params* p) {
  FilterLayout L;
  const size_t hw = (size_t)H * W;
  const int F = p->n_scales * p->n_orient;
  Carver c;
  L.rrow = c.take(hw * sizeof(float2));
  L.yplanes = c.take(hw * F * sizeof(float2));
  L.a0 = c.take(hw * p->n_orient * sizeof(float));
  L.cand = c.take(hw * p->n_orient * sizeof(uint32_t));
  L.spc = c.take(hw * p->n_orient * sizeof(float2));
  L.zero_words = p->n_orient * (kHist1 + 2 * kHist2 + 2 * kHist3 + 8 + kNoiseRegions);
  L.zero = c.take((size_t)L.zero_words * sizeof(uint32_t));
  L.t32 = c.take(p->n_orient * sizeof(float));
  L.t64 = c.take(p->n_orient * sizeof(double));
  L.ostat = c.take(2 * p->n_orient * sizeof(float));
  L.total = c.off;
  return L;
}

struct DetectLayout {
  size_t hdr, mm, hist, tile_cnt, cand, sel_cnt, sel, fin, part, above, cursor, total;
  int n_tiles, n_part;
  bool count_sort;
  uint32_t region;
};

// maps = 2: the corner + edge union, whose candidate lists are twice the tiles.
DetectLayout detect_layout(int H, int W, const rift2_detect_params* d, int maps = 1) {
  DetectLayout L;
  Carver c;
  L.n_tiles = maps * ((W + kTileX - 1) / kTileX) * ((H + kTileY - 1) / kTileY);
  const size_t slots = (size_t)L.n_tiles * kTileCap;
  L.region = (uint32_t)(((L.n_tiles + kSelBlocks - 1) / kSelBlocks) * kTileCap);  // k_det_select1 tiles per block
  L.hdr = c.take(64);
  L.mm = c.take(2 * maps * kMinMaxBlocks * sizeof(uint32_t));
  L.hist = c.take(kDetHistBins * sizeof(uint32_t));
  L.tile_cnt = c.take((size_t)L.n_tiles * sizeof(uint32_t));
  L.cand = c.take(slots * sizeof(uint64_t));
  L.sel_cnt = c.take(kSelBlocks * sizeof(uint32_t));
  L.sel = c.take((size_t)L.region * kSelBlocks * sizeof(uint64_t));
  const size_t kmax = d ? (size_t)d->max_keypoints : 0;
  L.fin = c.take(kmax * sizeof(uint64_t) + 8);
  L.count_sort = kmax >= kCountSortMin;
  const int blocks = (int)((kmax + 255) / 256);
  L.n_part = std::max(1, std::min(32, 512 / std::max(1, blocks)));
  if (L.count_sort) {
    // the winners in score-bin order, the bins' offsets and scatter cursors
    L.part = c.take(kmax * sizeof(uint64_t) + 8);
    L.above = c.take(kDetHistBins * sizeof(uint32_t));
    L.cursor = c.take(kDetHistBins * sizeof(uint32_t));
  } else {
    L.part = c.take((size_t)L.n_part * kmax * sizeof(uint32_t) + 8);
    L.above = L.cursor = 0;
  }
  L.total = c.off;
  return L;
}

// How one GEMM direction splits its candidate rows into slices.
struct SliceShape {
  int slices, slice_rows;
};

int round_up(int v, int m) { return (v + m - 1) / m * m; }

SliceShape slice_shape(int rows_q, int rows_c, bool fp32) {
  SliceShape s;
  const int blocks_x = (rows_q + 127) / 128;
  // enough blocks to fill the chip several times over (256 CUs x 2 blocks), slices of >= 2 tiles; the
  // FP32 kernel (long MFMA chain per tile, one tile buffer) measured best with more, shorter slices
  const int target_blocks = fp32 ? 6144 : 4096;
  int slices = (target_blocks + blocks_x - 1) / blocks_x;
  const int max_slices = (rows_c + 63) / 64;
  if (slices > max_slices) slices = max_slices;
  if (slices < 1) slices = 1;
  s.slice_rows = round_up((rows_c + slices - 1) / slices, 32);
  s.slices = (rows_c + s.slice_rows - 1) / s.slice_rows;
  return s;
}

// Mutual mode adds the reverse GEMM's lists (B rows as queries, A rows as
// candidates) and each B row's nearest A row.
struct MatchLayout {
  size_t ta, tb, wa, wb, part, best, rowj, rowd, part_r, a1, total;
  int dp, rs, rows_a, rows_b, slices, slice_rows, topk, slices_r, slice_rows_r;
};

MatchLayout match_layout(int cap_a, int cap_b, int D, int precision, bool mutual = false) {
  MatchLayout L;
  const bool bf = precision == RIFT2_PREC_BF16;
  const bool f8 = precision == RIFT2_PREC_FP8;
  // table row stride = the GEMM kernels' LDS row stride (elements)
  if (f8) {
    L.dp = round_up(D, 64);
    L.rs = L.dp + 16;
  } else if (bf) {
    L.dp = round_up(D, 16);
    L.rs = L.dp + 8;
  } else {
    L.dp = round_up(D, 8);
    L.rs = L.dp + 4;
  }
  L.topk = f8 ? kTopK8 : kTopK;
  L.rows_a = round_up(cap_a, 32);
  L.rows_b = round_up(cap_b, 32);
  const SliceShape fw = slice_shape(L.rows_a, L.rows_b, !(bf || f8));
  L.slices = fw.slices;
  L.slice_rows = fw.slice_rows;
  const SliceShape rv = slice_shape(L.rows_b, L.rows_a, !(bf || f8));
  L.slices_r = mutual ? rv.slices : 0;
  L.slice_rows_r = mutual ? rv.slice_rows : 0;
  const size_t el = f8 ? 1 : (bf ? 2 : 4);
  Carver c;
  L.ta = c.take((size_t)L.rows_a * L.rs * el);
  L.tb = c.take((size_t)L.rows_b * L.rs * el);
  L.wa = c.take((size_t)L.rows_a * sizeof(float));
  L.wb = c.take((size_t)L.rows_b * sizeof(float));
  L.part = c.take((size_t)L.rows_a * L.slices * 2 * L.topk * sizeof(int2));
  L.best = c.take((size_t)cap_a * sizeof(uint64_t));
  L.rowj = c.take((size_t)cap_a * sizeof(int32_t));
  L.rowd = c.take((size_t)cap_a * sizeof(float));
  L.part_r = c.take(mutual ? (size_t)L.rows_b * L.slices_r * 2 * L.topk * sizeof(int2) : 0);
  L.a1 = c.take(mutual ? (size_t)cap_b * sizeof(int32_t) : 0);
  L.total = c.off;
  return L;
}

struct RansacLayout {
  size_t xy, flags, key, sums, counts, total;
  int n_flags;
};

bool ransac_layout(int match_cap, int n_hyp, RansacLayout* L) {
  if (match_cap < 1 || match_cap > kRansacMaxMatches || n_hyp < 0 || n_hyp > kRansacMaxHyp) return false;
  Carver c;
  L->n_flags = (match_cap + 255) / 256;
  L->xy = c.take((size_t)match_cap * sizeof(int4));
  L->flags = c.take((size_t)L->n_flags * sizeof(int32_t));
  L->key = c.take(sizeof(unsigned long long));
  L->sums = c.take((size_t)kRansacMaxRefine * 8 * sizeof(unsigned long long));
  L->counts = c.take((size_t)n_hyp * sizeof(int32_t));
  L->total = c.off;
  return true;
}

rift2_status launch_status() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? RIFT2_OK : RIFT2_ERR_DEVICE;
}

std::mutex g_init_mu;
bool g_init_done[64] = {};
// Device address of `scratch` on each device, taken by rift2_init with that device current.
void* g_scratch_dev[64] = {};

// The FFT kernels read the twiddle tables that rift2_init loads per device.
bool current_device_ready() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
  std::lock_guard<std::mutex> lock(g_init_mu);
  return g_init_done[dev];
}

// ---- stage timing (diagnostics)
constexpr int kProfGroups = 12;
struct ProfRec {
  int group;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;

// Records an event pair around the kernels enqueued during its lifetime.
struct ProfScope {
  int group;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(int g, hipStream_t s, bool timed = true) : group(g), st(s) {
    if (!g_prof_on || !timed) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess ||
        hipEventRecord(a, st) != hipSuccess) {
      a = b = nullptr;
    }
  }
  void finish() {
    if (!a) return;
    if (hipEventRecord(b, st) == hipSuccess) {
      std::lock_guard<std::mutex> lock(g_prof_mu);
      g_prof.push_back({group, a, b});
    } else {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
    a = b = nullptr;
  }
  ~ProfScope() { finish(); }
};

}  // namespace

// ---------------------------------------------------------------- kernel dispatch tables

namespace {

// Every filter-bank launch covers the n images of a batch (grid z).
template <int W, int P, typename Tin>
void launch_fwd_rows(const FilterBatch& B, int n, int64_t pitch, int H, int n_zero, hipStream_t st) {
  constexpr int LINES = 256 / FftPlan<W, P>::T;
  hipLaunchKernelGGL((k_fwd_rows<W, P, Tin>), dim3(H / LINES, 1, n), dim3(256), 0, st, B, pitch, n_zero);
}

template <int W, int P>
bool fwd_rows_dtype(int dtype, const FilterBatch& B, int n, int64_t pitch, int H, int n_zero, hipStream_t st) {
  switch (dtype) {
    case RIFT2_U8: launch_fwd_rows<W, P, uint8_t>(B, n, pitch, H, n_zero, st); return true;
    case RIFT2_U16: launch_fwd_rows<W, P, uint16_t>(B, n, pitch, H, n_zero, st); return true;
    case RIFT2_F32: launch_fwd_rows<W, P, float>(B, n, pitch, H, n_zero, st); return true;
    default: return false;
  }
}

bool dispatch_fwd_rows(int W, int dtype, const FilterBatch& B, int n, int64_t pitch, int H, int n_zero,
                       hipStream_t st) {
  switch (W) {
    case 256: return fwd_rows_dtype<256, 16>(dtype, B, n, pitch, H, n_zero, st);
    case 512: return fwd_rows_dtype<512, 16>(dtype, B, n, pitch, H, n_zero, st);
    case 768: return fwd_rows_dtype<768, 12>(dtype, B, n, pitch, H, n_zero, st);
    case 1024: return fwd_rows_dtype<1024, 16>(dtype, B, n, pitch, H, n_zero, st);
    case 1536: return fwd_rows_dtype<1536, 12>(dtype, B, n, pitch, H, n_zero, st);
    case 2048: return fwd_rows_dtype<2048, 16>(dtype, B, n, pitch, H, n_zero, st);
    case 4096: return fwd_rows_dtype<4096, 16>(dtype, B, n, pitch, H, n_zero, st);
    default: return false;
  }
}

template <int H, int P, int C>
void launch_pass_a(int W, const FilterBatch& B, int n, const FilterConsts& fc, hipStream_t st, int min_blocks = 512) {
  // Split the orientations over grid.y until there are >= min_blocks blocks
  // per image; each group recomputes the column DFT of its block (an extra
  // read of Rrow).
  const int xblocks = W / C;
  int groups = (min_blocks + xblocks - 1) / xblocks;
  if (groups > fc.n_orient) groups = fc.n_orient;
  if (groups < 1) groups = 1;
  hipLaunchKernelGGL((k_pass_a<H, P, C>), dim3(xblocks, groups, n), dim3(C * (H / P)), 0, st, B, fc);
}

bool dispatch_pass_a(int H, int W, const FilterBatch& B, int n, const FilterConsts& fc, hipStream_t st) {
  switch (H) {
    case 256: launch_pass_a<256, 16, 16>(W, B, n, fc, st); return true;
    case 512: launch_pass_a<512, 16, 16>(W, B, n, fc, st); return true;
    case 768: launch_pass_a<768, 12, 8>(W, B, n, fc, st); return true;
    case 1024: launch_pass_a<1024, 8, 8>(W, B, n, fc, st, 256); return true;
    case 1536: launch_pass_a<1536, 12, 4>(W, B, n, fc, st); return true;
    case 2048: launch_pass_a<2048, 16, 4>(W, B, n, fc, st); return true;
    case 4096: launch_pass_a<4096, 16, 2>(W, B, n, fc, st); return true;
    default: return false;
  }
}

template <int W, int P>
void launch_noise_pre(int H, int n_orient, int n_scales, const FilterBatch& B, int n, hipStream_t st) {
  constexpr int LINES = 256 / FftPlan<W, P>::T;
  hipLaunchKernelGGL((k_noise_pre<W, P>), dim3(H / LINES, n_orient, n), dim3(256), 0, st, B, H, n_scales, n_orient,
                     kNoiseRegions);
}

bool dispatch_noise_pre(int W, int H, int n_orient, int n_scales, const FilterBatch& B, int n, hipStream_t st) {
  switch (W) {
    case 256: launch_noise_pre<256, 16>(H, n_orient, n_scales, B, n, st); return true;
    case 512: launch_noise_pre<512, 16>(H, n_orient, n_scales, B, n, st); return true;
    case 768: launch_noise_pre<768, 12>(H, n_orient, n_scales, B, n, st); return true;
    case 1024: launch_noise_pre<1024, 16>(H, n_orient, n_scales, B, n, st); return true;
    case 1536: launch_noise_pre<1536, 12>(H, n_orient, n_scales, B, n, st); return true;
    case 2048: launch_noise_pre<2048, 16>(H, n_orient, n_scales, B, n, st); return true;
    case 4096: launch_noise_pre<4096, 16>(H, n_orient, n_scales, B, n, st); return true;
    default: return false;
  }
}

template <int W, int P>
void launch_rows_inverse(int H, const float2* y, float2* out, hipStream_t st) {
  constexpr int LINES = 256 / FftPlan<W, P>::T;
  hipLaunchKernelGGL((k_rows_inverse<W, P>), dim3(H / LINES), dim3(256), 0, st, y, out);
}

bool dispatch_rows_inverse(int W, int H, const float2* y, float2* out, hipStream_t st) {
  switch (W) {
    case 256: launch_rows_inverse<256, 16>(H, y, out, st); return true;
    case 512: launch_rows_inverse<512, 16>(H, y, out, st); return true;
    case 768: launch_rows_inverse<768, 12>(H, y, out, st); return true;
    case 1024: launch_rows_inverse<1024, 16>(H, y, out, st); return true;
    case 1536: launch_rows_inverse<1536, 12>(H, y, out, st); return true;
    case 2048: launch_rows_inverse<2048, 16>(H, y, out, st); return true;
    case 4096: launch_rows_inverse<4096, 16>(H, y, out, st); return true;
    default: return false;
  }
}

template <int W, int P, int NS, int NO>
void launch_pass_b_split(int H, const FilterBatch& B, int n, const PCConsts& pcc, hipStream_t st) {
  {
    ProfScope ps(4, st);
    hipLaunchKernelGGL((k_pass_b_orient<W, P, NS>), dim3(H, NO, n), dim3(W / P), 0, st, B, H, pcc);
  }
  const int hw = H * W;
  ProfScope ps(10, st);
  hipLaunchKernelGGL((k_pass_b_reduce<NO>), dim3((hw / 4 + 255) / 256, 1, n), dim3(256), 0, st, B, hw, pcc);
}

// Rows of one wave with N_s = 4, N_o = 6: the fused row pass, two
// orientations per wave (3-wave blocks, so two blocks share a CU): 69.7 ->
// 64.7 us per 1024^2 image against the split pair of launches, with
// bit-identical results.  Other filter counts and longer rows keep the split
// form.
template <int W, int P, int NS, int NO>
void launch_pass_b(int H, const FilterBatch& B, int n, const PCConsts& pcc, hipStream_t st) {
  if constexpr (NS == 4 && NO == 6 && W / P == 64) {
    ProfScope ps(4, st);
    hipLaunchKernelGGL((k_pass_b_fused<W, P, NS, NO, 2>), dim3(H, 1, n), dim3(64 * NO / 2), 0, st, B, H, pcc);
  } else {
    launch_pass_b_split<W, P, NS, NO>(H, B, n, pcc, st);
  }
}

template <int NS, int NO>
bool pass_b_w(int W, int H, const FilterBatch& B, int n, const PCConsts& pcc, hipStream_t st) {
  switch (W) {
    case 256: launch_pass_b<256, 4, NS, NO>(H, B, n, pcc, st); return true;
    case 512: launch_pass_b<512, 8, NS, NO>(H, B, n, pcc, st); return true;
    case 768: launch_pass_b<768, 12, NS, NO>(H, B, n, pcc, st); return true;
    case 1024: launch_pass_b<1024, 16, NS, NO>(H, B, n, pcc, st); return true;
    case 1536: launch_pass_b_split<1536, 12, NS, NO>(H, B, n, pcc, st); return true;
    case 2048: launch_pass_b_split<2048, 8, NS, NO>(H, B, n, pcc, st); return true;
    case 4096: launch_pass_b_split<4096, 16, NS, NO>(H, B, n, pcc, st); return true;
    default: return false;
  }
}

bool dispatch_pass_b(int ns, int no, int W, int H, const FilterBatch& B, int n, const PCConsts& pcc, hipStream_t st) {
  if (ns == 4 && no == 6) return pass_b_w<4, 6>(W, H, B, n, pcc, st);
  if (ns == 5 && no == 8) return pass_b_w<5, 8>(W, H, B, n, pcc, st);
  if (ns == 4 && no == 8) return pass_b_w<4, 8>(W, H, B, n, pcc, st);
  if (ns == 5 && no == 6) return pass_b_w<5, 6>(W, H, B, n, pcc, st);
  return false;
}

// FP32 or BF16 distance GEMM of one direction: queries q against candidates c.
template <bool CF>
void launch_gemm_exact(bool bf, int dp, const void* tq, const float* inv_q, const int32_t* nq_dev, int cap_q,
                       const void* tc, const float* inv_c, const int32_t* nc_dev, int cap_c, int rows_q,
                       int slice_rows, int slices, int2* part, hipStream_t st) {
  const dim3 grid((rows_q + 127) / 128, slices);
  if (bf) {
    // the BF16 GEMM deals its cells to the XCDs itself (gemm_cell): 1-D grid
    const dim3 grid_xcd(8 * ((grid.x + 1) / 2) * ((slices + 3) / 4));
    if (dp == 224)
      hipLaunchKernelGGL((k_match_gemm_bf16<224, CF>), grid_xcd, dim3(256), 0, st, (const uint16_t*)tq, inv_q, nq_dev,
                         (const uint16_t*)tc, inv_c, nc_dev, cap_q, cap_c, slice_rows, slices, part);
    else
      hipLaunchKernelGGL((k_match_gemm_bf16<288, CF>), grid_xcd, dim3(256), 0, st, (const uint16_t*)tq, inv_q, nq_dev,
                         (const uint16_t*)tc, inv_c, nc_dev, cap_q, cap_c, slice_rows, slices, part);
  } else {
    if (dp == 216)
      hipLaunchKernelGGL((k_match_gemm_f32<216, CF>), grid, dim3(256), 0, st, (const float*)tq, inv_q, nq_dev,
                         (const float*)tc, inv_c, nc_dev, cap_q, cap_c, slice_rows, part);
    else
      hipLaunchKernelGGL((k_match_gemm_f32<288, CF>), grid, dim3(256), 0, st, (const float*)tq, inv_q, nq_dev,
                         (const float*)tc, inv_c, nc_dev, cap_q, cap_c, slice_rows, part);
  }
}

void launch_gemm_fp8(int dp, const uint8_t* tq, const float* wq, const int32_t* nq_dev, int cap_q, const uint8_t* tc,
                     const float* wc, const int32_t* nc_dev, int cap_c, int rows_q, int slice_rows, int slices,
                     int2* part, hipStream_t st) {
  const dim3 grid((rows_q + 127) / 128, slices);
  if (dp == 256)
    hipLaunchKernelGGL(k_match_gemm_fp8<256>, grid, dim3(256), 0, st, tq, wq, nq_dev, tc, wc, nc_dev, cap_q, cap_c,
                       slice_rows, part);
  else
    hipLaunchKernelGGL(k_match_gemm_fp8<320>, grid, dim3(256), 0, st, tq, wq, nq_dev, tc, wc, nc_dev, cap_q, cap_c,
                       slice_rows, part);
}

// Constants of the filter bank, phase congruency and noise model for the kernels.
void filter_consts(int H, int W, const rift2_pc_params* pc, FilterConsts* fcp, PCConsts* pccp, NoiseConsts* ncp) {
  FilterConsts& fc = *fcp;
  std::memset(&fc, 0, sizeof(fc));
  fc.H = H;
  fc.W = W;
  fc.n_scales = pc->n_scales;
  fc.n_orient = pc->n_orient;
  const double ls = std::log((double)pc->sigma_onf);
  fc.inv_2ln2_sigma = (float)(1.0 / (2.0 * ls * ls));
  for (int s = 0; s < pc->n_scales; ++s)
    fc.log_f0[s] = (float)std::log(1.0 / ((double)pc->min_wavelength * std::pow((double)pc->mult, (double)s)));
  fc.log_lp_cutoff = (float)std::log((double)pc->lp_cutoff);
  fc.two_n = (float)(2 * pc->lp_order);
  PCConsts& pcc = *pccp;
  std::memset(&pcc, 0, sizeof(pcc));
  for (int o = 0; o < pc->n_orient; ++o) {
    const double th = o * M_PI / pc->n_orient;
    fc.theta_o[o] = (float)th;
    pcc.cos_o[o] = (float)std::cos(th);
    pcc.sin_o[o] = (float)std::sin(th);
  }
  const double sig_th = (M_PI / pc->n_orient) / (double)pc->dtheta_on_sigma;
  fc.inv_2sig_theta2 = (float)(1.0 / (2.0 * sig_th * sig_th));
  fc.inv_hw = (float)(1.0 / ((double)H * (double)W));
  pcc.eps = pc->eps;
  pcc.g = pc->g;
  pcc.cutoff = pc->cutoff;
  NoiseConsts& nc = *ncp;
  nc.mult = pc->mult;
  nc.k = pc->k;
  nc.n_scales = pc->n_scales;

}

}  // namespace

// ---------------------------------------------------------------- C ABI

extern "C" {

void rift2_default_params(rift2_pc_params* pc, rift2_detect_params* det, rift2_desc_params* desc,
                          rift2_match_params* match) {
  if (pc) {
    pc->n_scales = 4;
    pc->n_orient = 6;
    pc->min_wavelength = 3.0f;
    pc->mult = 2.1f;
    pc->sigma_onf = 0.55f;
    pc->dtheta_on_sigma = 1.2f;
    pc->lp_cutoff = 0.45f;
    pc->lp_order = 15;
    pc->k = 2.0f;
    pc->cutoff = 0.5f;
    pc->g = 10.0f;
    pc->eps = 1e-4f;
  }
  if (det) {
    det->fast_threshold = 0.001f;
    det->max_keypoints = 5000;
    det->patch_size = 96;
  }
  if (desc) {
    desc->patch_size = 96;
    desc->grid = 6;
    desc->n_orient = 6;
    desc->dominant_num = 4;
    desc->dominant_den = 5;
    desc->mode = RIFT2_DESC_DOMINANT;
  }
  if (match) {
    match->ratio_sq = 0.81f;
    match->precision = RIFT2_PREC_FP32;
    match->ring = 0;
    match->mutual = 0;
  }
}

const char* rift2_status_string(rift2_status s) {
  switch (s) {
    case RIFT2_OK: return "ok";
    case RIFT2_ERR_INVALID_ARG: return "invalid argument";
    case RIFT2_ERR_UNSUPPORTED: return "unsupported size or parameter";
    case RIFT2_ERR_WORKSPACE: return "workspace too small";
    case RIFT2_ERR_DEVICE: return "device error";
    case RIFT2_ERR_NOT_INITIALIZED: return "rift2_init has not run on the current device";
    default: return "unknown status";
  }
}

int rift2_size_supported(int n) { return size_ok(n) ? 1 : 0; }

rift2_status rift2_init(int device) {
  if (device < 0 || device >= 64) return RIFT2_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_init_mu);
  if (g_init_done[device]) return RIFT2_OK;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return RIFT2_ERR_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return RIFT2_ERR_DEVICE;
  static float2 host_tw[kTwTotal];
  for (int len : kTwLengths) {
    float2* tab = host_tw + tw_offset(len);
    for (int m = 0; m < len; ++m) {
      const double a = -2.0 * M_PI * (double)m / (double)len;
      tab[m] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
  }
  const hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_twiddle), host_tw, sizeof(host_tw), 0, hipMemcpyHostToDevice);
  void* sp = nullptr;
  const hipError_t es = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
  (void)hipSetDevice(prev);
  if (e != hipSuccess || es != hipSuccess || sp == nullptr) return RIFT2_ERR_DEVICE;
  g_scratch_dev[device] = sp;
  g_init_done[device] = true;
  return RIFT2_OK;
}

size_t rift2_filter_workspace_size(int H, int W, const rift2_pc_params* pc) {
  if (!size_ok(H) || !size_ok(W) || !pc_ok(pc)) return 0;
  return filter_layout(H, W, pc).total;
}

size_t rift2_detect_workspace_size(int H, int W, const rift2_detect_params* det) {
  if (H <= 0 || W <= 0 || !det || det->max_keypoints <= 0) return 0;
  return detect_layout(H, W, det).total;
}

size_t rift2_detect_union_workspace_size(int H, int W, const rift2_detect_params* det) {
  if (H <= 0 || W <= 0 || !det || det->max_keypoints <= 0) return 0;
  return detect_layout(H, W, det, 2).total;
}

// info word per keypoint, then the turned-grid form's staged second rows
// (largest descriptor, 6 x 6 x 8) and their inverse norms.
struct DescLayout {
  size_t info, stage, stage_inv, total;
};
constexpr int kDescMaxD = 6 * 6 * 8;

DescLayout desc_layout(int kpt_cap) {
  DescLayout L;
  Carver c;
  L.info = c.take((size_t)kpt_cap * sizeof(uint32_t));
  L.stage = c.take((size_t)kpt_cap * kDescMaxD * sizeof(uint16_t));
  L.stage_inv = c.take((size_t)kpt_cap * sizeof(float));
  L.total = c.off;
  return L;
}

size_t rift2_describe_workspace_size(int32_t kpt_cap) {
  if (kpt_cap <= 0) return 0;
  return desc_layout(kpt_cap).total;
}

size_t rift2_match_workspace_size(int32_t cap_a, int32_t cap_b, int32_t D, const rift2_match_params* mp) {
  if (cap_a <= 0 || cap_b <= 0 || D <= 0 || !mp) return 0;
  return match_layout(cap_a, cap_b, D, mp->precision, mp->mutual != 0).total;
}

namespace {

// One image's pointers inside the batch record (workspace regions carved by
// the filter layout).
FilterImage filter_image(const FilterLayout& L, const void* img, void* workspace, uint8_t* mim, float* mmax,
                         float* mmin, float* amp) {
  char* ws = (char*)workspace;
  FilterImage I;
  I.img = img;
  I.rrow = (float2*)(ws + L.rrow);
  I.yplanes = (float2*)(ws + L.yplanes);
  I.a0 = (float*)(ws + L.a0);
  I.cand = (uint32_t*)(ws + L.cand);
  I.zero = (uint32_t*)(ws + L.zero);
  I.t32 = (float*)(ws + L.t32);
  I.t64 = (double*)(ws + L.t64);
  I.ostat = (float*)(ws + L.ostat);
  I.spc = (float2*)(ws + L.spc);
  I.mim = mim;
  I.mmax = mmax;
  I.mmin = mmin;
  I.amp = amp;
  return I;
}

rift2_status filter_batch(int32_t n, const rift2_filter_job* jobs, int32_t dtype, int32_t H, int32_t W, int64_t pitch,
                          const rift2_pc_params* pc, void* stream) {
  if (n < 1 || n > RIFT2_MAX_FILTER_BATCH || !jobs || !pc) return RIFT2_ERR_INVALID_ARG;
  if (dtype != RIFT2_U8 && dtype != RIFT2_U16 && dtype != RIFT2_F32) return RIFT2_ERR_INVALID_ARG;
  if (pitch < W) return RIFT2_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    const rift2_filter_job& j = jobs[i];
    if (!j.img || !j.mim || !j.max_moment || !j.workspace) return RIFT2_ERR_INVALID_ARG;
    // the per-pixel reduction stores 4 pixels at a time
    if (((uintptr_t)j.mim & 3u) || ((uintptr_t)j.max_moment & 15u) || ((uintptr_t)j.min_moment & 15u) ||
        ((uintptr_t)j.amp_sums & 3u))
      return RIFT2_ERR_INVALID_ARG;
  }
  if (!pc_ok(pc)) return RIFT2_ERR_INVALID_ARG;
  if (!size_ok(H) || !size_ok(W) || !pc_built(pc)) return RIFT2_ERR_UNSUPPORTED;
  const FilterLayout L = filter_layout(H, W, pc);
  for (int i = 0; i < n; ++i)
    if (jobs[i].workspace_bytes < L.total) return RIFT2_ERR_WORKSPACE;
  // the images of one launch write their workspaces concurrently
  for (int i = 0; i < n; ++i)
    for (int k = i + 1; k < n; ++k) {
      const uintptr_t a = (uintptr_t)jobs[i].workspace, b = (uintptr_t)jobs[k].workspace;
      if (a < b + L.total && b < a + L.total) return RIFT2_ERR_INVALID_ARG;
    }
  if (!current_device_ready()) return RIFT2_ERR_NOT_INITIALIZED;
  hipStream_t st = (hipStream_t)stream;
  FilterBatch B;
  std::memset(&B, 0, sizeof(B));
  for (int i = 0; i < n; ++i) {
    const rift2_filter_job& j = jobs[i];
    B.im[i] = filter_image(L, j.img, j.workspace, j.mim, j.max_moment, j.min_moment, j.amp_sums);
  }
  FilterConsts fc;
  PCConsts pcc;
  NoiseConsts nc;
  filter_consts(H, W, pc, &fc, &pcc, &nc);
  (void)hipGetLastError();
  {
    ProfScope ps(0, st);
    dispatch_fwd_rows(W, dtype, B, n, pitch, H, L.zero_words, st);
  }
  {
    ProfScope ps(1, st);
    dispatch_pass_a(H, W, B, n, fc, st);
  }
  {
    ProfScope ps(2, st);
    dispatch_noise_pre(W, H, pc->n_orient, pc->n_scales, B, n, st);
  }
  const int hw = H * W;
  {
    ProfScope ps(3, st);
    hipLaunchKernelGGL(k_noise_sel1, dim3(kNoiseRegions, pc->n_orient, n), dim3(256), 0, st, B, hw, pc->n_orient,
                       kNoiseRegions);
    hipLaunchKernelGGL(k_noise_sel2, dim3(kNoiseRegions, pc->n_orient, n), dim3(256), 0, st, B, hw, pc->n_orient,
                       kNoiseRegions);
    hipLaunchKernelGGL(k_noise_threshold, dim3(pc->n_orient, 1, n), dim3(256), 0, st, B, hw, pc->n_orient,
                       kNoiseRegions, nc);
  }
  dispatch_pass_b(pc->n_scales, pc->n_orient, W, H, B, n, pcc, st);
  return launch_status();
}

}  // namespace

rift2_status rift2_filter_mim(const void* img, int32_t dtype, int32_t H, int32_t W, int64_t pitch,
                              const rift2_pc_params* pc, uint8_t* mim, float* max_moment, float* min_moment,
                              float* amp_sums, void* workspace, size_t workspace_bytes, void* stream) {
  const rift2_filter_job job{img, mim, max_moment, min_moment, amp_sums, workspace, workspace_bytes};
  return filter_batch(1, &job, dtype, H, W, pitch, pc, stream);
}

rift2_status rift2_filter_mim_batch(int32_t n, const rift2_filter_job* jobs, int32_t dtype, int32_t H, int32_t W,
                                    int64_t pitch, const rift2_pc_params* pc, void* stream) {
  return filter_batch(n, jobs, dtype, H, W, pitch, pc, stream);
}

rift2_status rift2_debug_response(const void* img, int32_t dtype, int32_t H, int32_t W, int64_t pitch,
                                  const rift2_pc_params* pc, int32_t scale, int32_t orient, float* eo,
                                  void* workspace, size_t workspace_bytes, void* stream) {
  if (!img || !pc || !eo || !workspace) return RIFT2_ERR_INVALID_ARG;
  if (dtype != RIFT2_U8 && dtype != RIFT2_U16 && dtype != RIFT2_F32) return RIFT2_ERR_INVALID_ARG;
  if (pitch < W || ((uintptr_t)eo & 7u)) return RIFT2_ERR_INVALID_ARG;
  if (!pc_ok(pc)) return RIFT2_ERR_INVALID_ARG;
  if (scale < 0 || scale >= pc->n_scales || orient < 0 || orient >= pc->n_orient) return RIFT2_ERR_INVALID_ARG;
  if (!size_ok(H) || !size_ok(W)) return RIFT2_ERR_UNSUPPORTED;
  const FilterLayout L = filter_layout(H, W, pc);
  if (workspace_bytes < L.total) return RIFT2_ERR_WORKSPACE;
  if (!current_device_ready()) return RIFT2_ERR_NOT_INITIALIZED;
  hipStream_t st = (hipStream_t)stream;
  FilterBatch B;
  std::memset(&B, 0, sizeof(B));
  B.im[0] = filter_image(L, img, workspace, nullptr, nullptr, nullptr, nullptr);
  const float2* yp = B.im[0].yplanes;
  FilterConsts fc;
  PCConsts pcc;
  NoiseConsts nc;
  filter_consts(H, W, pc, &fc, &pcc, &nc);
  (void)hipGetLastError();
  dispatch_fwd_rows(W, dtype, B, 1, pitch, H, 0, st);
  dispatch_pass_a(H, W, B, 1, fc, st);
  const float2* plane = yp + (size_t)(orient * pc->n_scales + scale) * H * W;
  dispatch_rows_inverse(W, H, plane, (float2*)eo, st);
  return launch_status();
}

rift2_status rift2_debug_noise(const void* workspace, size_t workspace_bytes, int32_t H, int32_t W,
                               const rift2_pc_params* pc, float* a0, float* order_stats, double* t_o, void* stream) {
  if (!workspace || !pc || !pc_ok(pc)) return RIFT2_ERR_INVALID_ARG;
  if (!size_ok(H) || !size_ok(W)) return RIFT2_ERR_UNSUPPORTED;
  const FilterLayout L = filter_layout(H, W, pc);
  if (workspace_bytes < L.total) return RIFT2_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  const char* ws = (const char*)workspace;
  const size_t no = (size_t)pc->n_orient;
  bool ok = true;
  if (a0) ok = ok && hipMemcpyAsync(a0, ws + L.a0, no * H * W * sizeof(float), hipMemcpyDeviceToDevice, st) == hipSuccess;
  if (order_stats)
    ok = ok && hipMemcpyAsync(order_stats, ws + L.ostat, 2 * no * sizeof(float), hipMemcpyDeviceToDevice, st) == hipSuccess;
  if (t_o) ok = ok && hipMemcpyAsync(t_o, ws + L.t64, no * sizeof(double), hipMemcpyDeviceToDevice, st) == hipSuccess;
  return ok ? RIFT2_OK : RIFT2_ERR_DEVICE;
}

rift2_status rift2_desc_normalize(const uint16_t* desc, const float* inv_norm, const int32_t* n_rows_dev, int32_t cap,
                                  int32_t D, float* out, void* stream) {
  if (!desc || !inv_norm || !n_rows_dev || !out || cap <= 0 || D <= 0) return RIFT2_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  const int64_t total = (int64_t)cap * D;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_desc_normalize, dim3(blocks), dim3(256), 0, st, desc, inv_norm, n_rows_dev, cap, D, out);
  return launch_status();
}

rift2_status rift2_debug_mfma_rate(int32_t precision, int32_t waves_per_simd, int32_t iters, int32_t reps, float* sink,
                                   float* ms, void* stream) {
  if (precision != RIFT2_PREC_FP32 && precision != RIFT2_PREC_BF16) return RIFT2_ERR_INVALID_ARG;
  if (waves_per_simd < 1 || waves_per_simd > 4 || iters < 1 || reps < 1 || !sink || !ms) return RIFT2_ERR_INVALID_ARG;
  int dev = -1, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess)
    return RIFT2_ERR_DEVICE;
  if (cus != kCalibCUs) return RIFT2_ERR_UNSUPPORTED;  // the sink's size assumes the full chip
  hipStream_t st = (hipStream_t)stream;
  // waves_per_simd blocks of 4 waves per CU: every SIMD runs waves_per_simd waves
  const dim3 grid(kCalibCUs * waves_per_simd);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess) return RIFT2_ERR_DEVICE;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return RIFT2_ERR_DEVICE;
  }
  (void)hipGetLastError();
  auto launch = [&]() {
    if (precision == RIFT2_PREC_FP32)
      hipLaunchKernelGGL(k_calib_mfma_f32, grid, dim3(256), 0, st, sink, iters, 1.0f);
    else
      hipLaunchKernelGGL(k_calib_mfma_bf16, grid, dim3(256), 0, st, sink, iters, 1.0f);
  };
  launch();  // warm-up
  rift2_status r = hipEventRecord(a, st) == hipSuccess ? RIFT2_OK : RIFT2_ERR_DEVICE;
  for (int i = 0; i < reps && r == RIFT2_OK; ++i) launch();
  if (r == RIFT2_OK) r = launch_status();
  if (r == RIFT2_OK && (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                        hipEventElapsedTime(ms, a, b) != hipSuccess))
    r = RIFT2_ERR_DEVICE;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return r;
}

static rift2_status detect_launch(const float* edge, const float* corner, int32_t H, int32_t W,
                                  const rift2_detect_params* det, rift2_keypoint* kpts, int32_t* n_kpts_dev,
                                  void* workspace, size_t workspace_bytes, void* stream, bool timed = true) {
  if (!edge || !det || !kpts || !n_kpts_dev || !workspace) return RIFT2_ERR_INVALID_ARG;
  if (((uintptr_t)edge & 15u) || ((uintptr_t)corner & 15u)) return RIFT2_ERR_INVALID_ARG;  // 16-byte loads
  if (H < 8 || W < 8 || (int64_t)H * W >= (1ll << 31)) return RIFT2_ERR_INVALID_ARG;
  if (!(det->fast_threshold >= 0.0f) || det->max_keypoints <= 0 || det->patch_size < 0 || (det->patch_size & 1))
    return RIFT2_ERR_INVALID_ARG;
  const int maps = corner ? 2 : 1;
  const DetectLayout L = detect_layout(H, W, det, maps);
  if (workspace_bytes < L.total) return RIFT2_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  uint32_t* hdr = (uint32_t*)(ws + L.hdr);
  uint32_t* mm = (uint32_t*)(ws + L.mm);
  uint32_t* hist = (uint32_t*)(ws + L.hist);
  uint32_t* tile_cnt = (uint32_t*)(ws + L.tile_cnt);
  uint64_t* cand = (uint64_t*)(ws + L.cand);
  uint32_t* sel_cnt = (uint32_t*)(ws + L.sel_cnt);
  uint64_t* sel = (uint64_t*)(ws + L.sel);
  uint64_t* fin = (uint64_t*)(ws + L.fin);
  uint32_t* part = (uint32_t*)(ws + L.part);
  (void)hipGetLastError();
  ProfScope ps(5, st, timed);
  const int n = H * W;
  const dim3 tiles((W + kTileX - 1) / kTileX, (H + kTileY - 1) / kTileY);
  hipLaunchKernelGGL(k_det_minmax, dim3(kMinMaxBlocks), dim3(256), 0, st, edge, n, mm, hist);
  if (corner) {
    uint32_t* mm2 = mm + 2 * kMinMaxBlocks;
    hipLaunchKernelGGL(k_det_minmax, dim3(kMinMaxBlocks), dim3(256), 0, st, corner, n, mm2, hist);
    hipLaunchKernelGGL(k_det_fast_union, tiles, dim3(kTileX * kTileY), 0, st, edge, corner, H, W, det->fast_threshold,
                       det->patch_size / 2, (const uint32_t*)mm, (const uint32_t*)mm2, hist, tile_cnt, cand);
  } else {
    hipLaunchKernelGGL(k_det_fast, tiles, dim3(kTileX * kTileY), 0, st, edge, H, W, det->fast_threshold,
                       det->patch_size / 2, mm, hist, tile_cnt, cand);
  }
  const uint32_t kmax = (uint32_t)det->max_keypoints;
  hipLaunchKernelGGL(k_det_bin, dim3(1), dim3(1024), 0, st, hdr, hist, kmax);
  hipLaunchKernelGGL(k_det_select1, dim3(kSelBlocks), dim3(256), 0, st, hdr, tile_cnt, L.n_tiles, cand, sel, sel_cnt);
  hipLaunchKernelGGL(k_det_select2, dim3(1), dim3(1024), 0, st, hdr, sel, sel_cnt, L.region, fin, kmax);
  const int blocks = (int)((kmax + 255) / 256);
  if (L.count_sort) {
    uint64_t* grouped = (uint64_t*)(ws + L.part);
    uint32_t* above = (uint32_t*)(ws + L.above);
    uint32_t* cursor = (uint32_t*)(ws + L.cursor);
    hipLaunchKernelGGL(k_det_offsets, dim3(1), dim3(1024), 0, st, (const uint32_t*)hist, above, cursor);
    hipLaunchKernelGGL(k_det_group, dim3(blocks), dim3(256), 0, st, (const uint32_t*)hdr, (const uint64_t*)fin, cursor,
                       grouped);
    hipLaunchKernelGGL(k_det_rank_bins, dim3(blocks), dim3(256), 0, st, (const uint32_t*)hdr,
                       (const uint64_t*)grouped, (const uint32_t*)above, (const uint32_t*)hist, W, (KeypointOut*)kpts,
                       n_kpts_dev);
  } else {
    hipLaunchKernelGGL(k_det_rank, dim3(blocks, L.n_part), dim3(256), 0, st, hdr, fin, part, kmax);
    hipLaunchKernelGGL(k_det_emit, dim3(blocks), dim3(256), 0, st, hdr, fin, part, L.n_part, kmax, W,
                       (KeypointOut*)kpts, n_kpts_dev);
  }
  return launch_status();
}

rift2_status rift2_detect(const float* moment, int32_t H, int32_t W, const rift2_detect_params* det,
                          rift2_keypoint* kpts, int32_t* n_kpts_dev, void* workspace, size_t workspace_bytes,
                          void* stream) {
  return detect_launch(moment, nullptr, H, W, det, kpts, n_kpts_dev, workspace, workspace_bytes, stream);
}

rift2_status rift2_detect_noalloc(const float* moment, int32_t H, int32_t W, const rift2_detect_params* det,
                                  rift2_keypoint* kpts, int32_t* n_kpts_dev, void* stream) {
  if (!moment || !det || !kpts || !n_kpts_dev) return RIFT2_ERR_INVALID_ARG;
  if (H < 8 || W < 8 || (int64_t)H * W >= (1ll << 31) || det->max_keypoints <= 0) return RIFT2_ERR_INVALID_ARG;
  if (rift2_detect_workspace_size(H, W, det) > kNoAllocScratchBytes) return RIFT2_ERR_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return RIFT2_ERR_NOT_INITIALIZED;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_init_mu);
    if (g_init_done[dev]) ws = g_scratch_dev[dev];
  }
  if (!ws) return RIFT2_ERR_NOT_INITIALIZED;
  // no stage timing: its events are allocated by the runtime
  return detect_launch(moment, nullptr, H, W, det, kpts, n_kpts_dev, ws, kNoAllocScratchBytes, stream, false);
}

rift2_status rift2_detect_union(const float* max_moment, const float* min_moment, int32_t H, int32_t W,
                                const rift2_detect_params* det, rift2_keypoint* kpts, int32_t* n_kpts_dev,
                                void* workspace, size_t workspace_bytes, void* stream) {
  if (!min_moment) return RIFT2_ERR_INVALID_ARG;
  return detect_launch(max_moment, min_moment, H, W, det, kpts, n_kpts_dev, workspace, workspace_bytes, stream);
}

rift2_status rift2_describe(const uint8_t* mim, int32_t H, int32_t W, const rift2_keypoint* kpts,
                            const int32_t* n_kpts_dev, int32_t kpt_cap, const rift2_desc_params* dp, uint16_t* desc,
                            float* inv_norm, int32_t* desc_kp, int32_t desc_cap, int32_t* n_desc_dev, void* workspace,
                            size_t workspace_bytes, void* stream) {
  if (!mim || !kpts || !n_kpts_dev || !dp || !desc || !inv_norm || !desc_kp || !n_desc_dev || !workspace)
    return RIFT2_ERR_INVALID_ARG;
  if (H <= 0 || W <= 0 || kpt_cap <= 0) return RIFT2_ERR_INVALID_ARG;
  if (dp->mode != RIFT2_DESC_DOMINANT && dp->mode != RIFT2_DESC_PLAIN && dp->mode != RIFT2_DESC_RING &&
      dp->mode != RIFT2_DESC_TURNED)
    return RIFT2_ERR_INVALID_ARG;
  const int rows_per_kp = dp->mode == RIFT2_DESC_RING ? dp->n_orient : (dp->mode == RIFT2_DESC_PLAIN ? 1 : 2);
  if ((int64_t)desc_cap < (int64_t)rows_per_kp * kpt_cap) return RIFT2_ERR_INVALID_ARG;
  if (dp->dominant_num < 0 || dp->dominant_den <= 0) return RIFT2_ERR_INVALID_ARG;
  if (workspace_bytes < rift2_describe_workspace_size(kpt_cap)) return RIFT2_ERR_WORKSPACE;
  const DescLayout DL = desc_layout(kpt_cap);
  hipStream_t st = (hipStream_t)stream;
  char* wsb = (char*)workspace;
  uint32_t* info = (uint32_t*)(wsb + DL.info);
  uint16_t* stage = (uint16_t*)(wsb + DL.stage);
  float* stage_inv = (float*)(wsb + DL.stage_inv);
  const int* kp = (const int*)kpts;
  (void)hipGetLastError();
  const int blocks2 = (kpt_cap + kDesc2Kpts - 1) / kDesc2Kpts;
  const bool turned = dp->mode == RIFT2_DESC_TURNED;
  const bool second = dp->mode == RIFT2_DESC_DOMINANT || turned;  // forms with second rows
  TurnTable tt{};
  for (int k = 0; k < dp->n_orient && k < 8; ++k) {
    tt.c[k] = (int)std::lround(std::cos(k * M_PI / dp->n_orient) * 65536.0);
    tt.s[k] = (int)std::lround(std::sin(k * M_PI / dp->n_orient) * 65536.0);
  }
  const uint16_t* src_rows = turned ? stage : desc;
  const float* src_inv = turned ? stage_inv : inv_norm;
  // k_describe2's word-wide form (taken only where N_o is even)
  const bool wide2 = ((uintptr_t)info & 15u) == 0 && ((uintptr_t)desc & 3u) == 0 && ((uintptr_t)src_rows & 3u) == 0;
  ProfScope ps(6, st);
#define RIFT2_DESCRIBE_CASE(P_, G_, NO_)                                                                              \
  if (dp->patch_size == P_ && dp->grid == G_ && dp->n_orient == NO_) {                                               \
    constexpr int KPB = desc_kpb<P_>();                                                                               \
    const dim3 grid((kpt_cap + KPB - 1) / KPB);                                                                       \
    if (turned)                                                                                                        \
      hipLaunchKernelGGL((k_describe_turn<P_, G_, NO_>), grid, dim3(P_ * KPB), 0, st, mim, H, W, kp, n_kpts_dev,       \
                         kpt_cap, dp->dominant_num, dp->dominant_den, tt, desc, inv_norm, desc_kp, info, stage,      \
                         stage_inv);                                                                                   \
    else                                                                                                               \
      hipLaunchKernelGGL((k_describe<P_, G_, NO_>), grid, dim3(P_ * KPB), 0, st, mim, H, W, kp, n_kpts_dev, kpt_cap,   \
                         dp->dominant_num, dp->dominant_den, dp->mode, desc, inv_norm, desc_kp, info, n_desc_dev);   \
    if (second && wide2)                                                                                               \
      hipLaunchKernelGGL((k_describe2<G_, NO_, NO_ % 2 == 0>), dim3(blocks2), dim3(256), 0, st, n_kpts_dev, kpt_cap,    \
                         info, src_rows, src_inv, desc, inv_norm, desc_kp, n_desc_dev);                               \
    else if (second)                                                                                                   \
      hipLaunchKernelGGL((k_describe2<G_, NO_, false>), dim3(blocks2), dim3(256), 0, st, n_kpts_dev, kpt_cap, info,     \
                         src_rows, src_inv, desc, inv_norm, desc_kp, n_desc_dev);                                     \
    return launch_status();                                                                                           \
  }
  RIFT2_DESCRIBE_CASE(96, 6, 6)
  RIFT2_DESCRIBE_CASE(96, 6, 8)
  RIFT2_DESCRIBE_CASE(64, 4, 6)
#undef RIFT2_DESCRIBE_CASE
  return RIFT2_ERR_UNSUPPORTED;
}

rift2_status rift2_match(const uint16_t* desc_a, const float* inv_a, const int32_t* kp_a, const int32_t* nA_dev,
                         int32_t cap_a, const uint16_t* desc_b, const float* inv_b, const int32_t* kp_b,
                         const int32_t* nB_dev, int32_t cap_b, int32_t D, const rift2_match_params* mp,
                         rift2_correspondence* out, int32_t* n_out_dev, void* workspace, size_t workspace_bytes, void* stream) {
  if (!desc_a || !inv_a || !kp_a || !nA_dev || !desc_b || !inv_b || !kp_b || !nB_dev || !mp || !out || !n_out_dev ||
      !workspace)
    return RIFT2_ERR_INVALID_ARG;
  if (cap_a <= 0 || cap_b <= 0 || D <= 0) return RIFT2_ERR_INVALID_ARG;
  if (!(mp->ratio_sq > 0.0f) ||
      (mp->precision != RIFT2_PREC_FP32 && mp->precision != RIFT2_PREC_BF16 && mp->precision != RIFT2_PREC_FP8))
    return RIFT2_ERR_INVALID_ARG;
  if (mp->mutual != 0 && mp->mutual != 1) return RIFT2_ERR_INVALID_ARG;
  if (D != 216 && D != 288) return RIFT2_ERR_UNSUPPORTED;
  if (mp->ring < 0 || mp->ring == 1 || mp->ring > kMaxOrient) return RIFT2_ERR_INVALID_ARG;
  if (mp->ring && (mp->precision == RIFT2_PREC_FP8 || mp->mutual)) return RIFT2_ERR_UNSUPPORTED;
  // the table preparation reads descriptor rows as 16-byte vectors
  if (((uintptr_t)desc_a & 15u) || ((uintptr_t)desc_b & 15u)) return RIFT2_ERR_INVALID_ARG;
  const bool mutual = mp->mutual != 0;
  const MatchLayout L = match_layout(cap_a, cap_b, D, mp->precision, mutual);
  if (workspace_bytes < L.total) return RIFT2_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  void* ta = ws + L.ta;
  void* tb = ws + L.tb;
  int2* part = (int2*)(ws + L.part);
  int2* part_r = (int2*)(ws + L.part_r);
  int32_t* a1 = mutual ? (int32_t*)(ws + L.a1) : nullptr;
  uint64_t* best = (uint64_t*)(ws + L.best);
  int32_t* rowj = (int32_t*)(ws + L.rowj);
  float* rowd = (float*)(ws + L.rowd);
  const bool bf = mp->precision == RIFT2_PREC_BF16;
  (void)hipGetLastError();
  if (mp->precision == RIFT2_PREC_FP8) {
    float* wa = (float*)(ws + L.wa);
    float* wb = (float*)(ws + L.wb);
    {
      ProfScope ps7(7, st);
      hipLaunchKernelGGL(k_match_prep_fp8, dim3(1024), dim3(256), 0, st, desc_a, inv_a, nA_dev, cap_a, D, L.rs,
                         L.rows_a, (uint8_t*)ta, wa, best, cap_a);
      hipLaunchKernelGGL(k_match_prep_fp8, dim3(1024), dim3(256), 0, st, desc_b, inv_b, nB_dev, cap_b, D, L.rs,
                         L.rows_b, (uint8_t*)tb, wb, (uint64_t*)nullptr, 0);
    }
    {
      ProfScope ps8(8, st);
      launch_gemm_fp8(L.dp, (const uint8_t*)ta, wa, nA_dev, cap_a, (const uint8_t*)tb, wb, nB_dev, cap_b, L.rows_a,
                      L.slice_rows, L.slices, part, st);
      if (mutual)
        launch_gemm_fp8(L.dp, (const uint8_t*)tb, wb, nB_dev, cap_b, (const uint8_t*)ta, wa, nA_dev, cap_a, L.rows_b,
                        L.slice_rows_r, L.slices_r, part_r, st);
    }
    ProfScope ps9(9, st);
    if (mutual)
      hipLaunchKernelGGL(k_match_rnn8, dim3((cap_b + 3) / 4), dim3(256), 0, st, part_r, 2 * L.slices_r, nB_dev, cap_b,
                         desc_a, inv_a, desc_b, inv_b, D, a1);
    hipLaunchKernelGGL(k_match_merge8, dim3((cap_a + 3) / 4), dim3(256), 0, st, part, 2 * L.slices, nA_dev, desc_a, inv_a,
                       kp_a, desc_b, inv_b, kp_b, D, mp->ratio_sq, cap_a, (const int32_t*)a1, best, rowj, rowd);
    hipLaunchKernelGGL(k_match_emit, dim3((cap_a + 255) / 256), dim3(256), 0, st, best, cap_a, rowj, rowd, kp_b,
                       (MatchOut*)out, n_out_dev);
    return launch_status();
  }
  ProfScope ps7(7, st);
  {
    const PrepJob ja{desc_a, nA_dev, cap_a, L.rows_a, ta, best, cap_a};
    const PrepJob jb{desc_b, nB_dev, cap_b, L.rows_b, tb, nullptr, 0};
    if (bf)
      hipLaunchKernelGGL(k_match_prep<true>, dim3(512, 2), dim3(256), 0, st, ja, jb, D, L.rs);
    else
      hipLaunchKernelGGL(k_match_prep<false>, dim3(512, 2), dim3(256), 0, st, ja, jb, D, L.rs);
  }
  ps7.finish();
  ProfScope ps8(8, st);
  launch_gemm_exact<false>(bf, L.dp, ta, inv_a, nA_dev, cap_a, tb, inv_b, nB_dev, cap_b, L.rows_a, L.slice_rows,
                           L.slices, part, st);
  if (mutual)
    launch_gemm_exact<true>(bf, L.dp, tb, inv_b, nB_dev, cap_b, ta, inv_a, nA_dev, cap_a, L.rows_b, L.slice_rows_r,
                            L.slices_r, part_r, st);
  ps8.finish();
  ProfScope ps9(9, st);
  if (mutual)
    hipLaunchKernelGGL(k_match_rnn, dim3((cap_b + 3) / 4), dim3(256), 0, st, part_r, 2 * L.slices_r, nB_dev, cap_b, a1);
  if (mp->ring)
    hipLaunchKernelGGL(k_match_merge_ring, dim3((cap_a / mp->ring + 3) / 4), dim3(256), 0, st, part, 2 * L.slices,
                       (int)mp->ring, nA_dev, kp_a, kp_b, mp->ratio_sq, cap_a, best, rowj, rowd);
  else
    hipLaunchKernelGGL(k_match_merge, dim3((cap_a + 3) / 4), dim3(256), 0, st, part, 2 * L.slices, nA_dev, kp_a, kp_b,
                       mp->ratio_sq, cap_a, (const int32_t*)a1, best, rowj, rowd);
  // ring rows come R per keypoint, so keypoint indices stay below cap_a / R
  const int kp_range = mp->ring ? cap_a / mp->ring : cap_a;
  hipLaunchKernelGGL(k_match_emit, dim3((kp_range + 255) / 256), dim3(256), 0, st, best, kp_range, rowj, rowd, kp_b,
                     (MatchOut*)out, n_out_dev);
  return launch_status();
}

size_t rift2_ransac_workspace_size(int32_t match_cap, int32_t n_hyp) {
  RansacLayout L;
  return ransac_layout(match_cap, n_hyp, &L) ? L.total : 0;
}

rift2_status rift2_ransac(const rift2_correspondence* matches, const int32_t* n_matches_dev, int32_t match_cap,
                          const rift2_keypoint* kpts_a, int32_t kpt_cap_a, const rift2_keypoint* kpts_b,
                          int32_t kpt_cap_b, const uint32_t* words, int32_t n_hyp, const rift2_ransac_params* rp,
                          int32_t* counts, uint8_t* inlier_mask, rift2_similarity* result, void* workspace,
                          size_t workspace_bytes, void* stream) {
  if (!matches || !n_matches_dev || !kpts_a || !kpts_b || !words || !rp || !inlier_mask || !result || !workspace)
    return RIFT2_ERR_INVALID_ARG;
  if (kpt_cap_a < 1 || kpt_cap_b < 1 || n_hyp < 1 || rp->refine < 0 || rp->refine > kRansacMaxRefine ||
      !std::isfinite(rp->threshold) || !(rp->threshold > 0.0))
    return RIFT2_ERR_INVALID_ARG;
  if ((uintptr_t)words & 7u || (uintptr_t)result & 7u || (uintptr_t)workspace & 15u) return RIFT2_ERR_INVALID_ARG;
  RansacLayout L;
  if (!ransac_layout(match_cap, n_hyp, &L)) return RIFT2_ERR_UNSUPPORTED;
  if (workspace_bytes < L.total) return RIFT2_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  int4* xy = (int4*)(ws + L.xy);
  int32_t* flags = (int32_t*)(ws + L.flags);
  int32_t* cnt = counts ? counts : (int32_t*)(ws + L.counts);
  unsigned long long* key = (unsigned long long*)(ws + L.key);
  unsigned long long* sums = (unsigned long long*)(ws + L.sums);
  const double tau2 = rp->threshold * rp->threshold;
  const int refine = (int)rp->refine;
  (void)hipGetLastError();
  ProfScope ps(11, st);
  // the gather's first block clears the refit sums: it has at least 8 * refine <= 128 threads
  hipLaunchKernelGGL(k_ransac_gather, dim3(L.n_flags), dim3(256), 0, st, (const RansacMatch*)matches, n_matches_dev,
                     match_cap, (const RansacKp*)kpts_a, kpt_cap_a, (const RansacKp*)kpts_b, kpt_cap_b, xy, flags,
                     key, sums, 8 * refine);
  hipLaunchKernelGGL(k_ransac_score, dim3((n_hyp + kRansacHypPerBlock - 1) / kRansacHypPerBlock), dim3(256), 0, st,
                     (const int4*)xy, n_matches_dev, match_cap, (const int32_t*)flags, L.n_flags,
                     (const uint2*)words, n_hyp, tau2, cnt, key);
  const int refit_blocks = (match_cap + 256 * kRefitPerThread - 1) / (256 * kRefitPerThread);
  for (int it = 0; it < refine; ++it)
    hipLaunchKernelGGL(k_ransac_refit_sums, dim3(refit_blocks), dim3(256), 0, st, (const int4*)xy, n_matches_dev,
                       match_cap, (const uint2*)words, (const unsigned long long*)key, tau2, (const int32_t*)flags,
                       L.n_flags, sums, it);
  hipLaunchKernelGGL(k_ransac_refine, dim3(1), dim3(1024), 0, st, (const int4*)xy, n_matches_dev, match_cap,
                     (const uint2*)words, (const unsigned long long*)key, tau2, refine,
                     (const unsigned long long*)sums, (const int32_t*)flags, L.n_flags, inlier_mask,
                     (RansacResult*)result);
  return launch_status();
}

rift2_status rift2_consensus(const double* model, const rift2_correspondence* matches, const int32_t* n_matches_dev,
                             int32_t match_cap, const rift2_keypoint* kpts_a, int32_t kpt_cap_a,
                             const rift2_keypoint* kpts_b, int32_t kpt_cap_b, double threshold, uint8_t* mask,
                             rift2_consensus_result* result, void* workspace, size_t workspace_bytes, void* stream) {
  if (!model || !matches || !n_matches_dev || !kpts_a || !kpts_b || !result || !workspace)
    return RIFT2_ERR_INVALID_ARG;
  if (kpt_cap_a < 1 || kpt_cap_b < 1 || !std::isfinite(threshold) || !(threshold > 0.0)) return RIFT2_ERR_INVALID_ARG;
  if ((uintptr_t)model & 7u || (uintptr_t)result & 7u || (uintptr_t)workspace & 15u) return RIFT2_ERR_INVALID_ARG;
  RansacLayout L;
  if (!ransac_layout(match_cap, 0, &L)) return RIFT2_ERR_UNSUPPORTED;
  if (workspace_bytes < L.total) return RIFT2_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  int4* xy = (int4*)(ws + L.xy);
  int32_t* flags = (int32_t*)(ws + L.flags);
  (void)hipGetLastError();
  ProfScope ps(11, st);
  hipLaunchKernelGGL(k_ransac_gather, dim3(L.n_flags), dim3(256), 0, st, (const RansacMatch*)matches, n_matches_dev,
                     match_cap, (const RansacKp*)kpts_a, kpt_cap_a, (const RansacKp*)kpts_b, kpt_cap_b, xy, flags,
                     (unsigned long long*)nullptr, (unsigned long long*)nullptr, 0);
  hipLaunchKernelGGL(k_consensus, dim3(1), dim3(1024), 0, st, (const int4*)xy, n_matches_dev, match_cap,
                     (const int32_t*)flags, L.n_flags, model, threshold * threshold, mask, (ConsensusOut*)result);
  return launch_status();
}

size_t rift2_engine_request_bytes(int32_t H, int32_t W, int32_t max_keypoints, const rift2_pc_params* pc,
                                  const rift2_detect_params* det, const rift2_desc_params* dp,
                                  const rift2_match_params* mp) {
  if (!pc || !det || !dp || !mp) return 0;
  rift2_request r{};
  r.H = H;
  r.W = W;
  r.max_keypoints = max_keypoints;
  ReqLayout L;
  if (!req_layout(H, W, engine_keypoints(r), pc, det, dp, mp, &L)) return 0;
  return L.total;
}

rift2_status rift2_engine_create(int device, void* arena, size_t arena_bytes, int32_t max_inflight,
                                 const rift2_pc_params* pc, const rift2_detect_params* det,
                                 const rift2_desc_params* dp, const rift2_match_params* mp, rift2_engine** out) {
  if (!out || !arena || !arena_bytes || !pc || !det || !dp || !mp || max_inflight <= 0 || max_inflight > 64)
    return RIFT2_ERR_INVALID_ARG;
  if (dp->mode != RIFT2_DESC_DOMINANT || mp->ring != 0) return RIFT2_ERR_UNSUPPORTED;  // the engine serves RIFT2
  if ((uintptr_t)arena & 255u) return RIFT2_ERR_INVALID_ARG;
  *out = nullptr;
  const rift2_status st = rift2_init(device);
  if (st != RIFT2_OK) return st;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return RIFT2_ERR_DEVICE;
  rift2_engine* e = new rift2_engine();
  e->device = device;
  e->arena = (char*)arena;
  e->arena_bytes = arena_bytes;
  e->pc = *pc;
  e->det = *det;
  e->dp = *dp;
  e->mp = *mp;
  e->alloc.reset(arena_bytes);
  bool ok = hipEventCreate(&e->epoch) == hipSuccess;
  e->slots.resize(max_inflight);
  for (int i = 0; ok && i < max_inflight; ++i) {
    EngineSlot& s = e->slots[i];
    ok = hipStreamCreateWithFlags(&s.sa, hipStreamNonBlocking) == hipSuccess &&
         hipStreamCreateWithFlags(&s.sb, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreate(&s.b_done) == hipSuccess && hipEventCreate(&s.admit) == hipSuccess &&
         hipEventCreate(&s.done) == hipSuccess && hipEventCreate(&s.filt) == hipSuccess;
    e->free_slots.push_back(max_inflight - 1 - i);
  }
  if (ok) ok = hipEventRecord(e->epoch, e->slots[0].sa) == hipSuccess && hipEventSynchronize(e->epoch) == hipSuccess;
  (void)hipSetDevice(prev);
  if (!ok) {
    rift2_engine_destroy(e);
    return RIFT2_ERR_DEVICE;
  }
  *out = e;
  return RIFT2_OK;
}

rift2_status rift2_engine_submit(rift2_engine* e, const rift2_request* r) {
  if (!e || !r || !r->img_a || !r->img_b || !r->out || !r->n_out) return RIFT2_ERR_INVALID_ARG;
  if (r->dtype != RIFT2_U8 && r->dtype != RIFT2_U16 && r->dtype != RIFT2_F32) return RIFT2_ERR_INVALID_ARG;
  if (!size_ok(r->H) || !size_ok(r->W)) return RIFT2_ERR_UNSUPPORTED;
  EngineReq q;
  q.req = *r;
  q.H = r->H;
  q.W = r->W;
  q.K = engine_keypoints(*r);
  if (q.K <= 0) return RIFT2_ERR_INVALID_ARG;
  e->pending.push_back(q);
  return RIFT2_OK;
}

int32_t rift2_engine_poll(rift2_engine* e, rift2_completion* done, int32_t max_done) {
  if (!e || (!done && max_done > 0) || max_done < 0) return -RIFT2_ERR_INVALID_ARG;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(e->device) != hipSuccess) return -RIFT2_ERR_DEVICE;
  int32_t n = 0;
  while (n < max_done && !e->finished.empty()) {
    done[n++] = e->finished.front();
    e->finished.pop_front();
  }
  // reap finished requests (any order), then admit from the queue
  for (auto it = e->inflight.begin(); it != e->inflight.end() && n < max_done;) {
    const EngineSlot& s = e->slots[it->slot];
    const hipError_t q = hipEventQuery(s.done);
    if (q == hipErrorNotReady) {
      ++it;
      continue;
    }
    rift2_completion c{};
    c.id = it->req.id;
    c.status = q == hipSuccess ? it->status : RIFT2_ERR_DEVICE;
    c.batch = it->batch;
    float t_admit = 0.0f, t_done = 0.0f;
    if (q == hipSuccess && hipEventElapsedTime(&t_admit, e->epoch, s.admit) == hipSuccess &&
        hipEventElapsedTime(&t_done, e->epoch, s.done) == hipSuccess) {
      c.admit_ms = t_admit;
      c.done_ms = t_done;
      c.gpu_ms = t_done - t_admit;
    }
    done[n++] = c;
    e->alloc.release(it->off, it->bytes);
    e->free_slots.push_back(it->slot);
    it = e->inflight.erase(it);
  }
  engine_pump(e);
  (void)hipSetDevice(prev);
  return n;
}

rift2_status rift2_engine_set_batch(rift2_engine* e, int32_t max_requests) {
  if (!e || max_requests < 1 || max_requests > RIFT2_MAX_FILTER_BATCH / 2) return RIFT2_ERR_INVALID_ARG;
  e->batch = max_requests;
  return RIFT2_OK;
}

int32_t rift2_engine_pending(const rift2_engine* e) {
  if (!e) return 0;
  return (int32_t)(e->pending.size() + e->inflight.size() + e->finished.size());
}

rift2_status rift2_engine_destroy(rift2_engine* e) {
  if (!e) return RIFT2_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(e->device);
  for (EngineSlot& s : e->slots) {
    if (s.sa) (void)hipStreamSynchronize(s.sa);
    if (s.sb) (void)hipStreamSynchronize(s.sb);
    if (s.sa) (void)hipStreamDestroy(s.sa);
    if (s.sb) (void)hipStreamDestroy(s.sb);
    if (s.b_done) (void)hipEventDestroy(s.b_done);
    if (s.admit) (void)hipEventDestroy(s.admit);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.filt) (void)hipEventDestroy(s.filt);
  }
  if (e->epoch) (void)hipEventDestroy(e->epoch);
  (void)hipSetDevice(prev);
  delete e;
  return RIFT2_OK;
}

rift2_status rift2_profile_enable(int on) {
  std::lock_guard<std::mutex> lock(g_prof_mu);
  g_prof_on = on != 0;
  return RIFT2_OK;
}

int rift2_profile_read(double* ms, int64_t* count, int n_groups) {
  std::vector<ProfRec> recs;
  {
    std::lock_guard<std::mutex> lock(g_prof_mu);
    recs.swap(g_prof);
  }
  for (const ProfRec& r : recs) {
    float t = 0.0f;
    const bool ok = hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess;
    if (ok && r.group < n_groups) {
      if (ms) ms[r.group] += (double)t;
      if (count) count[r.group] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  return kProfGroups;
}

}  // extern "C"
