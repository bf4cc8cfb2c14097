// Outlier removal of the putative matches (Section 1 and Fig. 1: the matches
// are filtered by RANSAC, Fischler and Bolles 1981) and the consensus of a
// given transform, which also yields the correct-match count and RMSE of
// Section 4 when the transform is the ground truth.
//
// Model: the similarity u = a x - b y + tx, v = b x + a y + ty, i.e.
// w = (a + ib) z + t for z = x + iy, w = u + iv.
//
//   k_ransac_gather  match list + keypoint tables -> int4 (xa, ya, xb, yb),
//                    range check of every coordinate
//   k_ransac_score   one block per group of hypotheses: the exact fit to the
//                    hypothesis' two sampled matches, then its consensus
//                    count over all matches (ballot + popcount per 64)
//   k_ransac_refit_sums  one launch per least-squares refit: every block
//                    takes the model so far (the hypothesis with the largest
//                    count, lowest index on ties, then the earlier refits) and
//                    adds its matches' exact integer normal-equation sums
//                    into the refit's sums (atomic int64 adds: exact, so the
//                    order does not matter)
//   k_ransac_refine  one block: the final model from the hypothesis and the
//                    refits' sums, the inlier mask and count
//   k_consensus      one block: residuals of a given model, mask, count and
//                    the sum of the inliers' squared residuals
//
// Every floating-point step is one IEEE double operation in the order
// written (contraction into FMA is switched off in each function), so the
// consensus decisions are reproducible by any implementation that follows
// the same formulas.  Coordinates are integers below 2^13 and there are at
// most 2^17 matches, so every least-squares sum is an exact int64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rift2 {

constexpr int kRansacMaxMatches = 1 << 17;
constexpr int kRansacCoordLimit = 1 << 13;
constexpr int kRansacMaxHyp = 1 << 20;
constexpr int kRansacHypPerBlock = 4;
constexpr int kRansacMaxRefine = 16;
constexpr int kRefitPerThread = 4;  // matches per thread of a refit-sums block (loads issued together)

struct RansacKp {  // layout of rift2_keypoint
  int x, y;
  float score;
};

struct RansacMatch {  // layout of rift2_correspondence
  int kp_a, kp_b;
  float dist2;
};

struct RansacResult {  // layout of rift2_similarity
  double a, b, tx, ty;
  int32_t best;
  int32_t n_inliers;
  int32_t n_matches;
  int32_t status;
};

struct Sim {
  double a, b, tx, ty;
};

// Exact fit to the minimal sample p -> (p.z, p.w), q -> (q.z, q.w): with
// d = q - p in A and e likewise in B, (a + ib) = e / d = e conj(d) / |d|^2,
// t = w_p - (a + ib) z_p.  False when the two A points coincide.
__device__ __forceinline__ bool sim_fit_pair(int4 p, int4 q, Sim& m) {
#pragma clang fp contract(off)
  const long long dx = (long long)q.x - p.x, dy = (long long)q.y - p.y;
  const long long du = (long long)q.z - p.z, dv = (long long)q.w - p.w;
  const long long den = dx * dx + dy * dy;
  if (den == 0) return false;
  const double fden = (double)den;
  m.a = (double)(dx * du + dy * dv) / fden;
  m.b = (double)(dx * dv - dy * du) / fden;
  const double x1 = (double)p.x, y1 = (double)p.y;
  m.tx = (double)p.z - (m.a * x1 - m.b * y1);
  m.ty = (double)p.w - (m.b * x1 + m.a * y1);
  return true;
}

// Squared distance between the model's image of (x, y) and (u, v).
__device__ __forceinline__ double sim_residual_sq(const Sim& m, double x, double y, double u, double v) {
#pragma clang fp contract(off)
  const double ex = ((m.a * x - m.b * y) + m.tx) - u;
  const double ey = ((m.b * x + m.a * y) + m.ty) - v;
  return ex * ex + ey * ey;
}

// Sums of the least-squares normal equations over a set of correspondences.
struct LsqSums {
  long long n, sx, sy, su, sv, sxx_yy, sxu_yv, sxv_yu;
};

__device__ __forceinline__ void lsq_add(LsqSums& s, int4 p) {
  const long long x = p.x, y = p.y, u = p.z, v = p.w;
  s.n += 1;
  s.sx += x;
  s.sy += y;
  s.su += u;
  s.sv += v;
  s.sxx_yy += x * x + y * y;
  s.sxu_yv += x * u + y * v;
  s.sxv_yu += x * v - y * u;
}

// Least squares: minimising sum |(a + ib) z + t - w|^2 gives
// (a + ib) = sum conj(z - zbar)(w - wbar) / sum |z - zbar|^2 and
// t = wbar - (a + ib) zbar, here from the n-scaled integer sums.
__device__ __forceinline__ bool sim_fit_lsq(const LsqSums& s, Sim& m) {
#pragma clang fp contract(off)
  if (s.n < 2) return false;
  const long long den = s.n * s.sxx_yy - (s.sx * s.sx + s.sy * s.sy);
  if (den == 0) return false;
  const long long num_a = s.n * s.sxu_yv - (s.sx * s.su + s.sy * s.sv);
  const long long num_b = s.n * s.sxv_yu - (s.sx * s.sv - s.sy * s.su);
  const double fden = (double)den;
  m.a = (double)num_a / fden;
  m.b = (double)num_b / fden;
  const double fx = (double)s.sx, fy = (double)s.sy, fn = (double)s.n;
  m.tx = ((double)s.su - (m.a * fx - m.b * fy)) / fn;
  m.ty = ((double)s.sv - (m.b * fx + m.a * fy)) / fn;
  return true;
}

// Sample index of a uniform 32-bit word: floor(u * n / 2^32).
__device__ __forceinline__ int sample_index(uint32_t u, int n) {
  return (int)(((uint64_t)u * (uint64_t)(uint32_t)n) >> 32);
}

// grid = ceil(cap / 256).  Block z writes flags[z] = 1 when one of its
// matches refers to a keypoint index outside [0, cap_k) or to a coordinate
// outside [0, kRansacCoordLimit), else 0 (every block writes its flag, so
// nothing needs clearing between calls).  Also clears *best_key and the
// n_refit_sums refit sums (if given).
__global__ void __launch_bounds__(256) k_ransac_gather(const RansacMatch* __restrict__ m, const int32_t* __restrict__ n_dev,
                                                       int cap, const RansacKp* __restrict__ ka, int cap_ka,
                                                       const RansacKp* __restrict__ kb, int cap_kb,
                                                       int4* __restrict__ xy, int32_t* __restrict__ flags,
                                                       unsigned long long* __restrict__ best_key,
                                                       unsigned long long* __restrict__ refit_sums, int n_refit_sums) {
  const int n = min(*n_dev, cap);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i == 0 && best_key) *best_key = 0ull;  // the scoring kernel that follows takes maxima into it
  if (refit_sums && i < n_refit_sums) refit_sums[i] = 0ull;  // the refit kernels add into them
  bool bad = false;
  if (i < n) {
    const RansacMatch c = m[i];
    int4 p = make_int4(0, 0, 0, 0);
    bool ok = c.kp_a >= 0 && c.kp_a < cap_ka && c.kp_b >= 0 && c.kp_b < cap_kb;
    if (ok) {
      const RansacKp a = ka[c.kp_a], b = kb[c.kp_b];
      p = make_int4(a.x, a.y, b.x, b.y);
      ok = (unsigned)p.x < (unsigned)kRansacCoordLimit && (unsigned)p.y < (unsigned)kRansacCoordLimit &&
           (unsigned)p.z < (unsigned)kRansacCoordLimit && (unsigned)p.w < (unsigned)kRansacCoordLimit;
    }
    if (!ok) p = make_int4(0, 0, 0, 0);
    bad = !ok;
    xy[i] = p;
  }
  const int any = __syncthreads_or(bad ? 1 : 0);
  if (threadIdx.x == 0) flags[blockIdx.x] = any ? 1 : 0;
}

// True in every lane of the calling wave when one of flags[0..nf) is set.
__device__ __forceinline__ bool wave_any_flag(const int32_t* __restrict__ flags, int nf) {
  bool any = false;
  for (int base = 0; base < nf; base += 64) {
    const int i = base + (threadIdx.x & 63);
    any = any || __ballot(i < nf && flags[i] != 0) != 0ull;
  }
  return any;
}

// grid = ceil(n_hyp / kRansacHypPerBlock), block 256: block z scores
// hypotheses [z G, z G + G); its four waves take interleaved 64-match chunks
// and their counts are added through LDS.  counts[h] = consensus size, or -1
// when the sample is degenerate, there are fewer than two matches or a
// gather flag (n_flags of them) is set; every counted hypothesis also takes
// the maximum of (count << 32 | ~h) into *best_key (cleared by the gather).
__global__ void __launch_bounds__(256) k_ransac_score(const int4* __restrict__ xy, const int32_t* __restrict__ n_dev,
                                                      int cap, const int32_t* __restrict__ flags, int n_flags,
                                                      const uint2* __restrict__ words, int n_hyp, double tau2,
                                                      int32_t* __restrict__ counts,
                                                      unsigned long long* __restrict__ best_key) {
#pragma clang fp contract(off)
  constexpr int G = kRansacHypPerBlock;
  __shared__ int sh_cnt[4][G];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int h0 = blockIdx.x * G;
  // an invalid match list counts as empty: every hypothesis gets -1
  const int n = wave_any_flag(flags, n_flags) ? 0 : min(*n_dev, cap);
  // lane g fits hypothesis h0 + g; every lane then reads the G models
  Sim mine{0.0, 0.0, 0.0, 0.0};
  bool mine_ok = false;
  if (lane < G && h0 + lane < n_hyp && n >= 2) {
    const uint2 w = words[h0 + lane];
    mine_ok = sim_fit_pair(xy[sample_index(w.x, n)], xy[sample_index(w.y, n)], mine);
  }
  Sim m[G];
  bool ok[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    m[g].a = __shfl(mine.a, g, 64);
    m[g].b = __shfl(mine.b, g, 64);
    m[g].tx = __shfl(mine.tx, g, 64);
    m[g].ty = __shfl(mine.ty, g, 64);
    ok[g] = __shfl((int)mine_ok, g, 64) != 0;
  }
  int cnt[G];
#pragma unroll
  for (int g = 0; g < G; ++g) cnt[g] = 0;
  const int n_eff = n >= 2 ? n : 0;
  const int4 zero = make_int4(0, 0, 0, 0);
  int base = wave * 64;
  int4 p = base + lane < n_eff ? xy[base + lane] : zero;
  for (; base < n_eff; base += 256) {
    const int nxt = base + 256 + lane;
    const int4 pn = nxt < n_eff ? xy[nxt] : zero;  // next chunk in flight during this one
    const bool live = base + lane < n_eff;
    const double x = (double)p.x, y = (double)p.y, u = (double)p.z, v = (double)p.w;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const bool in = live && sim_residual_sq(m[g], x, y, u, v) < tau2;
      cnt[g] += __popcll(__ballot(in));
    }
    p = pn;
  }
  if (lane == 0) {
#pragma unroll
    for (int g = 0; g < G; ++g) sh_cnt[wave][g] = cnt[g];
  }
  __syncthreads();
  if (threadIdx.x < G) {
    const int g = threadIdx.x;
    const int h = h0 + g;
    if (h < n_hyp) {
      const int c = sh_cnt[0][g] + sh_cnt[1][g] + sh_cnt[2][g] + sh_cnt[3][g];
      counts[h] = ok[g] ? c : -1;
      // count << 32 | ~h: the maximum has the largest count, then the lowest index
      if (ok[g]) atomicMax(best_key, ((unsigned long long)(unsigned)c << 32) | (unsigned long long)(~(uint32_t)h));
    }
  }
}

__device__ __forceinline__ int block_sum_int(int v, int* sh /* 16 */) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = 0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q];
  return t;
}

// The model after the first `upto` least-squares refits: the exact fit to the
// best hypothesis' sample, then each refit's fit to its sums (8 int64 per
// refit), stopping at the first set without a unique fit.  *go: whether the
// model came through all `upto` refits (so a further refit would run).
// *best = the hypothesis index, -1 when there is none.
__device__ __forceinline__ Sim refit_chain(const int4* __restrict__ xy, int n, const uint2* __restrict__ words,
                                           unsigned long long key, const unsigned long long* __restrict__ sums,
                                           int upto, int* best, bool* go) {
  Sim m{0.0, 0.0, 0.0, 0.0};
  *best = -1;
  *go = false;
  if (key == 0 || n < 2) return m;
  const int h = (int)(~(uint32_t)(key & 0xffffffffull));
  const uint2 w = words[h];
  if (!sim_fit_pair(xy[sample_index(w.x, n)], xy[sample_index(w.y, n)], m)) return m;  // cannot happen: counted
  *best = h;
  *go = true;
  for (int j = 0; j < upto; ++j) {
    const unsigned long long* q = sums + 8 * j;
    const LsqSums t{(long long)q[0], (long long)q[1], (long long)q[2], (long long)q[3],
                    (long long)q[4], (long long)q[5], (long long)q[6], (long long)q[7]};
    Sim f;
    if (!sim_fit_lsq(t, f)) {
      *go = false;
      break;
    }
    m = f;
  }
  return m;
}

// Refit `it` (grid = ceil(cap / (256 kRefitPerThread)), block 256): the
// normal-equation sums of the matches within the threshold of the model after
// refits 0..it-1, added into sums[8 it .. 8 it + 8).  Nothing is added when
// the match list is invalid or the chain stopped earlier.
__global__ void __launch_bounds__(256) k_ransac_refit_sums(const int4* __restrict__ xy, const int32_t* __restrict__ n_dev,
                                                           int cap, const uint2* __restrict__ words,
                                                           const unsigned long long* __restrict__ best_key, double tau2,
                                                           const int32_t* __restrict__ flags, int n_flags,
                                                           unsigned long long* __restrict__ sums, int it) {
#pragma clang fp contract(off)
  __shared__ long long sh[4 * 8];
  __shared__ double sh_m[4];
  __shared__ int sh_go;
  const int tid = threadIdx.x;
  const int n = min(*n_dev, cap);
  const int beg = blockIdx.x * 256 * kRefitPerThread;
  if (beg >= n) return;  // uniform: no matches here
  if (tid < 64) {
    const bool invalid = wave_any_flag(flags, n_flags);
    if (tid == 0) {
      int best;
      bool go;
      const Sim m = refit_chain(xy, n, words, invalid ? 0ull : *best_key, sums, it, &best, &go);
      sh_m[0] = m.a;
      sh_m[1] = m.b;
      sh_m[2] = m.tx;
      sh_m[3] = m.ty;
      sh_go = go ? 1 : 0;
    }
  }
  __syncthreads();
  if (!sh_go) return;  // uniform
  const Sim m{sh_m[0], sh_m[1], sh_m[2], sh_m[3]};
  LsqSums s{0, 0, 0, 0, 0, 0, 0, 0};
  int4 p[kRefitPerThread];
  const int4 zero = make_int4(0, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < kRefitPerThread; ++r) {
    const int i = beg + r * 256 + tid;
    p[r] = i < n ? xy[i] : zero;
  }
#pragma unroll
  for (int r = 0; r < kRefitPerThread; ++r) {
    const int i = beg + r * 256 + tid;
    if (i < n && sim_residual_sq(m, (double)p[r].x, (double)p[r].y, (double)p[r].z, (double)p[r].w) < tau2)
      lsq_add(s, p[r]);
  }
  long long v[8] = {s.n, s.sx, s.sy, s.su, s.sv, s.sxx_yy, s.sxu_yv, s.sxv_yu};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  }
  if ((tid & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) sh[(tid >> 6) * 8 + k] = v[k];
  }
  __syncthreads();
  if (tid < 8) {
    const long long t = sh[tid] + sh[8 + tid] + sh[16 + tid] + sh[24 + tid];
    // two's-complement addition: the signed sums come out exact
    if (t != 0) atomicAdd(sums + 8 * it + tid, (unsigned long long)t);
  }
}

constexpr int kRefineBatch = 8;  // matches per thread whose loads are issued together

// One block of 1024 threads.  The model: the best hypothesis from *best_key
// (count << 32 | ~h, the maximum over all hypotheses, so the largest count
// and among equal counts the lowest index) refined by the `refine` refits
// whose sums k_ransac_refit_sums left (stopping at the first set without a
// unique fit); then the final mask over [0, cap) and the result.
__global__ void __launch_bounds__(1024) k_ransac_refine(const int4* __restrict__ xy, const int32_t* __restrict__ n_dev,
                                                        int cap, const uint2* __restrict__ words,
                                                        const unsigned long long* __restrict__ best_key, double tau2,
                                                        int refine, const unsigned long long* __restrict__ sums,
                                                        const int32_t* __restrict__ flags, int n_flags,
                                                        uint8_t* __restrict__ mask, RansacResult* __restrict__ out) {
#pragma clang fp contract(off)
  __shared__ int sh_cnt[16];
  __shared__ double sh_m[4];
  __shared__ int sh_best;
  const int tid = threadIdx.x;
  const bool invalid = wave_any_flag(flags, n_flags);
  const int n = invalid ? 0 : min(*n_dev, cap);
  if (tid == 0) {
    int b;
    bool go;
    const Sim f = refit_chain(xy, n, words, invalid ? 0ull : *best_key, sums, refine, &b, &go);
    sh_m[0] = f.a;
    sh_m[1] = f.b;
    sh_m[2] = f.tx;
    sh_m[3] = f.ty;
    sh_best = b;
  }
  __syncthreads();
  const Sim m{sh_m[0], sh_m[1], sh_m[2], sh_m[3]};
  const int best = sh_best;
  const int4 zero = make_int4(0, 0, 0, 0);
  int local = 0;
  for (int b0 = 0; b0 < cap; b0 += 1024 * kRefineBatch) {
    int4 p[kRefineBatch];
#pragma unroll
    for (int r = 0; r < kRefineBatch; ++r) {
      const int i = b0 + r * 1024 + tid;
      p[r] = (best >= 0 && i < n) ? xy[i] : zero;
    }
#pragma unroll
    for (int r = 0; r < kRefineBatch; ++r) {
      const int i = b0 + r * 1024 + tid;
      if (i < cap) {
        const uint8_t in = (best >= 0 && i < n &&
                            sim_residual_sq(m, (double)p[r].x, (double)p[r].y, (double)p[r].z, (double)p[r].w) < tau2)
                               ? 1 : 0;
        mask[i] = in;
        local += in;
      }
    }
  }
  const int total = block_sum_int(local, sh_cnt);
  if (tid == 0) {
    RansacResult r;
    r.a = m.a;
    r.b = m.b;
    r.tx = m.tx;
    r.ty = m.ty;
    r.best = best;
    r.n_inliers = total;
    r.n_matches = n;
    r.status = invalid ? 1 : 0;
    *out = r;
  }
}

struct ConsensusOut {  // layout of rift2_consensus_result
  int32_t n_inliers;
  int32_t status;
  double sum_sq;
};

// One block of 1024 threads: consensus of the model (a, b, tx, ty) read from
// `model` (device).  Writes mask[0..cap) (if not null) and the inlier count
// and sum of the inliers' squared residuals, added in a fixed order: per
// thread over its strided matches, then a fixed tree over the block.
__global__ void __launch_bounds__(1024) k_consensus(const int4* __restrict__ xy, const int32_t* __restrict__ n_dev,
                                                    int cap, const int32_t* __restrict__ flags, int n_flags,
                                                    const double* __restrict__ model, double tau2,
                                                    uint8_t* __restrict__ mask, ConsensusOut* __restrict__ out) {
#pragma clang fp contract(off)
  __shared__ double sh_d[16];
  __shared__ int sh_cnt[16];
  const bool invalid = wave_any_flag(flags, n_flags);
  const int n = invalid ? 0 : min(*n_dev, cap);
  const Sim m{model[0], model[1], model[2], model[3]};
  int local = 0;
  double ssq = 0.0;
  for (int i = threadIdx.x; i < cap; i += 1024) {
    uint8_t in = 0;
    if (i < n) {
      const int4 p = xy[i];
      const double r2 = sim_residual_sq(m, (double)p.x, (double)p.y, (double)p.z, (double)p.w);
      if (r2 < tau2) {
        in = 1;
        ssq = ssq + r2;
      }
    }
    if (mask) mask[i] = in;
    local += in;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) ssq = ssq + __shfl_xor(ssq, off, 64);
  if ((threadIdx.x & 63) == 0) sh_d[threadIdx.x >> 6] = ssq;
  const int total = block_sum_int(local, sh_cnt);  // its barriers also publish sh_d
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < 16; ++q) t = t + sh_d[q];
    ConsensusOut r;
    r.n_inliers = total;
    r.status = invalid ? 1 : 0;
    r.sum_sq = t;
    *out = r;
  }
}

}  // namespace rift2
