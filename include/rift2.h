/*
 * rift2.h -- C ABI of the MI355X (gfx950) RIFT2 hot-path library (librift2.so).
 *
 * RIFT2 (Li, Shi, Hu, Zhang, "RIFT2: Speeding-up RIFT with a New
 * Rotation-Invariance Technique") matches multimodal images in three stages
 * (Section 1; Fig. 1 workflow): keypoint detection on phase-congruency
 * moment maps, description by a maximum index map (MIM) made rotation
 * invariant by the dominant index of its patch histogram (Section 3,
 * Eqs. 1-2), and brute-force nearest-neighbour matching (Section 4).
 * The four compute calls below are those stages:
 *
 *   rift2_filter_mim  log-Gabor bank -> orientation amplitude sums -> MIM,
 *                     phase congruency -> max/min moment maps
 *   rift2_detect      FAST keypoints on a moment map
 *   rift2_describe    dominant-index 6x6xN_o histogram descriptors
 *   rift2_match       nearest-neighbour matching with a ratio test
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers named *_dev and every image, map, keypoint, descriptor and
 *   workspace pointer are DEVICE pointers on the current HIP device; the
 *   caller owns all of them.  Parameter records are host pointers.
 * - The library allocates no device memory.  Scratch space comes from the
 *   caller as (workspace, workspace_bytes); size it with the matching
 *   rift2_*_workspace_size call.  A workspace may be reused by consecutive
 *   calls on one stream but not by calls that can overlap.
 * - `stream` is a hipStream_t (NULL = default stream).  Calls only enqueue
 *   work and return; arguments are validated on the host before anything is
 *   enqueued.  Counts produced on the device (keypoints, descriptor rows,
 *   matches) stay in device memory so stages chain without a host sync.
 * - Images and maps are row-major H x W with x = column, y = row, 0-based.
 * - Errors: RIFT2_ERR_INVALID_ARG (null pointer, bad parameter),
 *   RIFT2_ERR_UNSUPPORTED (size or parameter outside what the kernels are
 *   built for), RIFT2_ERR_WORKSPACE (workspace too small), RIFT2_ERR_DEVICE
 *   (a HIP call or launch failed; device faults surface at the next
 *   synchronisation), RIFT2_ERR_NOT_INITIALIZED (a call that runs FFTs on a
 *   device where rift2_init has not run).  On error nothing further is
 *   enqueued.
 * - Capacities cannot overflow: detect writes at most max_keypoints records,
 *   describe at most rows-per-keypoint x kpt_cap rows (checked against
 *   desc_cap on the host) and match at most one record per A keypoint, so no
 *   call truncates its output.
 */
#ifndef RIFT2_H
#define RIFT2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RIFT2_OK = 0,
  RIFT2_ERR_INVALID_ARG = 1,
  RIFT2_ERR_UNSUPPORTED = 2,
  RIFT2_ERR_WORKSPACE = 3,
  RIFT2_ERR_DEVICE = 4,
  RIFT2_ERR_NOT_INITIALIZED = 5
} rift2_status;

typedef enum { RIFT2_U8 = 0, RIFT2_U16 = 1, RIFT2_F32 = 2 } rift2_dtype;

/* Distance GEMM precision: FP32 and BF16 give the same exact dots on the
 * integer counts; FP8 (E4M3, power-of-two scale per row) selects 8
 * candidates per query approximately and re-ranks them with exact dots. */
typedef enum { RIFT2_PREC_FP32 = 0, RIFT2_PREC_BF16 = 1, RIFT2_PREC_FP8 = 2 } rift2_precision;

/* Log-Gabor bank and phase-congruency constants (Sections 2.1-2.2 name the
 * log-Gabor convolution sequence and one-dimensional phase congruency per
 * orientation; the paper prints no constants).  Filter of scale s and
 * orientation o on DFT bin (k, l):
 *   G = exp(-ln^2(r f0_s^-1) / (2 ln^2 sigma_onf)) * 1/(1 + (r/lp_cutoff)^(2 lp_order))
 *       * exp(-dtheta^2 / (2 sigma_theta^2)),
 *   f0_s = 1/(min_wavelength mult^s), theta_o = o pi / n_orient,
 *   sigma_theta = (pi / n_orient) / dtheta_on_sigma, G = 0 at DC and on the
 *   Nyquist row/column.  Supported: 2 <= n_scales <= 8, 2 <= n_orient <= 8. */
typedef struct {
  int32_t n_scales;
  int32_t n_orient;
  float min_wavelength;
  float mult;
  float sigma_onf;
  float dtheta_on_sigma;
  float lp_cutoff;
  int32_t lp_order;
  float k;      /* noise threshold: mean + k sigma of the noise energy */
  float cutoff; /* frequency-spread cutoff of the sigmoid weight */
  float g;      /* sigmoid gain */
  float eps;
} rift2_pc_params;

/* FAST detector (Section 2.1; Table 1: threshold 0.001, 5000 keypoints,
 * patch 96).  Points whose patch would leave the image are dropped. */
typedef struct {
  float fast_threshold;
  int32_t max_keypoints;
  int32_t patch_size;
} rift2_detect_params;

/* Row forms of rift2_describe.  RIFT2_DESC_DOMINANT is the paper's method
 * (Section 3).  The other two serve RIFT's convolution-sequence ring
 * (Section 2.3), the baseline RIFT2 replaces: RIFT2_DESC_PLAIN is one row of
 * the cell histograms as computed (the ring's first member), RIFT2_DESC_RING
 * is n_orient rows per keypoint, row k n_orient + w built from the MIM with
 * layer w as the ring's first (bin b counts MIM value (b + w) mod n_orient).
 * RIFT2_DESC_TURNED is RIFT2's descriptor with the sampling grid also turned
 * by the dominant index, as SIFT turns its grid by its dominant orientation
 * (Section 3 takes SIFT as its model): s and s2 come from the MIM values in
 * the disc of diameter patch_size around the keypoint; sample (i, j) of the
 * patch_size^2 grid reads the pixel (x + ((c U + s V) >> 17),
 * y + ((-s U + c V) >> 17)) with U = 2i - patch_size + 1,
 * V = 2j - patch_size + 1 and (c, s) = round(2^16 (cos, sin)(k pi / n_orient))
 * for the row's index k; samples outside the image are not counted; rows
 * as in RIFT2_DESC_DOMINANT (second row on its own turned grid). */
typedef enum { RIFT2_DESC_DOMINANT = 0, RIFT2_DESC_PLAIN = 1, RIFT2_DESC_RING = 2, RIFT2_DESC_TURNED = 3 } rift2_desc_mode;

/* Descriptor (Section 2.2: 6x6 grid of N_o-bin MIM histograms; Section 3:
 * dominant index and second MIM when the second peak reaches the dominant
 * ratio, Table 1: 0.8).  The ratio is the exact fraction num/den. */
typedef struct {
  int32_t patch_size;
  int32_t grid;
  int32_t n_orient;
  int32_t dominant_num;
  int32_t dominant_den;
  int32_t mode; /* rift2_desc_mode */
} rift2_desc_params;

/* Matching (Section 4: brute force, nearest feature distance) with a
 * second-neighbour ratio test d1^2 < ratio_sq * d2^2.
 * ring = 0: the rows of A and B are matched as they are.
 * ring = R (2..8, FP32 or BF16): RIFT's ring matching (Section 2.3).  A holds
 * R rows per keypoint in RIFT2_DESC_RING form and B one RIFT2_DESC_PLAIN row
 * per keypoint.  The result is that of matching each A keypoint's plain row
 * against all R ring rows of every B keypoint (candidate order: B keypoint
 * r's ring row w is candidate r R + w); A row g R + w paired with B row r
 * gives the same dot product as A's plain row with ring row (R - w) mod R of
 * B keypoint r, so A carries the R-fold rows and the cost.
 * mutual = 1 (a stricter form of Section 4's nearest-distance rule): an A row
 * that passes the ratio test with nearest B row j1 is kept only if the
 * nearest A row of j1 -- the smallest argmin over all A rows of the same d2
 * values, ties to the lowest row -- belongs to its own A keypoint.  The check
 * runs a second distance GEMM with the roles swapped (twice the matching
 * work); in the FP8 form that reverse nearest row is the exact nearest of its
 * 8 re-ranked candidates.  Not combined with ring. */
typedef struct {
  float ratio_sq;
  int32_t precision; /* rift2_precision of the distance GEMM */
  int32_t ring;      /* 0, or rows per A keypoint of a ring matching */
  int32_t mutual;    /* 0 or 1: mutual nearest-neighbour check (ring = 0 only) */
} rift2_match_params;

typedef struct {
  int32_t x;
  int32_t y;
  float score;
} rift2_keypoint;

typedef struct {
  int32_t kp_a;
  int32_t kp_b;
  float dist2;
} rift2_correspondence;

/* Defaults: n_scales 4, n_orient 6, min_wavelength 3, mult 2.1, sigma_onf
 * 0.55, dtheta_on_sigma 1.2, lp 0.45/15, k 2, cutoff 0.5, g 10, eps 1e-4;
 * FAST 0.001, 5000 keypoints, patch 96; grid 6, ratio 4/5; ratio_sq 0.81,
 * FP32, no ring, no mutual check; descriptor form RIFT2_DESC_DOMINANT.  Any
 * argument may be NULL. */
void rift2_default_params(rift2_pc_params* pc, rift2_detect_params* det, rift2_desc_params* desc,
                          rift2_match_params* match);

const char* rift2_status_string(rift2_status s);

/* Loads the constant tables (FFT twiddles) onto `device`.  Must be called
 * once per device before the first compute call on it; idempotent. */
rift2_status rift2_init(int device);

/* Supported image sides are 2^a * 3^b in {256, 512, 768, 1024, 1536, 2048,
 * 4096}; H and W may differ. */
int rift2_size_supported(int n);

/* Workspace byte counts (0 if the arguments are unsupported). */
size_t rift2_filter_workspace_size(int H, int W, const rift2_pc_params* pc);
size_t rift2_detect_workspace_size(int H, int W, const rift2_detect_params* det);
size_t rift2_describe_workspace_size(int32_t kpt_cap);
size_t rift2_match_workspace_size(int32_t cap_a, int32_t cap_b, int32_t D, const rift2_match_params* mp);

/* Filter bank, MIM and moments of one image (Section 2.2: A_o = sum over
 * scales of the response amplitudes, MIM = argmax_o A_o; Section 2.1: phase
 * congruency per orientation and its max/min moment over orientation).
 *   img         H x W pixels of type `dtype`, row pitch `pitch` elements
 *   mim         H x W uint8, 0-based orientation index (ties -> lowest)
 *   max_moment  H x W float, M
 *   min_moment  H x W float, m (may be NULL)
 *   amp_sums    n_orient x H x W float, A_o (may be NULL)
 * mim must be 4-byte aligned, max_moment and min_moment 16-byte aligned
 * (RIFT2_ERR_INVALID_ARG otherwise).  Circular (periodic) convolution, raw
 * pixel values.  RIFT2_ERR_NOT_INITIALIZED if rift2_init has not run on the
 * current device. */
rift2_status rift2_filter_mim(const void* img, int32_t dtype, int32_t H, int32_t W, int64_t pitch,
                              const rift2_pc_params* pc, uint8_t* mim, float* max_moment,
                              float* min_moment, float* amp_sums, void* workspace,
                              size_t workspace_bytes, void* stream);

/* The filter bank of several images of one size in shared launches: every
 * kernel of rift2_filter_mim covers all n images (1 <= n <=
 * RIFT2_MAX_FILTER_BATCH), so small images fill the device together instead
 * of one after another.  Each job is one image's rift2_filter_mim arguments
 * (same rules; its own workspace of rift2_filter_workspace_size bytes, which
 * must not overlap another job's: RIFT2_ERR_INVALID_ARG); the results are
 * those of n separate calls.  Errors as rift2_filter_mim, checked for every
 * job before anything is enqueued. */
#define RIFT2_MAX_FILTER_BATCH 8
typedef struct {
  const void* img;
  uint8_t* mim;
  float* max_moment;
  float* min_moment;
  float* amp_sums;
  void* workspace;
  size_t workspace_bytes;
} rift2_filter_job;

rift2_status rift2_filter_mim_batch(int32_t n, const rift2_filter_job* jobs, int32_t dtype, int32_t H, int32_t W,
                                    int64_t pitch, const rift2_pc_params* pc, void* stream);

/* Diagnostics of the filter stage (not needed for computing).
 *
 * rift2_debug_response: the complex response EO_{s,o} = IDFT2(DFT2(img) G_{s,o})
 * of one filter of the bank (Section 2.2: the response components of the
 * log-Gabor filter, whose amplitudes rift2_filter_mim sums per orientation),
 * computed by the same kernels as rift2_filter_mim.
 *   scale, orient  0 <= scale < n_scales, 0 <= orient < n_orient
 *   eo             H x W complex values as interleaved float pairs (re, im),
 *                  8-byte aligned
 *   workspace      as for rift2_filter_mim (rift2_filter_workspace_size);
 *                  its previous contents are overwritten
 * Errors as rift2_filter_mim; RIFT2_ERR_INVALID_ARG for a filter index out of
 * range. */
rift2_status rift2_debug_response(const void* img, int32_t dtype, int32_t H, int32_t W, int64_t pitch,
                                  const rift2_pc_params* pc, int32_t scale, int32_t orient, float* eo,
                                  void* workspace, size_t workspace_bytes, void* stream);

/* rift2_debug_noise: the noise-threshold intermediates (Section 2.1's phase
 * congruency; median of the smallest-scale amplitude, Rayleigh model) that
 * the last rift2_filter_mim call on `workspace` left in it, copied on
 * `stream` (enqueue it after that call, on the same stream):
 *   a0           n_orient x H x W float, A0_o = |EO_{0,o}| as the selection
 *                saw it (may be NULL)
 *   order_stats  n_orient x 2 float: the order statistics of rank HW/2 - 1
 *                and HW/2 of A0_o (their mean is the median; may be NULL)
 *   t_o          n_orient double: the threshold T_o, evaluated in FP64
 *                (may be NULL)
 * H, W and pc must be those of the rift2_filter_mim call. */
rift2_status rift2_debug_noise(const void* workspace, size_t workspace_bytes, int32_t H, int32_t W,
                               const rift2_pc_params* pc, float* a0, float* order_stats, double* t_o,
                               void* stream);

/* rift2_debug_mfma_rate: calibration for the distance GEMMs' rooflines (the
 * matching step of Section 4 is a dense contraction on the matrix cores).
 * Runs register-only chains of a GEMM's MFMA instruction -- precision
 * RIFT2_PREC_FP32: v_mfma_f32_32x32x2f32, 4096 flops each; RIFT2_PREC_BF16:
 * v_mfma_f32_32x32x16_bf16, 32768 flops each -- with `waves_per_simd` waves
 * on every SIMD of the chip, each wave 2 x 16 x `iters` instructions, `reps`
 * launches back to back after one warm-up launch, and writes their elapsed
 * milliseconds to *ms (host memory; the call synchronises `stream`).  The
 * sustained rate is reps x 256 x 4 x waves_per_simd x 32 x iters x (flops per
 * instruction) / ms.
 *   waves_per_simd  1..4
 *   sink            device float, 256 x 256 x waves_per_simd entries (the
 *                   chains' sums, written so they are kept)
 * Errors: RIFT2_ERR_INVALID_ARG (precision, range, null pointer),
 * RIFT2_ERR_UNSUPPORTED (a device without 256 compute units),
 * RIFT2_ERR_DEVICE. */
rift2_status rift2_debug_mfma_rate(int32_t precision, int32_t waves_per_simd, int32_t iters, int32_t reps, float* sink,
                                   float* ms, void* stream);

/* FAST keypoints on `moment` (H x W float, normally the max moment map):
 * min-max normalisation to [0, 1], 16-pixel segment test with arc 9 and
 * score = largest passing threshold, corner iff score > fast_threshold, 3x3
 * non-maximum suppression (ties: lower raster index wins), patch-border
 * mask, then the max_keypoints strongest by (score desc, y*W+x asc).
 *   moment      16-byte aligned
 *   kpts        capacity det->max_keypoints, sorted strongest first
 *   n_kpts_dev  device int32: number of keypoints written */
rift2_status rift2_detect(const float* moment, int32_t H, int32_t W, const rift2_detect_params* det,
                          rift2_keypoint* kpts, int32_t* n_kpts_dev, void* workspace,
                          size_t workspace_bytes, void* stream);

/* rift2_detect without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The scratch is a 20 MiB array that the
 * library keeps in device memory on every device where rift2_init has run,
 * until the process ends; the call itself allocates nothing.  It covers every
 * image and keypoint count whose rift2_detect_workspace_size is at most
 * 20 MiB (e.g. 2048 x 2048 with 50 000 keypoints; not 4096 x 4096).
 * Results are those of rift2_detect on the same arguments.
 *   RIFT2_ERR_WORKSPACE        rift2_detect_workspace_size(H, W, det) > 20 MiB
 *   RIFT2_ERR_NOT_INITIALIZED  rift2_init has not run on the current device
 * Every call on one device shares that device's array, and it keeps the last
 * call's contents (each call initialises what it reads): calls that can
 * overlap on one device (concurrent streams, host threads) race and give
 * wrong results; serialise them on one stream.  No stage timing is recorded. */
rift2_status rift2_detect_noalloc(const float* moment, int32_t H, int32_t W, const rift2_detect_params* det,
                                  rift2_keypoint* kpts, int32_t* n_kpts_dev, void* stream);

/* RIFT's full detector (Section 2.1): FAST points on the maximum-moment map
 * (edge features) and on the minimum-moment map (corners), each map with its
 * own min-max normalisation, scores, 3x3 suppression and border mask as in
 * rift2_detect, then their union: a pixel kept on both maps appears once with
 * the larger of its two scores, and the max_keypoints strongest of the union
 * are taken by (score desc, y*W+x asc).  Both maps 16-byte aligned; the
 * workspace comes from rift2_detect_union_workspace_size. */
size_t rift2_detect_union_workspace_size(int H, int W, const rift2_detect_params* det);
rift2_status rift2_detect_union(const float* max_moment, const float* min_moment, int32_t H, int32_t W,
                                const rift2_detect_params* det, rift2_keypoint* kpts, int32_t* n_kpts_dev,
                                void* workspace, size_t workspace_bytes, void* stream);

/* Dominant-index descriptors (Section 3, Eqs. 1-2) of the first *n_kpts_dev
 * keypoints (at most kpt_cap) on a 0-based MIM.  Row layout: uint16 counts
 * desc[row][(cy*grid + cx)*n_orient + b] = #{pixels of cell (cy, cx) whose
 * MIM value is (b + s) mod n_orient}; primary rows (s = dominant index) for
 * keypoints 0..n-1 come first, then the secondary rows (s = second peak)
 * in keypoint order.  inv_norm[row] = fl(1 / fl(sqrt(sum counts^2))),
 * desc_kp[row] = keypoint index.  desc_cap must be >= 2 * kpt_cap
 * (RIFT2_DESC_DOMINANT, RIFT2_DESC_TURNED), kpt_cap (RIFT2_DESC_PLAIN) or
 * n_orient * kpt_cap (RIFT2_DESC_RING, rows k n_orient + w).
 *   n_desc_dev  device int32: number of rows written */
rift2_status rift2_describe(const uint8_t* mim, int32_t H, int32_t W, const rift2_keypoint* kpts,
                            const int32_t* n_kpts_dev, int32_t kpt_cap, const rift2_desc_params* dp,
                            uint16_t* desc, float* inv_norm, int32_t* desc_kp, int32_t desc_cap,
                            int32_t* n_desc_dev, void* workspace, size_t workspace_bytes,
                            void* stream);

/* FP32 view of descriptor rows: out[r][d] = fl(desc[r][d] * inv_norm[r]),
 * the L2-normalised vectors whose Euclidean distances rift2_match compares
 * (Section 2.2 concatenates the cell histograms into the feature vector),
 * for the first *n_rows_dev rows (at most cap rows of D values).  out is
 * cap x D floats; rows past *n_rows_dev are left alone. */
rift2_status rift2_desc_normalize(const uint16_t* desc, const float* inv_norm, const int32_t* n_rows_dev,
                                  int32_t cap, int32_t D, float* out, void* stream);

/* Brute-force matching of descriptor rows A against B (Section 4).  The
 * squared distance of normalised count vectors is evaluated as
 * t = fl(fl(dot * invA_i) * invB_j), d2 = fl(2 - 2t), with the dot product
 * exact (integer counts; BF16 holds counts <= 256 exactly and FP32
 * accumulation of sums < 2^24 is exact, so both precisions give the same
 * dots).  Per A row: j1 = nearest row (ties -> lowest j), j2 = nearest row of
 * a different B keypoint; accepted iff d2(j1) < fl(ratio_sq * d2(j2)).  Per A
 * keypoint the accepted row with the smallest d2 (ties -> lowest row) is
 * kept.  Output sorted by kp_a; capacity cap_a entries.
 *   desc_a, desc_b  rows of D uint16 counts, 16-byte aligned
 *   nA_dev, nB_dev  device int32 row counts (<= cap_a, cap_b)
 *   n_out_dev       device int32: number of matches written */
rift2_status rift2_match(const uint16_t* desc_a, const float* inv_a, const int32_t* kp_a,
                         const int32_t* nA_dev, int32_t cap_a, const uint16_t* desc_b,
                         const float* inv_b, const int32_t* kp_b, const int32_t* nB_dev,
                         int32_t cap_b, int32_t D, const rift2_match_params* mp, rift2_correspondence* out,
                         int32_t* n_out_dev, void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------- outlier removal
 * The putative matches are filtered by RANSAC (Section 1 and Fig. 1 name
 * RANSAC, Fischler and Bolles 1981, as the step after matching), here over
 * the similarity model u = a x - b y + tx, v = b x + a y + ty (the class of
 * a rotation plus a translation, which the paper's image pairs differ by).
 * Section 4 counts a match as correct when its residual under the
 * ground-truth transform is below 3 pixels; rift2_consensus computes that
 * count and the inliers' squared residuals for any given model.
 *
 * Matches are rift2_correspondence records (as rift2_match writes them)
 * whose kp_a / kp_b index the keypoint tables kpts_a / kpts_b (as
 * rift2_detect writes them); a descriptor row's keypoint index is what
 * rift2_match reports.  Coordinates must lie in [0, 8192), keypoint indices
 * in [0, kpt_cap); a list that breaks this is treated as empty and its
 * result carries status RIFT2_ERR_INVALID_ARG.  Every floating-point step is
 * one IEEE double operation in a fixed order, so counts, model and mask are
 * reproducible bit for bit. */
typedef struct {
  double threshold; /* inlier iff squared residual < threshold^2 (pixels); Section 4 uses 3 */
  int32_t refine;   /* least-squares refits of the chosen hypothesis, 0..16 */
} rift2_ransac_params;

typedef struct {
  double a, b, tx, ty; /* final model (all 0 when best < 0) */
  int32_t best;        /* chosen hypothesis, -1 when none has a model */
  int32_t n_inliers;   /* consensus-set size of the final model */
  int32_t n_matches;   /* number of matches used (0 for an invalid list) */
  int32_t status;      /* RIFT2_OK or RIFT2_ERR_INVALID_ARG (see above) */
} rift2_similarity;

typedef struct {
  int32_t n_inliers; /* matches with squared residual < threshold^2 */
  int32_t status;    /* RIFT2_OK or RIFT2_ERR_INVALID_ARG */
  double sum_sq;     /* sum of the inliers' squared residuals (RMSE = sqrt(sum_sq / n_inliers)) */
} rift2_consensus_result;

/* Workspace of rift2_ransac / rift2_consensus (0 if the arguments are out of range). */
size_t rift2_ransac_workspace_size(int32_t match_cap, int32_t n_hyp);

/* RANSAC over the first *n_matches_dev matches (at most match_cap <= 131072):
 *  1. hypothesis h (0 <= h < n_hyp <= 2^20) samples matches
 *     i = floor(u * N / 2^32) for its two uniform words u = words[2h],
 *     words[2h + 1] (device uint32, drawn by the caller) and fits the
 *     similarity to them exactly: (a + ib) = (w2 - w1) / (z2 - z1),
 *     t = w1 - (a + ib) z1 with z = x + iy in A and w in B;
 *  2. counts[h] = #{matches with squared residual < threshold^2}, or -1 when
 *     z1 = z2 or N < 2;
 *  3. the hypothesis with the largest count wins (lowest h on ties);
 *  4. `refine` times: least-squares fit to the current consensus set, then
 *     the set is recomputed (stops early when the set has no unique fit).
 *   counts       device int32 [n_hyp], or NULL (kept in the workspace)
 *   inlier_mask  device uint8 [match_cap]: 1 for the final consensus set
 *   result       device rift2_similarity */
rift2_status rift2_ransac(const rift2_correspondence* matches, const int32_t* n_matches_dev, int32_t match_cap,
                          const rift2_keypoint* kpts_a, int32_t kpt_cap_a, const rift2_keypoint* kpts_b,
                          int32_t kpt_cap_b, const uint32_t* words, int32_t n_hyp, const rift2_ransac_params* rp,
                          int32_t* counts, uint8_t* inlier_mask, rift2_similarity* result, void* workspace,
                          size_t workspace_bytes, void* stream);

/* Consensus of the model (a, b, tx, ty) read from `model` (device, 4
 * doubles; a rift2_similarity's first four fields qualify) over the first
 * *n_matches_dev matches: mask (device uint8 [match_cap], may be NULL) and
 * result (device).  sum_sq is accumulated in a fixed order. */
rift2_status rift2_consensus(const double* model, const rift2_correspondence* matches, const int32_t* n_matches_dev,
                             int32_t match_cap, const rift2_keypoint* kpts_a, int32_t kpt_cap_a,
                             const rift2_keypoint* kpts_b, int32_t kpt_cap_b, double threshold, uint8_t* mask,
                             rift2_consensus_result* result, void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------- serving
 * Continuous batching of image-pair requests of mixed sizes (the paper
 * times one pair at a time; this serves a stream of them).  Requests wait in
 * a host queue and are admitted in arrival order as soon as a stream pair is
 * free and the request's buffers fit into the caller's HBM arena (the
 * memory budget); queued requests of the same size are admitted with it and
 * their filter banks share launches (rift2_engine_set_batch); admitted pairs
 * then run concurrently on their own streams.
 * Every stage is the same call as above, so a request's result does not
 * depend on what else is in flight.  One engine per host thread. */
typedef struct rift2_engine rift2_engine;

typedef struct {
  int64_t id;                 /* caller's tag, returned with the completion */
  const void* img_a;          /* device, H x W of `dtype`, row pitch W, resident until completion */
  const void* img_b;
  int32_t dtype, H, W;        /* both images of a pair share one size */
  int32_t max_keypoints;      /* K per image; <= 0 selects floor(2e-3 * H * W) */
  rift2_correspondence* out;  /* device, capacity 2 K entries (written by the match stage) */
  int32_t* n_out;             /* device int32: number of matches */
  void* ready;                /* hipEvent_t recorded once the images and out / n_out are ready
                                 (the request's first stage waits for it), or NULL if they
                                 already are */
} rift2_request;

typedef struct {
  int64_t id;
  int32_t status;   /* rift2_status of the request */
  float gpu_ms;     /* admission to completion, on the GPU clock */
  double admit_ms;  /* admission, ms after the engine's creation (GPU clock) */
  double done_ms;   /* completion, ms after the engine's creation (GPU clock) */
  int32_t batch;    /* requests admitted together with it, itself included (their filter banks
                       shared launches; 1 = alone) */
} rift2_completion;

/* Arena bytes one request of this size needs (0 if unsupported); the
 * detector, descriptor and matcher parameters are those given to create. */
size_t rift2_engine_request_bytes(int32_t H, int32_t W, int32_t max_keypoints, const rift2_pc_params* pc,
                                  const rift2_detect_params* det, const rift2_desc_params* dp,
                                  const rift2_match_params* mp);

/* arena: device memory of arena_bytes (256-byte aligned), owned by the
 * caller and used only by the engine until rift2_engine_destroy returns.
 * max_inflight (1..64): requests running at once (two streams each).  The
 * parameter records are copied; det->max_keypoints is ignored (per
 * request).  Calls rift2_init(device). */
rift2_status rift2_engine_create(int device, void* arena, size_t arena_bytes, int32_t max_inflight,
                                 const rift2_pc_params* pc, const rift2_detect_params* det,
                                 const rift2_desc_params* dp, const rift2_match_params* mp,
                                 rift2_engine** out);

/* Queues a request (host only; nothing is launched until the next poll).
 * Errors: RIFT2_ERR_INVALID_ARG, RIFT2_ERR_UNSUPPORTED (size). */
rift2_status rift2_engine_submit(rift2_engine* e, const rift2_request* r);

/* Reaps finished requests into done[0..max_done) and admits queued ones;
 * returns the number of completions written, or minus a rift2_status.  A
 * request that can never fit the arena completes with RIFT2_ERR_WORKSPACE. */
int32_t rift2_engine_poll(rift2_engine* e, rift2_completion* done, int32_t max_done);

/* Up to max_requests (1..RIFT2_MAX_FILTER_BATCH / 2, default 4) queued
 * requests of one size, type and keypoint count are admitted together and
 * their filter banks run as one batch (rift2_filter_mim_batch); 1 admits
 * requests one at a time.  A request's results do not depend on it. */
rift2_status rift2_engine_set_batch(rift2_engine* e, int32_t max_requests);

/* Requests queued, running, or finished but not yet reported. */
int32_t rift2_engine_pending(const rift2_engine* e);

/* Waits for the running requests, then frees the engine's streams and events. */
rift2_status rift2_engine_destroy(rift2_engine* e);

/* Stage timing (diagnostics, not needed for computing).  While enabled, each
 * compute call records a HIP event pair on its stream around each of its
 * kernel groups: 0 row DFT, 1 column DFT + filter products + column IDFT,
 * 2 noise pre-pass, 3 noise median / threshold, 4 row IDFT + amplitude
 * sums + phase congruency per orientation, 5 detect (all kernels),
 * 6 describe (all kernels), 7 match table preparation, 8 match distance
 * GEMM + top-k, 9 match merge / ratio test / output, 10 per-pixel reduction
 * over orientations (MIM, moments), 11 outlier removal / consensus.
 * rift2_profile_read waits for the recorded events, adds the elapsed
 * milliseconds and the number of launches per group into ms[group] and
 * count[group] (arrays of n_groups >= 12 host
 * elements), forgets them and returns the number of groups.  Events are
 * owned by the library; enabling on one thread while another computes is
 * not supported. */
rift2_status rift2_profile_enable(int on);
int rift2_profile_read(double* ms, int64_t* count, int n_groups);

#ifdef __cplusplus
}
#endif

#endif /* RIFT2_H */
