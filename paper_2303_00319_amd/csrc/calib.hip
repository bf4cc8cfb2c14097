// Matrix-core calibration: the MFMA rate this chip sustains when the
// instruction stream holds nothing else.  The distance GEMMs' roofline
// fractions are quoted against the published peaks; these kernels measure how
// much of those peaks register-only chains of the GEMMs' own instructions
// (v_mfma_f32_32x32x2f32 for FP32, v_mfma_f32_32x32x16_bf16 for BF16) reach
// at a given number of waves per SIMD, so the GEMMs' fractions can be read
// against what the matrix cores deliver.
#pragma once

#include <hip/hip_runtime.h>

namespace rift2 {

constexpr int kCalibCUs = 256;  // MI355X compute units

typedef float calib_floatx16 __attribute__((ext_vector_type(16)));

// One wave: two independent accumulator chains of 16 x iters MFMAs each on
// register operands; the sums go to `sink` so the chains are not removed.
__global__ void __launch_bounds__(256) k_calib_mfma_f32(float* __restrict__ sink, int iters, float seed) {
  calib_floatx16 acc0 = {}, acc1 = {};
  const float a = seed + (float)threadIdx.x * 1e-3f, b = 0.5f * seed;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(b, a, acc1, 0, 0, 0);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) s += acc0[e] + acc1[e];
  sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// The same for the BF16 GEMM's instruction (v_mfma_f32_32x32x16_bf16,
// 32768 flops each).
typedef __bf16 calib_bf16x8 __attribute__((ext_vector_type(8)));

__global__ void __launch_bounds__(256) k_calib_mfma_bf16(float* __restrict__ sink, int iters, float seed) {
  calib_floatx16 acc0 = {}, acc1 = {};
  calib_bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(seed + (float)(threadIdx.x + e) * 1e-3f);
    b[e] = (__bf16)(0.5f * seed - (float)e * 1e-3f);
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b, a, acc1, 0, 0, 0);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int e = 0; e < 16; ++e) s += acc0[e] + acc1[e];
  sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace rift2
