// Matrix-core calibration: the FP32 MFMA rate this chip sustains when the
// instruction stream holds nothing else.  The distance GEMM's roofline
// fraction is quoted against the published peak; this kernel measures how
// much of that peak register-only chains of the GEMM's own instruction
// (v_mfma_f32_32x32x2f32) reach at a given number of waves per SIMD, so the
// GEMM's fraction can be read against what the matrix cores deliver.
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

}  // namespace rift2
