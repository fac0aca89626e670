// Matrix-core helpers shared by the GEMM and M2L kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

namespace kifmm {

typedef float v16f __attribute__((ext_vector_type(16)));

// One 32x32x2 FP32 matrix-core step (wave64): lane (i, h) = (l % 32, l / 32)
// holds A[i][h] and B[h][i]; the accumulator holds D[8 (v / 4) + 4 h + v % 4][i]
// in element v.
__device__ __forceinline__ v16f mfma32(float a, float b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Four 16x16x4 steps over 16 consecutive k.  Lane (i, q) holds a = A[i][4q ..
// 4q+3] and b = B^T[j][4q .. 4q+3]; step r contracts k = 4q + r.  The
// accumulator holds D[4q + v][i] in element v.
__device__ __forceinline__ v4f mfma16x4(const float4 a, const float4 b, v4f c) {
  c = mfma16(a.x, b.x, c);
  c = mfma16(a.y, b.y, c);
  c = mfma16(a.z, b.z, c);
  c = mfma16(a.w, b.w, c);
  return c;
}

}  // namespace kifmm
