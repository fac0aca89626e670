// Matrix-core and buffer-load helpers of the GEMM, M2L and leaf kernels (gfx950, wave64).
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

// Buffer loads: a wave-uniform base in the resource (SGPRs), the lane's byte
// offset (below 2^31) in one VGPR instead of a 64-bit address; 0x00020000 is
// gfx9's raw 32-bit data-format word.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const float* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ float4 bload(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

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
