// Batched FP32 GEMM of the kiFMM evaluate on the matrix cores (gfx950): the
// check-to-equivalent factors, U2U, compression, post and D2D products
// (v_mfma_f32_16x16x4_f32).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "mfma.hpp"

namespace kifmm {

// ---------------------------------------------------------------- GEMM ---
// Y[yrow(b)][o] = alpha * sum_k W[o][k] X[xrow(b)][k]  (+ Y[yrow(b)][o] when beta)
// W: [>= round_up(nout, 64)][ldw] row-major, rows >= nout zero.  X rows: ldx.
// K, nout, ldx, ldy, ldw are multiples of 4; pointers 16-byte aligned.
// Each wave computes a 32 (outputs) x 32 (boxes) tile as 2 x 2 blocks of
// v_mfma_f32_16x16x4_f32 over 16-k steps: lane (i, q) = (l % 16, l / 16) loads
// one float4 of each of two W rows and two X rows (64 contiguous bytes of a
// row per four lanes), and the four independent accumulators keep the matrix
// core busy.  Operands are loaded one step ahead of their use; a K that is not
// a multiple of 16 ends with 4-k steps.  SPLIT = 1: a 64 x 64 tile per
// workgroup, its 4 waves as 2 (outputs) x 2 (boxes), each over the whole K.
// SPLIT = 4: a 32 x 32 tile per workgroup, each wave over a quarter of the
// 16-k steps, the four partial tiles added through LDS in a fixed order (long K
// with few tiles: U2U of the upper levels).
struct GemmOps {
  float4 a[2], b[2];
};

template <int SPLIT>
__global__ __launch_bounds__(256) void k_gemm_nt(const float* __restrict__ W, int ldw, const float* __restrict__ X,
                                                 int ldx, const int* __restrict__ xrow, float* __restrict__ Y, int ldy,
                                                 const int* __restrict__ yrow, int nbox, int nout, int K, float alpha,
                                                 int beta, long long xbs, long long ybs, int ywide) {
  X += blockIdx.z * xbs;  // batch (right-hand side) blockIdx.z
  if (!ywide) Y += blockIdx.z * ybs;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int i16 = lane & 15, q = lane >> 4;
  const int nstep = K >> 4;  // whole 16-k steps
  int o0, b0, s0, s1;
  if (SPLIT == 1) {
    o0 = blockIdx.y * 64 + (wave & 1) * 32;
    b0 = blockIdx.x * 64 + (wave >> 1) * 32;
    s0 = 0;
    s1 = nstep;
  } else {
    o0 = blockIdx.y * 32;
    b0 = blockIdx.x * 32;
    s0 = wave * nstep / 4;
    s1 = (wave + 1) * nstep / 4;
  }
  const float* wp[2];
  const float* xp[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) wp[m] = W + (size_t)(o0 + 16 * m + i16) * ldw + 4 * q;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int bb = min(b0 + 16 * nb + i16, nbox - 1);
    xp[nb] = X + (size_t)(xrow ? xrow[bb] : bb) * ldx + 4 * q;
  }
  v4f acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) acc[m][nb] = v4f{0.f, 0.f, 0.f, 0.f};
  auto load = [&](GemmOps& r, int st) {
#pragma unroll
    for (int m = 0; m < 2; ++m) r.a[m] = *reinterpret_cast<const float4*>(wp[m] + 16 * st);
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) r.b[nb] = *reinterpret_cast<const float4*>(xp[nb] + 16 * st);
  };
  auto compute = [&](const GemmOps& r) {
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) acc[m][nb] = mfma16x4(r.a[m], r.b[nb], acc[m][nb]);
  };
  if (s0 < s1) {
    // Two register sets, each loaded one step ahead of its use.  An odd step
    // count takes its first step alone, so that every load and product in the
    // loop is unconditional (the compiler keeps the loads ahead and the wait
    // counts exact; past the end the last step is loaded again, unused).
    GemmOps r0, r1;
    load(r0, s0);
    int st = s0;
    if ((s1 - s0) & 1) {
      compute(r0);
      st = s0 + 1;
      load(r0, min(st, s1 - 1));
    }
    for (; st < s1; st += 2) {
      load(r1, st + 1);
      __builtin_amdgcn_sched_barrier(0);
      compute(r0);
      __builtin_amdgcn_sched_barrier(0);
      load(r0, min(st + 2, s1 - 1));
      __builtin_amdgcn_sched_barrier(0);
      compute(r1);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if (SPLIT == 1 || wave == 3) {
    // the last K mod 16: 4-k steps, lane (i, q) holding k = k0 + q
    for (int k = 16 * nstep; k < K; k += 4) {
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          acc[m][nb] = mfma16(wp[m][k - 3 * q], xp[nb][k - 3 * q], acc[m][nb]);  // element k + q
    }
  }
  // acc[m][nb][v]: output row o0 + 16 m + 4 q + v, box column b0 + 16 nb + i16
  int g0 = 0, g1 = 4;  // the (m, nb) blocks g = m + 2 nb this lane stores
  if (SPLIT == 4) {
    __shared__ float red[4][16][64];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wave][4 * (m + 2 * nb) + v][lane] = acc[m][nb][v];
    __syncthreads();
    // wave w adds the four partial tiles of block w in wave order
    const int m = wave & 1, nb = wave >> 1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float t = red[0][4 * wave + v][lane];
#pragma unroll
      for (int w = 1; w < 4; ++w) t += red[w][4 * wave + v][lane];
      acc[m][nb][v] = t;
    }
    g0 = wave;
    g1 = wave + 1;
  }
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    if (g < g0 || g >= g1) continue;
    const int m = g & 1, nb = g >> 1;
    const int b = b0 + 16 * nb + i16;
    const int o = o0 + 16 * m + 4 * q;
    if (b >= nbox || o >= nout) continue;
    const int r = yrow ? yrow[b] : b;
    // ywide: the 32-right-hand-side lane order of k_m2l_wide, [row][o / 8][32][8]
    float4* yp = reinterpret_cast<float4*>(
        ywide ? Y + (((size_t)r * (nout >> 3) + (o >> 3)) * 32 + blockIdx.z) * 8 + (o & 7) : Y + (size_t)r * ldy + o);
    float4 v = make_float4(alpha * acc[m][nb][0], alpha * acc[m][nb][1], alpha * acc[m][nb][2], alpha * acc[m][nb][3]);
    if (beta) {
      const float4 old = *yp;
      v.x += old.x;
      v.y += old.y;
      v.z += old.z;
      v.w += old.w;
    }
    *yp = v;
  }
}

void launch_gemm_nt(const float* W, int ldw, const float* X, int ldx, const int* xrow, float* Y, int ldy,
                    const int* yrow, int nbox, int nout, int K, float alpha, int beta, hipStream_t s, int batch,
                    long long xbs, long long ybs, int ywide) {
  if (nbox <= 0 || batch <= 0) return;
  const long long tiles64 = (long long)((nbox + 63) / 64) * ((nout + 63) / 64) * batch;
  if (tiles64 < 512 && K >= 256) {
    dim3 grid((nbox + 31) / 32, (nout + 31) / 32, batch);
    hipLaunchKernelGGL(k_gemm_nt<4>, grid, dim3(256), 0, s, W, ldw, X, ldx, xrow, Y, ldy, yrow, nbox, nout, K, alpha,
                       beta, xbs, ybs, ywide);
  } else {
    dim3 grid((nbox + 63) / 64, (nout + 63) / 64, batch);
    hipLaunchKernelGGL(k_gemm_nt<1>, grid, dim3(256), 0, s, W, ldw, X, ldx, xrow, Y, ldy, yrow, nbox, nout, K, alpha,
                       beta, xbs, ybs, ywide);
  }
}

}  // namespace kifmm
