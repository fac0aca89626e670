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

// ------------------------------------------------ GEMM, 32 batch entries ---
// The same product for a batch of exactly 32 (the 32 right-hand sides), with
// the batch entries as the 32 columns of v_mfma_f32_32x32x2_f32: per box, the
// 32 entries' rows of X form the B operand, so that a chunk of W staged in LDS
// serves 32 x kR32Boxes columns and every X row is fetched once.  A workgroup
// is nrb waves (32-row blocks of W: rows o_base .. o_base + 32 nrb - 1) over
// kR32Boxes boxes; W is staged in LDS kR32Slab k at a time (row stride
// kR32Slab / 4 + 1 float4, odd), zero beyond nout and K.  Lane (j, h) = (l % 32,
// l / 32) reads A[row j][8c + 4h .. +3] from LDS and B[8c + 4h .. +3][entry j]
// (entry j's row of the box) from global memory; the accumulator of a box holds
// D[8 (v / 4) + 4 h + v % 4][entry j].  With ywide a lane's four outputs of one
// box are 16 contiguous bytes of a 1 KiB block.
// The X chunks go to two register sets that take turns, so that each chunk's
// loads are in flight while the previous chunk's products run (with one set
// refilled by a copy, the compiler waits for each load before the products).
// Past K (the upper half of a last 4-k chunk) a lane reads the row's last four
// values again, which meet zeros of the staged W.  At each slab the accumulators
// are added into running totals and restart, so that the FP32 chains are 16
// products long whatever K (the 16x16x4 kernel adds four k per step over the
// whole K); the totals' registers hold the kernel to five waves per SIMD.
constexpr int kR32Boxes = 2;
constexpr int kR32Slab = 32;  // four 8-k chunks: slab boundaries fall on even chunks

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_gemm_r32(const float* __restrict__ W, int ldw, const float* __restrict__ X,
                                                  int ldx, const int* __restrict__ xrow, float* __restrict__ Y,
                                                  int ldy, const int* __restrict__ yrow, int nbox, int nout, int K,
                                                  float alpha, int beta, long long xbs, long long ybs, int ywide) {
  extern __shared__ float4 s_wr[];  // [32 nrb][kR32Slab / 4 + 1]
  constexpr int ld4 = kR32Slab / 4 + 1;
  const int nrb = blockDim.x >> 6;
  const int o_base = blockIdx.y * 32 * nrb;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = lane & 31, h = lane >> 5;
  const int b0 = blockIdx.x * kR32Boxes;
  const float* xp[kR32Boxes];  // entry j's row of each box
#pragma unroll
  for (int bb = 0; bb < kR32Boxes; ++bb) {
    const int b = min(b0 + bb, nbox - 1);
    xp[bb] = X + j * xbs + (size_t)(xrow ? xrow[b] : b) * ldx;
  }
  v16f acc[kR32Boxes], tot[kR32Boxes];
#pragma unroll
  for (int bb = 0; bb < kR32Boxes; ++bb)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[bb][e] = tot[bb][e] = 0.f;
  auto flush = [&]() {
#pragma unroll
    for (int bb = 0; bb < kR32Boxes; ++bb)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        tot[bb][e] += acc[bb][e];
        acc[bb][e] = 0.f;
      }
  };
  const int nch_all = (K + 7) >> 3;  // 8-k chunks over the whole K (the last may hold 4)
  auto load_b = [&](float4* b, int g) {
    const int k = min(8 * g + 4 * h, K - 4);  // this lane's first k of chunk g
#pragma unroll
    for (int bb = 0; bb < kR32Boxes; ++bb) b[bb] = *reinterpret_cast<const float4*>(xp[bb] + k);
  };
  auto stage = [&](int slab) {
    const int k0 = slab * kR32Slab;
    const int kw = min(kR32Slab, K - k0);  // a multiple of 4
    const int w4 = ((kw + 7) >> 3) * 2;    // float4 columns staged (whole chunks)
    if (slab) __syncthreads();             // the previous slab fully read
    for (int idx = threadIdx.x; idx < 32 * nrb * w4; idx += blockDim.x) {
      const int r = idx / w4, c4 = idx - r * w4;
      const int o = o_base + r;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (o < nout && 4 * c4 < kw) v = *reinterpret_cast<const float4*>(W + (size_t)o * ldw + k0 + 4 * c4);
      s_wr[r * ld4 + c4] = v;
    }
    __syncthreads();
  };
  const float4* arow = s_wr + (32 * wave + j) * ld4 + h;
  auto compute = [&](const float4* b, int g) {
    const float4 a = arow[2 * (g & 3)];
#pragma unroll
    for (int bb = 0; bb < kR32Boxes; ++bb) {
      acc[bb] = mfma32(a.x, b[bb].x, acc[bb]);
      acc[bb] = mfma32(a.y, b[bb].y, acc[bb]);
      acc[bb] = mfma32(a.z, b[bb].z, acc[bb]);
      acc[bb] = mfma32(a.w, b[bb].w, acc[bb]);
    }
  };
  float4 bA[kR32Boxes], bB[kR32Boxes];
  load_b(bA, 0);
  int g = 0;
  for (; g + 1 < nch_all; g += 2) {
    if ((g & 3) == 0) {
      if (g) flush();
      stage(g >> 2);
    }
    load_b(bB, g + 1);
    __builtin_amdgcn_sched_barrier(0);
    compute(bA, g);
    __builtin_amdgcn_sched_barrier(0);
    load_b(bA, g + 2);
    __builtin_amdgcn_sched_barrier(0);
    compute(bB, g + 1);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (g < nch_all) {
    if ((g & 3) == 0) {
      if (g) flush();
      stage(g >> 2);
    }
    compute(bA, g);
  }
#pragma unroll
  for (int bb = 0; bb < kR32Boxes; ++bb)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[bb][e] += tot[bb][e];
  const int ob = o_base + 32 * wave;
#pragma unroll
  for (int bb = 0; bb < kR32Boxes; ++bb) {
    const int b = b0 + bb;
    if (b >= nbox) continue;
    const int r = yrow ? yrow[b] : b;
#pragma unroll
    for (int b4 = 0; b4 < 4; ++b4) {
      const int o = ob + 8 * b4 + 4 * h;
      if (o >= nout) continue;
      float* yp = ywide ? Y + (((size_t)r * (nout >> 3) + (o >> 3)) * 32 + j) * 8 + (o & 7)
                        : Y + j * ybs + (size_t)r * ldy + o;
      float4 v = make_float4(alpha * acc[bb][4 * b4], alpha * acc[bb][4 * b4 + 1], alpha * acc[bb][4 * b4 + 2],
                             alpha * acc[bb][4 * b4 + 3]);
      if (beta) {
        const float4 old = *reinterpret_cast<const float4*>(yp);
        v.x += old.x;
        v.y += old.y;
        v.z += old.z;
        v.w += old.w;
      }
      *reinterpret_cast<float4*>(yp) = v;
    }
  }
}

size_t gemm_r32_lds_bytes(int nrb) { return (size_t)32 * nrb * (kR32Slab / 4 + 1) * 16; }

void launch_gemm_nt(const float* W, int ldw, const float* X, int ldx, const int* xrow, float* Y, int ldy,
                    const int* yrow, int nbox, int nout, int K, float alpha, int beta, hipStream_t s, int batch,
                    long long xbs, long long ybs, int ywide) {
  if (nbox <= 0 || batch <= 0) return;
  if (batch == 32) {
    // row blocks of 32 outputs, at most 8 per workgroup, spread evenly over the row tiles
    const int rb_all = (nout + 31) / 32;
    const int tiles = (rb_all + 7) / 8;
    const int nrb = (rb_all + tiles - 1) / tiles;
    hipLaunchKernelGGL(k_gemm_r32, dim3((nbox + kR32Boxes - 1) / kR32Boxes, tiles), dim3(64 * nrb),
                       gemm_r32_lds_bytes(nrb), s, W, ldw, X, ldx, xrow, Y, ldy, yrow, nbox, nout, K, alpha, beta,
                       xbs, ybs, ywide);
    return;
  }
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

// Dynamic LDS limit of the 32-entry GEMM on the current device (see
// configure_kernels).
hipError_t configure_gemm_kernels() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_r32), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kMaxDynamicLds);
}

}  // namespace kifmm
