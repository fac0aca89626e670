// HIP kernels of the kiFMM evaluate for gfx950 (CDNA4).
//
// Dense contractions run on the FP32 matrix cores: the check-to-equivalent
// factors, U2U, compression, post and D2D through v_mfma_f32_16x16x4_f32, the
// U2D translations (M2L) through v_mfma_f32_32x32x2_f32 (the split-bfloat16 M2L
// through v_mfma_f32_32x32x16_bf16 with FP32 accumulation).  The kernel sums
// (S2U check fields, D2T and the U-list direct sum) run on the vector ALUs.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace kifmm {

typedef float v16f __attribute__((ext_vector_type(16)));

// One 32x32x2 FP32 matrix-core step (wave64): lane (i, h) = (l % 32, l / 32)
// holds A[i][h] and B[h][i]; the accumulator holds D[8 (v / 4) + 4 h + v % 4][i]
// in element v.
__device__ __forceinline__ v16f mfma32(float a, float b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

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

// ----------------------------------------------------------------- M2L ---
// Compressed VLI over blocks.  A work item is (level, an aligned 4 x 4 x 4 block
// of parent boxes, target position o, source position o').  Its targets are the
// children at position o of the block's parents (up to 64); its sources are the
// children at position o' of the 6 x 6 x 6 parents around the block (216 rows,
// staged in LDS, missing boxes as zero rows).  Every V-list offset between such
// a target and source is a parent shift d in {-1,0,1}^3, i.e. a fixed row shift
// in the staged block, and the item computes for each target
//   chat_part[o'][target] = sum_{d} C_{t(o, o', d)} uhat[child o' of (parent + d)].
// The eight source positions' partial sums are added afterwards (k_sum_parts).
//
// Matrix-core mapping (v_mfma_f32_32x32x2_f32): one wave per 32 output rows,
// covering the 64 targets as two 32-column blocks.  The k dimension (padded
// with zeros to a multiple of 8) runs in "chunks" of 8: lane (i, h) = (l % 32,
// l / 32) loads A[i][8c + 4h .. +3] and B^T[j][8c + 4h .. +3] as float4 and the
// four MFMA steps contract k = 8c + 4h + r (the order of the sum over k is
// free).  Sources are staged in LDS in slabs of 40 k.  The operators are read
// from global memory (L2: the items of one (o, o') pair are dealt to one XCD),
// stored in lane order so that a wave's float4 loads of one chunk cover 1 KiB
// of contiguous memory; each chunk's operands are fetched two chunks ahead of
// their use.

struct M2LRegs {
  float4 a;
  float4 b[2];
  bool first;  // first chunk of a group of offsets in this slab
};

extern __shared__ float4 s_m2l[];  // [216][ld4] float4: the current k-slab of the staged sources

// A slab holds 4 (ld4 - 1) k of each staged row (a multiple of 8); the row
// stride ld4 is an odd number of float4, so lanes reading different rows
// spread over the LDS banks.

// The contribution of each group of kM2LFlush offsets over a slab is
// accumulated from zero and added into the running total when the next group
// starts: FP32 rounding then grows with the length of these short chains
// rather than with that of the whole sum (about 23 offsets x k terms, of both
// signs for signed charges).  Groups of 4 keep almost all of the gain of
// single offsets at a quarter of the vector-ALU cost.
constexpr int kM2LFlush = 4;

// Position (offset j, chunk c) in an item's sequence of 8-k chunks over one
// slab, with the offset's wave-uniform address parts.  Stepping past the end
// stays on the last chunk, so the loads it drives remain unconditional.
struct M2LCursor {
  int j, c, nch, noffs, ld4, po_reg;
  size_t core_stride, aoff;
  int sh;
  __device__ __forceinline__ void set_offset() {
    const int e = __builtin_amdgcn_readlane(po_reg, j);
    aoff = (size_t)(e & 511) * core_stride;
    sh = (e >> 9) * ld4;
  }
  __device__ __forceinline__ void next() {
    if (++c == nch) {
      if (j + 1 < noffs) {
        c = 0;
        ++j;
        set_offset();
      } else {
        c = nch - 1;
      }
    }
  }
};

// Operands of the cursor's chunk.  alane: this lane's float4 of the wave's row
// block in the slab's first chunk; bq[nb]: the float4 index of its target's
// staged row plus h.
__device__ __forceinline__ void m2l_load(M2LRegs& r, const float* __restrict__ alane, const int* bq,
                                         const M2LCursor& cu) {
  r.a = *reinterpret_cast<const float4*>(alane + cu.aoff + 256 * cu.c);
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) r.b[nb] = s_m2l[bq[nb] + cu.sh + 2 * cu.c];
  r.first = cu.c == 0 && cu.j % kM2LFlush == 0;
}

// Adds the group's accumulator into the running total and restarts it.
__device__ __forceinline__ void m2l_flush(v16f* acc, v16f* tot) {
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    tot[nb] += acc[nb];
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[nb][e] = 0.f;
  }
}

__device__ __forceinline__ void m2l_compute(const M2LRegs& r, v16f* acc, v16f* tot) {
  if (r.first) m2l_flush(acc, tot);
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) acc[nb] = mfma32(r.a.x, r.b[nb].x, acc[nb]);
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) acc[nb] = mfma32(r.a.y, r.b[nb].y, acc[nb]);
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) acc[nb] = mfma32(r.a.z, r.b[nb].z, acc[nb]);
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) acc[nb] = mfma32(r.a.w, r.b[nb].w, acc[nb]);
}

// All offsets of the item over one slab of nch chunks, with two register sets.
__device__ __forceinline__ void m2l_slab(v16f* acc, v16f* tot, const float* alane, size_t core_stride, int po_reg,
                                         int noffs, const int* bq, int nch, int ld4) {
  const int nv = noffs * nch;
  M2LCursor cu{0, 0, nch, noffs, ld4, po_reg, core_stride, 0, 0};
  cu.set_offset();
  M2LRegs r0, r1;
  m2l_load(r0, alane, bq, cu);
  cu.next();
  for (int v = 0; v < nv; v += 2) {
    m2l_load(r1, alane, bq, cu);
    cu.next();
    __builtin_amdgcn_sched_barrier(0);
    m2l_compute(r0, acc, tot);
    __builtin_amdgcn_sched_barrier(0);
    m2l_load(r0, alane, bq, cu);
    cu.next();
    __builtin_amdgcn_sched_barrier(0);
    if (v + 1 < nv) m2l_compute(r1, acc, tot);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// UPPER = 1 for the launch of the levels above the leaves that runs on a
// second stream beside the leaf level's (same code; a name of its own in traces).
template <int UPPER>
__global__ __launch_bounds__(512) void k_m2l(const float* __restrict__ cores, int core_rows, int ldk, int ld4,
                                             const M2LItem* __restrict__ items, const int* __restrict__ tgt_blk,
                                             const int* __restrict__ src_blk, const int* __restrict__ pair_offs,
                                             const float* __restrict__ uhat, float* __restrict__ chat_part,
                                             long long part_stride, long long rhs_stride) {
  const M2LItem it = items[blockIdx.x];
  uhat += blockIdx.y * rhs_stride;  // right-hand side blockIdx.y
  chat_part += blockIdx.y * rhs_stride;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;  // 32-row block of the output
  const int i32 = lane & 31, h = lane >> 5;

  int tslot[2], bq[2], bbase[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int pi = 32 * nb + i32;  // position in the 4x4x4 parent block, x fastest
    tslot[nb] = tgt_blk[it.tgt_base + pi];
    bbase[nb] = ((pi & 3) + 1) + 6 * (((pi >> 2) & 3) + 1) + 36 * ((pi >> 4) + 1) - 43;
    bq[nb] = bbase[nb] * ld4 + h;
  }
  v16f acc[2], tot[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[nb][e] = tot[nb][e] = 0.f;
  // offset table of the item in one VGPR (lane j holds entry j), read with readlane
  const int po_reg = pair_offs[it.pair * 27 + min(lane, 26)];
  // this lane's float4 in the wave's row block of the lane-ordered operators
  const float* ablk = cores + (size_t)wave * 32 * ldk + 4 * lane;
  const size_t core_stride = (size_t)core_rows * ldk;
  const int* srcs = src_blk + it.src_base;

  const int slab = 4 * (ld4 - 1);
  for (int k0 = 0; k0 < ldk; k0 += slab) {
    const int kw = min(slab, ldk - k0);  // slab width, a multiple of 8
    const int w4 = kw >> 2;
    if (k0) __syncthreads();  // previous slab fully consumed
    for (int idx = tid; idx < 216 * w4; idx += blockDim.x) {
      const int r = idx / w4, c4 = idx - r * w4;
      const int slot = srcs[r];
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (slot >= 0) v = *reinterpret_cast<const float4*>(uhat + (size_t)slot * ldk + k0 + 4 * c4);
      s_m2l[r * ld4 + c4] = v;
    }
    __syncthreads();
    m2l_slab(acc, tot, ablk + 32 * k0, core_stride, po_reg, it.noffs, bq, kw >> 3, ld4);
  }
  m2l_flush(acc, tot);
  // tot[nb][v]: row 32 wave + 8 (v / 4) + 4 h + v % 4, target column 32 nb + i32
  float* out = chat_part + (size_t)it.part * part_stride;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    if (tslot[nb] < 0) continue;
#pragma unroll
    for (int b4 = 0; b4 < 4; ++b4) {
      const int o = 32 * wave + 8 * b4 + 4 * h;
      if (o < ldk)
        *reinterpret_cast<float4*>(out + (size_t)tslot[nb] * ldk + o) =
            make_float4(tot[nb][4 * b4], tot[nb][4 * b4 + 1], tot[nb][4 * b4 + 2], tot[nb][4 * b4 + 3]);
    }
  }
}

bool m2l_supported(int row_blocks, int ldk, int lds_ld) {
  // lds_ld = slab + 4 floats, the slab a multiple of 8 k
  return row_blocks >= 1 && row_blocks <= 8 && (ldk & 7) == 0 && lds_ld >= 12 && ((lds_ld - 4) & 7) == 0 &&
         (size_t)216 * lds_ld * sizeof(float) <= kMaxDynamicLds;
}

bool launch_m2l(int row_blocks, const float* cores, int core_rows, int ldk, int lds_ld, const M2LItem* items,
                int nitems, const int* tgt_blk, const int* src_blk, const int* pair_offs, const float* uhat,
                float* chat_part, long long part_stride, int nrhs, long long rhs_stride, hipStream_t s, bool upper) {
  if (nitems <= 0 || nrhs <= 0) return true;
  if (!m2l_supported(row_blocks, ldk, lds_ld)) return false;
  const size_t lds = (size_t)216 * lds_ld * sizeof(float);
  const dim3 grid(nitems, nrhs), block(64 * row_blocks);
  if (upper)
    hipLaunchKernelGGL(k_m2l<1>, grid, block, lds, s, cores, core_rows, ldk, lds_ld / 4, items, tgt_blk, src_blk,
                       pair_offs, uhat, chat_part, part_stride, rhs_stride);
  else
    hipLaunchKernelGGL(k_m2l<0>, grid, block, lds, s, cores, core_rows, ldk, lds_ld / 4, items, tgt_blk, src_blk,
                       pair_offs, uhat, chat_part, part_stride, rhs_stride);
  return true;
}

// ------------------------------------------------------ M2L, gathered ---
// The compressed VLI with targets as columns, for one right-hand side: a group
// is up to 32 target boxes of one level and one position among siblings (hence
// one V-list offset set), and one wave per (group, 32-row block of C) walks the
// union of the group's offsets.  Per entry lane j gathers its own target's
// source row of uhat (a zero row where the target has no source at that offset)
// and the MFMA columns are the group's targets, so sparse trees, whose blocked
// items are mostly empty columns, keep full columns.  Operators in the lane
// order of k_m2l; chat written once per target (no partial sums); accumulators
// restarted every kM2LFlush entries (short FP32 chains).
template <int UPPER>  // as in k_m2l
__global__ __launch_bounds__(64) void k_m2l_gather(const float* __restrict__ cores, long long core_stride, int nch,
                                                   const int4* __restrict__ units, const int* __restrict__ ent_core,
                                                   const int* __restrict__ ent_src, const int* __restrict__ grp_tgt,
                                                   const float* __restrict__ uhat, float* __restrict__ chat, int ldk) {
  const int4 u = units[blockIdx.x];  // (group, row block, first entry, end entry)
  const int lane = threadIdx.x;
  const int j = lane & 31, h = lane >> 5;
  const float* alane = cores + (size_t)u.y * nch * 256 + 4 * lane;
  v16f acc, tot;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = tot[e] = 0.f;
  for (int e0 = u.z; e0 < u.w; e0 += kM2LFlush) {
    const int e1 = min(e0 + kM2LFlush, u.w);
    for (int e = e0; e < e1; ++e) {
      const float* ap = alane + (size_t)ent_core[e] * core_stride;
      const float* bp = uhat + (size_t)ent_src[(size_t)e * 32 + j] * ldk + 4 * h;
      float4 a = *reinterpret_cast<const float4*>(ap);
      float4 b = *reinterpret_cast<const float4*>(bp);
      for (int c = 0; c < nch; ++c) {
        const int cn = min(c + 1, nch - 1);  // next chunk (the last one repeats, unused)
        const float4 an = *reinterpret_cast<const float4*>(ap + 256 * cn);
        const float4 bn = *reinterpret_cast<const float4*>(bp + 8 * cn);
        acc = mfma32(a.x, b.x, acc);
        acc = mfma32(a.y, b.y, acc);
        acc = mfma32(a.z, b.z, acc);
        acc = mfma32(a.w, b.w, acc);
        a = an;
        b = bn;
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      tot[e] += acc[e];
      acc[e] = 0.f;
    }
  }
  const int tgt = grp_tgt[(size_t)u.x * 32 + j];
  if (tgt < 0) return;
  // tot[v]: row 32 u.y + 8 (v / 4) + 4 h + v % 4 of target column j
  float* out = chat + (size_t)tgt * ldk;
#pragma unroll
  for (int b4 = 0; b4 < 4; ++b4) {
    const int row = 32 * u.y + 8 * b4 + 4 * h;
    if (row < ldk)
      *reinterpret_cast<float4*>(out + row) = make_float4(tot[4 * b4], tot[4 * b4 + 1], tot[4 * b4 + 2], tot[4 * b4 + 3]);
  }
}

void launch_m2l_gather(const float* cores, long long core_stride, int ldk, const int4* units, int nunits,
                       const int* ent_core, const int* ent_src, const int* grp_tgt, const float* uhat, float* chat,
                       hipStream_t s, bool upper) {
  if (nunits <= 0) return;
  if (upper)
    hipLaunchKernelGGL(k_m2l_gather<1>, dim3(nunits), dim3(64), 0, s, cores, core_stride, ldk / 8, units, ent_core,
                       ent_src, grp_tgt, uhat, chat, ldk);
  else
    hipLaunchKernelGGL(k_m2l_gather<0>, dim3(nunits), dim3(64), 0, s, cores, core_stride, ldk / 8, units, ent_core,
                       ent_src, grp_tgt, uhat, chat, ldk);
}

// -------------------------------------------------- M2L, 32 right-hand sides ---
// The compressed VLI for 32 right-hand sides as wide products: per target box
// and V-list entry (offset t, source box), chat[:, target] += C_t uhat[:, source]
// with the 32 right-hand sides as the 32 columns of v_mfma_f32_32x32x2_f32.
// One wave per (target box, 32-row block of C) walks the target's V list.
// Operators are in the lane order of k_m2l; uhat is [box][k / 8][32][8], so
// that lane (j, h) reads B[8c + 4h .. +3][right-hand side j] as one float4 and
// a wave's read of one chunk is 1 KiB of contiguous memory.  No partial sums:
// the wave writes chat[r][target][rows] once.  The accumulators restart every
// kM2LFlush entries and are added into a running total (short FP32 chains).
__global__ __launch_bounds__(64) void k_m2l_wide(const float* __restrict__ cores, long long core_stride, int nch,
                                                 const int4* __restrict__ units, const int2* __restrict__ vlist,
                                                 const float* __restrict__ uhat, float* __restrict__ chat,
                                                 long long chat_rs, int ldk) {
  const int4 u = units[blockIdx.x];  // (target slot, row block, first entry, end entry)
  const int lane = threadIdx.x;
  const int j = lane & 31, h = lane >> 5;
  const float* alane = cores + (size_t)u.y * nch * 256 + 4 * lane;
  const float* blane = uhat + 8 * j + 4 * h;
  const size_t box_stride = (size_t)nch * 256;
  v16f acc, tot;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = tot[e] = 0.f;
  for (int e0 = u.z; e0 < u.w; e0 += kM2LFlush) {
    const int e1 = min(e0 + kM2LFlush, u.w);
    for (int e = e0; e < e1; ++e) {
      const int2 pr = vlist[e];
      const float* ap = alane + (size_t)pr.x * core_stride;
      const float* bp = blane + (size_t)pr.y * box_stride;
      float4 a = *reinterpret_cast<const float4*>(ap);
      float4 b = *reinterpret_cast<const float4*>(bp);
      for (int c = 0; c < nch; ++c) {
        const int cn = min(c + 1, nch - 1);  // next chunk (the last one repeats, unused)
        const float4 an = *reinterpret_cast<const float4*>(ap + 256 * cn);
        const float4 bn = *reinterpret_cast<const float4*>(bp + 256 * cn);
        acc = mfma32(a.x, b.x, acc);
        acc = mfma32(a.y, b.y, acc);
        acc = mfma32(a.z, b.z, acc);
        acc = mfma32(a.w, b.w, acc);
        a = an;
        b = bn;
      }
    }
    // a group of kM2LFlush entries: into the running total, restart
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      tot[e] += acc[e];
      acc[e] = 0.f;
    }
  }
  // tot[v]: row 32 u.y + 8 (v / 4) + 4 h + v % 4 of right-hand side j
  float* out = chat + j * chat_rs + (size_t)u.x * ldk;
#pragma unroll
  for (int b4 = 0; b4 < 4; ++b4) {
    const int row = 32 * u.y + 8 * b4 + 4 * h;
    if (row < ldk)
      *reinterpret_cast<float4*>(out + row) = make_float4(tot[4 * b4], tot[4 * b4 + 1], tot[4 * b4 + 2], tot[4 * b4 + 3]);
  }
}

void launch_m2l_wide(const float* cores, long long core_stride, int ldk, const int4* units, int nunits,
                     const int2* vlist, const float* uhat, float* chat, long long chat_rs, hipStream_t s) {
  if (nunits <= 0) return;
  hipLaunchKernelGGL(k_m2l_wide, dim3(nunits), dim3(64), 0, s, cores, core_stride, ldk / 8, units, vlist, uhat, chat,
                     chat_rs, ldk);
}

// ------------------------------------------------- M2L, split bfloat16 ---
// The same work items and staging as k_m2l, with every product of the
// translation computed from bfloat16 pieces on the matrix cores with FP32
// accumulation.  A value x is split into NP bfloat16 pieces, x_0 the bfloat16
// rounding of x and x_p that of x - x_0 - ... - x_{p-1}, so that the pieces hold
// 8 NP significant bits.  The products kept are those of pieces p of the
// operator and q of the source with p + q < NP, of order 2^-8 (p + q):
//   NP = 2: a0 b0 + a0 b1 + a1 b0                        (three passes, ~3 * 2^-16)
//   NP = 3: a0 b0 + a0 b1 + a1 b0 + a0 b2 + a1 b1 + a2 b0 (six passes,  ~2^-24)
// Operators are split once at plan creation; sources are split while they are
// staged in LDS.
//
// Matrix-core mapping (v_mfma_f32_32x32x16_bf16): one wave per 32 output rows,
// two 32-column target blocks, k in chunks of 16 (k padded with zeros to a
// multiple of 16).  Lane (i, h) holds A[i][16c + 8h .. +7] and
// B^T[j][16c + 8h .. +7] as 8 bfloat16 per piece; the accumulator layout is
// that of the FP32 kernel.  Per chunk a lane loads the NP operator pieces (16
// bytes each, global, in lane order) and the NP source pieces of both column
// blocks (LDS).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v16f mfma_bf16(const uint4& a, const uint4& b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

template <int NP>
struct M2LRegsB {
  uint4 a[NP];
  uint4 b[2][NP];
  bool first;  // first chunk of a group of offsets in this slab
};

// Staged sources, 16-byte units: a row holds, per group g of 8 k values of the
// slab, the NP pieces of those 8 values in units NP g .. NP g + NP - 1.
extern __shared__ uint4 s_m2lb[];

constexpr int kM2LSlabB = 32;  // k per LDS slab (two chunks); row stride 8 NP / 2 + 1 units, odd

template <int NP>
__device__ __forceinline__ void m2lb_load(M2LRegsB<NP>& r, const uint4* __restrict__ alane, const int* bq,
                                          const M2LCursor& cu) {
  const uint4* a = alane + cu.aoff + 64 * NP * cu.c;
#pragma unroll
  for (int p = 0; p < NP; ++p) r.a[p] = a[64 * p];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int p = 0; p < NP; ++p) r.b[nb][p] = s_m2lb[bq[nb] + cu.sh + 2 * NP * cu.c + p];
  r.first = cu.c == 0 && cu.j % kM2LFlush == 0;
}

template <int NP>
__device__ __forceinline__ void m2lb_compute(const M2LRegsB<NP>& r, v16f* acc, v16f* tot) {
  // (operator piece, source piece), largest terms first
  constexpr int kTerms = NP == 2 ? 3 : 6;
  constexpr int kPa[6] = {0, 0, 1, 0, 1, 2};
  constexpr int kPb[6] = {0, 1, 0, 2, 1, 0};
  // Short FP32 chains, as in k_m2l, for the three-piece form (whose products are as
  // accurate as FP32's); the two-piece form's error is that of its split, and the
  // registers of a second accumulator would cost it occupancy.
  if (NP == 3 && r.first) m2l_flush(acc, tot);
#pragma unroll
  for (int t = 0; t < kTerms; ++t)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) acc[nb] = mfma_bf16(r.a[kPa[t]], r.b[nb][kPb[t]], acc[nb]);
}

// All offsets of the item over one slab of nch chunks, with two register sets.
template <int NP>
__device__ __forceinline__ void m2lb_slab(v16f* acc, v16f* tot, const uint4* alane, size_t core_stride, int po_reg,
                                          int noffs, const int* bq, int nch, int ld16) {
  const int nv = noffs * nch;
  M2LCursor cu{0, 0, nch, noffs, ld16, po_reg, core_stride, 0, 0};
  cu.set_offset();
  M2LRegsB<NP> r0, r1;
  m2lb_load<NP>(r0, alane, bq, cu);
  cu.next();
  for (int v = 0; v < nv; v += 2) {
    m2lb_load<NP>(r1, alane, bq, cu);
    cu.next();
    __builtin_amdgcn_sched_barrier(0);
    m2lb_compute<NP>(r0, acc, tot);
    __builtin_amdgcn_sched_barrier(0);
    m2lb_load<NP>(r0, alane, bq, cu);
    cu.next();
    __builtin_amdgcn_sched_barrier(0);
    if (v + 1 < nv) m2lb_compute<NP>(r1, acc, tot);
    __builtin_amdgcn_sched_barrier(0);
  }
}

__device__ __forceinline__ uint32_t bf16_bits(__bf16 x) { return __builtin_bit_cast(uint16_t, x); }

// Eight FP32 values split into NP bfloat16 pieces each (piece p of value e in
// the low (e even) or high (e odd) half of word e / 2 of out[p]).  Each
// remainder x - x_0 - ... is exact in FP32.
template <int NP>
__device__ __forceinline__ void split8(const float4& u, const float4& v, uint4* out) {
  float x[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    uint32_t w[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const __bf16 h0 = (__bf16)x[2 * e], h1 = (__bf16)x[2 * e + 1];
      w[e] = bf16_bits(h0) | (bf16_bits(h1) << 16);
      x[2 * e] -= (float)h0;
      x[2 * e + 1] -= (float)h1;
    }
    out[p] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

template <int NP, int UPPER>  // UPPER as in k_m2l
__global__ __launch_bounds__(512) void k_m2l_bf16(const uint4* __restrict__ cores, size_t core_stride, int ldk,
                                                  int ld16, const M2LItem* __restrict__ items,
                                                  const int* __restrict__ tgt_blk, const int* __restrict__ src_blk,
                                                  const int* __restrict__ pair_offs, const float* __restrict__ uhat,
                                                  float* __restrict__ chat_part, long long part_stride,
                                                  long long rhs_stride) {
  const M2LItem it = items[blockIdx.x];
  uhat += blockIdx.y * rhs_stride;  // right-hand side blockIdx.y
  chat_part += blockIdx.y * rhs_stride;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;  // 32-row block of the output
  const int i32 = lane & 31, h = lane >> 5;
  const int nchunk = ldk >> 4;

  int tslot[2], bq[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int pi = 32 * nb + i32;  // position in the 4x4x4 parent block, x fastest
    tslot[nb] = tgt_blk[it.tgt_base + pi];
    const int bbase = ((pi & 3) + 1) + 6 * (((pi >> 2) & 3) + 1) + 36 * ((pi >> 4) + 1) - 43;
    bq[nb] = bbase * ld16 + NP * h;
  }
  v16f acc[2], tot[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[nb][e] = tot[nb][e] = 0.f;
  const int po_reg = pair_offs[it.pair * 27 + min(lane, 26)];
  // this lane's piece-0 unit in the wave's row block of the lane-ordered operators
  const uint4* ablk = cores + (size_t)wave * nchunk * 64 * NP + lane;
  const int* srcs = src_blk + it.src_base;

  for (int k0 = 0; k0 < ldk; k0 += kM2LSlabB) {
    const int kw = min(kM2LSlabB, ldk - k0);  // a multiple of 16
    const int ng = kw >> 3;                    // groups of 8 k
    if (k0) __syncthreads();
    for (int idx = tid; idx < 216 * ng; idx += blockDim.x) {
      const int r = idx / ng, g = idx - r * ng;
      const int slot = srcs[r];
      float4 u = make_float4(0.f, 0.f, 0.f, 0.f), v = u;
      if (slot >= 0) {
        const float4* src = reinterpret_cast<const float4*>(uhat + (size_t)slot * ldk + k0 + 8 * g);
        u = src[0];
        v = src[1];
      }
      uint4 pcs[NP];
      split8<NP>(u, v, pcs);
#pragma unroll
      for (int p = 0; p < NP; ++p) s_m2lb[r * ld16 + NP * g + p] = pcs[p];
    }
    __syncthreads();
    m2lb_slab<NP>(acc, tot, ablk + (size_t)(k0 >> 4) * 64 * NP, core_stride, po_reg, it.noffs, bq, kw >> 4, ld16);
  }
  m2l_flush(acc, tot);
  float* out = chat_part + (size_t)it.part * part_stride;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    if (tslot[nb] < 0) continue;
#pragma unroll
    for (int b4 = 0; b4 < 4; ++b4) {
      const int o = 32 * wave + 8 * b4 + 4 * h;
      if (o < ldk)
        *reinterpret_cast<float4*>(out + (size_t)tslot[nb] * ldk + o) =
            make_float4(tot[nb][4 * b4], tot[nb][4 * b4 + 1], tot[nb][4 * b4 + 2], tot[nb][4 * b4 + 3]);
    }
  }
}

int m2l_bf16_lds_ld16(int pieces) { return 4 * pieces + 1; }

bool m2l_bf16_supported(int pieces, int row_blocks, int ldk) {
  return row_blocks >= 1 && row_blocks <= 8 && (ldk & 15) == 0 && (pieces == 2 || pieces == 3) &&
         (size_t)216 * m2l_bf16_lds_ld16(pieces) * 16 <= kMaxDynamicLds;
}

bool launch_m2l_bf16(int pieces, int row_blocks, const uint16_t* cores, size_t core_stride16, int ldk, int lds_ld16,
                     const M2LItem* items, int nitems, const int* tgt_blk, const int* src_blk, const int* pair_offs,
                     const float* uhat, float* chat_part, long long part_stride, int nrhs, long long rhs_stride,
                     hipStream_t s, bool upper) {
  if (nitems <= 0 || nrhs <= 0) return true;
  if (!m2l_bf16_supported(pieces, row_blocks, ldk) || lds_ld16 < m2l_bf16_lds_ld16(pieces)) return false;
  const size_t lds = (size_t)216 * lds_ld16 * 16;
  const dim3 grid(nitems, nrhs), block(64 * row_blocks);
  const uint4* c = reinterpret_cast<const uint4*>(cores);
#define KIFMM_M2L_BF16(NP, UP)                                                                                     \
  hipLaunchKernelGGL((k_m2l_bf16<NP, UP>), grid, block, lds, s, c, core_stride16, ldk, lds_ld16, items, tgt_blk, \
                     src_blk, pair_offs, uhat, chat_part, part_stride, rhs_stride)
  if (pieces == 2) {
    if (upper) KIFMM_M2L_BF16(2, 1);
    else KIFMM_M2L_BF16(2, 0);
  } else {
    if (upper) KIFMM_M2L_BF16(3, 1);
    else KIFMM_M2L_BF16(3, 0);
  }
#undef KIFMM_M2L_BF16
  return true;
}

// Sum of the eight source positions' partial sums, in a fixed order:
// chat[i] = sum_p part[p][i] over n4 float4s.
__global__ void k_sum_parts(const float4* __restrict__ part, float4* __restrict__ chat, long long n4,
                            long long stride4) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n4) return;
  float4 acc = part[i];
#pragma unroll
  for (int p = 1; p < 8; ++p) {
    const float4 v = part[i + p * stride4];
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
    acc.w += v.w;
  }
  chat[i] = acc;
}

void launch_sum_parts(const float* part, float* chat, long long n, long long stride, hipStream_t s) {
  const long long n4 = n / 4;
  if (n4 <= 0) return;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(part), reinterpret_cast<float4*>(chat), n4, stride / 4);
}

// ----------------------------------------------------------------- VJP ---
// dL/dx_k = w_k grad f_s(x_k) + s_k grad f_w(x_k), elementwise over [n][3].
__global__ void k_vjp_combine(const float* __restrict__ s, const float* __restrict__ w, const float* __restrict__ fs,
                              const float* __restrict__ fw, float* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n) return;
  const int k = i / 3;
  out[i] = w[k] * fs[i] + s[k] * fw[i];
}

void launch_vjp_combine(const float* s, const float* w, const float* fs, const float* fw, float* out, int n,
                        hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_vjp_combine, dim3((3 * n + 255) / 256), dim3(256), 0, st, s, w, fs, fw, out, n);
}

// ------------------------------------------------------------- permute ---
// Sorted sources: pts[i].w = charges[order[i]] (xyz are set at plan creation).
__global__ void k_permute(float4* __restrict__ pts, const float* __restrict__ charges, const int* __restrict__ order,
                          int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pts[i].w = charges[order[i]];
}

void launch_permute(float4* pts, const float* charges, const int* order, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_permute, dim3((n + 255) / 256), dim3(256), 0, s, pts, charges, order, n);
}

// ----------------------------------------------------------------- P2M ---
// S2U, first half: field of each non-empty leaf's sources on its upward-check
// surface c + alpha_outer r S_m.  One wave per leaf; lane l owns the check
// points l, l + 64, ... (NR = ceil(n / 64) of them, in registers), and the
// sources are read uniformly by the whole wave, so that a source's position
// relative to the leaf centre is formed once for all of the lane's check
// points.  Geometry is relative to the leaf centre c = c_hi + c_lo (two
// floats), so rounding is relative to the box size rather than to |c|.
template <int NR>
__global__ __launch_bounds__(256) void k_p2m(const float4* __restrict__ pts, const int* __restrict__ start,
                                             const int* __restrict__ leaves, const float4* __restrict__ centers,
                                             const float* __restrict__ surf, int n, float alpha, float* __restrict__ q,
                                             int ldq, int nleaves) {
  // the leaf, and with it every source address, is wave-uniform: scalar loads
  const int leaf = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (leaf >= nleaves) return;
  const int lane = threadIdx.x & 63;
  const int slot = leaves[leaf];
  const float4 ch = centers[2 * slot], cl = centers[2 * slot + 1];
  const float sc = alpha * ch.w;
  const int s0 = start[slot], s1 = start[slot + 1];  // s1 > s0: the leaf is not empty
  float px[NR], py[NR], pz[NR], acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int m = min(lane + 64 * r, n - 1);  // lanes past n repeat the last point, not stored
    px[r] = sc * surf[3 * m];
    py[r] = sc * surf[3 * m + 1];
    pz[r] = sc * surf[3 * m + 2];
    acc[r] = 0.f;
  }
  // four sources per step, their loads issued together; past the end the last
  // source repeats with charge 0 (it lies inside the leaf, away from the check
  // surface, so its term is exactly 0)
  for (int j = s0; j < s1; j += 4) {
    float4 y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      y[u] = pts[min(j + u, s1 - 1)];
      if (j + u >= s1) y[u].w = 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float rx = (y[u].x - ch.x) - cl.x, ry = (y[u].y - ch.y) - cl.y, rz = (y[u].z - ch.z) - cl.z;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const float dx = px[r] - rx, dy = py[r] - ry, dz = pz[r] - rz;
        acc[r] += y[u].w * __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int m = lane + 64 * r;
    if (m < n) q[(size_t)slot * ldq + m] = acc[r];
  }
}

bool p2m_supported(int n) { return n >= 1 && n <= 768; }

bool launch_p2m(const float4* pts, const int* start, const int* leaves, const float4* centers, const float* surf, int n,
                float alpha, float* q, int ldq, int nleaves, hipStream_t s) {
  if (nleaves <= 0) return true;
  const dim3 grid((nleaves + 3) / 4);
  switch ((n + 63) / 64) {
#define KIFMM_P2M_CASE(R)                                                                                    \
  case R:                                                                                                    \
    hipLaunchKernelGGL(k_p2m<R>, grid, dim3(256), 0, s, pts, start, leaves, centers, surf, n, alpha, q, ldq, \
                       nleaves);                                                                             \
    break;
    KIFMM_P2M_CASE(1)
    KIFMM_P2M_CASE(2)
    KIFMM_P2M_CASE(3)
    KIFMM_P2M_CASE(4)
    KIFMM_P2M_CASE(5)
    KIFMM_P2M_CASE(6)
    KIFMM_P2M_CASE(7)
    KIFMM_P2M_CASE(8)
    KIFMM_P2M_CASE(9)
    KIFMM_P2M_CASE(10)
    KIFMM_P2M_CASE(11)
    KIFMM_P2M_CASE(12)
#undef KIFMM_P2M_CASE
    default:
      return false;  // more than 768 check points
  }
  return true;
}

// ----------------------------------------------------------------- P2P ---
// Fused D2T and ULI (Algorithm 1 steps 3b, 3c) for the leaves of one parent
// (up to 8 siblings) per workgroup, written straight to input order.
//
// The siblings' U lists together cover the 4 x 4 x 4 block of leaves around
// the parent; `blk` lists their slots (x fastest, -1 = none).  Their sources
// are staged once in LDS, each leaf's range padded to a multiple of 4 with
// zero-charge dummies at (FLT_MAX, FLT_MAX, FLT_MAX): r^2 overflows to +inf,
// rsqrt gives 0 and the dummy adds exactly zero.  Each thread owns one target
// and walks the 27 block entries around its own leaf, 4 sources per step.  Only
// the leaf's own entry can hold a source at zero distance, so only that loop
// tests r > 0.  D2T evaluates the downward-equivalent surface (alpha_outer r S_m
// relative to the leaf centre, density d[m]) as n more sources, in
// centre-relative coordinates.  A block whose padded sources exceed `cap` reads
// them from global memory instead.
//
// Dynamic LDS: [cap] float4 sources, [n] float4 surface points, [8 n] floats d.
//
// Four or five waves per workgroup (the plan's choice).  At 30.5 points per
// leaf a parent's siblings hold 244 targets on average (Poisson): 320 threads
// take nearly every parent in one pass, where 256 leave about a fifth of the
// workgroups a second pass on a few lanes while the workgroup keeps its LDS.
// Each target's sums do not depend on the choice.
extern __shared__ float4 s_p2p[];

__device__ __forceinline__ void p2p_pair(float xx, float xy, float xz, float4 y, float& phi, float& gx, float& gy,
                                         float& gz) {
  const float dx = xx - y.x, dy = xy - y.y, dz = xz - y.z;
  const float rinv = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
  const float qr = y.w * rinv;
  const float qr3 = qr * rinv * rinv;
  phi += qr;
  gx -= qr3 * dx;
  gy -= qr3 * dy;
  gz -= qr3 * dz;
}

__device__ __forceinline__ void p2p_pair_masked(float xx, float xy, float xz, float4 y, float& phi, float& gx,
                                                float& gy, float& gz) {
  const float dx = xx - y.x, dy = xy - y.y, dz = xz - y.z;
  const float r2 = dx * dx + dy * dy + dz * dz;
  const float rinv = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
  const float qr = y.w * rinv;
  const float qr3 = qr * rinv * rinv;
  phi += qr;
  gx -= qr3 * dx;
  gy -= qr3 * dy;
  gz -= qr3 * dz;
}

// FP32 partial sums over at most this many sources, added into FP64 totals: the
// sums over a leaf block's sources are long (hundreds of terms in dense leaves)
// and, for charges of both signs, cancel.
constexpr int kP2PChunk = 32;

struct Sum4 {
  double phi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  __device__ __forceinline__ void add(float p, float x, float y, float z) {
    phi += p;
    gx += x;
    gy += y;
    gz += z;
  }
};

// The pairs of one run of staged sources [a, b) (b - a a multiple of 4), eight
// per step and a last step of four, in order, in chunks of kP2PChunk sources.
template <bool MASKED>
__device__ __forceinline__ void p2p_run(const float4* src, int a, int b, const float4& x, Sum4& acc) {
  for (int c = a; c < b; c += kP2PChunk) {
    const int e = min(c + kP2PChunk, b);  // e - c is a multiple of 4
    float phi = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
    int j = c;
    for (; j + 8 <= e; j += 8) {
      float4 y[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) y[u] = src[j + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (MASKED) p2p_pair_masked(x.x, x.y, x.z, y[u], phi, gx, gy, gz);
        else p2p_pair(x.x, x.y, x.z, y[u], phi, gx, gy, gz);
      }
    }
    if (j < e) {
      float4 y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) y[u] = src[j + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (MASKED) p2p_pair_masked(x.x, x.y, x.z, y[u], phi, gx, gy, gz);
        else p2p_pair(x.x, x.y, x.z, y[u], phi, gx, gy, gz);
      }
    }
    acc.add(phi, gx, gy, gz);
  }
}

// MODE 0: fused near + far field; MODE 1: near field only, written in sorted
// order to `near` (phi, grad) for a later MODE 2 launch; MODE 2: far field only,
// added to `near` and written to input order.
template <int MODE>
__global__ __launch_bounds__(kP2PMaxThreads) void k_p2p(const float4* __restrict__ pts, const int* __restrict__ start,
                                             const int* __restrict__ blk, int group_slots, int cap,
                                             const float4* __restrict__ centers, const float* __restrict__ surf,
                                             int n, float alpha, const float* __restrict__ d, int ldd, int far,
                                             const int* __restrict__ order, float* __restrict__ pot,
                                             float* __restrict__ grad, float4* __restrict__ near) {
  constexpr bool kNear = MODE != 2;
  constexpr bool kFar = MODE != 1;
  float4* s_src = s_p2p;
  float4* s_de = s_p2p + cap;
  float* s_d = reinterpret_cast<float*>(s_p2p + cap + n);
  __shared__ int s_off[65];
  __shared__ int s_slot[64];
  __shared__ int s_cnt[64];
  __shared__ int s_cs[9];

  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int c0 = group_slots * g;  // first leaf slot of this parent

  if (kNear && tid < 64) {
    const int slot = blk[(size_t)g * 64 + tid];
    const int cnt = slot >= 0 ? start[slot + 1] - start[slot] : 0;
    int incl = (cnt + 3) & ~3;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o);
      if (tid >= o) incl += v;
    }
    s_slot[tid] = slot;
    s_cnt[tid] = cnt;
    s_off[tid + 1] = incl;
    if (tid == 0) s_off[0] = 0;
  }
  if (tid <= group_slots) s_cs[tid] = start[c0 + tid];
  __syncthreads();
  const int total = kNear ? s_off[64] : 0;
  const bool in_lds = total <= cap;
  if (kNear && in_lds) {
    const float big = 3.402823466e38f;
    for (int i = tid; i < total; i += (int)blockDim.x) {
      int lo = 0, hi = 64;  // entry e with s_off[e] <= i < s_off[e + 1]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_off[mid] <= i) lo = mid;
        else hi = mid;
      }
      const int r = i - s_off[lo];
      s_src[i] = r < s_cnt[lo] ? pts[start[s_slot[lo]] + r] : make_float4(big, big, big, 0.f);
    }
  }
  const float sc = alpha * centers[2 * c0].w;
  if (kFar && far) {
    for (int m = tid; m < n; m += (int)blockDim.x)
      s_de[m] = make_float4(sc * surf[3 * m], sc * surf[3 * m + 1], sc * surf[3 * m + 2], 0.f);
    for (int i = tid; i < group_slots * n; i += (int)blockDim.x) {
      const int o = i / n, m = i - o * n;
      s_d[o * n + m] = d[(size_t)(c0 + o) * ldd + m];
    }
  }
  __syncthreads();

  const int t0 = s_cs[0], t1 = s_cs[group_slots];
  for (int tb = t0; tb < t1; tb += (int)blockDim.x) {
    const int ti = tb + tid;
    if (ti >= t1) break;
    int o = 0;
    while (o + 1 < group_slots && s_cs[o + 1] <= ti) ++o;
    const float4 x = pts[ti];
    const int bx = 1 + (o & 1), by = 1 + ((o >> 1) & 1), bz = 1 + ((o >> 2) & 1);
    // Two-level summation: FP32 partial sums over at most kP2PChunk sources and per block
    // of 8 surface points, accumulated in FP64 (the sums cancel heavily).
    double aphi = 0.0, agx = 0.0, agy = 0.0, agz = 0.0;
    if (kNear) {
      // The three leaves dx = -1, 0, 1 of a (dy, dz) row are consecutive in the
      // x-fastest block order, so their staged sources form one run: nine runs
      // per target.  The run holding the target's own leaf tests r > 0.
      Sum4 acc;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
          const int e0 = (bx - 1) + 4 * (by + dy) + 16 * (bz + dz);
          const bool own = (dy == 0) & (dz == 0);
          if (in_lds) {
            const int a = s_off[e0], b = s_off[e0 + 3];  // b - a is a multiple of 4
            if (own)
              p2p_run<true>(s_src, a, b, x, acc);
            else
              p2p_run<false>(s_src, a, b, x, acc);
          } else {
            for (int dx = 0; dx < 3; ++dx) {
              const int slot = s_slot[e0 + dx];
              if (slot < 0) continue;
              const int a = start[slot], b = start[slot + 1];
              for (int c = a; c < b; c += kP2PChunk) {
                float phi = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
                const int e = min(c + kP2PChunk, b);
                if (own)
                  for (int j = c; j < e; ++j) p2p_pair_masked(x.x, x.y, x.z, pts[j], phi, gx, gy, gz);
                else
                  for (int j = c; j < e; ++j) p2p_pair(x.x, x.y, x.z, pts[j], phi, gx, gy, gz);
                acc.add(phi, gx, gy, gz);
              }
            }
          }
        }
      aphi = acc.phi;
      agx = acc.gx;
      agy = acc.gy;
      agz = acc.gz;
    } else {
      const float4 v = near[ti];
      aphi = v.x;
      agx = v.y;
      agy = v.z;
      agz = v.w;
    }
    if (kFar && far) {
      const float4 ch = centers[2 * (c0 + o)], cl = centers[2 * (c0 + o) + 1];
      const float xx = (x.x - ch.x) - cl.x, xy = (x.y - ch.y) - cl.y, xz = (x.z - ch.z) - cl.z;
      const float* dl = s_d + o * n;
      for (int m0 = 0; m0 < n; m0 += 8) {
        float phi = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
        const int m1 = min(m0 + 8, n);
        for (int m = m0; m < m1; ++m) {
          const float4 de = s_de[m];
          p2p_pair(xx, xy, xz, make_float4(de.x, de.y, de.z, dl[m]), phi, gx, gy, gz);
        }
        aphi += phi;
        agx += gx;
        agy += gy;
        agz += gz;
      }
    }
    if (MODE == 1) {
      near[ti] = make_float4((float)aphi, (float)agx, (float)agy, (float)agz);
    } else {
      const int oi = order[ti];
      if (pot) pot[oi] = (float)aphi;
      if (grad) {
        grad[3 * (size_t)oi] = (float)agx;
        grad[3 * (size_t)oi + 1] = (float)agy;
        grad[3 * (size_t)oi + 2] = (float)agz;
      }
    }
  }
}

size_t p2p_lds_bytes(int cap, int n) { return (size_t)cap * 16 + (size_t)n * 16 + (size_t)8 * n * 4; }

bool p2p_supported(int threads, int cap, int n) {
  return (threads == 256 || threads == kP2PMaxThreads) && cap >= 0 && p2p_lds_bytes(cap, n) <= kMaxDynamicLds;
}

bool launch_p2p(int mode, const float4* pts, const int* start, const int* blk, int ngroups, int group_slots, int cap,
                const float4* centers, const float* surf, int n, float alpha, const float* d, int ldd, int far,
                const int* order, float* pot, float* grad, float4* near, int threads, hipStream_t s) {
  if (ngroups <= 0) return true;
  if (!p2p_supported(threads, cap, n) || mode < 0 || mode > 2) return false;
  const int c = mode == 2 ? 0 : cap;
  const size_t lds = mode == 1 ? (size_t)cap * 16 : p2p_lds_bytes(c, n);  // near-only: sources alone
  const dim3 grid(ngroups), block(threads);
#define KIFMM_P2P(M)                                                                                            \
  hipLaunchKernelGGL(k_p2p<M>, grid, block, lds, s, pts, start, blk, group_slots, c, centers, surf, n, alpha, d, \
                     ldd, far, order, pot, grad, near)
  if (mode == 0) KIFMM_P2P(0);
  else if (mode == 1) KIFMM_P2P(1);
  else KIFMM_P2P(2);
#undef KIFMM_P2P
  return true;
}

// ---------------------------------------------------- leaf work queue ---
// Fused D2T and ULI (Algorithm 1 steps 3b, 3c) as a persistent kernel over a
// work queue of target tiles.  A tile is up to 64 consecutive targets of one
// leaf, one per lane, so all lanes of a wave share the tile's U list and D2T
// surface: every source is read at a wave-uniform address (scalar loads) and
// used by the whole wave, and loop bounds are wave-uniform.  Tiles are ordered
// longest first at plan creation; each wave takes its next tiles from a counter
// in device memory (cleared by k_clear_queue before the launch) until none is
// left, so the waves finish together on trees whose leaves hold very different
// numbers of points (points on a surface).
//
// The sums are those of k_p2p: the sources of each leaf in sorted order (a step
// past a leaf's end repeats its last source with charge zero, which adds exactly
// zero), FP32 partials over at most kP2PChunk sources and over 8 surface points,
// accumulated in FP64; the two kernels agree to FP32 rounding.  MODE as in k_p2p.
constexpr int kQueueGrab = 4;  // tiles a wave takes from its counter at a time

__global__ void k_clear_queue(int* queue, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) queue[i] = 0;
}

// Sources j .. j + 3 of a leaf range ending at b (clamped to b - 1).  The index
// is the same on every lane, but `lane0` (zero, opaque to the compiler) makes
// them vector loads: those complete in order, so a wait for one step's sources
// leaves the next step's loads in flight (scalar loads complete out of order,
// and a wait for any of them is a wait for all).
__device__ __forceinline__ void queue_load4(const float4* __restrict__ pts, int j, int b, int lane0, float4* y) {
#pragma unroll
  for (int u = 0; u < 4; ++u) y[u] = pts[min(j + u, b - 1) + lane0];
}

// The pairs of a target with the sources [a, b) of one leaf (a < b), four per step,
// the next step's sources loaded while this step's are used.  A source position at
// or past b (its load repeats the last source) gets charge zero and adds exactly
// nothing.
template <bool MASKED>
__device__ __forceinline__ void queue_leaf(const float4* __restrict__ pts, int a, int b, const float4& x, Sum4& acc) {
  int lane0;
  asm volatile("v_mov_b32 %0, 0" : "=v"(lane0));
  float4 y[4];
  queue_load4(pts, a, b, lane0, y);
  float phi = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
  for (int j = a; j < b; j += 4) {
    float4 yn[4];
    queue_load4(pts, j + 4, b, lane0, yn);  // past the end: unused
    __builtin_amdgcn_sched_barrier(0);  // the loads stay ahead of this step's arithmetic
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      float4 yu = y[u];
      if (j + u >= b) yu.w = 0.f;
      if (MASKED) p2p_pair_masked(x.x, x.y, x.z, yu, phi, gx, gy, gz);
      else p2p_pair(x.x, x.y, x.z, yu, phi, gx, gy, gz);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) y[u] = yn[u];
    if ((j - a + 4) % kP2PChunk == 0 || j + 4 >= b) {
      acc.add(phi, gx, gy, gz);
      phi = gx = gy = gz = 0.f;
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_leaf_queue(const float4* __restrict__ pts, const int* __restrict__ start,
                                                    const int4* __restrict__ tiles, int ntiles, int* queue,
                                                    const int* __restrict__ blk, int group_slots,
                                                    const float4* __restrict__ centers,
                                                    const float* __restrict__ surf, int n, float alpha,
                                                    const float* __restrict__ d, int ldd, int far,
                                                    const int* __restrict__ order, float* __restrict__ pot,
                                                    float* __restrict__ grad, float4* __restrict__ near) {
  constexpr bool kNear = MODE != 2;
  constexpr bool kFar = MODE != 1;
  // the downward-equivalent surface alpha r S_m of a leaf (every leaf has the same
  // half-width), staged once per workgroup as k_p2p stages it
  __shared__ float4 s_de[kMaxLeafSurface];
  // each wave's copy of its tile's downward-equivalent density (read by every lane)
  __shared__ float s_dens[4][kMaxLeafSurface];
  const int lane = threadIdx.x & 63;
  float* dens = s_dens[threadIdx.x >> 6];
  if (kFar && far) {
    const float sc = alpha * centers[0].w;
    for (int m = threadIdx.x; m < n; m += blockDim.x)
      s_de[m] = make_float4(sc * surf[3 * m], sc * surf[3 * m + 1], sc * surf[3 * m + 2], 0.f);
    __syncthreads();
  }
  // The tiles t = xcd + 8 i (i < n_x) belong to the workgroups of one XCD (the
  // hardware deals workgroups to the eight XCDs in turn), each XCD with a counter
  // of its own, so that eight counters share the atomic traffic.  A wave takes
  // tile i = its index among the XCD's waves first, then groups of kQueueGrab
  // tiles from the counter; every wave leaves once its group starts past n_x.
  const int xcd = blockIdx.x & 7;
  const int n_x = ntiles > xcd ? (ntiles - xcd + 7) / 8 : 0;
  const int waves_x = (int)(gridDim.x >> 3) * 4;  // the grid is a multiple of 8 workgroups
  int i = (int)(blockIdx.x >> 3) * 4 + (int)(threadIdx.x >> 6);
  int left = 1;
  for (;;) {
    if (left == 0) {
      int mine = 0;
      if (lane == 0) mine = atomicAdd(queue + 16 * xcd, 1);
      i = waves_x + kQueueGrab * __builtin_amdgcn_readfirstlane(mine);
      left = kQueueGrab;
    }
    if (i >= n_x) break;
    const int t = xcd + 8 * i;
    ++i;
    --left;
    const int4 tile = tiles[t];
    const int slot = tile.x, cnt = tile.z;
    const int ti = tile.y + min(lane, cnt - 1);
    const float4 x = pts[ti];
    const int g = slot / group_slots, o = slot - g * group_slots;
    const int bx = 1 + (o & 1), by = 1 + ((o >> 1) & 1), bz = 1 + ((o >> 2) & 1);
    double aphi = 0.0, agx = 0.0, agy = 0.0, agz = 0.0;
    if (kNear) {
      // the 27 leaves of the block around the tile's leaf; a leaf's sources four per
      // step, the next step's loaded while this one is used
      Sum4 acc;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
          const bool own = (dy == 0) & (dz == 0);
          for (int dx = -1; dx <= 1; ++dx) {
            const int ns = blk[(size_t)g * 64 + (bx + dx) + 4 * (by + dy) + 16 * (bz + dz)];
            if (ns < 0) continue;
            const int a = start[ns], b = start[ns + 1];
            if (a >= b) continue;
            if (own)
              queue_leaf<true>(pts, a, b, x, acc);
            else
              queue_leaf<false>(pts, a, b, x, acc);
          }
        }
      aphi = acc.phi;
      agx = acc.gx;
      agy = acc.gy;
      agz = acc.gz;
    } else {
      const float4 v = near[ti];
      aphi = v.x;
      agx = v.y;
      agy = v.z;
      agz = v.w;
    }
    if (kFar && far) {
      const float4 ch = centers[2 * slot], cl = centers[2 * slot + 1];
      const float xx = (x.x - ch.x) - cl.x, xy = (x.y - ch.y) - cl.y, xz = (x.z - ch.z) - cl.z;
      const float* dl = d + (size_t)slot * ldd;
      // the density through LDS: one coalesced load per 64 values instead of a
      // scalar load per value
      for (int m = lane; m < n; m += 64) dens[m] = dl[m];
      __builtin_amdgcn_wave_barrier();  // LDS accesses of one wave complete in order
      for (int m0 = 0; m0 < n; m0 += 8) {
        float phi = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
        const int m1 = min(m0 + 8, n);
        for (int m = m0; m < m1; ++m) {
          const float4 de = s_de[m];
          p2p_pair(xx, xy, xz, make_float4(de.x, de.y, de.z, dens[m]), phi, gx, gy, gz);
        }
        aphi += phi;
        agx += gx;
        agy += gy;
        agz += gz;
      }
    }
    if (lane < cnt) {
      if (MODE == 1) {
        near[ti] = make_float4((float)aphi, (float)agx, (float)agy, (float)agz);
      } else {
        const int oi = order[ti];
        if (pot) pot[oi] = (float)aphi;
        if (grad) {
          grad[3 * (size_t)oi] = (float)agx;
          grad[3 * (size_t)oi + 1] = (float)agy;
          grad[3 * (size_t)oi + 2] = (float)agz;
        }
      }
    }
  }
}

void launch_clear_queue(int* queue, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_queue, dim3(1), dim3(256), 0, s, queue, n);
}

bool launch_leaf_queue(int mode, const float4* pts, const int* start, const int4* tiles, int ntiles, int* queue,
                       int grid, const int* blk, int group_slots, const float4* centers, const float* surf, int n,
                       float alpha, const float* d, int ldd, int far, const int* order, float* pot, float* grad,
                       float4* near, hipStream_t s) {
  if (ntiles <= 0) return true;
  if (grid < 8 || (grid & 7) || mode < 0 || mode > 2) return false;
#define KIFMM_LEAF_QUEUE(M)                                                                                  \
  hipLaunchKernelGGL(k_leaf_queue<M>, dim3(grid), dim3(256), 0, s, pts, start, tiles, ntiles, queue, blk,  \
                     group_slots, centers, surf, n, alpha, d, ldd, far, order, pot, grad, near)
  if (mode == 0) KIFMM_LEAF_QUEUE(0);
  else if (mode == 1) KIFMM_LEAF_QUEUE(1);
  else KIFMM_LEAF_QUEUE(2);
#undef KIFMM_LEAF_QUEUE
  return true;
}

// ---------------------------------------------------- multi-RHS leaves ---
// R right-hand sides (R = 2, 4, ..., 32), potentials only.  Sorted charges are
// [N][R] (a point's R charges contiguous) and every leaf kernel runs one wave
// per leaf (or per 64 of its points) with the sources of a step common to the
// whole wave, so that a source's position and charges are wave-uniform loads
// and the geometry and reciprocal distance of a pair serve all R sums.

// qs[i][r] = charges[order[i]][r].
__global__ void k_permute_multi(float* __restrict__ qs, const float* __restrict__ charges,
                                const int* __restrict__ order, int n, int R) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * R) return;
  const long long p = i / R;
  qs[i] = charges[(long long)order[p] * R + (i - p * R)];
}

void launch_permute_multi(float* qs, const float* charges, const int* order, int n, int R, hipStream_t s) {
  const long long total = (long long)n * R;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_permute_multi, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, qs, charges, order, n,
                     R);
}

// S2U first half for R right-hand sides: q[r][slot][m] for the check points m
// (lanes) of one leaf per wave; sources in the leaf's order, centre-relative.
template <int R>
__global__ __launch_bounds__(256) void k_p2m_multi(const float4* __restrict__ pts, const float* __restrict__ qs,
                                                   const int* __restrict__ start, const int* __restrict__ leaves,
                                                   const float4* __restrict__ centers, const float* __restrict__ surf,
                                                   int n, float alpha, float* __restrict__ q, int ldq, long long qrs,
                                                   int nleaves) {
  const int leaf = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (leaf >= nleaves) return;
  const int lane = threadIdx.x & 63;
  const int slot = leaves[leaf];
  const float4 ch = centers[2 * slot], cl = centers[2 * slot + 1];
  const float sc = alpha * ch.w;
  const int s0 = start[slot], s1 = start[slot + 1];
  for (int m0 = 0; m0 < n; m0 += 64) {
    const int m = m0 + lane;
    const int mc = min(m, n - 1);  // lanes past n repeat the last point and store nothing
    const float px = sc * surf[3 * mc], py = sc * surf[3 * mc + 1], pz = sc * surf[3 * mc + 2];
    float acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.f;
#pragma unroll 1
    for (int j = s0; j < s1; ++j) {
      const float4 y = pts[j];
      const float dx = px - ((y.x - ch.x) - cl.x);
      const float dy = py - ((y.y - ch.y) - cl.y);
      const float dz = pz - ((y.z - ch.z) - cl.z);
      const float rinv = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
      const float* qj = qs + (size_t)j * R;
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += qj[r] * rinv;
    }
    if (m < n) {
      float* out = q + (size_t)slot * ldq + m;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        *out = acc[r];
        out += qrs;
      }
    }
  }
}

bool launch_p2m_multi(int R, const float4* pts, const float* qs, const int* start, const int* leaves,
                      const float4* centers, const float* surf, int n, float alpha, float* q, int ldq, long long qrs,
                      int nleaves, hipStream_t s) {
  if (nleaves <= 0) return true;
  const dim3 grid((nleaves + 3) / 4), block(256);
  switch (R) {
    case 2: hipLaunchKernelGGL(k_p2m_multi<2>, grid, block, 0, s, pts, qs, start, leaves, centers, surf, n, alpha, q, ldq, qrs, nleaves); return true;
    case 4: hipLaunchKernelGGL(k_p2m_multi<4>, grid, block, 0, s, pts, qs, start, leaves, centers, surf, n, alpha, q, ldq, qrs, nleaves); return true;
    case 8: hipLaunchKernelGGL(k_p2m_multi<8>, grid, block, 0, s, pts, qs, start, leaves, centers, surf, n, alpha, q, ldq, qrs, nleaves); return true;
    case 16: hipLaunchKernelGGL(k_p2m_multi<16>, grid, block, 0, s, pts, qs, start, leaves, centers, surf, n, alpha, q, ldq, qrs, nleaves); return true;
    case 32: hipLaunchKernelGGL(k_p2m_multi<32>, grid, block, 0, s, pts, qs, start, leaves, centers, surf, n, alpha, q, ldq, qrs, nleaves); return true;
    default: return false;
  }
}

// D2T + ULI for R right-hand sides, potentials, written to input order
// (pot[i][r]).  A task is up to 64 consecutive points of one leaf, one wave
// each; lanes are targets.  The leaf's 27 neighbours come from the 4 x 4 x 4
// leaf block of its parent group (as in k_p2p); the far field treats the n
// downward-equivalent points (centre-relative) as sources with densities
// d[r][slot][m], 4 consecutive m per load.  FP32 partial sums per source leaf
// and per 8 surface points are accumulated in FP64.
template <int R>
__global__ __launch_bounds__(256) void k_leaf_multi(const float4* __restrict__ pts, const float* __restrict__ qs,
                                                    const int* __restrict__ start, const int4* __restrict__ tasks,
                                                    int ntasks, const int* __restrict__ blk, int group_slots,
                                                    const float4* __restrict__ centers,
                                                    const float* __restrict__ surf, int n, float alpha,
                                                    const float* __restrict__ d, int ldd, long long drs, int far,
                                                    const int* __restrict__ order, float* __restrict__ pot) {
  const int t = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (t >= ntasks) return;
  const int lane = threadIdx.x & 63;
  const int4 task = tasks[t];
  const int slot = task.x, cnt = task.z;
  const int ti = start[slot] + task.y + min(lane, cnt - 1);
  const float4 x = pts[ti];
  const int g = slot / group_slots, o = slot - g * group_slots;
  const int bx = 1 + (o & 1), by = 1 + ((o >> 1) & 1), bz = 1 + ((o >> 2) & 1);
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int ns = blk[(size_t)g * 64 + (bx + dx) + 4 * (by + dy) + 16 * (bz + dz)];
        if (ns < 0) continue;
        const int a = start[ns], b = start[ns + 1];
        const bool self = ns == slot;
        float part[R];
#pragma unroll
        for (int r = 0; r < R; ++r) part[r] = 0.f;
        if (a < b) {
          // the next source's position and charges are fetched while this one is used
          float4 yn = pts[a];
          float qn[R];
#pragma unroll
          for (int r = 0; r < R; ++r) qn[r] = qs[(size_t)a * R + r];
          for (int j = a; j < b; ++j) {
            const float4 y = yn;
            float qj[R];
#pragma unroll
            for (int r = 0; r < R; ++r) qj[r] = qn[r];
            const int jn = min(j + 1, b - 1);
            yn = pts[jn];
#pragma unroll
            for (int r = 0; r < R; ++r) qn[r] = qs[(size_t)jn * R + r];
            const float ex = x.x - y.x, ey = x.y - y.y, ez = x.z - y.z;
            const float r2 = ex * ex + ey * ey + ez * ez;
            float rinv = __builtin_amdgcn_rsqf(r2);
            if (self) rinv = r2 > 0.f ? rinv : 0.f;  // the target itself
#pragma unroll
            for (int r = 0; r < R; ++r) part[r] += qj[r] * rinv;
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += part[r];
      }
  if (far) {
    const float4 ch = centers[2 * slot], cl = centers[2 * slot + 1];
    const float xx = (x.x - ch.x) - cl.x, xy = (x.y - ch.y) - cl.y, xz = (x.z - ch.z) - cl.z;
    const float sc = alpha * ch.w;
    const float* dl = d + (size_t)slot * ldd;
    for (int m0 = 0; m0 < n; m0 += 8) {
      float part[R];
#pragma unroll
      for (int r = 0; r < R; ++r) part[r] = 0.f;
#pragma unroll
      for (int h = 0; h < 8; h += 4) {
        // d rows are zero beyond n (padded to a multiple of 4); surface indices are clamped
        if (m0 + h >= n) break;
        float rinv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int mc = min(m0 + h + e, n - 1);
          const float fx = xx - sc * surf[3 * mc], fy = xy - sc * surf[3 * mc + 1], fz = xz - sc * surf[3 * mc + 2];
          rinv[e] = __builtin_amdgcn_rsqf(fx * fx + fy * fy + fz * fz);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const float4 dv = *reinterpret_cast<const float4*>(dl + r * drs + m0 + h);
          part[r] += dv.x * rinv[0];
          part[r] += dv.y * rinv[1];
          part[r] += dv.z * rinv[2];
          part[r] += dv.w * rinv[3];
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += part[r];
    }
  }
  if (lane < cnt) {
    float* out = pot + (size_t)order[ti] * R;
#pragma unroll
    for (int r = 0; r < R; ++r) out[r] = (float)acc[r];
  }
}

bool launch_leaf_multi(int R, const float4* pts, const float* qs, const int* start, const int4* tasks, int ntasks,
                       const int* blk, int group_slots, const float4* centers, const float* surf, int n, float alpha,
                       const float* d, int ldd, long long drs, int far, const int* order, float* pot, hipStream_t s) {
  if (ntasks <= 0) return true;
  const dim3 grid((ntasks + 3) / 4), block(256);
#define KIFMM_LEAF_MULTI(RR)                                                                                        \
  hipLaunchKernelGGL(k_leaf_multi<RR>, grid, block, 0, s, pts, qs, start, tasks, ntasks, blk, group_slots, centers, \
                     surf, n, alpha, d, ldd, drs, far, order, pot)
  switch (R) {
    case 2: KIFMM_LEAF_MULTI(2); return true;
    case 4: KIFMM_LEAF_MULTI(4); return true;
    case 8: KIFMM_LEAF_MULTI(8); return true;
    case 16: KIFMM_LEAF_MULTI(16); return true;
    case 32: KIFMM_LEAF_MULTI(32); return true;
    default: return false;
  }
#undef KIFMM_LEAF_MULTI
}

// Dynamic LDS limit of every kernel that stages data in LDS, for the current
// device.  Plans call this once per device (under a lock) before their first
// launch; the launchers then only check their sizes against kMaxDynamicLds.
hipError_t configure_kernels() {
  const void* kernels[] = {
      reinterpret_cast<const void*>(&k_m2l<0>),          reinterpret_cast<const void*>(&k_m2l<1>),
      reinterpret_cast<const void*>(&k_m2l_bf16<2, 0>), reinterpret_cast<const void*>(&k_m2l_bf16<2, 1>),
      reinterpret_cast<const void*>(&k_m2l_bf16<3, 0>), reinterpret_cast<const void*>(&k_m2l_bf16<3, 1>),
      reinterpret_cast<const void*>(&k_p2p<0>),          reinterpret_cast<const void*>(&k_p2p<1>),
      reinterpret_cast<const void*>(&k_p2p<2>)};
  for (const void* k : kernels) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynamicLds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace kifmm
