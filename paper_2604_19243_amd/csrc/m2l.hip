// The compressed U2D translations (M2L, VLI) of the kiFMM evaluate on the
// gfx950 matrix cores: blocked FP32 (v_mfma_f32_32x32x2_f32), gathered FP32,
// 32 right-hand sides as columns, and split bfloat16 (v_mfma_f32_32x32x16_bf16
// with FP32 accumulation); and the sum of the blocked forms' partial sums.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "mfma.hpp"

namespace kifmm {

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

// Operands of the cursor's chunk.  ablk: the wave's row block of the operators
// in the slab's first chunk (wave-uniform: a buffer load's base, the lane's
// float4 at byte 16 lane); bq[nb]: the float4 index of its target's staged row
// plus h.
__device__ __forceinline__ void m2l_load(M2LRegs& r, const float* __restrict__ ablk, const int* bq,
                                         const M2LCursor& cu) {
  r.a = bload(buf_rsrc(ablk + cu.aoff), 16 * (int)(threadIdx.x & 63) + 1024 * cu.c);
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
__device__ __forceinline__ void m2l_slab(v16f* acc, v16f* tot, const float* ablk, size_t core_stride, int po_reg,
                                         int noffs, const int* bq, int nch, int ld4) {
  const int nv = noffs * nch;
  M2LCursor cu{0, 0, nch, noffs, ld4, po_reg, core_stride, 0, 0};
  cu.set_offset();
  M2LRegs r0, r1;
  m2l_load(r0, ablk, bq, cu);
  cu.next();
  for (int v = 0; v < nv; v += 2) {
    m2l_load(r1, ablk, bq, cu);
    cu.next();
    __builtin_amdgcn_sched_barrier(0);
    m2l_compute(r0, acc, tot);
    __builtin_amdgcn_sched_barrier(0);
    m2l_load(r0, ablk, bq, cu);
    cu.next();
    __builtin_amdgcn_sched_barrier(0);
    if (v + 1 < nv) m2l_compute(r1, acc, tot);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Staging of one k-slab of an item's 216 source rows into LDS.  The rows' box
// slots (-1 for none) are read once per item into s_src.  Each thread takes a
// fixed column unit of the slab and every rpp-th row, and issues the global
// loads of kStageBatch rows before it waits for any of them (a missing box
// reads row 0 and stores zeros), so that a slab costs a few memory latencies
// rather than one dependent pair of loads per row.
constexpr int kStageBatch = 8;

__device__ __forceinline__ void m2l_load_src(int* s_src, const int* __restrict__ srcs) {
  for (int r = threadIdx.x; r < 216; r += blockDim.x) s_src[r] = srcs[r];
  __syncthreads();
}

// units: column units per row in this slab; load(slot, u) returns unit u of the
// row of box slot; store(r, u, v) writes it to LDS.
template <int B, typename Load, typename Store>
__device__ __forceinline__ void m2l_stage(const int* s_src, int units, Load load, Store store) {
  const int rpp = blockDim.x / units;  // rows per pass
  const int r0 = threadIdx.x / units, u = threadIdx.x - r0 * units;
  if (r0 >= rpp) return;
  for (int rb = r0; rb < 216; rb += B * rpp) {
    decltype(load(0, 0)) v[B];
#pragma unroll
    for (int j = 0; j < B; ++j) v[j] = load(max(s_src[min(rb + j * rpp, 215)], 0), u);
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int r = rb + j * rpp;
      if (r < 216) store(r, u, v[j], s_src[r] >= 0);
    }
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
  // the wave's row block of the lane-ordered operators (buffer-load base)
  const float* ablk = cores + (size_t)__builtin_amdgcn_readfirstlane(wave) * 32 * ldk;
  const size_t core_stride = (size_t)core_rows * ldk;
  __shared__ int s_src[216];
  m2l_load_src(s_src, src_blk + it.src_base);

  const int slab = 4 * (ld4 - 1);
  for (int k0 = 0; k0 < ldk; k0 += slab) {
    const int kw = min(slab, ldk - k0);  // slab width, a multiple of 8
    if (k0) __syncthreads();  // previous slab fully consumed
    m2l_stage<kStageBatch>(
        s_src, kw >> 2,
        [&](int slot, int c4) { return *reinterpret_cast<const float4*>(uhat + (size_t)slot * ldk + k0 + 4 * c4); },
        [&](int r, int c4, float4 v, bool live) { s_m2l[r * ld4 + c4] = live ? v : make_float4(0.f, 0.f, 0.f, 0.f); });
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
// restarted every kM2LFlush entries (short FP32 chains).  The chunk steps of all
// entries form one sequence with two register sets taking turns, each step's
// loads in flight while the previous step's products run.
// Position (entry e, 8-k chunk c) in a unit's sequence of chunk steps: the
// entry's core (wave-uniform) and this lane's source row, and the next entry's,
// loaded when the cursor enters an entry.  Past the end it stays on the last chunk.
struct GatherCursor {
  int e, c, end, nch;
  int core, ncore, src, nsrc;
  const int* ent_core;
  const int* ent_src;
  int j;
  __device__ __forceinline__ void fetch_next() {
    const int e2 = min(e + 1, end - 1);
    ncore = ent_core[e2];
    nsrc = ent_src[(size_t)e2 * 32 + j];
  }
  __device__ __forceinline__ void next() {
    if (++c == nch) {
      if (e + 1 < end) {
        c = 0;
        ++e;
        core = ncore;
        src = nsrc;
        fetch_next();
      } else {
        c = nch - 1;
      }
    }
  }
};

struct GatherRegs {
  float4 a, b;
  bool first;
};

template <int UPPER>  // as in k_m2l
__global__ __launch_bounds__(64) void k_m2l_gather(const float* __restrict__ cores, long long core_stride, int nch,
                                                   const int4* __restrict__ units, const int* __restrict__ ent_core,
                                                   const int* __restrict__ ent_src, const int* __restrict__ grp_tgt,
                                                   const float* __restrict__ uhat, float* __restrict__ chat, int ldk) {
  const int4 u = units[blockIdx.x];  // (group, row block, first entry, end entry)
  const int lane = threadIdx.x;
  const int j = lane & 31, h = lane >> 5;
  const float* ablk = cores + (size_t)u.y * nch * 256;
  const float* blane = uhat + 4 * h;
  v16f acc, tot;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = tot[e] = 0.f;
  if (u.z < u.w) {
    GatherCursor cu{u.z, 0, u.w, nch, ent_core[u.z], 0, ent_src[(size_t)u.z * 32 + j], 0, ent_core, ent_src, j};
    cu.fetch_next();
    auto load = [&](GatherRegs& r) {
      r.a = bload(buf_rsrc(ablk + (size_t)cu.core * core_stride), 16 * lane + 1024 * cu.c);
      r.b = *reinterpret_cast<const float4*>(blane + (size_t)cu.src * ldk + 8 * cu.c);
      r.first = cu.c == 0 && (cu.e - u.z) % kM2LFlush == 0;
    };
    auto compute = [&](const GatherRegs& r) {
      if (r.first) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          tot[e] += acc[e];
          acc[e] = 0.f;
        }
      }
      acc = mfma32(r.a.x, r.b.x, acc);
      acc = mfma32(r.a.y, r.b.y, acc);
      acc = mfma32(r.a.z, r.b.z, acc);
      acc = mfma32(r.a.w, r.b.w, acc);
    };
    const int nv = (u.w - u.z) * nch;
    GatherRegs r0, r1;
    load(r0);
    cu.next();
    int v = 0;
    for (; v + 1 < nv; v += 2) {
      load(r1);
      cu.next();
      __builtin_amdgcn_sched_barrier(0);
      compute(r0);
      __builtin_amdgcn_sched_barrier(0);
      load(r0);
      cu.next();
      __builtin_amdgcn_sched_barrier(0);
      compute(r1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (v < nv) compute(r0);
#pragma unroll
    for (int e = 0; e < 16; ++e) tot[e] += acc[e];
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
// * Two targets of one level and one position among siblings (neighbours in
//   Morton order, so their V lists hold many of the same offsets) share a
//   workgroup.  Its entries come in three runs: the offsets both targets have
//   (one fetch of C_t's chunk serves both products), then those of the first
//   target alone, then those of the second alone.  Each run is a loop with one
//   fixed set of products, so the accumulators stay in place across entries.
// * The workgroup's waves are the 32-row blocks of C, walking the same entries
//   in the same order, so that each uhat chunk is fetched once for all of them.
// * Within a run the chunk steps of successive entries form one sequence; two
//   register sets take turns, so each step's loads are in flight while the
//   previous step's products run.  The loads are buffer loads (the base of an
//   operator's row block or of a source box in the resource, so offsets stay
//   within a few KiB).
// Operators are in the lane order of k_m2l; uhat is [box][k / 8][32][8], so
// that lane (j, h) reads B[8c + 4h .. +3][right-hand side j] as one float4 and
// a wave's read of one chunk is 1 KiB of contiguous memory.  No partial sums:
// each wave writes chat[r][target][rows] once per target.  The accumulators
// restart every kM2LFlush entries of a run and are added into running totals
// (short FP32 chains).

__device__ __forceinline__ void wide_store(const v16f& tot, float* chat, long long chat_rs, int slot, int rb, int ldk,
                                           int j, int h) {
  // tot[v]: row 32 rb + 8 (v / 4) + 4 h + v % 4 of right-hand side j
  float* out = chat + j * chat_rs + (size_t)slot * ldk;
#pragma unroll
  for (int b4 = 0; b4 < 4; ++b4) {
    const int row = 32 * rb + 8 * b4 + 4 * h;
    if (row < ldk)
      *reinterpret_cast<float4*>(out + row) = make_float4(tot[4 * b4], tot[4 * b4 + 1], tot[4 * b4 + 2], tot[4 * b4 + 3]);
  }
}

// Position (entry e, 8-k chunk c) in a run's sequence of chunk steps, with
// the entry's fields and the next entry's.  Stepping past the end stays on the
// last chunk, so the loads it drives remain unconditional.
struct WideCursor {
  int e, c, end, nch;
  int4 en, nx;
  const int4* ents;
  __device__ __forceinline__ void next() {
    if (++c == nch) {
      if (e + 1 < end) {
        c = 0;
        ++e;
        en = nx;
        nx = ents[min(e + 1, end - 1)];
      } else {
        c = nch - 1;
      }
    }
  }
};

struct WideRegs {
  float4 a, b0, b1;
  bool first;
};

struct WideCtx {
  const float* ablk;   // the wave's row block of core 0
  const float* uhat;
  size_t core_stride, box_stride;
  int oa, ob;          // the lane's byte offsets in an operator chunk and in a source chunk
};

// P: 0 both targets, 1 target 0 only, 2 target 1 only.
template <int P>
__device__ __forceinline__ void wide_load(WideRegs& r, const WideCtx& x, int e0, const WideCursor& cu) {
  r.a = bload(buf_rsrc(x.ablk + (size_t)cu.en.x * x.core_stride), x.oa + 1024 * cu.c);
  if (P != 2) r.b0 = bload(buf_rsrc(x.uhat + (size_t)cu.en.y * x.box_stride), x.ob + 1024 * cu.c);
  if (P != 1) r.b1 = bload(buf_rsrc(x.uhat + (size_t)cu.en.z * x.box_stride), x.ob + 1024 * cu.c);
  r.first = cu.c == 0 && (cu.e - e0) % kM2LFlush == 0;
}

template <int P>
__device__ __forceinline__ void wide_compute(const WideRegs& r, v16f& acc0, v16f& acc1, v16f& tot0, v16f& tot1) {
  if (r.first) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      tot0[e] += acc0[e];
      tot1[e] += acc1[e];
      acc0[e] = acc1[e] = 0.f;
    }
  }
  if (P == 0) {
    acc0 = mfma32(r.a.x, r.b0.x, acc0);
    acc1 = mfma32(r.a.x, r.b1.x, acc1);
    acc0 = mfma32(r.a.y, r.b0.y, acc0);
    acc1 = mfma32(r.a.y, r.b1.y, acc1);
    acc0 = mfma32(r.a.z, r.b0.z, acc0);
    acc1 = mfma32(r.a.z, r.b1.z, acc1);
    acc0 = mfma32(r.a.w, r.b0.w, acc0);
    acc1 = mfma32(r.a.w, r.b1.w, acc1);
  } else if (P == 1) {
    acc0 = mfma32(r.a.x, r.b0.x, acc0);
    acc0 = mfma32(r.a.y, r.b0.y, acc0);
    acc0 = mfma32(r.a.z, r.b0.z, acc0);
    acc0 = mfma32(r.a.w, r.b0.w, acc0);
  } else {
    acc1 = mfma32(r.a.x, r.b1.x, acc1);
    acc1 = mfma32(r.a.y, r.b1.y, acc1);
    acc1 = mfma32(r.a.z, r.b1.z, acc1);
    acc1 = mfma32(r.a.w, r.b1.w, acc1);
  }
}

// The chunk steps of the run of entries [e0, e1), all of kind P, two register
// sets taking turns: each step's loads are issued one step ahead of its
// products, across entry boundaries.  The accumulators restart every
// kM2LFlush entries.
template <int P>
__device__ __forceinline__ void wide_run(const WideCtx& x, const int4* ents, int e0, int e1, int nch, v16f& acc0,
                                         v16f& acc1, v16f& tot0, v16f& tot1) {
  if (e0 >= e1) return;
  const int nv = (e1 - e0) * nch;
  WideCursor cu{e0, 0, e1, nch, ents[e0], ents[min(e0 + 1, e1 - 1)], ents};
  WideRegs r0, r1;
  wide_load<P>(r0, x, e0, cu);
  cu.next();
  int v = 0;
  for (; v + 1 < nv; v += 2) {
    wide_load<P>(r1, x, e0, cu);
    cu.next();
    __builtin_amdgcn_sched_barrier(0);
    wide_compute<P>(r0, acc0, acc1, tot0, tot1);
    __builtin_amdgcn_sched_barrier(0);
    wide_load<P>(r0, x, e0, cu);
    cu.next();
    __builtin_amdgcn_sched_barrier(0);
    wide_compute<P>(r1, acc0, acc1, tot0, tot1);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (v < nv) wide_compute<P>(r0, acc0, acc1, tot0, tot1);
}

__global__ __launch_bounds__(512) void k_m2l_wide(const float* __restrict__ cores, long long core_stride, int nch,
                                                  const int4* __restrict__ units, const int4* __restrict__ ents,
                                                  const float* __restrict__ uhat, float* __restrict__ chat,
                                                  long long chat_rs, int ldk) {
  // units[2 b]: (slot of target 0, slot of target 1 or -1, first entry, end entry);
  // units[2 b + 1]: (end of the entries of both targets, end of those of target 0 alone, 0, 0),
  // then those of target 1 alone up to the end.  Wave = row block.
  const int4 u = units[2 * blockIdx.x];
  const int4 sg = units[2 * blockIdx.x + 1];
  const int rb = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int j = lane & 31, h = lane >> 5;
  const WideCtx x{cores + (size_t)rb * nch * 256, uhat, (size_t)core_stride, (size_t)nch * 256, 16 * lane,
                  4 * (8 * j + 4 * h)};
  v16f acc0, acc1, tot0, tot1;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc0[e] = acc1[e] = tot0[e] = tot1[e] = 0.f;
  wide_run<0>(x, ents, u.z, sg.x, nch, acc0, acc1, tot0, tot1);
  wide_run<1>(x, ents, sg.x, sg.y, nch, acc0, acc1, tot0, tot1);
  wide_run<2>(x, ents, sg.y, u.w, nch, acc0, acc1, tot0, tot1);
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    tot0[e] += acc0[e];
    tot1[e] += acc1[e];
  }
  wide_store(tot0, chat, chat_rs, u.x, rb, ldk, j, h);
  if (u.y >= 0) wide_store(tot1, chat, chat_rs, u.y, rb, ldk, j, h);
}

bool launch_m2l_wide(int row_blocks, const float* cores, long long core_stride, int ldk, const int4* units,
                     int nunits, const int4* ents, const float* uhat, float* chat, long long chat_rs, hipStream_t s) {
  if (nunits <= 0) return true;
  if (row_blocks < 1 || row_blocks > 8) return false;
  hipLaunchKernelGGL(k_m2l_wide, dim3(nunits), dim3(64 * row_blocks), 0, s, cores, core_stride, ldk / 8, units, ents,
                     uhat, chat, chat_rs, ldk);
  return true;
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
__device__ __forceinline__ void m2lb_load(M2LRegsB<NP>& r, const uint4* __restrict__ ablk, const int* bq,
                                          const M2LCursor& cu) {
  // ablk: the wave's row block in the slab's first chunk (a buffer load's base)
  const __amdgpu_buffer_rsrc_t ra = buf_rsrc(reinterpret_cast<const float*>(ablk + cu.aoff));
  const int oa = 16 * ((int)(threadIdx.x & 63) + 64 * NP * cu.c);
#pragma unroll
  for (int p = 0; p < NP; ++p)
    r.a[p] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(ra, oa + 1024 * p, 0, 0));
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
__device__ __forceinline__ void m2lb_slab(v16f* acc, v16f* tot, const uint4* ablk, size_t core_stride, int po_reg,
                                          int noffs, const int* bq, int nch, int ld16) {
  const int nv = noffs * nch;
  M2LCursor cu{0, 0, nch, noffs, ld16, po_reg, core_stride, 0, 0};
  cu.set_offset();
  M2LRegsB<NP> r0, r1;
  m2lb_load<NP>(r0, ablk, bq, cu);
  cu.next();
  for (int v = 0; v < nv; v += 2) {
    m2lb_load<NP>(r1, ablk, bq, cu);
    cu.next();
    __builtin_amdgcn_sched_barrier(0);
    m2lb_compute<NP>(r0, acc, tot);
    __builtin_amdgcn_sched_barrier(0);
    m2lb_load<NP>(r0, ablk, bq, cu);
    cu.next();
    __builtin_amdgcn_sched_barrier(0);
    if (v + 1 < nv) m2lb_compute<NP>(r1, acc, tot);
    __builtin_amdgcn_sched_barrier(0);
  }
}

struct Float4x2 {
  float4 a, b;
};
__device__ __forceinline__ Float4x2 make_float4x2(const float4& a, const float4& b) { return Float4x2{a, b}; }

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
  // the wave's row block of the lane-ordered operators (buffer-load base)
  const uint4* ablk = cores + (size_t)__builtin_amdgcn_readfirstlane(wave) * nchunk * 64 * NP;
  __shared__ int s_src[216];
  m2l_load_src(s_src, src_blk + it.src_base);

  for (int k0 = 0; k0 < ldk; k0 += kM2LSlabB) {
    const int kw = min(kM2LSlabB, ldk - k0);  // a multiple of 16
    if (k0) __syncthreads();
    // column units of 8 k (two float4), split into NP pieces as they are stored
    m2l_stage<kStageBatch / 2>(
        s_src, kw >> 3,
        [&](int slot, int g) {
          const float4* src = reinterpret_cast<const float4*>(uhat + (size_t)slot * ldk + k0 + 8 * g);
          return make_float4x2(src[0], src[1]);
        },
        [&](int r, int g, Float4x2 v, bool live) {
          const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
          uint4 pcs[NP];
          split8<NP>(live ? v.a : z, live ? v.b : z, pcs);
#pragma unroll
          for (int p = 0; p < NP; ++p) s_m2lb[r * ld16 + NP * g + p] = pcs[p];
        });
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

// Dynamic LDS limit of the M2L kernels on the current device (see
// configure_kernels).
hipError_t configure_m2l_kernels() {
  const void* kernels[] = {
      reinterpret_cast<const void*>(&k_m2l<0>),          reinterpret_cast<const void*>(&k_m2l<1>),
      reinterpret_cast<const void*>(&k_m2l_bf16<2, 0>), reinterpret_cast<const void*>(&k_m2l_bf16<2, 1>),
      reinterpret_cast<const void*>(&k_m2l_bf16<3, 0>), reinterpret_cast<const void*>(&k_m2l_bf16<3, 1>)};
  for (const void* k : kernels) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynamicLds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace kifmm
