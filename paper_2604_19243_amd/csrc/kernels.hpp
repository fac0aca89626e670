// Launchers of the HIP kernels (gemm.hip, m2l.hip, leaf.hip).  All pointers are device memory;
// every launch is asynchronous on stream `s`.
#pragma once

#include <hip/hip_runtime.h>

namespace kifmm {

// Dynamic LDS any launch here may request (gfx950 has 160 KiB per CU; the rest
// covers the kernels' static LDS).
constexpr size_t kMaxDynamicLds = 156 * 1024;
// Surface points the leaf kernels hold in LDS (p <= 8).
constexpr int kMaxLeafSurface = 304;
// Sets the dynamic LDS limit of every LDS-staging kernel on the current device.
hipError_t configure_kernels();
hipError_t configure_m2l_kernels();
hipError_t configure_gemm_kernels();

// An M2L work item (see k_m2l in m2l.hip): one aligned 4x4x4 block of
// parents at one level, target sibling position o and source position o'.
struct M2LItem {
  int pair;      // 8 o + o'
  int noffs;     // number of V-list offsets of the pair (19 to 26)
  int part;      // o': which partial sum this item writes
  int tgt_base;  // 64 target slots (or -1) in block position order, x fastest
  int src_base;  // 216 source slots (or -1): position o' children of the 6x6x6 parents around the block
};

// batch > 1: the same product for `batch` right-hand sides, X and Y advanced by
// xbs and ybs floats per right-hand side (batch = 32: the right-hand sides are the
// matrix-core columns, k_gemm_r32).
// ywide: write Y in the 32-right-hand-side lane order of k_m2l_wide ([row][nout / 8][32][8],
// batch index = right-hand side; ybs unused), nout a multiple of 8 and batch = 32.
void launch_gemm_nt(const float* W, int ldw, const float* X, int ldx, const int* xrow, float* Y, int ldy,
                    const int* yrow, int nbox, int nout, int K, float alpha, int beta, hipStream_t s, int batch = 1,
                    long long xbs = 0, long long ybs = 0, int ywide = 0);
// Whether a kernel instance fits (row blocks, padded rank, LDS row stride).
bool m2l_supported(int row_blocks, int ldk, int lds_ld);
// Returns false if no kernel instance fits (rb, ldk).
// nrhs right-hand sides: uhat and each partial sum advance by rhs_stride floats per right-hand side.
// upper: the launch for the levels above the leaves (a kernel instance of its own name).
bool launch_m2l(int row_blocks, const float* cores, int core_rows, int ldk, int lds_ld, const M2LItem* items, int nitems,
                const int* tgt_blk, const int* src_blk, const int* pair_offs, const float* uhat, float* chat_part,
                long long part_stride, int nrhs, long long rhs_stride, hipStream_t s, bool upper = false);
// The same translation from split-bfloat16 pieces (2 pieces: three matrix-core
// passes; 3 pieces: six): cores are [316][row block][16-k chunk][piece][64
// lanes][8] bfloat16 bit patterns; core_stride16 is the size of one offset's
// operator in 16-byte units; lds_ld16 >= m2l_bf16_lds_ld16(pieces).
int m2l_bf16_lds_ld16(int pieces);
bool m2l_bf16_supported(int pieces, int row_blocks, int ldk);
bool launch_m2l_bf16(int pieces, int row_blocks, const uint16_t* cores, size_t core_stride16, int ldk, int lds_ld16,
                     const M2LItem* items, int nitems, const int* tgt_blk, const int* src_blk, const int* pair_offs,
                     const float* uhat, float* chat_part, long long part_stride, int nrhs, long long rhs_stride,
                     hipStream_t s, bool upper = false);
// M2L for 32 right-hand sides: one workgroup of row_blocks waves (<= 8, false otherwise)
// per unit, two int4 each: (slot of target 0, slot of target 1 or -1, first, end entry)
// and (end of the entries of both targets, end of those of target 0 alone, 0, 0), those
// of target 1 alone last; entries (core index, source slot of target 0 or -1, of target
// 1 or -1, 0); uhat in the lane order written by launch_gemm_nt(ywide); chat
// [32][slots][ldk] (chat_rs = slots * ldk).
bool launch_m2l_wide(int row_blocks, const float* cores, long long core_stride, int ldk, const int4* units,
                     int nunits, const int4* ents, const float* uhat, float* chat, long long chat_rs, hipStream_t s);
// M2L with gathered sources, one right-hand side: units (group, row block, first, end entry);
// per entry the core index and 32 source rows of uhat (zero row where none); grp_tgt: 32
// target slots per group (-1 = none); chat [slots][ldk].
void launch_m2l_gather(const float* cores, long long core_stride, int ldk, const int4* units, int nunits,
                       const int* ent_core, const int* ent_src, const int* grp_tgt, const float* uhat, float* chat,
                       hipStream_t s, bool upper = false);
void launch_sum_parts(const float* part, float* chat, long long n, long long stride, hipStream_t s);
// out[k][c] = w[k] fs[k][c] + s[k] fw[k][c] for k < n, c < 3.
void launch_vjp_combine(const float* s, const float* w, const float* fs, const float* fw, float* out, int n,
                        hipStream_t st);
void launch_permute(float4* pts, const float* charges, const int* order, int n, hipStream_t s);
// False if n > 768 (no kernel instance).
bool p2m_supported(int n);
bool launch_p2m(const float4* pts, const int* start, const int* leaves, const float4* centers, const float* surf, int n,
                float alpha, float* q, int ldq, int nleaves, hipStream_t s);
// centers: per leaf slot two float4, (c_hi, r) and (c_lo, 0) with c = c_hi + c_lo.
// blk: per parent group, the 64 leaf slots of the 4x4x4 block around it (-1 = none).
// cap: sources staged in LDS per block (each leaf padded to a multiple of 4).
size_t p2p_lds_bytes(int cap, int n);
// mode 0: near + far field fused, written to input order; mode 1: near field only,
// written in sorted order to `near` (phi, grad); mode 2: far field added to `near`,
// written to input order.  threads: 256 or kP2PMaxThreads per workgroup (false
// otherwise); the results do not depend on it.
constexpr int kP2PMaxThreads = 320;
bool p2p_supported(int threads, int cap, int n);
bool launch_p2p(int mode, const float4* pts, const int* start, const int* blk, int ngroups, int group_slots, int cap,
                const float4* centers, const float* surf, int n, float alpha, const float* d, int ldd, int far,
                const int* order, float* pot, float* grad, float4* near, int threads, hipStream_t s);

// The same sums as k_p2p (modes as there) by a persistent kernel over tiles
// (leaf slot, first sorted point, count <= 64, 0) taken with the counters
// queue[16 x], x = 0..7 (one per XCD), which launch_clear_queue zeroes (n ints)
// before each launch.  `grid` workgroups of four waves, a multiple of 8.
constexpr int kQueueInts = 128;  // counters of one launch (eight, 64 bytes apart)
void launch_clear_queue(int* queue, int n, hipStream_t s);
bool launch_leaf_queue(int mode, const float4* pts, const int* start, const int4* tiles, int ntiles, int* queue,
                       int grid, const int* blk, int group_slots, const float4* centers, const float* surf, int n,
                       float alpha, const float* d, int ldd, int far, const int* order, float* pot, float* grad,
                       float4* near, hipStream_t s);

// Multi-RHS leaf kernels (R = 2, 4, 8, 16, 32; potentials only; R = 32 on the
// matrix cores: k_p2m_r32, k_leaf_r32).  qs: sorted charges [N][R].  q: check
// fields [R][leaf slots][ldq], qrs = leaf slots * ldq.
// tasks: (leaf slot, first point offset in the leaf, point count, 0), at most
// kMultiTile(R) points.
// d: leaf-level downward densities, slot row `slot` at d + slot * ldd, right-hand
// side r at + r * drs.  Return false for an unsupported R.
constexpr int kMultiTile(int R) { return R == 32 ? 32 : 64; }
void launch_permute_multi(float* qs, const float* charges, const int* order, int n, int R, hipStream_t s);
bool launch_p2m_multi(int R, const float4* pts, const float* qs, const int* start, const int* leaves,
                      const float4* centers, const float* surf, int n, float alpha, float* q, int ldq, long long qrs,
                      int nleaves, hipStream_t s);
bool launch_leaf_multi(int R, const float4* pts, const float* qs, const int* start, const int4* tasks, int ntasks,
                       const int* blk, int group_slots, const float4* centers, const float* surf, int n, float alpha,
                       const float* d, int ldd, long long drs, int far, const int* order, float* pot, hipStream_t s);

}  // namespace kifmm
