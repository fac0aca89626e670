// Launchers of the HIP kernels (kernels.hip).  All pointers are device memory;
// every launch is asynchronous on stream `s`.
#pragma once

#include <hip/hip_runtime.h>

namespace kifmm {

// A block of up to 64 M2L targets of one level and one sibling position.
struct M2LTile {
  int octant;     // position among siblings, 0..7 (selects the 189 offsets)
  int i0;         // first target index within its group
  int count;      // targets in this tile (<= 64)
  int stride;     // targets in the group: row stride of the group's source table
  int tgt_base;   // group's first entry in the target list
  long long vsrc_base;  // group's first entry in the source table [189][stride]
};

void launch_gemm_nt(const float* W, int ldw, const float* X, int ldx, const int* xrow, float* Y, int ldy,
                    const int* yrow, int nbox, int nout, int K, float alpha, int beta, hipStream_t s);
void launch_m2l(int rb, const float* cores, int core_rows, int ldk, int K, const int* offidx, const float* uhat,
                float* chat, const float* zero_row, const M2LTile* tiles, int ntiles, const int* tgt,
                const int* vsrc, hipStream_t s);
void launch_permute(float4* pts, const float* charges, const int* order, int n, hipStream_t s);
void launch_p2m(const float4* pts, const int* start, const int* leaves, const float4* centers, const float* surf, int n,
                float alpha, float* q, int ldq, int nleaves, hipStream_t s);
// centers: per leaf slot two float4, (c_hi, r) and (c_lo, 0) with c = c_hi + c_lo.
// blk: per parent group, the 64 leaf slots of the 4x4x4 block around it (-1 = none).
void launch_p2p(const float4* pts, const int* start, const int* blk, int ngroups, int group_slots,
                const float4* centers, const float* surf, int n, float alpha, const float* d, int ldd, int far,
                const int* order, float* pot, float* grad, hipStream_t s);

}  // namespace kifmm
