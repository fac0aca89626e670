// HIP kernels of the kiFMM evaluate for gfx950 (CDNA4).
//
// Dense contractions (check-to-equivalent factors, U2U, compression, U2D, post,
// D2D) run on the FP32 matrix cores through v_mfma_f32_16x16x4_f32; the kernel
// sums (S2U check fields, D2T and the U-list direct sum) run on the vector
// ALUs.  All arithmetic is FP32.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace kifmm {

typedef float v4f __attribute__((ext_vector_type(4)));

// One 16x16x4 FP32 matrix-core step.  Operand layout (wave64): lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; the accumulator holds
// D[4 (l / 16) + v][l % 16] in element v.
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Four MFMA steps over 16 consecutive k.  Lane (i, q) = (l % 16, l / 16) holds
// a = A[i][4q .. 4q+3] and b = B^T[j][4q .. 4q+3]; step r contracts k = 4q + r,
// which covers all 16 k because the sum over k does not depend on its order.
__device__ __forceinline__ v4f mfma16x4(const float4 a, const float4 b, v4f c) {
  c = mfma16(a.x, b.x, c);
  c = mfma16(a.y, b.y, c);
  c = mfma16(a.z, b.z, c);
  c = mfma16(a.w, b.w, c);
  return c;
}

// ---------------------------------------------------------------- GEMM ---
// Y[yrow(b)][o] = alpha * sum_k W[o][k] X[xrow(b)][k]  (+ Y[yrow(b)][o] when beta)
// W: [>= round_up(nout, 64)][ldw] row-major, rows >= nout zero.  X rows: ldx.
// K, nout, ldx, ldy, ldw are multiples of 4; pointers 16-byte aligned.
// Block tile: 64 outputs x 64 boxes; 4 waves as 2 (outputs) x 2 (boxes), each
// wave 32 x 32 = 2 x 2 MFMA blocks.
__global__ __launch_bounds__(256) void k_gemm_nt(const float* __restrict__ W, int ldw, const float* __restrict__ X,
                                                 int ldx, const int* __restrict__ xrow, float* __restrict__ Y, int ldy,
                                                 const int* __restrict__ yrow, int nbox, int nout, int K, float alpha,
                                                 int beta) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int i16 = lane & 15, q = lane >> 4;
  const int o0 = blockIdx.y * 64 + (wave & 1) * 32;
  const int b0 = blockIdx.x * 64 + (wave >> 1) * 32;

  const float* wp[2];
  const float* xp[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) wp[m] = W + (size_t)(o0 + 16 * m + i16) * ldw;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    int b = min(b0 + 16 * nb + i16, nbox - 1);
    int r = xrow ? xrow[b] : b;
    xp[nb] = X + (size_t)r * ldx;
  }
  v4f acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) acc[m][nb] = v4f{0.f, 0.f, 0.f, 0.f};

  int k = 0;
  for (; k + 16 <= K; k += 16) {
    float4 a[2], b[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) a[m] = *reinterpret_cast<const float4*>(wp[m] + k + 4 * q);
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) b[nb] = *reinterpret_cast<const float4*>(xp[nb] + k + 4 * q);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) acc[m][nb] = mfma16x4(a[m], b[nb], acc[m][nb]);
  }
  for (; k < K; k += 4) {
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) acc[m][nb] = mfma16(wp[m][k + q], xp[nb][k + q], acc[m][nb]);
  }
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int b = b0 + 16 * nb + i16;
    if (b >= nbox) continue;
    const int r = yrow ? yrow[b] : b;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int o = o0 + 16 * m + 4 * q;
      if (o >= nout) continue;
      float4* yp = reinterpret_cast<float4*>(Y + (size_t)r * ldy + o);
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
}

void launch_gemm_nt(const float* W, int ldw, const float* X, int ldx, const int* xrow, float* Y, int ldy,
                    const int* yrow, int nbox, int nout, int K, float alpha, int beta, hipStream_t s) {
  if (nbox <= 0) return;
  dim3 grid((nbox + 63) / 64, (nout + 63) / 64);
  hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, s, W, ldw, X, ldx, xrow, Y, ldy, yrow, nbox, nout, K, alpha, beta);
}

// ----------------------------------------------------------------- M2L ---
// Compressed VLI: for every target box B of a tile,
//   chat[B][o] = sum_{j < 189} sum_k C_{t(j)}[o][k] uhat[src(B, j)][k],
// where t(j) is the j-th V-list offset of B's position among its siblings and
// src(B, j) is the source box at that offset (-1: none).  One workgroup owns
// 64 targets of one level and one sibling position, and all output rows.
// Waves are 2 (row halves) x 2 (32 targets); a wave holds RB row blocks of 16.
template <int RB>
__global__ __launch_bounds__(256) void k_m2l(const float* __restrict__ cores, int core_rows, int ldk, int K,
                                             const int* __restrict__ offidx, const float* __restrict__ uhat,
                                             float* __restrict__ chat, const float* __restrict__ zero_row,
                                             const M2LTile* __restrict__ tiles, const int* __restrict__ tgt,
                                             const int* __restrict__ vsrc) {
  const M2LTile tile = tiles[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int i16 = lane & 15, q = lane >> 4;
  const int row0 = (wave & 1) * RB * 16;
  const int col0 = (wave >> 1) * 32;

  v4f acc[RB][2];
#pragma unroll
  for (int m = 0; m < RB; ++m)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) acc[m][nb] = v4f{0.f, 0.f, 0.f, 0.f};

  int col_ok[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) col_ok[nb] = (col0 + 16 * nb + i16) < tile.count;
  const int* vs = vsrc + tile.vsrc_base + tile.i0 + col0 + i16;
  const int* offs = offidx + tile.octant * 189;

  for (int j = 0; j < 189; ++j) {
    int s[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) s[nb] = col_ok[nb] ? vs[(size_t)j * tile.stride + 16 * nb] : -1;
    if (!__any(s[0] >= 0 || s[1] >= 0)) continue;
    const float* ap[RB];
    const float* base = cores + (size_t)offs[j] * core_rows * ldk;
#pragma unroll
    for (int m = 0; m < RB; ++m) ap[m] = base + (size_t)(row0 + 16 * m + i16) * ldk;
    const float* bp[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) bp[nb] = s[nb] >= 0 ? uhat + (size_t)s[nb] * ldk : zero_row;
    int k = 0;
    for (; k + 16 <= K; k += 16) {
      float4 a[RB], b[2];
#pragma unroll
      for (int m = 0; m < RB; ++m) a[m] = *reinterpret_cast<const float4*>(ap[m] + k + 4 * q);
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) b[nb] = *reinterpret_cast<const float4*>(bp[nb] + k + 4 * q);
#pragma unroll
      for (int m = 0; m < RB; ++m)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[m][nb] = mfma16x4(a[m], b[nb], acc[m][nb]);
    }
    for (; k < K; k += 4) {
#pragma unroll
      for (int m = 0; m < RB; ++m)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[m][nb] = mfma16(ap[m][k + q], bp[nb][k + q], acc[m][nb]);
    }
  }
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    if (!col_ok[nb]) continue;
    const int b = tgt[tile.tgt_base + tile.i0 + col0 + 16 * nb + i16];
#pragma unroll
    for (int m = 0; m < RB; ++m) {
      const int o = row0 + 16 * m + 4 * q;
      if (o >= K) continue;
      *reinterpret_cast<float4*>(chat + (size_t)b * ldk + o) =
          make_float4(acc[m][nb][0], acc[m][nb][1], acc[m][nb][2], acc[m][nb][3]);
    }
  }
}

void launch_m2l(int rb, const float* cores, int core_rows, int ldk, int K, const int* offidx, const float* uhat,
                float* chat, const float* zero_row, const M2LTile* tiles, int ntiles, const int* tgt,
                const int* vsrc, hipStream_t s) {
  if (ntiles <= 0) return;
#define KIFMM_M2L_CASE(R)                                                                                         \
  case R:                                                                                                         \
    hipLaunchKernelGGL(k_m2l<R>, dim3(ntiles), dim3(256), 0, s, cores, core_rows, ldk, K, offidx, uhat, chat,     \
                       zero_row, tiles, tgt, vsrc);                                                               \
    break;
  switch (rb) {
    KIFMM_M2L_CASE(1)
    KIFMM_M2L_CASE(2)
    KIFMM_M2L_CASE(3)
    KIFMM_M2L_CASE(4)
    KIFMM_M2L_CASE(5)
    KIFMM_M2L_CASE(6)
    KIFMM_M2L_CASE(7)
    KIFMM_M2L_CASE(8)
    KIFMM_M2L_CASE(9)
    KIFMM_M2L_CASE(10)
    default:
      break;
  }
#undef KIFMM_M2L_CASE
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
// surface c + alpha_outer r S_m.  One wave per leaf; lanes over the n check
// points, sources read uniformly by the whole wave.  Geometry is relative to
// the leaf centre c = c_hi + c_lo (two floats), so rounding is relative to the
// box size rather than to |c|.
__global__ __launch_bounds__(256) void k_p2m(const float4* __restrict__ pts, const int* __restrict__ start,
                                             const int* __restrict__ leaves, const float4* __restrict__ centers,
                                             const float* __restrict__ surf, int n, float alpha, float* __restrict__ q,
                                             int ldq, int nleaves) {
  const int leaf = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (leaf >= nleaves) return;
  const int lane = threadIdx.x & 63;
  const int slot = leaves[leaf];
  const float4 ch = centers[2 * slot], cl = centers[2 * slot + 1];
  const float sc = alpha * ch.w;
  const int s0 = start[slot], s1 = start[slot + 1];
  for (int m = lane; m < n; m += 64) {
    const float px = sc * surf[3 * m], py = sc * surf[3 * m + 1], pz = sc * surf[3 * m + 2];
    float acc = 0.f;
    for (int j = s0; j < s1; ++j) {
      const float4 y = pts[j];
      const float dx = px - ((y.x - ch.x) - cl.x);
      const float dy = py - ((y.y - ch.y) - cl.y);
      const float dz = pz - ((y.z - ch.z) - cl.z);
      acc += y.w * __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
    }
    q[(size_t)slot * ldq + m] = acc;
  }
}

void launch_p2m(const float4* pts, const int* start, const int* leaves, const float4* centers, const float* surf, int n,
                float alpha, float* q, int ldq, int nleaves, hipStream_t s) {
  if (nleaves <= 0) return;
  hipLaunchKernelGGL(k_p2m, dim3((nleaves + 3) / 4), dim3(256), 0, s, pts, start, leaves, centers, surf, n, alpha, q,
                     ldq, nleaves);
}

// ----------------------------------------------------------------- P2P ---
// Fused D2T and ULI (Algorithm 1 steps 3b, 3c) for the leaves of one parent
// (up to 8 siblings) per workgroup, written straight to input order.
//
// The siblings' U lists together cover the 4 x 4 x 4 block of leaves around
// the parent; `blk` lists their slots (x fastest, -1 = none).  Their sources
// are staged once in LDS; each thread owns one target and walks the 27 block
// entries around its own leaf.  Only the leaf's own entry can hold a source at
// zero distance, so only that loop tests r > 0.  D2T evaluates the downward-
// equivalent surface (alpha_outer r S_m relative to the leaf centre, density
// d[m]) as n more sources, in centre-relative coordinates.  If a block's
// sources exceed the LDS capacity they are read from global memory instead.
constexpr int kP2PCap = 2560;   // sources staged per block (40 KB)
constexpr int kP2PMaxN = 304;   // largest n (p <= 8) rounded up to 16

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

__global__ __launch_bounds__(256) void k_p2p(const float4* __restrict__ pts, const int* __restrict__ start,
                                             const int* __restrict__ blk, int group_slots,
                                             const float4* __restrict__ centers, const float* __restrict__ surf,
                                             int n, float alpha, const float* __restrict__ d, int ldd, int far,
                                             const int* __restrict__ order, float* __restrict__ pot,
                                             float* __restrict__ grad) {
  __shared__ float4 s_src[kP2PCap];
  __shared__ float4 s_de[kP2PMaxN];
  __shared__ float s_d[8 * kP2PMaxN];
  __shared__ int s_off[65];
  __shared__ int s_slot[64];
  __shared__ int s_cs[9];

  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int c0 = group_slots * g;  // first leaf slot of this parent

  if (tid < 64) {
    const int slot = blk[(size_t)g * 64 + tid];
    const int cnt = slot >= 0 ? start[slot + 1] - start[slot] : 0;
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o);
      if (tid >= o) incl += v;
    }
    s_slot[tid] = slot;
    s_off[tid + 1] = incl;
    if (tid == 0) s_off[0] = 0;
  }
  if (tid <= group_slots) s_cs[tid] = start[c0 + tid];
  __syncthreads();
  const int total = s_off[64];
  const bool in_lds = total <= kP2PCap;
  if (in_lds) {
    for (int i = tid; i < total; i += 256) {
      int lo = 0, hi = 64;  // entry e with s_off[e] <= i < s_off[e + 1]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_off[mid] <= i) lo = mid;
        else hi = mid;
      }
      s_src[i] = pts[start[s_slot[lo]] + (i - s_off[lo])];
    }
  }
  const float sc = alpha * centers[2 * c0].w;
  if (far) {
    for (int m = tid; m < n; m += 256)
      s_de[m] = make_float4(sc * surf[3 * m], sc * surf[3 * m + 1], sc * surf[3 * m + 2], 0.f);
    for (int i = tid; i < group_slots * n; i += 256) {
      const int o = i / n, m = i - o * n;
      s_d[o * n + m] = d[(size_t)(c0 + o) * ldd + m];
    }
  }
  __syncthreads();

  const int t0 = s_cs[0], t1 = s_cs[group_slots];
  for (int tb = t0; tb < t1; tb += 256) {
    const int ti = tb + tid;
    if (ti >= t1) break;
    int o = 0;
    while (o + 1 < group_slots && s_cs[o + 1] <= ti) ++o;
    const float4 x = pts[ti];
    const int bx = 1 + (o & 1), by = 1 + ((o >> 1) & 1), bz = 1 + ((o >> 2) & 1);
    // Two-level summation: FP32 partial sums per source leaf and per block of 8
    // surface points, accumulated in FP64 (the D2T sum cancels heavily).
    double aphi = 0.0, agx = 0.0, agy = 0.0, agz = 0.0;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int e = (bx + dx) + 4 * (by + dy) + 16 * (bz + dz);
          const bool self = (dx == 0) & (dy == 0) & (dz == 0);
          float phi = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
          if (in_lds) {
            const int a = s_off[e], b = s_off[e + 1];
            if (self)
              for (int j = a; j < b; ++j) p2p_pair_masked(x.x, x.y, x.z, s_src[j], phi, gx, gy, gz);
            else
              for (int j = a; j < b; ++j) p2p_pair(x.x, x.y, x.z, s_src[j], phi, gx, gy, gz);
          } else {
            const int slot = s_slot[e];
            if (slot >= 0) {
              const int a = start[slot], b = start[slot + 1];
              if (self)
                for (int j = a; j < b; ++j) p2p_pair_masked(x.x, x.y, x.z, pts[j], phi, gx, gy, gz);
              else
                for (int j = a; j < b; ++j) p2p_pair(x.x, x.y, x.z, pts[j], phi, gx, gy, gz);
            }
          }
          aphi += phi;
          agx += gx;
          agy += gy;
          agz += gz;
        }
    if (far) {
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
    const float phi = (float)aphi, gx = (float)agx, gy = (float)agy, gz = (float)agz;
    const int oi = order[ti];
    if (pot) pot[oi] = phi;
    if (grad) {
      grad[3 * (size_t)oi] = gx;
      grad[3 * (size_t)oi + 1] = gy;
      grad[3 * (size_t)oi + 2] = gz;
    }
  }
}

void launch_p2p(const float4* pts, const int* start, const int* blk, int ngroups, int group_slots,
                const float4* centers, const float* surf, int n, float alpha, const float* d, int ldd, int far,
                const int* order, float* pot, float* grad, hipStream_t s) {
  if (ngroups <= 0) return;
  hipLaunchKernelGGL(k_p2p, dim3(ngroups), dim3(256), 0, s, pts, start, blk, group_slots, centers, surf, n, alpha, d,
                     ldd, far, order, pot, grad);
}

}  // namespace kifmm
