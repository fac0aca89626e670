// Leaf and point kernels of the kiFMM evaluate for gfx950: the charge
// permutation, the S2U check fields (P2M), the fused D2T and U-list sums (L2P
// and P2P) per parent or over a work queue (vector ALUs), their multi-RHS forms
// (32 right-hand sides on the matrix cores), and the derivative's combination.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "kernels.hpp"
#include "mfma.hpp"

namespace kifmm {

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
  const int lane = tid & 63;
  for (int tb = t0; tb < t1; tb += (int)blockDim.x) {
    const int wb = tb + (tid & ~63);  // the wave's first target
    if (wb >= t1) break;              // the whole wave leaves
    const int nt = min(64, t1 - wb);  // the wave's targets
    // A wave with at most 32 targets (the last of a parent) gives each target k
    // lanes, each summing a share of the nine runs (parts [9q/k, 9(q+1)/k)); the
    // shares are added in part order below.  Full waves keep k = 1.
    const int k = (!kNear || !in_lds || nt > 32) ? 1 : nt > 21 ? 2 : nt > 7 ? 3 : 9;
    const int part = lane / nt;
    const int ti = wb + (lane - part * nt);  // a target of this wave for every lane
    const bool act = part < k;
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
      if (in_lds && k == 1) {
        // (lanes past the wave's targets repeat a target's sums; they are dropped)
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy) {
            const int e0 = (bx - 1) + 4 * (by + dy) + 16 * (bz + dz);
            const int a = s_off[e0], b = s_off[e0 + 3];  // b - a is a multiple of 4
            if ((dy == 0) & (dz == 0))
              p2p_run<true>(s_src, a, b, x, acc);
            else
              p2p_run<false>(s_src, a, b, x, acc);
          }
      } else if (in_lds) {
        // runs r = 3 (dz + 1) + (dy + 1) of part q, every pair testing r > 0
        const int r0 = act ? 9 * part / k : 0, r1 = act ? 9 * (part + 1) / k : 0;
        for (int r = r0; r < r1; ++r) {
          const int dz = r / 3 - 1, dy = r - 3 * (r / 3) - 1;
          const int e0 = (bx - 1) + 4 * (by + dy) + 16 * (bz + dz);
          p2p_run<true>(s_src, s_off[e0], s_off[e0 + 3], x, acc);
        }
        const double p0 = acc.phi, x0 = acc.gx, y0 = acc.gy, z0 = acc.gz;
        for (int q = 1; q < k; ++q) {
          const int from = lane + q * nt;  // part q of this lane's target (lanes of part 0)
          acc.add(__shfl(p0, from), __shfl(x0, from), __shfl(y0, from), __shfl(z0, from));
        }
      } else if (act) {
#pragma unroll 1
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll 1
          for (int dy = -1; dy <= 1; ++dy) {
            const int e0 = (bx - 1) + 4 * (by + dy) + 16 * (bz + dz);
            const bool own = (dy == 0) & (dz == 0);
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
    } else if (act) {
      const float4 v = near[ti];
      aphi = v.x;
      agx = v.y;
      agy = v.z;
      agz = v.w;
    }
    if (part != 0) continue;  // the other parts' sums are in part 0's lanes
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

// The source ranges [a, b) of the 27 leaves around leaf slot o of parent group g
// (its 4 x 4 x 4 leaf block, x fastest; neighbour nb = (dx + 1) + 3 (dy + 1) +
// 9 (dz + 1), the leaf itself nb = 13), one per lane of lanes 0..26 (a = b for
// a missing or empty leaf).  All 27 are loaded at once, so that a kernel walking
// the neighbours reads each range with readlane instead of waiting on two
// dependent loads per neighbour.
struct NbRange {
  int a, b;
};

__device__ __forceinline__ NbRange neighbour_ranges(const int* __restrict__ blk, const int* __restrict__ start, int g,
                                                    int o, int lane) {
  NbRange r{0, 0};
  if (lane < 27) {
    const int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
    const int bx = 1 + (o & 1), by = 1 + ((o >> 1) & 1), bz = 1 + ((o >> 2) & 1);
    const int ns = blk[(size_t)g * 64 + (bx + dx) + 4 * (by + dy) + 16 * (bz + dz)];
    if (ns >= 0) {
      r.a = start[ns];
      r.b = start[ns + 1];
    }
  }
  return r;
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
    double aphi = 0.0, agx = 0.0, agy = 0.0, agz = 0.0;
    if (kNear) {
      // the 27 leaves of the block around the tile's leaf; a leaf's sources four per
      // step, the next step's loaded while this one is used
      Sum4 acc;
      const NbRange nr = neighbour_ranges(blk, start, g, o, lane);
      for (int nb = 0; nb < 27; ++nb) {
        const int a = __builtin_amdgcn_readlane(nr.a, nb), b = __builtin_amdgcn_readlane(nr.b, nb);
        if (a >= b) continue;
        if (nb / 3 == 4)  // the row (dy = dz = 0) that holds the tile's own leaf
          queue_leaf<true>(pts, a, b, x, acc);
        else
          queue_leaf<false>(pts, a, b, x, acc);
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

// S2U first half for 32 right-hand sides on the matrix cores: per leaf (one
// wave) the check field Q[m][r] = sum over sources s of K(p_m, y_s) C[s][r] is a
// product of the kernel matrix with the leaf's 32-column charge block, two
// sources per v_mfma_f32_32x32x2_f32 step.  Lane (i, h) = (l % 32, l / 32)
// computes K(p_{32 b + i}, y_{j+h}) for NB blocks b of 32 check points (the A
// operands) and loads C[j+h][i] (the B operand); the accumulator of block b
// holds Q[32 b + 8 (v / 4) + 4 h + v % 4][r = i].  Check points past n repeat
// the last one and store nothing; a source past the leaf's end (the last one
// again) has K = 0.  The sources' positions and charges are loaded one step
// ahead, in two register sets that take turns.  FP32 sums over the leaf's
// sources, as in k_p2m_multi.
template <int NB>
__global__ __launch_bounds__(256) void k_p2m_r32(const float4* __restrict__ pts, const float* __restrict__ qs,
                                                 const int* __restrict__ start, const int* __restrict__ leaves,
                                                 const float4* __restrict__ centers, const float* __restrict__ surf,
                                                 int n, float alpha, float* __restrict__ q, int ldq, long long qrs,
                                                 int nleaves) {
  __shared__ float s_tile[4][32][36];  // per wave: one block's 32 right-hand sides x 32 check points
  const int leaf = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (leaf >= nleaves) return;
  const int lane = threadIdx.x & 63;
  const int i = lane & 31, h = lane >> 5;
  float(*tile)[36] = s_tile[threadIdx.x >> 6];
  const int slot = leaves[leaf];
  const float4 ch = centers[2 * slot], cl = centers[2 * slot + 1];
  const float sc = alpha * ch.w;
  const int s0 = start[slot], s1 = start[slot + 1];
  const int nsteps = (s1 - s0 + 1) >> 1;
  struct Step {
    float4 y;
    float c;
  };
  auto load = [&](Step& s, int t) {
    const int js = min(s0 + 2 * t + h, s1 - 1);
    s.y = pts[js];
    s.c = qs[(size_t)js * 32 + i];
  };
  for (int b0 = 0; b0 < n; b0 += 32 * NB) {
    float px[NB], py[NB], pz[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int mc = min(b0 + 32 * b + i, n - 1);
      px[b] = sc * surf[3 * mc];
      py[b] = sc * surf[3 * mc + 1];
      pz[b] = sc * surf[3 * mc + 2];
    }
    v16f acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[b][v] = 0.f;
    auto add = [&](const Step& s, int t) {
      const float yx = (s.y.x - ch.x) - cl.x, yy = (s.y.y - ch.y) - cl.y, yz = (s.y.z - ch.z) - cl.z;
      const bool live = s0 + 2 * t + h < s1;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const float dx = px[b] - yx, dy = py[b] - yy, dz = pz[b] - yz;
        const float k = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
        acc[b] = mfma32(live ? k : 0.f, s.c, acc[b]);
      }
    };
    if (nsteps > 0) {
      Step sa, sb;
      load(sa, 0);
      int t = 0;
      for (; t + 1 < nsteps; t += 2) {
        load(sb, t + 1);
        __builtin_amdgcn_sched_barrier(0);
        add(sa, t);
        __builtin_amdgcn_sched_barrier(0);
        load(sa, t + 2);
        __builtin_amdgcn_sched_barrier(0);
        add(sb, t + 1);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (t < nsteps) add(sa, t);
    }
    // Each block goes out through the wave's LDS tile, so that 8 lanes write 128
    // contiguous bytes of one right-hand side's row.
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int g = 0; g < 4; ++g)
        *reinterpret_cast<float4*>(&tile[i][8 * g + 4 * h]) =
            make_float4(acc[b][4 * g], acc[b][4 * g + 1], acc[b][4 * g + 2], acc[b][4 * g + 3]);
      const int seg = lane & 7, m = b0 + 32 * b + 4 * seg;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = 8 * k + (lane >> 3);
        const float4 v = *reinterpret_cast<const float4*>(&tile[r][4 * seg]);
        float* out = q + r * qrs + (size_t)slot * ldq + m;
        if (m + 3 < n) {
          *reinterpret_cast<float4*>(out) = v;
        } else {
          if (m < n) out[0] = v.x;
          if (m + 1 < n) out[1] = v.y;
          if (m + 2 < n) out[2] = v.z;
        }
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
    case 32: {
      // as many 32-point check blocks per pass as the surface needs, at most five
      const int nb = std::min(5, (n + 31) / 32);
#define KIFMM_P2M_R32(NB)                                                                                          \
  hipLaunchKernelGGL(k_p2m_r32<NB>, grid, block, 0, s, pts, qs, start, leaves, centers, surf, n, alpha, q, ldq, qrs, \
                     nleaves)
      switch (nb) {
        case 1: KIFMM_P2M_R32(1); break;
        case 2: KIFMM_P2M_R32(2); break;
        case 3: KIFMM_P2M_R32(3); break;
        case 4: KIFMM_P2M_R32(4); break;
        default: KIFMM_P2M_R32(5); break;
      }
#undef KIFMM_P2M_R32
      return true;
    }
    default: return false;
  }
}

// D2T + ULI for R right-hand sides, potentials, written to input order
// (pot[i][r]).  A task is up to 64 consecutive points of one leaf, one wave
// each; lanes are targets.  The leaf's 27 neighbours come from the 4 x 4 x 4
// leaf block of its parent group (as in k_p2p).  A neighbour's sources are
// taken kMultiChunk at a time: the wave copies their positions and R charges
// ([N][R], contiguous) into its own LDS with coalesced loads, then every lane
// reads each source back at one address (a broadcast), so a pair's geometry and
// reciprocal distance serve all R sums: 9 + 2R FLOP per pair.  The far field
// treats the n downward-equivalent points (centre-relative) as sources with
// densities d[r][slot][m], staged 8 points at a time the same way.  FP32
// partial sums per source leaf and per 8 surface points are accumulated in
// FP64.
constexpr int kMultiChunk = 32;

template <int R>
__global__ __launch_bounds__(256) void k_leaf_multi(const float4* __restrict__ pts, const float* __restrict__ qs,
                                                    const int* __restrict__ start, const int4* __restrict__ tasks,
                                                    int ntasks, const int* __restrict__ blk, int group_slots,
                                                    const float4* __restrict__ centers,
                                                    const float* __restrict__ surf, int n, float alpha,
                                                    const float* __restrict__ d, int ldd, long long drs, int far,
                                                    const int* __restrict__ order, float* __restrict__ pot) {
  // per wave: kMultiChunk source positions and their R charges
  __shared__ float4 s_pos[4][kMultiChunk];
  __shared__ float4 s_q[4][kMultiChunk * R / 4 + (R < 4 ? 1 : 0)];
  const int wv = threadIdx.x >> 6;
  const int t = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + wv);
  if (t >= ntasks) return;
  const int lane = threadIdx.x & 63;
  float4* pos = s_pos[wv];
  float* q = reinterpret_cast<float*>(s_q[wv]);
  const int4 task = tasks[t];
  const int slot = task.x, cnt = task.z;
  const int ti = start[slot] + task.y + min(lane, cnt - 1);
  const float4 x = pts[ti];
  const int g = slot / group_slots, o = slot - g * group_slots;
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  const NbRange nr = neighbour_ranges(blk, start, g, o, lane);
  for (int nb = 0; nb < 27; ++nb) {
    const int a = __builtin_amdgcn_readlane(nr.a, nb), b = __builtin_amdgcn_readlane(nr.b, nb);
    const bool self = nb == 13;
    float part[R];
#pragma unroll
    for (int r = 0; r < R; ++r) part[r] = 0.f;
    for (int c = a; c < b; c += kMultiChunk) {
      const int m = min(kMultiChunk, b - c);
      __builtin_amdgcn_wave_barrier();  // the previous chunk's reads come first
      if (lane < m) pos[lane] = pts[c + lane];
      for (int f = lane; f < m * R; f += 64) q[f] = qs[(size_t)c * R + f];
      __builtin_amdgcn_wave_barrier();  // LDS accesses of one wave complete in order
      for (int j = 0; j < m; ++j) {
        const float4 y = pos[j];
        const float ex = x.x - y.x, ey = x.y - y.y, ez = x.z - y.z;
        const float r2 = ex * ex + ey * ey + ez * ez;
        float rinv = __builtin_amdgcn_rsqf(r2);
        if (self) rinv = r2 > 0.f ? rinv : 0.f;  // the target itself
        const float* qj = q + j * R;
        if constexpr (R % 4 == 0) {
#pragma unroll
          for (int r = 0; r < R; r += 4) {
            const float4 q4 = *reinterpret_cast<const float4*>(qj + r);
            part[r] += q4.x * rinv;
            part[r + 1] += q4.y * rinv;
            part[r + 2] += q4.z * rinv;
            part[r + 3] += q4.w * rinv;
          }
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) part[r] += qj[r] * rinv;
        }
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
      const int mc = min(8, n - m0);
      __builtin_amdgcn_wave_barrier();
      if (lane < mc) {
        const int mm = m0 + lane;
        pos[lane] = make_float4(sc * surf[3 * mm], sc * surf[3 * mm + 1], sc * surf[3 * mm + 2], 0.f);
      }
      // densities of the 8 points for every right-hand side, [point][r]
      for (int f = lane; f < mc * R; f += 64) {
        const int pt = f / R, r = f - pt * R;
        q[f] = dl[r * drs + m0 + pt];
      }
      __builtin_amdgcn_wave_barrier();
      float part[R];
#pragma unroll
      for (int r = 0; r < R; ++r) part[r] = 0.f;
      for (int j = 0; j < mc; ++j) {
        const float4 y = pos[j];
        const float fx = xx - y.x, fy = xy - y.y, fz = xz - y.z;
        const float rinv = __builtin_amdgcn_rsqf(fx * fx + fy * fy + fz * fz);
        const float* qj = q + j * R;
        if constexpr (R % 4 == 0) {
#pragma unroll
          for (int r = 0; r < R; r += 4) {
            const float4 q4 = *reinterpret_cast<const float4*>(qj + r);
            part[r] += q4.x * rinv;
            part[r + 1] += q4.y * rinv;
            part[r + 2] += q4.z * rinv;
            part[r + 3] += q4.w * rinv;
          }
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) part[r] += qj[r] * rinv;
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

// D2T + ULI for 32 right-hand sides on the matrix cores.  For a tile of up to
// 32 targets of one leaf, the potentials of 32 right-hand sides are the product
// of the kernel matrix K[target][source] with the charges Q[source][rhs]: a
// dense contraction over the sources, computed two sources per
// v_mfma_f32_32x32x2_f32 step.  Lane (i, h) = (l % 32, l / 32) computes the
// A operand K(x_i, y_{j+h}) of target i and source j + h on the vector ALUs
// (the geometry and reciprocal distance, once per pair) and loads the B
// operand Q[j + h][i] (right-hand side i, 32 consecutive charges per source);
// the accumulator holds D[8 (v / 4) + 4 h + v % 4][i], 16 targets of right-hand
// side i per lane.  FP32 accumulation per source leaf and per 16 surface points,
// added into FP64 totals.  The U-list steps of all 27 neighbour leaves form one
// sequence with kR32Ahead steps in flight; a lane past its leaf's end (it reads
// the leaf's last source again) and coincident points (only in the target's own
// leaf) have K = 0.
constexpr int kR32Ahead = 4;  // source steps in flight per lane in k_leaf_r32

// One 2-source step of k_leaf_r32: first source j, range end lim (INT_MIN past
// the last range: no lane's source counts), the target's own leaf, first step of
// its range.
struct LeafStep {
  int j, lim;
  bool self, first;
};

// Wave-uniform position in the non-empty ranges of the 27 neighbours (lane nb of
// ra / rb holds range nb; bit nb of `left` is set for the non-empty ranges not
// yet started).  Past the last range it stays on the last source.
struct LeafCursor {
  int ra, rb;
  unsigned long long left;
  int nb = 0, a = 0, b = 1, j = 0;
  bool done = false;
  __device__ __forceinline__ void start_next() {
    if (left == 0) {
      done = true;
      j = b - 1;
      return;
    }
    nb = __builtin_ctzll(left);
    left &= left - 1;
    a = __builtin_amdgcn_readlane(ra, nb);
    b = __builtin_amdgcn_readlane(rb, nb);
    j = a;
  }
  __device__ __forceinline__ void next() {
    if (done) return;
    j += 2;
    if (j >= b) start_next();
  }
  __device__ __forceinline__ LeafStep step() const { return {j, done ? INT_MIN : b, nb == 13, !done && j == a}; }
};


__global__ __launch_bounds__(256) void k_leaf_r32(const float4* __restrict__ pts, const float* __restrict__ qs,
                                                  const int* __restrict__ start, const int4* __restrict__ tasks,
                                                  int ntasks, const int* __restrict__ blk, int group_slots,
                                                  const float4* __restrict__ centers, const float* __restrict__ surf,
                                                  int n, float alpha, const float* __restrict__ d, int ldd,
                                                  long long drs, int far, const int* __restrict__ order,
                                                  float* __restrict__ pot) {
  __shared__ float s_surf[3 * kMaxLeafSurface];  // the unit surface (far field)
  if (far) {
    for (int e = threadIdx.x; e < 3 * n; e += blockDim.x) s_surf[e] = surf[e];
    __syncthreads();
  }
  const int t = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (t >= ntasks) return;
  const int lane = threadIdx.x & 63;
  const int i = lane & 31, h = lane >> 5;
  const int4 task = tasks[t];
  const int slot = task.x, cnt = task.z;
  const int t0 = start[slot] + task.y;  // sorted index of the tile's first target
  const float4 x = pts[t0 + min(i, cnt - 1)];
  const int g = slot / group_slots, o = slot - g * group_slots;
  double tot[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) tot[v] = 0.0;
  auto flush = [&](v16f& acc) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      tot[v] += acc[v];
      acc[v] = 0.f;
    }
  };
  v16f acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  // The U-list sources as one sequence of 2-source steps over the non-empty
  // neighbour ranges (wave-uniform cursor), kR32Ahead steps in flight: step u of
  // a group is computed, then its registers take the step kR32Ahead later.
  const NbRange nr = neighbour_ranges(blk, start, g, o, lane);
  LeafCursor cu{nr.a, nr.b, __builtin_amdgcn_ballot_w64(lane < 27 && nr.a < nr.b)};
  cu.start_next();
  float4 y[kR32Ahead];
  float q[kR32Ahead];
  LeafStep st[kR32Ahead];
  auto fetch = [&](int u) {
    const int js = min(cu.j + h, cu.b - 1);
    y[u] = pts[js];
    q[u] = qs[js * 32 + i];
    st[u] = cu.step();
    cu.next();
  };
#pragma unroll
  for (int u = 0; u < kR32Ahead; ++u) fetch(u);
  do {
#pragma unroll
    for (int u = 0; u < kR32Ahead; ++u) {
      if (st[u].first) flush(acc);
      const float ex = x.x - y[u].x, ey = x.y - y[u].y, ez = x.z - y[u].z;
      const float r2 = ex * ex + ey * ey + ez * ez;
      float k = __builtin_amdgcn_rsqf(r2);
      if (st[u].self) k = r2 > 0.f ? k : 0.f;  // the target itself
      k = st[u].j + h < st[u].lim ? k : 0.f;
      acc = mfma32(k, q[u], acc);
      fetch(u);
    }
  } while (st[0].lim > INT_MIN);
  flush(acc);
  if (far) {
    const float4 ch = centers[2 * slot], cl = centers[2 * slot + 1];
    const float xx = (x.x - ch.x) - cl.x, xy = (x.y - ch.y) - cl.y, xz = (x.z - ch.z) - cl.z;
    const float sc = alpha * ch.w;
    const float* dl = d + (size_t)i * drs + (size_t)slot * ldd;  // density of right-hand side i
    // 16 surface points per FP32 partial: their 8 densities per lane are loaded
    // one group ahead (two register sets taking turns); the surface points come
    // from LDS.  Steps past n add zero.
    const int ngrp = (n + 15) / 16;
    float dA[8], dB[8];
    auto load_d = [&](float* dv, int c) {
#pragma unroll
      for (int s = 0; s < 8; ++s) dv[s] = dl[min(16 * c + 2 * s + h, n - 1)];
    };
    auto group = [&](const float* dv, int c) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int m = 16 * c + 2 * s;
        const int mm = min(m + h, n - 1);
        const float fx = xx - sc * s_surf[3 * mm], fy = xy - sc * s_surf[3 * mm + 1], fz = xz - sc * s_surf[3 * mm + 2];
        const float k = __builtin_amdgcn_rsqf(fx * fx + fy * fy + fz * fz);
        acc = mfma32(k, m + h < n ? dv[s] : 0.f, acc);
      }
      flush(acc);
    };
    load_d(dA, 0);
    int c = 0;
    for (; c + 1 < ngrp; c += 2) {
      load_d(dB, c + 1);
      __builtin_amdgcn_sched_barrier(0);
      group(dA, c);
      __builtin_amdgcn_sched_barrier(0);
      load_d(dA, c + 2);
      __builtin_amdgcn_sched_barrier(0);
      group(dB, c + 1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (c < ngrp) group(dA, c);
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = 8 * (v >> 2) + 4 * h + (v & 3);  // target of the tile
    if (row < cnt) pot[(size_t)order[t0 + row] * 32 + i] = (float)tot[v];
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
    case 32:
      hipLaunchKernelGGL(k_leaf_r32, grid, block, 0, s, pts, qs, start, tasks, ntasks, blk, group_slots, centers, surf,
                         n, alpha, d, ldd, drs, far, order, pot);
      return true;
    default: return false;
  }
#undef KIFMM_LEAF_MULTI
}

// Dynamic LDS limit of every kernel that stages data in LDS, for the current
// device.  Plans call this once per device (under a lock) before their first
// launch; the launchers then only check their sizes against kMaxDynamicLds.
hipError_t configure_kernels() {
  hipError_t e = configure_m2l_kernels();
  if (e == hipSuccess) e = configure_gemm_kernels();
  if (e != hipSuccess) return e;
  const void* kernels[] = {reinterpret_cast<const void*>(&k_p2p<0>), reinterpret_cast<const void*>(&k_p2p<1>),
                           reinterpret_cast<const void*>(&k_p2p<2>)};
  for (const void* k : kernels) {
    const hipError_t e2 = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynamicLds);
    if (e2 != hipSuccess) return e2;
  }
  return hipSuccess;
}

}  // namespace kifmm
