// Device plan of the kiFMM evaluate: data layout in HBM, interaction tables,
// and the launch sequence of Algorithm 1.
//
// Box layout ("slots").  Level 0 has one slot.  At level l >= 1 the slots are
// 8 per non-empty box of level l-1, in Morton order: the child at position o
// (x bit 0, y bit 1, z bit 2) of the j-th non-empty parent is slot 8 j + o.
// Siblings are therefore contiguous, so U2U reads and D2D writes the eight
// children of a parent as one row, and slot order is Morton order.  Slots of
// empty boxes hold zeros.  Per-box vectors of levels 2..L are stored in one
// array per kind (u, d: row stride nst = n rounded up to 4; uhat, chat: kst),
// indexed by base[l] + slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>

#include "common.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace kifmm {

void autotune(Plan* P, hipStream_t st);
void vjp_enqueue(Plan* P, const float* charges, const float* weights, const float* field, float* grad_charges,
                 float* grad_points, float* fs_buf, float* fw_buf, hipStream_t st);

namespace {

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// bfloat16 bit pattern of x: x rounded to FP32, then to its top 16 bits, to
// nearest with ties to even (finite values).
uint16_t bf16_round(double x) {
  const float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

double bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  (void)hipGetLastError();
  fail(e == hipErrorOutOfMemory ? KIFMM_E_NOMEM : KIFMM_E_DEVICE,
       std::string(what) + ": " + hipGetErrorString(e));
}

// Makes `device` current for a scope and restores the previous device.
struct DeviceScope {
  int prev = -1;
  explicit DeviceScope(int device) {
    hip_check(hipGetDevice(&prev), "hipGetDevice");
    if (prev != device) hip_check(hipSetDevice(device), "hipSetDevice");
  }
  ~DeviceScope() { (void)hipSetDevice(prev); }
};

// The device arrays of a plan, gathered on the host first, so that their total
// size is known (and checked against the device memory limit) before anything
// is allocated or enqueued.
struct Staging {
  struct Item {
    void** dst;
    size_t bytes;           // allocation size
    size_t copy_bytes;      // bytes copied from `data` (0: the array is zeroed)
    const void* data;
    std::shared_ptr<const void> keep;
  };
  std::vector<Item> items;
  int64_t total = 0;
  static size_t padded(size_t b) { return (b + 255) / 256 * 256; }
  template <class T>
  void data(void** dst, std::vector<T> host) {
    auto keep = std::make_shared<const std::vector<T>>(std::move(host));
    const size_t copy = keep->size() * sizeof(T);
    const size_t bytes = std::max<size_t>(copy, sizeof(T));
    items.push_back({dst, bytes, copy, copy ? keep->data() : nullptr, keep});
    total += (int64_t)padded(bytes);
  }
  template <class T>
  void zeros(void** dst, size_t count) {
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    items.push_back({dst, bytes, 0, nullptr, nullptr});
    total += (int64_t)padded(bytes);
  }
};

// Kernel attributes are set once per device.
std::mutex g_config_mu;
std::set<int> g_configured;

// Workspace of kifmm_evaluate_vjp_noalloc: the two [n][3] fields of the
// derivative for n <= kNoAllocMaxPoints, in a device array of the library
// rather than in memory a plan allocates.  Each GPU the library runs on holds
// its own copy until the process ends.  In host code `scratch` names a host-side
// stand-in: kernels and copies get the device address that hipGetSymbolAddress
// gives on each device (g_scratch), never the array's name.
constexpr int64_t kNoAllocMaxPoints = KIFMM_NOALLOC_MAX_POINTS;
static __device__ __align__(256) float scratch[2 * 3 * kNoAllocMaxPoints];
std::map<int, float*> g_scratch;  // device -> address of `scratch` there (under g_config_mu)

// Once per device, with the device current: kernel attributes and the address
// of the no-allocation workspace.
void configure_device(int device) {
  std::lock_guard<std::mutex> lock(g_config_mu);
  if (g_configured.count(device)) return;
  hip_check(configure_kernels(), "kernel LDS configuration");
  void* ptr = nullptr;
  hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "address of the no-allocation workspace");
  g_scratch[device] = static_cast<float*>(ptr);
  g_configured.insert(device);
}

float* scratch_address(int device) {
  std::lock_guard<std::mutex> lock(g_config_mu);
  auto it = g_scratch.find(device);
  if (it == g_scratch.end()) fail(KIFMM_E_STATE, "internal: the device was not configured by a plan");
  return it->second;
}

constexpr unsigned kAllFlags = KIFMM_POTENTIAL | KIFMM_GRADIENT | KIFMM_SERIAL | KIFMM_M2L_BF16X3 |
                               KIFMM_M2L_BF16X6 | KIFMM_VJP | KIFMM_M2L_BLOCKED | KIFMM_M2L_GATHER |
                               KIFMM_UPPER_STREAM | KIFMM_NO_UPPER_STREAM | KIFMM_LEAF_THREADS_256 |
                               KIFMM_LEAF_THREADS_320 | KIFMM_LEAF_QUEUE | KIFMM_LEAF_BLOCKS | KIFMM_NO_AUTOTUNE;

void check_plan_args(Tree* tree, Ops* ops, int nrhs, unsigned flags) {
  require(tree && ops, "null tree or ops");
  require((flags & ~kAllFlags) == 0 && (flags & (KIFMM_POTENTIAL | KIFMM_GRADIENT)) != 0,
          "flags must hold POTENTIAL and/or GRADIENT plus only the documented KIFMM_ flags");
  require(!((flags & KIFMM_M2L_BF16X3) && (flags & KIFMM_M2L_BF16X6)), "M2L_BF16X3 and M2L_BF16X6 exclude each other");
  require(nrhs == 1 || nrhs == 2 || nrhs == 4 || nrhs == 8 || nrhs == 16 || nrhs == 32,
          "nrhs must be 1, 2, 4, 8, 16 or 32");
  require(!((flags & KIFMM_M2L_BLOCKED) && (flags & KIFMM_M2L_GATHER)), "M2L_BLOCKED and M2L_GATHER exclude each other");
  require(!((flags & KIFMM_UPPER_STREAM) && (flags & KIFMM_NO_UPPER_STREAM)),
          "UPPER_STREAM and NO_UPPER_STREAM exclude each other");
  require(!((flags & KIFMM_LEAF_THREADS_256) && (flags & KIFMM_LEAF_THREADS_320)),
          "LEAF_THREADS_256 and LEAF_THREADS_320 exclude each other");
  require(!((flags & KIFMM_LEAF_QUEUE) && (flags & KIFMM_LEAF_BLOCKS)), "LEAF_QUEUE and LEAF_BLOCKS exclude each other");
  require(!(flags & KIFMM_M2L_GATHER) || (nrhs == 1 && !(flags & (KIFMM_M2L_BF16X3 | KIFMM_M2L_BF16X6))),
          "M2L_GATHER needs one right-hand side and the FP32 M2L");
  require(nrhs == 1 || !(flags & (KIFMM_GRADIENT | KIFMM_VJP | KIFMM_LEAF_QUEUE)),
          "gradients, KIFMM_VJP and KIFMM_LEAF_QUEUE need nrhs = 1 (plans with more right-hand sides give potentials)");
  require(tree->depth < 2 || ops->n <= kMaxLeafSurface, "the leaf kernel supports p <= 8 when the tree has a far field");
}

// Median of a few timings.
double median(std::vector<double> v) {
  std::sort(v.begin(), v.end());
  return v.empty() ? 0.0 : v[v.size() / 2];
}

}  // namespace

Plan::~Plan() {
  if (on_device) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_up0) (void)hipEventDestroy(ev_up0);
    if (ev_up1) (void)hipEventDestroy(ev_up1);
    if (side) (void)hipStreamDestroy(side);
    if (up) (void)hipStreamDestroy(up);
    for (void* p : owned) (void)hipFree(p);
    (void)hipSetDevice(prev);
  }
  release(tree);
  release(ops);
}

Tree* build_tree_device(const float* xyz, int64_t n, int depth, const double* cube, hipStream_t st) {
  require(xyz != nullptr, "xyz is null");
  require(n >= 1 && n < (1ll << 31), "n must be in [1, 2^31)");
  require(depth >= 0 && depth <= KIFMM_MAX_DEPTH, "depth must be in [0, " + std::to_string(KIFMM_MAX_DEPTH) + "]");
  std::vector<float> host((size_t)3 * n);
  hip_check(hipMemcpyAsync(host.data(), xyz, host.size() * sizeof(float), hipMemcpyDeviceToHost, st),
            "copy of the points to the host");
  hip_check(hipStreamSynchronize(st), "copy of the points to the host");
  return build_tree(host.data(), n, depth, cube);
}

namespace {

// Host-side preparation of a plan: sizes, interaction tables and FP32 operators
// in their device layout, registered in `S`.  Touches no device.
void prepare(Plan* P, Staging& S) {
  const Tree& T = *P->tree;
  const Ops& O = *P->ops;
  const unsigned flags = P->flags;
  const int nrhs = P->nrhs;
  const int L = T.depth;
  P->L = L;
  P->N = T.n;
  P->far = L >= 2;
  P->n = O.n;
  P->nst = round_up(O.n, 4);
  P->k = O.k;
  P->m2l_pieces = (flags & KIFMM_M2L_BF16X3) ? 2 : (flags & KIFMM_M2L_BF16X6) ? 3 : 0;
  // M2L runs k in chunks of 8 (FP32) or 16 (bfloat16), with zero padding
  P->kst = round_up(O.k, P->m2l_pieces ? 16 : 8);
  P->kc = O.kc;
  P->kcst = round_up(O.kc, 4);

  // Slots per level and the slot of every non-empty box.
  std::vector<std::vector<int>> slot_of(L + 1);  // [level][compact index] -> local slot
  P->slots.assign(L + 1, 0);
  for (int l = 0; l <= L; ++l) {
    const auto& keys = T.keys[l];
    slot_of[l].resize(keys.size());
    if (l == 0) {
      P->slots[0] = 1;
      slot_of[0][0] = 0;
      continue;
    }
    P->slots[l] = 8 * (int64_t)T.keys[l - 1].size();
    int64_t parent = 0;
    for (size_t i = 0; i < keys.size(); ++i) {
      while (T.keys[l - 1][parent] != (keys[i] >> 3)) ++parent;
      slot_of[l][i] = (int)(8 * parent + (keys[i] & 7));
    }
  }
  const int64_t SL = P->slots[L];
  const int64_t NBL = (int64_t)T.keys[L].size();
  P->n_leaves = NBL;

  // Sorted points (xyz; the charge is written per evaluate) and order.
  {
    std::vector<float> pts4(4 * T.n);
    std::vector<int> order(T.n);
    for (int64_t s = 0; s < T.n; ++s) {
      const int64_t i = T.order[s];
      order[s] = (int)i;
      for (int d = 0; d < 3; ++d) pts4[4 * s + d] = T.xyz[3 * i + d];
      pts4[4 * s + 3] = 0.f;
    }
    S.data((void**)&P->d_pts, std::move(pts4));
    S.data((void**)&P->d_order, std::move(order));
  }

  // Leaf slots: CSR point ranges (empty slots have empty ranges) and centres as
  // two floats per coordinate (c = hi + lo), so that kernels can form
  // centre-relative coordinates with rounding relative to the box size.
  std::vector<int> start(SL + 1, 0), leaves(NBL);
  {
    std::vector<float> centers(8 * SL, 0.f);
    const double rL = T.radius(L);
    std::vector<int> cnt(SL, 0);
    for (int64_t i = 0; i < NBL; ++i) {
      const int s = slot_of[L][i];
      leaves[i] = s;
      cnt[s] = (int)(T.leaf_start[i + 1] - T.leaf_start[i]);
    }
    for (int64_t s = 0; s < SL; ++s) {
      start[s + 1] = start[s] + cnt[s];
      // every slot's centre, empty ones included (a slot is a child position of a known parent)
      int32_t pc[3] = {0, 0, 0};
      if (L > 0) morton_decode(T.keys[L - 1][s / 8], L - 1, pc);
      for (int d = 0; d < 3; ++d) {
        const int c = L > 0 ? 2 * pc[d] + (int)((s % 8) >> d & 1) : 0;
        const double v = (T.center[d] - T.half) + (2.0 * c + 1.0) * rL;
        const float hi = (float)v;
        centers[8 * s + d] = hi;
        centers[8 * s + 4 + d] = (float)(v - (double)hi);
      }
      centers[8 * s + 3] = (float)rL;
    }
    S.data((void**)&P->d_centers, std::move(centers));
  }
  S.data((void**)&P->d_start, start);
  S.data((void**)&P->d_leaves, leaves);

  // Leaf groups (the children of each non-empty parent, or the root alone when
  // L = 0) and the 4 x 4 x 4 block of leaves around each group that holds the
  // U lists of its members.
  const int64_t m = 1ll << L;
  const int64_t ngroups = L > 0 ? (int64_t)T.keys[L - 1].size() : 1;
  P->n_groups = ngroups;
  P->group_slots = L > 0 ? 8 : 1;
  std::vector<int> blk(64 * ngroups, -1);
  for (int64_t g = 0; g < ngroups; ++g) {
    int32_t pc[3] = {0, 0, 0};
    if (L > 0) morton_decode(T.keys[L - 1][g], L - 1, pc);
    for (int bz = 0; bz < 4; ++bz)
      for (int by = 0; by < 4; ++by)
        for (int bx = 0; bx < 4; ++bx) {
          const int64_t x = 2 * pc[0] - 1 + bx, y = 2 * pc[1] - 1 + by, z = 2 * pc[2] - 1 + bz;
          if (x < 0 || y < 0 || z < 0 || x >= m || y >= m || z >= m) continue;
          const int64_t j = T.find(L, morton_encode((uint32_t)x, (uint32_t)y, (uint32_t)z, L));
          if (j >= 0) blk[64 * g + bx + 4 * by + 16 * bz] = slot_of[L][j];
        }
  }
  // LDS capacity of the leaf kernel: the largest block's padded source count
  // (rounded up to 64), limited so that at least two workgroups fit on a CU.
  {
    int64_t most = 0;
    for (int64_t g = 0; g < ngroups; ++g) {
      int64_t tot = 0;
      for (int e = 0; e < 64; ++e) {
        const int sl = blk[64 * g + e];
        if (sl >= 0) tot += (start[sl + 1] - start[sl] + 3) & ~3;
      }
      most = std::max(most, tot);
    }
    const int64_t budget = (72 * 1024 - (int64_t)O.n * 16 - 8 * (int64_t)O.n * 4) / 16;
    P->p2p_cap = (int)std::max<int64_t>(64, std::min<int64_t>((most + 63) / 64 * 64, budget / 64 * 64));
  }
  // U-list pairs (target, source) per leaf, for throughput accounting and the
  // cost order of the work-queue tiles.
  std::vector<int64_t> leaf_sources(SL, 0);
  int64_t pairs = 0;
  for (int64_t i = 0; i < NBL; ++i) {
    int32_t c[3];
    morton_decode(T.keys[L][i], L, c);
    int64_t src = 0;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int64_t x = c[0] + dx, y = c[1] + dy, z = c[2] + dz;
          if (x < 0 || y < 0 || z < 0 || x >= m || y >= m || z >= m) continue;
          const int64_t j = T.find(L, morton_encode((uint32_t)x, (uint32_t)y, (uint32_t)z, L));
          if (j >= 0) src += T.leaf_start[j + 1] - T.leaf_start[j];
        }
    leaf_sources[slot_of[L][i]] = src;
    pairs += (T.leaf_start[i + 1] - T.leaf_start[i]) * src;
  }
  P->p2p_pairs = pairs;
  S.data((void**)&P->d_blk, std::move(blk));

  // Target tiles of the leaf sums: up to 64 consecutive points of one non-empty
  // leaf (32 for the 32-right-hand-side kernel), as (slot, first sorted point,
  // count, 0).  The work queue takes them longest first (U-list sources plus
  // surface points per target); the multi-RHS kernels take them in leaf order.
  std::vector<int> tk;
  std::vector<int64_t> cost;
  const int tile = nrhs > 1 ? kMultiTile(nrhs) : 64;
  for (int64_t i = 0; i < NBL; ++i) {
    const int s = leaves[i];
    const int c = start[s + 1] - start[s];
    for (int t0 = 0; t0 < c; t0 += tile) {
      tk.insert(tk.end(), {s, start[s] + t0, std::min(tile, c - t0), 0});
      cost.push_back(leaf_sources[s] + (P->far ? O.n : 0));
    }
  }
  const bool queue_possible = nrhs == 1 && !(flags & KIFMM_LEAF_BLOCKS);
  if (nrhs > 1 || queue_possible) {
    std::vector<int> tiles(tk.size());
    const size_t nt = tk.size() / 4;
    if (nrhs > 1) {
      tiles = tk;  // multi-RHS tasks: the first point is leaf-relative
      for (size_t t = 0; t < nt; ++t) tiles[4 * t + 1] -= start[tiles[4 * t]];
    } else {
      std::vector<size_t> idx(nt);
      for (size_t t = 0; t < nt; ++t) idx[t] = t;
      std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
      for (size_t t = 0; t < nt; ++t)
        for (int c = 0; c < 4; ++c) tiles[4 * t + c] = tk[4 * idx[t] + c];
    }
    P->n_tiles = (int)nt;
    if (nrhs > 1) {
      P->n_tasks = (int)nt;
      if (nt) S.data((void**)&P->d_tasks, std::move(tiles));
    } else if (nt) {
      S.data((void**)&P->d_tiles, std::move(tiles));
      S.zeros<int>((void**)&P->d_queue, 2 * kQueueInts);
    }
  }

  // Surface and operators (rounded once to FP32, zero-padded).
  {
    std::vector<float> surf(3 * O.n);
    for (int i = 0; i < 3 * O.n; ++i) surf[i] = (float)O.surf[i];
    S.data((void**)&P->d_surf, std::move(surf));
  }

  if (P->far) {
    const int n = O.n, nst = P->nst, k = O.k, kst = P->kst, kc = O.kc, kcst = P->kcst;
    // Level bases of the per-box arrays (levels 2..L).
    P->base.assign(L + 1, 0);
    int64_t total = 0;
    for (int l = 2; l <= L; ++l) {
      P->base[l] = total;
      total += P->slots[l];
    }
    P->total_slots = total;
    // Per-box arrays hold the nrhs right-hand sides one after the other: [nrhs][slots][row].
    const size_t R = (size_t)nrhs;
    S.zeros<float>((void**)&P->d_q, R * SL * nst);
    S.zeros<float>((void**)&P->d_t, R * SL * kcst);
    S.zeros<float>((void**)&P->d_u, R * total * nst);
    S.zeros<float>((void**)&P->d_d, R * total * nst);
    // one more zero row: the gathered M2L's source for "no source"
    S.zeros<float>((void**)&P->d_uhat, R * total * kst + kst);
    S.zeros<float>((void**)&P->d_chat, R * total * kst);
    // M2L partial sums, one per source position among siblings: [8][nrhs][total][kst]
    // (the wide 32-right-hand-side M2L writes chat directly and needs none).
    P->m2l_wide = nrhs == 32 && P->m2l_pieces == 0;
    if (!P->m2l_wide) S.zeros<float>((void**)&P->d_chat_part, 8 * R * total * kst);
    S.zeros<float>((void**)&P->d_zero, (size_t)kst + nst);

    auto pad_rows = [](int rows) { return round_up(rows, 64); };
    {
      // f1: [kc][n] -> W [pad(kcst)][nst]
      std::vector<float> w1((size_t)pad_rows(kcst) * nst, 0.f);
      for (int c = 0; c < kc; ++c)
        for (int i = 0; i < n; ++i) w1[(size_t)c * nst + i] = (float)O.f1[(size_t)c * n + i];
      S.data((void**)&P->d_f1, std::move(w1));
      // f2: [n][kc] -> W [pad(nst)][kcst]
      std::vector<float> w2((size_t)pad_rows(nst) * kcst, 0.f);
      for (int i = 0; i < n; ++i)
        for (int c = 0; c < kc; ++c) w2[(size_t)i * kcst + c] = (float)O.f2[(size_t)i * kc + c];
      S.data((void**)&P->d_f2, std::move(w2));
      // U2U: W[i][oc * nst + c] = M2M_oc[i][c]
      std::vector<float> wm((size_t)pad_rows(nst) * 8 * nst, 0.f);
      for (int oc = 0; oc < 8; ++oc)
        for (int i = 0; i < n; ++i)
          for (int c = 0; c < n; ++c)
            wm[(size_t)i * 8 * nst + oc * nst + c] = (float)O.m2m[((size_t)oc * n + i) * n + c];
      S.data((void**)&P->d_m2m, std::move(wm));
      // compression: W[c][i] = V_k[i][c]
      std::vector<float> wv((size_t)pad_rows(kst) * nst, 0.f);
      for (int c = 0; c < k; ++c)
        for (int i = 0; i < n; ++i) wv[(size_t)c * nst + i] = (float)O.mv[(size_t)i * k + c];
      S.data((void**)&P->d_vt, std::move(wv));
      // post: W[i][c] = (DC2E U_k)[i][c]
      std::vector<float> wp((size_t)pad_rows(nst) * kst, 0.f);
      for (int i = 0; i < n; ++i)
        for (int c = 0; c < k; ++c) wp[(size_t)i * kst + c] = (float)O.post[(size_t)i * k + c];
      S.data((void**)&P->d_post, std::move(wp));
      // D2D: W[oc * nst + i][c] = L2L_oc[i][c]
      std::vector<float> wl((size_t)pad_rows(8 * nst) * nst, 0.f);
      for (int oc = 0; oc < 8; ++oc)
        for (int i = 0; i < n; ++i)
          for (int c = 0; c < n; ++c)
            wl[((size_t)oc * nst + i) * nst + c] = (float)O.l2l[((size_t)oc * n + i) * n + c];
      S.data((void**)&P->d_l2l, std::move(wl));
    }
    // M2L cores, rows padded to whole 32-row blocks (one wave each) and stored in
    // the matrix-core lane order of k_m2l: [316][row block][k chunk of 8][lane][4],
    // where lane (i, h) = (l % 32, l / 32) holds C[32 rb + i][8 c + 4 h .. + 3].
    // One wave's operand load for a chunk is then 1 KiB of contiguous memory.
    P->m2l_rb = (kst + 31) / 32;
    P->core_rows = 32 * P->m2l_rb;
    require(P->m2l_rb <= 8, "M2L rank too large for the M2L kernel (k <= 256)");
    if (!P->m2l_pieces) {
      const int nchunk = kst / 8;
      std::vector<float> wc((size_t)kNumOffsets * P->core_rows * kst, 0.f);
      for (int t = 0; t < kNumOffsets; ++t)
        for (int a = 0; a < k; ++a)
          for (int b = 0; b < k; ++b) {
            const size_t chunk = ((size_t)t * P->m2l_rb + a / 32) * nchunk + b / 8;
            const int lane = (a % 32) + 32 * ((b % 8) / 4);
            wc[(chunk * 64 + lane) * 4 + b % 4] = (float)O.cores[((size_t)t * k + a) * k + b];
          }
      S.data((void**)&P->d_cores, std::move(wc));
    } else {
      // Split-bfloat16 cores: C = C_0 + C_1 (+ C_2), C_0 the bfloat16 rounding
      // of C (to nearest, ties to even) and each further piece that of the
      // FP64 remainder.  Layout [316][row block][16-k chunk][piece][64 lanes][8],
      // lane (i, h) holding C[32 rb + i][16 c + 8 h .. + 7], so that one wave's
      // load of a piece of a chunk is 1 KiB of contiguous memory.
      const int nchunk = kst / 16;
      auto split_cores = [&](int np, size_t& stride16) {
        stride16 = (size_t)P->m2l_rb * nchunk * 64 * np;
        std::vector<uint16_t> wb((size_t)kNumOffsets * stride16 * 8, 0);
        for (int t = 0; t < kNumOffsets; ++t)
          for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) {
              double rem = O.cores[((size_t)t * k + a) * k + b];
              const size_t chunk = ((size_t)t * P->m2l_rb + a / 32) * nchunk + b / 16;
              const int lane = (a % 32) + 32 * ((b % 16) / 8);
              for (int q = 0; q < np; ++q) {
                const uint16_t piece = bf16_round(rem);
                rem -= bf16_value(piece);
                wb[((chunk * np + q) * 64 + lane) * 8 + b % 8] = piece;
              }
            }
        return wb;
      };
      S.data((void**)&P->d_cores_b, split_cores(P->m2l_pieces, P->core_stride16));
      // The three-product form runs the levels above the leaves with six products:
      // their translations carry the far field of many more sources (its magnitude
      // grows about as 2^(L-l)/2 towards the root for charges of random sign), so
      // their product error dominates the result's while they hold about an eighth
      // of the translations.
      if (P->m2l_pieces == 2 && L > 2) S.data((void**)&P->d_cores_b3, split_cores(3, P->core_stride16_3));
    }

    // Per-level lists of non-empty boxes' slots (U2U scatter, D2D gather).
    P->d_nbslot.assign(L + 1, nullptr);
    for (int l = 2; l <= L; ++l) S.data((void**)&P->d_nbslot[l], slot_of[l]);
    {
      std::vector<int> ne;
      for (int l = 2; l <= L; ++l)
        for (int sl : slot_of[l]) ne.push_back((int)(P->base[l] + sl));
      P->n_nonempty = (int)ne.size();
      S.data((void**)&P->d_nonempty, std::move(ne));
    }

    // VLI work items (see k_m2l).  For target position o and source position o'
    // (x bit 0, y bit 1, z bit 2) the V-list offsets are the parent shifts d in
    // {-1,0,1}^3 whose offset t = o - o' - 2 d (per axis) has max |t| >= 2
    // (Table 1: children of the parent's colleagues, not adjacent).
    std::vector<int> pair_offs(64 * 27, 0), pair_cnt(64, 0);
    {
      auto offset_index = [&](int tx, int ty, int tz) {
        for (int t = 0; t < kNumOffsets; ++t)
          if (O.offsets[3 * t] == tx && O.offsets[3 * t + 1] == ty && O.offsets[3 * t + 2] == tz) return t;
        fail(KIFMM_E_INVALID, "internal: V-list offset not in the operator table");
      };
      int total_offs = 0;
      for (int o = 0; o < 8; ++o)
        for (int o2 = 0; o2 < 8; ++o2) {
          const int pr = 8 * o + o2;
          for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
              for (int dx = -1; dx <= 1; ++dx) {
                const int t[3] = {(o & 1) - (o2 & 1) - 2 * dx, ((o >> 1) & 1) - ((o2 >> 1) & 1) - 2 * dy,
                                  ((o >> 2) & 1) - ((o2 >> 2) & 1) - 2 * dz};
                if (std::max({std::abs(t[0]), std::abs(t[1]), std::abs(t[2])}) < 2) continue;
                const int e = (dx + 1) + 6 * (dy + 1) + 36 * (dz + 1);
                pair_offs[27 * pr + pair_cnt[pr]++] = offset_index(t[0], t[1], t[2]) | (e << 9);
              }
          total_offs += pair_cnt[pr];
        }
      require(total_offs == 8 * kOffsetsPerOctant, "internal: V-list offsets per position != 189");
    }
    std::vector<int> tgt_blk, src_blk;
    // items of the leaf level and of the levels above it, kept apart so that the
    // upper levels can run beside the leaf level's M2L (see evaluate_plan)
    std::vector<std::vector<M2LItem>> per_xcd_l[2] = {std::vector<std::vector<M2LItem>>(8),
                                                       std::vector<std::vector<M2LItem>>(8)};
    int64_t vpairs = 0, ntargets = 0, vpairs_leaf = 0;
    for (int l = L; l >= 2; --l) {
      auto& per_xcd = per_xcd_l[l == L ? 0 : 1];
      const int64_t mp = 1ll << (l - 1);  // parents per axis
      const int64_t ml = 1ll << l;
      // aligned 4x4x4 blocks of parents that hold at least one non-empty parent
      std::vector<uint64_t> blocks;
      for (uint64_t pk : T.keys[l - 1]) {
        const uint64_t bk = pk >> 6;
        if (blocks.empty() || blocks.back() != bk) blocks.push_back(bk);
      }
      for (uint64_t bk : blocks) {
        int32_t bc[3];
        morton_decode(bk, std::max(l - 3, 0), bc);
        const int64_t px0 = 4 * (int64_t)bc[0], py0 = 4 * (int64_t)bc[1], pz0 = 4 * (int64_t)bc[2];
        auto box_slot = [&](int64_t x, int64_t y, int64_t z) -> int {
          if (x < 0 || y < 0 || z < 0 || x >= ml || y >= ml || z >= ml) return -1;
          const int64_t j = T.find(l, morton_encode((uint32_t)x, (uint32_t)y, (uint32_t)z, l));
          return j < 0 ? -1 : (int)(P->base[l] + slot_of[l][j]);
        };
        int src_base[8];
        for (int o2 = 0; o2 < 8; ++o2) {
          src_base[o2] = (int)src_blk.size();
          for (int ez = 0; ez < 6; ++ez)
            for (int ey = 0; ey < 6; ++ey)
              for (int ex = 0; ex < 6; ++ex) {
                const int64_t x = px0 - 1 + ex, y = py0 - 1 + ey, z = pz0 - 1 + ez;
                const bool inside = x >= 0 && y >= 0 && z >= 0 && x < mp && y < mp && z < mp;
                src_blk.push_back(inside ? box_slot(2 * x + (o2 & 1), 2 * y + ((o2 >> 1) & 1),
                                                    2 * z + ((o2 >> 2) & 1))
                                         : -1);
              }
        }
        for (int o = 0; o < 8; ++o) {
          const int tgt_base = (int)tgt_blk.size();
          int count = 0;
          for (int pi = 0; pi < 64; ++pi) {
            const int64_t x = px0 + (pi & 3), y = py0 + ((pi >> 2) & 3), z = pz0 + (pi >> 4);
            const bool inside = x < mp && y < mp && z < mp;
            const int sl = inside ? box_slot(2 * x + (o & 1), 2 * y + ((o >> 1) & 1), 2 * z + ((o >> 2) & 1)) : -1;
            tgt_blk.push_back(sl);
            if (sl < 0) continue;
            ++count;
            // V-list pairs of this target, for accounting
            for (int o2 = 0; o2 < 8; ++o2)
              for (int j = 0; j < pair_cnt[8 * o + o2]; ++j) {
                const int e = pair_offs[27 * (8 * o + o2) + j] >> 9;
                const int ex = e % 6, ey = (e / 6) % 6, ez = e / 36;  // (d + 1) per axis, in 0..2
                const int r = ((pi & 3) + ex) + 6 * (((pi >> 2) & 3) + ey) + 36 * ((pi >> 4) + ez);
                vpairs += src_blk[src_base[o2] + r] >= 0;
                if (l == L) vpairs_leaf += src_blk[src_base[o2] + r] >= 0;
              }
          }
          if (!count) {
            tgt_blk.resize(tgt_base);
            continue;
          }
          ntargets += count;
          // items of one (o, o') pair go to one XCD: source position o' -> XCD o'
          for (int o2 = 0; o2 < 8; ++o2)
            per_xcd[o2].push_back(M2LItem{8 * o + o2, pair_cnt[8 * o + o2], o2, tgt_base, src_base[o2]});
        }
      }
    }
    // Workgroups are dealt to the 8 XCDs round-robin: item b runs on XCD b % 8.
    // Within an XCD's list, items are ordered by (o, o') pair, so that the XCD's
    // L2 holds the ~24 translation cores of the pair its CUs are working on, and
    // pairs with more offsets (longer items) come first, so the end of the grid
    // is made of short items.
    std::vector<M2LItem> items;
    for (int part = 0; part < 2; ++part) {
      auto& per_xcd = per_xcd_l[part];
      for (auto& v : per_xcd)
        std::stable_sort(v.begin(), v.end(), [](const M2LItem& a, const M2LItem& b) {
          return a.noffs != b.noffs ? a.noffs > b.noffs : a.pair < b.pair;
        });
      size_t most = 0;
      for (auto& v : per_xcd) most = std::max(most, v.size());
      for (size_t i = 0; i < most; ++i)
        for (int x = 0; x < 8; ++x)
          if (i < per_xcd[x].size()) items.push_back(per_xcd[x][i]);
      if (part == 0) P->n_items_leaf = (int)items.size();
    }
    P->m2l_pairs = vpairs;
    P->m2l_pairs_leaf = vpairs_leaf;
    P->m2l_targets = ntargets;
    P->n_items = (int)items.size();
    // k per LDS slab of the staged sources (row stride slab + 4 floats, an odd
    // number of 16-byte units): the most resident waves per CU first (at most
    // 16 for the kernel's register use; rb waves per workgroup, 216 rows of
    // LDS each), then the fewest slabs.  (Timed at k = 94 on the 1M cube: 5,
    // 4 and 3 workgroups per CU take 1.21, 1.34 and 1.38 ms.)
    {
      int best_slab = 0, best_waves = -1, best_n = 0;
      for (int slab = 24; slab <= 48; slab += 8) {
        const int lds = 216 * (slab + 4) * 4;
        const int waves = std::min(16 / P->m2l_rb, (160 * 1024) / lds) * P->m2l_rb;
        const int nsl = (P->kst + slab - 1) / slab;
        if (waves > best_waves || (waves == best_waves && nsl < best_n)) {
          best_slab = slab;
          best_waves = waves;
          best_n = nsl;
        }
      }
      P->m2l_lds_ld = best_slab + 4;
    }
    S.data((void**)&P->d_pair_offs, std::move(pair_offs));
    S.data((void**)&P->d_tgt_blk, std::move(tgt_blk));
    S.data((void**)&P->d_src_blk, std::move(src_blk));
    S.data((void**)&P->d_items, std::move(items));
    P->keys_per_level.assign(L + 1, 0);
    for (int l = 0; l <= L; ++l) P->keys_per_level[l] = (int64_t)T.keys[l].size();

    // Explicit per-target V lists (Table 1: children of the parent's colleagues,
    // not adjacent, non-empty) as (core index, source slot), for the wide and
    // the gathered M2L forms.
    // The gathered form pays off only where most blocked columns would be empty
    // (sparse trees); on trees whose leaf slots are mostly full it is not built.
    const bool sparse = (double)NBL < 0.6 * (double)SL;
    const bool want_gather = nrhs == 1 && P->m2l_pieces == 0 && !(flags & KIFMM_M2L_BLOCKED) &&
                             ((flags & KIFMM_M2L_GATHER) || sparse);
    if (P->m2l_wide || want_gather) {
      std::vector<int> idx7(343, -1);
      for (int t = 0; t < kNumOffsets; ++t)
        idx7[(O.offsets[3 * t] + 3) + 7 * (O.offsets[3 * t + 1] + 3) + 49 * (O.offsets[3 * t + 2] + 3)] = t;
      std::vector<int> vl;
      std::vector<int64_t> tgt_first, tgt_end;
      std::vector<int> tgt_slot, tgt_pos, tgt_level;
      for (int l = 2; l <= L; ++l) {
        const int64_t mp = 1ll << (l - 1), ml = 1ll << l;
        for (size_t i = 0; i < T.keys[l].size(); ++i) {
          int32_t c[3];
          morton_decode(T.keys[l][i], l, c);
          const int64_t first = (int64_t)vl.size() / 2;
          for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
              for (int dx = -1; dx <= 1; ++dx) {
                const int64_t qx = (c[0] >> 1) + dx, qy = (c[1] >> 1) + dy, qz = (c[2] >> 1) + dz;
                if (qx < 0 || qy < 0 || qz < 0 || qx >= mp || qy >= mp || qz >= mp) continue;
                for (int o2 = 0; o2 < 8; ++o2) {
                  const int64_t sx = 2 * qx + (o2 & 1), sy = 2 * qy + ((o2 >> 1) & 1), sz = 2 * qz + (o2 >> 2);
                  const int64_t tx = c[0] - sx, ty = c[1] - sy, tz = c[2] - sz;
                  if (std::max({std::llabs(tx), std::llabs(ty), std::llabs(tz)}) < 2) continue;
                  if (sx >= ml || sy >= ml || sz >= ml) continue;
                  const int64_t jj = T.find(l, morton_encode((uint32_t)sx, (uint32_t)sy, (uint32_t)sz, l));
                  if (jj < 0) continue;
                  const int t = idx7[(tx + 3) + 7 * (ty + 3) + 49 * (tz + 3)];
                  require(t >= 0, "internal: V-list offset not in the operator table");
                  vl.push_back(t);
                  vl.push_back((int)(P->base[l] + slot_of[l][jj]));
                }
              }
          tgt_first.push_back(first);
          tgt_end.push_back((int64_t)vl.size() / 2);
          tgt_slot.push_back((int)(P->base[l] + slot_of[l][i]));
          tgt_pos.push_back((int)(T.keys[l][i] & 7));
          tgt_level.push_back(l);
        }
      }
      require(vl.size() / 2 < (size_t)INT32_MAX, "V lists too long for the M2L tables");
      // Units (w ints each) are dealt to XCDs by the target's position among its
      // siblings: an XCD then works through the ~189 cores of one position.
      auto deal = [&](const std::vector<std::vector<int>>& ux, size_t w = 4) {
        std::vector<int> units;
        size_t most = 0;
        for (auto& v : ux) most = std::max(most, v.size() / w);
        for (size_t i = 0; i < most; ++i)
          for (int x = 0; x < 8; ++x)
            if (i < ux[x].size() / w) units.insert(units.end(), ux[x].begin() + w * i, ux[x].begin() + w * (i + 1));
        return units;
      };
      if (P->m2l_wide) {
        // Wide form: targets of one level and position paired in Morton order; per
        // pair the entries (core, source of the first target or -1, source of the
        // second or -1, 0) of the offsets both have, then of those of the first
        // alone, then of those of the second alone, each run in core order; one
        // unit (workgroup) per pair: (slot 0, slot 1 or -1, first, end entry) and
        // (end of the first run, end of the second run, 0, 0).
        std::vector<int> ents, ux_all[8];
        std::vector<std::pair<int, int>> la, lb;
        auto sorted_list = [&](size_t i, std::vector<std::pair<int, int>>& out) {
          out.clear();
          for (int64_t e = tgt_first[i]; e < tgt_end[i]; ++e) out.push_back({vl[2 * e], vl[2 * e + 1]});
          std::sort(out.begin(), out.end());
        };
        for (int l = 2; l <= L; ++l)
          for (int x = 0; x < 8; ++x) {
            std::vector<size_t> members;
            for (size_t i = 0; i < tgt_slot.size(); ++i)
              if (tgt_level[i] == l && tgt_pos[i] == x) members.push_back(i);
            for (size_t m = 0; m < members.size(); m += 2) {
              const bool two = m + 1 < members.size();
              sorted_list(members[m], la);
              if (two) sorted_list(members[m + 1], lb);
              else lb.clear();
              // entries of both targets, then of target 0 alone, then of target 1 alone
              const int first = (int)(ents.size() / 4);
              std::vector<int> only0, only1;
              size_t ia = 0, ib = 0;
              while (ia < la.size() || ib < lb.size()) {
                const int ta = ia < la.size() ? la[ia].first : INT32_MAX;
                const int tb = ib < lb.size() ? lb[ib].first : INT32_MAX;
                if (ta == tb) {
                  ents.insert(ents.end(), {ta, la[ia].second, lb[ib].second, 0});
                  ++ia;
                  ++ib;
                } else if (ta < tb) {
                  only0.insert(only0.end(), {ta, la[ia].second, -1, 0});
                  ++ia;
                } else {
                  only1.insert(only1.end(), {tb, -1, lb[ib].second, 0});
                  ++ib;
                }
              }
              const int pair_end = (int)(ents.size() / 4);
              ents.insert(ents.end(), only0.begin(), only0.end());
              const int t0_end = (int)(ents.size() / 4);
              ents.insert(ents.end(), only1.begin(), only1.end());
              ux_all[x].insert(ux_all[x].end(), {tgt_slot[members[m]], two ? tgt_slot[members[m + 1]] : -1, first,
                                                 (int)(ents.size() / 4), pair_end, t0_end, 0, 0});
            }
          }
        require(ents.size() / 4 < (size_t)INT32_MAX, "V lists too long for the M2L tables");
        std::vector<int> units = deal(std::vector<std::vector<int>>(ux_all, ux_all + 8), 8);
        P->n_units = (int)(units.size() / 8);
        P->n_wide_entries = (int64_t)(ents.size() / 4);
        S.data((void**)&P->d_wents, std::move(ents));
        S.data((void**)&P->d_units, std::move(units));
      } else {
        // Gathered form: groups of up to 32 targets of one level and position; per
        // group the union of their offsets (ascending core index) and, per offset,
        // each target's source row (the zero row total_slots where it has none).
        std::vector<int> ent_core, ent_src, gtgt;
        std::vector<std::vector<int>> ux_leaf(8), ux_upper(8);
        std::vector<int> lane_src((size_t)kNumOffsets * 32);
        std::vector<char> used(kNumOffsets);
        const int zero_row = (int)total;
        for (int l = 2; l <= L; ++l)
          for (int x = 0; x < 8; ++x) {
            auto& ux = l == L ? ux_leaf : ux_upper;
            std::vector<int> members;
            for (size_t i = 0; i < tgt_slot.size(); ++i)
              if (tgt_level[i] == l && tgt_pos[i] == x) members.push_back((int)i);
            for (size_t g0 = 0; g0 < members.size(); g0 += 32) {
              const int g = (int)(gtgt.size() / 32);
              std::fill(lane_src.begin(), lane_src.end(), zero_row);
              std::fill(used.begin(), used.end(), 0);
              for (int jl = 0; jl < 32; ++jl) {
                const bool real = g0 + jl < members.size();
                const int i = real ? members[g0 + jl] : -1;
                gtgt.push_back(real ? tgt_slot[i] : -1);
                if (!real) continue;
                for (int64_t e = tgt_first[i]; e < tgt_end[i]; ++e) {
                  const int t = vl[2 * e];
                  used[t] = 1;
                  lane_src[(size_t)t * 32 + jl] = vl[2 * e + 1];
                }
              }
              const int first = (int)ent_core.size();
              for (int t = 0; t < kNumOffsets; ++t) {
                if (!used[t]) continue;
                ent_core.push_back(t);
                ent_src.insert(ent_src.end(), lane_src.begin() + (size_t)t * 32, lane_src.begin() + (size_t)t * 32 + 32);
              }
              const int end = (int)ent_core.size();
              for (int rb = 0; rb < P->m2l_rb; ++rb) ux[x].insert(ux[x].end(), {g, rb, first, end});
            }
          }
        std::vector<int> units = deal(ux_leaf);
        P->n_gunits_leaf = (int)(units.size() / 4);
        const std::vector<int> upper = deal(ux_upper);
        units.insert(units.end(), upper.begin(), upper.end());
        P->n_gunits = (int)(units.size() / 4);
        S.data((void**)&P->d_gent_core, std::move(ent_core));
        S.data((void**)&P->d_gent_src, std::move(ent_src));
        S.data((void**)&P->d_gtgt, std::move(gtgt));
        S.data((void**)&P->d_gunits, std::move(units));
        P->m2l_gather = (flags & KIFMM_M2L_GATHER) != 0;
      }
    }
  }
  P->slot_of = std::move(slot_of);
  if (nrhs > 1) S.zeros<float>((void**)&P->d_qs, (size_t)nrhs * T.n);
  // Streams of the plan: the U-list sum (one right-hand side, not serial, with a
  // far field) and the levels above the leaves (depth >= 3).
  P->want_up = P->far && !(flags & (KIFMM_SERIAL | KIFMM_NO_UPPER_STREAM)) && nrhs == 1 && L >= 3;
  P->want_side = P->far && !(flags & KIFMM_SERIAL) && nrhs == 1;
  if (P->want_side) S.zeros<float>((void**)&P->d_near, 4 * (size_t)T.n);
  if (flags & KIFMM_VJP) {
    S.zeros<float>((void**)&P->d_vjp_fs, 3 * (size_t)T.n);
    S.zeros<float>((void**)&P->d_vjp_fw, 3 * (size_t)T.n);
  }
  P->p2p_threads = (flags & KIFMM_LEAF_THREADS_256) ? 256 : kP2PMaxThreads;
}

// Buffers of the plan-time timing (zero charges, outputs), freed afterwards.
int64_t tuning_bytes(const Plan* P) {
  if (P->nrhs != 1) return 0;
  const int64_t n = P->N;
  return Staging::padded(4 * n) * 2 + ((P->flags & KIFMM_GRADIENT) ? Staging::padded(12 * n) : 0);
}

// Whether every launch of the plan has a kernel instance (checked once here, so
// that an evaluate cannot fail part-way through its launches).
void check_launches(const Plan* P) {
  if (!p2p_supported(P->p2p_threads, P->p2p_cap, P->n) || !p2p_supported(256, P->p2p_cap, P->n))
    fail(KIFMM_E_INVALID, "leaf kernel configuration not available for this tree and order");
  if (P->far) {
    if (!p2m_supported(P->n)) fail(KIFMM_E_INVALID, "the S2U kernel supports at most 768 surface points");
    const bool ok = P->m2l_pieces ? m2l_bf16_supported(P->m2l_pieces, P->m2l_rb, P->kst) &&
                                        m2l_bf16_supported(3, P->m2l_rb, P->kst)
                                  : m2l_supported(P->m2l_rb, P->kst, P->m2l_lds_ld);
    if (!ok) fail(KIFMM_E_INVALID, "M2L kernel configuration not available for this rank");
    if (P->m2l_wide && P->m2l_rb > 8) fail(KIFMM_E_INVALID, "M2L rank too large for the wide M2L kernel");
  }
}

}  // namespace

Plan* create_plan(Tree* tree, Ops* ops, int nrhs, unsigned flags, hipStream_t st) {
  check_plan_args(tree, ops, nrhs, flags);
  Plan* P = new Plan();
  tree->refs.fetch_add(1);
  ops->refs.fetch_add(1);
  P->tree = tree;
  P->ops = ops;
  P->flags = flags;
  P->nrhs = nrhs;
  try {
    Staging S;
    prepare(P, S);
    check_launches(P);
    const int64_t need = S.total + tuning_bytes(P);
    const int64_t limit = device_memory_limit();
    if (limit > 0 && need > limit)
      fail(KIFMM_E_NOMEM, "the plan needs " + std::to_string(need) + " device bytes, above the limit of " +
                              std::to_string(limit) + " set by kifmm_set_device_memory_limit");

    // The device of the stream (the current one for the null stream).
    int device = 0;
    if (st) hip_check(hipStreamGetDevice(st, &device), "hipStreamGetDevice");
    else hip_check(hipGetDevice(&device), "hipGetDevice");
    P->device = device;
    DeviceScope scope(device);
    configure_device(device);
    P->on_device = true;
    for (auto& it : S.items) {
      void* p = nullptr;
      hip_check(hipMalloc(&p, it.bytes), "plan allocation");
      P->owned.push_back(p);
      *it.dst = p;
      if (it.copy_bytes) hip_check(hipMemcpyAsync(p, it.data, it.copy_bytes, hipMemcpyHostToDevice, st), "plan upload");
      else hip_check(hipMemsetAsync(p, 0, it.bytes, st), "plan upload");
    }
    hip_check(hipStreamSynchronize(st), "plan upload");
    S.items.clear();
    if (P->want_up) {
      // the levels above the leaves run on a second plan stream (default priority)
      hip_check(hipStreamCreateWithFlags(&P->up, hipStreamNonBlocking), "hipStreamCreate");
      hip_check(hipEventCreateWithFlags(&P->ev_up0, hipEventDisableTiming), "hipEventCreate");
      hip_check(hipEventCreateWithFlags(&P->ev_up1, hipEventDisableTiming), "hipEventCreate");
    }
    if (P->want_side) {
      hip_check(hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking), "hipStreamCreate");
      hip_check(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming), "hipEventCreate");
      hip_check(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming), "hipEventCreate");
    }
    hip_check(hipDeviceGetAttribute(&P->n_cus, hipDeviceAttributeMultiprocessorCount, device),
              "hipDeviceGetAttribute");
    autotune(P, st);
  } catch (...) {
    delete P;
    throw;
  }
  return P;
}

int64_t plan_workspace_bytes(Tree* tree, Ops* ops, int nrhs, unsigned flags) {
  check_plan_args(tree, ops, nrhs, flags);
  Plan* P = new Plan();
  tree->refs.fetch_add(1);
  ops->refs.fetch_add(1);
  P->tree = tree;
  P->ops = ops;
  P->flags = flags;
  P->nrhs = nrhs;
  int64_t bytes = 0;
  try {
    Staging S;
    prepare(P, S);
    check_launches(P);
    bytes = S.total + tuning_bytes(P);
  } catch (...) {
    delete P;
    throw;
  }
  delete P;
  return bytes;
}

void plan_stats(const Plan* P, int64_t* v) {
  const int64_t form = P->m2l_pieces ? 3 : P->m2l_wide ? 2 : P->m2l_gather ? 1 : 0;
  const bool up = P->up && P->up_on;
  auto us = [](double ms) { return (int64_t)std::llround(ms * 1000.0); };
  const int64_t vals[KIFMM_N_STATS] = {
      P->p2p_pairs, P->m2l_pairs, P->far ? P->slots[P->L] : 0, P->m2l_targets, P->k, P->n, P->nrhs, form,
      up ? P->m2l_pairs_leaf : P->m2l_pairs, up ? 1 : 0,
      form == 0 ? P->m2l_lds_ld - 4 : form == 3 ? 32 : 0,
      P->nrhs == 1 ? P->p2p_threads : 0,
      P->leaf_queue ? 1 : 0, P->leaf_queue ? P->n_tiles : 0,
      us(P->tune_ms[0][0]), us(P->tune_ms[0][1]), us(P->tune_ms[1][0]), us(P->tune_ms[1][1]),
      us(P->m2l_tune_ms[0]), us(P->m2l_tune_ms[1]), us(P->leaf_tune_ms[0]), us(P->leaf_tune_ms[1]),
      P->m2l_pairs_leaf, P->tuned_from_cache ? 1 : 0, P->leaf_queue ? P->queue_per_cu : 0,
      us(P->slab_tune_ms[0]), us(P->slab_tune_ms[1]), us(P->slab_tune_ms[2]), us(P->slab_tune_ms[3])};
  for (int i = 0; i < KIFMM_N_STATS; ++i) v[i] = vals[i];
}

void Plan::set_timing(bool on) {
  if (on && ev.empty()) {
    // the events are created here, so that evaluates create nothing
    DeviceScope scope(device);
    std::vector<hipEvent_t> made((size_t)kRing * KIFMM_N_STAGES * 2, nullptr);
    for (auto& e : made) {
      const hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) {
        for (auto& d : made)
          if (d) (void)hipEventDestroy(d);
        hip_check(err, "hipEventCreate");
      }
    }
    ev = std::move(made);
    recorded.assign((size_t)kRing * KIFMM_N_STAGES, 0);
  }
  if (!on && timing) collect_times();
  timing = on;
}

void Plan::timing_begin_call() {
  ring_slot = -1;
  if (!timing) return;
  if (ring_used == kRing) collect_times();
  ring_slot = ring_used++;
}

void Plan::stage_begin(int s, hipStream_t st) {
  if (ring_slot < 0) return;
  hip_check(hipEventRecord(ev[((size_t)ring_slot * KIFMM_N_STAGES + s) * 2], st), "hipEventRecord");
}

void Plan::stage_end(int s, hipStream_t st) {
  if (ring_slot < 0) return;
  hip_check(hipEventRecord(ev[((size_t)ring_slot * KIFMM_N_STAGES + s) * 2 + 1], st), "hipEventRecord");
  recorded[(size_t)ring_slot * KIFMM_N_STAGES + s] = 1;
}

void Plan::collect_times() {
  for (int c = 0; c < ring_used; ++c)
    for (int s = 0; s < KIFMM_N_STAGES; ++s) {
      unsigned char& r = recorded[(size_t)c * KIFMM_N_STAGES + s];
      if (!r) continue;
      const size_t e = ((size_t)c * KIFMM_N_STAGES + s) * 2;
      hip_check(hipEventSynchronize(ev[e + 1]), "hipEventSynchronize");
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, ev[e], ev[e + 1]), "hipEventElapsedTime");
      stage_ms[s] += ms;
      stage_count[s] += 1;
      r = 0;
    }
  ring_used = 0;
}

// The M2L launch of the plan's form (uhat -> chat, or -> the partial sums that
// k_sum_parts adds), for all target levels (part 0), the leaf level (part 1) or
// the levels above it (part 2).  False if no kernel instance fits.
bool launch_m2l_form(Plan* P, hipStream_t st, int part) {
  const int kst = P->kst, R = P->nrhs;
  const long long TS = P->total_slots;
  if (P->m2l_wide) {
    if (part == 2) return true;
    return launch_m2l_wide(P->m2l_rb, P->d_cores, (long long)P->core_rows * kst, kst, P->d_units, P->n_units,
                           P->d_wents, P->d_uhat, P->d_chat, TS * kst, st);
  }
  if (P->m2l_gather) {
    const int u0 = part == 2 ? P->n_gunits_leaf : 0;
    const int u1 = part == 1 ? P->n_gunits_leaf : P->n_gunits;
    launch_m2l_gather(P->d_cores, (long long)P->core_rows * kst, kst, P->d_gunits + u0, u1 - u0, P->d_gent_core,
                      P->d_gent_src, P->d_gtgt, P->d_uhat, P->d_chat, st, part == 2);
    return true;
  }
  const int i0 = part == 2 ? P->n_items_leaf : 0;
  const int i1 = part == 1 ? P->n_items_leaf : P->n_items;
  if (P->m2l_pieces == 2 && P->d_cores_b3) {
    // three products at the leaf level, six above it
    const int split = P->n_items_leaf;
    bool ok = true;
    if (i0 < split)
      ok = launch_m2l_bf16(2, P->m2l_rb, P->d_cores_b, P->core_stride16, kst, m2l_bf16_lds_ld16(2), P->d_items + i0,
                           std::min(i1, split) - i0, P->d_tgt_blk, P->d_src_blk, P->d_pair_offs, P->d_uhat,
                           P->d_chat_part, R * TS * kst, R, TS * kst, st, part == 2);
    if (ok && i1 > split)
      ok = launch_m2l_bf16(3, P->m2l_rb, P->d_cores_b3, P->core_stride16_3, kst, m2l_bf16_lds_ld16(3),
                           P->d_items + std::max(i0, split), i1 - std::max(i0, split), P->d_tgt_blk, P->d_src_blk,
                           P->d_pair_offs, P->d_uhat, P->d_chat_part, R * TS * kst, R, TS * kst, st, true);
    return ok;
  }
  if (P->m2l_pieces)
    return launch_m2l_bf16(P->m2l_pieces, P->m2l_rb, P->d_cores_b, P->core_stride16, kst,
                           m2l_bf16_lds_ld16(P->m2l_pieces), P->d_items + i0, i1 - i0, P->d_tgt_blk, P->d_src_blk,
                           P->d_pair_offs, P->d_uhat, P->d_chat_part, R * TS * kst, R, TS * kst, st, part == 2);
  return launch_m2l(P->m2l_rb, P->d_cores, P->core_rows, kst, P->m2l_lds_ld, P->d_items + i0, i1 - i0, P->d_tgt_blk,
                    P->d_src_blk, P->d_pair_offs, P->d_uhat, P->d_chat_part, R * TS * kst, R, TS * kst, st,
                    part == 2);
}

namespace {

// Joins a plan stream back into the caller's stream if an enqueue fails after
// the fork (so that nothing of the call stays unordered with later work).
struct JoinGuard {
  hipStream_t from = nullptr, into = nullptr;
  hipEvent_t ev = nullptr;
  ~JoinGuard() {
    if (!from) return;
    (void)hipEventRecord(ev, from);
    (void)hipStreamWaitEvent(into, ev, 0);
  }
  void arm(hipStream_t f, hipStream_t i, hipEvent_t e) {
    from = f;
    into = i;
    ev = e;
  }
  void disarm() { from = nullptr; }
};

const char* kLeafInternal = "internal: leaf kernel configuration not available";

// Workgroups of the persistent leaf kernel: queue_per_cu per CU, at most one per
// four tiles, a multiple of 8 (one counter per XCD).
int queue_grid(const Plan* P) {
  const int want = std::min(P->queue_per_cu * P->n_cus, (P->n_tiles + 3) / 4);
  return std::max(8, (want + 7) / 8 * 8);
}

// The one-RHS leaf sums (U-list, D2T or both, see k_p2p) by the plan's kernel.
void launch_leaf_sums(Plan* P, int mode, const float* d_leaf, float* pot, float* grad, hipStream_t s) {
  bool ok;
  if (P->leaf_queue)
    ok = launch_leaf_queue(mode, P->d_pts, P->d_start, P->d_tiles, P->n_tiles,
                           P->d_queue + (mode == 2 ? kQueueInts : 0), queue_grid(P), P->d_blk, P->group_slots, P->d_centers, P->d_surf, P->n,
                           (float)P->ops->alpha_outer, d_leaf, P->nst, P->far ? 1 : 0, P->d_order, pot, grad,
                           P->d_near, s);
  else
    ok = launch_p2p(mode, P->d_pts, P->d_start, P->d_blk, (int)P->n_groups, P->group_slots, P->p2p_cap, P->d_centers,
                    P->d_surf, P->n, (float)P->ops->alpha_outer, d_leaf, P->nst, P->far ? 1 : 0, P->d_order, pot,
                    grad, P->d_near, P->p2p_threads, s);
  if (!ok) fail(KIFMM_E_DEVICE, kLeafInternal);
}

}  // namespace

void evaluate_plan(Plan* P, const float* charges, float* pot, float* grad, hipStream_t st) {
  // Every check before the first enqueue.
  require(charges != nullptr, "charges is null");
  require(pot || grad, "at least one of potential / gradient must be given");
  if (grad && !(P->flags & KIFMM_GRADIENT)) fail(KIFMM_E_STATE, "the plan was created without KIFMM_GRADIENT");
  const int R = P->nrhs;
  require(R == 1 || pot != nullptr, "plans with nrhs > 1 give potentials: potential must be given");
  DeviceScope scope(P->device);
  if (st) {
    int dev = -1;
    hip_check(hipStreamGetDevice(st, &dev), "hipStreamGetDevice");
    require(dev == P->device, "the stream belongs to another device than the plan");
  }
  P->timing_begin_call();

  const int N = (int)P->N;
  const int L = P->L;
  const float alpha = (float)P->ops->alpha_outer;
  if (P->leaf_queue) launch_clear_queue(P->d_queue, 2 * kQueueInts, st);
  P->stage_begin(KIFMM_STAGE_PERMUTE, st);
  if (R == 1)
    launch_permute(P->d_pts, charges, P->d_order, N, st);
  else
    launch_permute_multi(P->d_qs, charges, P->d_order, N, R, st);
  P->stage_end(KIFMM_STAGE_PERMUTE, st);
  const bool split = P->side != nullptr;
  const float* d_leaf = P->far ? P->d_d + P->base[L] * P->nst : nullptr;
  JoinGuard side_guard, up_guard;
  if (split) {
    // (3c) ULI needs only the sorted charges: it runs on the plan's stream beside
    // the upward pass and M2L, and is joined before D2T.
    hip_check(hipEventRecord(P->ev_fork, st), "hipEventRecord");
    hip_check(hipStreamWaitEvent(P->side, P->ev_fork, 0), "hipStreamWaitEvent");
    side_guard.arm(P->side, st, P->ev_join);
    P->stage_begin(KIFMM_STAGE_P2P, P->side);
    launch_leaf_sums(P, 1, d_leaf, nullptr, nullptr, P->side);
    P->stage_end(KIFMM_STAGE_P2P, P->side);
    hip_check(hipEventRecord(P->ev_join, P->side), "hipEventRecord");
  }

  if (P->far) {
    const int n = P->n, nst = P->nst, kst = P->kst, kcst = P->kcst;
    const int SL = (int)P->slots[L];
    const int nleaves = (int)P->n_leaves;
    const long long TS = P->total_slots;
    float* uL = P->d_u + P->base[L] * nst;
    // (1a) S2U: check field, then the two pseudo-inverse factors (scaled by r_L).
    // With nrhs > 1 every per-box array holds the right-hand sides one after
    // the other, and each product runs as one batch over them.
    P->stage_begin(KIFMM_STAGE_P2M, st);
    if (R == 1) {
      if (!launch_p2m(P->d_pts, P->d_start, P->d_leaves, P->d_centers, P->d_surf, n, alpha, P->d_q, nst, nleaves, st))
        fail(KIFMM_E_DEVICE, kLeafInternal);
    } else if (!launch_p2m_multi(R, P->d_pts, P->d_qs, P->d_start, P->d_leaves, P->d_centers, P->d_surf, n, alpha,
                                 P->d_q, nst, (long long)SL * nst, nleaves, st))
      fail(KIFMM_E_DEVICE, kLeafInternal);
    P->stage_end(KIFMM_STAGE_P2M, st);
    P->stage_begin(KIFMM_STAGE_UC2E, st);
    launch_gemm_nt(P->d_f1, nst, P->d_q, nst, P->d_leaves, P->d_t, kcst, P->d_leaves, nleaves, kcst, nst, 1.0f, 0, st,
                   R, (long long)SL * nst, (long long)SL * kcst);
    launch_gemm_nt(P->d_f2, kcst, P->d_t, kcst, P->d_leaves, uL, nst, P->d_leaves, nleaves, nst, kcst,
                   (float)P->tree->radius(L), 0, st, R, (long long)SL * kcst, TS * nst);
    P->stage_end(KIFMM_STAGE_UC2E, st);
    // (1b) U2U, (2a) compression and VLI, (2c) D2D.  The leaf level's VLI needs
    // only the leaf level's compressed densities, so with a second plan stream the
    // levels above it (U2U to level 2, their compression, VLI and downward pass,
    // and the D2D into the leaf level) run there, beside the leaf level's VLI, and
    // are joined before the leaf level's post product.
    const bool up = P->up != nullptr && P->up_on;
    const int n_upper = P->n_nonempty - (int)P->keys_per_level[L];  // non-empty rows of levels 2..L-1
    hipStream_t su = up ? P->up : st;
    // (2c) pieces: the sum of the eight M2L partial sums over a range of box rows,
    // D2D into level l (all 8 children of each non-empty parent, overwritten) and
    // the post product (DC2E U_k) of level l's non-empty boxes, added above level 2:
    // d = L2L d_parent + post chat.  Empty boxes' d is never read.
    auto sum_rows = [&](long long r0, long long r1, hipStream_t s) {
      if (!P->m2l_wide && !P->m2l_gather)
        launch_sum_parts(P->d_chat_part + r0 * kst, P->d_chat + r0 * kst, R * (r1 - r0) * kst, R * TS * kst, s);
    };
    auto d2d = [&](int l, hipStream_t s) {
      const int parents = (int)P->keys_per_level[l - 1];
      launch_gemm_nt(P->d_l2l, nst, P->d_d + P->base[l - 1] * nst, nst, P->d_nbslot[l - 1], P->d_d + P->base[l] * nst,
                     8 * nst, nullptr, parents, 8 * nst, nst, 1.0f, 0, s, R, TS * nst, TS * nst);
    };
    auto post = [&](int l, hipStream_t s) {
      launch_gemm_nt(P->d_post, kst, P->d_chat + P->base[l] * kst, kst, P->d_nbslot[l], P->d_d + P->base[l] * nst,
                     nst, P->d_nbslot[l], (int)P->keys_per_level[l], nst, kst, 1.0f, l > 2 ? 1 : 0, s, R, TS * kst,
                     TS * nst);
    };
    if (up) {
      hip_check(hipEventRecord(P->ev_up0, st), "hipEventRecord");
      hip_check(hipStreamWaitEvent(su, P->ev_up0, 0), "hipStreamWaitEvent");
      up_guard.arm(su, st, P->ev_up1);
    }
    P->stage_begin(KIFMM_STAGE_M2M, su);
    for (int l = L; l >= 3; --l) {
      const int parents = (int)P->keys_per_level[l - 1];
      launch_gemm_nt(P->d_m2m, 8 * nst, P->d_u + P->base[l] * nst, 8 * nst, nullptr, P->d_u + P->base[l - 1] * nst,
                     nst, P->d_nbslot[l - 1], parents, nst, 8 * nst, 1.0f, 0, su, R, TS * nst, TS * nst);
    }
    if (up) {
      // Compression, VLI and the downward pass of the levels above the leaves, and
      // D2D into the leaf level (it needs only the level above): all of it beside
      // the leaf level's VLI, whose result then only needs its sum and post.
      launch_gemm_nt(P->d_vt, nst, P->d_u, nst, P->d_nonempty, P->d_uhat, kst, P->d_nonempty, n_upper, kst, nst, 1.0f,
                     0, su, R, TS * nst, TS * kst, P->m2l_wide ? 1 : 0);
      if (!launch_m2l_form(P, su, 2)) fail(KIFMM_E_DEVICE, "internal: M2L kernel configuration not available");
      sum_rows(P->base[2], P->base[L], su);
      for (int l = 2; l < L; ++l) {
        if (l > 2) d2d(l, su);
        post(l, su);
      }
      d2d(L, su);
    }
    P->stage_end(KIFMM_STAGE_M2M, su);
    if (up) hip_check(hipEventRecord(P->ev_up1, su), "hipEventRecord");
    // (empty boxes keep uhat = 0 from allocation: their rows are never written)
    P->stage_begin(KIFMM_STAGE_COMPRESS, st);
    if (up)
      launch_gemm_nt(P->d_vt, nst, P->d_u, nst, P->d_nonempty + n_upper, P->d_uhat, kst, P->d_nonempty + n_upper,
                     P->n_nonempty - n_upper, kst, nst, 1.0f, 0, st, R, TS * nst, TS * kst, P->m2l_wide ? 1 : 0);
    else
      launch_gemm_nt(P->d_vt, nst, P->d_u, nst, P->d_nonempty, P->d_uhat, kst, P->d_nonempty, P->n_nonempty, kst, nst,
                     1.0f, 0, st, R, TS * nst, TS * kst, P->m2l_wide ? 1 : 0);
    P->stage_end(KIFMM_STAGE_COMPRESS, st);
    P->stage_begin(KIFMM_STAGE_M2L, st);
    if (!launch_m2l_form(P, st, up ? 1 : 0)) fail(KIFMM_E_DEVICE, "internal: M2L kernel configuration not available");
    P->stage_end(KIFMM_STAGE_M2L, st);
    // (2c) coarse to fine; with the second stream only the leaf level's sum and post remain here
    P->stage_begin(KIFMM_STAGE_L2L, st);
    if (up) {
      sum_rows(P->base[L], TS, st);
      hip_check(hipStreamWaitEvent(st, P->ev_up1, 0), "hipStreamWaitEvent");
      up_guard.disarm();
      post(L, st);
    } else {
      sum_rows(0, TS, st);
      for (int l = 2; l <= L; ++l) {
        if (l > 2) d2d(l, st);
        post(l, st);
      }
    }
    P->stage_end(KIFMM_STAGE_L2L, st);
  }
  if (split) {
    // (3b) D2T added to the ULI result, written in input order.
    hip_check(hipStreamWaitEvent(st, P->ev_join, 0), "hipStreamWaitEvent");
    side_guard.disarm();
    P->stage_begin(KIFMM_STAGE_L2P, st);
    launch_leaf_sums(P, 2, d_leaf, pot, grad, st);
    P->stage_end(KIFMM_STAGE_L2P, st);
  } else if (R > 1) {
    // (3b) D2T + (3c) ULI for all right-hand sides, potentials in input order.
    P->stage_begin(KIFMM_STAGE_P2P, st);
    if (!launch_leaf_multi(R, P->d_pts, P->d_qs, P->d_start, P->d_tasks, P->n_tasks, P->d_blk, P->group_slots,
                           P->d_centers, P->d_surf, P->n, alpha, d_leaf, P->nst,
                           P->far ? (long long)P->total_slots * P->nst : 0, P->far ? 1 : 0, P->d_order, pot, st))
      fail(KIFMM_E_DEVICE, kLeafInternal);
    P->stage_end(KIFMM_STAGE_P2P, st);
  } else {
    // (3b) D2T + (3c) ULI fused, written in input order.
    P->stage_begin(KIFMM_STAGE_P2P, st);
    launch_leaf_sums(P, 0, d_leaf, pot, grad, st);
    P->stage_end(KIFMM_STAGE_P2P, st);
  }
  hip_check(hipGetLastError(), "kernel launch");
}

void evaluate_vjp(Plan* P, const float* charges, const float* weights, const float* field, float* grad_charges,
                  float* grad_points, hipStream_t st) {
  if (!(P->flags & KIFMM_VJP)) fail(KIFMM_E_STATE, "the plan was created without KIFMM_VJP");
  require(charges != nullptr && weights != nullptr, "charges or weights is null");
  require(grad_charges || grad_points, "at least one of grad_charges / grad_points must be given");
  if (grad_points && !(P->flags & KIFMM_GRADIENT))
    fail(KIFMM_E_STATE, "grad_points needs a plan with KIFMM_GRADIENT");
  vjp_enqueue(P, charges, weights, field, grad_charges, grad_points, P->d_vjp_fs, P->d_vjp_fw, st);
}

void evaluate_vjp_noalloc(Plan* P, const float* charges, const float* weights, const float* field,
                          float* grad_charges, float* grad_points, hipStream_t st) {
  require(charges != nullptr && weights != nullptr, "charges or weights is null");
  require(grad_charges || grad_points, "at least one of grad_charges / grad_points must be given");
  if (grad_points && !(P->flags & KIFMM_GRADIENT))
    fail(KIFMM_E_STATE, "grad_points needs a plan with KIFMM_GRADIENT");
  require(P->nrhs == 1, "the derivative needs a plan with one right-hand side");
  require(P->N <= kNoAllocMaxPoints, "the no-allocation derivative takes at most " +
                                         std::to_string(kNoAllocMaxPoints) + " points (the plan has " +
                                         std::to_string(P->N) + ")");
  float* base = scratch_address(P->device);
  vjp_enqueue(P, charges, weights, field, grad_charges, grad_points, base, base + 3 * P->N, st);
}

// dL/ds = evaluate(w); dL/dx = w grad f_s + s grad f_w, with the two fields in fs_buf / fw_buf.
void vjp_enqueue(Plan* P, const float* charges, const float* weights, const float* field, float* grad_charges,
                 float* grad_points, float* fs_buf, float* fw_buf, hipStream_t st) {
  const float* fs = field;
  if (grad_points && !fs) {
    evaluate_plan(P, charges, nullptr, fs_buf, st);
    fs = fs_buf;
  }
  evaluate_plan(P, weights, grad_charges, grad_points ? fw_buf : nullptr, st);
  if (grad_points) {
    DeviceScope scope(P->device);
    launch_vjp_combine(charges, weights, fs, fw_buf, grad_points, (int)P->N, st);
    hip_check(hipGetLastError(), "kernel launch");
  }
}

namespace {

// Choices timed at plan creation, kept per process for plans of the same shape
// (device, sizes, order, rank, flags and the occupancy of the tree's levels and
// leaves), so that creating such a plan again times nothing.
struct Tuned {
  bool m2l_gather = false;
  int m2l_lds_ld = 0;
  bool up_on = false, leaf_queue = false;
  int p2p_threads = kP2PMaxThreads, queue_per_cu = 8;
  double m2l_tune_ms[2] = {0, 0}, slab_ms[4] = {0, 0, 0, 0}, tune_ms[2][2] = {{0, 0}, {0, 0}}, leaf_tune_ms[2] = {0, 0};
};
std::mutex g_tuned_mu;
std::map<std::string, Tuned> g_tuned;

std::string shape_key(const Plan* P) {
  const Tree& T = *P->tree;
  std::string key = std::to_string(P->device) + "|" + std::to_string(P->N) + "|" + std::to_string(P->L) + "|" +
                    std::to_string(P->n) + "|" + std::to_string(P->k) + "|" + std::to_string(P->nrhs) + "|" +
                    std::to_string(P->flags) + "|" + std::to_string(P->ops->alpha_inner) + "|";
  for (int l = 0; l <= P->L; ++l) key += std::to_string(T.keys[l].size()) + ",";
  // leaf occupancy histogram in powers of two
  int64_t hist[40] = {};
  for (size_t i = 0; i + 1 < T.leaf_start.size(); ++i) {
    const int64_t c = T.leaf_start[i + 1] - T.leaf_start[i];
    int b = 0;
    while (b < 39 && (int64_t(1) << (b + 1)) <= c) ++b;
    ++hist[b];
  }
  key += "|";
  for (int b = 0; b < 40; ++b)
    if (hist[b]) key += std::to_string(b) + ":" + std::to_string(hist[b]) + ",";
  return key;
}

}  // namespace

// Timed choices at plan creation, each by whole launches on the plan's own
// tables (the work does not depend on the values): one warm-up, then the
// median of the timed repeats.  A choice leaves its default only when it is at
// least 2 % faster, so that run-to-run noise does not flip it.
//   1. M2L form (one right-hand side, FP32): blocked or gathered.
//   2. M2L LDS slab of the blocked FP32 form: 24, 32, 40 or 48 k per slab (the
//      default is the slab that keeps the most waves resident).
//   3. Evaluate layout (one right-hand side): the second stream for the levels
//      above the leaves, and the leaf sums by the per-parent kernel (256 or 320
//      threads) or the persistent work queue (2, 4 or 8 workgroups per CU).
void autotune(Plan* P, hipStream_t st) {
  const unsigned flags = P->flags;
  if (flags & KIFMM_LEAF_QUEUE) P->leaf_queue = true;
  if (flags & KIFMM_NO_AUTOTUNE) {
    P->m2l_gather = (flags & KIFMM_M2L_GATHER) != 0;
    return;  // the defaults of prepare(); the second stream on where it exists
  }
  const std::string key = shape_key(P);
  {
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      const Tuned& t = it->second;
      P->m2l_gather = t.m2l_gather;
      if (t.m2l_lds_ld) P->m2l_lds_ld = t.m2l_lds_ld;
      if (P->up) P->up_on = t.up_on;
      P->leaf_queue = t.leaf_queue;
      P->p2p_threads = t.p2p_threads;
      P->queue_per_cu = t.queue_per_cu;
      std::copy(t.m2l_tune_ms, t.m2l_tune_ms + 2, P->m2l_tune_ms);
      std::copy(t.slab_ms, t.slab_ms + 4, P->slab_tune_ms);
      for (int i = 0; i < 2; ++i) std::copy(t.tune_ms[i], t.tune_ms[i] + 2, P->tune_ms[i]);
      std::copy(t.leaf_tune_ms, t.leaf_tune_ms + 2, P->leaf_tune_ms);
      P->tuned_from_cache = true;
      return;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hip_check(hipEventCreate(&e0), "hipEventCreate");
  hip_check(hipEventCreate(&e1), "hipEventCreate");
  struct Events {
    hipEvent_t a, b;
    ~Events() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } events{e0, e1};
  auto time_ms = [&](int reps, auto&& body) {
    std::vector<double> t;
    for (int rep = 0; rep <= reps; ++rep) {
      hip_check(hipEventRecord(e0, st), "hipEventRecord");
      body();
      hip_check(hipEventRecord(e1, st), "hipEventRecord");
      hip_check(hipEventSynchronize(e1), "plan-time timing");
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      if (rep > 0) t.push_back(ms);  // the first launch warms up
    }
    return median(t);
  };
  const long long n_red = (long long)P->nrhs * P->total_slots * P->kst;
  auto m2l_all = [&] {
    if (!launch_m2l_form(P, st, 0)) fail(KIFMM_E_DEVICE, "internal: M2L kernel configuration not available");
    if (!P->m2l_gather && !P->m2l_wide) launch_sum_parts(P->d_chat_part, P->d_chat, n_red, n_red, st);
  };

  // 1. The one-RHS M2L form.
  if (P->d_gunits && !(flags & (KIFMM_M2L_BLOCKED | KIFMM_M2L_GATHER))) {
    for (int form = 0; form < 2; ++form) {
      P->m2l_gather = form == 1;
      P->m2l_tune_ms[form] = time_ms(3, m2l_all);
    }
    P->m2l_gather = P->m2l_tune_ms[1] < 0.98 * P->m2l_tune_ms[0];
  }
  // 2. The LDS slab of the blocked FP32 M2L.
  if (P->far && !P->m2l_pieces && !P->m2l_gather && !P->m2l_wide) {
    const int def = P->m2l_lds_ld;
    double t_def = -1.0, best = -1.0;
    int pick = def;
    for (int i = 0; i < 4; ++i) {
      const int ld = 24 + 8 * i + 4;
      if (!m2l_supported(P->m2l_rb, P->kst, ld)) continue;
      P->m2l_lds_ld = ld;
      const double ms = time_ms(3, m2l_all);
      P->slab_tune_ms[i] = ms;
      if (ld == def) t_def = ms;
      if (best < 0.0 || ms < best) {
        best = ms;
        pick = ld;
      }
    }
    P->m2l_lds_ld = (t_def >= 0.0 && best > 0.98 * t_def) ? def : pick;
  }
  if (P->far && P->d_chat) hip_check(hipMemsetAsync(P->d_chat, 0, sizeof(float) * (size_t)n_red, st), "chat reset");

  // 3. The evaluate's layout.
  const bool tune_up = P->up != nullptr && !(flags & KIFMM_UPPER_STREAM);
  const bool tune_threads = P->side != nullptr && !(flags & (KIFMM_LEAF_THREADS_256 | KIFMM_LEAF_THREADS_320));
  const bool tune_queue = P->d_tiles != nullptr && !(flags & (KIFMM_LEAF_QUEUE | KIFMM_LEAF_BLOCKS));
  if (P->nrhs == 1 && (tune_up || tune_threads || tune_queue || P->leaf_queue)) {
    const int64_t n = P->N;
    float *q = nullptr, *pot = nullptr, *grad = nullptr;
    struct Buffers {
      float** p[3];
      ~Buffers() {
        for (float** b : p)
          if (*b) (void)hipFree(*b);
      }
    } buffers{{&q, &pot, &grad}};
    hip_check(hipMalloc(&q, sizeof(float) * (size_t)n), "timing charges");
    hip_check(hipMemsetAsync(q, 0, sizeof(float) * (size_t)n, st), "timing charges");
    hip_check(hipMalloc(&pot, sizeof(float) * (size_t)n), "timing potentials");
    if (flags & KIFMM_GRADIENT) hip_check(hipMalloc(&grad, 3 * sizeof(float) * (size_t)n), "timing field");

    struct Layout {
      bool up_on, queue;
      int threads, per_cu;
    };
    const Layout def{P->up != nullptr, P->leaf_queue, P->p2p_threads, 8};
    std::vector<Layout> cands;
    for (int on = 0; on < 2; ++on) {
      if (on != (int)def.up_on && !tune_up) continue;
      for (int qu = 0; qu < 2; ++qu) {
        if (qu != (int)def.queue && !tune_queue) continue;
        if (qu) {
          for (int per_cu : {2, 4, 8}) cands.push_back(Layout{on == 1, true, def.threads, per_cu});
        } else {
          for (int th : {256, kP2PMaxThreads})
            if (th == def.threads || tune_threads) cands.push_back(Layout{on == 1, false, th, def.per_cu});
        }
      }
    }
    double best = -1.0, t_def = -1.0, best_blocks = -1.0, best_queue = -1.0;
    Layout pick = def;
    for (const Layout& c : cands) {
      P->up_on = c.up_on;
      P->leaf_queue = c.queue;
      P->p2p_threads = c.threads;
      P->queue_per_cu = c.per_cu;
      const double ms = time_ms(5, [&] { evaluate_plan(P, q, pot, grad, st); });
      if (!c.queue) P->tune_ms[c.up_on ? 1 : 0][c.threads == 256 ? 0 : 1] = ms;
      double& slot = c.queue ? best_queue : best_blocks;
      if (slot < 0.0 || ms < slot) slot = ms;
      if (c.up_on == def.up_on && c.queue == def.queue && c.threads == def.threads && c.per_cu == def.per_cu)
        t_def = ms;
      if (best < 0.0 || ms < best) {
        best = ms;
        pick = c;
      }
    }
    if (t_def >= 0.0 && best > 0.98 * t_def) pick = def;
    P->up_on = pick.up_on;
    P->leaf_queue = pick.queue;
    P->p2p_threads = pick.threads;
    P->queue_per_cu = pick.per_cu;
    P->leaf_tune_ms[0] = std::max(best_blocks, 0.0);
    P->leaf_tune_ms[1] = std::max(best_queue, 0.0);
  }
  hip_check(hipStreamSynchronize(st), "plan-time timing");
  Tuned t;
  t.m2l_gather = P->m2l_gather;
  t.m2l_lds_ld = P->m2l_lds_ld;
  t.up_on = P->up_on;
  t.leaf_queue = P->leaf_queue;
  t.p2p_threads = P->p2p_threads;
  t.queue_per_cu = P->queue_per_cu;
  std::copy(P->m2l_tune_ms, P->m2l_tune_ms + 2, t.m2l_tune_ms);
  std::copy(P->slab_tune_ms, P->slab_tune_ms + 4, t.slab_ms);
  for (int i = 0; i < 2; ++i) std::copy(P->tune_ms[i], P->tune_ms[i] + 2, t.tune_ms[i]);
  std::copy(P->leaf_tune_ms, P->leaf_tune_ms + 2, t.leaf_tune_ms);
  std::lock_guard<std::mutex> lock(g_tuned_mu);
  g_tuned[key] = t;
}

void read_density(Plan* P, int kind, int level, float* out, int64_t capacity) {
  require(out != nullptr, "output is null");
  require(kind == 0 || kind == 1, "kind must be 0 (u) or 1 (d)");
  require(P->far, "the tree has no far field (depth < 2)");
  require(level >= 2 && level <= P->L, "level must be in [2, depth]");
  const int64_t nb = P->keys_per_level[level];
  require(capacity >= nb * P->n, "capacity too small");
  DeviceScope scope(P->device);
  hip_check(hipDeviceSynchronize(), "synchronise");
  std::vector<float> all((size_t)P->slots[level] * P->nst);
  const float* src = (kind == 0 ? P->d_u : P->d_d) + P->base[level] * P->nst;
  hip_check(hipMemcpy(all.data(), src, all.size() * sizeof(float), hipMemcpyDeviceToHost), "copy density");
  for (int64_t i = 0; i < nb; ++i)
    std::memcpy(out + i * P->n, all.data() + (size_t)P->slot_of[level][i] * P->nst, P->n * sizeof(float));
}

}  // namespace kifmm
