// Shared host-side definitions of the kiFMM library: error reporting and the
// tree / operator objects behind the C ABI handles.
#pragma once

#include <atomic>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "kifmm_mi355x.h"

namespace kifmm {

// Error carried to the C ABI boundary, where it becomes a status code and a
// thread-local message.
struct Error : std::runtime_error {
  kifmm_status status;
  Error(kifmm_status s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

[[noreturn]] inline void fail(kifmm_status s, const std::string& msg) { throw Error(s, msg); }
inline void require(bool ok, const std::string& msg) {
  if (!ok) fail(KIFMM_E_INVALID, msg);
}

void set_last_error(const std::string& msg);

// Reference-counted base of the three handle types.
struct Object {
  std::atomic<int> refs{1};
  virtual ~Object() = default;
};
template <class T>
void release(T* obj) {
  if (obj && obj->refs.fetch_sub(1) == 1) delete obj;
}

// Interleave the low `bits` bits of (ix, iy, iz): bit b of ix, iy, iz goes to
// key bits 3b, 3b+1, 3b+2 (three bits per level, Section 2.1).
inline uint64_t morton_encode(uint32_t ix, uint32_t iy, uint32_t iz, int bits) {
  uint64_t key = 0;
  for (int b = 0; b < bits; ++b) {
    key |= (uint64_t)((ix >> b) & 1u) << (3 * b);
    key |= (uint64_t)((iy >> b) & 1u) << (3 * b + 1);
    key |= (uint64_t)((iz >> b) & 1u) << (3 * b + 2);
  }
  return key;
}
inline void morton_decode(uint64_t key, int bits, int32_t* ijk) {
  ijk[0] = ijk[1] = ijk[2] = 0;
  for (int b = 0; b < bits; ++b) {
    ijk[0] |= (int32_t)((key >> (3 * b)) & 1u) << b;
    ijk[1] |= (int32_t)((key >> (3 * b + 1)) & 1u) << b;
    ijk[2] |= (int32_t)((key >> (3 * b + 2)) & 1u) << b;
  }
}

// Uniform octree over the input points (Section 2.1): levels 0..depth, leaves
// at `depth`, non-empty boxes of every level listed in Morton order.
struct Tree : Object {
  int64_t n = 0;
  int depth = 0;
  double center[3] = {0, 0, 0};
  double half = 1.0;
  std::vector<float> xyz;               // [n][3] input order
  std::vector<int32_t> ijk;             // [n][3] leaf coordinates, input order
  std::vector<int64_t> order;           // sorted position -> input index
  std::vector<std::vector<uint64_t>> keys;   // per level: Morton keys of non-empty boxes, sorted
  std::vector<int64_t> leaf_start;      // [nonempty leaves + 1]: first sorted position of each leaf
  int32_t max_leaf = 0;

  double radius(int level) const { return half / (double)(1ll << level); }
  // Compact index of the non-empty box with `key` at `level`, or -1.
  int64_t find(int level, uint64_t key) const;
};

// FP64 operators for expansion order p at unit box half-width (Table 1).
struct Ops : Object {
  int p = 0, n = 0, k = 0, kc = 0;      // surface size n, M2L rank k, pinv rank kc
  double eps_pinv = 0, eps_svd = 0;
  double alpha_inner = 0, alpha_outer = 0;  // surface radius factors (equivalent/check)
  std::vector<double> surf;             // [n][3]
  std::vector<double> uc2e, dc2e;       // [n][n]
  std::vector<double> f1, f2;           // UC2E = f2 * f1: f1 = U_kc^T [kc][n], f2 = V_kc S^-1 [n][kc]
  std::vector<double> m2m, l2l;         // [8][n][n]
  std::vector<double> mu, mv;           // U_k, V_k [n][k]
  std::vector<double> cores;            // [316][k][k]
  std::vector<int32_t> offsets;         // [316][3]
  std::vector<double> post;             // DC2E U_k [n][k]
};

Tree* build_tree(const float* xyz, int64_t n, int depth, const double* cube);
// eps_svd > 0: relative compression cutoff; eps_svd = -k (k >= 1 integral): rank k.
Ops* precompute_ops(int p, double alpha_inner, double alpha_outer, double eps_pinv, double eps_svd);

constexpr int kNumOffsets = 316;
constexpr int kOffsetsPerOctant = 189;

}  // namespace kifmm
