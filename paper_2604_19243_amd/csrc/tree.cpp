// Uniform octree build on the host (Section 2.1): enclosing cube, leaf grid
// coordinates in double precision, Morton keys, stable sort, and the
// non-empty boxes of every level in Morton order.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <utility>
#include <string>

#include "common.hpp"

namespace kifmm {

int64_t Tree::find(int level, uint64_t key) const {
  const auto& k = keys[level];
  auto it = std::lower_bound(k.begin(), k.end(), key);
  return (it != k.end() && *it == key) ? (int64_t)(it - k.begin()) : -1;
}

Tree* build_tree(const float* xyz, int64_t n, int depth, const double* cube) {
  require(xyz != nullptr, "xyz is null");
  require(n >= 1 && n < (1ll << 31), "n must be in [1, 2^31)");
  require(depth >= 0 && depth <= KIFMM_MAX_DEPTH, "depth must be in [0, " + std::to_string(KIFMM_MAX_DEPTH) + "]");
  for (int64_t i = 0; i < 3 * n; ++i)
    require(std::isfinite(xyz[i]) && std::fabs(xyz[i]) < 1e30f, "coordinates must be finite and below 1e30 in magnitude");

  Tree* t = new Tree();
  try {
    t->n = n;
    t->depth = depth;
    t->xyz.assign(xyz, xyz + 3 * n);
    if (cube) {
      for (int d = 0; d < 4; ++d) require(std::isfinite(cube[d]), "non-finite cube");
      require(cube[3] > 0.0, "cube half-width must be positive");
      for (int d = 0; d < 3; ++d) t->center[d] = cube[d];
      t->half = cube[3];
    } else {
      // Midpoint of the per-axis range; half-width 0.5 * max range * (1 + 1e-6).
      double lo[3], hi[3];
      for (int d = 0; d < 3; ++d) lo[d] = hi[d] = (double)xyz[d];
      for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
          lo[d] = std::min(lo[d], (double)xyz[3 * i + d]);
          hi[d] = std::max(hi[d], (double)xyz[3 * i + d]);
        }
      double ext = 0.0;
      for (int d = 0; d < 3; ++d) {
        t->center[d] = 0.5 * (lo[d] + hi[d]);
        ext = std::max(ext, hi[d] - lo[d]);
      }
      t->half = 0.5 * ext * (1.0 + 1e-6);
      if (!(t->half > 0.0)) t->half = 1.0;
    }

    // Leaf grid coordinates: floor((x - (c - R0)) / h), h = 2 R0 / 2^L, clamped.
    const int64_t m = 1ll << depth;
    const double h = (2.0 * t->half) / (double)m;
    t->ijk.resize(3 * n);
    std::vector<uint64_t> key(n);
    for (int64_t i = 0; i < n; ++i) {
      uint32_t c[3];
      for (int d = 0; d < 3; ++d) {
        const double lo = t->center[d] - t->half;
        double f = std::floor(((double)xyz[3 * i + d] - lo) / h);
        if (!(f >= 0.0)) f = 0.0;
        if (f > (double)(m - 1)) f = (double)(m - 1);
        c[d] = (uint32_t)f;
        t->ijk[3 * i + d] = (int32_t)f;
      }
      key[i] = morton_encode(c[0], c[1], c[2], depth);
    }
    // Sort (key, input index) pairs: equal keys keep input order.
    {
      std::vector<std::pair<uint64_t, int64_t>> kv(n);
      for (int64_t i = 0; i < n; ++i) kv[i] = {key[i], i};
      std::sort(kv.begin(), kv.end());
      t->order.resize(n);
      for (int64_t s = 0; s < n; ++s) t->order[s] = kv[s].second;
    }

    // Non-empty leaves and their point ranges in sorted order.
    t->keys.assign(depth + 1, {});
    for (int64_t s = 0; s < n; ++s) {
      const uint64_t k = key[t->order[s]];
      if (s == 0 || k != key[t->order[s - 1]]) {
        t->keys[depth].push_back(k);
        t->leaf_start.push_back(s);
      }
    }
    t->leaf_start.push_back(n);
    for (size_t b = 0; b + 1 < t->leaf_start.size(); ++b)
      t->max_leaf = std::max<int32_t>(t->max_leaf, (int32_t)(t->leaf_start[b + 1] - t->leaf_start[b]));
    // Coarser levels: parent key = key >> 3 (sorted keys are a pre-order traversal).
    for (int l = depth - 1; l >= 0; --l) {
      for (uint64_t k : t->keys[l + 1]) {
        const uint64_t pk = k >> 3;
        if (t->keys[l].empty() || t->keys[l].back() != pk) t->keys[l].push_back(pk);
      }
    }
  } catch (...) {
    delete t;
    throw;
  }
  return t;
}

}  // namespace kifmm
