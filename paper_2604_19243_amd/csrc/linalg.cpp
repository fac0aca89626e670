// FP64 Householder QR and one-sided Jacobi SVD for the operator precompute.
#include "linalg.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>

namespace kifmm {

namespace {

// In-place Householder triangularisation of the column-major m x n block `a`
// (leading dimension lda, m >= n); writes the n x n upper-triangular factor to r.
void householder_block(double* a, int64_t lda, int64_t m, int64_t n, double* r) {
  for (int64_t j = 0; j < n; ++j) {
    double* x = a + j * lda;
    double norm2 = 0.0;
    for (int64_t i = j; i < m; ++i) norm2 += x[i] * x[i];
    const double norm = std::sqrt(norm2);
    if (norm == 0.0) continue;
    const double alpha = x[j] > 0.0 ? -norm : norm;
    const double vv = 2.0 * norm * (norm + std::fabs(x[j]));  // |x - alpha e_j|^2 without cancellation
    x[j] -= alpha;  // v = x - alpha e_j, stored in place
    if (vv > 0.0) {
      for (int64_t c = j + 1; c < n; ++c) {
        double* y = a + c * lda;
        double dot = 0.0;
        for (int64_t i = j; i < m; ++i) dot += x[i] * y[i];
        const double f = 2.0 * dot / vv;
        for (int64_t i = j; i < m; ++i) y[i] -= f * x[i];
      }
    }
    x[j] = alpha;
  }
  for (int64_t c = 0; c < n; ++c)
    for (int64_t i = 0; i < n; ++i) r[c * n + i] = (i <= c) ? a[c * lda + i] : 0.0;
}

}  // namespace

std::vector<double> qr_r_factor(std::vector<double>& a, int64_t m, int64_t n) {
  std::vector<double> r(n * n, 0.0);
  int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(16, m / (8 * n)));
  unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  blocks = std::min<int64_t>(blocks, hw);
  if (blocks <= 1) {
    householder_block(a.data(), m, m, n, r.data());
    return r;
  }
  // Tall-skinny QR: factor row blocks independently, then the stacked R factors.
  std::vector<int64_t> start(blocks + 1);
  for (int64_t b = 0; b <= blocks; ++b) start[b] = (m * b) / blocks;
  std::vector<std::vector<double>> rb(blocks, std::vector<double>(n * n));
  std::vector<std::thread> pool;
  for (int64_t b = 0; b < blocks; ++b) {
    pool.emplace_back([&, b]() {
      const int64_t mb = start[b + 1] - start[b];
      std::vector<double> blk(mb * n);
      for (int64_t c = 0; c < n; ++c)
        std::copy(a.begin() + c * m + start[b], a.begin() + c * m + start[b + 1], blk.begin() + c * mb);
      householder_block(blk.data(), mb, mb, n, rb[b].data());
    });
  }
  for (auto& t : pool) t.join();
  const int64_t ms = blocks * n;
  std::vector<double> stacked(ms * n);
  for (int64_t b = 0; b < blocks; ++b)
    for (int64_t c = 0; c < n; ++c)
      for (int64_t i = 0; i < n; ++i) stacked[c * ms + b * n + i] = rb[b][c * n + i];
  householder_block(stacked.data(), ms, ms, n, r.data());
  return r;
}

void jacobi_svd(std::vector<double>& g, int64_t n, std::vector<double>& s, std::vector<double>& v) {
  v.assign(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i) v[i * n + i] = 1.0;
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 80; ++sweep) {
    double off = 0.0;
    for (int64_t ci = 0; ci < n - 1; ++ci) {
      for (int64_t cj = ci + 1; cj < n; ++cj) {
        double* gi = &g[ci * n];
        double* gj = &g[cj * n];
        double alpha = 0.0, beta = 0.0, gamma = 0.0;
        for (int64_t i = 0; i < n; ++i) {
          alpha += gi[i] * gi[i];
          beta += gj[i] * gj[i];
          gamma += gi[i] * gj[i];
        }
        if (alpha == 0.0 || beta == 0.0) continue;
        const double rel = std::fabs(gamma) / std::sqrt(alpha * beta);
        off = std::max(off, rel);
        if (rel <= tol) continue;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t);
        const double sn = c * t;
        for (int64_t i = 0; i < n; ++i) {
          const double a = gi[i], b = gj[i];
          gi[i] = c * a - sn * b;
          gj[i] = sn * a + c * b;
        }
        double* vi = &v[ci * n];
        double* vj = &v[cj * n];
        for (int64_t i = 0; i < n; ++i) {
          const double a = vi[i], b = vj[i];
          vi[i] = c * a - sn * b;
          vj[i] = sn * a + c * b;
        }
      }
    }
    if (off <= tol) break;
  }
  std::vector<double> sv(n);
  for (int64_t c = 0; c < n; ++c) {
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += g[c * n + i] * g[c * n + i];
    sv[c] = std::sqrt(acc);
  }
  std::vector<int64_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return sv[a] > sv[b]; });
  std::vector<double> u2(n * n), v2(n * n);
  s.assign(n, 0.0);
  for (int64_t c = 0; c < n; ++c) {
    const int64_t src = perm[c];
    s[c] = sv[src];
    for (int64_t i = 0; i < n; ++i) {
      u2[c * n + i] = sv[src] > 0.0 ? g[src * n + i] / sv[src] : 0.0;
      v2[c * n + i] = v[src * n + i];
    }
  }
  g.swap(u2);
  v.swap(v2);
}

bool splits_cluster(const std::vector<double>& s, int64_t k) {
  return k > 0 && k < (int64_t)s.size() && (s[k - 1] - s[k]) <= 1e-8 * s[k - 1];
}

int64_t kept_rank(const std::vector<double>& s, double eps) {
  int64_t k = 0;
  for (double x : s)
    if (x > eps * s[0]) ++k;
  while (splits_cluster(s, k)) ++k;
  return k;
}

}  // namespace kifmm
