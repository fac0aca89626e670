// FP64 operator precompute (Table 1) at unit box half-width.
//
// For the Laplace kernel, K(a x, a y) = K(x, y) / a, so every operator below
// except the leaf S2U factor is the same at all levels:
//   U2U:  pinv(K(UC_P, UE_P)) K(UC_P, UE_C)   (parent radius 2, child radius 1)
//   D2D:  pinv(K(DC_C, DE_C)) K(DC_C, DE_P)
//   U2D:  pinv(K(DC_B, DE_B)) K(DC_B, UE_A)  = post C_t V_k^T after compression,
// and the S2U pseudo-inverse at a leaf of radius r is r times the unit one.
#include <algorithm>
#include <cmath>
#include <functional>
#include <string>
#include <thread>

#include "common.hpp"
#include "linalg.hpp"

namespace kifmm {

namespace {

void parallel_for(int64_t count, const std::function<void(int64_t)>& body) {
  const int64_t workers = std::max<int64_t>(1, std::min<int64_t>(count, std::max(1u, std::thread::hardware_concurrency())));
  std::vector<std::thread> pool;
  for (int64_t w = 0; w < workers; ++w)
    pool.emplace_back([&, w]() {
      for (int64_t i = w; i < count; i += workers) body(i);
    });
  for (auto& t : pool) t.join();
}

inline double lap(double dx, double dy, double dz) {
  const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
  return r > 0.0 ? 1.0 / r : 0.0;
}

// Row-major K[a][b] = K(cx + ax S_a, cy + ay S_b) for surfaces scaled by ax, ay
// and centred at cx, cy.
std::vector<double> surface_kernel(const std::vector<double>& S, int n, double ax, const double* cx, double ay,
                                   const double* cy) {
  std::vector<double> k((size_t)n * n);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      k[(size_t)a * n + b] = lap(cx[0] + ax * S[3 * a] - cy[0] - ay * S[3 * b],
                                 cx[1] + ax * S[3 * a + 1] - cy[1] - ay * S[3 * b + 1],
                                 cx[2] + ax * S[3 * a + 2] - cy[2] - ay * S[3 * b + 2]);
  return k;
}

// c[m][n] = a[m][k] * b[k][n], row-major.
std::vector<double> matmul(const std::vector<double>& a, const std::vector<double>& b, int m, int k, int n) {
  std::vector<double> c((size_t)m * n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int l = 0; l < k; ++l) {
      const double av = a[(size_t)i * k + l];
      if (av == 0.0) continue;
      const double* br = &b[(size_t)l * n];
      double* cr = &c[(size_t)i * n];
      for (int j = 0; j < n; ++j) cr[j] += av * br[j];
    }
  return c;
}

void check_finite(const std::vector<double>& v, const char* what) {
  for (double x : v)
    if (!std::isfinite(x)) fail(KIFMM_E_NUMERIC, std::string("non-finite value in ") + what);
}

}  // namespace

Ops* precompute_ops(int p, double alpha_inner, double alpha_outer, double eps_pinv, double eps_svd) {
  require(p >= 2 && p <= 12, "p must be in [2, 12]");
  // The equivalent surface must enclose the box (alpha_inner > 1) inside the check
  // surface (alpha_inner < alpha_outer), and a V-list source's equivalent surface
  // must stay outside the target's check surface: V-list centres are at least 4 r
  // apart in the max norm, so alpha_inner + alpha_outer <= 4.
  require(std::isfinite(alpha_inner) && std::isfinite(alpha_outer) && alpha_inner > 1.0 &&
              alpha_inner < alpha_outer && alpha_inner + alpha_outer <= 4.0 + 1e-12,
          "surface radii must satisfy 1 < alpha_inner < alpha_outer and alpha_inner + alpha_outer <= 4");
  require(eps_pinv > 0.0 && eps_pinv < 1.0, "eps_pinv must be in (0, 1)");
  const int n = 6 * (p - 1) * (p - 1) + 2;
  int rank = 0;
  if (eps_svd < 0.0) {
    require(eps_svd == std::floor(eps_svd) && -eps_svd <= (double)n,
            "a negative eps_svd gives the rank: it must be an integer -k with 1 <= k <= n");
    rank = (int)(-eps_svd);
  } else {
    require(eps_svd > 0.0 && eps_svd < 1.0, "eps_svd must be in (0, 1), or a negative integer rank");
  }

  Ops* o = new Ops();
  try {
    o->p = p;
    o->n = n;
    o->eps_pinv = eps_pinv;
    o->eps_svd = eps_svd;
    o->alpha_inner = alpha_inner;
    o->alpha_outer = alpha_outer;
    const double ai = alpha_inner, ao = alpha_outer;
    // Surface: grid points of {-1..1}^3, p per edge, on the cube boundary; each
    // coordinate is (2i - (p-1)) / (p-1).
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j)
        for (int k = 0; k < p; ++k)
          if (i == 0 || i == p - 1 || j == 0 || j == p - 1 || k == 0 || k == p - 1) {
            o->surf.push_back((double)(2 * i - (p - 1)) / (double)(p - 1));
            o->surf.push_back((double)(2 * j - (p - 1)) / (double)(p - 1));
            o->surf.push_back((double)(2 * k - (p - 1)) / (double)(p - 1));
          }
    const std::vector<double>& S = o->surf;
    const double zero[3] = {0, 0, 0};

    // Check-to-equivalent pseudo-inverses.  K(DC, DE) = K(UC, UE)^T at equal radius,
    // so DC2E = UC2E^T.
    std::vector<double> kuc = surface_kernel(S, n, ao, zero, ai, zero);
    std::vector<double> g((size_t)n * n);  // column-major copy
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) g[(size_t)b * n + a] = kuc[(size_t)a * n + b];
    std::vector<double> sv, vv;
    jacobi_svd(g, n, sv, vv);  // g <- U, vv <- V (column-major)
    const int kc = (int)kept_rank(sv, eps_pinv);
    o->kc = kc;
    o->f1.assign((size_t)kc * n, 0.0);
    o->f2.assign((size_t)n * kc, 0.0);
    for (int c = 0; c < kc; ++c)
      for (int i = 0; i < n; ++i) {
        o->f1[(size_t)c * n + i] = g[(size_t)c * n + i];              // U^T row c
        o->f2[(size_t)i * kc + c] = vv[(size_t)c * n + i] / sv[c];    // V S^-1 column c
      }
    o->uc2e = matmul(o->f2, o->f1, n, kc, n);
    o->dc2e.assign((size_t)n * n, 0.0);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) o->dc2e[(size_t)a * n + b] = o->uc2e[(size_t)b * n + a];

    // U2U and D2D for the 8 child positions (x in bit 0, y bit 1, z bit 2).
    o->m2m.resize((size_t)8 * n * n);
    o->l2l.resize((size_t)8 * n * n);
    std::vector<double> uc2e_parent(o->uc2e);
    for (double& x : uc2e_parent) x *= 2.0;  // parent radius 2
    for (int oc = 0; oc < 8; ++oc) {
      const double off[3] = {(double)(2 * (oc & 1) - 1), (double)(2 * ((oc >> 1) & 1) - 1),
                             (double)(2 * ((oc >> 2) & 1) - 1)};
      std::vector<double> kup = surface_kernel(S, n, 2.0 * ao, zero, ai, off);
      std::vector<double> m = matmul(uc2e_parent, kup, n, n, n);
      std::copy(m.begin(), m.end(), o->m2m.begin() + (size_t)oc * n * n);
      std::vector<double> kdn = surface_kernel(S, n, ai, off, 2.0 * ao, zero);
      std::vector<double> l = matmul(o->dc2e, kdn, n, n, n);
      std::copy(l.begin(), l.end(), o->l2l.begin() + (size_t)oc * n * n);
    }

    // U2D operators of the 316 V-list offsets t (|t|_inf in {2, 3}), lexicographic order.
    for (int tx = -3; tx <= 3; ++tx)
      for (int ty = -3; ty <= 3; ++ty)
        for (int tz = -3; tz <= 3; ++tz)
          if (std::max({std::abs(tx), std::abs(ty), std::abs(tz)}) >= 2) {
            o->offsets.push_back(tx);
            o->offsets.push_back(ty);
            o->offsets.push_back(tz);
          }
    const int nt = (int)o->offsets.size() / 3;
    std::vector<std::vector<double>> kt(nt);
    parallel_for(nt, [&](int64_t t) {
      const double c[3] = {2.0 * o->offsets[3 * t], 2.0 * o->offsets[3 * t + 1], 2.0 * o->offsets[3 * t + 2]};
      kt[t] = surface_kernel(S, n, ai, c, ai, zero);
    });
    // Column-major stacks: fat^T = [K_1^T; ...; K_m^T] and tall = [K_1; ...; K_m], both (m n) x n.
    const int64_t rows = (int64_t)nt * n;
    std::vector<double> fat_t((size_t)rows * n), tall((size_t)rows * n);
    for (int t = 0; t < nt; ++t)
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          const double v = kt[t][(size_t)a * n + b];
          fat_t[(size_t)a * rows + (int64_t)t * n + b] = v;  // row t n + b, column a
          tall[(size_t)b * rows + (int64_t)t * n + a] = v;   // row t n + a, column b
        }
    std::vector<double> rf = qr_r_factor(fat_t, rows, n);
    std::vector<double> rt = qr_r_factor(tall, rows, n);
    fat_t.clear();
    fat_t.shrink_to_fit();
    tall.clear();
    tall.shrink_to_fit();
    std::vector<double> sf, wf, st, wt;
    jacobi_svd(rf, n, sf, wf);  // left singular vectors of the fat stack = right ones of its R
    jacobi_svd(rt, n, st, wt);  // right singular vectors of the tall stack
    int k = rank > 0 ? rank : 0;
    if (rank == 0)
      for (double x : sf)
        if (x > eps_svd * sf[0]) ++k;
    k = std::max(1, std::min(k, n));
    while (k < n && (splits_cluster(sf, k) || splits_cluster(st, k))) ++k;
    o->k = k;
    o->mu.assign((size_t)n * k, 0.0);
    o->mv.assign((size_t)n * k, 0.0);
    for (int c = 0; c < k; ++c)
      for (int i = 0; i < n; ++i) {
        o->mu[(size_t)i * k + c] = wf[(size_t)c * n + i];
        o->mv[(size_t)i * k + c] = wt[(size_t)c * n + i];
      }
    // C_t = U_k^T K_t V_k.
    std::vector<double> mut((size_t)k * n);
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < k; ++c) mut[(size_t)c * n + i] = o->mu[(size_t)i * k + c];
    o->cores.resize((size_t)nt * k * k);
    parallel_for(nt, [&](int64_t t) {
      std::vector<double> kv = matmul(kt[t], o->mv, n, n, k);
      std::vector<double> c = matmul(mut, kv, k, n, k);
      std::copy(c.begin(), c.end(), o->cores.begin() + (size_t)t * k * k);
    });
    o->post = matmul(o->dc2e, o->mu, n, n, k);

    check_finite(o->f1, "UC2E factor");
    check_finite(o->f2, "UC2E factor");
    check_finite(o->m2m, "M2M");
    check_finite(o->l2l, "L2L");
    check_finite(o->cores, "M2L cores");
    check_finite(o->post, "M2L post");
  } catch (...) {
    delete o;
    throw;
  }
  return o;
}

}  // namespace kifmm
