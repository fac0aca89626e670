// FP64 dense linear algebra for the operator precompute: Householder QR (R
// factor only) and one-sided Jacobi SVD.  Matrices are column-major.
#pragma once

#include <cstdint>
#include <vector>

namespace kifmm {

// R factor (n x n, upper triangular, column-major) of the QR factorisation of
// the column-major m x n matrix `a` (m >= n).  `a` is overwritten.  Rows are
// split into blocks factorised in parallel, then the stacked block R factors
// are factorised again (a tall-skinny QR).
std::vector<double> qr_r_factor(std::vector<double>& a, int64_t m, int64_t n);

// One-sided Jacobi SVD of the column-major n x n matrix `g`:
//   g = U diag(s) V^T with s sorted in decreasing order.
// On return `g` holds U (columns with s = 0 are zero), `v` holds V.
void jacobi_svd(std::vector<double>& g, int64_t n, std::vector<double>& s, std::vector<double>& v);

// Number of leading singular values kept for relative cutoff eps, extended so
// that no cluster of equal values (relative gap <= 1e-8) is split.
int64_t kept_rank(const std::vector<double>& s, double eps);
bool splits_cluster(const std::vector<double>& s, int64_t k);

}  // namespace kifmm
