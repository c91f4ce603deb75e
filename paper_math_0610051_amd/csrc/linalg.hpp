// Small dense FP64 linear algebra of the plan (host side): Hermitian
// eigen-decomposition (Householder tridiagonalisation and implicit QL) and a
// pseudo-inverse of a tall matrix through its Gram matrix.  Sizes are the
// separation's sample counts (r <= 256).
#pragma once

#include <complex>
#include <vector>

namespace fio {

using zd = std::complex<double>;

// A: n x n Hermitian (row-major, overwritten).  w: eigenvalues, descending.
// V: n x n, eigenvectors as columns (row-major).
// Householder tridiagonalisation and implicit QL, O(n^3) with a small
// constant; returns the QL iterations.
int eigh(int n, std::vector<zd> &A, std::vector<double> &w, std::vector<zd> &V);

// P = pinv(U) for U (m x k, m >= k, row-major), singular values below
// rcond * s_max discarded.  P is k x m (row-major).
void pinv_tall(int m, int k, const std::vector<zd> &U, std::vector<zd> &P, double rcond);

// Column interpolative decomposition of A (m x n, row-major): returns k and
// a column order perm such that A(:, perm[k..n)) ~ A(:, perm[0..k)) T (T is
// k x (n - k), row-major); pivoting stops at a remaining column norm of
// tol times the first pivot's.
int column_id(int m, int n, std::vector<zd> A, double tol, std::vector<int> &perm, std::vector<zd> &T);

}  // namespace fio
