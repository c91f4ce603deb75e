// Host FP64 linear algebra used at plan time (see linalg.hpp).
#include "linalg.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace fio {

// Householder tridiagonalisation and implicit QL (Golub and Van Loan,
// "Matrix Computations", Sections 8.3.1 and 8.3.5).
//  1. For k = 0 .. n-3 a reflector H_k = I - 2 v v^H (|v| = 1, v zero in
//     rows 0..k) maps column k below the diagonal onto a multiple of e_{k+1};
//     A <- H_k A H_k is applied as A - v w^H - w v^H with p = 2 A v,
//     w = p - (v^H p) v, and Q <- Q H_k accumulates the reflectors.
//  2. The Hermitian tridiagonal result has complex off-diagonals b_k; the
//     unitary diagonal D with D_{k+1} = D_k b_k / |b_k| turns it into the
//     real symmetric tridiagonal T = D^H (Q^H A Q) D with off-diagonal |b_k|.
//  3. Implicit QL with Wilkinson shifts diagonalises T by plane rotations,
//     applied to the columns of Z = Q D, which then hold the eigenvectors.
int eigh(int n, std::vector<zd> &A, std::vector<double> &w, std::vector<zd> &V) {
    auto at = [&](int i, int j) -> zd & { return A[(size_t)i * n + j]; };
    std::vector<zd> Q((size_t)n * n, zd(0, 0));
    for (int i = 0; i < n; ++i)
        Q[(size_t)i * n + i] = 1.0;
    std::vector<zd> v(n), pv(n), wv(n);
    for (int k = 0; k + 2 < n; ++k) {
        double nx = 0;
        for (int i = k + 1; i < n; ++i)
            nx += std::norm(at(i, k));
        nx = std::sqrt(nx);
        if (nx == 0)
            continue;
        const zd x0 = at(k + 1, k);
        const double ax0 = std::abs(x0);
        const zd ph = ax0 > 0 ? x0 / ax0 : zd(1, 0);
        const zd alpha = -ph * nx;  // the image of x: alpha e_{k+1}
        // v = (x - alpha e_{k+1}) / |x - alpha e_{k+1}|
        for (int i = 0; i <= k; ++i)
            v[i] = 0;
        for (int i = k + 1; i < n; ++i)
            v[i] = at(i, k);
        v[k + 1] -= alpha;
        double nv = 0;
        for (int i = k + 1; i < n; ++i)
            nv += std::norm(v[i]);
        nv = std::sqrt(nv);
        if (nv == 0)
            continue;
        for (int i = k + 1; i < n; ++i)
            v[i] /= nv;
        // p = 2 A v over rows and columns k .. n-1 (column k included, so that
        // the reflected column comes out of the same update)
        for (int i = k; i < n; ++i) {
            zd sacc(0, 0);
            for (int j = k + 1; j < n; ++j)
                sacc += at(i, j) * v[j];
            pv[i] = 2.0 * sacc;
        }
        zd vhp(0, 0);
        for (int i = k + 1; i < n; ++i)
            vhp += std::conj(v[i]) * pv[i];
        for (int i = k; i < n; ++i)
            wv[i] = pv[i] - vhp * v[i];
        for (int i = k; i < n; ++i)
            for (int j = k; j < n; ++j)
                at(i, j) -= v[i] * std::conj(wv[j]) + wv[i] * std::conj(v[j]);
        // exact zeros below the sub-diagonal and the reflected entry
        for (int i = k + 2; i < n; ++i)
            at(i, k) = at(k, i) = 0;
        at(k + 1, k) = alpha;
        at(k, k + 1) = std::conj(alpha);
        // Q <- Q H_k
        for (int i = 0; i < n; ++i) {
            zd qv(0, 0);
            for (int j = k + 1; j < n; ++j)
                qv += Q[(size_t)i * n + j] * v[j];
            qv *= 2.0;
            for (int j = k + 1; j < n; ++j)
                Q[(size_t)i * n + j] -= qv * std::conj(v[j]);
        }
    }
    // real tridiagonal: d (diagonal), e[k] between k and k+1
    std::vector<double> d(n), e(n, 0.0);
    std::vector<zd> D(n);
    D[0] = 1;
    for (int k = 0; k < n; ++k)
        d[k] = at(k, k).real();
    for (int k = 0; k + 1 < n; ++k) {
        const zd b = at(k + 1, k);
        const double ab = std::abs(b);
        e[k] = ab;
        D[k + 1] = ab > 0 ? D[k] * (b / ab) : D[k];
    }
    V.assign((size_t)n * n, zd(0, 0));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            V[(size_t)i * n + j] = Q[(size_t)i * n + j] * D[j];
    // implicit QL on (d, e)
    int iters = 0;
    for (int l = 0; l < n; ++l) {
        for (int guard = 0; guard < 60; ++guard) {
            int m = l;
            for (; m + 1 < n; ++m) {
                // e[m] is negligible when adding it to |d[m]| + |d[m+1]| changes nothing
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                volatile double sum = std::fabs(e[m]) + dd;
                if (sum == dd)
                    break;
            }
            if (m == l)
                break;
            ++iters;
            // Wilkinson-type shift from the leading 2 x 2 block
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double s = 1, c = 1, p = 0;
            int i = m - 1;
            for (; i >= l; --i) {
                const double f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0) {
                    d[i + 1] -= p;
                    e[m] = 0;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                for (int k = 0; k < n; ++k) {
                    const zd zf = V[(size_t)k * n + i + 1], zi = V[(size_t)k * n + i];
                    V[(size_t)k * n + i + 1] = s * zi + c * zf;
                    V[(size_t)k * n + i] = c * zi - s * zf;
                }
            }
            if (r == 0 && i >= l)
                continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0;
        }
    }
    // sort descending
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] > d[b]; });
    w.resize(n);
    std::vector<zd> Vs((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        w[j] = d[idx[j]];
        for (int k = 0; k < n; ++k)
            Vs[(size_t)k * n + j] = V[(size_t)k * n + idx[j]];
    }
    V.swap(Vs);
    return iters;
}

void pinv_tall(int m, int k, const std::vector<zd> &U, std::vector<zd> &P, double rcond) {
    // H = U^H U (k x k) = W diag(lam) W^H;  pinv = W diag(1/lam) W^H U^H
    std::vector<zd> H((size_t)k * k, zd(0, 0));
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            zd s(0, 0);
            for (int i = 0; i < m; ++i)
                s += std::conj(U[(size_t)i * k + a]) * U[(size_t)i * k + b];
            H[(size_t)a * k + b] = s;
        }
    std::vector<double> lam;
    std::vector<zd> W;
    eigh(k, H, lam, W);
    const double lmax = lam.empty() ? 0 : lam[0];
    // M = W diag(1/lam) W^H
    std::vector<zd> Mi((size_t)k * k, zd(0, 0));
    for (int j = 0; j < k; ++j) {
        if (!(lam[j] > rcond * rcond * lmax) || lam[j] <= 0)
            continue;
        const double inv = 1.0 / lam[j];
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
                Mi[(size_t)a * k + b] += W[(size_t)a * k + j] * inv * std::conj(W[(size_t)b * k + j]);
    }
    P.assign((size_t)k * m, zd(0, 0));
    for (int a = 0; a < k; ++a)
        for (int i = 0; i < m; ++i) {
            zd s(0, 0);
            for (int b = 0; b < k; ++b)
                s += Mi[(size_t)a * k + b] * std::conj(U[(size_t)i * k + b]);
            P[(size_t)a * m + i] = s;
        }
}

// Column interpolative decomposition by Householder QR with column pivoting
// (Golub and Van Loan, Section 5.4.1; Cheng, Gimbutas, Martinsson and
// Rokhlin, "On the compression of low rank matrices", 2005).  Step j swaps
// the remaining column of largest norm into place and stops once that norm
// is at most tol times the first pivot's; with k steps taken, A P = Q [R11
// R12] on the leading k rows gives A(:, P(k..n)) ~ A(:, P(0..k)) T,
// T = R11^-1 R12.
int column_id(int m, int n, std::vector<zd> A, double tol, std::vector<int> &perm, std::vector<zd> &T) {
    auto at = [&](int i, int j) -> zd & { return A[(size_t)i * n + j]; };
    perm.resize(n);
    std::iota(perm.begin(), perm.end(), 0);
    const int kmax = std::min(m, n);
    double first = 0;
    int k = 0;
    std::vector<zd> v(m);
    for (; k < kmax; ++k) {
        // column of largest norm in rows k..m-1
        int best = k;
        double bn = -1;
        for (int j = k; j < n; ++j) {
            double s = 0;
            for (int i = k; i < m; ++i)
                s += std::norm(at(i, j));
            if (s > bn) {
                bn = s;
                best = j;
            }
        }
        bn = std::sqrt(bn);
        if (k == 0)
            first = bn;
        if (bn <= tol * first || bn == 0)
            break;
        if (best != k) {
            for (int i = 0; i < m; ++i)
                std::swap(at(i, k), at(i, best));
            std::swap(perm[k], perm[best]);
        }
        // reflector mapping column k (rows k..) onto alpha e_k
        const zd x0 = at(k, k);
        const double ax0 = std::abs(x0);
        const zd alpha = -(ax0 > 0 ? x0 / ax0 : zd(1, 0)) * bn;
        double vn = 0;
        for (int i = k; i < m; ++i) {
            v[i] = at(i, k) - (i == k ? alpha : zd(0, 0));
            vn += std::norm(v[i]);
        }
        vn = std::sqrt(vn);
        if (vn > 0) {
            for (int i = k; i < m; ++i)
                v[i] /= vn;
            for (int j = k; j < n; ++j) {
                zd d(0, 0);
                for (int i = k; i < m; ++i)
                    d += std::conj(v[i]) * at(i, j);
                for (int i = k; i < m; ++i)
                    at(i, j) -= 2.0 * v[i] * d;
            }
        }
    }
    // T = R11^-1 R12 by back substitution, k x (n - k)
    T.assign((size_t)k * (n - k), zd(0, 0));
    for (int c = 0; c < n - k; ++c)
        for (int i = k - 1; i >= 0; --i) {
            zd s = at(i, k + c);
            for (int j = i + 1; j < k; ++j)
                s -= at(i, j) * T[(size_t)j * (n - k) + c];
            T[(size_t)i * (n - k) + c] = s / at(i, i);
        }
    return k;
}

}  // namespace fio
