// Host FP64 linear algebra used at plan time (see linalg.hpp).
#include "linalg.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace fio {

// Cyclic Jacobi for a complex Hermitian matrix.  Each rotation acts on the
// pair (p, q) with a_pq = |a_pq| e^{i phi}:
//   J = [[c, s e^{i phi}], [-s e^{-i phi}, c]],  A <- J^H A J,  V <- V J,
// with t = s / c the smaller root of t^2 + 2 tau t - 1 = 0,
// tau = (a_qq - a_pp) / (2 |a_pq|), which zeroes the (p, q) entry.
int eigh_jacobi(int n, std::vector<zd> &A, std::vector<double> &w, std::vector<zd> &V) {
    V.assign((size_t)n * n, zd(0, 0));
    for (int i = 0; i < n; ++i)
        V[(size_t)i * n + i] = 1.0;
    auto at = [&](int i, int j) -> zd & { return A[(size_t)i * n + j]; };
    double fro = 0;
    for (const zd &z : A)
        fro += std::norm(z);
    fro = std::sqrt(fro);
    int sweep = 0;
    for (; sweep < 60; ++sweep) {
        double off = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                off += std::norm(at(i, j));
        if (std::sqrt(2 * off) <= 1e-16 * fro || fro == 0)
            break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const zd apq = at(p, q);
                const double mag = std::abs(apq);
                if (mag == 0 || mag < 1e-300)
                    continue;
                const double app = at(p, p).real(), aqq = at(q, q).real();
                const double tau = (aqq - app) / (2 * mag);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1 + tau * tau));
                const double c = 1 / std::sqrt(1 + t * t), s = t * c;
                const zd e = apq / mag;              // e^{i phi}
                const zd se = s * e, sec = s * std::conj(e);
                // columns: A <- A J
                for (int k = 0; k < n; ++k) {
                    const zd akp = at(k, p), akq = at(k, q);
                    at(k, p) = c * akp - sec * akq;
                    at(k, q) = se * akp + c * akq;
                }
                // rows: A <- J^H A
                for (int k = 0; k < n; ++k) {
                    const zd apk = at(p, k), aqk = at(q, k);
                    at(p, k) = c * apk - se * aqk;
                    at(q, k) = sec * apk + c * aqk;
                }
                at(p, q) = 0;
                at(q, p) = 0;
                at(p, p) = at(p, p).real();
                at(q, q) = at(q, q).real();
                for (int k = 0; k < n; ++k) {
                    zd &vp = V[(size_t)k * n + p];
                    zd &vq = V[(size_t)k * n + q];
                    const zd a0 = vp, b0 = vq;
                    vp = c * a0 - sec * b0;
                    vq = se * a0 + c * b0;
                }
            }
        }
    }
    // sort descending
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::vector<double> d(n);
    for (int i = 0; i < n; ++i)
        d[i] = at(i, i).real();
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] > d[b]; });
    w.resize(n);
    std::vector<zd> Vs((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        w[j] = d[idx[j]];
        for (int k = 0; k < n; ++k)
            Vs[(size_t)k * n + j] = V[(size_t)k * n + idx[j]];
    }
    V.swap(Vs);
    return sweep;
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
    eigh_jacobi(k, H, lam, W);
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

}  // namespace fio
