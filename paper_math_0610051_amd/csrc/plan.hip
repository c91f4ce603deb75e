// Plan construction: the preprocessing step of Section 3 for the wedge FIO.
//
//   1. partition Omega into angular wedges (Section 1.3) or dyadic coronae cut
//      into angular wedges;
//   2. per wedge, an integer shear M and translation xi_c giving a small centred
//      box (Section 3.4), and an oversampled FFT grid for the type-2 NUFFT;
//   3. per wedge, the randomized separation of exp(2 pi i Phi_ell) (Section 3.2):
//      r sampled columns, their FP64 Gram matrix reduced on the GPU, a host
//      Hermitian eigen-decomposition (the SVD of A_[C] through its Gram matrix),
//      rank q from the singular-value threshold, r sampled rows and the
//      pseudo-inverse U_[R]^+, the compressed form A_[C] (V S^-1) U_[R]^+ A_[R]
//      of eq. (probnewfac), an s x s error estimate (Section 4), and adaptive
//      doubling of r (accept when q <= r/3);
//   4. the factors gamma^x = A_[C] V S^-1 (all x) and gamma^xi = U_[R]^+ A_[R]
//      (all members, deconvolution and 1/N folded in) evaluated on the GPU in
//      FP64 and stored in the plan's precision.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>

#include "apply.hpp"
#include "errors.hpp"
#include "linalg.hpp"
#include "learned.hpp"
#include "plan_build.hpp"

namespace fio {

// ---------------------------------------------------------------------------
// Partitions (host, FP64).  Same half-open rule for both: the wedge of angle
// index k among n covers [(2k - 1) pi/n, (2k + 1) pi/n) with arg in [0, 2 pi).
// ---------------------------------------------------------------------------
static int angular_index(int k1, int k2, int n) {
    double a = std::atan2((double)k2, (double)k1);
    if (a < 0)
        a += kTwoPi;
    const double width = kTwoPi / n;
    long long id = (long long)std::floor((a + M_PI / n) / width);
    return (int)(id % n);
}

void partition_equiangular(int N, int L, std::vector<int> &ids, std::vector<double> &thetas) {
    ids.assign((size_t)N * N, 0);
    const int h = N / 2;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            const int k1 = i - h, k2 = j - h;
            ids[(size_t)i * N + j] = (k1 == 0 && k2 == 0) ? 0 : angular_index(k1, k2, L);
        }
    thetas.resize(L);
    for (int l = 0; l < L; ++l)
        thetas[l] = kTwoPi * l / L;
}

// Corona 0 holds |xi| < 8 (and xi = 0); corona j >= 1 holds 2^(j+2) <= |xi| < 2^(j+3);
// corona j is cut into n_j = 8 * 2^ceil(j/2) angular wedges.
void partition_coronae(int N, std::vector<int> &ids, std::vector<double> &thetas) {
    const int h = N / 2;
    ids.assign((size_t)N * N, 0);
    double rmax = 0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            const double k1 = i - h, k2 = j - h;
            rmax = std::max(rmax, std::sqrt(k1 * k1 + k2 * k2));
        }
    thetas.clear();
    int base = 0;
    for (int jc = 0;; ++jc) {
        const double lo = jc == 0 ? 0.0 : std::ldexp(1.0, jc + 2);
        const double hi = std::ldexp(1.0, jc + 3);
        if (lo > rmax)
            break;
        const int nj = 8 << ((jc + 1) / 2);
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                const int k1 = i - h, k2 = j - h;
                const double rad = std::sqrt((double)k1 * k1 + (double)k2 * k2);
                if (rad >= lo && rad < hi)
                    ids[(size_t)i * N + j] = base + angular_index(k1, k2, nj);
            }
        for (int k = 0; k < nj; ++k)
            thetas.push_back(kTwoPi * k / nj);
        base += nj;
    }
    ids[(size_t)h * N + h] = 0;
}

// ---------------------------------------------------------------------------
// Geometry of one wedge: an integer unimodular shear M and the smallest box of
// the sheared members.  Every M with entries in [-2, 2] and determinant +-1
// is a candidate (the box of the sheared members is that of their convex
// hull).  A candidate is scored by the work it implies per rank and
// right-hand side: the oversampled grid's cells times its FFT passes, plus
// kWindowWeight times the staged interpolation windows, estimated over all
// 16 x 16 output tiles as the tile's image under M^{-T} on the grid plus the
// kernel width (the warp's own spread is left out).  kWindowWeight is the
// measured cost of a staged window unit per transformed cell and pass.
// ---------------------------------------------------------------------------
constexpr int kShearMax = 2;
constexpr double kWindowWeight = 0.34;

static int fft_pass_count(int n) {
    FftPlan pl;
    fft_make_plan(n, pl);
    return std::max(1, pl.npass - 1);  // the leading radix-2 pass is folded into the load
}

// Convex hull of lattice points (Andrew's monotone chain), counter-clockwise.
static std::vector<std::pair<int, int>> hull_of(std::vector<std::pair<int, int>> pts) {
    std::sort(pts.begin(), pts.end());
    pts.erase(std::unique(pts.begin(), pts.end()), pts.end());
    if (pts.size() < 3)
        return pts;
    auto cross = [](const std::pair<int, int> &o, const std::pair<int, int> &a, const std::pair<int, int> &b) {
        return (long long)(a.first - o.first) * (b.second - o.second) -
               (long long)(a.second - o.second) * (b.first - o.first);
    };
    std::vector<std::pair<int, int>> h(2 * pts.size());
    size_t k = 0;
    for (size_t i = 0; i < pts.size(); ++i) {
        while (k >= 2 && cross(h[k - 2], h[k - 1], pts[i]) <= 0)
            --k;
        h[k++] = pts[i];
    }
    for (size_t i = pts.size() - 1, t = k + 1; i > 0; --i) {
        while (k >= t && cross(h[k - 2], h[k - 1], pts[i - 1]) <= 0)
            --k;
        h[k++] = pts[i - 1];
    }
    h.resize(k - 1);
    return h;
}

void wedge_geometry(int N, double sigma, int w, WedgeHost &W) {
    const int h = N / 2;
    std::vector<std::pair<int, int>> pts;
    pts.reserve(W.members.size());
    for (int om : W.members)
        pts.emplace_back(om / N - h, om % N - h);
    const std::vector<std::pair<int, int>> hull = hull_of(pts);
    const double tiles = std::ceil(N / 16.0) * std::ceil(N / 16.0);
    // entries tried in the order 0, 1, -1, 2, -2, and among equal costs the
    // smallest entries win, so an unsheared wedge keeps the identity
    int vals[2 * kShearMax + 1];
    vals[0] = 0;
    for (int v = 1; v <= kShearMax; ++v) {
        vals[2 * v - 1] = v;
        vals[2 * v] = -v;
    }
    double best = -1;
    int best_norm = 0;
    for (int m0 : vals)
        for (int m1 : vals)
            for (int m2 : vals)
                for (int m3 : vals) {
                    const int det = m0 * m3 - m1 * m2;
                    if (det != 1 && det != -1)
                        continue;
                    int M[4] = {m0, m1, m2, m3};
                    int mn1 = 1 << 30, mx1 = -(1 << 30), mn2 = 1 << 30, mx2 = -(1 << 30);
                    for (const auto &pq : hull) {
                        const int a1 = M[0] * pq.first + M[1] * pq.second, a2 = M[2] * pq.first + M[3] * pq.second;
                        mn1 = std::min(mn1, a1);
                        mx1 = std::max(mx1, a1);
                        mn2 = std::min(mn2, a2);
                        mx2 = std::max(mx2, a2);
                    }
                    int B[2] = {mx1 - mn1 + 1, mx2 - mn2 + 1}, xc[2] = {mn1 + B[0] / 2, mn2 + B[1] / 2};
                    // axis 1 is the long side of the box (its FFT runs in the column stage);
                    // swapping the rows of M keeps it unimodular
                    if (B[1] > B[0]) {
                        std::swap(M[0], M[2]);
                        std::swap(M[1], M[3]);
                        std::swap(B[0], B[1]);
                        std::swap(xc[0], xc[1]);
                    }
                    int n[2];
                    for (int d = 0; d < 2; ++d)
                        n[d] = fft_nice_size(std::max((int)std::ceil(sigma * B[d]), 2 * w));
                    const double fft = (double)n[0] * n[1] * (fft_pass_count(n[0]) + fft_pass_count(n[1]));
                    // a tile spans 16 / N of the unit square; row d of M^{-T} = column d of M^{-1}, and
                    // |M^{-1}| has the entries of M up to order and sign
                    const double s1 = std::abs(M[3]) + std::abs(M[2]), s2 = std::abs(M[1]) + std::abs(M[0]);
                    const double f1 = s1 * 16.0 * n[0] / N + w, f2 = s2 * 16.0 * n[1] / N + w;
                    const double win = std::ceil(f2 * (f1 + 2) / 64.0) * 64.0 * tiles;
                    const double cost = fft + kWindowWeight * win;
                    const int norm = std::abs(m0) + std::abs(m1) + std::abs(m2) + std::abs(m3);
                    if (best < 0 || cost < best * (1 - 1e-12) || (cost <= best * (1 + 1e-12) && norm < best_norm)) {
                        best = cost;
                        best_norm = norm;
                        std::memcpy(W.M, M, sizeof(W.M));
                        W.B[0] = B[0];
                        W.B[1] = B[1];
                        W.xc[0] = xc[0];
                        W.xc[1] = xc[1];
                    }
                }
    W.lo[0] = -(W.B[0] / 2);
    W.lo[1] = -(W.B[1] / 2);
    // inverse of a unimodular [[a, b], [c, d]]: [[d, -b], [-c, a]] / det
    const int det = W.M[0] * W.M[3] - W.M[1] * W.M[2];
    W.Minv[0] = W.M[3] * det;
    W.Minv[1] = -W.M[1] * det;
    W.Minv[2] = -W.M[2] * det;
    W.Minv[3] = W.M[0] * det;
}

// ---------------------------------------------------------------------------
// NUFFT kernel: width and shape from the tolerance, Fourier transform by
// Gauss-Legendre quadrature.
// ---------------------------------------------------------------------------
void es_parameters(double eps, double sigma, int forced_w, int &w, double &beta) {
    if (forced_w > 0) {
        w = forced_w;
    } else {
        w = (int)std::ceil(std::log(1.0 / eps) / (M_PI * std::sqrt(1.0 - 1.0 / sigma)));
        w = std::max(w, 4);
    }
    // round up to a compiled width
    int wc = 16;
    for (int v : kInterpWidths)
        if (v >= w) {
            wc = v;
            break;
        }
    w = std::min(wc, 16);
    beta = 0.97 * M_PI * (1.0 - 0.5 / sigma) * w;
}

static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &wt) {
    x.resize(n);
    wt.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16)
                break;
        }
        x[i] = z;
        wt[i] = 2.0 / ((1 - z * z) * dp * dp);
    }
}

// phi_hat(omega) = int_{-w/2}^{w/2} phi(z) exp(-2 pi i omega z) dz (phi even).
double es_fourier(int w, double beta, double omega) {
    static thread_local std::vector<double> gx, gw;
    if (gx.empty())
        gauss_legendre(200, gx, gw);
    const double half = 0.5 * w;
    double s = 0;
    for (size_t i = 0; i < gx.size(); ++i) {
        const double z = half * gx[i];
        s += gw[i] * es_kernel<double>(z, 2.0 / w, beta) * std::cos(kTwoPi * omega * z);
    }
    return s * half;
}

// ---------------------------------------------------------------------------
// Separation kernels (FP64).
// ---------------------------------------------------------------------------
__global__ void k_xcoef(Phase ph, int N, double2 *out) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (long long)N * N)
        return;
    const int n1 = (int)(p / N), n2 = (int)(p % N);
    XCoef c = phase_xcoef(ph, (double)n1 / N, (double)n2 / N);
    out[p] = make_double2(c.a, c.b);
}

__device__ inline double2 residual_at(const Phase &ph, double2 xc, double e1, double e2, double k1, double k2) {
    XCoef c{xc.x, xc.y};
    double g1, g2;
    phase_grad(ph, c, e1, e2, g1, g2);
    double cs, sn;
    residual_entry(ph, c, g1, g2, k1, k2, cs, sn);
    return make_double2(cs, sn);
}

constexpr int kGramTile = 16;
constexpr int kMaxSamples = 256;  // cap on r: the host eigen-solve is O(r^3)
constexpr int kGramRows = 64;

// Partial Gram G = A_C^H A_C over a row range, one 16 x 16 tile per block.
__global__ __launch_bounds__(256) void k_gram(Phase ph, const double2 *__restrict__ xcoef, long long NN, double e1,
                                              double e2, const double2 *__restrict__ cols, int r,
                                              long long rows_per_block, double2 *__restrict__ partial) {
    const int ti = blockIdx.y, tj = blockIdx.z;
    if (ti > tj)
        return;
    __shared__ double2 Ai[kGramRows][kGramTile];
    __shared__ double2 Aj[kGramRows][kGramTile];
    const int tid = threadIdx.x;
    const int ii = tid / kGramTile, jj = tid % kGramTile;
    const int gi = ti * kGramTile + ii, gj = tj * kGramTile + jj;
    const long long x0 = (long long)blockIdx.x * rows_per_block;
    const long long x1 = (x0 + rows_per_block < NN) ? x0 + rows_per_block : NN;
    double sr = 0, si = 0;
    for (long long xb = x0; xb < x1; xb += kGramRows) {
        for (int e = tid; e < 2 * kGramRows * kGramTile; e += blockDim.x) {
            const int which = e / (kGramRows * kGramTile);
            const int rr = (e % (kGramRows * kGramTile)) / kGramTile;
            const int cc = e % kGramTile;
            const long long x = xb + rr;
            const int col = (which ? tj : ti) * kGramTile + cc;
            double2 v = make_double2(0, 0);
            if (x < x1 && col < r)
                v = residual_at(ph, xcoef[x], e1, e2, cols[col].x, cols[col].y);
            if (which)
                Aj[rr][cc] = v;
            else
                Ai[rr][cc] = v;
        }
        __syncthreads();
#pragma unroll 8
        for (int rr = 0; rr < kGramRows; ++rr) {
            const double2 a = Ai[rr][ii], b = Aj[rr][jj];
            // conj(a) * b
            sr += a.x * b.x + a.y * b.y;
            si += a.x * b.y - a.y * b.x;
        }
        __syncthreads();
    }
    if (gi < r && gj < r)
        partial[((long long)blockIdx.x * r + gi) * r + gj] = make_double2(sr, si);
}

__global__ void k_gram_reduce(const double2 *__restrict__ partial, int nblk, int r, double2 *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= r * r)
        return;
    const int i = e / r, j = e % r;
    if (i > j)
        return;
    double sr = 0, si = 0;
    for (int b = 0; b < nblk; ++b) {
        const double2 v = partial[(long long)b * r * r + e];
        sr += v.x;
        si += v.y;
    }
    out[e] = make_double2(sr, si);
}

// gamma^x(x, t) = sum_c A(x, C_c) Z(c, t) for every grid point, stored as T (stride qpad).
template <typename T>
__global__ void k_gamma_x(Phase ph, const double2 *__restrict__ xcoef, long long NN, double e1, double e2,
                          const double2 *__restrict__ cols, int r, const double2 *__restrict__ Z, int q, int qpad,
                          cplx<T> *__restrict__ out) {
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= NN)
        return;
    constexpr int kQ = 32;
    double ar[kQ], ai[kQ];
    for (int t0 = 0; t0 < q; t0 += kQ) {
        const int nt = min(kQ, q - t0);
#pragma unroll
        for (int t = 0; t < kQ; ++t)
            ar[t] = ai[t] = 0;
        const double2 xc = xcoef[x];
        for (int c = 0; c < r; ++c) {
            const double2 a = residual_at(ph, xc, e1, e2, cols[c].x, cols[c].y);
            const double2 *zr = Z + (long long)c * q + t0;
#pragma unroll
            for (int t = 0; t < kQ; ++t)
                if (t < nt) {
                    const double2 z = zr[t];
                    ar[t] += a.x * z.x - a.y * z.y;
                    ai[t] += a.x * z.y + a.y * z.x;
                }
        }
#pragma unroll
        for (int t = 0; t < kQ; ++t)
            if (t < nt)
                out[x * qpad + t0 + t] = cmake<T>((T)ar[t], (T)ai[t]);
    }
    for (int t = q; t < qpad; ++t)
        out[x * qpad + t] = cmake<T>(0, 0);
}

// gamma^xi(m, t) = scale(m) * sum_i P(t, i) A(R_i, xi_m) for every member, stride qpad.
template <typename T>
__global__ void k_gamma_xi(Phase ph, int N, const int *__restrict__ omega, const double *__restrict__ scale, int nmem,
                           const double4 *__restrict__ rows, int r, const double2 *__restrict__ P, int q, int qpad,
                           cplx<T> *__restrict__ out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nmem)
        return;
    const int h = N / 2;
    const int om = omega[m];
    const double k1 = om / N - h, k2 = om % N - h;
    constexpr int kQ = 32;
    double ar[kQ], ai[kQ];
    for (int t0 = 0; t0 < q; t0 += kQ) {
        const int nt = min(kQ, q - t0);
#pragma unroll
        for (int t = 0; t < kQ; ++t)
            ar[t] = ai[t] = 0;
        for (int i = 0; i < r; ++i) {
            const double4 rw = rows[i];  // a, b, g1, g2 of row R_i
            XCoef c{rw.x, rw.y};
            double cs, sn;
            residual_entry(ph, c, rw.z, rw.w, k1, k2, cs, sn);
#pragma unroll
            for (int t = 0; t < kQ; ++t)
                if (t < nt) {
                    const double2 pv = P[(long long)(t0 + t) * r + i];
                    ar[t] += pv.x * cs - pv.y * sn;
                    ai[t] += pv.x * sn + pv.y * cs;
                }
        }
        const double s = scale[m];
#pragma unroll
        for (int t = 0; t < kQ; ++t)
            if (t < nt)
                out[(long long)m * qpad + t0 + t] = cmake<T>((T)(s * ar[t]), (T)(s * ai[t]));
    }
    for (int t = q; t < qpad; ++t)
        out[(long long)m * qpad + t] = cmake<T>(0, 0);
}

__global__ void k_warp(Phase ph, int N, double e1, double e2, const long long *__restrict__ xidx, int nx,
                       double *__restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx)
        return;
    const long long p = xidx[i];
    const int n1 = (int)(p / N), n2 = (int)(p % N);
    const double x1 = (double)n1 / N, x2 = (double)n2 / N;
    const XCoef c = phase_xcoef(ph, x1, x2);
    double g1, g2;
    phase_grad(ph, c, e1, e2, g1, g2);
    y[2 * i] = x1 + g1;
    y[2 * i + 1] = x2 + g2;
}

template __global__ void k_gamma_x<float>(Phase, const double2 *, long long, double, double, const double2 *, int,
                                          const double2 *, int, int, cplx<float> *);
template __global__ void k_gamma_x<double>(Phase, const double2 *, long long, double, double, const double2 *, int,
                                           const double2 *, int, int, cplx<double> *);

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
// Host FP64 residual entry a(x, xi) exp(2 pi i Phi_ell(x, xi)) for flat grid index p.
zd host_residual(const Phase &ph, int N, long long p, double e1, double e2, double k1, double k2) {
    const double x1 = (double)(p / N) / N, x2 = (double)(p % N) / N;
    XCoef c = phase_xcoef(ph, x1, x2);
    double g1, g2;
    phase_grad(ph, c, e1, e2, g1, g2);
    double cs, sn;
    residual_entry(ph, c, g1, g2, k1, k2, cs, sn);
    return zd(cs, sn);
}

// k distinct values in [0, n) from the splitmix64 stream `state`.
template <typename I>
static std::vector<I> sample_distinct(I n, int k, uint64_t &state) {
    std::vector<I> out;
    if ((long long)k >= (long long)n) {
        out.resize((size_t)n);
        for (I i = 0; i < n; ++i)
            out[(size_t)i] = i;
        return out;
    }
    std::map<I, I> swaps;  // sparse Fisher-Yates
    for (int i = 0; i < k; ++i) {
        state = splitmix64(state);
        const I j = (I)(i + (long long)(state % (uint64_t)(n - i)));
        auto get = [&](I v) {
            auto it = swaps.find(v);
            return it == swaps.end() ? v : it->second;
        };
        const I vi = get((I)i), vj = get(j);
        swaps[j] = vi;
        swaps[(I)i] = vj;
        out.push_back(vj);
    }
    std::sort(out.begin(), out.end());
    return out;
}

template std::vector<int> sample_distinct<int>(int, int, uint64_t &);
template std::vector<long long> sample_distinct<long long>(long long, int, uint64_t &);

std::vector<int> sample_members(int n, int k, uint64_t &state) { return sample_distinct<int>(n, k, state); }
std::vector<long long> sample_points(long long n, int k, uint64_t &state) {
    return sample_distinct<long long>(n, k, state);
}

// Gram matrix A_C^H A_C (r x r, full Hermitian) of the residual kernel columns
// at frequencies `cols` over every grid point, reduced on the GPU in FP64.
// d_xcoef (N^2) is filled with the phase's per-point coefficients when fill_xcoef.
fio_status gram_of_columns(const Phase &ph, int N, double2 *d_xcoef, double theta, const std::vector<double2> &cols,
                           DeviceScratch &scr, std::vector<zd> &G, bool fill_xcoef) {
    const long long NN = (long long)N * N;
    const int rc = (int)cols.size();
    if (fill_xcoef) {
        k_xcoef<<<(unsigned)((NN + 255) / 256), 256>>>(ph, N, d_xcoef);
        FIO_HIP_TRY(hipGetLastError());
    }
    FIO_HIP_TRY(scr.ensure_cols(rc));
    FIO_HIP_TRY(hipMemcpy(scr.cols, cols.data(), rc * sizeof(double2), hipMemcpyHostToDevice));
    const int nt = (rc + kGramTile - 1) / kGramTile;
    const int nblk = (int)std::min<long long>(256, (NN + 4095) / 4096);
    const long long rpb = (NN + nblk - 1) / nblk;
    FIO_HIP_TRY(scr.ensure_partial((size_t)nblk * rc * rc, (size_t)rc * rc));
    k_gram<<<dim3(nblk, nt, nt), 256>>>(ph, d_xcoef, NN, std::cos(theta), std::sin(theta), scr.cols, rc, rpb,
                                        scr.partial);
    FIO_HIP_TRY(hipGetLastError());
    k_gram_reduce<<<(rc * rc + 255) / 256, 256>>>(scr.partial, nblk, rc, scr.gram);
    FIO_HIP_TRY(hipGetLastError());
    std::vector<double2> g((size_t)rc * rc);
    FIO_HIP_TRY(hipMemcpy(g.data(), scr.gram, (size_t)rc * rc * sizeof(double2), hipMemcpyDeviceToHost));
    G.assign((size_t)rc * rc, zd(0, 0));
    for (int i = 0; i < rc; ++i)
        for (int j = i; j < rc; ++j) {
            G[(size_t)i * rc + j] = zd(g[(size_t)i * rc + j].x, g[(size_t)i * rc + j].y);
            G[(size_t)j * rc + i] = std::conj(G[(size_t)i * rc + j]);
        }
    return FIO_OK;
}

// s x s estimate of the relative separation error (Section 4): U at rows Gam
// from `ugam(i, t)`, T at columns Del as P A_[R, Del], A exactly on the host.
static double separation_estimate(const fio_plan_s *P, const WedgeHost &W, const std::vector<long long> &Gam,
                                  const std::vector<int> &Del, const std::vector<zd> &UG) {
    const int N = P->N, h = N / 2, q = W.q;
    const int rr = (int)W.R.size(), sg = (int)Gam.size(), sd = (int)Del.size();
    const double e1 = std::cos(W.theta), e2 = std::sin(W.theta);
    std::vector<zd> TD((size_t)q * sd, zd(0, 0));
    for (int j = 0; j < sd; ++j) {
        const int om = W.members[Del[j]];
        const double k1 = om / N - h, k2 = om % N - h;
        for (int i = 0; i < rr; ++i) {
            const zd a = host_residual(P->phase, N, W.R[i], e1, e2, k1, k2);
            for (int t = 0; t < q; ++t)
                TD[(size_t)t * sd + j] += W.P[(size_t)t * rr + i] * a;
        }
    }
    double num = 0, den = 0;
    for (int i = 0; i < sg; ++i)
        for (int j = 0; j < sd; ++j) {
            const int om = W.members[Del[j]];
            const zd a = host_residual(P->phase, N, Gam[i], e1, e2, om / N - h, om % N - h);
            zd v(0, 0);
            for (int t = 0; t < q; ++t)
                v += UG[(size_t)i * q + t] * TD[(size_t)t * sd + j];
            num += std::norm(a - v);
            den += std::norm(a);
        }
    return std::sqrt(num / std::max(den, 1e-300));
}

// Randomized separation of one wedge (Section 3.2) with verification.
fio_status separate_wedge(fio_plan_s *P, int l, const double2 *d_xcoef, DeviceScratch &scr) {
    WedgeHost &W = P->wedges[l];
    const int N = P->N;
    const long long NN = (long long)N * N;
    const int nmem = (int)W.members.size();
    const double e1 = std::cos(W.theta), e2 = std::sin(W.theta);
    const int h = N / 2;
    double thr = P->tol * P->opt.sep_tol_frac;
    const double target = 0.5 * P->tol;
    int r = std::max(4, P->opt.r0);
    const int rmax = std::max(r, kMaxSamples);
    const int sv = std::max(8, P->opt.verify_samples);
    uint64_t state = splitmix64(P->opt.seed ^ (0x51ED2701ull * (uint64_t)(l + 1)));
    for (int attempt = 0; attempt < 10; ++attempt) {
        W.attempts = attempt + 1;
        const int rc = std::min(r, nmem);
        W.C = sample_distinct<int>(nmem, rc, state);
        std::vector<double2> cols(rc);
        for (int c = 0; c < rc; ++c) {
            const int om = W.members[W.C[c]];
            cols[c] = make_double2(om / N - h, om % N - h);
        }
        // --- Gram of A_[C] on the GPU (FP64), eigen-decomposition on the host
        std::vector<zd> G;
        fio_status gs = gram_of_columns(P->phase, N, const_cast<double2 *>(d_xcoef), W.theta, cols, scr, G, false);
        if (gs != FIO_OK)
            return gs;
        std::vector<double> lam;
        std::vector<zd> V;
        eigh(rc, G, lam, V);
        const double s1 = std::sqrt(std::max(lam[0], 0.0));
        int q = 0;
        while (q < rc && std::sqrt(std::max(lam[q], 0.0)) > thr * s1)
            ++q;
        q = std::max(q, 1);
        if (3 * q > rc && rc < nmem && r < rmax) {
            r = std::min(2 * r, rmax);
            continue;
        }
        // Z = V_q S_q^-1
        W.Z.assign((size_t)rc * q, zd(0, 0));
        for (int c = 0; c < rc; ++c)
            for (int t = 0; t < q; ++t)
                W.Z[(size_t)c * q + t] = V[(size_t)c * rc + t] / std::sqrt(lam[t]);
        // rows R, U_R = A_RC Z, P = pinv(U_R)
        const int rr = (int)std::min<long long>(std::max(rc, 2 * q), NN);
        W.R = sample_distinct<long long>(NN, rr, state);
        std::vector<zd> UR((size_t)rr * q, zd(0, 0));
        for (int i = 0; i < rr; ++i)
            for (int c = 0; c < rc; ++c) {
                const zd a = host_residual(P->phase, N, W.R[i], e1, e2, cols[c].x, cols[c].y);
                for (int t = 0; t < q; ++t)
                    UR[(size_t)i * q + t] += a * W.Z[(size_t)c * q + t];
            }
        pinv_tall(rr, q, UR, W.P, 1e-7);
        W.q = q;
        W.r = rc;
        // --- s x s estimate (Section 4)
        const int sg = (int)std::min<long long>(sv, NN), sd = std::min(sv, nmem);
        std::vector<long long> Gam = sample_distinct<long long>(NN, sg, state);
        std::vector<int> Del = sample_distinct<int>(nmem, sd, state);
        std::vector<zd> UG((size_t)sg * q, zd(0, 0));
        for (int i = 0; i < sg; ++i)
            for (int c = 0; c < rc; ++c) {
                const zd a = host_residual(P->phase, N, Gam[i], e1, e2, cols[c].x, cols[c].y);
                for (int t = 0; t < q; ++t)
                    UG[(size_t)i * q + t] += a * W.Z[(size_t)c * q + t];
            }
        W.sep_err = separation_estimate(P, W, Gam, Del, UG);
        if (W.sep_err <= target || attempt == 9)
            return FIO_OK;
        // the estimate missed the target: tighten the threshold and, while
        // columns remain unsampled, sample more of them
        thr *= 0.5;
        if (rc < nmem && r < rmax)
            r = std::min(2 * r, rmax);
    }
    return FIO_OK;
}

hipError_t DeviceScratch::ensure_cols(int n) {
    if (n <= ncols)
        return hipSuccess;
    if (cols)
        (void)hipFree(cols);
    ncols = n;
    return hipMalloc(&cols, (size_t)n * sizeof(double2));
}
hipError_t DeviceScratch::ensure_partial(size_t npart, size_t ngram) {
    if (npart > npartial) {
        if (partial)
            (void)hipFree(partial);
        npartial = npart;
        hipError_t e = hipMalloc(&partial, npart * sizeof(double2));
        if (e != hipSuccess)
            return e;
    }
    if (ngram > ngram_) {
        if (gram)
            (void)hipFree(gram);
        ngram_ = ngram;
        return hipMalloc(&gram, ngram * sizeof(double2));
    }
    return hipSuccess;
}
DeviceScratch::~DeviceScratch() {
    if (cols)
        (void)hipFree(cols);
    if (partial)
        (void)hipFree(partial);
    if (gram)
        (void)hipFree(gram);
}

// ---------------------------------------------------------------------------
// Device storage of factors, tables and workspace
// ---------------------------------------------------------------------------
// Factor folded into gamma^xi of every member: the kernel's deconvolution
// 1 / phi_hat along both axes of the sheared box, and 1/N.
std::vector<double> member_scale(int N, const WedgeHost &W) {
    const int h = N / 2;
    std::vector<double> scale(W.members.size());
    for (size_t m = 0; m < W.members.size(); ++m) {
        const int om = W.members[m];
        const int k1 = om / N - h, k2 = om % N - h;
        const int a1 = W.M[0] * k1 + W.M[1] * k2 - W.xc[0], a2 = W.M[2] * k1 + W.M[3] * k2 - W.xc[1];
        scale[m] = W.dec1[a1 - W.lo[0]] * W.dec2[a2 - W.lo[1]] / N;
    }
    return scale;
}

// gamma^xi = scale * (P A_[R]) for every member (and gamma^x = A_[C] Z for
// every grid point when exact_x), evaluated in FP64 and stored as T.
template <typename T>
static fio_status store_factors(fio_plan_s *P, const double2 *d_xcoef, bool exact_x) {
    const int N = P->N;
    const long long NN = (long long)N * N;
    const int h = N / 2;
    double2 *d_cols = nullptr, *d_mat = nullptr;
    double4 *d_rows = nullptr;
    double *d_scale = nullptr;
    struct Guard {
        std::vector<void *> p;
        ~Guard() {
            for (void *v : p)
                if (v)
                    (void)hipFree(v);
        }
    } guard;
    size_t maxr = 1, maxm = 1, maxz = 1;
    for (const WedgeHost &W : P->wedges) {
        maxr = std::max(maxr, std::max(W.C.size(), W.R.size()));
        maxm = std::max(maxm, W.members.size());
        maxz = std::max(maxz, std::max(W.Z.size(), W.P.size()));
    }
    FIO_HIP_TRY(hipMalloc(&d_cols, maxr * sizeof(double2)));
    guard.p.push_back(d_cols);
    FIO_HIP_TRY(hipMalloc(&d_rows, maxr * sizeof(double4)));
    guard.p.push_back(d_rows);
    FIO_HIP_TRY(hipMalloc(&d_mat, maxz * sizeof(double2)));
    guard.p.push_back(d_mat);
    FIO_HIP_TRY(hipMalloc(&d_scale, maxm * sizeof(double)));
    guard.p.push_back(d_scale);
    cplx<T> *gx = static_cast<cplx<T> *>(P->d_gx);
    cplx<T> *gxi = static_cast<cplx<T> *>(P->d_gxi);
    for (int l = 0; l < P->L; ++l) {
        WedgeHost &W = P->wedges[l];
        const WedgeDev &D = P->wdev[l];
        if (W.q == 0)
            continue;
        const double e1 = std::cos(W.theta), e2 = std::sin(W.theta);
        const int rc = (int)W.C.size(), rr = (int)W.R.size();
        if (exact_x && P->regen) {
            // the compressed factors: column frequencies and Z zero-padded to qpad ranks
            std::vector<double2> cols(rc), zp((size_t)rc * W.qpad, make_double2(0, 0));
            for (int c = 0; c < rc; ++c) {
                const int om = W.members[W.C[c]];
                cols[c] = make_double2(om / N - h, om % N - h);
                for (int t = 0; t < W.q; ++t)
                    zp[(size_t)c * W.qpad + t] = make_double2(W.Z[(size_t)c * W.q + t].real(), W.Z[(size_t)c * W.q + t].imag());
            }
            FIO_HIP_TRY(hipMemcpy(static_cast<double2 *>(P->d_zcol) + D.zc_off, cols.data(), rc * sizeof(double2),
                                  hipMemcpyHostToDevice));
            FIO_HIP_TRY(hipMemcpy(static_cast<double2 *>(P->d_zmat) + D.zm_off, zp.data(), zp.size() * sizeof(double2),
                                  hipMemcpyHostToDevice));
            std::vector<float2> zf(zp.size());
            for (size_t i = 0; i < zp.size(); ++i)
                zf[i] = make_float2((float)zp[i].x, (float)zp[i].y);
            FIO_HIP_TRY(hipMemcpy(static_cast<float2 *>(P->d_zmat32) + D.zm_off, zf.data(), zf.size() * sizeof(float2),
                                  hipMemcpyHostToDevice));
        } else if (exact_x) {
            std::vector<double2> cols(rc);
            for (int c = 0; c < rc; ++c) {
                const int om = W.members[W.C[c]];
                cols[c] = make_double2(om / N - h, om % N - h);
            }
            FIO_HIP_TRY(hipMemcpy(d_cols, cols.data(), rc * sizeof(double2), hipMemcpyHostToDevice));
            FIO_HIP_TRY(hipMemcpy(d_mat, W.Z.data(), W.Z.size() * sizeof(double2), hipMemcpyHostToDevice));
            k_gamma_x<T><<<(unsigned)((NN + 255) / 256), 256>>>(P->phase, d_xcoef, NN, e1, e2, d_cols, rc, d_mat, W.q,
                                                                W.qpad, gx + D.gx_off);
            FIO_HIP_TRY(hipGetLastError());
        }
        // gamma^xi with deconvolution and 1/N
        std::vector<double4> rows(rr);
        for (int i = 0; i < rr; ++i) {
            const long long p = W.R[i];
            const double x1 = (double)(p / N) / N, x2 = (double)(p % N) / N;
            XCoef c = phase_xcoef(P->phase, x1, x2);
            double g1, g2;
            phase_grad(P->phase, c, e1, e2, g1, g2);
            rows[i] = make_double4(c.a, c.b, g1, g2);
        }
        const std::vector<double> scale = member_scale(N, W);
        FIO_HIP_TRY(hipMemcpy(d_rows, rows.data(), rr * sizeof(double4), hipMemcpyHostToDevice));
        FIO_HIP_TRY(hipMemcpy(d_mat, W.P.data(), W.P.size() * sizeof(double2), hipMemcpyHostToDevice));
        FIO_HIP_TRY(hipMemcpy(d_scale, scale.data(), scale.size() * sizeof(double), hipMemcpyHostToDevice));
        const int nmem = (int)W.members.size();
        k_gamma_xi<T><<<(nmem + 255) / 256, 256>>>(P->phase, N, P->d_omega + D.mem_off, d_scale, nmem, d_rows, rr,
                                                   d_mat, W.q, W.qpad, gxi + D.gxi_off);
        FIO_HIP_TRY(hipGetLastError());
        FIO_HIP_TRY(hipDeviceSynchronize());
    }
    return FIO_OK;
}

// Default number of equiangular wedges.  Section 1.3 takes L ~ sqrt(N) with
// a free constant.  The residual phase of a wedge grows like
// S |xi| (theta - theta_ell)^2 / 2, with S = max |grad_xi h| the phase's
// strength, so its peak S (N / sqrt 2) (pi / L)^2 / 2 is held at 0.75 or
// below (the c1/c2 family at scale 1 stays on 8 ceil(sqrt(N) / 8)); L is
// never below 8 ceil(sqrt(N) / 8) and is rounded up to a multiple of 8.
int default_wedge_count(int N, const Phase &ph) {
    const double a0 = std::fabs(ph.p[0]);
    double S = 0;
    switch (ph.kind) {
    case 1: S = a0; break;
    case 2: S = a0 * 3.0 / 16.0; break;
    case 3: S = a0 * (1.0 + std::fabs(ph.p[1])); break;
    case 4:
    case 5: S = a0; break;
    default: S = 0; break;
    }
    const int base = 8 * (int)std::ceil(std::sqrt((double)N) / 8.0);
    const double Ls = kTwoPi / 2 * std::sqrt(S * N / (std::sqrt(2.0) * 1.5));
    return std::max(base, 8 * (int)std::ceil(Ls / 8.0));
}

// Partition, NUFFT kernel, shears, boxes, grids and FFT plans.
static fio_status plan_geometry(fio_plan_s *P) {
    const int N = P->N;
    const long long NN = (long long)N * N;
    std::vector<double> thetas;
    if (P->opt.partition == FIO_PART_CORONAE) {
        partition_coronae(N, P->wedge_of, thetas);
    } else {
        int L = P->opt.n_wedges;
        // a learned network fixes the partition it was trained on
        const LearnedModel *net = static_cast<const LearnedModel *>(P->opt.learned);
        if (L <= 0)
            L = net && net->N == N ? net->L : default_wedge_count(N, P->phase);
        partition_equiangular(N, L, P->wedge_of, thetas);
    }
    P->L = (int)thetas.size();
    P->wedges.assign(P->L, WedgeHost());
    for (int l = 0; l < P->L; ++l)
        P->wedges[l].theta = thetas[l];
    for (long long i = 0; i < NN; ++i)
        P->wedges[P->wedge_of[i]].members.push_back((int)i);
    P->sigma = P->opt.sigma > 0 ? P->opt.sigma : 2.0;
    es_parameters(P->tol * P->opt.nufft_tol_frac, P->sigma, P->opt.kernel_width, P->w, P->beta);
    std::map<int, int> fft_index;
    auto fft_for = [&](int n) -> int {
        auto it = fft_index.find(n);
        if (it != fft_index.end())
            return it->second;
        FftPlan pl;
        fft_make_plan(n, pl);
        const int id = (int)P->fftplans.size();
        P->fftplans.push_back(pl);
        P->fft_len.push_back(n);
        P->tw_off.push_back((int)P->tw_total);
        P->tw_total += n;
        fft_index[n] = id;
        return id;
    };
    for (WedgeHost &W : P->wedges) {
        if (W.members.empty())
            continue;
        wedge_geometry(N, P->sigma, P->w, W);
        for (int d = 0; d < 2; ++d) {
            W.n[d] = fft_nice_size(std::max((int)std::ceil(P->sigma * W.B[d]), 2 * P->w));
            W.fft[d] = fft_for(W.n[d]);
        }
        W.dec1.resize(W.B[0]);
        W.dec2.resize(W.B[1]);
        for (int i = 0; i < W.B[0]; ++i)
            W.dec1[i] = 1.0 / es_fourier(P->w, P->beta, (double)(W.lo[0] + i) / W.n[0]);
        for (int i = 0; i < W.B[1]; ++i)
            W.dec2[i] = 1.0 / es_fourier(P->w, P->beta, (double)(W.lo[1] + i) / W.n[1]);
    }
    return FIO_OK;
}

void release_layout(fio_plan_s *P) {
    void **bufs[] = {(void **)&P->d_wedges, (void **)&P->d_fftplans, (void **)&P->d_rows, (void **)&P->d_cols,
                     (void **)&P->d_map,    (void **)&P->d_omega,    &P->d_gxi,             &P->d_gx,
                     &P->d_tw,              &P->d_H,                 &P->d_G,               &P->d_zcol,
                     &P->d_zmat,            &P->d_zmat32,            (void **)&P->d_adj_bins, (void **)&P->d_adj_pts,
                     (void **)&P->d_adj_ref, (void **)&P->d_win};
    for (void **b : bufs) {
        if (*b)
            (void)hipFree(*b);
        *b = nullptr;
    }
    P->rows.clear();
    P->cols.clear();
    P->wdev.clear();
    P->n_adj_bins = 0;
    P->n_adj_pts = 0;
    P->adjoint_ready = false;
}

// Offsets, work items, device tables, factor storage and workspace for the
// ranks currently in P->wedges[*].q.
fio_status plan_layout(fio_plan_s *P) {
    const int N = P->N;
    const long long NN = (long long)N * N;
    const int h = N / 2;
    P->esize = P->precision == FIO_F64 ? 16 : 8;
    // complex elements of the in-place FFT buffers of the row and column stages
    const long long cap = kRowLdsBytes / (long long)P->esize, capc = kColLdsBytes / (long long)P->esize;
    P->qmax = 0;
    P->wdev.assign(P->L, WedgeDev());
    P->rows.clear();
    P->cols.clear();
    long long map_off = 0, mem_off = 0, gxi_off = 0, gx_off = 0, H_off = 0, G_off = 0, zc_off = 0, zm_off = 0;
    P->row_first.assign(P->L + 1, 0);
    P->col_first.assign(P->L + 1, 0);
    size_t lds_rows = 0, lds_cols = 0;
    for (int l = 0; l < P->L; ++l) {
        WedgeHost &W = P->wedges[l];
        WedgeDev &D = P->wdev[l];
        std::memset(&D, 0, sizeof(D));
        D.e1 = std::cos(W.theta);
        D.e2 = std::sin(W.theta);
        P->row_first[l] = (int)P->rows.size();
        P->col_first[l] = (int)P->cols.size();
        if (W.members.empty() || W.q == 0)
            continue;
        W.qpad = W.q + (W.q & 1);
        P->qmax = std::max(P->qmax, W.qpad);
        // y' = M^{-T} y ; psi = y . M^{-1} xi_c
        D.mt[0] = W.Minv[0];
        D.mt[1] = W.Minv[2];
        D.mt[2] = W.Minv[1];
        D.mt[3] = W.Minv[3];
        D.cvec[0] = W.Minv[0] * W.xc[0] + W.Minv[1] * W.xc[1];
        D.cvec[1] = W.Minv[2] * W.xc[0] + W.Minv[3] * W.xc[1];
        D.n1 = W.n[0];
        D.n2 = W.n[1];
        D.B1 = W.B[0];
        D.B2 = W.B[1];
        D.lo1 = W.lo[0];
        D.lo2 = W.lo[1];
        D.q = W.qpad;
        D.fq = FastDiv((unsigned)std::max(1, W.qpad));
        D.fB1 = FastDiv((unsigned)W.B[0]);
        D.fB2 = FastDiv((unsigned)W.B[1]);
        D.fn1 = FastDiv((unsigned)W.n[0]);
        D.fn2 = FastDiv((unsigned)W.n[1]);
        D.nmem = (int)W.members.size();
        D.fft1 = W.fft[0];
        D.fft2 = W.fft[1];
        D.tw1 = P->tw_off[D.fft1];
        D.tw2 = P->tw_off[D.fft2];
        if (W.n[0] > capc || W.n[1] > cap)
            return (set_error("oversampled grid too long for the LDS transform"), FIO_ENOTSUP);
        D.map_off = map_off;
        map_off += (long long)W.B[0] * W.B[1];
        D.mem_off = mem_off;
        mem_off += W.members.size();
        D.gxi_off = gxi_off;
        gxi_off += (long long)W.members.size() * W.qpad;
        D.gx_off = gx_off;
        D.zc_off = zc_off;
        D.zm_off = zm_off;
        D.zrc = 0;
        if (P->regen) {
            D.zrc = (int)W.C.size();
            zc_off += W.C.size();
            zm_off += (long long)W.C.size() * W.qpad;
        } else {
            gx_off += NN * W.qpad;
        }
        D.H_off = H_off;
        H_off += (long long)W.B[0] * W.n[1] * W.qpad;
        D.G_off = G_off;
        G_off += (long long)W.n[0] * W.n[1] * W.qpad;
        // H is plane-major: plane P = j2 * qu + t / cpu holds ranks
        // [cpu (t / cpu), cpu (t / cpu + 1)) of grid column j2, element
        // [(P * B1 + k1) * cpu + t % cpu] (cpu = complex per 16 bytes); G is
        // plane-major as well, [((P * n2 + j2) * n1 + j1) * cpu + t % cpu].
        const int cpu = (int)(16 / P->esize), qu = W.qpad / cpu;
        // stage-1 items: nr adjacent box rows and tn ranks (whole planes),
        // aiming at 8 or more rows so each (column, plane) leaves as a run of
        // at least 128 bytes
        int tn = cpu * (int)std::max<long long>(1, std::min<long long>(qu, cap / ((long long)W.n[1] * 8 * cpu)));
        if ((long long)W.n[1] * tn > cap)
            tn = (int)std::max<long long>(1, cap / W.n[1]);  // sub-plane chunks (very long rows)
        const int nr = (int)std::max<long long>(1, std::min<long long>(W.B[0], cap / ((long long)W.n[1] * tn)));
        for (int k1 = 0; k1 < W.B[0]; k1 += nr)
            for (int t0 = 0; t0 < W.qpad; t0 += tn)
                P->rows.push_back(make_row_item(l, k1, std::min(nr, W.B[0] - k1), t0, std::min(tn, W.qpad - t0), cpu));
        lds_rows = std::max(lds_rows, (size_t)W.n[1] * (nr * tn + 1) * P->esize);  // buffer + twiddles
        // stage-2 items: whole planes (one contiguous block of H per item), or
        // single ranks when one plane does not fit the buffer
        const long long plsz = (long long)W.n[0] * cpu;
        if (plsz <= capc) {
            const long long npl = (long long)W.n[1] * qu;
            const int np = (int)std::min<long long>(npl, capc / plsz);
            for (long long p0 = 0; p0 < npl; p0 += np)
                P->cols.push_back(make_col_item(l, (int)(p0 * cpu), (int)(std::min<long long>(np, npl - p0) * cpu)));
            lds_cols = std::max(lds_cols, (size_t)(plsz * np + W.n[0]) * P->esize);  // buffer + twiddles
        } else {
            for (long long t0 = 0; t0 < (long long)W.n[1] * W.qpad; ++t0)
                P->cols.push_back(make_col_item(l, (int)t0, 1));
            lds_cols = std::max(lds_cols, (size_t)W.n[0] * 2 * P->esize);  // buffer + twiddles
        }
    }
    P->row_first[P->L] = (int)P->rows.size();
    P->col_first[P->L] = (int)P->cols.size();
    P->lds_rows = lds_rows;
    P->lds_cols = lds_cols;
    P->map_total = map_off;
    P->mem_total = mem_off;
    P->gxi_total = gxi_off;
    P->gx_total = gx_off;
    P->H_total = H_off;
    P->G_total = G_off;
    if (P->qmax == 0)
        return (set_error("no wedge has a nonzero rank"), FIO_EINVAL);
    std::vector<int> map(std::max<long long>(1, map_off), -1), omega(std::max<long long>(1, mem_off));
    for (int l = 0; l < P->L; ++l) {
        WedgeHost &W = P->wedges[l];
        const WedgeDev &D = P->wdev[l];
        if (W.members.empty() || W.q == 0)
            continue;
        for (size_t m = 0; m < W.members.size(); ++m) {
            const int om = W.members[m];
            const int k1 = om / N - h, k2 = om % N - h;
            const int a1 = W.M[0] * k1 + W.M[1] * k2 - W.xc[0] - W.lo[0];
            const int a2 = W.M[2] * k1 + W.M[3] * k2 - W.xc[1] - W.lo[1];
            map[D.map_off + (long long)a1 * W.B[1] + a2] = (int)m;
            omega[D.mem_off + m] = om;
        }
    }
    const size_t es = P->esize;
    FIO_HIP_TRY(hipMalloc(&P->d_wedges, sizeof(WedgeDev) * P->L));
    FIO_HIP_TRY(hipMemcpy(P->d_wedges, P->wdev.data(), sizeof(WedgeDev) * P->L, hipMemcpyHostToDevice));
    FIO_HIP_TRY(hipMalloc(&P->d_fftplans, sizeof(FftPlan) * P->fftplans.size()));
    FIO_HIP_TRY(hipMemcpy(P->d_fftplans, P->fftplans.data(), sizeof(FftPlan) * P->fftplans.size(),
                          hipMemcpyHostToDevice));
    FIO_HIP_TRY(hipMalloc(&P->d_rows, sizeof(RowItem) * std::max<size_t>(1, P->rows.size())));
    FIO_HIP_TRY(hipMemcpy(P->d_rows, P->rows.data(), sizeof(RowItem) * P->rows.size(), hipMemcpyHostToDevice));
    FIO_HIP_TRY(hipMalloc(&P->d_cols, sizeof(ColItem) * std::max<size_t>(1, P->cols.size())));
    FIO_HIP_TRY(hipMemcpy(P->d_cols, P->cols.data(), sizeof(ColItem) * P->cols.size(), hipMemcpyHostToDevice));
    FIO_HIP_TRY(hipMalloc(&P->d_map, sizeof(int) * map.size()));
    FIO_HIP_TRY(hipMemcpy(P->d_map, map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice));
    FIO_HIP_TRY(hipMalloc(&P->d_omega, sizeof(int) * omega.size()));
    FIO_HIP_TRY(hipMemcpy(P->d_omega, omega.data(), sizeof(int) * omega.size(), hipMemcpyHostToDevice));
    // twiddles exp(+2 pi i m / n) in FP64, stored in the plan precision
    {
        std::vector<double> tw(2 * P->tw_total);
        for (size_t f = 0; f < P->fftplans.size(); ++f) {
            const int n = P->fft_len[f];
            for (int m = 0; m < n; ++m) {
                tw[2 * (P->tw_off[f] + m)] = std::cos(kTwoPi * m / n);
                tw[2 * (P->tw_off[f] + m) + 1] = std::sin(kTwoPi * m / n);
            }
        }
        FIO_HIP_TRY(hipMalloc(&P->d_tw, es * P->tw_total));
        if (P->precision == FIO_F64) {
            FIO_HIP_TRY(hipMemcpy(P->d_tw, tw.data(), es * P->tw_total, hipMemcpyHostToDevice));
        } else {
            std::vector<float> twf(tw.begin(), tw.end());
            FIO_HIP_TRY(hipMemcpy(P->d_tw, twf.data(), es * P->tw_total, hipMemcpyHostToDevice));
        }
    }
    FIO_HIP_TRY(hipMalloc(&P->d_gxi, es * std::max<long long>(1, gxi_off)));
    FIO_HIP_TRY(hipMalloc(&P->d_gx, es * std::max<long long>(1, gx_off)));
    P->factor_bytes = (long long)es * (gxi_off + gx_off);
    if (P->regen) {
        FIO_HIP_TRY(hipMalloc(&P->d_zcol, sizeof(double2) * std::max<long long>(1, zc_off)));
        FIO_HIP_TRY(hipMalloc(&P->d_zmat, sizeof(double2) * std::max<long long>(1, zm_off)));
        // padded: the regeneration reads kRegenMaxRank values of a column at once
        FIO_HIP_TRY(hipMalloc(&P->d_zmat32, sizeof(float2) * (zm_off + kRegenMaxRank)));
        FIO_HIP_TRY(hipMemset(P->d_zmat32, 0, sizeof(float2) * (zm_off + kRegenMaxRank)));
        P->factor_bytes += (long long)sizeof(double2) * (zc_off + zm_off);
    }
    // workspace: bchunk right-hand sides
    P->bchunk = std::max(1, P->opt.max_batch);
    const long long per_rhs = (long long)es * (H_off + G_off);
    const long long budget = 24LL << 30;
    while (P->bchunk > 1 && per_rhs * P->bchunk > budget)
        P->bchunk /= 2;
    FIO_HIP_TRY(hipMalloc(&P->d_H, es * std::max<long long>(1, H_off) * P->bchunk));
    FIO_HIP_TRY(hipMalloc(&P->d_G, es * std::max<long long>(1, G_off) * P->bchunk));
    P->workspace_bytes = per_rhs * P->bchunk;
    return FIO_OK;
}

// FIO_FACTORS_REGEN regenerates gamma^x(x) = A(x, C) Z with a sum over all r
// sampled columns.  A column interpolative decomposition of A(R, C) on the
// sampled rows keeps k of them, A(:, C) ~ A(:, C') [I T] P^T, so that
// gamma^x = A(x, C') Z' with Z' = [I T] P^T Z: k (near the rank) columns per
// point instead of r.  Errors in A(:, C) reach the operator through Z, which
// scales the weakest directions up, so the decomposition is cut far below
// the separation threshold; the s x s estimate then decides whether the
// wedge keeps it.
static void regen_column_id(fio_plan_s *P, int l) {
    WedgeHost &W = P->wedges[l];
    const int N = P->N, h = N / 2, rc = (int)W.C.size(), rr = (int)W.R.size(), q = W.q;
    if (q == 0 || rc <= q + 2)
        return;
    const double e1 = std::cos(W.theta), e2 = std::sin(W.theta);
    auto col = [&](int c, double &k1, double &k2) {
        const int om = W.members[W.C[c]];
        k1 = om / N - h;
        k2 = om % N - h;
    };
    std::vector<zd> M((size_t)rr * rc);
    for (int i = 0; i < rr; ++i)
        for (int c = 0; c < rc; ++c) {
            double k1, k2;
            col(c, k1, k2);
            M[(size_t)i * rc + c] = host_residual(P->phase, N, W.R[i], e1, e2, k1, k2);
        }
    std::vector<int> perm;
    std::vector<zd> T;
    const double thr = P->tol * P->opt.sep_tol_frac;
    const int k = column_id(rr, rc, M, 1e-3 * thr, perm, T);
    if (k <= 0 || k >= rc)
        return;
    std::vector<zd> Z2((size_t)k * q);
    for (int j = 0; j < k; ++j)
        for (int t = 0; t < q; ++t) {
            zd s = W.Z[(size_t)perm[j] * q + t];
            for (int i = k; i < rc; ++i)
                s += T[(size_t)j * (rc - k) + (i - k)] * W.Z[(size_t)perm[i] * q + t];
            Z2[(size_t)j * q + t] = s;
        }
    // s x s estimate with the reduced columns
    uint64_t state = splitmix64(P->opt.seed ^ (0x1DC0ull * (uint64_t)(l + 1)));
    const long long NN = (long long)N * N;
    const int sv = std::max(8, P->opt.verify_samples), nmem = (int)W.members.size();
    const std::vector<long long> Gam = sample_distinct<long long>(NN, (int)std::min<long long>(sv, NN), state);
    const std::vector<int> Del = sample_distinct<int>(nmem, std::min(sv, nmem), state);
    std::vector<zd> UG(Gam.size() * (size_t)q, zd(0, 0));
    for (size_t i = 0; i < Gam.size(); ++i)
        for (int j = 0; j < k; ++j) {
            double k1, k2;
            col(perm[j], k1, k2);
            const zd a = host_residual(P->phase, N, Gam[i], e1, e2, k1, k2);
            for (int t = 0; t < q; ++t)
                UG[i * q + t] += a * Z2[(size_t)j * q + t];
        }
    const double err = separation_estimate(P, W, Gam, Del, UG);
    if (err > std::max(0.5 * P->tol, 1.2 * W.sep_err))
        return;
    std::vector<int> C2(k);
    for (int j = 0; j < k; ++j)
        C2[j] = W.C[perm[j]];
    W.C = C2;
    W.Z = Z2;
    W.sep_err = std::max(W.sep_err, err);
}

// Exact factors: randomized separation of every wedge, then storage.
static fio_status plan_exact(fio_plan_s *P, const double2 *d_xcoef) {
    {
        DeviceScratch scr;
        for (int l = 0; l < P->L; ++l) {
            if (P->wedges[l].members.empty())
                continue;
            fio_status st = separate_wedge(P, l, d_xcoef, scr);
            if (st != FIO_OK)
                return st;
            // the verification retries tighten the threshold; an estimate
            // still above the whole budget means the tolerance is out of reach
            if (P->wedges[l].sep_err > P->tol)
                return (set_error("wedge " + std::to_string(l) + ": separation error estimate " +
                                  std::to_string(P->wedges[l].sep_err) + " exceeds tol"),
                        FIO_EACCURACY);
        }
    }
    P->regen = P->opt.factor_mode == FIO_FACTORS_REGEN;
    if (P->regen)
        for (int l = 0; l < P->L; ++l)
            regen_column_id(P, l);
    if (P->regen) {
        int qmax = 0;
        for (const WedgeHost &W : P->wedges)
            qmax = std::max(qmax, W.q + (W.q & 1));
        if (qmax > kRegenMaxRank / (P->precision == FIO_F64 ? 2 : 1))
            return (set_error("FIO_FACTORS_REGEN needs a padded rank of at most " +
                              std::to_string(kRegenMaxRank / (P->precision == FIO_F64 ? 2 : 1)) + " (have " +
                              std::to_string(qmax) + ")"),
                    FIO_ENOTSUP);
    }
    fio_status st = plan_layout(P);
    if (st != FIO_OK)
        return st;
    P->factor_mode = P->regen ? FIO_FACTORS_REGEN : FIO_FACTORS_STORED;
    return P->precision == FIO_F64 ? store_factors<double>(P, d_xcoef, true) : store_factors<float>(P, d_xcoef, true);
}

// The network's 16 factors at sampled grid points, FP64 on the host
// ([i * 16 + t], row-major).
static fio_status infer_rows(fio_plan_s *P, LearnedModel *net, double theta, const std::vector<long long> &rows,
                             std::vector<zd> &out) {
    const int n = (int)rows.size();
    long long *d_x = nullptr;
    float *d_y = nullptr;
    FIO_HIP_TRY(hipMalloc(&d_x, sizeof(long long) * n));
    hipError_t e = hipMalloc(&d_y, sizeof(float) * (size_t)n * kNetOut);
    if (e == hipSuccess)
        e = hipMemcpy(d_x, rows.data(), sizeof(long long) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = learned_infer_points(net, theta, P->opt.learned_scale, d_x, n, d_y, 0);
    std::vector<float> h((size_t)n * kNetOut);
    if (e == hipSuccess)
        e = hipMemcpy(h.data(), d_y, sizeof(float) * h.size(), hipMemcpyDeviceToHost);
    (void)hipFree(d_x);
    if (d_y)
        (void)hipFree(d_y);
    if (e != hipSuccess)
        return hip_fail(e, "learned inference at sampled rows");
    out.resize((size_t)n * kNetRank);
    for (size_t i = 0; i < out.size(); ++i)
        out[i] = zd(h[2 * i], h[2 * i + 1]);
    return FIO_OK;
}

// Learned factors.  For each wedge the network gives alpha_t (t < 16) at the
// sampled rows R and at the rows Gamma of the s x s estimate (Section 4);
// gamma^xi is the least-squares refit alpha_[R]^+ A_[R] of the leading q
// factors, and q is the smallest rank whose estimate meets the separation
// target (the factors are ordered by the singular values of their targets,
// so the leading ones carry the most energy).  Only then are the q factors
// inferred on the whole grid and stored, at the plan's padded rank, so the
// apply runs at the rank the tolerance needs.  *ok is false if even the 16
// factors miss the target on some wedge.
static fio_status plan_learned(fio_plan_s *P, LearnedModel *net, const double2 *d_xcoef, bool *ok) {
    *ok = true;
    const int N = P->N, h = N / 2;
    const long long NN = (long long)N * N;
    P->factor_mode = FIO_FACTORS_LEARNED;
    const double target = 0.5 * P->tol;
    const int sv = std::max(8, P->opt.verify_samples);
    const int rr = std::max(4 * kNetRank, std::min(512, std::max(P->opt.r0, 8 * kNetRank)));
    for (int l = 0; l < P->L; ++l) {
        WedgeHost &W = P->wedges[l];
        W.q = 0;
        if (W.members.empty())
            continue;
        uint64_t state = splitmix64(P->opt.seed ^ (0x1EA2Dull * (uint64_t)(l + 1)));
        W.R = sample_distinct<long long>(NN, (int)std::min<long long>(rr, NN), state);
        W.C.clear();
        W.Z.clear();
        W.r = (int)W.R.size();
        const int nmem = (int)W.members.size(), nr = W.r;
        const int sg = (int)std::min<long long>(sv, NN), sd = std::min(sv, nmem);
        std::vector<long long> Gam = sample_distinct<long long>(NN, sg, state);
        std::vector<int> Del = sample_distinct<int>(nmem, sd, state);
        std::vector<zd> aR, aG;
        fio_status st = infer_rows(P, net, W.theta, W.R, aR);
        if (st == FIO_OK)
            st = infer_rows(P, net, W.theta, Gam, aG);
        if (st != FIO_OK)
            return st;
        // residual kernel at (R, Delta) and (Gamma, Delta), once for every trial rank
        const double e1 = std::cos(W.theta), e2 = std::sin(W.theta);
        std::vector<zd> ARD((size_t)nr * sd), AGD((size_t)sg * sd);
        double den = 0;
        for (int j = 0; j < sd; ++j) {
            const int om = W.members[Del[j]];
            const double k1 = om / N - h, k2 = om % N - h;
            for (int i = 0; i < nr; ++i)
                ARD[(size_t)i * sd + j] = host_residual(P->phase, N, W.R[i], e1, e2, k1, k2);
            for (int i = 0; i < sg; ++i) {
                AGD[(size_t)i * sd + j] = host_residual(P->phase, N, Gam[i], e1, e2, k1, k2);
                den += std::norm(AGD[(size_t)i * sd + j]);
            }
        }
        // estimate of the rank-q refit; Pq = alpha_[R](:, :q)^+
        auto estimate = [&](int q, std::vector<zd> &Pq) {
            std::vector<zd> U((size_t)nr * q);
            for (int i = 0; i < nr; ++i)
                for (int t = 0; t < q; ++t)
                    U[(size_t)i * q + t] = aR[(size_t)i * kNetRank + t];
            pinv_tall(nr, q, U, Pq, 1e-6);
            std::vector<zd> TD((size_t)q * sd, zd(0, 0));
            for (int t = 0; t < q; ++t)
                for (int i = 0; i < nr; ++i) {
                    const zd pv = Pq[(size_t)t * nr + i];
                    const zd *arow = &ARD[(size_t)i * sd];
                    zd *trow = &TD[(size_t)t * sd];
                    for (int j = 0; j < sd; ++j)
                        trow[j] += pv * arow[j];
                }
            double num = 0;
            for (int i = 0; i < sg; ++i)
                for (int j = 0; j < sd; ++j) {
                    zd v(0, 0);
                    for (int t = 0; t < q; ++t)
                        v += aG[(size_t)i * kNetRank + t] * TD[(size_t)t * sd + j];
                    num += std::norm(AGD[(size_t)i * sd + j] - v);
                }
            return std::sqrt(num / std::max(den, 1e-300));
        };
        std::vector<zd> Pq;
        double err = estimate(kNetRank, Pq);
        int q = kNetRank;
        if (err > target) {
            *ok = false;
        } else {
            // smallest rank meeting the target; the error falls with the rank
            int lo = 1, hi = kNetRank;
            while (lo < hi) {
                const int mid = (lo + hi) / 2;
                std::vector<zd> Pm;
                if (estimate(mid, Pm) <= target)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            q = lo;
            err = estimate(q, Pq);
        }
        W.q = q;
        W.P = Pq;
        W.sep_err = err;
        P->learned_sep_err = std::max(P->learned_sep_err, err);
    }
    if (!*ok)
        return FIO_OK;
    fio_status st = plan_layout(P);
    if (st != FIO_OK)
        return st;
    for (int l = 0; l < P->L; ++l) {
        WedgeHost &W = P->wedges[l];
        if (W.q == 0)
            continue;
        FIO_HIP_TRY(learned_infer_wedge(net, W.theta, P->opt.learned_scale,
                                        static_cast<cplx<float> *>(P->d_gx) + P->wdev[l].gx_off, W.q, W.qpad,
                                        P->precision, 0));
    }
    FIO_HIP_TRY(hipDeviceSynchronize());
    return store_factors<float>(P, d_xcoef, false);
}

// ---------------------------------------------------------------------------
// Plan files.  A plan is saved as its build inputs (N, phase, tol, options)
// and, per wedge, the compressed factors of its randomized separation: the
// sampled columns C and rows R, Z = V S^-1 and U_[R]^+ (eq. (probnewfac)),
// the rank and the error estimate.  Loading rebuilds the geometry (a
// deterministic function of N and the options), checks it against the file
// and evaluates gamma^x and gamma^xi on the device from the saved factors,
// exactly as a fresh build stores them, so a loaded plan applies bit for bit
// like the plan that was saved; only the sampling and the eigen-solves of
// the separation are skipped.  Little-endian binary with an FNV-1a checksum.
// ---------------------------------------------------------------------------
namespace {
constexpr char kPlanMagic[8] = {'F', 'I', 'O', 'P', 'L', 'A', 'N', '1'};
constexpr uint32_t kPlanVersion = 2;  // 2: the amplitude kind follows the phase kind

struct PlanWriter {
    FILE *f;
    uint64_t h = 1469598103934665603ull;
    bool ok = true;
    void raw(const void *p, size_t n) {
        if (!ok)
            return;
        ok = std::fwrite(p, 1, n, f) == n;
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i)
            h = (h ^ c[i]) * 1099511628211ull;
    }
    template <typename V>
    void put(V v) {
        raw(&v, sizeof v);
    }
    template <typename V>
    void vec(const std::vector<V> &v) {
        put<int64_t>((int64_t)v.size());
        if (!v.empty())
            raw(v.data(), v.size() * sizeof(V));
    }
};

struct PlanReader {
    FILE *f;
    uint64_t h = 1469598103934665603ull;
    bool ok = true;
    void raw(void *p, size_t n) {
        if (!ok)
            return;
        ok = std::fread(p, 1, n, f) == n;
        if (!ok)
            return;
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i)
            h = (h ^ c[i]) * 1099511628211ull;
    }
    template <typename V>
    V get() {
        V v{};
        raw(&v, sizeof v);
        return v;
    }
    // a vector of at most `limit` elements
    template <typename V>
    bool vec(std::vector<V> &v, int64_t limit) {
        const int64_t n = get<int64_t>();
        if (!ok || n < 0 || n > limit)
            return ok = false;
        v.resize((size_t)n);
        if (n)
            raw(v.data(), (size_t)n * sizeof(V));
        return ok;
    }
};

struct SavedWedge {
    int32_t members = 0, q = 0, qpad = 0, r = 0, attempts = 0;
    double sep_err = 0;
    std::vector<int32_t> C;
    std::vector<int64_t> R;
    std::vector<zd> Z, Pinv;
};
}  // namespace

fio_status save_plan(const fio_plan_s *P, const char *path) {
    if (P->factor_mode == FIO_FACTORS_LEARNED)
        return (set_error("a plan with learned factors is kept by saving its network (fio_learned_save)"),
                FIO_ENOTSUP);
    if (P->factor_mode == FIO_FACTORS_TAYLOR)
        return (set_error("plan files hold the randomized separation; Taylor factors are rebuilt"), FIO_ENOTSUP);
    FILE *f = std::fopen(path, "wb");
    if (!f)
        return (set_error(std::string("cannot open ") + path + " for writing"), FIO_EINVAL);
    PlanWriter w{f};
    w.raw(kPlanMagic, sizeof kPlanMagic);
    w.put<uint32_t>(kPlanVersion);
    w.put<int32_t>(P->N);
    w.put<int32_t>(P->phase.kind);
    w.put<int32_t>(P->phase.amp);
    for (double v : P->phase.p)
        w.put<double>(v);
    w.put<double>(P->tol);
    const fio_options &o = P->opt;
    w.put<int32_t>(o.precision);
    w.put<int32_t>(o.partition);
    w.put<int32_t>(o.n_wedges);
    w.put<int32_t>(P->factor_mode);
    w.put<int32_t>(o.max_batch);
    w.put<int32_t>(o.kernel_width);
    w.put<int32_t>(o.r0);
    w.put<int32_t>(o.verify_samples);
    w.put<uint64_t>(o.seed);
    w.put<double>(o.sep_tol_frac);
    w.put<double>(o.nufft_tol_frac);
    w.put<double>(o.sigma);
    w.put<int32_t>(P->L);
    w.put<int32_t>(P->w);
    for (const WedgeHost &W : P->wedges) {
        w.put<int32_t>((int32_t)W.members.size());
        w.put<int32_t>(W.q);
        w.put<int32_t>(W.qpad);
        w.put<int32_t>(W.r);
        w.put<int32_t>(W.attempts);
        w.put<double>(W.sep_err);
        w.vec(std::vector<int32_t>(W.C.begin(), W.C.end()));
        w.vec(std::vector<int64_t>(W.R.begin(), W.R.end()));
        w.vec(W.Z);
        w.vec(W.P);
    }
    const uint64_t sum = w.h;
    w.put<uint64_t>(sum);
    const bool closed = std::fclose(f) == 0;
    if (!w.ok || !closed)
        return (set_error(std::string("write error on ") + path), FIO_EINVAL);
    return FIO_OK;
}

fio_status load_plan(fio_plan_s *P, const char *path) {
    using clock = std::chrono::steady_clock;
    const auto t_start = clock::now();
    FILE *f = std::fopen(path, "rb");
    if (!f)
        return (set_error(std::string("cannot open ") + path), FIO_EINVAL);
    PlanReader r{f};
    char magic[8] = {};
    r.raw(magic, sizeof magic);
    const uint32_t version = r.get<uint32_t>();
    auto bad = [&](const std::string &why) {
        std::fclose(f);
        set_error(std::string(path) + ": " + why);
        return FIO_EINVAL;
    };
    if (!r.ok || std::memcmp(magic, kPlanMagic, sizeof magic) != 0)
        return bad("not a plan file");
    if (version != kPlanVersion)
        return bad("unsupported plan file version " + std::to_string(version));
    const int N = r.get<int32_t>();
    Phase ph{};
    ph.kind = r.get<int32_t>();
    ph.amp = r.get<int32_t>();
    if (ph.amp != 0 && ph.amp != 1)
        return bad("unknown amplitude kind");
    for (double &v : ph.p)
        v = r.get<double>();
    const double tol = r.get<double>();
    fio_options o;
    fio_default_options(&o);
    o.precision = r.get<int32_t>();
    o.partition = r.get<int32_t>();
    o.n_wedges = r.get<int32_t>();
    const int mode = r.get<int32_t>();
    o.max_batch = r.get<int32_t>();
    o.kernel_width = r.get<int32_t>();
    o.r0 = r.get<int32_t>();
    o.verify_samples = r.get<int32_t>();
    o.seed = r.get<uint64_t>();
    o.sep_tol_frac = r.get<double>();
    o.nufft_tol_frac = r.get<double>();
    o.sigma = r.get<double>();
    o.factor_mode = mode;
    const int L = r.get<int32_t>(), w = r.get<int32_t>();
    if (!r.ok)
        return bad("truncated header");
    if (N < 8 || (N & 1) || N > 4096 || ph.kind < 0 || ph.kind > 5 || !(tol >= 5e-7 && tol < 1) ||
        (o.precision != FIO_F32 && o.precision != FIO_F64) ||
        (o.partition != FIO_PART_EQUIANGULAR && o.partition != FIO_PART_CORONAE) ||
        (mode != FIO_FACTORS_STORED && mode != FIO_FACTORS_REGEN) || o.max_batch < 1 || o.kernel_width < 0 ||
        o.kernel_width > 16 || o.n_wedges < 0 || o.n_wedges > 4096 || o.sigma < 0 ||
        (o.sigma > 0 && o.sigma < 1.25) || !(o.nufft_tol_frac > 0 && o.nufft_tol_frac <= 1) || L < 1 ||
        L > (long long)N * N)
        return bad("header out of range");
    const int64_t NN = (int64_t)N * N;
    std::vector<SavedWedge> saved((size_t)L);
    for (SavedWedge &S : saved) {
        S.members = r.get<int32_t>();
        S.q = r.get<int32_t>();
        S.qpad = r.get<int32_t>();
        S.r = r.get<int32_t>();
        S.attempts = r.get<int32_t>();
        S.sep_err = r.get<double>();
        if (!r.ok || S.members < 0 || S.members > NN || S.q < 0 || S.q > S.members || S.qpad != S.q + (S.q & 1))
            return bad("wedge record out of range");
        r.vec(S.C, S.members);
        r.vec(S.R, NN);
        r.vec(S.Z, (int64_t)S.C.size() * S.q);
        r.vec(S.Pinv, (int64_t)S.q * (int64_t)S.R.size());
        if (!r.ok)
            return bad("truncated wedge record");
        if (S.Z.size() != S.C.size() * (size_t)S.q || S.Pinv.size() != (size_t)S.q * S.R.size())
            return bad("inconsistent factor sizes");
        for (int32_t c : S.C)
            if (c < 0 || c >= S.members)
                return bad("column sample out of range");
        for (int64_t x : S.R)
            if (x < 0 || x >= NN)
                return bad("row sample out of range");
    }
    const uint64_t expect = r.h;
    const uint64_t sum = r.get<uint64_t>();
    char extra;
    const bool at_end = std::fread(&extra, 1, 1, f) == 0;
    std::fclose(f);
    if (!r.ok || sum != expect || !at_end)
        return (set_error(std::string(path) + ": checksum mismatch or trailing bytes"), FIO_EINVAL);

    P->N = N;
    P->phase = ph;
    P->tol = tol;
    P->opt = o;
    P->precision = o.precision;
    FIO_HIP_TRY(hipGetDevice(&P->device));
    fio_status st = plan_geometry(P);
    if (st != FIO_OK)
        return st;
    if (P->L != L || P->w != w)
        return (set_error(std::string(path) + ": wedge count or kernel width differs from this library's geometry"),
                FIO_EINVAL);
    for (int l = 0; l < L; ++l) {
        WedgeHost &W = P->wedges[l];
        SavedWedge &S = saved[(size_t)l];
        if ((int)W.members.size() != S.members)
            return (set_error(std::string(path) + ": wedge " + std::to_string(l) +
                              " has another member count in this library's partition"),
                    FIO_EINVAL);
        W.q = S.q;
        W.qpad = S.qpad;
        W.r = S.r;
        W.attempts = S.attempts;
        W.sep_err = S.sep_err;
        W.C.assign(S.C.begin(), S.C.end());
        W.R.assign(S.R.begin(), S.R.end());
        W.Z = std::move(S.Z);
        W.P = std::move(S.Pinv);
    }
    P->regen = mode == FIO_FACTORS_REGEN;
    if (P->regen) {
        int qmax = 0;
        for (const WedgeHost &W : P->wedges)
            qmax = std::max(qmax, W.qpad);
        if (qmax > kRegenMaxRank / (P->precision == FIO_F64 ? 2 : 1))
            return (set_error("FIO_FACTORS_REGEN rank bound exceeded in the plan file"), FIO_ENOTSUP);
    }
    st = plan_layout(P);
    if (st != FIO_OK)
        return st;
    P->factor_mode = mode;
    double2 *d_xcoef = nullptr;
    FIO_HIP_TRY(hipMalloc(&d_xcoef, NN * sizeof(double2)));
    k_xcoef<<<(unsigned)((NN + 255) / 256), 256>>>(P->phase, N, d_xcoef);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        st = P->precision == FIO_F64 ? store_factors<double>(P, d_xcoef, true) : store_factors<float>(P, d_xcoef, true);
    } else {
        st = hip_fail(e, "k_xcoef");
    }
    (void)hipFree(d_xcoef);
    if (st != FIO_OK)
        return st;
    FIO_HIP_TRY(apply_prepare(P));
    FIO_HIP_TRY(hipDeviceSynchronize());
    P->plan_ms = std::chrono::duration<double, std::milli>(clock::now() - t_start).count();
    return FIO_OK;
}

fio_status build_plan(fio_plan_s *P) {
    using clock = std::chrono::steady_clock;
    const auto t_start = clock::now();
    const int N = P->N;
    const long long NN = (long long)N * N;
    FIO_HIP_TRY(hipGetDevice(&P->device));
    fio_status st = plan_geometry(P);
    if (st != FIO_OK)
        return st;
    double2 *d_xcoef = nullptr;
    FIO_HIP_TRY(hipMalloc(&d_xcoef, NN * sizeof(double2)));
    struct XGuard {
        double2 *p;
        ~XGuard() {
            if (p)
                (void)hipFree(p);
        }
    } xg{d_xcoef};
    k_xcoef<<<(unsigned)((NN + 255) / 256), 256>>>(P->phase, N, d_xcoef);
    FIO_HIP_TRY(hipGetLastError());
    LearnedModel *net = static_cast<LearnedModel *>(const_cast<void *>(P->opt.learned));
    const bool want_net =
        net && (P->opt.factor_mode == FIO_FACTORS_AUTO || P->opt.factor_mode == FIO_FACTORS_LEARNED);
    bool use_net = want_net;
    if (want_net && (net->N != N || net->L != P->L || P->opt.partition != FIO_PART_EQUIANGULAR ||
                     P->precision != FIO_F32 || net->family.kind != P->phase.kind || P->phase.amp != 0)) {
        if (P->opt.factor_mode == FIO_FACTORS_LEARNED)
            return (set_error("the network was trained for another N, wedge count, partition, precision, "
                              "phase family or amplitude"),
                    FIO_EINVAL);
        use_net = false;
    }
    if (use_net) {
        bool ok = false;
        const auto t_net = clock::now();
        st = plan_learned(P, net, d_xcoef, &ok);
        if (st != FIO_OK)
            return st;
        FIO_HIP_TRY(hipDeviceSynchronize());
        P->learned_ms = std::chrono::duration<double, std::milli>(clock::now() - t_net).count();
        if (!ok) {
            if (P->opt.factor_mode == FIO_FACTORS_LEARNED)
                return (set_error("learned factors miss the error budget"), FIO_EACCURACY);
            // fall back to the exact randomized separation
            release_layout(P);
            for (WedgeHost &W : P->wedges) {
                W.q = 0;
                W.P.clear();
                W.R.clear();
            }
            P->fallback = 1;
            use_net = false;
        }
    }
    if (!use_net) {
        st = P->opt.factor_mode == FIO_FACTORS_TAYLOR ? plan_taylor(P, d_xcoef) : plan_exact(P, d_xcoef);
        if (st != FIO_OK)
            return st;
    }
    FIO_HIP_TRY(apply_prepare(P));
    FIO_HIP_TRY(hipDeviceSynchronize());
    P->plan_ms = std::chrono::duration<double, std::milli>(clock::now() - t_start).count();
    return FIO_OK;
}

}  // namespace fio
