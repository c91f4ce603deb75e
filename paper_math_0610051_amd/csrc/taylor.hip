// Deterministic separated factors (Section 3.1), FIO_FACTORS_TAYLOR.
//
// For wedge ell with centre angle theta_ell, write xi = |xi| (cos theta,
// sin theta).  For a phase h of degree 1 in xi the residual phase is
// Phi_ell(x, xi) = |xi| phi_ell(x, theta) with
//   phi_ell(x, theta) = h(x, e(theta)) - grad_xi h(x, e(theta_ell)) . e(theta),
// which is analytic in theta and vanishes with its first derivative at
// theta_ell.  The construction, in the section's order:
//   1. the polar Taylor coefficients c_k(x) of phi_ell(x, theta_ell + t), from
//      the Cauchy integral over |t| = rho evaluated by the trapezoidal rule at
//      M points: c_k = (1/M) sum_m phi_ell(theta_ell + rho w^m) w^(-mk) / rho^k,
//      w = exp(2 pi i / M) (device kernel, FP64, complex theta); rho lies
//      between the wedge's half-width and the nearest complex singularity of
//      phi_ell, beyond which the series cannot converge;
//   2. exp(2 pi i Phi_ell) = prod_k exp(2 pi i c_k(x) |xi| t^k), each factor a
//      truncated exponential series
//        sum_{m < d_k} (2 pi i s_k c_k(x))^m / m! * (|xi| t^k / s_k)^m,
//      with s_k the largest |xi| |t|^k over the wedge and d_k the first m at
//      which the largest term drops below a tenth of the threshold; the
//      orders k run while a term can still exceed a hundredth of it;
//   3. the running product X Y (X: N^2 x q on the grid, Y: q x |W_ell| on the
//      wedge) is multiplied by factor k (a Khatri-Rao product of the columns
//      on each side) and compressed: QR of both sides through their Gram
//      matrices (rocBLAS zgemm), an SVD of the small core through the
//      eigen-decomposition of its Gram matrix (host), singular values below
//      the threshold (relative to the largest) dropped.
// The factors are then checked with the s x s estimate of Section 4 against
// the exact residual kernel; a miss tightens the threshold and repeats the
// wedge.  gamma^x = X and gamma^xi = Y (with the kernel's deconvolution and
// 1/N folded in) are stored as for the randomized factors.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "apply.hpp"
#include "errors.hpp"
#include "interp_util.hpp"
#include "linalg.hpp"
#include "plan_build.hpp"

namespace fio {

constexpr int kCauchyM = 96;          // trapezoidal points on the circle
constexpr int kTaylorK = 32;          // coefficients c_0 .. c_31
constexpr double kCauchyMaxRadius = 0.25;
constexpr int kTaylorMaxCols = 1024;  // columns of a product before compression

using cd = cplx<double>;

__host__ __device__ inline cd zsqrt(cd z) {
    // principal square root, without cancellation on either half-plane
    const double r = hypot(z.re, z.im);
    if (r == 0.0)
        return cmake(0.0, 0.0);
    if (z.re >= 0.0) {
        const double t = sqrt(0.5 * (r + z.re));
        return cmake(t, z.im / (2.0 * t));
    }
    const double t = sqrt(0.5 * (r - z.re));
    return cmake(fabs(z.im) / (2.0 * t), copysign(t, z.im));
}

// Distance from theta_ell to the nearest complex singularity of
// phi_ell(x, .) over the grid.  Only the elliptic families have one: h is
// p0 sqrt(a^2 cos^2 + b^2 sin^2), and a^2 cos^2 theta + b^2 sin^2 theta =
// (a^2 + b^2)/2 + (a^2 - b^2)/2 cos 2 theta vanishes at
// theta = pi/2 + i acosh(kappa)/2 (a > b) or theta = i acosh(kappa)/2
// (a < b), modulo pi, with kappa = (a^2 + b^2) / |a^2 - b^2|.
static double singularity_distance(const Phase &ph, const std::vector<double2> &xc, double theta) {
    if (ph.kind == 0 || phase_isotropic(ph.kind))
        return INFINITY;
    double best = INFINITY;
    for (const double2 &c : xc) {
        const double aa = c.x * c.x, bb = c.y * c.y;
        if (aa == bb)
            continue;
        const double im = 0.5 * std::acosh((aa + bb) / std::fabs(aa - bb));
        const double re0 = aa > bb ? 0.5 * M_PI : 0.0;
        double dre = std::remainder(theta - re0, M_PI);
        best = std::min(best, std::hypot(dre, im));
    }
    return best;
}

// c_k(x), k < kTaylorK, of every grid point; cmax[k] gathers max_x |c_k(x)|
// as the bit patterns of non-negative doubles (ordered like the values).
// E[m] = (cos, sin)(theta_ell + rho w^m) as (re, im, re, im);
// F[m * kTaylorK + k] = w^(-mk) / (M rho^k).
__global__ __launch_bounds__(256) void k_taylor_coef(Phase ph, const double2 *__restrict__ xcoef, long long NN,
                                                     double e1, double e2, const double4 *__restrict__ E,
                                                     const double2 *__restrict__ F, double *__restrict__ C,
                                                     unsigned long long *__restrict__ cmax) {
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = x < NN;
    double acc[kTaylorK];
#pragma unroll
    for (int k = 0; k < kTaylorK; ++k)
        acc[k] = 0.0;
    if (live) {
        const double2 xc = xcoef[x];
        const XCoef c{xc.x, xc.y};
        double g1, g2;
        phase_grad(ph, c, e1, e2, g1, g2);
        for (int m = 0; m < kCauchyM; ++m) {
            const double4 em = E[m];
            const cd c1 = cmake(em.x, em.y), c2 = cmake(em.z, em.w);
            cd hv;
            if (ph.kind == 0) {
                hv = cmake(ph.p[0] * c1.re + ph.p[1] * c2.re, ph.p[0] * c1.im + ph.p[1] * c2.im);
            } else if (phase_isotropic(ph.kind)) {
                const cd s = zsqrt(cadd(cmul(c1, c1), cmul(c2, c2)));
                hv = cmake(c.a * s.re, c.a * s.im);
            } else {
                const cd u = cmul(c1, c1), v = cmul(c2, c2);
                const double aa = c.a * c.a, bb = c.b * c.b;
                const cd s = zsqrt(cmake(aa * u.re + bb * v.re, aa * u.im + bb * v.im));
                hv = cmake(ph.p[0] * s.re, ph.p[0] * s.im);
            }
            const cd res = cmake(hv.re - (g1 * c1.re + g2 * c2.re), hv.im - (g1 * c1.im + g2 * c2.im));
            const double2 *fm = F + m * kTaylorK;
#pragma unroll
            for (int k = 0; k < kTaylorK; ++k)
                acc[k] += res.re * fm[k].x - res.im * fm[k].y;
        }
#pragma unroll
        for (int k = 0; k < kTaylorK; ++k)
            C[x * kTaylorK + k] = acc[k];
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < kTaylorK; ++k) {
        const double mx = wave_max(live ? fabs(acc[k]) : 0.0);
        if (lane == 0)
            atomicMax(cmax + k, (unsigned long long)__double_as_longlong(mx));
    }
}

// Xp[x, t d + m] = X[x, t] z(x)^m / m!, z(x) = i zs c_k(x) (row-major, r = q d).
__global__ void k_taylor_xp(const double2 *__restrict__ X, int q, const double *__restrict__ C, int k, double zs,
                            int d, long long NN, double2 *__restrict__ Xp) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NN * q)
        return;
    const long long x = i / q;
    const int t = (int)(i - x * q);
    const double zi = zs * C[x * kTaylorK + k];
    double2 v = X[i];
    double2 *out = Xp + x * (long long)q * d + (long long)t * d;
    out[0] = v;
    for (int m = 1; m < d; ++m) {
        // v * (i zi) / m
        const double re = -v.y * zi / m, im = v.x * zi / m;
        v = make_double2(re, im);
        out[m] = v;
    }
}

// Yp[t d + m, j] = Y[t, j] u_j^m (row-major, rows of length nmem).
__global__ void k_taylor_yp(const double2 *__restrict__ Y, int q, const double *__restrict__ u, int nmem, int d,
                            double2 *__restrict__ Yp) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)q * nmem)
        return;
    const int t = (int)(i / nmem), j = (int)(i - (long long)t * nmem);
    double2 v = Y[i];
    const double uj = u[j];
    for (int m = 0; m < d; ++m) {
        Yp[((long long)t * d + m) * nmem + j] = v;
        v = make_double2(v.x * uj, v.y * uj);
    }
}

template <typename T>
__global__ void k_taylor_store_x(const double2 *__restrict__ X, int q, int qpad, long long NN,
                                 cplx<T> *__restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NN * qpad)
        return;
    const long long x = i / qpad;
    const int t = (int)(i - x * qpad);
    const double2 v = t < q ? X[x * q + t] : make_double2(0.0, 0.0);
    out[i] = cmake<T>((T)v.x, (T)v.y);
}

template <typename T>
__global__ void k_taylor_store_xi(const double2 *__restrict__ Y, int q, int qpad, int nmem,
                                  const double *__restrict__ scale, cplx<T> *__restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)nmem * qpad)
        return;
    const int m = (int)(i / qpad), t = (int)(i - (long long)m * qpad);
    const double2 v = t < q ? Y[(long long)t * nmem + m] : make_double2(0.0, 0.0);
    const double s = scale[m];
    out[i] = cmake<T>((T)(s * v.x), (T)(s * v.y));
}

namespace {

const char *rocblas_name(rocblas_status s) { return rocblas_status_to_string(s); }

#define FIO_BLAS_TRY(expr)                                                                      \
    do {                                                                                        \
        const rocblas_status s_ = (expr);                                                       \
        if (s_ != rocblas_status_success)                                                       \
            return (set_error(std::string("rocBLAS: ") + rocblas_name(s_)), FIO_EDEVICE);        \
    } while (0)

struct DevMem {
    void *p = nullptr;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem() {
        if (p)
            (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes) {
        if (p)
            (void)hipFree(p);
        p = nullptr;
        return hipMalloc(&p, std::max<size_t>(bytes, 16));
    }
    template <typename U>
    U *as() const {
        return static_cast<U *>(p);
    }
};

struct Blas {
    rocblas_handle h = nullptr;
    ~Blas() {
        if (h)
            (void)rocblas_destroy_handle(h);
    }
};

// Row-major host matrices of complex doubles.
using Mat = std::vector<zd>;

// Per-wedge result kept on the device until the layout is known.
struct TaylorFactors {
    DevMem X, Y;  // N^2 x q and q x nmem, row-major complex double
    int q = 0;
};

// One compression of X Y times the expansion of order k (step 3).
fio_status taylor_step(Blas &bl, long long NN, int nmem, int k, double zs, const std::vector<double> &u, int d,
                       double thr, const DevMem &dC, TaylorFactors &F, int &q_out) {
    const int q = F.q, r = q * d;
    if (r > kTaylorMaxCols)
        return (set_error("Taylor factors: a product of " + std::to_string(r) + " columns exceeds " +
                          std::to_string(kTaylorMaxCols) + " (use more wedges)"),
                FIO_ENOTSUP);
    DevMem Xp, Yp, du, G;
    FIO_HIP_TRY(Xp.alloc(sizeof(double2) * (size_t)NN * r));
    FIO_HIP_TRY(Yp.alloc(sizeof(double2) * (size_t)r * nmem));
    FIO_HIP_TRY(du.alloc(sizeof(double) * nmem));
    FIO_HIP_TRY(G.alloc(sizeof(double2) * (size_t)r * r));
    FIO_HIP_TRY(hipMemcpy(du.p, u.data(), sizeof(double) * nmem, hipMemcpyHostToDevice));
    const long long nx = NN * q, ny = (long long)q * nmem;
    k_taylor_xp<<<(unsigned)((nx + 255) / 256), 256>>>(F.X.as<double2>(), q, dC.as<double>(), k, zs, d, NN,
                                                       Xp.as<double2>());
    FIO_HIP_TRY(hipGetLastError());
    k_taylor_yp<<<(unsigned)((ny + 255) / 256), 256>>>(F.Y.as<double2>(), q, du.as<double>(), nmem, d,
                                                       Yp.as<double2>());
    FIO_HIP_TRY(hipGetLastError());
    const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
    auto *xp = Xp.as<rocblas_double_complex>(), *yp = Yp.as<rocblas_double_complex>();
    auto *g = G.as<rocblas_double_complex>();
    // Gram of the grid side, Gx = Xp^H Xp (read row-major from the column-major result)
    Mat Gx((size_t)r * r), Gy((size_t)r * r);
    FIO_BLAS_TRY(rocblas_zgemm(bl.h, rocblas_operation_none, rocblas_operation_conjugate_transpose, r, r, (int)NN,
                               &one, xp, r, xp, r, &zero, g, r));
    FIO_HIP_TRY(hipMemcpy(Gx.data(), g, sizeof(zd) * r * r, hipMemcpyDeviceToHost));
    // Gram of the wedge side, Gy = Yp Yp^H
    FIO_BLAS_TRY(rocblas_zgemm(bl.h, rocblas_operation_conjugate_transpose, rocblas_operation_none, r, r, nmem, &one,
                               yp, nmem, yp, nmem, &zero, g, r));
    FIO_HIP_TRY(hipMemcpy(Gy.data(), g, sizeof(zd) * r * r, hipMemcpyDeviceToHost));
    // Xp = Q_X R_X with R_X = Lx^1/2 Vx^H, Yp = R_Y^H Q_Y^H with R_Y = Ly^1/2 Vy^H
    // (eigen-directions with negligible weight dropped)
    std::vector<double> lx, ly;
    Mat Vx, Vy;
    eigh(r, Gx, lx, Vx);
    eigh(r, Gy, ly, Vy);
    auto kept = [](const std::vector<double> &l) {
        int n = 0;
        while (n < (int)l.size() && l[n] > 1e-30 * std::max(l[0], 1e-300))
            ++n;
        return std::max(n, 1);
    };
    const int rx = kept(lx), ry = kept(ly);
    // B = Vx^H Vy (rx x ry), core M = Lx^1/2 B Ly^1/2
    Mat Bm((size_t)rx * ry, zd(0, 0)), M((size_t)rx * ry);
    for (int i = 0; i < rx; ++i)
        for (int j = 0; j < ry; ++j) {
            zd s(0, 0);
            for (int a = 0; a < r; ++a)
                s += std::conj(Vx[(size_t)a * r + i]) * Vy[(size_t)a * r + j];
            Bm[(size_t)i * ry + j] = s;
            M[(size_t)i * ry + j] = std::sqrt(std::max(lx[i], 0.0)) * s * std::sqrt(std::max(ly[j], 0.0));
        }
    // SVD of the core from M^H M = W S^2 W^H
    Mat MhM((size_t)ry * ry, zd(0, 0));
    for (int i = 0; i < ry; ++i)
        for (int j = 0; j < ry; ++j) {
            zd s(0, 0);
            for (int a = 0; a < rx; ++a)
                s += std::conj(M[(size_t)a * ry + i]) * M[(size_t)a * ry + j];
            MhM[(size_t)i * ry + j] = s;
        }
    std::vector<double> s2;
    Mat Wv;
    eigh(ry, MhM, s2, Wv);
    const double s1 = std::sqrt(std::max(s2[0], 0.0));
    int qn = 0;
    while (qn < ry && std::sqrt(std::max(s2[qn], 0.0)) > thr * s1)
        ++qn;
    qn = std::max(qn, 1);
    // X~ = Q_X U_q S_q = Xp Vx B Ly^1/2 W_q  ->  TX (r x qn)
    // Y~ = W_q^H Q_Y^H = S_q^-1 U_q^H Lx^1/2 B Vy^H Yp, U_q = M W_q S_q^-1  ->  TY (qn x r)
    Mat LW((size_t)ry * qn);  // Ly^1/2 W_q
    for (int j = 0; j < ry; ++j)
        for (int t = 0; t < qn; ++t)
            LW[(size_t)j * qn + t] = std::sqrt(std::max(ly[j], 0.0)) * Wv[(size_t)j * ry + t];
    Mat BLW((size_t)rx * qn, zd(0, 0));  // B Ly^1/2 W_q
    for (int i = 0; i < rx; ++i)
        for (int j = 0; j < ry; ++j) {
            const zd b = Bm[(size_t)i * ry + j];
            for (int t = 0; t < qn; ++t)
                BLW[(size_t)i * qn + t] += b * LW[(size_t)j * qn + t];
        }
    Mat TX((size_t)r * qn, zd(0, 0));
    for (int a = 0; a < r; ++a)
        for (int i = 0; i < rx; ++i) {
            const zd v = Vx[(size_t)a * r + i];
            for (int t = 0; t < qn; ++t)
                TX[(size_t)a * qn + t] += v * BLW[(size_t)i * qn + t];
        }
    // U_q^H Lx^1/2 = (M W_q S_q^-1)^H Lx^1/2 ; with M W_q = Lx^1/2 B Ly^1/2 W_q = Lx^1/2 BLW
    Mat UL((size_t)qn * rx);  // S_q^-1 U_q^H Lx^1/2, then times B Vy^H
    for (int t = 0; t < qn; ++t) {
        const double st = std::sqrt(std::max(s2[t], 0.0));
        for (int i = 0; i < rx; ++i) {
            const double li = std::max(lx[i], 0.0);
            UL[(size_t)t * rx + i] = std::conj(BLW[(size_t)i * qn + t]) * li / (st * st);
        }
    }
    Mat ULB((size_t)qn * ry, zd(0, 0));
    for (int t = 0; t < qn; ++t)
        for (int i = 0; i < rx; ++i) {
            const zd v = UL[(size_t)t * rx + i];
            for (int j = 0; j < ry; ++j)
                ULB[(size_t)t * ry + j] += v * Bm[(size_t)i * ry + j];
        }
    Mat TY((size_t)qn * r, zd(0, 0));
    for (int t = 0; t < qn; ++t)
        for (int j = 0; j < ry; ++j) {
            const zd v = ULB[(size_t)t * ry + j];
            for (int a = 0; a < r; ++a)
                TY[(size_t)t * r + a] += v * std::conj(Vy[(size_t)a * r + j]);
        }
    // X <- Xp TX, Y <- TY Yp
    DevMem dT, Xn, Yn;
    FIO_HIP_TRY(dT.alloc(sizeof(zd) * (size_t)r * qn));
    FIO_HIP_TRY(Xn.alloc(sizeof(double2) * (size_t)NN * qn));
    FIO_HIP_TRY(Yn.alloc(sizeof(double2) * (size_t)qn * nmem));
    FIO_HIP_TRY(hipMemcpy(dT.p, TX.data(), sizeof(zd) * r * qn, hipMemcpyHostToDevice));
    FIO_BLAS_TRY(rocblas_zgemm(bl.h, rocblas_operation_none, rocblas_operation_none, qn, (int)NN, r, &one,
                               dT.as<rocblas_double_complex>(), qn, xp, r, &zero,
                               Xn.as<rocblas_double_complex>(), qn));
    FIO_HIP_TRY(hipDeviceSynchronize());  // dT is reused for TY
    FIO_HIP_TRY(hipMemcpy(dT.p, TY.data(), sizeof(zd) * r * qn, hipMemcpyHostToDevice));
    FIO_BLAS_TRY(rocblas_zgemm(bl.h, rocblas_operation_none, rocblas_operation_none, nmem, qn, r, &one, yp, nmem,
                               dT.as<rocblas_double_complex>(), r, &zero, Yn.as<rocblas_double_complex>(), nmem));
    FIO_HIP_TRY(hipDeviceSynchronize());
    std::swap(F.X.p, Xn.p);
    std::swap(F.Y.p, Yn.p);
    F.q = qn;
    q_out = qn;
    return FIO_OK;
}

// s x s estimate of the relative error of X Y against the exact residual kernel.
fio_status taylor_estimate(const fio_plan_s *P, const WedgeHost &W, const TaylorFactors &F, uint64_t &state,
                           double &err) {
    const int N = P->N, h = N / 2, q = F.q, nmem = (int)W.members.size();
    const long long NN = (long long)N * N;
    const int sv = std::max(8, P->opt.verify_samples);
    const std::vector<long long> Gam = sample_points(NN, (int)std::min<long long>(sv, NN), state);
    const std::vector<int> Del = sample_members(nmem, std::min(sv, nmem), state);
    std::vector<zd> Y((size_t)q * nmem), XG((size_t)Gam.size() * q);
    FIO_HIP_TRY(hipMemcpy(Y.data(), F.Y.p, sizeof(zd) * Y.size(), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < Gam.size(); ++i)
        FIO_HIP_TRY(hipMemcpy(XG.data() + i * q, F.X.as<double2>() + Gam[i] * q, sizeof(zd) * q,
                              hipMemcpyDeviceToHost));
    const double e1 = std::cos(W.theta), e2 = std::sin(W.theta);
    double num = 0, den = 0;
    for (size_t i = 0; i < Gam.size(); ++i)
        for (int j : Del) {
            const int om = W.members[j];
            const zd a = host_residual(P->phase, N, Gam[i], e1, e2, om / N - h, om % N - h);
            zd v(0, 0);
            for (int t = 0; t < q; ++t)
                v += XG[i * q + t] * Y[(size_t)t * nmem + j];
            num += std::norm(a - v);
            den += std::norm(a);
        }
    err = std::sqrt(num / std::max(den, 1e-300));
    return FIO_OK;
}

template <typename T>
fio_status taylor_store(fio_plan_s *P, std::vector<TaylorFactors> &fac) {
    const long long NN = (long long)P->N * P->N;
    cplx<T> *gx = static_cast<cplx<T> *>(P->d_gx);
    cplx<T> *gxi = static_cast<cplx<T> *>(P->d_gxi);
    DevMem dscale;
    for (int l = 0; l < P->L; ++l) {
        const WedgeHost &W = P->wedges[l];
        const WedgeDev &D = P->wdev[l];
        if (W.q == 0)
            continue;
        const int nmem = (int)W.members.size();
        const std::vector<double> scale = member_scale(P->N, W);
        FIO_HIP_TRY(dscale.alloc(sizeof(double) * nmem));
        FIO_HIP_TRY(hipMemcpy(dscale.p, scale.data(), sizeof(double) * nmem, hipMemcpyHostToDevice));
        k_taylor_store_x<T><<<(unsigned)((NN * W.qpad + 255) / 256), 256>>>(fac[l].X.as<double2>(), W.q, W.qpad, NN,
                                                                           gx + D.gx_off);
        FIO_HIP_TRY(hipGetLastError());
        k_taylor_store_xi<T><<<(unsigned)(((long long)nmem * W.qpad + 255) / 256), 256>>>(
            fac[l].Y.as<double2>(), W.q, W.qpad, nmem, dscale.as<double>(), gxi + D.gxi_off);
        FIO_HIP_TRY(hipGetLastError());
        FIO_HIP_TRY(hipDeviceSynchronize());
    }
    return FIO_OK;
}

}  // namespace

fio_status plan_taylor(fio_plan_s *P, const double2 *d_xcoef) {
    if (P->phase.amp != 0)
        return (set_error("FIO_FACTORS_TAYLOR expands the phase alone (amplitude a = 1 only)"), FIO_ENOTSUP);
    const int N = P->N, h = N / 2;
    const long long NN = (long long)N * N;
    Blas bl;
    FIO_BLAS_TRY(rocblas_create_handle(&bl.h));
    DevMem dC, dmax, dE, dF;
    FIO_HIP_TRY(dC.alloc(sizeof(double) * NN * kTaylorK));
    FIO_HIP_TRY(dmax.alloc(sizeof(unsigned long long) * kTaylorK));
    FIO_HIP_TRY(dE.alloc(sizeof(double4) * kCauchyM));
    FIO_HIP_TRY(dF.alloc(sizeof(double2) * kCauchyM * kTaylorK));
    std::vector<double2> xc(NN);
    FIO_HIP_TRY(hipMemcpy(xc.data(), d_xcoef, sizeof(double2) * NN, hipMemcpyDeviceToHost));
    std::vector<TaylorFactors> fac(P->L);
    for (int l = 0; l < P->L; ++l) {
        WedgeHost &W = P->wedges[l];
        const int nmem = (int)W.members.size();
        if (nmem == 0)
            continue;
        // |xi| and the angle to the wedge centre of every member
        std::vector<double> rad(nmem), dth(nmem);
        double half = 0;
        for (int j = 0; j < nmem; ++j) {
            const int om = W.members[j];
            const double k1 = om / N - h, k2 = om % N - h;
            rad[j] = std::hypot(k1, k2);
            dth[j] = std::arg(std::polar(1.0, std::atan2(k2, k1) - W.theta));
            if (rad[j] > 0)
                half = std::max(half, std::fabs(dth[j]));
        }
        // the polar series converges inside the nearest singularity; the
        // Cauchy circle stays inside it too
        const double Rs = singularity_distance(P->phase, xc, W.theta);
        if (half >= 0.9 * Rs)
            return (set_error("wedge " + std::to_string(l) + ": the polar Taylor series of the residual phase " +
                              "converges within " + std::to_string(Rs) + " rad of the wedge centre, the wedge " +
                              "reaches " + std::to_string(half) + " (use more wedges)"),
                    FIO_EACCURACY);
        const double rho = std::min(kCauchyMaxRadius, 0.5 * (half + Rs));
        // 1. Taylor coefficients of the angular residual: trapezoidal weights
        // w^(-mk) / (M rho^k) and the points of the circle
        std::vector<double2> Fw(kCauchyM * kTaylorK);
        for (int m = 0; m < kCauchyM; ++m)
            for (int k = 0; k < kTaylorK; ++k) {
                const double ang = -kTwoPi * (double)((m * k) % kCauchyM) / kCauchyM;
                const double sc = 1.0 / (kCauchyM * std::pow(rho, k));
                Fw[m * kTaylorK + k] = make_double2(sc * std::cos(ang), sc * std::sin(ang));
            }
        FIO_HIP_TRY(hipMemcpy(dF.p, Fw.data(), sizeof(double2) * Fw.size(), hipMemcpyHostToDevice));
        std::vector<double4> E(kCauchyM);
        for (int m = 0; m < kCauchyM; ++m) {
            const zd th = W.theta + rho * std::polar(1.0, kTwoPi * m / kCauchyM);
            const zd c = std::cos(th), s = std::sin(th);
            E[m] = make_double4(c.real(), c.imag(), s.real(), s.imag());
        }
        FIO_HIP_TRY(hipMemcpy(dE.p, E.data(), sizeof(double4) * kCauchyM, hipMemcpyHostToDevice));
        FIO_HIP_TRY(hipMemset(dmax.p, 0, sizeof(unsigned long long) * kTaylorK));
        k_taylor_coef<<<(unsigned)((NN + 255) / 256), 256>>>(P->phase, d_xcoef, NN, std::cos(W.theta),
                                                             std::sin(W.theta), dE.as<double4>(), dF.as<double2>(),
                                                             dC.as<double>(), dmax.as<unsigned long long>());
        FIO_HIP_TRY(hipGetLastError());
        std::vector<unsigned long long> bits(kTaylorK);
        FIO_HIP_TRY(hipMemcpy(bits.data(), dmax.p, sizeof(unsigned long long) * kTaylorK, hipMemcpyDeviceToHost));
        std::vector<double> cmax(kTaylorK);
        for (int k = 0; k < kTaylorK; ++k)
            std::memcpy(&cmax[k], &bits[k], sizeof(double));
        std::vector<double> sk(kTaylorK, 0.0), zmax(kTaylorK, 0.0);
        for (int k = 1; k < kTaylorK; ++k) {
            for (int j = 0; j < nmem; ++j)
                sk[k] = std::max(sk[k], rad[j] * std::pow(std::fabs(dth[j]), k));
            zmax[k] = kTwoPi * cmax[k] * sk[k];
        }
        double thr = P->tol * P->opt.sep_tol_frac;
        uint64_t state = splitmix64(P->opt.seed ^ (0x7A1108ull * (uint64_t)(l + 1)));
        for (int attempt = 0;; ++attempt) {
            W.attempts = attempt + 1;
            // the series must have converged within the computed orders
            if (zmax[kTaylorK - 1] > 0.01 * thr)
                return (set_error("wedge " + std::to_string(l) + ": the polar Taylor series of the residual phase "
                                  "needs more than " + std::to_string(kTaylorK - 1) + " orders (use more wedges)"),
                        FIO_EACCURACY);
            TaylorFactors &F = fac[l];
            const double2 unit = make_double2(1.0, 0.0);
            std::vector<double2> ones((size_t)std::max<long long>(NN, nmem), unit);
            FIO_HIP_TRY(F.X.alloc(sizeof(double2) * NN));
            FIO_HIP_TRY(F.Y.alloc(sizeof(double2) * nmem));
            FIO_HIP_TRY(hipMemcpy(F.X.p, ones.data(), sizeof(double2) * NN, hipMemcpyHostToDevice));
            FIO_HIP_TRY(hipMemcpy(F.Y.p, ones.data(), sizeof(double2) * nmem, hipMemcpyHostToDevice));
            F.q = 1;
            // 2-3. the exponential of every order that matters, multiplied in and compressed
            for (int k = 2; k < kTaylorK; ++k) {
                if (zmax[k] <= 0.01 * thr)
                    continue;
                int d = 1;
                double term = 1.0;
                while (term > 0.1 * thr && d < 200) {
                    term *= zmax[k] / d;
                    ++d;
                }
                std::vector<double> u(nmem);
                for (int j = 0; j < nmem; ++j)
                    u[j] = sk[k] > 0 ? rad[j] * std::pow(dth[j], k) / sk[k] : 0.0;
                int qn = 0;
                const fio_status st = taylor_step(bl, NN, nmem, k, kTwoPi * sk[k], u, d, thr, dC, F, qn);
                if (st != FIO_OK)
                    return st;
            }
            W.q = F.q;
            W.r = 0;
            double err = 0;
            const fio_status st = taylor_estimate(P, W, F, state, err);
            if (st != FIO_OK)
                return st;
            W.sep_err = err;
            if (err <= 0.5 * P->tol || attempt == 3)
                break;
            thr *= 0.25;
        }
        if (W.sep_err > P->tol)
            return (set_error("wedge " + std::to_string(l) + ": Taylor separation error estimate " +
                              std::to_string(W.sep_err) + " exceeds tol"),
                    FIO_EACCURACY);
        W.C.clear();
        W.R.clear();
        W.Z.clear();
        W.P.clear();
    }
    P->regen = false;
    fio_status st = plan_layout(P);
    if (st != FIO_OK)
        return st;
    P->factor_mode = FIO_FACTORS_TAYLOR;
    return P->precision == FIO_F64 ? taylor_store<double>(P, fac) : taylor_store<float>(P, fac);
}

}  // namespace fio
