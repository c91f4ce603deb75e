// Shared host/device building blocks of the FIO library: complex numbers,
// the FP64 phase families, the exponential-of-semicircle NUFFT kernel and a
// counter-based random generator.  Everything here is header-only so that
// the same code runs in kernels and in the host-side plan.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace fio {

constexpr double kTwoPi = 6.283185307179586476925286766559;

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T re, im;
};

template <typename T>
__host__ __device__ inline cplx<T> cmake(T re, T im) {
    cplx<T> c;
    c.re = re;
    c.im = im;
    return c;
}
template <typename T>
__host__ __device__ inline cplx<T> cadd(cplx<T> a, cplx<T> b) { return cmake(a.re + b.re, a.im + b.im); }
template <typename T>
__host__ __device__ inline cplx<T> csub(cplx<T> a, cplx<T> b) { return cmake(a.re - b.re, a.im - b.im); }
template <typename T>
__host__ __device__ inline cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return cmake(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// a += b * c
template <typename T>
__host__ __device__ inline void cfma(cplx<T> &a, cplx<T> b, cplx<T> c) {
    a.re += b.re * c.re - b.im * c.im;
    a.im += b.re * c.im + b.im * c.re;
}

// sin(2 pi x), cos(2 pi x) for FP64 x; exact-period device builtins on the GPU.
__host__ __device__ inline double sin2pi(double x) {
#ifdef __HIP_DEVICE_COMPILE__
    return sinpi(2.0 * x);
#else
    return std::sin(kTwoPi * x);
#endif
}
__host__ __device__ inline double cos2pi(double x) {
#ifdef __HIP_DEVICE_COMPILE__
    return cospi(2.0 * x);
#else
    return std::cos(kTwoPi * x);
#endif
}

// exp(2 pi i r) for a phase already reduced to |r| <= 1/2.
__host__ __device__ inline void expi2pi(double r, double &c, double &s) {
#ifdef __HIP_DEVICE_COMPILE__
    sincospi(2.0 * r, &s, &c);
#else
    s = std::sin(kTwoPi * r);
    c = std::cos(kTwoPi * r);
#endif
}
__device__ inline void expi2pi_f(float r, float &c, float &s) { sincospif(2.0f * r, &s, &c); }

// ---------------------------------------------------------------------------
// Phase families Phi(x, xi) = x.xi + h(x, xi) (kind numbers as in fio.h).
// The x-dependent coefficients are computed once per point (XCoef), then h
// and grad_xi h are cheap per frequency / per wedge.
// ---------------------------------------------------------------------------
struct Phase {
    int kind;
    int amp;  // amplitude kind (fio.h): 0 a = 1, 1 the Bessel amplitude of Section 4
    double p[8];
};

// Division of integers 0 <= x < 2^31 by an invariant divisor d >= 1 with a
// multiply-high and a shift (Granlund and Montgomery, "Division by invariant
// integers using multiplication", 1994): with l = ceil(log2 d) and
// m = ceil(2^(31 + l) / d), x / d = mulhi(x, m) >> (l - 1); d = 1 passes x.
// Used wherever a kernel splits flat indices by run-time extents.
struct FastDiv {
    unsigned d = 1, m = 0, s = 0;
    FastDiv() = default;
    __host__ __device__ explicit FastDiv(unsigned dd) : d(dd) {
        unsigned l = 0;
        while (l < 31 && (1u << l) < dd)
            ++l;
        if (l > 0) {
            m = (unsigned)((((unsigned long long)1 << (31 + l)) + dd - 1) / dd);
            s = l - 1;
        }
    }
    __device__ __forceinline__ int div(int x) const {
        return d == 1 ? x : (int)(__umulhi((unsigned)x, m) >> s);
    }
};

struct XCoef {
    double a, b;
};

__host__ __device__ inline bool phase_isotropic(int kind) { return kind == 1 || kind == 3 || kind == 5; }

__host__ __device__ inline XCoef phase_xcoef(const Phase &ph, double x1, double x2) {
    XCoef c{0.0, 0.0};
    switch (ph.kind) {
    case 1:
        c.a = c.b = ph.p[0];
        break;
    case 2:
        c.a = (2.0 + sin2pi(x1) * sin2pi(x2)) * 0.0625;
        c.b = (2.0 + cos2pi(x1) * cos2pi(x2)) * 0.0625;
        break;
    case 3:
        c.a = c.b = ph.p[0] * (1.0 + ph.p[1] * sin2pi(x1));
        break;
    case 4:
        c.a = (2.0 + sin2pi(2.0 * x1)) * (2.0 + sin2pi(2.0 * x2)) / 9.0;
        c.b = (2.0 + cos2pi(2.0 * x1)) * (2.0 + cos2pi(2.0 * x2)) / 9.0;
        break;
    case 5:
        c.a = c.b = ph.p[0] * (3.0 + sin2pi(2.0 * x1)) * (3.0 + sin2pi(2.0 * x2)) * 0.0625;
        break;
    default:
        break;
    }
    return c;
}

// h(x, xi)
__host__ __device__ inline double phase_h(const Phase &ph, XCoef c, double k1, double k2) {
    if (ph.kind == 0)
        return ph.p[0] * k1 + ph.p[1] * k2;
    if (phase_isotropic(ph.kind))
        return c.a * sqrt(k1 * k1 + k2 * k2);
    return ph.p[0] * sqrt(c.a * c.a * k1 * k1 + c.b * c.b * k2 * k2);
}

// grad_xi h(x, e) for a direction e (degree-0 homogeneous in e).
__host__ __device__ inline void phase_grad(const Phase &ph, XCoef c, double e1, double e2, double &g1, double &g2) {
    if (ph.kind == 0) {
        g1 = ph.p[0];
        g2 = ph.p[1];
        return;
    }
    if (phase_isotropic(ph.kind)) {
        double r = sqrt(e1 * e1 + e2 * e2);
        g1 = c.a * e1 / r;
        g2 = c.a * e2 / r;
        return;
    }
    double aa = c.a * c.a, bb = c.b * c.b;
    double q = sqrt(aa * e1 * e1 + bb * e2 * e2);
    g1 = ph.p[0] * aa * e1 / q;
    g2 = ph.p[0] * bb * e2 / q;
}

// Residual phase Phi_ell(x, xi) = h(x, xi) - grad_xi h(x, xi_hat_ell) . xi (Section 1.3),
// given g = grad_xi h(x, xi_hat_ell); reduced by its nearest integer.
__host__ __device__ inline double residual_reduced(const Phase &ph, XCoef c, double g1, double g2, double k1,
                                                   double k2) {
    double r = phase_h(ph, c, k1, k2) - (g1 * k1 + g2 * k2);
    return r - rint(r);
}

// The Bessel amplitude of the integration along ellipses (Section 4, eq.
// (ellipses_amp), '+' sign): a = (1/4pi)(J0(2 pi rho) + i Y0(2 pi rho))
// exp(-2 pi i rho) with rho = h(x, xi) >= 0, and a = 0 at xi = 0, where Y0 is
// singular (the paper states no value there).  J0 and Y0 are the math
// library's (the device library on the GPU, the C library on the host).
__host__ __device__ inline void amp_bessel(double rho, bool origin, double &ar, double &ai) {
    if (origin) {
        ar = ai = 0.0;
        return;
    }
    const double z = kTwoPi * rho;
#ifdef __HIP_DEVICE_COMPILE__
    const double jr = j0(z), yi = y0(z);
#else
    const double jr = ::j0(z), yi = ::y0(z);
#endif
    double c, s;
    expi2pi(rho - rint(rho), c, s);
    const double k = 1.0 / (2.0 * kTwoPi);
    ar = k * (jr * c + yi * s);  // (J0 + i Y0)(c - i s) / (4 pi)
    ai = k * (yi * c - jr * s);
}

// Entry a(x, xi) exp(2 pi i Phi_ell(x, xi)) of the residual kernel of wedge
// ell (Section 3.2, with the amplitude folded in as Section 4 describes),
// given g = grad_xi h(x, xi_hat_ell); the phase is reduced by its nearest
// integer before the exponential.
__host__ __device__ inline void residual_entry(const Phase &ph, XCoef c, double g1, double g2, double k1, double k2,
                                               double &re, double &im) {
    const double hv = phase_h(ph, c, k1, k2);
    double r = hv - (g1 * k1 + g2 * k2);
    r -= rint(r);
    expi2pi(r, re, im);
    if (ph.amp == 1) {
        double ar, ai;
        amp_bessel(hv, k1 == 0.0 && k2 == 0.0, ar, ai);
        const double tr = re * ar - im * ai;
        im = re * ai + im * ar;
        re = tr;
    }
}

// residual_entry for FP32 consumers (amplitude a = 1): the phase in FP64,
// reduced by its nearest integer to |r| <= 1/2, then exp(2 pi i r) from the
// hardware sine and cosine, which take their argument in revolutions (on
// gfx950 within 1.3e-7 of the FP64 values over |r| <= 1/2, measured on 4M
// points: FP32 rounding level).
__device__ inline void residual_entry_f32(const Phase &ph, XCoef c, double g1, double g2, double k1, double k2,
                                          float &re, float &im) {
    double r = phase_h(ph, c, k1, k2) - (g1 * k1 + g2 * k2);
    r -= rint(r);
    re = __builtin_amdgcn_cosf((float)r);
    im = __builtin_amdgcn_sinf((float)r);
}
// ---------------------------------------------------------------------------
// Exponential-of-semicircle kernel (Barnett, Magland, af Klinteberg 2019):
// phi(z) = exp(beta (sqrt(1 - (2z/w)^2) - 1)) on |z| < w/2, zero outside.
// ---------------------------------------------------------------------------
template <typename T>
__host__ __device__ inline T es_kernel(T z, T two_over_w, T beta) {
    T u = z * two_over_w;
    T s = T(1) - u * u;
    return s > T(0) ? exp(beta * (sqrt(s) - T(1))) : T(0);
}

// splitmix64 (Steele, Lea, Flood 2014): a counter-based 64-bit generator.
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace fio
