// Mixed-radix Stockham FFT passes (radices 2, 3, 4, 5, 8) used by the
// oversampled-grid transforms of the type-2 NUFFT, run in place in LDS.
//
// Layout: nb transforms of length n are interleaved, element j of transform
// b at index j*nb + b, so that consecutive lanes touch consecutive words.
// Sign: exp(+2 pi i j k / n), unnormalised (the inverse DFT without 1/n),
// which is what the interpolation step of a type-2 NUFFT needs.
#pragma once

#include "common.hpp"

namespace fio {

constexpr int kMaxPasses = 24;

// Radix plan of a length n = 2^a 3^b 5^c: for even n a radix-2 pass first
// (which a half-empty input lets the caller fold into its load, see
// fft_inplace's first_pass), then radix 8, 4/2, 3, 5.
// ns[p] divides flat butterfly indices by Ns = radix[0] * ... * radix[p-1].
struct FftPlan {
    int n;
    int npass;
    int radix[kMaxPasses];
    int tfac[kMaxPasses];  // n / (Ns radix[p]): twiddle stride per unit of k
    FastDiv ns[kMaxPasses];
};

inline bool fft_make_plan(int n, FftPlan &pl) {
    pl.n = n;
    pl.npass = 0;
    int m = n;
    if (n < 1)
        return false;
    if (m % 2 == 0) {
        pl.radix[pl.npass++] = 2;
        m /= 2;
    }
    while (m % 8 == 0 && pl.npass < kMaxPasses) {
        pl.radix[pl.npass++] = 8;
        m /= 8;
    }
    while (m % 4 == 0 && pl.npass < kMaxPasses) {
        pl.radix[pl.npass++] = 4;
        m /= 4;
    }
    while (m % 2 == 0 && pl.npass < kMaxPasses) {
        pl.radix[pl.npass++] = 2;
        m /= 2;
    }
    while (m % 3 == 0 && pl.npass < kMaxPasses) {
        pl.radix[pl.npass++] = 3;
        m /= 3;
    }
    while (m % 5 == 0 && pl.npass < kMaxPasses) {
        pl.radix[pl.npass++] = 5;
        m /= 5;
    }
    int Ns = 1;
    for (int p = 0; p < pl.npass; ++p) {
        pl.ns[p] = FastDiv((unsigned)Ns);
        pl.tfac[p] = n / (Ns * pl.radix[p]);
        Ns *= pl.radix[p];
    }
    return m == 1;
}

// Smallest 2^a 3^b 5^c >= n with a >= 1 (even lengths keep the grid symmetric).
inline int fft_nice_size(int n) {
    if (n < 2)
        n = 2;
    for (int m = n;; ++m) {
        if (m & 1)
            continue;
        int r = m;
        while (r % 2 == 0)
            r /= 2;
        while (r % 3 == 0)
            r /= 3;
        while (r % 5 == 0)
            r /= 5;
        if (r == 1)
            return m;
    }
}

template <typename T>
__host__ __device__ inline cplx<T> mul_i(cplx<T> a) {  // i * a
    return cmake(-a.im, a.re);
}

// In-register DFT of size R with the + sign: y_s = sum_r v_r exp(+2 pi i r s / R).
template <typename T, int R>
__host__ __device__ inline void dft_small(cplx<T> *v);

template <typename T>
__host__ __device__ inline void dft2(cplx<T> &a, cplx<T> &b) {
    cplx<T> t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <>
__host__ __device__ inline void dft_small<float, 2>(cplx<float> *v) { dft2(v[0], v[1]); }
template <>
__host__ __device__ inline void dft_small<double, 2>(cplx<double> *v) { dft2(v[0], v[1]); }

template <typename T>
__host__ __device__ inline void dft4(cplx<T> &v0, cplx<T> &v1, cplx<T> &v2, cplx<T> &v3) {
    cplx<T> t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = mul_i(csub(v1, v3));
    v0 = cadd(t0, t2);
    v2 = csub(t0, t2);
    v1 = cadd(t1, t3);
    v3 = csub(t1, t3);
}
template <>
__host__ __device__ inline void dft_small<float, 4>(cplx<float> *v) { dft4(v[0], v[1], v[2], v[3]); }
template <>
__host__ __device__ inline void dft_small<double, 4>(cplx<double> *v) { dft4(v[0], v[1], v[2], v[3]); }

template <typename T>
__host__ __device__ inline void dft8(cplx<T> *v) {
    // even / odd split, then y_s = E_s + W8^s O_s, y_{s+4} = E_s - W8^s O_s
    cplx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cplx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const T h = T(0.70710678118654752440084436210485);
    cplx<T> w1 = cmake(h * (o1.re - o1.im), h * (o1.re + o1.im));    // (1+i)/sqrt2 * o1
    cplx<T> w2 = mul_i(o2);                                          // i * o2
    cplx<T> w3 = cmake(-h * (o3.re + o3.im), h * (o3.re - o3.im));   // (-1+i)/sqrt2 * o3
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, w1);
    v[5] = csub(e1, w1);
    v[2] = cadd(e2, w2);
    v[6] = csub(e2, w2);
    v[3] = cadd(e3, w3);
    v[7] = csub(e3, w3);
}
template <>
__host__ __device__ inline void dft_small<float, 8>(cplx<float> *v) { dft8(v); }
template <>
__host__ __device__ inline void dft_small<double, 8>(cplx<double> *v) { dft8(v); }

template <typename T>
__host__ __device__ inline void dft3(cplx<T> *v) {
    const T c = T(-0.5), s = T(0.86602540378443864676372317075294);
    cplx<T> a = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    cplx<T> y0 = cadd(v[0], a);
    cplx<T> m = cmake(v[0].re + c * a.re, v[0].im + c * a.im);
    cplx<T> j = cmake(-s * d.im, s * d.re);  // i s (v1 - v2)
    v[0] = y0;
    v[1] = cadd(m, j);
    v[2] = csub(m, j);
}
template <>
__host__ __device__ inline void dft_small<float, 3>(cplx<float> *v) { dft3(v); }
template <>
__host__ __device__ inline void dft_small<double, 3>(cplx<double> *v) { dft3(v); }

template <typename T>
__host__ __device__ inline void dft5(cplx<T> *v) {
    const T c1 = T(0.30901699437494742410229341718282), s1 = T(0.95105651629515357211643933337938);
    const T c2 = T(-0.80901699437494742410229341718282), s2 = T(0.58778525229247312916870595463907);
    cplx<T> a1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
    cplx<T> a2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
    cplx<T> y0 = cadd(v[0], cadd(a1, a2));
    cplx<T> m1 = cmake(v[0].re + c1 * a1.re + c2 * a2.re, v[0].im + c1 * a1.im + c2 * a2.im);
    cplx<T> m2 = cmake(v[0].re + c2 * a1.re + c1 * a2.re, v[0].im + c2 * a1.im + c1 * a2.im);
    // i (s1 d1 + s2 d2) and i (s2 d1 - s1 d2)
    cplx<T> j1 = mul_i(cmake(s1 * d1.re + s2 * d2.re, s1 * d1.im + s2 * d2.im));
    cplx<T> j2 = mul_i(cmake(s2 * d1.re - s1 * d2.re, s2 * d1.im - s1 * d2.im));
    v[0] = y0;
    v[1] = cadd(m1, j1);
    v[4] = csub(m1, j1);
    v[2] = cadd(m2, j2);
    v[3] = csub(m2, j2);
}
template <>
__host__ __device__ inline void dft_small<float, 5>(cplx<float> *v) { dft5(v); }
template <>
__host__ __device__ inline void dft_small<double, 5>(cplx<double> *v) { dft5(v); }

// In-place Stockham pass of radix R (decimation in time) on one LDS buffer.
// Butterfly w = j * nb + b reads buf[(j + r m) nb + b], r < R, m = n / R,
// twiddles input r by W^(r k n / (Ns R)) with k = j mod Ns, W = exp(2 pi i / n),
// and writes output s to buf[((j / Ns) Ns R + k + s Ns) nb + b].  KB bounds
// the butterflies per worker: (n / R) * nb <= KB * nthreads.  twl: the n
// twiddles W^i, i < n, in LDS (twl[0] = 1, and a product with 1 is exact, so
// k = 0 needs no branch).  A worker issues the loads of all its butterflies,
// elements and twiddles, before the first product, so that the LDS latencies
// overlap; workers past the end read butterfly 0 and store nothing.  The
// workgroup synchronises, the results are written back, and it synchronises
// again.
template <typename T, int R, int KB>
__device__ __forceinline__ void stockham_pass_inplace(cplx<T> *buf, int n, int nb, const FastDiv &fnb, int Ns,
                                                      const FastDiv &fns, int tfac, const cplx<T> *twl, int tid,
                                                      int nthreads) {
    const int m = n / R;
    const int total = m * nb;
    cplx<T> v[KB][R], tw[KB][R];
    int dst[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        int w0 = tid + k * nthreads;
        // opaque to the compiler: the butterfly addresses are recomputed in
        // every pass instead of being held in registers across all passes
        asm volatile("" : "+v"(w0));
        const int w = w0 < total ? w0 : 0;
        const int j = fnb.div(w), b = w - j * nb;
        const int jq = fns.div(j), kk = j - jq * Ns;
        const int tstep = tfac * kk;
#pragma unroll
        for (int r = 0; r < R; ++r)
            v[k][r] = buf[(j + r * m) * nb + b];
#pragma unroll
        for (int r = 1; r < R; ++r)
            tw[k][r] = twl[r * tstep];
        dst[k] = w0 < total ? (jq * Ns * R + kk) * nb + b : -1;
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
#pragma unroll
        for (int r = 1; r < R; ++r)
            v[k][r] = cmul(v[k][r], tw[k][r]);
        dft_small<T, R>(v[k]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KB; ++k)
        if (dst[k] >= 0) {
#pragma unroll
            for (int s = 0; s < R; ++s)
                buf[dst[k] + s * Ns * nb] = v[k][s];
        }
    __syncthreads();
}

// All passes of a length-n transform of nb interleaved sequences in place;
// E = elements per worker the buffer holds at most (n * nb <= E * nthreads).
// first_pass = 1 starts after the plan's leading radix-2 pass, whose output
// the caller has already written: when every pair (x[j], x[j + n/2]) holds at
// most one nonzero x, that pass maps it to buf[2j] = x and buf[2j + 1] = +x
// (nonzero in the lower half) or -x (upper half).
template <typename T, int E>
__device__ __forceinline__ void fft_inplace(cplx<T> *buf, const FftPlan *pl, int n, int nb, const FastDiv &fnb,
                                            const cplx<T> *twl, int tid, int nthreads, int first_pass = 0) {
    int Ns = first_pass ? pl->radix[0] : 1;
    const int npass = pl->npass;
    for (int p = first_pass; p < npass; ++p) {
        const int R = pl->radix[p];
        const FastDiv fns = pl->ns[p];
        const int tfac = pl->tfac[p];
        switch (R) {
        case 8:
            stockham_pass_inplace<T, 8, (E + 7) / 8>(buf, n, nb, fnb, Ns, fns, tfac, twl, tid, nthreads);
            break;
        case 4:
            stockham_pass_inplace<T, 4, (E + 3) / 4>(buf, n, nb, fnb, Ns, fns, tfac, twl, tid, nthreads);
            break;
        case 2:
            stockham_pass_inplace<T, 2, (E + 1) / 2>(buf, n, nb, fnb, Ns, fns, tfac, twl, tid, nthreads);
            break;
        case 3:
            stockham_pass_inplace<T, 3, (E + 2) / 3>(buf, n, nb, fnb, Ns, fns, tfac, twl, tid, nthreads);
            break;
        default:
            stockham_pass_inplace<T, 5, (E + 4) / 5>(buf, n, nb, fnb, Ns, fns, tfac, twl, tid, nthreads);
            break;
        }
        Ns *= R;
    }
}

}  // namespace fio
