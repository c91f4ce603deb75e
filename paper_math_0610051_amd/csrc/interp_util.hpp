// Device helpers shared by the interpolation (type-2) and spreading (type-1)
// steps of the NUFFT: block reductions, the stencil origin of a nonuniform
// point on the oversampled grid, the ES kernel weight and exp(2 pi i r) in
// the plan's precision.
#pragma once

#include <cfloat>
#include <cstdint>

#include "common.hpp"

namespace fio {

__device__ inline int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ inline int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = max(v, __shfl_xor(v, o));
    return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Grid coordinate u = m (y - k) and the first cell floor(u - w/2) + 1 of the
// stencil, without floating-point contraction, so that every thread and the
// window bounds map equal inputs to equal results; the map is monotone in y.
template <int W>
__device__ inline int stencil_origin(double m, double y, double k, double &u) {
#pragma clang fp contract(off)
    u = m * (y - k);
    return (int)floor(u - 0.5 * W) + 1;
}

// Kernel weight phi(z) = exp(beta (sqrt(1 - (2z/w)^2) - 1)) of the ES kernel.
// In FP32 the hardware base-2 exponential and square root suffice: the
// argument of the exponential lies in [-beta log2(e), 0] and 1 - (2z/w)^2 is
// either at most 0 or at least 2^-23, so neither needs the range and
// denormal handling of the library functions; their error (about one ulp)
// is below that of the FP32 argument itself.
template <typename T>
__device__ __forceinline__ T es_weight(T z, T two_over_w, T beta) {
    if constexpr (sizeof(T) == 4) {
        const float u = z * two_over_w, s = 1.0f - u * u;
        return s > 0.0f ? __builtin_amdgcn_exp2f(beta * 1.44269504f * (__builtin_amdgcn_sqrtf(s) - 1.0f)) : 0.0f;
    } else {
        return es_kernel<T>(z, two_over_w, beta);
    }
}

// A plan constant read at wave-uniform addresses through the constant
// address space: the compiler then issues scalar loads, which batch and
// run ahead of the vector work, instead of one vector load and wait per value.
template <typename P>
__device__ __forceinline__ const __attribute__((address_space(4))) P *as_constant(const P *p) {
    return (const __attribute__((address_space(4))) P *)(uintptr_t)p;
}

// A plan record (a multiple of 4 bytes) copied word by word through the
// constant address space: scalar loads, of the words the caller uses only.
template <typename S>
__device__ __forceinline__ S load_constant(const S *p) {
    static_assert(sizeof(S) % 4 == 0, "record of whole words");
    S v;
    const __attribute__((address_space(4))) unsigned *src = as_constant(reinterpret_cast<const unsigned *>(p));
    unsigned *dst = reinterpret_cast<unsigned *>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(S) / 4); ++i)
        dst[i] = src[i];
    return v;
}

// FP32 regeneration of one point's separated factor (the storage-compressed
// form of the randomized separation): sums over the sampled columns c <
// zrc of A(x, C_c) Z(c, t), t < K, with each entry's phase in FP64, reduced
// by its nearest integer, and its exponential and the sums in FP32.  The K
// values Z(c, 0 .. K-1) of a column (row stride q <= K) are read at once as
// scalar loads; past q they belong to the next column or to the array's
// padding, and those sums are not used.
template <int K>
__device__ __forceinline__ void regen_sums_f32(const Phase &ph, XCoef c, double g1, double g2, const double2 *zcol,
                                               const float2 *zmat, int zrc, int q, float (&ar)[K], float (&ai)[K]) {
    const auto *zc = as_constant(reinterpret_cast<const double *>(zcol));  // (k1, k2) per column
    const auto *zm = as_constant(reinterpret_cast<const float *>(zmat));   // (re, im) per column and rank
#pragma unroll
    for (int t = 0; t < K; ++t)
        ar[t] = ai[t] = 0.0f;
    for (int cc = 0; cc < zrc; ++cc) {
        float cs, sn;
        residual_entry_f32(ph, c, g1, g2, zc[2 * cc], zc[2 * cc + 1], cs, sn);
        const auto *zr = zm + 2ll * cc * q;
        float zre[K], zim[K];
#pragma unroll
        for (int t = 0; t < K; ++t) {
            zre[t] = zr[2 * t];
            zim[t] = zr[2 * t + 1];
        }
#pragma unroll
        for (int t = 0; t < K; ++t) {
            ar[t] += cs * zre[t] - sn * zim[t];
            ai[t] += cs * zim[t] + sn * zre[t];
        }
    }
}

template <typename T>
__device__ inline void expi_t(double r, T &c, T &s);
template <>
__device__ inline void expi_t<float>(double r, float &c, float &s) {
    expi2pi_f((float)r, c, s);
}
template <>
__device__ inline void expi_t<double>(double r, double &c, double &s) {
    expi2pi(r, c, s);
}

}  // namespace fio
