// Device helpers shared by the interpolation (type-2) and spreading (type-1)
// steps of the NUFFT: block reductions, the stencil origin of a nonuniform
// point on the oversampled grid, the ES kernel weight and exp(2 pi i r) in
// the plan's precision.
#pragma once

#include <cfloat>

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
