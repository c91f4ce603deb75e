// The evaluation step of Section 3.4 as three gfx950 kernels:
//
//   stage 1 (k_rows):  fhat_{ell t} = gamma^xi_{ell t} chi_ell fhat placed in the
//                      sheared, centred box of W_ell (the deconvolution 1/phi_hat
//                      and the 1/N of eq. (dfio) are folded into gamma^xi), then
//                      the oversampled inverse FFT along axis 2 of every box row;
//   stage 2 (k_cols):  the inverse FFT along axis 1 of the zero-padded columns;
//   stage 3 (k_interp):type-2 interpolation of the q grids of every wedge at the
//                      warped points M^{-T} grad_xi Phi(x, xi_hat_ell), modulation
//                      by exp(2 pi i y . M^{-1} xi_c), combination with
//                      gamma^x_{ell t}(x) and accumulation over ell in registers.
//
// Stages 1 and 2 run LDS-resident Stockham transforms; stage 3 is atomic-free:
// each thread owns one output point and loops over all wedges.
#include <cfloat>
#include <climits>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "apply.hpp"
#include "interp_util.hpp"

namespace fio {

// ---------------------------------------------------------------------------
// Pruned first pass.  When the nonzeros of a length-n sequence fill at most
// half of it around index 0 (a centred box in an oversampled grid), every pair
// (x[j], x[j + n/2]) holds at most one of them, and the plan's leading
// radix-2 Stockham pass turns x into buf[2j] = x and buf[2j + 1] = +x for
// j < n/2, or -x above.  slot_code packs the buffer position of input index
// j at column col (row stride `stride`) with the sign in bit 0; store_slot
// writes the value (and, pruned, its partner).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int slot_code(bool pruned, int j, int n, int stride, int col) {
    if (!pruned)
        return (j * stride + col) << 1;
    const int h = n >> 1;
    return j < h ? ((2 * j * stride + col) << 1) : (((2 * (j - h)) * stride + col) << 1) | 1;
}

template <typename T>
__device__ __forceinline__ void store_slot(cplx<T> *buf, int code, int stride, bool pruned, cplx<T> v) {
    const int pos = code >> 1;
    buf[pos] = v;
    if (pruned)
        buf[pos + stride] = (code & 1) ? cmake<T>(-v.re, -v.im) : v;
}

// 16-byte unit of H, G and the staged window: two complex floats or one
// complex double.
template <typename T>
struct Unit16;
template <>
struct Unit16<float> {
    using type = float4;
};
template <>
struct Unit16<double> {
    using type = double2;
};

template <typename U>
__device__ __forceinline__ U neg_unit(U v);
template <>
__device__ __forceinline__ float4 neg_unit(float4 v) {
    return make_float4(-v.x, -v.y, -v.z, -v.w);
}
template <>
__device__ __forceinline__ double2 neg_unit(double2 v) {
    return make_double2(-v.x, -v.y);
}

// ---------------------------------------------------------------------------
// Stage 1: window x factor -> box rows, FFT along axis 2 (length n2, the short
// side of the box).  One workgroup per (wedge, nr adjacent box rows, rank
// chunk); loops over the batch; in-place LDS transform of nr * tn sequences.
// H is plane-major: plane P = j2 * qu + t / CPU (CPU complex per 16 bytes)
// holds element [(P * B1 + k1) * CPU + t % CPU], so the nr rows of one
// (column, plane) leave as one contiguous run.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void rows_body(const PlanArgs<T> &a, const RowItem it, const cplx<T> *__restrict__ fhat,
                                          long long fstride, int B) {
    constexpr int E = kRowLdsBytes / (int)sizeof(cplx<T>) / kFftThreads;
    using U = typename Unit16<T>::type;
    constexpr int CPU = 16 / (int)sizeof(cplx<T>);
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
    U *bu = reinterpret_cast<U *>(smem_raw);
    const WedgeDev &W = a.wedges[it.l];
    const int n = W.n2, nr = it.nr, tn = it.tn, nbt = nr * tn, q = W.q, B1 = W.B1, B2 = W.B2, lo2 = W.lo2;
    const int k1 = it.k1, t0 = it.t0;
    const long long H_off = W.H_off;
    const int tid = threadIdx.x, nt = blockDim.x;
    const FftPlan *pl = a.fftplans + W.fft2;
    cplx<T> *twl = buf + n * nbt;  // the n twiddles follow the transform buffer
    for (int i = tid; i < n; i += nt)
        twl[i] = a.tw[W.tw2 + i];
    // copies, not references: the stores to H could alias the wedge and item
    // records as far as the compiler knows
    const FastDiv ftn = it.ftn, fb2 = W.fB2, fnbt = it.fnbt, fnr = it.fnr, fnpl = it.fnpl;
    // the box fills at most half the row: the first radix-2 pass is folded into the scatter
    const bool pruned = pl->radix[0] == 2 && n >= 2 * B2;
    const int *map = a.map + W.map_off + (long long)k1 * B2;
    const int *omega = a.omega + W.mem_off;
    const cplx<T> *gxi = a.gxi + W.gxi_off + t0;
    // This thread's box cells (row r, box column k2, rank t; rank fastest):
    // buffer position, input index and frequency factor do not depend on
    // the right-hand side, so they are looked up once for the whole batch:
    // the box map of every cell first, then the input indices and factors,
    // two rounds of dependent loads.  (Cells beyond KR * nt, possible only
    // for oversampling below 2, are looked up per right-hand side.)
    constexpr int KR = (E + 1) / 2;
    const int ncell = nr * B2 * tn;
    int dst[KR], fidx[KR];
    cplx<T> g[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int i0 = tid + k * nt, i = i0 < ncell ? i0 : 0;
        const int rk = ftn.div(i), t = i - rk * tn;
        const int r = fb2.div(rk), k2 = rk - r * B2;
        const int m = map[r * B2 + k2];
        fidx[k] = i0 < ncell ? m : -1;  // the box map entry, for now
        int j2 = lo2 + k2;
        if (j2 < 0)
            j2 += n;
        dst[k] = slot_code(pruned, j2, n, nbt, r * tn + t);
    }
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int i0 = tid + k * nt, i = i0 < ncell ? i0 : 0;
        const int t = i - ftn.div(i) * tn;
        const int m = fidx[k] >= 0 ? fidx[k] : 0;
        if (fidx[k] < 0)
            dst[k] = -1;
        fidx[k] = omega[m];
        g[k] = gxi[(long long)m * q + t];
    }
    // this thread's inputs of the next right-hand side, fetched during the
    // current one's transform (FP32; FP64 has no registers to spare for them)
    constexpr bool kPrefetch = sizeof(T) == 4;
    cplx<T> fv[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k)
        fv[k] = fhat[dst[k] >= 0 ? fidx[k] : 0];
    const bool whole = tn % CPU == 0 && t0 % CPU == 0;
    const int qu = q / CPU;
    for (int b = 0; b < B; ++b) {
        // n is even, so the buffer is a whole number of 16-byte units
        for (int i = tid; i < n * nbt / CPU; i += nt)
            bu[i] = U{};
        __syncthreads();
        const cplx<T> *f = fhat + b * fstride;
        if (!kPrefetch && b > 0) {
#pragma unroll
            for (int k = 0; k < KR; ++k)
                fv[k] = f[dst[k] >= 0 ? fidx[k] : 0];
        }
#pragma unroll
        for (int k = 0; k < KR; ++k)
            if (dst[k] >= 0)
                store_slot(buf, dst[k], nbt, pruned, cmul(fv[k], g[k]));
        if (kPrefetch && b + 1 < B) {
#pragma unroll
            for (int k = 0; k < KR; ++k)
                fv[k] = f[fstride + (dst[k] >= 0 ? fidx[k] : 0)];
        }
        for (int i = tid + KR * nt; i < ncell; i += nt) {
            const int rk = ftn.div(i), t = i - rk * tn;
            const int r = fb2.div(rk), k2 = rk - r * B2;
            const int m = map[r * B2 + k2];
            if (m >= 0) {
                int j2 = lo2 + k2;
                if (j2 < 0)
                    j2 += n;
                store_slot(buf, slot_code(pruned, j2, n, nbt, r * tn + t), nbt, pruned,
                           cmul(f[omega[m]], gxi[(long long)m * q + t]));
            }
        }
        __syncthreads();
        fft_inplace<T, E>(buf, pl, n, nbt, fnbt, twl, tid, nt, pruned ? 1 : 0);
        // buf[j2 * nbt + r * tn + t] -> H[((j2 * qu + (t0 + t) / CPU) * B1 + k1 + r) * CPU + (t0 + t) % CPU]
        cplx<T> *H = a.H + b * a.H_stride + H_off;
        if (whole) {
            // whole planes: 16-byte unit u = (j2 * npl + pl) * nr + r follows H
            U *Hu = reinterpret_cast<U *>(H);
            const int npl = tn / CPU;
            for (int u = tid; u < n * nbt / CPU; u += nt) {
                const int jp = fnr.div(u), r = u - jp * nr;
                const int j2 = fnpl.div(jp), p = jp - j2 * npl;
                Hu[(long long)(j2 * qu + t0 / CPU + p) * B1 + k1 + r] = bu[(j2 * nbt + r * tn) / CPU + p];
            }
        } else {
            for (int i = tid; i < n * nbt; i += nt) {
                const int j2 = fnbt.div(i), cc = i - j2 * nbt, r = ftn.div(cc), t = t0 + cc - r * tn;
                H[((long long)(j2 * qu + t / CPU) * B1 + k1 + r) * CPU + t % CPU] = buf[i];
            }
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(kFftWavesPerEU))) void k_rows(PlanArgs<T> a, const RowItem *__restrict__ items,
                                                      const cplx<T> *__restrict__ fhat, long long fstride, int B) {
    rows_body<T>(a, items[blockIdx.x], fhat, fstride, B);
}

// A fused launch reads each instance's arguments from a device table, and
// pointers loaded from memory are generic (flat) to the compiler: the wedge
// records would be read with flat vector loads instead of scalar ones, and
// every buffer access would go through flat instructions.  All of these
// pointers address global memory; passing them through an integer into the
// global address space restores what a kernel argument gives for free.
template <typename P>
__device__ __forceinline__ P *as_global(P *p) {
    return (P *)(__attribute__((address_space(1))) P *)(uintptr_t)p;
}

template <typename T>
__device__ __forceinline__ InstArgs<T> load_inst(const InstArgs<T> *inst, int i) {
    InstArgs<T> I = inst[i];
    PlanArgs<T> &a = I.a;
    a.wedges = as_global(a.wedges);
    a.fftplans = as_global(a.fftplans);
    a.map = as_global(a.map);
    a.omega = as_global(a.omega);
    a.gxi = as_global(a.gxi);
    a.gx = as_global(a.gx);
    a.tw = as_global(a.tw);
    a.H = as_global(a.H);
    a.G = as_global(a.G);
    a.zcol = as_global(a.zcol);
    a.zmat = as_global(a.zmat);
    a.zmat32 = as_global(a.zmat32);
    I.fhat = as_global(I.fhat);
    I.u = as_global(I.u);
    return I;
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(kFftWavesPerEU))) void k_rows_multi(const InstArgs<T> *__restrict__ inst,
                                                            const MultiRowItem *__restrict__ items) {
    const MultiRowItem &m = items[blockIdx.x];
    const InstArgs<T> I = load_inst(inst, m.inst);
    rows_body<T>(I.a, m.it, I.fhat, (long long)I.a.N * I.a.N, I.B);
}

// ---------------------------------------------------------------------------
// Stage 2: FFT along axis 1 (length n1, the long side) of nb transforms
// tau = j2 * q + t, tau0 <= tau < tau0 + nb, of right-hand side b; rows
// outside the box are the implicit zero padding.  Items hold whole planes
// (16-byte rank groups of a column: nb and tau0 multiples of CPU) or single
// ranks of one plane.  H and G are both plane-major, so a whole-plane item
// reads one contiguous block and writes one contiguous column per plane.
// Many small workgroups per CU overlap one another's load, transform and
// store phases.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void cols_body(const PlanArgs<T> &a, const ColItem it, int b) {
    constexpr int E = kColLdsBytes / (int)sizeof(cplx<T>) / kColThreads;
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
    const WedgeDev &W = a.wedges[it.l];
    const int n = W.n1, nb = it.nb, B1 = W.B1, lo1 = W.lo1, q = W.q;
    const int tid = threadIdx.x, nt = blockDim.x;
    const FftPlan *pl = a.fftplans + W.fft1;
    cplx<T> *twl = buf + n * nb;  // the n twiddles follow the transform buffer
    for (int i = tid; i < n; i += nt)
        twl[i] = a.tw[W.tw1 + i];
    // the box fills at most half the column: the first radix-2 pass is folded
    // into the load, and only pairs without a box row are zeroed; otherwise
    // the padding rows j1 in [B1 - B1/2, n - B1/2) are zeroed
    const bool pruned = pl->radix[0] == 2 && n >= 2 * B1;
    const int z0 = pruned ? 2 * (B1 - B1 / 2) : B1 - B1 / 2, z1 = pruned ? n - 2 * (B1 / 2) : n - B1 / 2;
    for (int i = z0 * nb + tid; i < z1 * nb; i += nt)
        buf[i] = cmake<T>(0, 0);
    // copies, not references: the stores to G could alias the wedge record as
    // far as the compiler knows, and it would reload them after every store
    const FastDiv fnb = it.fnb, fq = W.fq, fb1 = W.fB1, fn = W.fn1;
    const int n2 = W.n2;
    const cplx<T> *H = a.H + (long long)b * a.H_stride + W.H_off;
    cplx<T> *G = a.G + (long long)b * a.G_stride + W.G_off;
    // H is plane-major (plane P = tau / CPU, element [(P * B1 + k1) * CPU + tau % CPU]): an item of
    // whole planes reads one contiguous block.  G is plane-major too (g_index), which makes the
    // window columns that the interpolation stages contiguous runs of each plane.
    using U = typename Unit16<T>::type;
    constexpr int CPU = 16 / (int)sizeof(cplx<T>);
    const bool whole = nb % CPU == 0 && it.tau0 % CPU == 0;
    if (whole) {
        // 16-byte unit g = p * B1 + k1 holds ranks p * CPU .. p * CPU + CPU - 1 of box row k1, which
        // land side by side in the buffer (nb and p * CPU are multiples of CPU); four loads in flight
        const U *src = reinterpret_cast<const U *>(H + (long long)it.tau0 * B1);
        U *bu = reinterpret_cast<U *>(buf);
        const int tot = B1 * (nb / CPU);
        constexpr int kIn = 4;
        for (int g0 = tid; g0 < tot; g0 += kIn * nt) {
            U v[kIn];
            int code[kIn];
#pragma unroll
            for (int k = 0; k < kIn; ++k) {
                const int g = g0 + k * nt < tot ? g0 + k * nt : g0;
                v[k] = src[g];
                const int p = fb1.div(g), k1 = g - p * B1;
                int j1 = lo1 + k1;
                if (j1 < 0)
                    j1 += n;
                code[k] = slot_code(pruned, j1, n, nb, p * CPU);
            }
#pragma unroll
            for (int k = 0; k < kIn; ++k)
                if (g0 + k * nt < tot) {
                    const int pos = (code[k] >> 1) / CPU;
                    bu[pos] = v[k];
                    if (pruned)
                        bu[pos + nb / CPU] = (code[k] & 1) ? neg_unit(v[k]) : v[k];
                }
        }
    } else {
        // single ranks of one plane
        const int P = it.tau0 / CPU, c0 = it.tau0 % CPU;
        for (int i = tid; i < B1 * nb; i += nt) {
            const int k1 = fnb.div(i), c = i - k1 * nb;
            int j1 = lo1 + k1;
            if (j1 < 0)
                j1 += n;
            store_slot(buf, slot_code(pruned, j1, n, nb, c), nb, pruned, H[((long long)P * B1 + k1) * CPU + c0 + c]);
        }
    }
    __syncthreads();
    fft_inplace<T, E>(buf, pl, n, nb, fnb, twl, tid, nt, pruned ? 1 : 0);
    // buffer element j1 * nb + c (transform tau = tau0 + c = j2 * q + t) -> G[g_index(j1, j2, t)]
    if (whole) {
        // one 16-byte unit per (plane, cell); consecutive threads take consecutive cells of a
        // plane, so each plane's column leaves as one contiguous run
        const U *bu = reinterpret_cast<const U *>(buf);
        U *Gu = reinterpret_cast<U *>(G);
        const int nbu = nb / CPU;
        for (int u = tid; u < n * nbu; u += nt) {
            const int cu = fn.div(u), j1 = u - cu * n;
            const int tau = it.tau0 + cu * CPU, j2 = fq.div(tau), t = tau - j2 * q;
            Gu[((long long)(t / CPU) * n2 + j2) * n + j1] = bu[j1 * nbu + cu];
        }
    } else {
        for (int i = tid; i < n * nb; i += nt) {
            const int j1 = fnb.div(i), c = i - j1 * nb;
            const int tau = it.tau0 + c, j2 = fq.div(tau), t = tau - j2 * q;
            G[g_index<CPU>(j1, j2, t, n, n2)] = buf[i];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kColThreads) __attribute__((amdgpu_waves_per_eu(kColWavesPerEU))) void k_cols(
    PlanArgs<T> a, const ColItem *__restrict__ items) {
    cols_body<T>(a, items[blockIdx.x], blockIdx.y);
}

template <typename T>
__global__ __launch_bounds__(kColThreads) __attribute__((amdgpu_waves_per_eu(kColWavesPerEU))) void k_cols_multi(
    const InstArgs<T> *__restrict__ inst, const MultiColItem *__restrict__ items) {
    const MultiColItem &m = items[blockIdx.x];
    const InstArgs<T> I = load_inst(inst, m.inst);
    cols_body<T>(I.a, m.it, m.b);
}

// ---------------------------------------------------------------------------
// Stage 3: interpolate + modulate + combine over t + accumulate over ell.
// A workgroup owns a kTileX x kTileX tile of output points (one per thread)
// and loops over the wedges.  For one wedge the stencils of the tile cover a
// small window of the oversampled grid.  The window is found by a block
// min/max reduction, with grid coordinates unwrapped around the tile's corner
// point so that the periodic wrap cannot split it; a launch without
// right-hand sides records it per tile and wedge at plan time, and applies
// read the record.  The window is staged into LDS plane by plane, each window
// column one contiguous run of the plane-major G, and every thread
// interpolates its point from LDS.  A window larger than the LDS budget
// (strongly folded warps) is read from the grid directly instead.  Up to
// kInterpBatch right-hand sides share the warped point, the kernel weights
// and gamma^x.
// ---------------------------------------------------------------------------
// Column stride (16-byte units) of the staged window, which holds each plane
// column-major: unit e = cc * S + rr is cell (J1 + rr, J2 + cc).  A
// ds_read_b128 serves 16 lanes of a wave per cycle from 64 four-byte banks,
// i.e. 16 unit residues: two different cells whose unit addresses agree mod
// 16 cost an extra cycle, while lanes reading the same cell share it.  The 16
// lanes of one cycle are not a contiguous quarter of the wave: on gfx950 they
// are the four lane quads that agree in lane bit 5 and in the parity of lane
// bits 2..4 (found with bank-conflict counters over single-lane address
// probes).  Such a lane set is closed under lane xor 1, 2, 12 and 24.  All
// lanes of one stencil read are the lanes' base cells (d1, d2) shifted by a
// common offset, so the conflicts follow from the base cells alone.  Each
// candidate stride F1 .. F1 + 7 is scored per lane set by the number of
// distinct cells minus the number of distinct residues, summed over the
// workgroup; the lowest score wins, ties going to the smaller stride.  Lane
// sets whose cells spread beyond 8 x 8 are not scored.  Contains one block
// barrier.
constexpr int kPassXor[4] = {1, 2, 12, 24};  // generators of one ds_read_b128 lane set
__device__ inline int pick_col_stride(bool active, int d1, int d2, int F1, int lane, int wave,
                                      unsigned long long *red2) {
    int m1 = active ? d1 : INT_MAX, m2 = active ? d2 : INT_MAX;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        m1 = min(m1, __shfl_xor(m1, kPassXor[k]));
        m2 = min(m2, __shfl_xor(m2, kPassXor[k]));
    }
    const int e1 = active ? d1 - m1 : 0, e2 = active ? d2 - m2 : 0;
    const bool fits = e1 < 8 && e2 < 8;
    unsigned long long cell = (active && fits) ? 1ull << (e2 * 8 + e1) : 0ull;
    int wide = fits ? 0 : 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        cell |= __shfl_xor(cell, kPassXor[k]);
        wide |= __shfl_xor(wide, kPassXor[k]);
    }
    const int ncell = __popcll(cell);
    unsigned long long packed = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        unsigned key = active ? 1u << ((e2 * (F1 + k) + e1) & 15) : 0u;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            key |= __shfl_xor(key, kPassXor[j]);
        const int score = wide ? 0 : ncell - __popc(key);  // 0..15 per lane set
        packed |= (unsigned long long)score << (8 * k);
    }
    // 8-bit fields: at most 4 x 4 x 15 = 240 per candidate over the workgroup;
    // lane xor 16 and then 32 visit the wave's other three lane sets
    packed += __shfl_xor(packed, 16);
    packed += __shfl_xor(packed, 32);
    if (lane == 0)
        red2[wave] = packed;
    __syncthreads();
    unsigned long long tot = 0;
#pragma unroll
    for (int k = 0; k < kThreads / 64; ++k)
        tot += red2[k];
    int best = 0, bs = 1 << 30;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int sc = (int)((tot >> (8 * k)) & 0xFF);
        if (sc < bs) {
            bs = sc;
            best = k;
        }
    }
    return F1 + best;
}

// Window of a tile's stencils on one wedge's grid from the sheared
// coordinates of its points.  The coordinates are unwrapped around floor of
// the smallest one, so the periodic wrap cannot split the window; the
// stencil origin is monotone in the coordinate, so the bounds follow from
// the extreme points with the same arithmetic.  Contains two block barriers
// (the second, in pick_col_stride, also separates these reads of red from
// the next call's writes).
template <int W>
__device__ __forceinline__ WinRec tile_window(bool active, double yp1, double yp2, int m1, int m2, int lane, int wave,
                                              double (*red)[4], unsigned long long *red2) {
    {
        const double mn1 = wave_min(active ? yp1 : DBL_MAX), mx1 = wave_max(active ? yp1 : -DBL_MAX);
        const double mn2 = wave_min(active ? yp2 : DBL_MAX), mx2 = wave_max(active ? yp2 : -DBL_MAX);
        if (lane == 0) {
            red[wave][0] = mn1;
            red[wave][1] = mx1;
            red[wave][2] = mn2;
            red[wave][3] = mx2;
        }
    }
    __syncthreads();
    double lo1 = red[0][0], hi1 = red[0][1], lo2 = red[0][2], hi2 = red[0][3];
#pragma unroll
    for (int k = 1; k < kThreads / 64; ++k) {
        lo1 = fmin(lo1, red[k][0]);
        hi1 = fmax(hi1, red[k][1]);
        lo2 = fmin(lo2, red[k][2]);
        hi2 = fmax(hi2, red[k][3]);
    }
    const double k1 = floor(lo1), k2 = floor(lo2);
    double u1, u2, ue;
    const int j1 = stencil_origin<W>(m1, yp1, k1, u1), j2 = stencil_origin<W>(m2, yp2, k2, u2);
    const int J1 = stencil_origin<W>(m1, lo1, k1, ue), X1 = stencil_origin<W>(m1, hi1, k1, ue);
    const int J2 = stencil_origin<W>(m2, lo2, k2, ue), X2 = stencil_origin<W>(m2, hi2, k2, ue);
    WinRec r;
    r.J1 = J1;
    r.J2 = J2;
    r.F1 = X1 - J1 + W;
    r.F2 = X2 - J2 + W;
    r.S = pick_col_stride(active, j1 - J1, j2 - J2, r.F1, lane, wave, red2);
    r.k1 = (int)k1;
    r.k2 = (int)k2;
    r.pad = 0;
    return r;
}

// a += b * c as four fused multiply-adds
template <typename T>
__device__ __forceinline__ void cfma4(cplx<T> &a, cplx<T> b, cplx<T> c) {
    a.re = fma(b.re, c.re, a.re);
    a.re = fma(-b.im, c.im, a.re);
    a.im = fma(b.re, c.im, a.im);
    a.im = fma(b.im, c.re, a.im);
}

// acc[vb] += mod * v, without floating-point contraction, so that every call
// site rounds alike (a batch then equals a loop of single right-hand sides bit
// for bit).
template <typename T>
__device__ __forceinline__ cplx<T> rotate_rhs(const cplx<T> &mod, const cplx<T> &v) {
#pragma clang fp contract(off)
    return cmake<T>(mod.re * v.re - mod.im * v.im, mod.re * v.im + mod.im * v.re);
}
// acc[vb] += mv for a uniform run-time vb: one branch per register of acc
// (the empty volatile asm keeps the compiler from turning the branches into
// selects over all of acc)
#define FIO_ACC_ADD(acc, vb, mv)                          \
    do {                                                  \
        _Pragma("unroll") for (int bb_ = 0; bb_ < kInterpBatch; ++bb_) if (bb_ == (vb)) { \
            asm volatile("");                             \
            acc[bb_].re += (mv).re;                       \
            acc[bb_].im += (mv).im;                       \
        }                                                 \
    } while (0)

// gamma^x(x, t) = sum_c A(x, C_c) Z(c, t) of one point in FP64 (FP64 plans,
// amplitude included), into the LDS rows [t / CPU][thread].
template <typename T>
__device__ __forceinline__ void regen_gx_f64(const PlanArgs<T> &a, const WedgeDev &wd, XCoef c, double g1, double g2,
                                          cplx<T> *gxl, int tid) {
    constexpr int CPU = 16 / (int)sizeof(cplx<T>);
    const int q = wd.q;
    const double2 *zc = a.zcol + wd.zc_off;
    const double2 *zm = a.zmat + wd.zm_off;
    constexpr int kC = 8;
    for (int t0 = 0; t0 < q; t0 += kC) {
        double ar[kC], ai[kC];
#pragma unroll
        for (int t = 0; t < kC; ++t)
            ar[t] = ai[t] = 0;
        for (int cc = 0; cc < wd.zrc; ++cc) {
            const double2 k = zc[cc];
            double cs2, sn2;
            residual_entry(a.phase, c, g1, g2, k.x, k.y, cs2, sn2);
            const double2 *zr = zm + (long long)cc * q + t0;
#pragma unroll
            for (int t = 0; t < kC; ++t)
                if (t0 + t < q) {
                    const double2 z = zr[t];
                    ar[t] += cs2 * z.x - sn2 * z.y;
                    ai[t] += cs2 * z.y + sn2 * z.x;
                }
        }
#pragma unroll
        for (int t = 0; t < kC; ++t)
            if (t0 + t < q) {
                const int tt = t0 + t;
                gxl[((tt / CPU) * kThreads + tid) * CPU + tt % CPU] = cmake<T>((T)ar[t], (T)ai[t]);
            }
    }
}

template <typename T, int W, bool REGEN>
__device__ __forceinline__ void interp_body(const PlanArgs<T> &a, cplx<T> *__restrict__ u, long long ustride, int B,
                                            int bofs, int l0, int l1, int tile) {
    using U = typename Unit16<T>::type;
    constexpr int CPU = 16 / (int)sizeof(cplx<T>);  // complex per 16-byte unit (rank pair / single rank)
    const int win_bytes = interp_window_bytes<T>(a.qmax);
    const int kUnits = win_bytes / 16;               // window capacity in units
    constexpr int kOff = 6;                          // staged cells per thread: windows up to 1536 cells
    extern __shared__ unsigned char smem_raw[];
    U *win = reinterpret_cast<U *>(smem_raw);
    __shared__ double red[kThreads / 64][4];
    __shared__ unsigned long long red2[kThreads / 64];
    const int N = a.N;
    const int tiles2 = (N + kTileX - 1) / kTileX, ntiles = tiles2 * tiles2;
    const int T1 = (tile / tiles2) * kTileX, T2 = (tile % tiles2) * kTileX;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // a wave covers an 8 x 8 block of the tile and each 16-lane set that one
    // ds_read_b128 cycle serves (lane bit 5, parity of lane bits 2..4) a 4 x 4
    // block: row from lane bits 3..4, column from lane bits 0..1, so that the
    // lanes of one cycle read nearby window cells
    const int grp = ((lane >> 5) << 1) | (((lane >> 2) ^ (lane >> 3) ^ (lane >> 4)) & 1);
    const int n1 = T1 + (wave >> 1) * 8 + (grp >> 1) * 4 + ((lane >> 3) & 3);
    const int n2 = T2 + (wave & 1) * 8 + (grp & 1) * 4 + (lane & 3);
    const bool active = n1 < N && n2 < N;
    const long long p = (long long)n1 * N + n2;
    const double x1 = (double)n1 / N, x2 = (double)n2 / N;
    const XCoef c = phase_xcoef(a.phase, x1, x2);
    cplx<T> acc[kInterpBatch];
#pragma unroll
    for (int b = 0; b < kInterpBatch; ++b)
        acc[b] = cmake<T>(0, 0);
    for (int l = l0; l < l1; ++l) {
        // plan constants through the constant address space: scalar loads
        // that run ahead, instead of vector loads waited on at every wedge
        const WedgeDev wd = load_constant(a.wedges + l);
        if (wd.q == 0)
            continue;
        const int m1 = wd.n1, m2 = wd.n2, q = wd.q, qu = q / CPU;
        double g1, g2;
        phase_grad(a.phase, c, wd.e1, wd.e2, g1, g2);
        // FIO_FACTORS_REGEN: gamma^x(x, t) = sum_c A(x, C_c) Z(c, t) for this
        // thread's point from the residual phase (reduced in FP64), into LDS
        // after the window ([t / CPU][thread] units; each thread reads only its own)
        cplx<T> *gxl = reinterpret_cast<cplx<T> *>(smem_raw + win_bytes);
        // the staged path reads gamma^x from LDS; larger ranks take the direct path
        const bool gx_lds = REGEN || a.qmax <= kGxLdsMaxRank<T>;
        if constexpr (REGEN && sizeof(T) == 8) {
            regen_gx_f64<T>(a, wd, c, g1, g2, gxl, tid);
        } else if constexpr (REGEN) {
            {
                // FP32 plans use gamma^x in FP32: the entries' phases in FP64,
                // their exponentials and the sums over the columns in FP32
                // (amplitude a = 1: FP32 plans do not regenerate with amplitudes)
                auto put = [&](auto kq) {
                    constexpr int K = decltype(kq)::value;
                    float ar[K], ai[K];
                    regen_sums_f32<K>(a.phase, c, g1, g2, a.zcol + wd.zc_off, a.zmat32 + wd.zm_off, wd.zrc, q, ar, ai);
#pragma unroll
                    for (int t = 0; t < K; ++t)
                        if (t < q)
                            gxl[((t / CPU) * kThreads + tid) * CPU + t % CPU] = cmake<T>(ar[t], ai[t]);
                };
                if (q <= 8)
                    put(std::integral_constant<int, 8>());
                else
                    put(std::integral_constant<int, kRegenMaxRank>());
            }
        }
        const double y1 = x1 + g1, y2 = x2 + g2;
        const double yp1 = wd.mt[0] * y1 + wd.mt[1] * y2;
        const double yp2 = wd.mt[2] * y1 + wd.mt[3] * y2;
        double psi = wd.cvec[0] * y1 + wd.cvec[1] * y2;
        psi -= rint(psi);
        T cs, sn;
        expi_t<T>(psi, cs, sn);
        // The tile's window on this wedge's grid: recorded at plan time by
        // this same kernel (so from these very coordinates), or found here.
        WinRec wr;
        if (a.win_mode == kWinUse) {
            wr = load_constant(a.win + (long long)l * ntiles + tile);
        } else {
            wr = tile_window<W>(active, yp1, yp2, m1, m2, lane, wave, red, red2);
            if (a.win_mode == kWinRecord) {
                if (tid == 0)
                    a.win[(long long)l * ntiles + tile] = wr;
                continue;  // a recording launch interpolates nothing
            }
        }
        double u1, u2;
        const int j1 = stencil_origin<W>(m1, yp1, (double)wr.k1, u1), j2 = stencil_origin<W>(m2, yp2, (double)wr.k2, u2);
        const int J1 = wr.J1, J2 = wr.J2;
        const T f1 = (T)(u1 - j1), f2 = (T)(u2 - j2);
        T w1[W], w2[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            w1[i] = es_weight<T>(f1 - T(i), a.two_over_w, a.beta);
            w2[i] = es_weight<T>(f2 - T(i), a.two_over_w, a.beta);
        }
        // small stencils use the W x W products of the weights: one FMA per
        // window value instead of a product and a row sum per stencil row
        constexpr bool k2D = sizeof(T) == 4 && W <= 6 && !REGEN;
        T w12[k2D ? W * W : 1];
        if constexpr (k2D) {
#pragma unroll
            for (int i1 = 0; i1 < W; ++i1)
#pragma unroll
                for (int i2 = 0; i2 < W; ++i2)
                    w12[i1 * W + i2] = w1[i1] * w2[i2];
        }
        const int F1 = wr.F1, F2 = wr.F2, S = wr.S;
        // The window of one plane (a rank pair in FP32) is F2 columns of S
        // units (unit e = cc * S + rr holds cell (J1 + rr, J2 + cc)), padded
        // to whole 64-unit wave chunks.  Rounds of planes are copied from G
        // straight into LDS by global_load_lds (lane i of a wave writes unit
        // 64 c + i of chunk c); a window column of a plane is one contiguous
        // run of G, so consecutive lanes read consecutive 16-byte units.
        // With two buffers the next round's copies run under the current
        // round's interpolation, with one a round is copied, then used.
        const int units = F2 * S;
        const int planeP = (units + 63) & ~63;
        const int nbuf = 2 * planeP <= kUnits ? 2 : 1;
        const int bufU = kUnits / nbuf / 64 * 64;
        const int ppr = bufU / planeP;           // planes per round
        const bool staged = gx_lds && ppr >= 1 && F1 <= m1 && F2 <= m2 && units <= kOff * kThreads;
        // lanes beyond a ragged edge of the grid run the plane loop on point 0
        // and window cell (0, 0), and their sums are never written
        const cplx<T> *gxp = a.gx + wd.gx_off + (active ? p : 0) * q;
        const cplx<T> mod = cmake(cs, sn);
        const cplx<T> *G0 = a.G + (long long)bofs * a.G_stride + wd.G_off;
        if (staged) {
            // source offsets (16-byte units within a plane) of this thread's
            // units tid + k kThreads; padding units copy cell 0 of the plane.
            // J1 > -W and J1 + F1 <= 2 m1 (likewise for axis 2), so one
            // conditional wrap brings every window cell onto the grid
            int off[kOff];
            const int c0 = J2 < 0 ? J2 + m2 : (J2 >= m2 ? J2 - m2 : J2);
            const int r0 = J1 < 0 ? J1 + m1 : (J1 >= m1 ? J1 - m1 : J1);
            const float rS = 1.0f / (float)S;
#pragma unroll
            for (int k = 0; k < kOff; ++k) {
                const int e = tid + k * kThreads;
                off[k] = 0;
                if (e < units) {
                    // e / S for e < 2^11: the float quotient is off by at most one
                    int cc = (int)((float)e * rS);
                    if (cc * S > e)
                        --cc;
                    else if ((cc + 1) * S <= e)
                        ++cc;
                    const int rr = e - cc * S;
                    if (rr < F1) {
                        int gr = r0 + rr;
                        if (gr >= m1)
                            gr -= m1;
                        int gc = c0 + cc;
                        if (gc >= m2)
                            gc -= m2;
                        off[k] = gc * m1 + gr;
                    }
                }
            }
            const int base = active ? (j2 - J2) * S + (j1 - J1) : 0;
            // stored gamma^x rows of the tile's points, copied into LDS
            // ([t / CPU][thread] units) with the first round; the interpolation
            // then never waits on a global load of its own
            if constexpr (!REGEN) {
                for (int tl = 0; tl < qu; ++tl)
                    __builtin_amdgcn_global_load_lds(
                        reinterpret_cast<const void *>(gxp + tl * CPU),
                        (__attribute__((address_space(3))) void *)(reinterpret_cast<U *>(gxl) + tl * kThreads +
                                                                    wave * 64),
                        16, 0, 0);
            }
            // Planes (b, tl), right-hand side major, go ppr to a round, so one
            // round serves several right-hand sides between two barriers.
            const int nplanes = B * qu;
            const int nrounds = (nplanes + ppr - 1) / ppr;
            int sb = 0, stl = 0;         // (b, tl) of the next plane to copy
            int cb = 0, ctl = 0;         // (b, tl) of the next plane to interpolate
            cplx<T> v = cmake<T>(0, 0);  // partial sum of right-hand side vb
            int vb = 0;
            for (int r = 0; r <= nrounds; ++r) {
                // copy round r (two buffers: while round r - 1 is interpolated)
                const bool copy_now = r < nrounds && (nbuf == 2 || r == 0);
                for (int pass = 0; pass < 2; ++pass) {
                    if (pass == 0 ? copy_now : (nbuf == 1 && r > 0 && r < nrounds)) {
                        if (pass == 1)
                            __syncthreads();  // one buffer: round r - 1 has been read
                        const int np = min(ppr, nplanes - r * ppr);
                        U *dst = win + (r & (nbuf - 1)) * bufU + wave * 64;
                        for (int k2 = 0; k2 < np; ++k2) {
                            const U *Gp = reinterpret_cast<const U *>(G0 + (long long)sb * a.G_stride) +
                                          (long long)stl * m2 * m1;
#pragma unroll
                            for (int k = 0; k < kOff; ++k)
                                if (wave * 64 + k * kThreads < units)
                                    __builtin_amdgcn_global_load_lds(
                                        reinterpret_cast<const void *>(Gp + off[k]),
                                        (__attribute__((address_space(3))) void *)(dst + k2 * planeP + k * kThreads), 16,
                                        0, 0);
                            if (++stl == qu) {
                                stl = 0;
                                ++sb;
                            }
                        }
                    }
                    if (pass == 1 || r == 0)
                        break;
                    // interpolate round r - 1; (b, tl, vb) stay uniform, so the
                    // accumulator of right-hand side vb is selected by scalar branches
                    const int np = min(ppr, nplanes - (r - 1) * ppr);
                    const U *src = win + ((r - 1) & (nbuf - 1)) * bufU + base;
                    for (int k2 = 0; k2 < np; ++k2) {
                        if (cb != vb) {
                            const cplx<T> mv = rotate_rhs<T>(mod, v);
                            FIO_ACC_ADD(acc, vb, mv);
                            v = cmake<T>(0, 0);
                            vb = cb;
                        }
                        const U *pw = src + k2 * planeP;
                        U sum;
                        if constexpr (CPU == 2)
                            sum = make_float4(0.f, 0.f, 0.f, 0.f);
                        else
                            sum = make_double2(0.0, 0.0);
                        // column by column (a window column is contiguous), one running pointer
                        if constexpr (k2D) {
                            const U *pc = pw;
#pragma unroll
                            for (int i2 = 0; i2 < W; ++i2, pc += S)
#pragma unroll
                                for (int i1 = 0; i1 < W; ++i1) {
                                    const U g = pc[i1];
                                    const T wk = w12[i1 * W + i2];
                                    sum.x += wk * g.x;
                                    sum.y += wk * g.y;
                                    if constexpr (CPU == 2) {
                                        sum.z += wk * g.z;
                                        sum.w += wk * g.w;
                                    }
                                }
                        } else {
                            const U *pc = pw;
#pragma unroll
                            for (int i2 = 0; i2 < W; ++i2, pc += S) {
                                U cs = pc[0];
                                cs.x *= w1[0];
                                cs.y *= w1[0];
                                if constexpr (CPU == 2) {
                                    cs.z *= w1[0];
                                    cs.w *= w1[0];
                                }
#pragma unroll
                                for (int i1 = 1; i1 < W; ++i1) {
                                    const U g = pc[i1];
                                    cs.x += w1[i1] * g.x;
                                    cs.y += w1[i1] * g.y;
                                    if constexpr (CPU == 2) {
                                        cs.z += w1[i1] * g.z;
                                        cs.w += w1[i1] * g.w;
                                    }
                                }
                                sum.x += w2[i2] * cs.x;
                                sum.y += w2[i2] * cs.y;
                                if constexpr (CPU == 2) {
                                    sum.z += w2[i2] * cs.z;
                                    sum.w += w2[i2] * cs.w;
                                }
                            }
                        }
                        const U gx = reinterpret_cast<const U *>(gxl)[ctl * kThreads + tid];
                        cfma4(v, cmake<T>(gx.x, gx.y), cmake<T>(sum.x, sum.y));
                        if constexpr (CPU == 2)
                            cfma4(v, cmake<T>(gx.z, gx.w), cmake<T>(sum.z, sum.w));
                        if (++ctl == qu) {
                            ctl = 0;
                            ++cb;
                        }
                    }
                }
                // this wave's copies have landed; after the barrier every wave's
                // have, and the buffer read in this round may be overwritten
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
            }
            {
                const cplx<T> mv = rotate_rhs<T>(mod, v);
                FIO_ACC_ADD(acc, vb, mv);
            }
        } else if (active) {
            // window too large for LDS (strongly folded warp): read the grid directly
            int g1i = j1 % m1, g2i = j2 % m2;
            if (g1i < 0)
                g1i += m1;
            if (g2i < 0)
                g2i += m2;
            for (int b = 0; b < B; ++b) {
                const cplx<T> *G = G0 + (long long)b * a.G_stride;
                cplx<T> v = cmake<T>(0, 0);
                for (int t = 0; t < q; ++t) {
                    cplx<T> sum = cmake<T>(0, 0);
#pragma unroll
                    for (int i1 = 0; i1 < W; ++i1) {
                        int r1 = g1i + i1;
                        if (r1 >= m1)
                            r1 -= m1;
                        cplx<T> rs = cmake<T>(0, 0);
#pragma unroll
                        for (int i2 = 0; i2 < W; ++i2) {
                            int r2 = g2i + i2;
                            if (r2 >= m2)
                                r2 -= m2;
                            const cplx<T> g = G[g_index<CPU>(r1, r2, t, m1, m2)];
                            rs.re += w2[i2] * g.re;
                            rs.im += w2[i2] * g.im;
                        }
                        sum.re += w1[i1] * rs.re;
                        sum.im += w1[i1] * rs.im;
                    }
                    cfma(v, REGEN ? gxl[((t / CPU) * kThreads + tid) * CPU + t % CPU] : gxp[t], sum);
                }
                const cplx<T> mv = rotate_rhs<T>(mod, v);
                FIO_ACC_ADD(acc, b, mv);
            }
        }
    }
    if (active && a.win_mode != kWinRecord) {
#pragma unroll
        for (int b = 0; b < kInterpBatch; ++b)
            if (b < B)
                u[b * ustride + p] = acc[b];
    }
}

// Occupancy targets of the FP32 interpolation: three waves per SIMD (168
// VGPRs, matching the three workgroups per CU that the window and gamma^x
// rows fit in LDS) for widths up to 6, two for wider stencils, whose planes
// need more registers, and one fewer when gamma^x is regenerated.  The cap
// also keeps the compiler from hoisting whole stencil planes into registers.
// FP64 keeps the compiler's choice, which it needs to avoid spills.
template <typename T, int W, bool REGEN>
constexpr int kInterpWavesPerEU =
    sizeof(T) == 4 ? (W <= 5 ? 3 : (W == 6 ? 3 : 2)) - (REGEN ? 1 : 0) : 1;
template <typename T, int W, bool REGEN>
constexpr int kInterpWavesPerEUMax = sizeof(T) == 4 ? kInterpWavesPerEU<T, W, REGEN> : 2;

template <typename T, int W, bool REGEN>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kInterpWavesPerEU<T, W, REGEN>, kInterpWavesPerEUMax<T, W, REGEN>))) void k_interp(
    PlanArgs<T> a, cplx<T> *__restrict__ u, long long ustride, int B, int bofs, int l0, int l1) {
    const int tiles = (a.N + kTileX - 1) / kTileX;
    interp_body<T, W, REGEN>(a, u, ustride, B, bofs, l0, l1,
                             chunked_tile(xcd_slot(blockIdx.x, gridDim.x), tiles));
}

template <typename T, int W, bool REGEN>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kInterpWavesPerEU<T, W, REGEN>, kInterpWavesPerEUMax<T, W, REGEN>))) void k_interp_multi(
    const InstArgs<T> *__restrict__ inst, const MultiTile *__restrict__ tiles) {
    // the table interleaves one stream of tiles per die (slot i runs on die
    // i % kXcds); padding entries have no right-hand sides
    const MultiTile m = tiles[blockIdx.x];
    if (m.nb == 0)
        return;
    const InstArgs<T> I = load_inst(inst, m.inst);
    interp_body<T, W, REGEN>(I.a, I.u + (long long)m.b0 * I.a.N * I.a.N, (long long)I.a.N * I.a.N, m.nb, m.b0, 0,
                             I.a.L, m.tile);
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
template <typename T>
PlanArgs<T> make_args(const fio_plan_s *P) {
    PlanArgs<T> a;
    a.phase = P->phase;
    a.N = P->N;
    a.L = P->L;
    a.w = P->w;
    a.qmax = P->qmax;
    a.beta = (T)P->beta;
    a.two_over_w = (T)(2.0 / P->w);
    a.wedges = P->d_wedges;
    a.fftplans = P->d_fftplans;
    a.map = P->d_map;
    a.omega = P->d_omega;
    a.gxi = static_cast<const cplx<T> *>(P->d_gxi);
    a.gx = static_cast<const cplx<T> *>(P->d_gx);
    a.tw = static_cast<const cplx<T> *>(P->d_tw);
    a.H = static_cast<cplx<T> *>(P->d_H);
    a.G = static_cast<cplx<T> *>(P->d_G);
    a.H_stride = P->H_total;
    a.G_stride = P->G_total;
    a.zcol = static_cast<const double2 *>(P->d_zcol);
    a.zmat = static_cast<const double2 *>(P->d_zmat);
    a.zmat32 = static_cast<const float2 *>(P->d_zmat32);
    a.win = P->d_win;
    a.win_mode = P->d_win ? kWinUse : kWinCompute;
    return a;
}

template PlanArgs<float> make_args<float>(const fio_plan_s *P);
template PlanArgs<double> make_args<double>(const fio_plan_s *P);

// Dynamic LDS of the interpolation: the window buffers, plus gamma^x of the
// tile's points (kThreads x qmax complex; regenerated in FIO_FACTORS_REGEN,
// copied from the stored factors otherwise, when qmax is small enough).
template <typename T>
size_t interp_lds_bytes(int qmax) {
    return (size_t)interp_window_bytes<T>(qmax) + interp_gx_lds_bytes<T>(qmax);
}

template <typename T, int W>
static hipError_t launch_interp_w(const fio_plan_s *P, const PlanArgs<T> &a, cplx<T> *u, long long ustride, int B,
                                  int bofs, int l0, int l1, hipStream_t s) {
    const int tiles = (P->N + kTileX - 1) / kTileX;
    if (P->regen)
        k_interp<T, W, true><<<(unsigned)(tiles * tiles), kThreads, interp_lds_bytes<T>(P->qmax), s>>>(
            a, u, ustride, B, bofs, l0, l1);
    else
        k_interp<T, W, false><<<(unsigned)(tiles * tiles), kThreads, interp_lds_bytes<T>(P->qmax), s>>>(
            a, u, ustride, B, bofs, l0, l1);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_interp(const fio_plan_s *P, const PlanArgs<T> &a, cplx<T> *u, long long ustride, int B,
                                int bofs, int l0, int l1, hipStream_t s) {
    switch (P->w) {
    case 4: return launch_interp_w<T, 4>(P, a, u, ustride, B, bofs, l0, l1, s);
    case 5: return launch_interp_w<T, 5>(P, a, u, ustride, B, bofs, l0, l1, s);
    case 6: return launch_interp_w<T, 6>(P, a, u, ustride, B, bofs, l0, l1, s);
    case 7: return launch_interp_w<T, 7>(P, a, u, ustride, B, bofs, l0, l1, s);
    case 8: return launch_interp_w<T, 8>(P, a, u, ustride, B, bofs, l0, l1, s);
    case 10: return launch_interp_w<T, 10>(P, a, u, ustride, B, bofs, l0, l1, s);
    case 12: return launch_interp_w<T, 12>(P, a, u, ustride, B, bofs, l0, l1, s);
    case 14: return launch_interp_w<T, 14>(P, a, u, ustride, B, bofs, l0, l1, s);
    case 16: return launch_interp_w<T, 16>(P, a, u, ustride, B, bofs, l0, l1, s);
    default: return hipErrorInvalidValue;
    }
}

// Event pair around one stage launch when the plan is profiling.
struct StageTimer {
    fio_plan_s *P;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(fio_plan_s *P_, int stage_, hipStream_t s_) : P(P_), stage(stage_), s(s_) {
        if (P && P->profiling && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, s);
    }
    ~StageTimer() {
        if (a && b) {
            (void)hipEventRecord(b, s);
            P->prof_events.push_back({stage, a, b});
        } else {
            if (a)
                (void)hipEventDestroy(a);
            if (b)
                (void)hipEventDestroy(b);
        }
    }
};

// One apply of B right-hand sides over wedges [l0, l1).  The row-stage output
// H and the grids G live in the plan's workspace, or, when `ws` is given, in
// the caller-provided device region ws (wsb bytes): H of `chunk` right-hand
// sides, then G of as many at the next 256-byte boundary, where chunk is what
// fits (at most the plan's batch chunk).  Every cell of H and G is written
// before it is read, so the region needs no clearing.  No events are created
// on the ws path.
template <typename T>
static hipError_t apply_t(fio_plan_s *P, int B, const void *fhat, void *u, hipStream_t s, int l0, int l1,
                          void *ws = nullptr, size_t wsb = 0) {
    PlanArgs<T> a = make_args<T>(P);
    int chunk = P->bchunk;
    if (ws) {
        const long long per = (long long)sizeof(cplx<T>) * (P->H_total + P->G_total);
        chunk = (int)std::min<long long>(P->bchunk, per > 0 ? (long long)(wsb - 256) / per : P->bchunk);
        if (chunk < 1)
            return hipErrorInvalidValue;
        const size_t hb = ((size_t)sizeof(cplx<T>) * P->H_total * chunk + 255) & ~size_t(255);
        a.H = static_cast<cplx<T> *>(ws);
        a.G = reinterpret_cast<cplx<T> *>(static_cast<unsigned char *>(ws) + hb);
    }
    const bool timed = ws == nullptr;
    const long long NN = (long long)P->N * P->N;
    const cplx<T> *f = static_cast<const cplx<T> *>(fhat);
    cplx<T> *out = static_cast<cplx<T> *>(u);
    const int r0 = P->row_first[l0], r1 = P->row_first[l1];
    const int c0 = P->col_first[l0], c1 = P->col_first[l1];
    for (int b0 = 0; b0 < B; b0 += chunk) {
        const int bc = std::min(chunk, B - b0);
        if (r1 > r0) {
            StageTimer tm(timed ? P : nullptr, 0, s);
            k_rows<T><<<r1 - r0, kFftThreads, P->lds_rows, s>>>(a, P->d_rows + r0, f + b0 * NN, NN, bc);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
        if (c1 > c0) {
            StageTimer tm(timed ? P : nullptr, 1, s);
            k_cols<T><<<dim3(c1 - c0, bc), kColThreads, P->lds_cols, s>>>(a, P->d_cols + c0);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
        for (int bs = 0; bs < bc; bs += kInterpBatch) {
            const int nb = std::min(kInterpBatch, bc - bs);
            StageTimer tm(timed ? P : nullptr, 2, s);
            hipError_t e = launch_interp<T>(P, a, out + (b0 + bs) * NN, NN, nb, bs, l0, l1, s);
            if (e != hipSuccess)
                return e;
        }
    }
    return hipSuccess;
}

template <typename T, int... Ws>
static hipError_t set_interp_lds_limits() {
    hipError_t e = hipSuccess;
    // the window plus up to kThreads x kGxLdsMaxRank complex of gamma^x
    ((e = e != hipSuccess ? e
                          : hipFuncSetAttribute(reinterpret_cast<const void *>(&k_interp<T, Ws, true>),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes)),
     ...);
    ((e = e != hipSuccess ? e
                          : hipFuncSetAttribute(reinterpret_cast<const void *>(&k_interp_multi<T, Ws, true>),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes)),
     ...);
    ((e = e != hipSuccess ? e
                          : hipFuncSetAttribute(reinterpret_cast<const void *>(&k_interp<T, Ws, false>),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes)),
     ...);
    ((e = e != hipSuccess ? e
                          : hipFuncSetAttribute(reinterpret_cast<const void *>(&k_interp_multi<T, Ws, false>),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes)),
     ...);
    return e;
}

template <typename T>
static hipError_t set_lds_limits() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rows<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
    if (e != hipSuccess)
        return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_cols<T>), hipFuncAttributeMaxDynamicSharedMemorySize,
                            kMaxLdsBytes);
    if (e != hipSuccess)
        return e;
    return set_interp_lds_limits<T, 4, 5, 6, 7, 8, 10, 12, 14, 16>();
}

__global__ void k_zero(unsigned long long *__restrict__ p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

hipError_t zero_fill(void *ptr, size_t bytes, hipStream_t s) {
    const long long n = (long long)(bytes / 8);
    const unsigned grid = (unsigned)std::min<long long>(4096, (n + kThreads - 1) / kThreads);
    if (n > 0)
        k_zero<<<std::max(1u, grid), kThreads, 0, s>>>(static_cast<unsigned long long *>(ptr), n);
    return hipGetLastError();
}

template <typename T, int W>
static void launch_multi_w(const MultiLaunch &ml, hipStream_t s, bool interp_only = false) {
    const InstArgs<T> *I = static_cast<const InstArgs<T> *>(ml.inst);
    if (interp_only) {
        if (ml.regen)
            k_interp_multi<T, W, true><<<ml.ntiles, kThreads, ml.lds_interp, s>>>(I, ml.tiles);
        else
            k_interp_multi<T, W, false><<<ml.ntiles, kThreads, ml.lds_interp, s>>>(I, ml.tiles);
        return;
    }
    if (ml.nrows)
        k_rows_multi<T><<<ml.nrows, kFftThreads, ml.lds_rows, s>>>(I, ml.rows);
    if (ml.ncols)
        k_cols_multi<T><<<ml.ncols, kColThreads, ml.lds_cols, s>>>(I, ml.cols);
    if (ml.ntiles) {
        if (ml.regen)
            k_interp_multi<T, W, true><<<ml.ntiles, kThreads, ml.lds_interp, s>>>(I, ml.tiles);
        else
            k_interp_multi<T, W, false><<<ml.ntiles, kThreads, ml.lds_interp, s>>>(I, ml.tiles);
    }
}

template <typename T>
static hipError_t launch_multi_t(const MultiLaunch &ml, hipStream_t s, bool interp_only) {
    switch (ml.w) {
    case 4: launch_multi_w<T, 4>(ml, s, interp_only); break;
    case 5: launch_multi_w<T, 5>(ml, s, interp_only); break;
    case 6: launch_multi_w<T, 6>(ml, s, interp_only); break;
    case 7: launch_multi_w<T, 7>(ml, s, interp_only); break;
    case 8: launch_multi_w<T, 8>(ml, s, interp_only); break;
    case 10: launch_multi_w<T, 10>(ml, s, interp_only); break;
    case 12: launch_multi_w<T, 12>(ml, s, interp_only); break;
    case 14: launch_multi_w<T, 14>(ml, s, interp_only); break;
    case 16: launch_multi_w<T, 16>(ml, s, interp_only); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t multi_launch(const MultiLaunch &ml, hipStream_t s) {
    return ml.precision == FIO_F64 ? launch_multi_t<double>(ml, s, false) : launch_multi_t<float>(ml, s, false);
}

hipError_t multi_record_windows(const MultiLaunch &ml, hipStream_t s) {
    if (!ml.ntiles)
        return hipSuccess;
    return ml.precision == FIO_F64 ? launch_multi_t<double>(ml, s, true) : launch_multi_t<float>(ml, s, true);
}

template <typename T>
static void fill_inst_t(const fio_plan_s *P, const void *fhat, void *u, int B, WinRec *win, int win_mode, void *out) {
    InstArgs<T> I;
    I.a = make_args<T>(P);
    // the fused kernel is another compilation of the interpolation (of the
    // widest width of the launch), so it records and reads windows of its own
    I.a.win = win;
    I.a.win_mode = win ? win_mode : kWinCompute;
    I.fhat = static_cast<const cplx<T> *>(fhat);
    I.u = static_cast<cplx<T> *>(u);
    I.B = B;
    std::memcpy(out, &I, sizeof(I));
}

size_t inst_args_size(int precision) {
    return precision == FIO_F64 ? sizeof(InstArgs<double>) : sizeof(InstArgs<float>);
}

void fill_inst_args(const fio_plan_s *P, const void *fhat, void *u, int B, WinRec *win, int win_mode, void *out) {
    if (P->precision == FIO_F64)
        fill_inst_t<double>(P, fhat, u, B, win, win_mode, out);
    else
        fill_inst_t<float>(P, fhat, u, B, win, win_mode, out);
}

template <typename T>
static hipError_t set_lds_limits_multi() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rows_multi<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
    if (e != hipSuccess)
        return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_cols_multi<T>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
}

// Record every tile's window on every wedge with the plan's own
// interpolation kernel (a launch without right-hand sides).  Without the
// table (it takes 32 bytes per tile and wedge) the kernel finds the windows
// in every apply.
template <typename T>
static hipError_t record_windows(fio_plan_s *P) {
    if (P->d_win) {
        (void)hipFree(P->d_win);
        P->d_win = nullptr;
    }
    const long long tiles = (P->N + kTileX - 1) / kTileX;
    if (hipMalloc(&P->d_win, sizeof(WinRec) * (size_t)(tiles * tiles * P->L)) != hipSuccess) {
        (void)hipGetLastError();
        P->d_win = nullptr;
        return hipSuccess;
    }
    PlanArgs<T> a = make_args<T>(P);
    a.win_mode = kWinRecord;
    hipError_t e = launch_interp<T>(P, a, nullptr, 0, 0, 0, 0, P->L, 0);
    if (e == hipSuccess)
        e = hipStreamSynchronize(0);
    if (e != hipSuccess) {
        (void)hipFree(P->d_win);
        P->d_win = nullptr;
    }
    return e;
}

hipError_t apply_prepare(fio_plan_s *P) {
    hipError_t e = P->precision == FIO_F64 ? set_lds_limits<double>() : set_lds_limits<float>();
    if (e == hipSuccess)
        e = P->precision == FIO_F64 ? set_lds_limits_multi<double>() : set_lds_limits_multi<float>();
    if (e == hipSuccess)
        e = P->precision == FIO_F64 ? record_windows<double>(P) : record_windows<float>(P);
    return e;
}

hipError_t apply_launch(fio_plan_s *P, int B, const void *fhat, void *u, hipStream_t s, int l0, int l1) {
    if (P->precision == FIO_F64)
        return apply_t<double>(P, B, fhat, u, s, l0, l1);
    return apply_t<float>(P, B, fhat, u, s, l0, l1);
}

// ---------------------------------------------------------------------------
// The apply without allocation.  Its H and G live in `scratch`, a fixed
// device array of this file (one copy per device, held until the process
// ends).  In host code `scratch` names a host-side stand-in, so kernels get
// its device address from hipGetSymbolAddress, taken once per device with
// that device current and kept in scratch_ptr.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_address(int device, void **out) {
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!p)
            return hipErrorInvalidSymbol;
        scratch_ptr[device] = p;
    }
    *out = scratch_ptr[device];
    return hipSuccess;
}

long long scratch_bytes_per_rhs(const fio_plan_s *P) {
    return (long long)P->esize * (P->H_total + P->G_total);
}

hipError_t apply_launch_scratch(fio_plan_s *P, int B, const void *fhat, void *u, hipStream_t s) {
    void *ws = nullptr;
    const hipError_t e = scratch_address(P->device, &ws);
    if (e != hipSuccess)
        return e;
    if (P->precision == FIO_F64)
        return apply_t<double>(P, B, fhat, u, s, 0, P->L, ws, kScratchBytes);
    return apply_t<float>(P, B, fhat, u, s, 0, P->L, ws, kScratchBytes);
}

}  // namespace fio
