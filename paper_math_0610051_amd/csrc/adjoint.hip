// The adjoint operator (Section 3.5).  With the separated factors of the
// forward plan, the Fourier coefficients of L*g are
//
//   hhat(xi) = (1/N) sum_ell chi_ell(xi) sum_t conj(gamma^xi_{ell t}(xi))
//              sum_y exp(-2 pi i grad_xi Phi(y, xi_hat_ell) . xi) conj(gamma^x_{ell t}(y)) g(y),
//
// the inner sum a type-1 NUFFT (eq. of the adjoint algorithm, steps 1-3).
// The three stages below are the conjugate transposes of the forward stages,
// on the same sheared boxes, oversampled grids and kernel, so that the
// computed map is the exact adjoint of the computed forward map up to
// rounding:
//   k_spread    conj(gamma^x) conj(modulation) g spread onto each wedge's
//               oversampled grid with the ES weights (the transpose of the
//               interpolation), accumulated per tile in an LDS window and
//               added to the grid with global atomics;
//   k_cols_adj  FFT with the - sign along axis 1, keeping the box rows;
//   k_rows_adj  FFT with the - sign along axis 2, keeping the box columns,
//               then the sum over ranks with conj(gamma^xi) (1/N and the
//               kernel's deconvolution are folded into gamma^xi), written to
//               the wedge's members of hhat.
// The - sign transforms reuse the + sign Stockham passes through
// conj(DFT+(conj(x))).  The row-stage buffer H and the grids G of the plan's
// workspace hold the intermediate results, as in the forward apply.
#include <algorithm>
#include <cstring>

#include "adjoint.hpp"
#include "apply.hpp"
#include "interp_util.hpp"

namespace fio {

constexpr int kSpreadLdsBytes = 65536;  // LDS window of the spreading (planes of several ranks and RHS)

template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) {
    return cmake<T>(a.re, -a.im);
}

template <typename T>
__device__ __forceinline__ void lds_add(T *p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);  // ds_add_f32 / ds_add_f64
}

template <typename T>
__device__ __forceinline__ void global_add(T *p, T v) {
    unsafeAtomicAdd(p, v);  // hardware global_atomic_add_f32 / _f64
}

// ---------------------------------------------------------------------------
// Stage A1: spreading.  A workgroup owns a kTileX x kTileX tile of input
// points (one per thread) and loops over the wedges.  Per wedge the stencils
// of the tile cover a window of the oversampled grid (found as in the
// interpolation); rounds of planes (right-hand side b, rank t) of that window
// are accumulated in LDS and then added to G.  Windows too large for one
// plane of LDS or wider than the grid (strongly folded warps) are added to G
// directly.
// ---------------------------------------------------------------------------
template <typename T, int W, bool REGEN>
__global__ __launch_bounds__(kThreads) void k_spread(PlanArgs<T> a, const cplx<T> *__restrict__ g, long long gstride,
                                                     int B, int bofs, int l0, int l1) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *win = reinterpret_cast<cplx<T> *>(smem_raw);
    constexpr int kCells = kSpreadLdsBytes / (int)sizeof(cplx<T>);
    __shared__ double red[kThreads / 64][4];
    const int N = a.N;
    const int tiles = (N + kTileX - 1) / kTileX;
    const int tile = chunked_tile(xcd_slot(blockIdx.x, gridDim.x), tiles);
    const int T1 = (tile / tiles) * kTileX, T2 = (tile % tiles) * kTileX;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n1 = T1 + tid / kTileX, n2 = T2 + tid % kTileX;
    const bool active = n1 < N && n2 < N;
    const long long p = active ? (long long)n1 * N + n2 : 0;
    const double x1 = (double)n1 / N, x2 = (double)n2 / N;
    const XCoef c = phase_xcoef(a.phase, x1, x2);
    // this point's inputs, one per right-hand side
    cplx<T> gv[kInterpBatch];
#pragma unroll
    for (int b = 0; b < kInterpBatch; ++b)
        gv[b] = (active && b < B) ? g[b * gstride + p] : cmake<T>(0, 0);
    // regenerated gamma^x of the tile's points follows the window in LDS
    cplx<T> *gxl = reinterpret_cast<cplx<T> *>(smem_raw + kSpreadLdsBytes);
    for (int l = l0; l < l1; ++l) {
        const WedgeDev &wd = a.wedges[l];
        if (wd.q == 0)
            continue;
        const int m1 = wd.n1, m2 = wd.n2, q = wd.q;
        double g1, g2;
        phase_grad(a.phase, c, wd.e1, wd.e2, g1, g2);
        if constexpr (REGEN) {
            const double2 *zc = a.zcol + wd.zc_off;
            const double2 *zm = a.zmat + wd.zm_off;
            for (int t = 0; t < q; ++t)
                gxl[t * kThreads + tid] = cmake<T>(0, 0);
            for (int cc = 0; cc < wd.zrc; ++cc) {
                const double2 k = zc[cc];
                double cs2, sn2;
                residual_entry(a.phase, c, g1, g2, k.x, k.y, cs2, sn2);
                const double2 *zr = zm + (long long)cc * q;
                for (int t = 0; t < q; ++t) {
                    const double2 z = zr[t];
                    cplx<T> &o = gxl[t * kThreads + tid];
                    o.re += (T)(cs2 * z.x - sn2 * z.y);
                    o.im += (T)(cs2 * z.y + sn2 * z.x);
                }
            }
        }
        const double y1 = x1 + g1, y2 = x2 + g2;
        const double yp1 = wd.mt[0] * y1 + wd.mt[1] * y2;
        const double yp2 = wd.mt[2] * y1 + wd.mt[3] * y2;
        double psi = wd.cvec[0] * y1 + wd.cvec[1] * y2;
        psi -= rint(psi);
        T cs, sn;
        expi_t<T>(psi, cs, sn);
        const cplx<T> cmod = cmake<T>(cs, -sn);  // conj(exp(2 pi i psi))
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
        __syncthreads();  // red is rewritten by the next wedge
        const double k1 = floor(lo1), k2 = floor(lo2);
        double u1, u2, ue;
        const int j1 = stencil_origin<W>(m1, yp1, k1, u1), j2 = stencil_origin<W>(m2, yp2, k2, u2);
        const int J1 = stencil_origin<W>(m1, lo1, k1, ue), X1 = stencil_origin<W>(m1, hi1, k1, ue);
        const int J2 = stencil_origin<W>(m2, lo2, k2, ue), X2 = stencil_origin<W>(m2, hi2, k2, ue);
        const T f1 = (T)(u1 - j1), f2 = (T)(u2 - j2);
        T w1[W], w2[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            w1[i] = es_weight<T>(f1 - T(i), a.two_over_w, a.beta);
            w2[i] = es_weight<T>(f2 - T(i), a.two_over_w, a.beta);
        }
        const int F1 = X1 - J1 + W, F2 = X2 - J2 + W;
        const int cells = F1 * F2;
        const cplx<T> *gxp = a.gx + wd.gx_off + p * q;
        cplx<T> *G0 = a.G + (long long)bofs * a.G_stride + wd.G_off;
        // grid cell of window row rr / column cc: 0 <= r0 < m1 and rr < F1 <= m1,
        // so one wrap brings r0 + rr onto the grid (likewise for axis 2)
        const int r0 = J1 < 0 ? J1 + m1 : (J1 >= m1 ? J1 - m1 : J1);
        const int c0 = J2 < 0 ? J2 + m2 : (J2 >= m2 ? J2 - m2 : J2);
        const int nplanes = B * q;
        if (cells <= kCells && F1 <= m1 && F2 <= m2) {
            const int ppr = kCells / cells;  // planes per round
            const int base = (j1 - J1) * F2 + (j2 - J2);
            for (int p0 = 0; p0 < nplanes; p0 += ppr) {
                const int np = min(ppr, nplanes - p0);
                for (int e = tid; e < np * cells; e += kThreads)
                    win[e] = cmake<T>(0, 0);
                __syncthreads();
                if (active) {
                    for (int k = 0; k < np; ++k) {
                        const int pl = p0 + k, b = pl / q, t = pl - b * q;
                        const cplx<T> gx = REGEN ? gxl[t * kThreads + tid] : gxp[t];
                        cplx<T> bv = cmake<T>(0, 0);
#pragma unroll
                        for (int bb = 0; bb < kInterpBatch; ++bb)
                            if (bb == b)
                                bv = gv[bb];
                        const cplx<T> v = cmul(cconj(gx), cmul(cmod, bv));
                        cplx<T> *pw = win + k * cells + base;
#pragma unroll
                        for (int i1 = 0; i1 < W; ++i1) {
                            const T ar = w1[i1] * v.re, ai = w1[i1] * v.im;
#pragma unroll
                            for (int i2 = 0; i2 < W; ++i2) {
                                lds_add(&pw[i1 * F2 + i2].re, w2[i2] * ar);
                                lds_add(&pw[i1 * F2 + i2].im, w2[i2] * ai);
                            }
                        }
                    }
                }
                __syncthreads();
                for (int e = tid; e < np * cells; e += kThreads) {
                    const cplx<T> v = win[e];
                    if (v.re == T(0) && v.im == T(0))
                        continue;
                    const int k = e / cells, cell = e - k * cells;
                    const int pl = p0 + k, b = pl / q, t = pl - b * q;
                    const int rr = cell / F2, cc = cell - rr * F2;
                    int gr = r0 + rr, gc = c0 + cc;
                    if (gr >= m1)
                        gr -= m1;
                    if (gc >= m2)
                        gc -= m2;
                    cplx<T> *dst = G0 + (long long)b * a.G_stride + ((long long)gc * m1 + gr) * q + t;
                    global_add(&dst->re, v.re);
                    global_add(&dst->im, v.im);
                }
                __syncthreads();  // the window is cleared for the next round
            }
        } else if (active) {
            // window beyond LDS: add each stencil value to the grid directly
            int g1i = j1 % m1, g2i = j2 % m2;
            if (g1i < 0)
                g1i += m1;
            if (g2i < 0)
                g2i += m2;
            for (int pl = 0; pl < nplanes; ++pl) {
                const int b = pl / q, t = pl - b * q;
                const cplx<T> gx = REGEN ? gxl[t * kThreads + tid] : gxp[t];
                cplx<T> bv = cmake<T>(0, 0);
#pragma unroll
                for (int bb = 0; bb < kInterpBatch; ++bb)
                    if (bb == b)
                        bv = gv[bb];
                const cplx<T> v = cmul(cconj(gx), cmul(cmod, bv));
                cplx<T> *G = G0 + (long long)b * a.G_stride + t;
                for (int i1 = 0; i1 < W; ++i1) {
                    int rr = g1i + i1;
                    if (rr >= m1)
                        rr -= m1;
                    for (int i2 = 0; i2 < W; ++i2) {
                        int cc = g2i + i2;
                        if (cc >= m2)
                            cc -= m2;
                        const T wk = w1[i1] * w2[i2];
                        cplx<T> *dst = G + ((long long)cc * m1 + rr) * q;
                        global_add(&dst->re, wk * v.re);
                        global_add(&dst->im, wk * v.im);
                    }
                }
            }
        }
        if constexpr (REGEN)
            __syncthreads();  // gxl is rewritten by the next wedge
    }
}

// ---------------------------------------------------------------------------
// Stage A2: the transpose of the column stage.  Item (wedge, transforms
// tau0 .. tau0 + nb of tau = j2 q + t) of right-hand side b: the full column
// of G, an FFT with the - sign along axis 1 (length n1), and the B1 box rows
// j1 = lo1 + k1 (mod n1) written to H in the forward stage's plane-major
// layout.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kColThreads) void k_cols_adj(PlanArgs<T> a, const ColItem *__restrict__ items) {
    constexpr int E = kColLdsBytes / (int)sizeof(cplx<T>) / kColThreads;
    constexpr int CPU = 16 / (int)sizeof(cplx<T>);
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
    const ColItem it = items[blockIdx.x];
    const int b = blockIdx.y;
    const WedgeDev &W = a.wedges[it.l];
    const int n = W.n1, nb = it.nb, B1 = W.B1, lo1 = W.lo1, q = W.q, qu = q / CPU;
    const int tid = threadIdx.x, nt = blockDim.x;
    const FftPlan *pl = a.fftplans + W.fft1;
    cplx<T> *twl = buf + n * nb;
    for (int i = tid; i < n; i += nt)
        twl[i] = a.tw[W.tw1 + i];
    const FastDiv &fnb = it.fnb, &fq = W.fq;
    const cplx<T> *G = a.G + (long long)b * a.G_stride + W.G_off;
    cplx<T> *H = a.H + (long long)b * a.H_stride + W.H_off;
    for (int i = tid; i < n * nb; i += nt) {
        const int j1 = fnb.div(i), cc = i - j1 * nb;
        const int tau = it.tau0 + cc, j2 = fq.div(tau), t = tau - j2 * q;
        buf[i] = cconj(G[((long long)j2 * n + j1) * q + t]);
    }
    __syncthreads();
    fft_inplace<T, E>(buf, pl, n, nb, fnb, twl, tid, nt, 0);
    for (int i = tid; i < B1 * nb; i += nt) {
        const int k1 = fnb.div(i), cc = i - k1 * nb;
        const int tau = it.tau0 + cc, j2 = fq.div(tau), t = tau - j2 * q;
        int j1 = lo1 + k1;
        if (j1 < 0)
            j1 += n;
        H[((long long)(j2 * qu + t / CPU) * B1 + k1) * CPU + t % CPU] = cconj(buf[j1 * nb + cc]);
    }
}

// ---------------------------------------------------------------------------
// Stage A3: the transpose of the row stage.  Item (wedge, box rows k1 .. k1 +
// nr, ranks t0 .. t0 + tn) of right-hand side b: the rows of H, an FFT with
// the - sign along axis 2 (length n2), and for every member xi of the wedge
// in these rows the sum over the item's ranks of conj(gamma^xi) times the
// box column j2 = lo2 + k2 (mod n2).  An item holding all ranks writes hhat
// directly; a rank chunk adds its share atomically (hhat is then cleared
// first).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_rows_adj(PlanArgs<T> a, const RowItem *__restrict__ items,
                                                         cplx<T> *__restrict__ hhat, long long hstride) {
    constexpr int E = kRowLdsBytes / (int)sizeof(cplx<T>) / kFftThreads;
    constexpr int CPU = 16 / (int)sizeof(cplx<T>);
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *buf = reinterpret_cast<cplx<T> *>(smem_raw);
    const RowItem it = items[blockIdx.x];
    const int b = blockIdx.y;
    const WedgeDev &W = a.wedges[it.l];
    const int n = W.n2, nr = it.nr, tn = it.tn, nbt = nr * tn, q = W.q, qu = q / CPU, B1 = W.B1, B2 = W.B2,
              lo2 = W.lo2;
    const int tid = threadIdx.x, nt = blockDim.x;
    const FftPlan *pl = a.fftplans + W.fft2;
    cplx<T> *twl = buf + n * nbt;
    for (int i = tid; i < n; i += nt)
        twl[i] = a.tw[W.tw2 + i];
    const cplx<T> *H = a.H + (long long)b * a.H_stride + W.H_off;
    for (int i = tid; i < n * nbt; i += nt) {
        const int j2 = it.fnbt.div(i), cc = i - j2 * nbt, r = it.ftn.div(cc), t = it.t0 + cc - r * tn;
        buf[i] = cconj(H[((long long)(j2 * qu + t / CPU) * B1 + it.k1 + r) * CPU + t % CPU]);
    }
    __syncthreads();
    fft_inplace<T, E>(buf, pl, n, nbt, it.fnbt, twl, tid, nt, 0);
    const int *map = a.map + W.map_off + (long long)it.k1 * B2;
    const int *omega = a.omega + W.mem_off;
    const cplx<T> *gxi = a.gxi + W.gxi_off + it.t0;
    const bool whole = it.t0 == 0 && tn == q;
    cplx<T> *hb = hhat + (long long)b * hstride;
    for (int i = tid; i < nr * B2; i += nt) {
        const int r = W.fB2.div(i), k2 = i - r * B2;
        const int m = map[r * B2 + k2];
        if (m < 0)
            continue;
        int j2 = lo2 + k2;
        if (j2 < 0)
            j2 += n;
        const cplx<T> *row = buf + j2 * nbt + r * tn;
        cplx<T> s = cmake<T>(0, 0);
        for (int t = 0; t < tn; ++t)
            cfma(s, cconj(gxi[(long long)m * q + t]), cconj(row[t]));
        cplx<T> *dst = hb + omega[m];
        if (whole) {
            *dst = s;
        } else {
            global_add(&dst->re, s.re);
            global_add(&dst->im, s.im);
        }
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
template <typename T, int W>
static hipError_t launch_spread_w(const fio_plan_s *P, const PlanArgs<T> &a, const cplx<T> *g, long long gstride,
                                  int B, int bofs, hipStream_t s) {
    const int tiles = (P->N + kTileX - 1) / kTileX;
    const size_t lds = kSpreadLdsBytes + (P->regen ? (size_t)kThreads * P->qmax * sizeof(cplx<T>) : 0);
    if (P->regen)
        k_spread<T, W, true><<<(unsigned)(tiles * tiles), kThreads, lds, s>>>(a, g, gstride, B, bofs, 0, P->L);
    else
        k_spread<T, W, false><<<(unsigned)(tiles * tiles), kThreads, lds, s>>>(a, g, gstride, B, bofs, 0, P->L);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_spread(const fio_plan_s *P, const PlanArgs<T> &a, const cplx<T> *g, long long gstride,
                                int B, int bofs, hipStream_t s) {
    switch (P->w) {
    case 4: return launch_spread_w<T, 4>(P, a, g, gstride, B, bofs, s);
    case 5: return launch_spread_w<T, 5>(P, a, g, gstride, B, bofs, s);
    case 6: return launch_spread_w<T, 6>(P, a, g, gstride, B, bofs, s);
    case 7: return launch_spread_w<T, 7>(P, a, g, gstride, B, bofs, s);
    case 8: return launch_spread_w<T, 8>(P, a, g, gstride, B, bofs, s);
    case 10: return launch_spread_w<T, 10>(P, a, g, gstride, B, bofs, s);
    case 12: return launch_spread_w<T, 12>(P, a, g, gstride, B, bofs, s);
    case 14: return launch_spread_w<T, 14>(P, a, g, gstride, B, bofs, s);
    case 16: return launch_spread_w<T, 16>(P, a, g, gstride, B, bofs, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int... Ws>
static hipError_t set_spread_lds_limits() {
    hipError_t e = hipSuccess;
    ((e = e != hipSuccess ? e
                          : hipFuncSetAttribute(reinterpret_cast<const void *>(&k_spread<T, Ws, false>),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes)),
     ...);
    ((e = e != hipSuccess ? e
                          : hipFuncSetAttribute(reinterpret_cast<const void *>(&k_spread<T, Ws, true>),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes)),
     ...);
    if (e != hipSuccess)
        return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_cols_adj<T>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
    if (e != hipSuccess)
        return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rows_adj<T>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
}

hipError_t adjoint_prepare(fio_plan_s *P) {
    return P->precision == FIO_F64 ? set_spread_lds_limits<double, 4, 5, 6, 7, 8, 10, 12, 14, 16>()
                                   : set_spread_lds_limits<float, 4, 5, 6, 7, 8, 10, 12, 14, 16>();
}

template <typename T>
static hipError_t adjoint_t(fio_plan_s *P, int B, const void *g, void *hhat, hipStream_t s) {
    const PlanArgs<T> a = make_args<T>(P);
    const long long NN = (long long)P->N * P->N;
    const cplx<T> *gin = static_cast<const cplx<T> *>(g);
    cplx<T> *out = static_cast<cplx<T> *>(hhat);
    bool partial = false;  // a row item holding a rank chunk adds into hhat
    for (const RowItem &r : P->rows)
        partial = partial || r.t0 != 0 || r.tn != P->wedges[r.l].qpad;
    // members of wedges of rank 0 receive nothing: clear hhat unless every
    // member is written by exactly one row item
    bool all_ranked = true;
    for (const WedgeHost &Wh : P->wedges)
        all_ranked = all_ranked && (Wh.members.empty() || Wh.qpad > 0);
    hipError_t e = hipSuccess;
    if (partial || !all_ranked) {
        e = zero_fill(out, sizeof(cplx<T>) * NN * B, s);
        if (e != hipSuccess)
            return e;
    }
    for (int b0 = 0; b0 < B; b0 += P->bchunk) {
        const int bc = std::min(P->bchunk, B - b0);
        e = zero_fill(P->d_G, sizeof(cplx<T>) * P->G_total * bc, s);
        if (e != hipSuccess)
            return e;
        for (int bs = 0; bs < bc; bs += kInterpBatch) {
            const int nb = std::min(kInterpBatch, bc - bs);
            e = launch_spread<T>(P, a, gin + (b0 + bs) * NN, NN, nb, bs, s);
            if (e != hipSuccess)
                return e;
        }
        if (!P->cols.empty()) {
            k_cols_adj<T><<<dim3((unsigned)P->cols.size(), bc), kColThreads, P->lds_cols, s>>>(a, P->d_cols);
            if ((e = hipGetLastError()) != hipSuccess)
                return e;
        }
        if (!P->rows.empty()) {
            k_rows_adj<T><<<dim3((unsigned)P->rows.size(), bc), kFftThreads, P->lds_rows, s>>>(a, P->d_rows,
                                                                                             out + b0 * NN, NN);
            if ((e = hipGetLastError()) != hipSuccess)
                return e;
        }
    }
    return hipSuccess;
}

hipError_t adjoint_launch(fio_plan_s *P, int B, const void *g, void *hhat, hipStream_t s) {
    if (!P->adjoint_ready) {
        const hipError_t e = adjoint_prepare(P);
        if (e != hipSuccess)
            return e;
        P->adjoint_ready = true;
    }
    return P->precision == FIO_F64 ? adjoint_t<double>(P, B, g, hhat, s) : adjoint_t<float>(P, B, g, hhat, s);
}

}  // namespace fio
