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
#include "apply.hpp"

namespace fio {

// ---------------------------------------------------------------------------
// Stage 1: window x factor -> box row, FFT along axis 2 (length n2).
// One workgroup per (wedge, box row, rank chunk); loops over the batch.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_rows(PlanArgs<T> a, const RowItem *__restrict__ items,
                                                   const cplx<T> *__restrict__ fhat, long long fstride, int B) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *buf0 = reinterpret_cast<cplx<T> *>(smem_raw);
    const RowItem it = items[blockIdx.x];
    const WedgeDev &W = a.wedges[it.l];
    const int n = W.n2, nb = it.tn, q = W.q, B2 = W.B2, lo2 = W.lo2;
    const int tid = threadIdx.x, nt = blockDim.x;
    cplx<T> *buf1 = buf0 + n * nb;
    const FftPlan *pl = a.fftplans + W.fft2;
    const int npass = pl->npass;
    const cplx<T> *tw = a.tw + W.tw2;
    const int *map = a.map + W.map_off + (long long)it.k1 * B2;
    const int *omega = a.omega + W.mem_off;
    const cplx<T> *gxi = a.gxi + W.gxi_off + it.t0;
    for (int b = 0; b < B; ++b) {
        for (int i = tid; i < n * nb; i += nt)
            buf0[i] = cmake<T>(0, 0);
        __syncthreads();
        const cplx<T> *f = fhat + b * fstride;
        for (int i = tid; i < B2 * nb; i += nt) {
            const int k2 = i / nb, t = i - k2 * nb;
            const int m = map[k2];
            if (m >= 0) {
                int j2 = lo2 + k2;
                if (j2 < 0)
                    j2 += n;
                buf0[j2 * nb + t] = cmul(f[omega[m]], gxi[(long long)m * q + t]);
            }
        }
        __syncthreads();
        cplx<T> *src = buf0, *dst = buf1;
        int Ns = 1;
        for (int p = 0; p < npass; ++p) {
            const int R = pl->radix[p];
            stockham_pass<T>(R, src, dst, n, nb, Ns, tw, tid, nt);
            __syncthreads();
            cplx<T> *tmp = src;
            src = dst;
            dst = tmp;
            Ns *= R;
        }
        cplx<T> *H = a.H + b * a.H_stride + W.H_off + (long long)it.k1 * n * q + it.t0;
        for (int i = tid; i < n * nb; i += nt) {
            const int j2 = i / nb, t = i - j2 * nb;
            H[(long long)j2 * q + t] = src[i];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Stage 2: FFT along axis 1 (length n1) of nb adjacent transforms
// tau = j2 * q + t; rows outside the box are the implicit zero padding.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cols(PlanArgs<T> a, const ColItem *__restrict__ items) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *buf0 = reinterpret_cast<cplx<T> *>(smem_raw);
    const ColItem it = items[blockIdx.x];
    const int b = blockIdx.y;
    const WedgeDev &W = a.wedges[it.l];
    const int n = W.n1, nb = it.nb, B1 = W.B1, lo1 = W.lo1;
    const long long rs = (long long)W.n2 * W.q;  // row stride of H and G
    const int tid = threadIdx.x, nt = blockDim.x;
    cplx<T> *buf1 = buf0 + n * nb;
    const FftPlan *pl = a.fftplans + W.fft1;
    const int npass = pl->npass;
    const cplx<T> *tw = a.tw + W.tw1;
    for (int i = tid; i < n * nb; i += nt)
        buf0[i] = cmake<T>(0, 0);
    __syncthreads();
    const cplx<T> *H = a.H + b * a.H_stride + W.H_off + it.tau0;
    for (int i = tid; i < B1 * nb; i += nt) {
        const int k1 = i / nb, c = i - k1 * nb;
        int j1 = lo1 + k1;
        if (j1 < 0)
            j1 += n;
        buf0[j1 * nb + c] = H[k1 * rs + c];
    }
    __syncthreads();
    cplx<T> *src = buf0, *dst = buf1;
    int Ns = 1;
    for (int p = 0; p < npass; ++p) {
        const int R = pl->radix[p];
        stockham_pass<T>(R, src, dst, n, nb, Ns, tw, tid, nt);
        __syncthreads();
        cplx<T> *tmp = src;
        src = dst;
        dst = tmp;
        Ns *= R;
    }
    cplx<T> *G = a.G + b * a.G_stride + W.G_off + it.tau0;
    for (int i = tid; i < n * nb; i += nt) {
        const int j1 = i / nb, c = i - j1 * nb;
        G[j1 * rs + c] = src[i];
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

// ---------------------------------------------------------------------------
// Stage 3: interpolate + modulate + combine over t + accumulate over ell.
// One thread per output point x; up to 4 right-hand sides per launch share
// the warped point, kernel weights and gamma^x.  W is the kernel width,
// QC the rank chunk held in registers.
// ---------------------------------------------------------------------------
template <typename T, int W, int QC>
__global__ __launch_bounds__(kThreads) void k_interp(PlanArgs<T> a, cplx<T> *__restrict__ u, long long ustride,
                                                     int B, int bofs, int l0, int l1) {
    const int N = a.N;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (long long)N * N)
        return;
    const int n1 = (int)(p / N), n2 = (int)(p - (long long)n1 * N);
    const double x1 = (double)n1 / N, x2 = (double)n2 / N;
    const XCoef c = phase_xcoef(a.phase, x1, x2);
    cplx<T> acc[kInterpBatch];
#pragma unroll
    for (int b = 0; b < kInterpBatch; ++b)
        acc[b] = cmake<T>(0, 0);
    for (int l = l0; l < l1; ++l) {
        const WedgeDev &wd = a.wedges[l];
        if (wd.q == 0)
            continue;
        double g1, g2;
        phase_grad(a.phase, c, wd.e1, wd.e2, g1, g2);
        const double y1 = x1 + g1, y2 = x2 + g2;
        const double yp1 = wd.mt[0] * y1 + wd.mt[1] * y2;
        const double yp2 = wd.mt[2] * y1 + wd.mt[3] * y2;
        double psi = wd.cvec[0] * y1 + wd.cvec[1] * y2;
        psi -= rint(psi);
        T cs, sn;
        expi_t<T>(psi, cs, sn);
        const int m1 = wd.n1, m2 = wd.n2, q = wd.q;
        const double u1 = m1 * (yp1 - floor(yp1));
        const double u2 = m2 * (yp2 - floor(yp2));
        int j1 = (int)floor(u1 - 0.5 * W) + 1;
        int j2 = (int)floor(u2 - 0.5 * W) + 1;
        const T f1 = (T)(u1 - j1), f2 = (T)(u2 - j2);
        T w2[W];
#pragma unroll
        for (int i = 0; i < W; ++i)
            w2[i] = es_kernel<T>(f2 - T(i), a.two_over_w, a.beta);
        if (j1 < 0)
            j1 += m1;
        if (j2 < 0)
            j2 += m2;
        const long long rs = (long long)m2 * q;
        const cplx<T> *gxp = a.gx + wd.gx_off + p * q;
        const cplx<T> mod = cmake(cs, sn);
        for (int b = 0; b < B; ++b) {
            const cplx<T> *G = a.G + (long long)(bofs + b) * a.G_stride + wd.G_off;
            cplx<T> v = cmake<T>(0, 0);
            for (int t0 = 0; t0 < q; t0 += QC) {
                cplx<T> s[QC];
#pragma unroll
                for (int t = 0; t < QC; ++t)
                    s[t] = cmake<T>(0, 0);
#pragma unroll 1
                for (int i1 = 0; i1 < W; ++i1) {
                    const T wa = es_kernel<T>(f1 - T(i1), a.two_over_w, a.beta);
                    int r1 = j1 + i1;
                    if (r1 >= m1)
                        r1 -= m1;
                    const cplx<T> *row = G + r1 * rs + t0;
#pragma unroll
                    for (int i2 = 0; i2 < W; ++i2) {
                        int r2 = j2 + i2;
                        if (r2 >= m2)
                            r2 -= m2;
                        const T wt = wa * w2[i2];
                        const cplx<T> *cell = row + (long long)r2 * q;
#pragma unroll
                        for (int t = 0; t < QC; ++t) {
                            if (t0 + t < q) {
                                const cplx<T> g = cell[t];
                                s[t].re += wt * g.re;
                                s[t].im += wt * g.im;
                            }
                        }
                    }
                }
#pragma unroll
                for (int t = 0; t < QC; ++t)
                    if (t0 + t < q)
                        cfma(v, gxp[t0 + t], s[t]);
            }
            const cplx<T> mv = cmul(mod, v);
#pragma unroll
            for (int bb = 0; bb < kInterpBatch; ++bb)
                if (bb == b) {
                    acc[bb].re += mv.re;
                    acc[bb].im += mv.im;
                }
        }
    }
#pragma unroll
    for (int b = 0; b < kInterpBatch; ++b)
        if (b < B)
            u[b * ustride + p] = acc[b];
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
    return a;
}

template <typename T, int W>
static hipError_t launch_interp_w(const fio_plan_s *P, const PlanArgs<T> &a, cplx<T> *u, long long ustride, int B,
                                  int bofs, int l0, int l1, hipStream_t s) {
    const long long npts = (long long)P->N * P->N;
    const unsigned grid = (unsigned)((npts + kThreads - 1) / kThreads);
    if (P->qmax <= 4)
        k_interp<T, W, 4><<<grid, kThreads, 0, s>>>(a, u, ustride, B, bofs, l0, l1);
    else if (P->qmax <= 8)
        k_interp<T, W, 8><<<grid, kThreads, 0, s>>>(a, u, ustride, B, bofs, l0, l1);
    else
        k_interp<T, W, 16><<<grid, kThreads, 0, s>>>(a, u, ustride, B, bofs, l0, l1);
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
        if (P->profiling && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
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

template <typename T>
static hipError_t apply_t(fio_plan_s *P, int B, const void *fhat, void *u, hipStream_t s, int l0, int l1) {
    const PlanArgs<T> a = make_args<T>(P);
    const long long NN = (long long)P->N * P->N;
    const cplx<T> *f = static_cast<const cplx<T> *>(fhat);
    cplx<T> *out = static_cast<cplx<T> *>(u);
    const int r0 = P->row_first[l0], r1 = P->row_first[l1];
    const int c0 = P->col_first[l0], c1 = P->col_first[l1];
    for (int b0 = 0; b0 < B; b0 += P->bchunk) {
        const int bc = std::min(P->bchunk, B - b0);
        if (r1 > r0) {
            StageTimer tm(P, 0, s);
            k_rows<T><<<r1 - r0, kThreads, P->lds_rows, s>>>(a, P->d_rows + r0, f + b0 * NN, NN, bc);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
        if (c1 > c0) {
            StageTimer tm(P, 1, s);
            k_cols<T><<<dim3(c1 - c0, bc), kThreads, P->lds_cols, s>>>(a, P->d_cols + c0);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
        for (int bs = 0; bs < bc; bs += kInterpBatch) {
            const int nb = std::min(kInterpBatch, bc - bs);
            StageTimer tm(P, 2, s);
            hipError_t e = launch_interp<T>(P, a, out + (b0 + bs) * NN, NN, nb, bs, l0, l1, s);
            if (e != hipSuccess)
                return e;
        }
    }
    return hipSuccess;
}

template <typename T>
static hipError_t set_lds_limits() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rows<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
    if (e != hipSuccess)
        return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_cols<T>), hipFuncAttributeMaxDynamicSharedMemorySize,
                               kMaxLdsBytes);
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

hipError_t apply_prepare(fio_plan_s *P) {
    return P->precision == FIO_F64 ? set_lds_limits<double>() : set_lds_limits<float>();
}

hipError_t apply_launch(fio_plan_s *P, int B, const void *fhat, void *u, hipStream_t s, int l0, int l1) {
    if (P->precision == FIO_F64)
        return apply_t<double>(P, B, fhat, u, s, l0, l1);
    return apply_t<float>(P, B, fhat, u, s, l0, l1);
}

}  // namespace fio
