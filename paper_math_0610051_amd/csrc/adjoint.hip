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
//               interpolation), gathered per block of grid cells from the
//               grid points whose stencils touch the block (lists built once
//               per plan) and accumulated in LDS;
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
#include <type_traits>

#include <rocprim/device/device_segmented_radix_sort.hpp>

#include "adjoint.hpp"
#include "apply.hpp"
#include "errors.hpp"
#include "interp_util.hpp"

namespace fio {


template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) {
    return cmake<T>(a.re, -a.im);
}

template <typename T>
__device__ __forceinline__ void global_add(T *p, T v) {
    unsafeAtomicAdd(p, v);  // hardware global_atomic_add_f32 / _f64
}

// ---------------------------------------------------------------------------
// Stage A1: spreading, gathered per strip of the oversampled grid.  Each
// wedge's grid is cut into strips of kStripRows<T> x kStripCols cells; at the
// first adjoint apply every grid point x is listed in the strips its w x w
// stencil touches (a point's warp and stencil do not depend on the input).
// One wave owns one strip and keeps its cells in registers: lane k carries
// plane k (RHS b, rank t) of every cell, and for each listed point it adds
// conj(gamma^x_t(x)) conj(exp(2 pi i psi(x))) g_b(x) times the ES weight of
// each tap row and column that falls in the strip (zero elsewhere).  The
// FP64 warp, stencil and weights of 64 listed points are formed lane-parallel
// and broadcast with readlane, and the next point's factor and input values
// are fetched while the current one is added.  Every grid cell belongs to
// exactly one strip, which writes it once: the grids need no clearing, and
// neither LDS nor global atomics are involved.
// ---------------------------------------------------------------------------
template <typename T>
constexpr int kStripRows = 4;  // cells along the long grid axis (1)
constexpr int kStripCols = 8;  // cells along the short grid axis (2)
constexpr int kSpreadLanes = 64;                     // planes per round: one per lane
constexpr int kSpreadMaxB = 16;                      // right-hand sides per round

// Warped point of x in wedge W, its stencil's first cell on each axis
// wrapped into [0, m), and the fractions f = u - j of the unwrapped grid
// coordinate u = m (y' - k).  The integer reference k is the one the
// interpolation uses for x's output tile (the floor of the tile's smallest
// coordinate, tabulated per tile and wedge), and u, j and f are formed with
// the interpolation's own arithmetic, so that every point spreads with
// exactly the stencil cells and weights it is interpolated with.
struct SpreadPoint {
    int j1, j2;
    double f1, f2;
    double y1, y2;
};
__device__ inline double warp_coord(const WedgeDev &wd, int axis, double y1, double y2) {
    return axis == 0 ? wd.mt[0] * y1 + wd.mt[1] * y2 : wd.mt[2] * y1 + wd.mt[3] * y2;
}
__device__ inline int origin_rt(double m, double y, double k, int W, double &u) {
#pragma clang fp contract(off)
    u = m * (y - k);
    return (int)floor(u - 0.5 * W) + 1;
}
__device__ inline SpreadPoint spread_point(const Phase &ph, const WedgeDev &wd, double x1, double x2, const XCoef &c,
                                           int W, int2 ref, double &g1, double &g2) {
    phase_grad(ph, c, wd.e1, wd.e2, g1, g2);
    SpreadPoint s;
    s.y1 = x1 + g1;
    s.y2 = x2 + g2;
    const double yp1 = warp_coord(wd, 0, s.y1, s.y2), yp2 = warp_coord(wd, 1, s.y1, s.y2);
    double u1, u2;
    const int j1 = origin_rt(wd.n1, yp1, (double)ref.x, W, u1), j2 = origin_rt(wd.n2, yp2, (double)ref.y, W, u2);
    s.f1 = u1 - j1;
    s.f2 = u2 - j2;
    int a = j1 % wd.n1, b = j2 % wd.n2;
    s.j1 = a < 0 ? a + wd.n1 : a;
    s.j2 = b < 0 ? b + wd.n2 : b;
    return s;
}

// Integer reference of every output tile and wedge: the floor of the
// smallest warped coordinate over the tile's points on each axis, as the
// interpolation forms its window (block-wide minimum).
__global__ __launch_bounds__(kThreads) void k_adj_tileref(Phase ph, int N, const WedgeDev *__restrict__ wedges,
                                                          int2 *__restrict__ ref) {
    __shared__ double red[kThreads / 64][2];
    const int tiles = (N + kTileX - 1) / kTileX;
    const int tile = blockIdx.x, l = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n1 = (tile / tiles) * kTileX + tid / kTileX, n2 = (tile % tiles) * kTileX + tid % kTileX;
    const bool active = n1 < N && n2 < N;
    const WedgeDev &wd = wedges[l];
    const double x1 = (double)n1 / N, x2 = (double)n2 / N;
    const XCoef c = phase_xcoef(ph, x1, x2);
    double g1, g2;
    phase_grad(ph, c, wd.e1, wd.e2, g1, g2);
    const double y1 = x1 + g1, y2 = x2 + g2;
    const double yp1 = warp_coord(wd, 0, y1, y2), yp2 = warp_coord(wd, 1, y1, y2);
    const double mn1 = wave_min(active ? yp1 : DBL_MAX), mn2 = wave_min(active ? yp2 : DBL_MAX);
    if (lane == 0) {
        red[wave][0] = mn1;
        red[wave][1] = mn2;
    }
    __syncthreads();
    if (tid == 0) {
        double lo1 = red[0][0], lo2 = red[0][1];
        for (int k = 1; k < kThreads / 64; ++k) {
            lo1 = fmin(lo1, red[k][0]);
            lo2 = fmin(lo2, red[k][1]);
        }
        ref[(long long)l * tiles * tiles + tile] = make_int2((int)floor(lo1), (int)floor(lo2));
    }
}

__device__ inline int2 tile_ref(const int2 *ref, int N, int l, int n1, int n2) {
    const int tiles = (N + kTileX - 1) / kTileX;
    return ref[(long long)l * tiles * tiles + (n1 / kTileX) * tiles + n2 / kTileX];
}

// Distinct strips (at most w per axis) that the w cells j, j+1, ... (mod m) touch.
__device__ inline int stencil_bins(int j, int W, int m, int bb, int *bins) {
    int n = 0, last = -1;
    for (int i = 0; i < W; ++i) {
        int c = j + i;
        if (c >= m)
            c -= m;
        const int b = c / bb;
        if (b != last) {
            bins[n++] = b;
            last = b;
        }
    }
    return n;
}

// Bin builder, pass 0 counts and pass 1 fills: thread = (grid point, wedge).
__global__ void k_adj_bins(Phase ph, int N, const WedgeDev *__restrict__ wedges, int W, const int2 *__restrict__ ref,
                           int bb1, int bb2, const long long *__restrict__ wbase, const int *__restrict__ nb2, int pass,
                           unsigned *__restrict__ counter, const long long *__restrict__ off, int *__restrict__ pts) {
    const long long NN = (long long)N * N;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (p >= NN)
        return;
    const WedgeDev &wd = wedges[l];
    if (wd.q == 0)
        return;
    const int n1 = (int)(p / N), n2 = (int)(p % N);
    const double x1 = (double)n1 / N, x2 = (double)n2 / N;
    const XCoef c = phase_xcoef(ph, x1, x2);
    double g1, g2;
    const SpreadPoint sp = spread_point(ph, wd, x1, x2, c, W, tile_ref(ref, N, l, n1, n2), g1, g2);
    int b1[16], b2[16];
    const int k1 = stencil_bins(sp.j1, W, wd.n1, bb1, b1), k2 = stencil_bins(sp.j2, W, wd.n2, bb2, b2);
    for (int a = 0; a < k1; ++a)
        for (int b = 0; b < k2; ++b) {
            const long long bin = wbase[l] + (long long)b1[a] * nb2[l] + b2[b];
            const unsigned slot = atomicAdd(&counter[bin], 1u);
            if (pass == 1)
                pts[off[bin] + slot] = (int)p;
        }
}

__device__ __forceinline__ int lane_bcast(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ __forceinline__ float lane_bcast(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ double lane_bcast(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), k), hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <typename T, int W, bool REGEN>
__global__ __launch_bounds__(kThreads) void k_spread(PlanArgs<T> a, const AdjBin *__restrict__ bins, int nbins,
                                                     const int *__restrict__ pts, const int2 *__restrict__ ref,
                                                     const cplx<T> *__restrict__ g, long long gstride, int B,
                                                     int bofs, int qstage) {
    constexpr int R = kStripRows<T>, C = kStripCols;
    constexpr int CPU = 16 / (int)sizeof(cplx<T>);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int bi = blockIdx.x * (kThreads / 64) + wave;
    if (bi >= nbins)
        return;  // waves are independent: no barrier below
    extern __shared__ unsigned char smem_raw[];
    // FIO_FACTORS_REGEN: gamma^x of the wave's 64 staged points, [point][rank]
    cplx<T> *sgx = reinterpret_cast<cplx<T> *>(smem_raw) + (size_t)wave * 64 * qstage;
    const AdjBin bin = bins[bi];
    const WedgeDev &wd = a.wedges[bin.l];
    const int N = a.N, m1 = wd.n1, m2 = wd.n2, q = wd.q;
    cplx<T> *G0 = a.G + (long long)bofs * a.G_stride + wd.G_off;
    const cplx<T> *gx0 = a.gx + wd.gx_off;
    for (int t0 = 0; t0 < q; t0 += kSpreadLanes) {
        const int tn = min(kSpreadLanes, q - t0);
        const int bmax = min(kSpreadMaxB, kSpreadLanes / tn);
        for (int b0 = 0; b0 < B; b0 += bmax) {
            const int nb = min(bmax, B - b0);
            // this lane's plane: RHS b0 + bl, rank t0 + tl (lanes past nb tn compute a copy of a live plane)
            const int bl = min(lane / tn, nb - 1), tl = lane % tn;
            const cplx<T> *gb = g + (long long)(b0 + bl) * gstride;
            cplx<T> acc[R][C];
#pragma unroll
            for (int j = 0; j < R; ++j)
#pragma unroll
                for (int c = 0; c < C; ++c)
                    acc[j][c] = cmake<T>(0, 0);
            for (int kb = 0; kb < bin.n; kb += 64) {
                const int nbt = min(64, bin.n - kb);
                // lane i forms the record of listed point kb + i
                int p = 0, r0 = 0;
                T wr[R], wc[C];
                cplx<T> md = cmake<T>(0, 0);
#pragma unroll
                for (int j = 0; j < R; ++j)
                    wr[j] = T(0);
#pragma unroll
                for (int c = 0; c < C; ++c)
                    wc[c] = T(0);
                if (lane < nbt) {
                    p = pts[bin.off + kb + lane];
                    const int n1 = p / N, n2 = p - n1 * N;
                    const double x1 = (double)n1 / N, x2 = (double)n2 / N;
                    const XCoef c = phase_xcoef(a.phase, x1, x2);
                    double g1, g2;
                    const SpreadPoint sp =
                        spread_point(a.phase, wd, x1, x2, c, W, tile_ref(ref, N, bin.l, n1, n2), g1, g2);
                    double psi = wd.cvec[0] * sp.y1 + wd.cvec[1] * sp.y2;
                    psi -= rint(psi);
                    T cs, sn;
                    expi_t<T>(psi, cs, sn);
                    md = cmake<T>(cs, -sn);
                    // first stencil cell relative to the strip, wrapped next to it
                    r0 = sp.j1 - bin.o1;
                    int c0 = sp.j2 - bin.o2;
                    if (r0 < -W)
                        r0 += m1;
                    else if (r0 >= R)
                        r0 -= m1;
                    if (c0 < -W)
                        c0 += m2;
                    else if (c0 >= C)
                        c0 -= m2;
                    const T f1 = (T)sp.f1, f2 = (T)sp.f2;
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        const int k = j - r0;
                        wr[j] = k >= 0 && k < W ? es_weight<T>(f1 - T(k), a.two_over_w, a.beta) : T(0);
                    }
#pragma unroll
                    for (int cc = 0; cc < C; ++cc) {
                        const int k = cc - c0;
                        wc[cc] = k >= 0 && k < W ? es_weight<T>(f2 - T(k), a.two_over_w, a.beta) : T(0);
                    }
                    if constexpr (REGEN && sizeof(T) == 4) {  // as the interpolation regenerates it
                        auto put = [&](auto kq) {
                            constexpr int K = decltype(kq)::value;
                            float ar[K], ai[K];
                            regen_sums_f32<K>(a.phase, c, g1, g2, a.zcol + wd.zc_off, a.zmat32 + wd.zm_off, wd.zrc,
                                              q, ar, ai);
#pragma unroll
                            for (int t = 0; t < K; ++t)
                                if (t < q)
                                    sgx[lane * qstage + t] = cmake<T>(ar[t], ai[t]);
                        };
                        if (q <= 8)
                            put(std::integral_constant<int, 8>());
                        else
                            put(std::integral_constant<int, kRegenMaxRank>());
                    }
                    if constexpr (REGEN && sizeof(T) == 8) {  // q <= kRegenMaxRank: one round of ranks
                        const double2 *zc = a.zcol + wd.zc_off;
                        const double2 *zm = a.zmat + wd.zm_off;
                        double ar[kRegenMaxRank], ai[kRegenMaxRank];
#pragma unroll
                        for (int t = 0; t < kRegenMaxRank; ++t)
                            ar[t] = ai[t] = 0;
                        for (int cc = 0; cc < wd.zrc; ++cc) {
                            const double2 kk = zc[cc];
                            double cs2, sn2;
                            residual_entry(a.phase, c, g1, g2, kk.x, kk.y, cs2, sn2);
                            const double2 *zr = zm + (long long)cc * q;
#pragma unroll
                            for (int t = 0; t < kRegenMaxRank; ++t)
                                if (t < q) {
                                    const double2 z = zr[t];
                                    ar[t] += cs2 * z.x - sn2 * z.y;
                                    ai[t] += cs2 * z.y + sn2 * z.x;
                                }
                        }
#pragma unroll
                        for (int t = 0; t < kRegenMaxRank; ++t)
                            if (t < q)
                                sgx[lane * qstage + t] = cmake<T>((T)ar[t], (T)ai[t]);
                    }
                }
                if constexpr (REGEN)
                    __builtin_amdgcn_wave_barrier();  // the wave's LDS writes precede its reads (in-order LDS)
                // point k of the batch: its factor and input values are loaded one point ahead
                auto fetch = [&](int k, cplx<T> &x, cplx<T> &y) {
                    const int pk = lane_bcast(p, k);
                    if constexpr (REGEN)
                        x = sgx[k * qstage + t0 + tl];
                    else
                        x = gx0[(long long)pk * q + t0 + tl];
                    y = gb[pk];
                };
                cplx<T> nx, ny;
                fetch(0, nx, ny);
                for (int k = 0; k < nbt; ++k) {
                    const cplx<T> cx = nx, cy = ny;
                    if (k + 1 < nbt)
                        fetch(k + 1, nx, ny);
                    const int rk = lane_bcast(r0, k);
                    const cplx<T> mk = cmake<T>(lane_bcast(md.re, k), lane_bcast(md.im, k));
                    const cplx<T> v = cmul(cconj(cx), cmul(mk, cy));
                    T wcol[C];
#pragma unroll
                    for (int cc = 0; cc < C; ++cc)
                        wcol[cc] = lane_bcast(wc[cc], k);
#pragma unroll
                    for (int j = 0; j < R; ++j)
                        if (j - rk >= 0 && j - rk < W) {  // a tap row of the point (uniform branch)
                            const T w = lane_bcast(wr[j], k);
                            const T ar = w * v.re, ai = w * v.im;
#pragma unroll
                            for (int cc = 0; cc < C; ++cc) {
                                acc[j][cc].re += wcol[cc] * ar;
                                acc[j][cc].im += wcol[cc] * ai;
                            }
                        }
                }
            }
            // the strip's cells (G is plane-major, g_index)
            if (lane < nb * tn) {
#pragma unroll
                for (int cc = 0; cc < C; ++cc) {
                    const int gc = bin.o2 + cc;
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        const int gr = bin.o1 + j;
                        if (gr < m1 && gc < m2)
                            G0[(long long)(b0 + bl) * a.G_stride + g_index<CPU>(gr, gc, t0 + tl, m1, m2)] =
                                acc[j][cc];
                    }
                }
            }
        }
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
        buf[i] = cconj(G[g_index<CPU>(j1, j2, t, n, W.n2)]);
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
                                  int B, hipStream_t s) {
    const unsigned grid = (unsigned)((P->n_adj_bins + kThreads / 64 - 1) / (kThreads / 64));
    if (P->regen) {
        const int qstage = P->qmax;
        const size_t lds = (size_t)(kThreads / 64) * 64 * qstage * sizeof(cplx<T>);
        if (lds > (size_t)kMaxLdsBytes)
            return hipErrorInvalidConfiguration;
        k_spread<T, W, true><<<grid, kThreads, lds, s>>>(a, P->d_adj_bins, P->n_adj_bins, P->d_adj_pts, P->d_adj_ref,
                                                        g, gstride, B, 0, qstage);
    } else {
        k_spread<T, W, false><<<grid, kThreads, 0, s>>>(a, P->d_adj_bins, P->n_adj_bins, P->d_adj_pts,
                                                       P->d_adj_ref, g, gstride, B, 0, 0);
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_spread(const fio_plan_s *P, const PlanArgs<T> &a, const cplx<T> *g, long long gstride,
                                int B, hipStream_t s) {
    switch (P->w) {
    case 4: return launch_spread_w<T, 4>(P, a, g, gstride, B, s);
    case 5: return launch_spread_w<T, 5>(P, a, g, gstride, B, s);
    case 6: return launch_spread_w<T, 6>(P, a, g, gstride, B, s);
    case 7: return launch_spread_w<T, 7>(P, a, g, gstride, B, s);
    case 8: return launch_spread_w<T, 8>(P, a, g, gstride, B, s);
    case 10: return launch_spread_w<T, 10>(P, a, g, gstride, B, s);
    case 12: return launch_spread_w<T, 12>(P, a, g, gstride, B, s);
    case 14: return launch_spread_w<T, 14>(P, a, g, gstride, B, s);
    case 16: return launch_spread_w<T, 16>(P, a, g, gstride, B, s);
    default: return hipErrorInvalidValue;
    }
}

// The spreading blocks of every wedge and their point lists (two passes of
// k_adj_bins: counts, then the lists at their exclusive prefix offsets).
static fio_status build_adj_bins(fio_plan_s *P) {
    const int L = P->L, N = P->N;
    const int bb1 = P->precision == FIO_F64 ? kStripRows<double> : kStripRows<float>, bb2 = kStripCols;
    const long long NN = (long long)N * N;
    std::vector<long long> wbase(L + 1, 0);
    std::vector<int> nb1(L, 0), nb2(L, 0);
    for (int l = 0; l < L; ++l) {
        const WedgeDev &wd = P->wdev[l];
        if (wd.q > 0) {
            nb1[l] = (wd.n1 + bb1 - 1) / bb1;
            nb2[l] = (wd.n2 + bb2 - 1) / bb2;
        }
        wbase[l + 1] = wbase[l] + (long long)nb1[l] * nb2[l];
    }
    const long long nbins = wbase[L];
    struct Tmp {
        std::vector<void *> p;
        ~Tmp() {
            for (void *v : p)
                if (v)
                    (void)hipFree(v);
        }
    } tmp;
    long long *d_wbase = nullptr, *d_off = nullptr;
    int *d_nb2 = nullptr;
    unsigned *d_cnt = nullptr;
    FIO_HIP_TRY(hipMalloc(&d_wbase, sizeof(long long) * (L + 1)));
    tmp.p.push_back(d_wbase);
    FIO_HIP_TRY(hipMalloc(&d_nb2, sizeof(int) * L));
    tmp.p.push_back(d_nb2);
    FIO_HIP_TRY(hipMalloc(&d_cnt, sizeof(unsigned) * std::max<long long>(1, nbins)));
    tmp.p.push_back(d_cnt);
    FIO_HIP_TRY(hipMalloc(&d_off, sizeof(long long) * std::max<long long>(1, nbins)));
    tmp.p.push_back(d_off);
    FIO_HIP_TRY(hipMemcpy(d_wbase, wbase.data(), sizeof(long long) * (L + 1), hipMemcpyHostToDevice));
    FIO_HIP_TRY(hipMemcpy(d_nb2, nb2.data(), sizeof(int) * L, hipMemcpyHostToDevice));
    const int tiles = (N + kTileX - 1) / kTileX;
    FIO_HIP_TRY(hipMalloc(&P->d_adj_ref, sizeof(int2) * (size_t)L * tiles * tiles));
    k_adj_tileref<<<dim3((unsigned)(tiles * tiles), (unsigned)L), kThreads>>>(P->phase, N, P->d_wedges,
                                                                               P->d_adj_ref);
    FIO_HIP_TRY(hipGetLastError());
    const dim3 grid((unsigned)((NN + 255) / 256), (unsigned)L);
    FIO_HIP_TRY(hipMemset(d_cnt, 0, sizeof(unsigned) * std::max<long long>(1, nbins)));
    k_adj_bins<<<grid, 256>>>(P->phase, N, P->d_wedges, P->w, P->d_adj_ref, bb1, bb2, d_wbase, d_nb2, 0, d_cnt,
                              nullptr, nullptr);
    FIO_HIP_TRY(hipGetLastError());
    std::vector<unsigned> cnt(nbins);
    FIO_HIP_TRY(hipMemcpy(cnt.data(), d_cnt, sizeof(unsigned) * nbins, hipMemcpyDeviceToHost));
    std::vector<long long> off(nbins);
    long long total = 0;
    for (long long i = 0; i < nbins; ++i) {
        off[i] = total;
        total += cnt[i];
    }
    std::vector<AdjBin> bins(nbins);
    for (int l = 0; l < L; ++l)
        for (int b1 = 0; b1 < nb1[l]; ++b1)
            for (int b2 = 0; b2 < nb2[l]; ++b2) {
                const long long i = wbase[l] + (long long)b1 * nb2[l] + b2;
                bins[i] = AdjBin{l, b1 * bb1, b2 * bb2, (int)cnt[i], off[i]};
            }
    FIO_HIP_TRY(hipMalloc(&P->d_adj_pts, sizeof(int) * std::max<long long>(1, total)));
    FIO_HIP_TRY(hipMalloc(&P->d_adj_bins, sizeof(AdjBin) * std::max<long long>(1, nbins)));
    FIO_HIP_TRY(hipMemcpy(P->d_adj_bins, bins.data(), sizeof(AdjBin) * nbins, hipMemcpyHostToDevice));
    FIO_HIP_TRY(hipMemcpy(d_off, off.data(), sizeof(long long) * nbins, hipMemcpyHostToDevice));
    FIO_HIP_TRY(hipMemset(d_cnt, 0, sizeof(unsigned) * std::max<long long>(1, nbins)));
    k_adj_bins<<<grid, 256>>>(P->phase, N, P->d_wedges, P->w, P->d_adj_ref, bb1, bb2, d_wbase, d_nb2, 1, d_cnt,
                              d_off, P->d_adj_pts);
    FIO_HIP_TRY(hipGetLastError());
    // Every list in point order (the fill above takes atomic slots): the
    // spreading then sums each cell in a fixed order, so adjoint applies are
    // reproducible bit for bit, and it walks gamma^x and g in memory order.
    if (total > 1 && total < (1ll << 32) && nbins < (1ll << 32)) {
        std::vector<unsigned> off32(nbins + 1);
        for (long long i = 0; i < nbins; ++i)
            off32[i] = (unsigned)off[i];
        off32[nbins] = (unsigned)total;
        unsigned *d_off32 = nullptr;
        int *sorted = nullptr;
        void *work = nullptr;
        FIO_HIP_TRY(hipMalloc(&d_off32, sizeof(unsigned) * (nbins + 1)));
        tmp.p.push_back(d_off32);
        FIO_HIP_TRY(hipMemcpy(d_off32, off32.data(), sizeof(unsigned) * (nbins + 1), hipMemcpyHostToDevice));
        FIO_HIP_TRY(hipMalloc(&sorted, sizeof(int) * total));
        tmp.p.push_back(sorted);
        const size_t slot = tmp.p.size() - 1;
        unsigned bits = 1;
        while ((1ll << bits) < NN)
            ++bits;
        size_t work_bytes = 0;
        FIO_HIP_TRY(rocprim::segmented_radix_sort_keys(nullptr, work_bytes, P->d_adj_pts, sorted, (unsigned)total,
                                                       (unsigned)nbins, d_off32, d_off32 + 1, 0, bits));
        FIO_HIP_TRY(hipMalloc(&work, std::max<size_t>(work_bytes, 1)));
        tmp.p.push_back(work);
        FIO_HIP_TRY(rocprim::segmented_radix_sort_keys(work, work_bytes, P->d_adj_pts, sorted, (unsigned)total,
                                                       (unsigned)nbins, d_off32, d_off32 + 1, 0, bits));
        FIO_HIP_TRY(hipDeviceSynchronize());
        tmp.p[slot] = P->d_adj_pts;  // the unsorted lists are freed with the temporaries
        P->d_adj_pts = sorted;
    }
    FIO_HIP_TRY(hipDeviceSynchronize());
    P->n_adj_bins = (int)nbins;
    P->n_adj_pts = total;
    return FIO_OK;
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
        if (P->n_adj_bins > 0) {
            e = launch_spread<T>(P, a, gin + b0 * NN, NN, bc, s);
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

fio_status adjoint_launch(fio_plan_s *P, int B, const void *g, void *hhat, hipStream_t s) {
    if (!P->adjoint_ready) {
        FIO_HIP_TRY(adjoint_prepare(P));
        const fio_status st = build_adj_bins(P);
        if (st != FIO_OK)
            return st;
        P->adjoint_ready = true;
    }
    FIO_HIP_TRY(P->precision == FIO_F64 ? adjoint_t<double>(P, B, g, hhat, s) : adjoint_t<float>(P, B, g, hhat, s));
    return FIO_OK;
}

}  // namespace fio
