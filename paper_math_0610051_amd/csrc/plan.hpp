// Internal plan structures of the FIO library (host side and the POD
// descriptors the kernels read).
#pragma once

#include <algorithm>
#include <complex>
#include <string>
#include <vector>

#include "../../include/fio.h"
#include "common.hpp"
#include "fft.hpp"

namespace fio {

using zd = std::complex<double>;

// Device-visible descriptor of one wedge W_ell and its NUFFT box (Section 3.4).
struct WedgeDev {
    double e1, e2;       // centre direction xi_hat_ell
    double mt[4];        // M^{-T} (row-major): y' = M^{-T} y
    double cvec[2];      // M^{-1} xi_c: modulation phase psi(x) = y . M^{-1} xi_c
    int n1, n2;          // oversampled grid
    int B1, B2;          // sheared, centred box
    int lo1, lo2;        // centred frequency of box index 0 (lo = -floor(B/2))
    int q;               // stored rank (even, zero-padded factors)
    int nmem;            // |W_ell|
    int tw1, tw2;        // twiddle-table offsets for lengths n1, n2
    int fft1, fft2;      // FFT plan indices for n1, n2
    int pad0, pad1;
    long long map_off;   // box map: int32 per box cell -> member index or -1
    long long mem_off;   // member tables: centred Omega index per member
    long long gxi_off;   // gamma^xi (deconvolved, 1/N folded in), nmem * q complex
    long long gx_off;    // gamma^x, N^2 * q complex
    long long H_off;     // per-RHS row-transformed box, plane-major [j2][plane][k1][rank in plane]: n2 * B1 * q complex
    long long G_off;     // per-RHS oversampled grid, plane-major [plane][j2][j1] (g_index): n2 * n1 * q complex
    FastDiv fq, fB1, fB2, fn1, fn2;  // dividers by q, B1, B2, n1, n2 (constants built on the host)
    long long zc_off;    // regenerated factors: sampled column frequencies (zrc of them)
    long long zm_off;    // and Z = V S^-1, zrc * q complex double (zero-padded ranks)
    int zrc, pad2;       // number of sampled columns (0 when gamma^x is stored)
};

// Position of element t of cell (j1, j2) in one wedge's oversampled grid G
// (one right-hand side).  G is plane-major: plane P = t / CPU (CPU complex
// per 16 bytes: a rank pair in FP32, one rank in FP64) holds the n2 columns
// of n1 cells as 16-byte units, so a window column of one plane is one
// contiguous run.
template <int CPU>
__host__ __device__ inline long long g_index(int j1, int j2, int t, int n1, int n2) {
    return (((long long)(t / CPU) * n2 + j2) * n1 + j1) * CPU + t % CPU;
}

// One block of an oversampled grid for the adjoint's spreading: wedge l,
// first cell (o1, o2), and its n points at pts[off ...].
struct AdjBin {
    int l, o1, o2, n;
    long long off;
};

// Work items of the two FFT stages.
struct RowItem {   // stage 1: box rows [k1, k1 + nr) of wedge ell, ranks [t0, t0 + tn)
    int l, k1, nr, t0, tn, pad;
    FastDiv ftn, fnbt, fnr, fnpl;  // dividers by tn, nr * tn, nr and the planes tn / cpu
};
struct ColItem {   // stage 2: transforms tau in [tau0, tau0 + nb) of wedge ell (tau = j2 * q + t, plane tau / cpu)
    int l, tau0, nb, pad;
    FastDiv fnb;        // divider by nb
};
inline RowItem make_row_item(int l, int k1, int nr, int t0, int tn, int cpu) {
    return RowItem{l,  k1, nr, t0, tn, 0, FastDiv((unsigned)tn), FastDiv((unsigned)(nr * tn)), FastDiv((unsigned)nr),
                   FastDiv((unsigned)std::max(1, tn / cpu))};
}
inline ColItem make_col_item(int l, int tau0, int nb) { return ColItem{l, tau0, nb, 0, FastDiv((unsigned)nb)}; }

// Kernel-side view of a plan (passed by value).
// Interpolation window of one tile on one wedge's grid: first stencil cell
// (J1, J2), extent F1 x F2, LDS column stride S >= F1 (16-byte units) and the
// integer reference (k1, k2) the tile's sheared coordinates are unwrapped
// around.
struct WinRec {
    int J1, J2, F1, F2, S, k1, k2, pad;
};
// How the interpolation finds its windows: from the tile's points (block
// reductions), the same and recorded in the plan's table, or read from it.
enum WinMode { kWinCompute = 0, kWinRecord = 1, kWinUse = 2 };

template <typename T>
struct PlanArgs {
    Phase phase;
    int N, L, w, qmax;
    T beta, two_over_w;
    const WedgeDev *wedges;
    const FftPlan *fftplans;
    const int *map;
    const int *omega;
    const cplx<T> *gxi;
    const cplx<T> *gx;
    const cplx<T> *tw;
    cplx<T> *H;
    cplx<T> *G;
    long long H_stride, G_stride;  // per right-hand side
    const double2 *zcol;           // regenerated factors (FIO_FACTORS_REGEN)
    const double2 *zmat;
    const float2 *zmat32;          // Z in FP32 (FP32 plans)
    WinRec *win;                   // [wedge][tile] windows (WinMode)
    int win_mode;
};

struct WedgeHost {
    double theta = 0;
    std::vector<int> members;   // centred Omega indices
    int M[4] = {1, 0, 0, 1}, Minv[4] = {1, 0, 0, 1};
    int xc[2] = {0, 0}, B[2] = {1, 1}, lo[2] = {0, 0}, n[2] = {2, 2}, fft[2] = {0, 0};
    int q = 0, qpad = 0, r = 0, attempts = 0;
    double sep_err = 0;
    std::vector<int> C;          // sampled member positions (columns)
    std::vector<long long> R;    // sampled grid rows
    std::vector<zd> Z;           // r x q, V S^-1 (row-major)
    std::vector<zd> P;           // q x r, U_[R]^+ (row-major)
    std::vector<double> dec1, dec2;  // 1 / phi_hat along each box axis
};

}  // namespace fio

struct fio_plan_s {
    unsigned long long serial = 0;  // unique per plan built in this process
    void *multi_state = nullptr;    // cached multi-instance launch owned by this plan
    int N = 0, L = 0, precision = FIO_F32, device = 0;
    fio::Phase phase{};
    double tol = 0;
    fio_options opt{};
    int w = 0;
    double sigma = 2.0, beta = 0;
    int qmax = 0;
    int fallback = 0, factor_mode = FIO_FACTORS_STORED;
    double plan_ms = 0;
    double learned_sep_err = 0, learned_ms = 0;  // the learned attempt, if any
    bool regen = false;                          // gamma^x recomputed in the apply
    void *d_zcol = nullptr, *d_zmat = nullptr, *d_zmat32 = nullptr;
    std::vector<fio::WedgeHost> wedges;
    std::vector<int> wedge_of;   // N*N, centred
    std::vector<fio::WedgeDev> wdev;
    std::vector<fio::RowItem> rows;
    std::vector<fio::ColItem> cols;
    std::vector<fio::FftPlan> fftplans;
    std::vector<int> fft_len;    // length of each fft plan
    std::vector<int> tw_off;     // twiddle offset per fft plan
    long long tw_total = 0;
    long long map_total = 0, mem_total = 0, gxi_total = 0, gx_total = 0, H_total = 0, G_total = 0;
    int bchunk = 8;
    size_t esize = 8;            // bytes of one complex element
    size_t lds_rows = 0, lds_cols = 0;  // dynamic LDS of the two FFT stages
    // device buffers
    fio::WedgeDev *d_wedges = nullptr;
    fio::FftPlan *d_fftplans = nullptr;
    fio::RowItem *d_rows = nullptr;
    fio::ColItem *d_cols = nullptr;
    int *d_map = nullptr, *d_omega = nullptr;
    void *d_gxi = nullptr, *d_gx = nullptr, *d_tw = nullptr, *d_H = nullptr, *d_G = nullptr;
    long long factor_bytes = 0, workspace_bytes = 0;
    // rows of the row/column work tables restricted to a wedge range are
    // found by scanning: rows and cols are sorted by wedge.
    std::vector<int> row_first, col_first;   // L+1 prefix offsets
    bool adjoint_ready = false;  // LDS limits of the adjoint kernels set, spreading bins built
    // Spreading bins of the adjoint: every wedge's oversampled grid cut into
    // blocks of cells, each with the grid points whose stencil
    // touches it (built at the first adjoint apply)
    fio::AdjBin *d_adj_bins = nullptr;
    int *d_adj_pts = nullptr;
    int2 *d_adj_ref = nullptr;  // integer reference of every output tile and wedge
    fio::WinRec *d_win = nullptr;  // interpolation window of every tile and wedge (recorded at plan time)
    int n_adj_bins = 0;
    long long n_adj_pts = 0;
    // optional per-stage event timing
    int profiling = 0;
    struct StageEvents {
        int stage;
        hipEvent_t start, stop;
    };
    std::vector<StageEvents> prof_events;
    double prof_ms[3] = {0, 0, 0};
    long long prof_launches[3] = {0, 0, 0};
};
