// Internal interface between the plan builder and the apply kernels.
#pragma once

#include <algorithm>

#include "plan.hpp"

namespace fio {

constexpr int kThreads = 256;       // workgroup size of every apply kernel
constexpr int kInterpBatch = 8;     // right-hand sides per interpolation launch
constexpr int kTileX = 16;          // interpolation tile: kTileX x kTileX output points per workgroup
constexpr int kRegenMaxRank = 16;      // padded rank bound of FIO_FACTORS_REGEN (FP32; half in FP64)
constexpr int kInterpLdsTarget = 53248;  // interpolation LDS (window + gamma^x) per workgroup: three per CU
constexpr int kInterpWindowMax = 36864;  // LDS window buffers (rank planes of several right-hand sides)
constexpr int kInterpWindowMin = 16384;
constexpr int kMaxLdsBytes = 131072;  // largest dynamic LDS request of any apply kernel
constexpr int kFftThreads = 512;     // workgroup size of the two FFT stages
constexpr int kFftWavesPerEU = 4;    // register budget of the row stage: two workgroups per CU overlap load, transform and store
constexpr int kColWavesPerEU = 6;    // at least three column-stage workgroups per CU
constexpr int kRowLdsBytes = 32768;   // in-place FFT buffer of a row-stage workgroup
constexpr int kColLdsBytes = 32768;   // in-place FFT buffer of a column-stage workgroup
constexpr int kColThreads = 512;      // workgroup size of the column stage
constexpr int kInterpWidths[] = {4, 5, 6, 7, 8, 10, 12, 14, 16};
// gamma^x of a workgroup's points (kThreads x padded rank complex, at most
// 96 KB) follows the window in LDS when the padded rank is at most this; plans
// of larger rank interpolate straight from global memory
template <typename T>
constexpr int kGxLdsMaxRank = sizeof(T) == 4 ? 48 : 24;
template <typename T>
__host__ __device__ inline int interp_gx_lds_bytes(int qmax) {
    return qmax <= kGxLdsMaxRank<T> ? kThreads * qmax * 2 * (int)sizeof(T) : 0;
}
// window bytes: what the target leaves beside gamma^x, within [min, max]
template <typename T>
__host__ __device__ inline int interp_window_bytes(int qmax) {
    const int w = kInterpLdsTarget - interp_gx_lds_bytes<T>(qmax);
    return w > kInterpWindowMax ? kInterpWindowMax : (w < kInterpWindowMin ? kInterpWindowMin : w / 1024 * 1024);
}
constexpr int kXcds = 8;              // accelerator dies; workgroup i of a launch runs on die i % kXcds
constexpr int kTileChunk = 8;         // interpolation tiles are walked in kTileChunk x kTileChunk squares

// Workgroup id -> position in a list of n work items such that each die runs
// one contiguous run of the list (die x gets items [x * n / 8 ...) in order).
__host__ __device__ inline int xcd_slot(int bid, int n) {
    const int q = n / kXcds, r = n % kXcds, x = bid % kXcds, s = bid / kXcds;
    return x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

// Position li in the walk of a tiles x tiles grid of interpolation tiles ->
// row-major tile index.  The walk covers bands of kTileChunk tile rows, each
// band square by square, each square row by row: tiles that run together on
// one die are neighbours in both directions, and the halos of their windows
// are read from that die's L2.
__host__ __device__ inline int chunked_tile(int li, int tiles) {
    const int band = li / (kTileChunk * tiles);
    const int hb = tiles - band * kTileChunk < kTileChunk ? tiles - band * kTileChunk : kTileChunk;
    const int rem = li - band * kTileChunk * tiles;
    const int c = rem / (hb * kTileChunk);
    const int rc = rem - c * hb * kTileChunk;
    const int wc = tiles - c * kTileChunk < kTileChunk ? tiles - c * kTileChunk : kTileChunk;
    const int row = rc / wc, col = rc - row * wc;
    return (band * kTileChunk + row) * tiles + c * kTileChunk + col;
}

// Per-instance arguments of the multi-instance kernels.
template <typename T>
struct InstArgs {
    PlanArgs<T> a;
    const cplx<T> *fhat;
    cplx<T> *u;
    int B;
};
struct MultiRowItem {
    int inst;
    RowItem it;
};
struct MultiColItem {  // one column item of one instance and right-hand side
    int inst, b;
    ColItem it;
};
struct MultiTile {
    int inst, tile, b0, nb;
};
// One fused launch per stage over every instance, wedge and right-hand side.
struct MultiLaunch {
    int precision = FIO_F32, w = 0;
    const void *inst = nullptr;  // device array of InstArgs<T>
    const MultiRowItem *rows = nullptr;
    const MultiColItem *cols = nullptr;
    const MultiTile *tiles = nullptr;
    unsigned nrows = 0, ncols = 0, ntiles = 0;
    size_t lds_rows = 0, lds_cols = 0;
    bool regen = false;          // FIO_FACTORS_REGEN plans (all instances alike)
    size_t lds_interp = 0;       // dynamic LDS of the interpolation launch
};
hipError_t multi_launch(const MultiLaunch &ml, hipStream_t s);
// The fused interpolation alone, its instances' arguments in record mode:
// fills each instance's window table (WinRec per tile and wedge).
hipError_t multi_record_windows(const MultiLaunch &ml, hipStream_t s);
size_t inst_args_size(int precision);
// win: the instance's window table for the fused kernel (nullptr: windows
// found in every launch), read or recorded as win_mode says.
void fill_inst_args(const fio_plan_s *P, const void *fhat, void *u, int B, WinRec *win, int win_mode, void *out);

hipError_t apply_prepare(fio_plan_s *P);
// Kernel-side view of a plan (instantiated for float and double).
template <typename T>
PlanArgs<T> make_args(const fio_plan_s *P);
// Zero `bytes` (a multiple of 8) with a fill kernel on stream s (no memset node).
hipError_t zero_fill(void *ptr, size_t bytes, hipStream_t s);
hipError_t apply_launch(fio_plan_s *P, int B, const void *fhat, void *u, hipStream_t s, int l0, int l1);

// The apply without allocation: H and G in a fixed device array of
// kScratchBytes per device instead of the plan's workspace.
constexpr size_t kScratchBytes = size_t(128) << 20;
long long scratch_bytes_per_rhs(const fio_plan_s *P);  // H + G of one right-hand side
hipError_t apply_launch_scratch(fio_plan_s *P, int B, const void *fhat, void *u, hipStream_t s);

}  // namespace fio
