// Internal interface between the plan builder and the apply kernels.
#pragma once

#include <algorithm>

#include "plan.hpp"

namespace fio {

constexpr int kThreads = 256;       // workgroup size of every apply kernel
constexpr int kInterpBatch = 8;     // right-hand sides per interpolation launch
constexpr int kTileX = 16;          // interpolation tile: kTileX x kTileX output points per workgroup
constexpr int kRegenMaxRank = 16;      // padded rank bound of FIO_FACTORS_REGEN (FP32; half in FP64)
constexpr int kInterpLdsBytes = 38912;  // LDS windows (rank planes of several right-hand sides) per interpolation workgroup: four per CU
constexpr int kMaxLdsBytes = 131072;  // largest dynamic LDS request of any apply kernel
constexpr int kFftThreads = 512;     // workgroup size of the two FFT stages
constexpr int kFftWavesPerEU = 4;    // register budget: two FFT workgroups per CU overlap load, transform and store
constexpr int kRowLdsBytes = 32768;   // in-place FFT buffer of a row-stage workgroup
constexpr int kColLdsBytes = 32768;   // in-place FFT buffer of a column-stage workgroup
constexpr int kColThreads = 512;      // workgroup size of the column stage
constexpr int kInterpWidths[] = {4, 5, 6, 7, 8, 10, 12, 14, 16};

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
size_t inst_args_size(int precision);
void fill_inst_args(const fio_plan_s *P, const void *fhat, void *u, int B, void *out);

hipError_t apply_prepare(fio_plan_s *P);
// Zero `bytes` (a multiple of 8) with a fill kernel on stream s (no memset node).
hipError_t zero_fill(void *ptr, size_t bytes, hipStream_t s);
hipError_t apply_launch(fio_plan_s *P, int B, const void *fhat, void *u, hipStream_t s, int l0, int l1);

}  // namespace fio
