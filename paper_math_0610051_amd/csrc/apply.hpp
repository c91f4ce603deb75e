// Internal interface between the plan builder and the apply kernels.
#pragma once

#include <algorithm>

#include "plan.hpp"

namespace fio {

constexpr int kThreads = 256;       // workgroup size of every apply kernel
constexpr int kInterpBatch = 4;     // right-hand sides per interpolation launch
constexpr int kMaxLdsBytes = 131072;  // two ping-pong FFT buffers per workgroup
constexpr int kInterpWidths[] = {4, 5, 6, 7, 8, 10, 12, 14, 16};

hipError_t apply_prepare(fio_plan_s *P);
// Zero `bytes` (a multiple of 8) with a fill kernel on stream s (no memset node).
hipError_t zero_fill(void *ptr, size_t bytes, hipStream_t s);
hipError_t apply_launch(fio_plan_s *P, int B, const void *fhat, void *u, hipStream_t s, int l0, int l1);

}  // namespace fio
