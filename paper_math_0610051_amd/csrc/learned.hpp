// Learned spatial factors: a small network that maps (x, theta_ell, s) to the
// 16 complex spatial factors alpha_t(x) of wedge ell at phase scale s.
#pragma once

#include <vector>

#include "plan.hpp"

namespace fio {

constexpr int kNetIn = 16, kNetHidden = 128, kNetOut = 32, kNetRank = 16;
constexpr int kNetLayers = 4;
// layer i maps kNetDims[i] -> kNetDims[i + 1]
constexpr int kNetDims[kNetLayers + 1] = {kNetIn, kNetHidden, kNetHidden, kNetHidden, kNetOut};

struct LearnedModel {
    int N = 0, L = 0, device = 0;
    Phase family{};          // p0 is replaced by the scale input
    unsigned long long seed = 0;
    int nparams = 0;
    int offW[kNetLayers] = {}, offb[kNetLayers] = {};
    // device: FP32 master parameters (flat, W row-major [in][out] then b per layer),
    // Adam moments, BF16 copies of the weights, gradients
    float *d_p = nullptr, *d_m = nullptr, *d_v = nullptr, *d_g = nullptr;
    unsigned short *d_wb = nullptr;  // bf16 weights, same offsets as the W blocks of d_p
    long long adam_t = 0;
    // training data
    long long nsamples = 0;
    unsigned short *d_feat = nullptr;  // [n][16] bf16
    float *d_target = nullptr;         // [n][32]
    // per-wedge column samples and joint right singular vectors (targets)
    std::vector<std::vector<int>> cols;   // member positions per wedge
    std::vector<std::vector<int>> colk;   // their centred frequencies, (k1, k2) interleaved
    std::vector<double> theta;            // wedge centre angles
    std::vector<std::vector<zd>> V;       // r x 16 per wedge
    std::vector<double> s1;               // leading joint singular value per wedge
    // scratch of the training step
    int batch_cap = 0;
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    double last_loss = 0;
    ~LearnedModel();
};

// Inference of the leading q factors alpha_t for all grid points of wedge
// ell at scale s into out (N^2 rows of qpad complex; columns q .. qpad
// zeroed), in the precision of the plan (FP32 only).
hipError_t learned_infer_wedge(LearnedModel *M, double theta, double s, void *out, int q, int qpad, int precision,
                               hipStream_t st);
// All 16 factors at n given grid points (device index list) into d_out (n x 32 floats).
hipError_t learned_infer_points(LearnedModel *M, double theta, double s, const long long *d_x, int n, float *d_out,
                                hipStream_t st);

}  // namespace fio
