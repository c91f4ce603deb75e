// Plan-construction internals shared by plan.hip and abi.hip.
#pragma once

#include <vector>

#include "plan.hpp"

namespace fio {

// Device scratch reused across the wedges of one plan build.
struct DeviceScratch {
    double2 *cols = nullptr, *partial = nullptr, *gram = nullptr;
    int ncols = 0;
    size_t npartial = 0, ngram_ = 0;
    hipError_t ensure_cols(int n);
    hipError_t ensure_partial(size_t npart, size_t ngram);
    ~DeviceScratch();
};

int default_wedge_count(int N, const Phase &ph);
void partition_equiangular(int N, int L, std::vector<int> &ids, std::vector<double> &thetas);
void partition_coronae(int N, std::vector<int> &ids, std::vector<double> &thetas);
void wedge_geometry(int N, double sigma, int w, WedgeHost &W);
void es_parameters(double eps, double sigma, int forced_w, int &w, double &beta);
double es_fourier(int w, double beta, double omega);
zd host_residual(const Phase &ph, int N, long long p, double e1, double e2, double k1, double k2);
fio_status build_plan(fio_plan_s *P);
fio_status save_plan(const fio_plan_s *P, const char *path);
fio_status load_plan(fio_plan_s *P, const char *path);
void release_layout(fio_plan_s *P);
std::vector<int> sample_members(int n, int k, uint64_t &state);
std::vector<long long> sample_points(long long n, int k, uint64_t &state);
std::vector<double> member_scale(int N, const WedgeHost &W);
// Device layout of the plan's tables, factors and workspace from the wedge ranks.
fio_status plan_layout(fio_plan_s *P);
// Deterministic separated factors of Section 3.1 (FIO_FACTORS_TAYLOR).
fio_status plan_taylor(fio_plan_s *P, const double2 *d_xcoef);
fio_status gram_of_columns(const Phase &ph, int N, double2 *d_xcoef, double theta, const std::vector<double2> &cols,
                           DeviceScratch &scr, std::vector<zd> &G, bool fill_xcoef = true);

__global__ void k_warp(Phase ph, int N, double e1, double e2, const long long *__restrict__ xidx, int nx,
                       double *__restrict__ y);

}  // namespace fio
