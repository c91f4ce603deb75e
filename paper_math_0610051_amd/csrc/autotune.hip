// Autotuner and the on-device accuracy probe.
//
// fio_probe_error evaluates the operator by FP64 direct summation (eq. (dfio))
// on the device at sampled output points and returns the relative l2 error of
// a computed u there (the Section 4 estimator).  fio_autotune builds candidate
// plans over the wedge count, the oversampling factor and the split of the
// tolerance between separation and NUFFT, times a batched apply with HIP
// events, probes its accuracy, and keeps the fastest candidate within the
// budget; choices are cached in a text file keyed by the problem.  fio_copy
// is a plain streaming copy whose hardware counters and event time calibrate
// the traffic and bandwidth figures of the other kernels.
#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "apply.hpp"
#include "errors.hpp"
#include "plan_build.hpp"

namespace fio {

// One block per sample point: u(x) = (1/N) sum_xi a(x, xi) exp(2 pi i Phi(x, xi)) fhat(xi),
// x.xi reduced exactly in integers, h in FP64, FP64 accumulation.
template <typename T>
__global__ __launch_bounds__(256) void k_direct_probe(Phase ph, int N, const cplx<T> *__restrict__ fhat,
                                                      const long long *__restrict__ xs, double2 *__restrict__ out) {
    __shared__ double sr[256], si[256];
    const long long p = xs[blockIdx.x];
    const int n1 = (int)(p / N), n2 = (int)(p % N), h = N / 2;
    const XCoef c = phase_xcoef(ph, (double)n1 / N, (double)n2 / N);
    double ar = 0, ai = 0;
    const long long NN = (long long)N * N;
    for (long long i = threadIdx.x; i < NN; i += blockDim.x) {
        const int k1 = (int)(i / N) - h, k2 = (int)(i % N) - h;
        long long ip = ((long long)n1 * k1 + (long long)n2 * k2) % N;
        if (ip < 0)
            ip += N;
        const double hv = phase_h(ph, c, (double)k1, (double)k2);
        double phs = (double)ip / N + hv;
        phs -= rint(phs);
        double cs, sn;
        expi2pi(phs, cs, sn);
        if (ph.amp == 1) {
            double ar, ai;
            amp_bessel(hv, k1 == 0 && k2 == 0, ar, ai);
            const double tr = cs * ar - sn * ai;
            sn = cs * ai + sn * ar;
            cs = tr;
        }
        const cplx<T> f = fhat[i];
        ar += cs * (double)f.re - sn * (double)f.im;
        ai += cs * (double)f.im + sn * (double)f.re;
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sr[threadIdx.x] += sr[threadIdx.x + o];
            si[threadIdx.x] += si[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[blockIdx.x] = make_double2(sr[0] / N, si[0] / N);
}

template <typename T>
__global__ void k_gather_points(const cplx<T> *__restrict__ u, const long long *__restrict__ xs, int n,
                                double2 *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const cplx<T> v = u[xs[i]];
        out[i] = make_double2((double)v.re, (double)v.im);
    }
}

// Complex Gaussian test input (Box-Muller on a counter-based stream), centred layout.
template <typename T>
__global__ void k_random_fhat(cplx<T> *__restrict__ f, long long n, unsigned long long key, double scale) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const uint64_t a = splitmix64(key + 2 * (unsigned long long)i), b = splitmix64(key + 2 * (unsigned long long)i + 1);
        const double u1 = ((a >> 11) + 1.0) / 9007199254740993.0, u2 = (b >> 11) / 9007199254740992.0;
        const double r = scale * sqrt(-2.0 * log(u1));
        double cs, sn;
        expi2pi(u2, cs, sn);
        f[i] = cmake<T>((T)(r * cs), (T)(r * sn));
    }
}

template <typename T>
static fio_status probe_t(fio_plan_s *P, const void *fhat, const void *u, int ns, unsigned long long seed, double *err,
                          hipStream_t s) {
    const long long NN = (long long)P->N * P->N;
    ns = (int)std::min<long long>(ns, NN);
    std::vector<long long> xs(ns);
    uint64_t st = splitmix64(seed ^ 0x9B0BEull);
    for (int i = 0; i < ns; ++i) {
        st = splitmix64(st);
        xs[i] = (long long)(st % (uint64_t)NN);
    }
    long long *d_xs = nullptr;
    double2 *d_ref = nullptr, *d_got = nullptr;
    FIO_HIP_TRY(hipMalloc(&d_xs, sizeof(long long) * ns));
    hipError_t e = hipMalloc(&d_ref, sizeof(double2) * ns);
    if (e == hipSuccess)
        e = hipMalloc(&d_got, sizeof(double2) * ns);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_xs, xs.data(), sizeof(long long) * ns, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        k_direct_probe<T><<<ns, 256, 0, s>>>(P->phase, P->N, static_cast<const cplx<T> *>(fhat), d_xs, d_ref);
        k_gather_points<T><<<(ns + 255) / 256, 256, 0, s>>>(static_cast<const cplx<T> *>(u), d_xs, ns, d_got);
        e = hipGetLastError();
    }
    std::vector<double2> ref(ns), got(ns);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ref.data(), d_ref, sizeof(double2) * ns, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(got.data(), d_got, sizeof(double2) * ns, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    (void)hipFree(d_xs);
    if (d_ref)
        (void)hipFree(d_ref);
    if (d_got)
        (void)hipFree(d_got);
    if (e != hipSuccess)
        return hip_fail(e, "fio_probe_error");
    double num = 0, den = 0;
    for (int i = 0; i < ns; ++i) {
        const double dr = got[i].x - ref[i].x, di = got[i].y - ref[i].y;
        num += dr * dr + di * di;
        den += ref[i].x * ref[i].x + ref[i].y * ref[i].y;
    }
    *err = std::sqrt(num / std::max(den, 1e-300));
    return FIO_OK;
}

fio_status probe_error(fio_plan_s *P, const void *fhat, const void *u, int ns, unsigned long long seed, double *err,
                       hipStream_t s) {
    return P->precision == FIO_F64 ? probe_t<double>(P, fhat, u, ns, seed, err, s)
                                   : probe_t<float>(P, fhat, u, ns, seed, err, s);
}

// Cache key: everything a choice depends on, including the library build
// (a cached choice of an older kernel build is not reused).
static std::string tune_key(int N, const fio_phase *ph, int amp, double tol, const fio_options &o, int B) {
    char buf[512];
    std::snprintf(buf, sizeof(buf),
                  "N=%d kind=%d p=%.9g,%.9g,%.9g amp=%d tol=%.3g prec=%d part=%d mode=%d seed=%llu B=%d build=%s",
                  N, ph->kind, ph->p[0], ph->p[1], ph->p[2], amp, tol, o.precision, o.partition, o.factor_mode,
                  o.seed, B, fio_version());
    return buf;
}

static bool cache_lookup(const char *path, const std::string &key, fio_tune_result_t *best) {
    if (!path || !*path)
        return false;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char *bar = std::strchr(line, '|');
        if (!bar)
            continue;
        *bar = 0;
        if (key != line)
            continue;
        fio_tune_result_t r{};
        if (std::sscanf(bar + 1, "%d %lf %d %lf %lf %lf %lf", &r.n_wedges, &r.sigma, &r.kernel_width,
                        &r.sep_tol_frac, &r.nufft_tol_frac, &r.ms_per_rhs, &r.error) == 7) {
            *best = r;
            found = true;  // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

static void cache_store(const char *path, const std::string &key, const fio_tune_result_t &r) {
    if (!path || !*path)
        return;
    FILE *f = std::fopen(path, "a");
    if (!f)
        return;
    std::fprintf(f, "%s|%d %.6g %d %.6g %.6g %.6g %.6g\n", key.c_str(), r.n_wedges, r.sigma, r.kernel_width,
                 r.sep_tol_frac, r.nufft_tol_frac, r.ms_per_rhs, r.error);
    std::fclose(f);
}

// Grid-stride copy of n 16-byte units; each lane moves one unit per iteration
// so consecutive lanes touch consecutive addresses.
__global__ __launch_bounds__(256) void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

}  // namespace fio

using namespace fio;

extern "C" {

fio_status fio_probe_error(fio_plan_t plan, const void *fhat, const void *u, int nsamples, unsigned long long seed,
                           double *err, void *stream) {
    set_error("");
    if (!plan || !fhat || !u || !err || nsamples < 1)
        return (set_error("bad argument"), FIO_EINVAL);
    return probe_error(plan, fhat, u, nsamples, seed, err, static_cast<hipStream_t>(stream));
}

fio_status fio_copy(const void *src, void *dst, size_t bytes, void *stream) {
    set_error("");
    if (!src || !dst || (bytes & 15) || ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15))
        return (set_error("fio_copy needs non-null 16-byte aligned pointers and a multiple of 16 bytes"), FIO_EINVAL);
    const size_t n = bytes / 16;
    if (n == 0)
        return FIO_OK;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 256 * 32);
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n);
    FIO_HIP_TRY(hipGetLastError());
    return FIO_OK;
}

fio_status fio_autotune(int N, const fio_phase *phase, const fio_amplitude *amp, double tol, const fio_options *base,
                        int B, fio_tune_result_t *tried, int max_tried, int *ntried, fio_tune_result_t *best) {
    set_error("");
    if (!phase || !best || B < 1 || (max_tried > 0 && !tried))
        return (set_error("bad argument"), FIO_EINVAL);
    fio_options o;
    if (base)
        o = *base;
    else
        fio_default_options(&o);
    const char *cache = std::getenv("FIO_TUNE_CACHE");
    const std::string key = tune_key(N, phase, amp ? amp->kind : FIO_AMP_ONE, tol, o, B);
    if (ntried)
        *ntried = 0;
    if (cache_lookup(cache, key, best))
        return FIO_OK;
    Phase ph0{};
    ph0.kind = phase->kind;
    std::memcpy(ph0.p, phase->p, sizeof(ph0.p));
    const int L0 = o.n_wedges > 0 ? o.n_wedges : default_wedge_count(N, ph0);
    // fewer wedges rarely pay at large N, where ranks grow fastest with the angular width
    std::vector<int> Ls;
    if (N <= 256)
        Ls.push_back(std::max(8, L0 - 8));
    for (int L : {L0, L0 + 8, L0 + 16})
        Ls.push_back(L);
    const double splits[][2] = {{0.25, 0.1}, {0.4, 0.15}};
    // oversampling: below 2 the grids (and FFT stages) shrink while the kernel widens
    const double sigmas[] = {1.5, 1.75, 2.0, 2.5};
    const size_t es = o.precision == FIO_F64 ? 16 : 8;
    const long long NN = (long long)N * N;
    void *d_f = nullptr, *d_u = nullptr;
    FIO_HIP_TRY(hipMalloc(&d_f, es * NN * B));
    hipError_t he = hipMalloc(&d_u, es * NN * B);
    if (he != hipSuccess) {
        (void)hipFree(d_f);
        return hip_fail(he, "fio_autotune");
    }
    if (o.precision == FIO_F64)
        k_random_fhat<double><<<1024, 256>>>(static_cast<cplx<double> *>(d_f), NN * B, 0x7A11ull, 1.0 / N);
    else
        k_random_fhat<float><<<1024, 256>>>(static_cast<cplx<float> *>(d_f), NN * B, 0x7A11ull, 1.0 / N);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    bool have = false;
    int count = 0;
    fio_status result = FIO_OK;
    // kernel widths: the one the NUFFT tolerance asks for, and the next
    // compiled width below it (the width formula is a bound; the probe decides)
    auto widths = [&](double eps, double sg) {
        int w = 0;
        double beta = 0;
        es_parameters(eps, sg, 0, w, beta);
        std::vector<int> ws{w};
        int lower = 0;
        for (int v : kInterpWidths)
            if (v < w)
                lower = v;
        if (lower >= 4)
            ws.push_back(lower);
        return ws;
    };
    bool failed = false;  // a failed launch or probe ends the whole search
    for (double sg : sigmas)
        for (const auto &sp : splits)
            for (int kw : widths(tol * sp[1], sg))
            for (int L : Ls) {
                if (failed)
                    break;
                fio_options c = o;
                c.n_wedges = L;
                c.sigma = sg;
                c.sep_tol_frac = sp[0];
                c.nufft_tol_frac = sp[1];
                c.kernel_width = kw;
                c.max_batch = std::max(c.max_batch, B);
                fio_plan_t P = nullptr;
                fio_status st = fio_plan_ex(N, phase, amp, tol, &c, &P);
                if (st != FIO_OK)
                    continue;  // e.g. a grid too long for this oversampling
                fio_tune_result_t r{};
                r.n_wedges = L;
                r.sigma = sg;
                r.kernel_width = P->w;
                r.sep_tol_frac = sp[0];
                r.nufft_tol_frac = sp[1];
                // the fastest of five timed applies after two warm-ups: the
                // minimum is what the candidate sustains, free of one-off stalls
                float ms = 0;
                hipError_t ae = apply_launch(P, B, d_f, d_u, 0, 0, P->L);
                if (ae == hipSuccess)
                    ae = apply_launch(P, B, d_f, d_u, 0, 0, P->L);
                for (int rep = 0; rep < 5 && ae == hipSuccess; ++rep) {
                    float t = 0;
                    ae = hipEventRecord(e0, 0);
                    if (ae == hipSuccess)
                        ae = apply_launch(P, B, d_f, d_u, 0, 0, P->L);
                    if (ae == hipSuccess)
                        ae = hipEventRecord(e1, 0);
                    if (ae == hipSuccess)
                        ae = hipEventSynchronize(e1);
                    if (ae == hipSuccess)
                        ae = hipEventElapsedTime(&t, e0, e1);
                    if (ae == hipSuccess && (rep == 0 || t < ms))
                        ms = t;
                }
                if (ae != hipSuccess) {
                    fio_destroy(P);
                    result = hip_fail(ae, "fio_autotune apply");
                    failed = true;
                    break;
                }
                r.ms_per_rhs = ms / B;
                double err = 1;
                st = probe_error(P, d_f, d_u, 256, 0x5EEDull + count, &err, 0);
                fio_destroy(P);
                if (st != FIO_OK) {
                    result = st;
                    failed = true;
                    break;
                }
                r.error = err;
                if (tried && count < max_tried)
                    tried[count] = r;
                ++count;
                if (err <= 0.8 * tol && (!have || r.ms_per_rhs < best->ms_per_rhs)) {
                    *best = r;
                    have = true;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(d_f);
    (void)hipFree(d_u);
    if (ntried)
        *ntried = std::min(count, std::max(0, max_tried));
    if (result != FIO_OK)
        return result;
    if (!have)
        return (set_error("no candidate met the tolerance"), FIO_EACCURACY);
    cache_store(cache, key, *best);
    return FIO_OK;
}

}  // extern "C"
