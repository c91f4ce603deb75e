// C ABI of the FIO library (declared in include/fio.h).  Argument checks,
// device selection and error reporting live here; the plan builder is in
// plan.hip and the apply kernels in apply.hip.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <new>

#include "adjoint.hpp"
#include "apply.hpp"
#include "errors.hpp"
#include "linalg.hpp"
#include "multi.hpp"
#include "plan_build.hpp"

namespace fio {

static thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }
const char *get_error() { return g_error.c_str(); }

fio_status hip_fail(hipError_t e, const char *what) {
    char buf[512];
    std::snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    set_error(buf);
    return e == hipErrorOutOfMemory ? FIO_ENOMEM : FIO_EDEVICE;
}

// Makes the plan's device current for the duration of a call.
struct DeviceScope {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceScope(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev)
            err = hipSetDevice(dev);
    }
    ~DeviceScope() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
            (void)hipSetDevice(prev);
    }
};

static void drop_events(fio_plan_s *P) {
    for (auto &ev : P->prof_events) {
        (void)hipEventDestroy(ev.start);
        (void)hipEventDestroy(ev.stop);
    }
    P->prof_events.clear();
}

// unique per plan made in this process (built or loaded)
static unsigned long long next_plan_serial() {
    static std::atomic<unsigned long long> next{1};
    return next++;
}

static void free_plan(fio_plan_s *P) {
    if (!P)
        return;
    drop_events(P);
    release_layout(P);
    multi_release(P);
    delete P;
}

template <typename T>
__global__ void k_gather(const cplx<T> *__restrict__ src, const long long *__restrict__ rows, int n, int stride, int q,
                         double2 *__restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * q)
        return;
    const int r = i / q, t = i % q;
    const cplx<T> v = src[rows[r] * stride + t];
    dst[i] = make_double2((double)v.re, (double)v.im);
}

}  // namespace fio

using namespace fio;

extern "C" {

void fio_default_options(fio_options *o) {
    if (!o)
        return;
    std::memset(o, 0, sizeof(*o));
    o->precision = FIO_F32;
    o->partition = FIO_PART_EQUIANGULAR;
    o->n_wedges = 0;
    o->factor_mode = FIO_FACTORS_AUTO;
    o->seed = 0x5EED0FF10ull;
    o->max_batch = 8;
    o->sep_tol_frac = 0.25;
    o->nufft_tol_frac = 0.1;
    o->sigma = 2.0;
    o->kernel_width = 0;
    o->r0 = 32;
    o->verify_samples = 200;
    o->learned = nullptr;
    o->learned_scale = 1.0;
}

const char *fio_last_error(void) { return get_error(); }

#ifndef FIO_BUILD_ID
#define FIO_BUILD_ID "unstamped"
#endif
const char *fio_version(void) { return "fio-mi355x 0.2 (gfx950, sources " FIO_BUILD_ID ")"; }

fio_status fio_plan_ex(int N, const fio_phase *phase, const fio_amplitude *amp, double tol, const fio_options *opt,
                       fio_plan_t *out) {
    set_error("");
    if (!out || !phase)
        return (set_error("null argument"), FIO_EINVAL);
    *out = nullptr;
    if (N < 8 || (N & 1) || N > 4096)
        return (set_error("N must be even and in [8, 4096]"), FIO_EINVAL);
    if (phase->kind < 0 || phase->kind > 5)
        return (set_error("unknown phase kind"), FIO_EINVAL);
    const int ak = amp ? amp->kind : FIO_AMP_ONE;
    if (ak != FIO_AMP_ONE && ak != FIO_AMP_BESSEL)
        return (set_error("unknown amplitude kind"), FIO_ENOTSUP);
    if (ak == FIO_AMP_BESSEL) {
        // rho = h(x, xi) must be nonnegative
        const double *pp = phase->p;
        const bool nonneg = (phase->kind == 1 && pp[0] >= 0) || (phase->kind == 2 && pp[0] >= 0) ||
                            (phase->kind == 3 && pp[0] >= 0 && std::fabs(pp[1]) <= 1) ||
                            (phase->kind == 4 && pp[0] >= 0) || (phase->kind == 5 && pp[0] >= 0);
        if (!nonneg)
            return (set_error("the Bessel amplitude needs a phase with h(x, xi) >= 0"), FIO_EINVAL);
    }
    if (!(tol > 0 && tol < 1))
        return (set_error("tol must lie in (0, 1)"), FIO_EINVAL);
    fio_options o;
    if (opt)
        o = *opt;
    else
        fio_default_options(&o);
    if (o.precision != FIO_F32 && o.precision != FIO_F64)
        return (set_error("precision must be FIO_F32 or FIO_F64"), FIO_EINVAL);
    if (o.partition != FIO_PART_EQUIANGULAR && o.partition != FIO_PART_CORONAE)
        return (set_error("unknown partition"), FIO_EINVAL);
    if (o.n_wedges < 0 || o.n_wedges > 4096 || o.max_batch < 1 || o.r0 < 0 || o.kernel_width < 0 ||
        o.kernel_width > 16 || o.sigma < 0 || (o.sigma > 0 && o.sigma < 1.25) || o.verify_samples < 0)
        return (set_error("option out of range"), FIO_EINVAL);
    if (!(o.sep_tol_frac > 0 && o.sep_tol_frac <= 1) || !(o.nufft_tol_frac > 0 && o.nufft_tol_frac <= 1))
        return (set_error("tolerance fractions must lie in (0, 1]"), FIO_EINVAL);
    // the separation reads singular values off the eigenvalues of the FP64
    // Gram matrix of the sampled columns, which resolves them down to about
    // 1e-7 of the largest (its threshold is tol * sep_tol_frac)
    if (tol < 5e-7)
        return (set_error("tol below the floor (5e-7) of the Gram-matrix separation"), FIO_ENOTSUP);
    if (o.factor_mode < FIO_FACTORS_AUTO || o.factor_mode > FIO_FACTORS_TAYLOR)
        return (set_error("unknown factor mode"), FIO_EINVAL);
    if (o.factor_mode == FIO_FACTORS_LEARNED && !o.learned)
        return (set_error("FIO_FACTORS_LEARNED needs a trained network"), FIO_EINVAL);
    // FP32 plans regenerate gamma^x in FP32 from the phase alone
    if (o.factor_mode == FIO_FACTORS_REGEN && o.precision == FIO_F32 && ak != FIO_AMP_ONE)
        return (set_error("FIO_FACTORS_REGEN with an amplitude needs FIO_F64 (or use FIO_FACTORS_STORED)"),
                FIO_ENOTSUP);
    fio_plan_s *P = new (std::nothrow) fio_plan_s();
    if (!P)
        return (set_error("host allocation failed"), FIO_ENOMEM);
    P->serial = next_plan_serial();
    P->N = N;
    P->phase.kind = phase->kind;
    P->phase.amp = ak;
    std::memcpy(P->phase.p, phase->p, sizeof(P->phase.p));
    P->tol = tol;
    P->opt = o;
    P->precision = o.precision;
    fio_status st;
    try {
        st = build_plan(P);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        st = FIO_ENOMEM;
    } catch (...) {
        set_error("unexpected host exception while building the plan");
        st = FIO_EDEVICE;
    }
    if (st != FIO_OK) {
        free_plan(P);
        return st;
    }
    *out = P;
    return FIO_OK;
}

fio_status fio_plan(int N, const fio_phase *phase, const fio_amplitude *amp, double tol, fio_plan_t *out) {
    return fio_plan_ex(N, phase, amp, tol, nullptr, out);
}

fio_status fio_plan_save(fio_plan_t plan, const char *path) {
    set_error("");
    if (!plan || !path)
        return (set_error("null argument"), FIO_EINVAL);
    try {
        return save_plan(plan, path);
    } catch (const std::bad_alloc &) {
        return (set_error("host allocation failed"), FIO_ENOMEM);
    }
}

fio_status fio_plan_load(const char *path, fio_plan_t *out) {
    set_error("");
    if (!path || !out)
        return (set_error("null argument"), FIO_EINVAL);
    *out = nullptr;
    fio_plan_s *P = new (std::nothrow) fio_plan_s();
    if (!P)
        return (set_error("host allocation failed"), FIO_ENOMEM);
    P->serial = next_plan_serial();
    fio_status st;
    try {
        st = load_plan(P, path);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        st = FIO_ENOMEM;
    } catch (...) {
        set_error("unexpected host exception while loading the plan");
        st = FIO_EDEVICE;
    }
    if (st != FIO_OK) {
        free_plan(P);
        return st;
    }
    *out = P;
    return FIO_OK;
}

static fio_status apply_common(fio_plan_t P, int l0, int l1, int B, const void *fhat, void *u, void *stream) {
    set_error("");
    if (!P || !fhat || !u)
        return (set_error("null argument"), FIO_EINVAL);
    if (B < 1)
        return (set_error("B must be >= 1"), FIO_EINVAL);
    if (l0 < 0 || l1 > P->L || l0 > l1)
        return (set_error("wedge range out of bounds"), FIO_EINVAL);
    DeviceScope ds(P->device);
    if (ds.err != hipSuccess)
        return hip_fail(ds.err, "hipSetDevice");
    if (l0 == l1) {
        const size_t bytes = (size_t)B * P->N * P->N * P->esize;
        FIO_HIP_TRY(zero_fill(u, bytes, static_cast<hipStream_t>(stream)));
        return FIO_OK;
    }
    FIO_HIP_TRY(apply_launch(P, B, fhat, u, static_cast<hipStream_t>(stream), l0, l1));
    return FIO_OK;
}

fio_status fio_apply(fio_plan_t plan, const void *fhat, void *u, void *stream) {
    return apply_common(plan, 0, plan ? plan->L : 0, 1, fhat, u, stream);
}

fio_status fio_apply_batch(fio_plan_t plan, int B, const void *fhat, void *u, void *stream) {
    return apply_common(plan, 0, plan ? plan->L : 0, B, fhat, u, stream);
}

fio_status fio_apply_batch_noalloc(fio_plan_t P, int B, const void *fhat, void *u, void *stream) {
    set_error("");
    if (!P || !fhat || !u)
        return (set_error("null argument"), FIO_EINVAL);
    if (B < 1)
        return (set_error("B must be >= 1"), FIO_EINVAL);
    const long long per = scratch_bytes_per_rhs(P);
    if (per + 256 > (long long)kScratchBytes) {
        char msg[200];
        std::snprintf(msg, sizeof(msg),
                      "one right-hand side needs %lld bytes of scratch, above the fixed %lld-byte array", per + 256,
                      (long long)kScratchBytes);
        return (set_error(msg), FIO_EINVAL);
    }
    DeviceScope ds(P->device);
    if (ds.err != hipSuccess)
        return hip_fail(ds.err, "hipSetDevice");
    FIO_HIP_TRY(apply_launch_scratch(P, B, fhat, u, static_cast<hipStream_t>(stream)));
    return FIO_OK;
}

fio_status fio_apply_adjoint_batch(fio_plan_t P, int B, const void *g, void *hhat, void *stream) {
    set_error("");
    if (!P || !g || !hhat)
        return (set_error("null argument"), FIO_EINVAL);
    if (B < 1)
        return (set_error("B must be >= 1"), FIO_EINVAL);
    DeviceScope ds(P->device);
    if (ds.err != hipSuccess)
        return hip_fail(ds.err, "hipSetDevice");
    try {
        return adjoint_launch(P, B, g, hhat, static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc &) {
        return (set_error("host allocation failed"), FIO_ENOMEM);
    }
}

fio_status fio_apply_adjoint(fio_plan_t plan, const void *g, void *hhat, void *stream) {
    return fio_apply_adjoint_batch(plan, 1, g, hhat, stream);
}

fio_status fio_apply_wedges(fio_plan_t plan, int l0, int l1, int B, const void *fhat, void *u, void *stream) {
    return apply_common(plan, l0, l1, B, fhat, u, stream);
}

fio_status fio_apply_multi(int n, const fio_plan_t *plans, const void *const *fhat, void *const *u, const int *B,
                           void *stream) {
    set_error("");
    if (n < 1 || !plans || !fhat || !u || !B)
        return (set_error("null argument or n < 1"), FIO_EINVAL);
    for (int i = 0; i < n; ++i) {
        if (!plans[i] || !fhat[i] || !u[i] || B[i] < 1)
            return (set_error("null plan/pointer or B < 1 in instance list"), FIO_EINVAL);
        if (plans[i]->precision != plans[0]->precision || plans[i]->device != plans[0]->device)
            return (set_error("instances must share precision and device"), FIO_EINVAL);
    }
    DeviceScope ds(plans[0]->device);
    if (ds.err != hipSuccess)
        return hip_fail(ds.err, "hipSetDevice");
    try {
        return multi_apply(n, plans, fhat, u, B, static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return FIO_ENOMEM;
    }
}

fio_status fio_plan_info(fio_plan_t P, fio_plan_info_t *o) {
    set_error("");
    if (!P || !o)
        return (set_error("null argument"), FIO_EINVAL);
    std::memset(o, 0, sizeof(*o));
    o->N = P->N;
    o->L = P->L;
    o->precision = P->precision;
    o->factor_mode = P->factor_mode;
    o->kernel_width = P->w;
    o->fallback = P->fallback;
    o->sigma = P->sigma;
    o->tol = P->tol;
    o->plan_ms = P->plan_ms;
    o->max_rank = 0;
    o->min_rank = 1 << 30;
    long long comp = 0;
    for (const WedgeHost &W : P->wedges) {
        if (W.members.empty())
            continue;
        o->max_rank = std::max(o->max_rank, W.q);
        o->min_rank = std::min(o->min_rank, W.q);
        o->max_sep_error = std::max(o->max_sep_error, W.sep_err);
        o->fine_cells += (long long)W.n[0] * W.n[1];
        o->box_cells += (long long)W.B[0] * W.B[1];
        comp += (long long)(W.Z.size() + W.P.size()) * 16 + (long long)(W.C.size() * 4 + W.R.size() * 8);
    }
    if (o->min_rank == (1 << 30))
        o->min_rank = 0;
    o->factor_bytes = P->factor_bytes;
    o->workspace_bytes = P->workspace_bytes;
    o->compressed_bytes = comp;
    o->learned_sep_error = P->learned_sep_err;
    o->learned_ms = P->learned_ms;
    return FIO_OK;
}

fio_status fio_wedge_info(fio_plan_t P, int l, fio_wedge_info_t *o) {
    set_error("");
    if (!P || !o)
        return (set_error("null argument"), FIO_EINVAL);
    if (l < 0 || l >= P->L)
        return (set_error("wedge index out of range"), FIO_EINVAL);
    const WedgeHost &W = P->wedges[l];
    std::memset(o, 0, sizeof(*o));
    o->theta = W.theta;
    o->members = (int)W.members.size();
    o->rank = W.q;
    o->samples = W.r;
    std::memcpy(o->M, W.M, sizeof(o->M));
    o->xi_c[0] = W.xc[0];
    o->xi_c[1] = W.xc[1];
    o->box[0] = W.B[0];
    o->box[1] = W.B[1];
    o->lo[0] = W.lo[0];
    o->lo[1] = W.lo[1];
    o->fine[0] = W.n[0];
    o->fine[1] = W.n[1];
    o->sep_error = W.sep_err;
    return FIO_OK;
}

fio_status fio_wedge_map(fio_plan_t P, int *ids) {
    set_error("");
    if (!P || !ids)
        return (set_error("null argument"), FIO_EINVAL);
    std::memcpy(ids, P->wedge_of.data(), sizeof(int) * P->wedge_of.size());
    return FIO_OK;
}

fio_status fio_wedge_factors(fio_plan_t P, int l, int nx, const long long *xidx, double *gx, int nxi,
                             const long long *xiidx, double *gxi) {
    set_error("");
    if (!P || l < 0 || l >= P->L || nx < 0 || nxi < 0 || (nx > 0 && (!xidx || !gx)) ||
        (nxi > 0 && (!xiidx || !gxi)))
        return (set_error("bad argument"), FIO_EINVAL);
    const WedgeHost &W = P->wedges[l];
    const WedgeDev &D = P->wdev[l];
    const long long NN = (long long)P->N * P->N;
    const int q = W.q;
    if (q == 0)
        return FIO_OK;
    std::vector<long long> mrows(nxi);
    std::vector<double> unscale(nxi);
    const int h = P->N / 2;
    for (int j = 0; j < nxi; ++j) {
        auto it = std::lower_bound(W.members.begin(), W.members.end(), (int)xiidx[j]);
        if (xiidx[j] < 0 || xiidx[j] >= NN || it == W.members.end() || *it != (int)xiidx[j])
            return (set_error("frequency index not in the wedge"), FIO_EINVAL);
        mrows[j] = it - W.members.begin();
        const int om = (int)xiidx[j], k1 = om / P->N - h, k2 = om % P->N - h;
        const int a1 = W.M[0] * k1 + W.M[1] * k2 - W.xc[0], a2 = W.M[2] * k1 + W.M[3] * k2 - W.xc[1];
        unscale[j] = P->N / (W.dec1[a1 - W.lo[0]] * W.dec2[a2 - W.lo[1]]);
    }
    for (int i = 0; i < nx; ++i)
        if (xidx[i] < 0 || xidx[i] >= NN)
            return (set_error("grid index out of range"), FIO_EINVAL);
    DeviceScope ds(P->device);
    if (ds.err != hipSuccess)
        return hip_fail(ds.err, "hipSetDevice");
    const int nmax = std::max(nx, nxi);
    if (nmax == 0)
        return FIO_OK;
    long long *d_idx = nullptr;
    double2 *d_out = nullptr;
    FIO_HIP_TRY(hipMalloc(&d_idx, sizeof(long long) * nmax));
    hipError_t e = hipMalloc(&d_out, sizeof(double2) * (size_t)nmax * q);
    if (e != hipSuccess) {
        (void)hipFree(d_idx);
        return hip_fail(e, "hipMalloc");
    }
    auto run = [&](const long long *rows, int n, bool xside, double *dst) -> hipError_t {
        hipError_t err = hipMemcpy(d_idx, rows, sizeof(long long) * n, hipMemcpyHostToDevice);
        if (err != hipSuccess)
            return err;
        const unsigned g = (unsigned)((n * q + 255) / 256);
        if (P->precision == FIO_F64) {
            const cplx<double> *src = static_cast<const cplx<double> *>(xside ? P->d_gx : P->d_gxi) +
                                      (xside ? D.gx_off : D.gxi_off);
            k_gather<double><<<g, 256>>>(src, d_idx, n, W.qpad, q, d_out);
        } else {
            const cplx<float> *src = static_cast<const cplx<float> *>(xside ? P->d_gx : P->d_gxi) +
                                     (xside ? D.gx_off : D.gxi_off);
            k_gather<float><<<g, 256>>>(src, d_idx, n, W.qpad, q, d_out);
        }
        err = hipGetLastError();
        if (err != hipSuccess)
            return err;
        return hipMemcpy(dst, d_out, sizeof(double2) * (size_t)n * q, hipMemcpyDeviceToHost);
    };
    if (nx > 0 && P->regen) {
        // regenerated factors: gamma^x(x, t) = sum_c A(x, C_c) Z(c, t) in FP64 on the host
        const double e1 = std::cos(W.theta), e2 = std::sin(W.theta);
        for (int i = 0; i < nx; ++i)
            for (int t = 0; t < q; ++t) {
                zd acc(0, 0);
                for (size_t c = 0; c < W.C.size(); ++c) {
                    const int om = W.members[W.C[c]];
                    acc += host_residual(P->phase, P->N, xidx[i], e1, e2, om / P->N - h, om % P->N - h) *
                           W.Z[c * q + t];
                }
                gx[((size_t)i * q + t) * 2] = acc.real();
                gx[((size_t)i * q + t) * 2 + 1] = acc.imag();
            }
    } else if (nx > 0) {
        e = run(xidx, nx, true, gx);
    }
    if (e == hipSuccess && nxi > 0) {
        e = run(mrows.data(), nxi, false, gxi);
        for (int j = 0; j < nxi && e == hipSuccess; ++j)
            for (int t = 0; t < 2 * q; ++t)
                gxi[(size_t)j * 2 * q + t] *= unscale[j];
    }
    (void)hipFree(d_idx);
    (void)hipFree(d_out);
    if (e != hipSuccess)
        return hip_fail(e, "fio_wedge_factors");
    return FIO_OK;
}

fio_status fio_wedge_warp(fio_plan_t P, int l, int nx, const long long *xidx, double *y) {
    set_error("");
    if (!P || l < 0 || l >= P->L || nx < 0 || (nx > 0 && (!xidx || !y)))
        return (set_error("bad argument"), FIO_EINVAL);
    const long long NN = (long long)P->N * P->N;
    for (int i = 0; i < nx; ++i)
        if (xidx[i] < 0 || xidx[i] >= NN)
            return (set_error("grid index out of range"), FIO_EINVAL);
    if (nx == 0)
        return FIO_OK;
    DeviceScope ds(P->device);
    if (ds.err != hipSuccess)
        return hip_fail(ds.err, "hipSetDevice");
    long long *d_idx = nullptr;
    double *d_y = nullptr;
    FIO_HIP_TRY(hipMalloc(&d_idx, sizeof(long long) * nx));
    hipError_t e = hipMalloc(&d_y, sizeof(double) * 2 * nx);
    if (e == hipSuccess)
        e = hipMemcpy(d_idx, xidx, sizeof(long long) * nx, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        const WedgeHost &W = P->wedges[l];
        k_warp<<<(nx + 255) / 256, 256>>>(P->phase, P->N, std::cos(W.theta), std::sin(W.theta), d_idx, nx, d_y);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpy(y, d_y, sizeof(double) * 2 * nx, hipMemcpyDeviceToHost);
    (void)hipFree(d_idx);
    if (d_y)
        (void)hipFree(d_y);
    if (e != hipSuccess)
        return hip_fail(e, "fio_wedge_warp");
    return FIO_OK;
}

fio_status fio_profile(fio_plan_t P, int on) {
    set_error("");
    if (!P)
        return (set_error("null plan"), FIO_EINVAL);
    DeviceScope ds(P->device);
    drop_events(P);
    P->profiling = on ? 1 : 0;
    for (int i = 0; i < 3; ++i) {
        P->prof_ms[i] = 0;
        P->prof_launches[i] = 0;
    }
    return FIO_OK;
}

fio_status fio_profile_read(fio_plan_t P, double ms[3], long long launches[3]) {
    set_error("");
    if (!P || !ms || !launches)
        return (set_error("null argument"), FIO_EINVAL);
    DeviceScope ds(P->device);
    for (auto &ev : P->prof_events) {
        FIO_HIP_TRY(hipEventSynchronize(ev.stop));
        float t = 0;
        FIO_HIP_TRY(hipEventElapsedTime(&t, ev.start, ev.stop));
        P->prof_ms[ev.stage] += t;
        P->prof_launches[ev.stage] += 1;
    }
    drop_events(P);
    for (int i = 0; i < 3; ++i) {
        ms[i] = P->prof_ms[i];
        launches[i] = P->prof_launches[i];
    }
    return FIO_OK;
}

fio_status fio_destroy(fio_plan_t plan) {
    set_error("");
    if (!plan)
        return FIO_OK;
    DeviceScope ds(plan->device);
    free_plan(plan);
    return FIO_OK;
}

fio_status fio_host_eigh(int n, const double *A, double *w, double *V) {
    set_error("");
    if (n < 1 || n > 4096 || !A || !w || !V)
        return (set_error("bad argument"), FIO_EINVAL);
    std::vector<zd> M((size_t)n * n), Vec;
    for (size_t i = 0; i < M.size(); ++i)
        M[i] = zd(A[2 * i], A[2 * i + 1]);
    std::vector<double> lam;
    eigh(n, M, lam, Vec);
    for (int i = 0; i < n; ++i)
        w[i] = lam[i];
    for (size_t i = 0; i < Vec.size(); ++i) {
        V[2 * i] = Vec[i].real();
        V[2 * i + 1] = Vec[i].imag();
    }
    return FIO_OK;
}

fio_status fio_host_column_id(int m, int n, const double *A, double tol, int *k, int *perm, double *T) {
    set_error("");
    if (m < 1 || n < 1 || m > 4096 || n > 4096 || !A || !k || !perm || !T || !(tol >= 0))
        return (set_error("bad argument"), FIO_EINVAL);
    std::vector<zd> M((size_t)m * n), Tm;
    for (size_t i = 0; i < M.size(); ++i)
        M[i] = zd(A[2 * i], A[2 * i + 1]);
    std::vector<int> pv;
    *k = column_id(m, n, M, tol, pv, Tm);
    for (int j = 0; j < n; ++j)
        perm[j] = pv[j];
    for (size_t i = 0; i < Tm.size(); ++i) {
        T[2 * i] = Tm[i].real();
        T[2 * i + 1] = Tm[i].imag();
    }
    return FIO_OK;
}

}  // extern "C"
