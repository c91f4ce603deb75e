// Learned spatial factors (the network part of the plan).
//
// The network: a fixed periodic feature map of (x1, x2, theta_ell, s) (16
// inputs), three hidden layers of width 128 with the tanh form of GELU, and 32
// outputs = the real and imaginary parts of 16 spatial factors alpha_t(x).
// Weights are kept as FP32 masters and fed to the matrix cores as BF16; every
// product accumulates in FP32 (v_mfma_f32_16x16x16_bf16).  Training (forward,
// backward, Adam) and plan-time inference run in the kernels of this file.
//
// Training targets come from the method's own randomized separation (Section
// 3.3), made free of the SVD's gauge: per wedge one set C of r columns of the
// residual kernel exp(2 pi i Phi_ell) is sampled once and shared by all
// training scales; the Gram matrices of A_s[:, C] are summed over the scales,
// and its leading 16 eigenvectors V give alpha*_s(x) = A_s(x, C) V / s_1,
// which is analytic in (x, s).  At plan time the network's alpha replaces
// gamma^x and gamma^xi is refit as T = alpha_[R]^+ A_[R] on sampled rows.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "apply.hpp"
#include "errors.hpp"
#include "learned.hpp"
#include "linalg.hpp"
#include "plan_build.hpp"

namespace fio {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ inline unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

constexpr float kGeluC = 0.79788456080286535588f;  // sqrt(2 / pi)
constexpr float kGeluA = 0.044715f;

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + tanhf(kGeluC * (z + kGeluA * z * z * z))); }
__device__ inline float gelu_grad_f(float z) {
    const float t = tanhf(kGeluC * (z + kGeluA * z * z * z));
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * kGeluC * (1.0f + 3.0f * kGeluA * z * z);
}

// Periodic feature map: harmonics 1 and 2 of x1, x2 and theta, then s - 1, (s - 1)^2, 1, 0.
__host__ __device__ inline void net_features(double x1, double x2, double th, double s, float *f) {
    f[0] = (float)sin2pi(x1);
    f[1] = (float)cos2pi(x1);
    f[2] = (float)sin2pi(x2);
    f[3] = (float)cos2pi(x2);
    f[4] = (float)sin2pi(2 * x1);
    f[5] = (float)cos2pi(2 * x1);
    f[6] = (float)sin2pi(2 * x2);
    f[7] = (float)cos2pi(2 * x2);
    f[8] = (float)cos(th);
    f[9] = (float)sin(th);
    f[10] = (float)cos(2 * th);
    f[11] = (float)sin(2 * th);
    f[12] = (float)(s - 1.0);
    f[13] = (float)((s - 1.0) * (s - 1.0));
    f[14] = 1.0f;
    f[15] = 0.0f;
}

// ---------------------------------------------------------------------------
// BF16 matrix-core GEMM: C (M x N) = A (M x K) B (K x N), FP32 accumulate.
// TA: A is stored K x M (row-major) and read transposed; TB: B stored N x K.
// One wave owns a 16 x 16 output tile; four waves per block stack along M.
// Lane layout of v_mfma_f32_16x16x16_bf16: lane l holds A[l%16][4(l/16)+j],
// B[4(l/16)+j][l%16] and D[4(l/16)+j][l%16], j = 0..3.
// M, N, K are multiples of 16; gridDim.z splits K into chunks of kchunk.
// ---------------------------------------------------------------------------
enum { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_DACT = 2, EPI_PARTIAL = 3 };

struct Epi {
    const float *bias = nullptr;
    float *Z = nullptr;              // pre-activation (optional)
    unsigned short *A = nullptr;     // bf16 activation out
    float *Y = nullptr;              // fp32 output
    const float *Zprev = nullptr;    // pre-activation of the layer below (backward)
    float *dZf = nullptr;            // fp32 gradient out
    unsigned short *dZb = nullptr;   // bf16 gradient out
    float *P = nullptr;              // split-K partials
    long long ldy = 0;               // row stride of Y (floats)
};

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const unsigned short *__restrict__ A, int lda,
                                              const unsigned short *__restrict__ B, int ldb, int M, int N, int K,
                                              int kchunk, Epi e) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = (blockIdx.x * 4 + wave) * 16, n0 = blockIdx.y * 16;
    if (m0 >= M)
        return;
    const int kb = blockIdx.z * kchunk;
    const int ke = min(K, kb + kchunk);
    const int r = lane & 15, g = lane >> 4;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += 16) {
        bf16x4_t a, b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + 4 * g + j;
            const int m = m0 + r, n = n0 + r;
            a[j] = (short)(TA ? A[(long long)k * lda + m] : A[(long long)m * lda + k]);
            b[j] = (short)(TB ? B[(long long)n * ldb + k] : B[(long long)k * ldb + n]);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    const int n = n0 + r;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int m = m0 + 4 * g + j;
        const long long o = (long long)m * N + n;
        const float v = acc[j];
        if constexpr (EPI == EPI_HIDDEN) {
            const float z = v + e.bias[n];
            if (e.Z)
                e.Z[o] = z;
            e.A[o] = f2bf(gelu_f(z));
        } else if constexpr (EPI == EPI_OUT) {
            e.Y[(long long)m * e.ldy + n] = v + e.bias[n];
        } else if constexpr (EPI == EPI_DACT) {
            const float dz = v * gelu_grad_f(e.Zprev[o]);
            e.dZf[o] = dz;
            e.dZb[o] = f2bf(dz);
        } else {
            e.P[(long long)blockIdx.z * M * N + o] = v;
        }
    }
}

template <bool TA, bool TB, int EPI>
static hipError_t gemm(const unsigned short *A, int lda, const unsigned short *B, int ldb, int M, int N, int K,
                       int splits, const Epi &e, hipStream_t s) {
    const int kchunk = ((K / splits + 15) / 16) * 16;
    dim3 grid((M + 63) / 64, N / 16, (K + kchunk - 1) / kchunk);
    k_gemm<TA, TB, EPI><<<grid, 256, 0, s>>>(A, lda, B, ldb, M, N, K, kchunk, e);
    return hipGetLastError();
}

// sum of split-K partials [splits][M][N] into dst (M x N)
__global__ void k_reduce_splits(const float *__restrict__ P, int splits, int MN, float *__restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MN)
        return;
    float s = 0;
#pragma unroll 8
    for (int k = 0; k < splits; ++k)
        s += P[(long long)k * MN + i];
    dst[i] = s;
}

// Column sums of an n x N fp32 matrix (bias gradients), first stage: block b
// sums rows [b rows_per_block, (b + 1) rows_per_block) of every column into
// partial[b][c].  N divides the block size: thread t takes column t % N and
// every (256 / N)-th row, so each row is read as one contiguous run.
constexpr int kColsumBlocks = 128;
static_assert(256 % kNetHidden == 0 && 256 % kNetOut == 0, "layer widths must divide the colsum block");
__global__ __launch_bounds__(256) void k_colsum_part(const float *__restrict__ X, int n, int N, int rows_per_block,
                                                     float *__restrict__ partial) {
    __shared__ float red[256];
    const int t = threadIdx.x, c = t % N, lanes = 256 / N, rl = t / N;
    const int r0 = blockIdx.x * rows_per_block, r1 = min(n, r0 + rows_per_block);
    // four independent sums keep four rows' loads in flight
    float s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int r = r0 + rl;
    for (; r + 3 * lanes < r1; r += 4 * lanes) {
        s0 += X[(long long)r * N + c];
        s1 += X[(long long)(r + lanes) * N + c];
        s2 += X[(long long)(r + 2 * lanes) * N + c];
        s3 += X[(long long)(r + 3 * lanes) * N + c];
    }
    for (; r < r1; r += lanes)
        s0 += X[(long long)r * N + c];
    float s = (s0 + s1) + (s2 + s3);
    red[t] = s;
    __syncthreads();
    if (rl == 0) {
        for (int k = 1; k < lanes; ++k)
            s += red[k * N + c];
        partial[(long long)blockIdx.x * N + c] = s;
    }
}

// dY = 2 (Y - T) / n; per-block partial sums of (Y - T)^2
__global__ void k_mse(const float *__restrict__ Y, const float *__restrict__ T, long long total, float inv_n,
                      float *__restrict__ dYf, unsigned short *__restrict__ dYb, float *__restrict__ part) {
    __shared__ float red[256];
    float s = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const float d = Y[i] - T[i];
        s += d * d;
        const float g = 2.0f * d * inv_n;
        dYf[i] = g;
        dYb[i] = f2bf(g);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = red[0];
}

// Adam on the flat FP32 parameters; refreshes the BF16 weight copies.
__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int n, float lr, float b1, float b2, float eps, float c1, float c2,
                       unsigned short *__restrict__ wb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1 - b1) * gi;
    const float vi = b2 * v[i] + (1 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    wb[i] = f2bf(pi);
}

__global__ void k_to_bf16(const float *__restrict__ x, long long n, unsigned short *__restrict__ y) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        y[i] = f2bf(x[i]);
}

// minibatch gather with a counter-based index stream
__global__ void k_gather_batch(const unsigned short *__restrict__ feat, const float *__restrict__ target,
                               long long nsamples, unsigned long long key, int n, unsigned short *__restrict__ X,
                               float *__restrict__ T) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const long long src = (long long)(splitmix64(key + (unsigned long long)i) % (unsigned long long)nsamples);
#pragma unroll
    for (int k = 0; k < kNetIn; ++k)
        X[(long long)i * kNetIn + k] = feat[src * kNetIn + k];
#pragma unroll 4
    for (int k = 0; k < kNetOut; ++k)
        T[(long long)i * kNetOut + k] = target[src * kNetOut + k];
}

// Training samples of one (scale, wedge) group: features and alpha* targets
// at nx grid points drawn from the group's counter-based stream, or at the
// given flat grid indices xlist when it is not null (feat may then be null).
__global__ void k_make_samples(Phase ph, int N, double theta, double s, const double2 *__restrict__ cols, int r,
                               const double2 *__restrict__ V, double inv_s1, unsigned long long key, int nx,
                               const long long *__restrict__ xlist, unsigned short *__restrict__ feat,
                               float *__restrict__ target) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx)
        return;
    const long long NN = (long long)N * N;
    const long long p = xlist ? xlist[i] : (long long)(splitmix64(key + (unsigned long long)i) % (unsigned long long)NN);
    const double x1 = (double)(p / N) / N, x2 = (double)(p % N) / N;
    const XCoef c = phase_xcoef(ph, x1, x2);
    double g1, g2;
    phase_grad(ph, c, cos(theta), sin(theta), g1, g2);
    double ar[kNetRank], ai[kNetRank];
#pragma unroll
    for (int t = 0; t < kNetRank; ++t)
        ar[t] = ai[t] = 0;
    for (int k = 0; k < r; ++k) {
        double cs, sn;
        residual_entry(ph, c, g1, g2, cols[k].x, cols[k].y, cs, sn);
#pragma unroll
        for (int t = 0; t < kNetRank; ++t) {
            const double2 v = V[k * kNetRank + t];
            ar[t] += cs * v.x - sn * v.y;
            ai[t] += cs * v.y + sn * v.x;
        }
    }
    if (feat) {
        float f[kNetIn];
        net_features(x1, x2, theta, s, f);
#pragma unroll
        for (int k = 0; k < kNetIn; ++k)
            feat[(long long)i * kNetIn + k] = f2bf(f[k]);
    }
#pragma unroll
    for (int t = 0; t < kNetRank; ++t) {
        target[(long long)i * kNetOut + 2 * t] = (float)(ar[t] * inv_s1);
        target[(long long)i * kNetOut + 2 * t + 1] = (float)(ai[t] * inv_s1);
    }
}

// Features of n given grid points (flat indices xs) at scale s; rows n .. npad
// (the padding to a multiple of 64) repeat the last point.
__global__ void k_point_features(int N, const long long *__restrict__ xs, int n, int npad, double theta, double s,
                                 unsigned short *__restrict__ X) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad)
        return;
    const long long p = xs[i < n ? i : n - 1];
    float f[kNetIn];
    net_features((double)(p / N) / N, (double)(p % N) / N, theta, s, f);
#pragma unroll
    for (int k = 0; k < kNetIn; ++k)
        X[(long long)i * kNetIn + k] = f2bf(f[k]);
}

// The leading ncols complex outputs of n rows of network outputs (32 floats
// per row) into dst with row stride ld complex; columns ncols .. ld are zeroed.
__global__ void k_take_factors(const float *__restrict__ Y, long long n, int ncols, int ld, float *__restrict__ dst) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * ld)
        return;
    const long long row = i / ld;
    const int t = (int)(i - row * ld);
    const float re = t < ncols ? Y[row * kNetOut + 2 * t] : 0.0f;
    const float im = t < ncols ? Y[row * kNetOut + 2 * t + 1] : 0.0f;
    dst[2 * i] = re;
    dst[2 * i + 1] = im;
}

// Features of every grid point of one wedge at scale s (inference).
__global__ void k_grid_features(int N, long long x0, int n, double theta, double s, unsigned short *__restrict__ X) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const long long p = x0 + i;
    float f[kNetIn];
    net_features((double)(p / N) / N, (double)(p % N) / N, theta, s, f);
#pragma unroll
    for (int k = 0; k < kNetIn; ++k)
        X[(long long)i * kNetIn + k] = f2bf(f[k]);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
LearnedModel::~LearnedModel() {
    void *bufs[] = {d_p, d_m, d_v, d_g, d_wb, d_feat, d_target, scratch};
    for (void *b : bufs)
        if (b)
            (void)hipFree(b);
}

struct StepBuffers {
    unsigned short *X, *A[3], *dYb, *dZb[2];
    float *T, *Z[3], *Y, *dYf, *dZf[2], *P, *part, *CP;
};

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr int kSplitMax = 32;

static hipError_t ensure_scratch(LearnedModel *M, int n) {
    if (n <= M->batch_cap && M->scratch)
        return hipSuccess;
    if (M->scratch)
        (void)hipFree(M->scratch);
    M->scratch = nullptr;
    const size_t h = (size_t)n * kNetHidden;
    size_t bytes = 0;
    bytes += align256(2 * (size_t)n * kNetIn);                       // X
    bytes += 3 * align256(2 * h);                                    // A1..3
    bytes += align256(2 * (size_t)n * kNetOut);                      // dYb
    bytes += 2 * align256(2 * h);                                    // dZb ping-pong
    bytes += align256(4 * (size_t)n * kNetOut);                      // T
    bytes += 3 * align256(4 * h);                                    // Z1..3
    bytes += 2 * align256(4 * (size_t)n * kNetOut);                  // Y, dYf
    bytes += 2 * align256(4 * h);                                    // dZf ping-pong
    bytes += align256(4 * (size_t)kSplitMax * kNetHidden * kNetHidden);  // split-K partials
    bytes += align256(4 * 4096);                                     // loss partials
    bytes += align256(4 * (size_t)kColsumBlocks * kNetHidden);        // bias-gradient partials
    hipError_t e = hipMalloc(&M->scratch, bytes);
    if (e != hipSuccess)
        return e;
    M->scratch_bytes = bytes;
    M->batch_cap = n;
    return hipSuccess;
}

static StepBuffers carve(LearnedModel *M, int n) {
    StepBuffers b;
    char *p = static_cast<char *>(M->scratch);
    const size_t h = (size_t)n * kNetHidden;
    auto take = [&](size_t bytes) {
        char *q = p;
        p += align256(bytes);
        return q;
    };
    b.X = (unsigned short *)take(2 * (size_t)n * kNetIn);
    for (int i = 0; i < 3; ++i)
        b.A[i] = (unsigned short *)take(2 * h);
    b.dYb = (unsigned short *)take(2 * (size_t)n * kNetOut);
    for (int i = 0; i < 2; ++i)
        b.dZb[i] = (unsigned short *)take(2 * h);
    b.T = (float *)take(4 * (size_t)n * kNetOut);
    for (int i = 0; i < 3; ++i)
        b.Z[i] = (float *)take(4 * h);
    b.Y = (float *)take(4 * (size_t)n * kNetOut);
    b.dYf = (float *)take(4 * (size_t)n * kNetOut);
    for (int i = 0; i < 2; ++i)
        b.dZf[i] = (float *)take(4 * h);
    b.P = (float *)take(4 * (size_t)kSplitMax * kNetHidden * kNetHidden);
    b.part = (float *)take(4 * 4096);
    b.CP = (float *)take(4 * (size_t)kColsumBlocks * kNetHidden);
    return b;
}

// Forward through all layers for n rows of X (bf16 features): hidden
// pre-activations into Z (if store_z), activations into A, output into Y.
static hipError_t forward(LearnedModel *M, const StepBuffers &b, int n, bool store_z, float *Y, long long ldy,
                          hipStream_t s) {
    const unsigned short *in = b.X;
    for (int l = 0; l < 3; ++l) {
        Epi e;
        e.bias = M->d_p + M->offb[l];
        e.Z = store_z ? b.Z[l] : nullptr;
        e.A = b.A[l];
        hipError_t err = gemm<false, false, EPI_HIDDEN>(in, kNetDims[l], M->d_wb + M->offW[l], kNetDims[l + 1], n,
                                                        kNetDims[l + 1], kNetDims[l], 1, e, s);
        if (err != hipSuccess)
            return err;
        in = b.A[l];
    }
    Epi e;
    e.bias = M->d_p + M->offb[3];
    e.Y = Y;
    e.ldy = ldy;
    return gemm<false, false, EPI_OUT>(in, kNetHidden, M->d_wb + M->offW[3], kNetOut, n, kNetOut, kNetHidden, 1, e, s);
}

// Backward of the mean squared error for n rows (after forward with store_z):
// flat gradients into M->d_g; returns the loss through *loss (synchronises).
static hipError_t backward(LearnedModel *M, const StepBuffers &b, int n, double *loss, hipStream_t s) {
    const int nblk = 256;
    k_mse<<<nblk, 256, 0, s>>>(b.Y, b.T, (long long)n * kNetOut, 1.0f / n, b.dYf, b.dYb, b.part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const unsigned short *dZb = b.dYb;
    const float *dZf = b.dYf;
    const int splits = std::min(kSplitMax, std::max(1, n / 256));
    for (int l = 3; l >= 0; --l) {
        const int din = kNetDims[l], dout = kNetDims[l + 1];
        const unsigned short *Ain = l == 0 ? b.X : b.A[l - 1];
        // dW = Ain^T dZ (split over the batch), db = column sums of dZ
        Epi ep;
        ep.P = b.P;
        e = gemm<true, false, EPI_PARTIAL>(Ain, din, dZb, dout, din, dout, n, splits, ep, s);
        if (e != hipSuccess)
            return e;
        const int kchunk = ((n / splits + 15) / 16) * 16;
        const int nsplit = (n + kchunk - 1) / kchunk;
        k_reduce_splits<<<(din * dout + 255) / 256, 256, 0, s>>>(b.P, nsplit, din * dout, M->d_g + M->offW[l]);
        // db: column sums of dZ in two stages (dout divides the block size)
        const int rpb = (n + kColsumBlocks - 1) / kColsumBlocks;
        k_colsum_part<<<kColsumBlocks, 256, 0, s>>>(dZf, n, dout, rpb, b.CP);
        k_reduce_splits<<<(dout + 255) / 256, 256, 0, s>>>(b.CP, kColsumBlocks, dout, M->d_g + M->offb[l]);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        if (l > 0) {
            // dA = dZ W^T, dZ_prev = dA * gelu'(Z_prev)
            Epi ed;
            ed.Zprev = b.Z[l - 1];
            ed.dZf = b.dZf[l & 1];
            ed.dZb = b.dZb[l & 1];
            e = gemm<false, true, EPI_DACT>(dZb, dout, M->d_wb + M->offW[l], dout, n, din, dout, 1, ed, s);
            if (e != hipSuccess)
                return e;
            dZb = b.dZb[l & 1];
            dZf = b.dZf[l & 1];
        }
    }
    if (loss) {
        std::vector<float> part(nblk);
        e = hipMemcpyAsync(part.data(), b.part, nblk * sizeof(float), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess)
            return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return e;
        double sum = 0;
        for (float v : part)
            sum += v;
        *loss = sum / n;
    }
    return hipSuccess;
}

hipError_t learned_infer_wedge(LearnedModel *M, double theta, double s, void *out, int q, int qpad, int precision,
                               hipStream_t st) {
    if (precision != FIO_F32 || q < 1 || q > kNetRank || qpad < q || qpad > kNetRank)
        return hipErrorInvalidValue;
    const long long NN = (long long)M->N * M->N;
    const int chunk = 1 << 16;
    hipError_t e = ensure_scratch(M, chunk);
    if (e != hipSuccess)
        return e;
    StepBuffers b = carve(M, chunk);
    float *Y = static_cast<float *>(out);
    for (long long x0 = 0; x0 < NN; x0 += chunk) {
        const int n = (int)std::min<long long>(chunk, NN - x0);
        const int npad = ((n + 63) / 64) * 64;
        k_grid_features<<<(npad + 255) / 256, 256, 0, st>>>(M->N, x0, npad, theta, s, b.X);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        // the output layer writes the interleaved (re, im) pairs of the 16
        // factors; the leading q are kept, at the plan's padded rank
        if (n == npad && q == kNetRank && qpad == kNetRank) {
            e = forward(M, b, npad, false, Y + x0 * kNetOut, kNetOut, st);
        } else {
            e = forward(M, b, npad, false, b.Y, kNetOut, st);
            if (e == hipSuccess) {
                const long long tot = (long long)n * qpad;
                k_take_factors<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(b.Y, n, q, qpad, Y + x0 * 2 * qpad);
                e = hipGetLastError();
            }
        }
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t learned_infer_points(LearnedModel *M, double theta, double s, const long long *d_x, int n, float *d_out,
                                hipStream_t st) {
    const int chunk = 1 << 16;
    hipError_t e = ensure_scratch(M, chunk);
    if (e != hipSuccess)
        return e;
    StepBuffers b = carve(M, chunk);
    for (int x0 = 0; x0 < n; x0 += chunk) {
        const int m = std::min(chunk, n - x0);
        const int npad = ((m + 63) / 64) * 64;
        k_point_features<<<(npad + 255) / 256, 256, 0, st>>>(M->N, d_x + x0, m, npad, theta, s, b.X);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        e = forward(M, b, npad, false, b.Y, kNetOut, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_out + (size_t)x0 * kNetOut, b.Y, (size_t)m * kNetOut * sizeof(float),
                               hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace fio

using namespace fio;

struct fio_learned_s : LearnedModel {};

static fio_status upload_weights_bf16(LearnedModel *M) {
    k_to_bf16<<<64, 256>>>(M->d_p, M->nparams, M->d_wb);
    FIO_HIP_TRY(hipGetLastError());
    return FIO_OK;
}

static fio_status init_model(LearnedModel *M) {
    int o = 0;
    for (int l = 0; l < kNetLayers; ++l) {
        M->offW[l] = o;
        o += kNetDims[l] * kNetDims[l + 1];
        M->offb[l] = o;
        o += kNetDims[l + 1];
    }
    M->nparams = o;
    FIO_HIP_TRY(hipGetDevice(&M->device));
    FIO_HIP_TRY(hipMalloc(&M->d_p, sizeof(float) * o));
    FIO_HIP_TRY(hipMalloc(&M->d_m, sizeof(float) * o));
    FIO_HIP_TRY(hipMalloc(&M->d_v, sizeof(float) * o));
    FIO_HIP_TRY(hipMalloc(&M->d_g, sizeof(float) * o));
    FIO_HIP_TRY(hipMalloc(&M->d_wb, sizeof(unsigned short) * o));
    FIO_HIP_TRY(hipMemset(M->d_m, 0, sizeof(float) * o));
    FIO_HIP_TRY(hipMemset(M->d_v, 0, sizeof(float) * o));
    // He-normal weights from the seed (Box-Muller on splitmix64 draws), zero biases
    std::vector<float> p(o, 0.0f);
    uint64_t st = splitmix64(M->seed ^ 0xA5A5A5A5ull);
    for (int l = 0; l < kNetLayers; ++l) {
        const double sd = std::sqrt(2.0 / kNetDims[l]);
        for (int i = 0; i < kNetDims[l] * kNetDims[l + 1]; ++i) {
            st = splitmix64(st);
            const double u1 = ((st >> 11) + 1.0) / 9007199254740993.0;
            st = splitmix64(st);
            const double u2 = (st >> 11) / 9007199254740992.0;
            p[M->offW[l] + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(kTwoPi * u2));
        }
    }
    FIO_HIP_TRY(hipMemcpy(M->d_p, p.data(), sizeof(float) * o, hipMemcpyHostToDevice));
    return upload_weights_bf16(M);
}

extern "C" {

fio_status fio_learned_create(int N, const fio_phase *family, int n_wedges, unsigned long long seed,
                              fio_learned_t *out) {
    set_error("");
    if (!out || !family || N < 8 || (N & 1) || N > 4096 || family->kind < 0 || family->kind > 5 || n_wedges < 0)
        return (set_error("bad argument"), FIO_EINVAL);
    *out = nullptr;
    fio_learned_s *M = new (std::nothrow) fio_learned_s();
    if (!M)
        return (set_error("host allocation failed"), FIO_ENOMEM);
    M->N = N;
    M->family.kind = family->kind;
    std::memcpy(M->family.p, family->p, sizeof(M->family.p));
    M->L = n_wedges > 0 ? n_wedges : default_wedge_count(N, M->family);
    M->seed = seed;
    fio_status st = init_model(M);
    if (st != FIO_OK) {
        delete M;
        return st;
    }
    *out = M;
    return FIO_OK;
}

fio_status fio_learned_destroy(fio_learned_t m) {
    delete m;
    return FIO_OK;
}

fio_status fio_learned_params(fio_learned_t m, int get, float *params, int n) {
    set_error("");
    if (!m || !params || n != m->nparams)
        return (set_error("bad argument (n must equal the parameter count)"), FIO_EINVAL);
    if (get) {
        FIO_HIP_TRY(hipMemcpy(params, m->d_p, sizeof(float) * n, hipMemcpyDeviceToHost));
        return FIO_OK;
    }
    FIO_HIP_TRY(hipMemcpy(m->d_p, params, sizeof(float) * n, hipMemcpyHostToDevice));
    FIO_HIP_TRY(hipMemset(m->d_m, 0, sizeof(float) * n));
    FIO_HIP_TRY(hipMemset(m->d_v, 0, sizeof(float) * n));
    m->adam_t = 0;
    return upload_weights_bf16(m);
}

int fio_learned_param_count(void) {
    int o = 0;
    for (int l = 0; l < kNetLayers; ++l)
        o += kNetDims[l] * kNetDims[l + 1] + kNetDims[l + 1];
    return o;
}

fio_status fio_learned_generate(fio_learned_t m, int nscales, const double *scales, int x_samples, int r_cols) {
    set_error("");
    if (!m || nscales < 1 || !scales || x_samples < 64 || r_cols < 16 || r_cols > 256)
        return (set_error("bad argument"), FIO_EINVAL);
    const int N = m->N, L = m->L, h = N / 2;
    const long long NN = (long long)N * N;
    std::vector<int> ids;
    std::vector<double> thetas;
    partition_equiangular(N, L, ids, thetas);
    std::vector<std::vector<int>> members(L);
    for (long long i = 0; i < NN; ++i)
        members[ids[i]].push_back((int)i);
    // samples: all (scale, wedge) groups of x_samples points
    const long long total = (long long)nscales * L * x_samples;
    if (m->d_feat)
        (void)hipFree(m->d_feat);
    if (m->d_target)
        (void)hipFree(m->d_target);
    m->d_feat = nullptr;
    m->d_target = nullptr;
    FIO_HIP_TRY(hipMalloc(&m->d_feat, sizeof(unsigned short) * total * kNetIn));
    FIO_HIP_TRY(hipMalloc(&m->d_target, sizeof(float) * total * kNetOut));
    m->nsamples = total;
    m->cols.assign(L, {});
    m->colk.assign(L, {});
    m->theta = thetas;
    m->V.assign(L, {});
    m->s1.assign(L, 1.0);
    double2 *d_xcoef = nullptr, *d_cols = nullptr, *d_V = nullptr;
    FIO_HIP_TRY(hipMalloc(&d_xcoef, NN * sizeof(double2)));
    struct G {
        std::vector<void *> p;
        ~G() {
            for (void *v : p)
                if (v)
                    (void)hipFree(v);
        }
    } guard;
    guard.p.push_back(d_xcoef);
    FIO_HIP_TRY(hipMalloc(&d_cols, 256 * sizeof(double2)));
    guard.p.push_back(d_cols);
    FIO_HIP_TRY(hipMalloc(&d_V, 256 * kNetRank * sizeof(double2)));
    guard.p.push_back(d_V);
    DeviceScratch scr;
    uint64_t state = splitmix64(m->seed ^ 0xC0FFEEull);
    for (int l = 0; l < L; ++l) {
        const int nm = (int)members[l].size();
        if (nm == 0)
            continue;
        const int r = std::min(r_cols, nm);
        m->cols[l] = sample_members(nm, r, state);
        std::vector<double2> cols(r);
        m->colk[l].resize(2 * (size_t)r);
        for (int c = 0; c < r; ++c) {
            const int om = members[l][m->cols[l][c]];
            cols[c] = make_double2(om / N - h, om % N - h);
            m->colk[l][2 * c] = om / N - h;
            m->colk[l][2 * c + 1] = om % N - h;
        }
        // joint Gram over the training scales
        std::vector<zd> Gsum((size_t)r * r, zd(0, 0));
        for (int si = 0; si < nscales; ++si) {
            Phase ph = m->family;
            ph.p[0] = scales[si];
            std::vector<zd> Gs;
            fio_status gs = gram_of_columns(ph, N, d_xcoef, thetas[l], cols, scr, Gs);
            if (gs != FIO_OK)
                return gs;
            for (size_t k = 0; k < Gs.size(); ++k)
                Gsum[k] += Gs[k];
        }
        std::vector<double> lam;
        std::vector<zd> Vr;
        eigh(r, Gsum, lam, Vr);
        m->s1[l] = std::sqrt(std::max(lam[0], 1e-300) / nscales);
        m->V[l].assign((size_t)r * kNetRank, zd(0, 0));
        for (int c = 0; c < r; ++c)
            for (int t = 0; t < std::min(kNetRank, r); ++t)
                m->V[l][(size_t)c * kNetRank + t] = Vr[(size_t)c * r + t];
        // samples: features and targets, normalised so that the leading factor has unit rms
        FIO_HIP_TRY(hipMemcpy(d_cols, cols.data(), r * sizeof(double2), hipMemcpyHostToDevice));
        FIO_HIP_TRY(hipMemcpy(d_V, m->V[l].data(), (size_t)r * kNetRank * sizeof(double2), hipMemcpyHostToDevice));
        const double inv_s1 = std::sqrt((double)NN) / m->s1[l];
        for (int si = 0; si < nscales; ++si) {
            Phase ph = m->family;
            ph.p[0] = scales[si];
            const long long g = (long long)si * L + l;
            const unsigned long long key = splitmix64(m->seed + 0x9E37ull * (unsigned long long)(g + 1));
            k_make_samples<<<(x_samples + 255) / 256, 256>>>(ph, N, thetas[l], scales[si], d_cols, r, d_V, inv_s1,
                                                             key, x_samples, nullptr,
                                                             m->d_feat + g * x_samples * kNetIn,
                                                             m->d_target + g * x_samples * kNetOut);
            FIO_HIP_TRY(hipGetLastError());
        }
    }
    FIO_HIP_TRY(hipDeviceSynchronize());
    return FIO_OK;
}

fio_status fio_learned_train(fio_learned_t m, int steps, int batch, double lr, double lr_final, double *loss_out) {
    set_error("");
    if (!m || steps < 0 || batch < 64 || (batch % 64) || lr <= 0 || !(lr_final > 0) || !m->d_feat)
        return (set_error("bad argument (batch a multiple of 64; generate data first)"), FIO_EINVAL);
    FIO_HIP_TRY(ensure_scratch(m, batch));
    StepBuffers b = carve(m, batch);
    hipStream_t s = 0;
    double loss = 0;
    for (int it = 0; it < steps; ++it) {
        const unsigned long long key = splitmix64(m->seed * 0x100000001B3ull + (unsigned long long)m->adam_t * 7919u);
        k_gather_batch<<<(batch + 255) / 256, 256, 0, s>>>(m->d_feat, m->d_target, m->nsamples, key, batch, b.X, b.T);
        FIO_HIP_TRY(hipGetLastError());
        FIO_HIP_TRY(forward(m, b, batch, true, b.Y, kNetOut, s));
        const bool want = (it == steps - 1) || (it % 500 == 0);
        FIO_HIP_TRY(backward(m, b, batch, want ? &loss : nullptr, s));
        // cosine decay from lr to lr_final
        const double frac = steps > 1 ? (double)it / (steps - 1) : 1.0;
        const double cur = lr_final + 0.5 * (lr - lr_final) * (1 + std::cos(M_PI * frac));
        m->adam_t += 1;
        const float c1 = (float)(1 - std::pow(0.9, (double)m->adam_t));
        const float c2 = (float)(1 - std::pow(0.999, (double)m->adam_t));
        k_adam<<<(m->nparams + 255) / 256, 256, 0, s>>>(m->d_p, m->d_m, m->d_v, m->d_g, m->nparams, (float)cur, 0.9f,
                                                        0.999f, 1e-8f, c1, c2, m->d_wb);
        FIO_HIP_TRY(hipGetLastError());
    }
    FIO_HIP_TRY(hipDeviceSynchronize());
    m->last_loss = loss;
    if (loss_out)
        *loss_out = loss;
    return FIO_OK;
}

fio_status fio_learned_forward(fio_learned_t m, int n, const float *feat, float *out) {
    set_error("");
    if (!m || n < 1 || !feat || !out)
        return (set_error("bad argument"), FIO_EINVAL);
    const int npad = ((n + 63) / 64) * 64;
    FIO_HIP_TRY(ensure_scratch(m, npad));
    StepBuffers b = carve(m, npad);
    std::vector<float> f((size_t)npad * kNetIn, 0.0f);
    std::memcpy(f.data(), feat, sizeof(float) * (size_t)n * kNetIn);
    float *d_f = nullptr;
    FIO_HIP_TRY(hipMalloc(&d_f, sizeof(float) * f.size()));
    hipError_t e = hipMemcpy(d_f, f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        k_to_bf16<<<64, 256>>>(d_f, (long long)f.size(), b.X);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = forward(m, b, npad, false, b.Y, kNetOut, 0);
    if (e == hipSuccess)
        e = hipMemcpy(out, b.Y, sizeof(float) * (size_t)n * kNetOut, hipMemcpyDeviceToHost);
    (void)hipFree(d_f);
    if (e != hipSuccess)
        return hip_fail(e, "fio_learned_forward");
    return FIO_OK;
}

fio_status fio_learned_grads(fio_learned_t m, int n, const float *feat, const float *target, float *grads,
                             double *loss) {
    set_error("");
    if (!m || n < 64 || (n % 64) || !feat || !target || !grads)
        return (set_error("bad argument (n a multiple of 64)"), FIO_EINVAL);
    FIO_HIP_TRY(ensure_scratch(m, n));
    StepBuffers b = carve(m, n);
    float *d_f = nullptr;
    FIO_HIP_TRY(hipMalloc(&d_f, sizeof(float) * (size_t)n * kNetIn));
    hipError_t e = hipMemcpy(d_f, feat, sizeof(float) * (size_t)n * kNetIn, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        k_to_bf16<<<64, 256>>>(d_f, (long long)n * kNetIn, b.X);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpy(b.T, target, sizeof(float) * (size_t)n * kNetOut, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = forward(m, b, n, true, b.Y, kNetOut, 0);
    if (e == hipSuccess)
        e = backward(m, b, n, loss, 0);
    if (e == hipSuccess)
        e = hipMemcpy(grads, m->d_g, sizeof(float) * m->nparams, hipMemcpyDeviceToHost);
    (void)hipFree(d_f);
    if (e != hipSuccess)
        return hip_fail(e, "fio_learned_grads");
    return FIO_OK;
}

fio_status fio_learned_eval(fio_learned_t m, double *loss) {
    set_error("");
    if (!m || !loss || !m->d_feat)
        return (set_error("bad argument (generate data first)"), FIO_EINVAL);
    const int chunk = 1 << 15;
    FIO_HIP_TRY(ensure_scratch(m, chunk));
    StepBuffers b = carve(m, chunk);
    double sum = 0;
    for (long long x0 = 0; x0 < m->nsamples; x0 += chunk) {
        const int n = (int)std::min<long long>(chunk, m->nsamples - x0);
        if (n % 64)
            break;
        FIO_HIP_TRY(hipMemcpy(b.X, m->d_feat + x0 * kNetIn, sizeof(unsigned short) * n * kNetIn,
                              hipMemcpyDeviceToDevice));
        FIO_HIP_TRY(hipMemcpy(b.T, m->d_target + x0 * kNetOut, sizeof(float) * n * kNetOut,
                              hipMemcpyDeviceToDevice));
        FIO_HIP_TRY(forward(m, b, n, true, b.Y, kNetOut, 0));
        double l = 0;
        FIO_HIP_TRY(backward(m, b, n, &l, 0));
        sum += l * n;
    }
    *loss = sum / (double)m->nsamples;
    return FIO_OK;
}

fio_status fio_learned_basis(fio_learned_t m, int ell, int cap, int *r, double *cols, double *V, double *s1) {
    set_error("");
    if (!m || !r || !s1 || cap < 0 || (cap > 0 && (!cols || !V)))
        return (set_error("bad argument"), FIO_EINVAL);
    if (ell < 0 || ell >= (int)m->colk.size())
        return (set_error("wedge out of range, or no training data generated"), FIO_EINVAL);
    const int rr = (int)m->colk[ell].size() / 2;
    *r = rr;
    *s1 = m->s1[ell];
    if (rr > cap)
        return (set_error("capacity below the column count"), FIO_EINVAL);
    for (int c = 0; c < rr; ++c) {
        cols[2 * c] = m->colk[ell][2 * c];
        cols[2 * c + 1] = m->colk[ell][2 * c + 1];
        for (int t = 0; t < kNetRank; ++t) {
            const zd v = m->V[ell][(size_t)c * kNetRank + t];
            V[2 * ((size_t)c * kNetRank + t)] = v.real();
            V[2 * ((size_t)c * kNetRank + t) + 1] = v.imag();
        }
    }
    return FIO_OK;
}

fio_status fio_learned_targets(fio_learned_t m, int ell, double scale, int nx, const long long *xidx, float *out) {
    set_error("");
    if (!m || nx < 0 || (nx > 0 && (!xidx || !out)))
        return (set_error("bad argument"), FIO_EINVAL);
    if (ell < 0 || ell >= (int)m->colk.size() || m->colk[ell].empty())
        return (set_error("wedge out of range, or no training data generated"), FIO_EINVAL);
    const long long NN = (long long)m->N * m->N;
    for (int i = 0; i < nx; ++i)
        if (xidx[i] < 0 || xidx[i] >= NN)
            return (set_error("grid index out of range"), FIO_EINVAL);
    if (nx == 0)
        return FIO_OK;
    const int r = (int)m->colk[ell].size() / 2;
    std::vector<double2> cols(r);
    for (int c = 0; c < r; ++c)
        cols[c] = make_double2(m->colk[ell][2 * c], m->colk[ell][2 * c + 1]);
    struct G {
        std::vector<void *> p;
        ~G() {
            for (void *v : p)
                if (v)
                    (void)hipFree(v);
        }
    } guard;
    double2 *d_cols = nullptr, *d_V = nullptr;
    long long *d_x = nullptr;
    float *d_t = nullptr;
    FIO_HIP_TRY(hipMalloc(&d_cols, r * sizeof(double2)));
    guard.p.push_back(d_cols);
    FIO_HIP_TRY(hipMalloc(&d_V, (size_t)r * kNetRank * sizeof(double2)));
    guard.p.push_back(d_V);
    FIO_HIP_TRY(hipMalloc(&d_x, sizeof(long long) * nx));
    guard.p.push_back(d_x);
    FIO_HIP_TRY(hipMalloc(&d_t, sizeof(float) * (size_t)nx * kNetOut));
    guard.p.push_back(d_t);
    FIO_HIP_TRY(hipMemcpy(d_cols, cols.data(), r * sizeof(double2), hipMemcpyHostToDevice));
    FIO_HIP_TRY(hipMemcpy(d_V, m->V[ell].data(), (size_t)r * kNetRank * sizeof(double2), hipMemcpyHostToDevice));
    FIO_HIP_TRY(hipMemcpy(d_x, xidx, sizeof(long long) * nx, hipMemcpyHostToDevice));
    Phase ph = m->family;
    ph.p[0] = scale;
    const double inv_s1 = std::sqrt((double)NN) / m->s1[ell];
    k_make_samples<<<(nx + 255) / 256, 256>>>(ph, m->N, m->theta[ell], scale, d_cols, r, d_V, inv_s1, 0ull, nx, d_x,
                                              nullptr, d_t);
    FIO_HIP_TRY(hipGetLastError());
    FIO_HIP_TRY(hipMemcpy(out, d_t, sizeof(float) * (size_t)nx * kNetOut, hipMemcpyDeviceToHost));
    return FIO_OK;
}

fio_status fio_learned_adam_step(fio_learned_t m, const float *grads, double lr) {
    set_error("");
    if (!m || !grads || !(lr > 0))
        return (set_error("bad argument"), FIO_EINVAL);
    FIO_HIP_TRY(hipMemcpy(m->d_g, grads, sizeof(float) * m->nparams, hipMemcpyHostToDevice));
    m->adam_t += 1;
    const float c1 = (float)(1 - std::pow(0.9, (double)m->adam_t));
    const float c2 = (float)(1 - std::pow(0.999, (double)m->adam_t));
    k_adam<<<(m->nparams + 255) / 256, 256>>>(m->d_p, m->d_m, m->d_v, m->d_g, m->nparams, (float)lr, 0.9f, 0.999f,
                                             1e-8f, c1, c2, m->d_wb);
    FIO_HIP_TRY(hipGetLastError());
    FIO_HIP_TRY(hipDeviceSynchronize());
    return FIO_OK;
}

fio_status fio_learned_save(fio_learned_t m, const char *path) {
    set_error("");
    if (!m || !path)
        return (set_error("bad argument"), FIO_EINVAL);
    std::vector<float> p(m->nparams);
    FIO_HIP_TRY(hipMemcpy(p.data(), m->d_p, sizeof(float) * p.size(), hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f)
        return (set_error("cannot open file for writing"), FIO_EINVAL);
    const char magic[8] = {'F', 'I', 'O', 'N', 'E', 'T', '0', '1'};
    int hdr[4] = {m->N, m->L, m->family.kind, m->nparams};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int), 4, f) == 4 &&
              std::fwrite(m->family.p, sizeof(double), 8, f) == 8 &&
              std::fwrite(&m->seed, sizeof(m->seed), 1, f) == 1 &&
              std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok)
        return (set_error("write failed"), FIO_EINVAL);
    return FIO_OK;
}

fio_status fio_learned_load(const char *path, fio_learned_t *out) {
    set_error("");
    if (!path || !out)
        return (set_error("bad argument"), FIO_EINVAL);
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f)
        return (set_error("cannot open file"), FIO_EINVAL);
    char magic[8];
    int hdr[4];
    fio_phase fam;
    unsigned long long seed = 0;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "FIONET01", 8) == 0 &&
              std::fread(hdr, sizeof(int), 4, f) == 4 && std::fread(fam.p, sizeof(double), 8, f) == 8 &&
              std::fread(&seed, sizeof(seed), 1, f) == 1;
    fam.kind = hdr[2];
    std::vector<float> p;
    if (ok && hdr[3] == fio_learned_param_count()) {
        p.resize(hdr[3]);
        ok = std::fread(p.data(), sizeof(float), p.size(), f) == p.size();
    } else {
        ok = false;
    }
    std::fclose(f);
    if (!ok)
        return (set_error("not a network file of this version"), FIO_EINVAL);
    fio_learned_t m = nullptr;
    fio_status st = fio_learned_create(hdr[0], &fam, hdr[1], seed, &m);
    if (st != FIO_OK)
        return st;
    st = fio_learned_params(m, 0, p.data(), (int)p.size());
    if (st != FIO_OK) {
        fio_learned_destroy(m);
        return st;
    }
    *out = m;
    return FIO_OK;
}

}  // extern "C"
