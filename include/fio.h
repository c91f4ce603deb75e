/*
 * fio.h -- C ABI of the MI355X (gfx950) library that applies a discrete
 * Fourier integral operator by the wedge-localised method of Candes,
 * Demanet and Ying, "Fast Computation of Fourier Integral Operators".
 *
 * The operator (Section 1.2, eq. (dfio)), in Egorov form a = 1 (Section 3,
 * eq. (Egorov)):
 *
 *     u(x) = (Lf)(x) = (1/N) sum_{xi in Omega} exp(2 pi i Phi(x, xi)) fhat(xi),
 *     x in X = {(n1/N, n2/N) : 0 <= n1, n2 < N},  Omega = [-N/2, N/2)^2,  N even,
 *
 * with fhat the 1/N-normalised DFT of f (eq. (dft)).  The apply follows the
 * evaluation step of Section 3.4: window fhat onto angular wedges W_ell
 * (Section 1.3), multiply by the separated frequency factors gamma^xi_{ell t},
 * evaluate each term with a type-2 NUFFT at the warped points
 * grad_xi Phi(x, xi_hat_ell) of a sheared, centred box, and combine with the
 * spatial factors gamma^x_{ell t}(x) (eq. (dfioalgo)).  The factors come from
 * the randomized separation of Section 3.2, built by fio_plan.
 *
 * Conventions shared by every entry point:
 *   - Arrays are plain device pointers (HIP device memory on the device that
 *     was current at fio_plan), complex numbers interleaved (re, im).
 *   - fhat: N*N complex, centred: element (k1 + N/2)*N + (k2 + N/2) holds
 *     fhat(k1, k2).  u: N*N complex, row-major: element n1*N + n2 holds
 *     u(n1/N, n2/N).  Batches are B such arrays back to back.
 *   - Element type: complex float (8 bytes) for FIO_F32 plans, complex
 *     double (16 bytes) for FIO_F64 plans.
 *   - stream: a hipStream_t passed as void*; NULL is the null stream.  Apply
 *     calls are asynchronous and stream-ordered; the caller keeps fhat and u
 *     alive until the stream has passed the call.  A plan owns a workspace,
 *     so one plan must not be applied on two streams at once.
 *   - Errors: every call returns a fio_status; nothing throws or aborts
 *     across the ABI.  fio_last_error() returns a thread-local message for
 *     the last failing call of this thread (valid until the next call).
 *   - Ownership: the plan owns all device memory it allocates and frees it
 *     in fio_destroy.  Host arrays passed in are only read during the call.
 */
#ifndef FIO_H
#define FIO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fio_plan_s *fio_plan_t;
typedef struct fio_learned_s *fio_learned_t;

typedef enum {
    FIO_OK = 0,
    FIO_EINVAL = -1,    /* bad argument: odd or too small N, null pointer, tol outside (0,1), ... */
    FIO_ENOMEM = -2,    /* device or host allocation failed */
    FIO_EDEVICE = -3,   /* a HIP call failed (message has the HIP error string) */
    FIO_EACCURACY = -4, /* the separation (exact or forced learned) could not meet the tolerance */
    FIO_ENOTSUP = -5    /* valid but unsupported request (e.g. amplitude kind, tol below 5e-7) */
} fio_status;

/* Phase families Phi(x, xi) = x.xi + h(x, xi), h homogeneous of degree 1 in xi.
 * A phase must be evaluable on the device, so it is a descriptor, not a callback. */
enum {
    FIO_PHASE_LINEAR = 0,        /* h = p0 xi1 + p1 xi2 (translation by (p0, p1)) */
    FIO_PHASE_WAVE = 1,          /* h = p0 |xi| (constant-speed wave, Section 1: p0 = +-c t) */
    FIO_PHASE_ELLIPSE_C1C2 = 2,  /* h = p0 sqrt(c1^2 xi1^2 + c2^2 xi2^2), c1 = (2 + sin 2pi x1 sin 2pi x2)/16,
                                    c2 = (2 + cos 2pi x1 cos 2pi x2)/16 (p0 = phase scale) */
    FIO_PHASE_RADIAL = 3,        /* h = rho(x)|xi|, rho = p0 (1 + p1 sin 2pi x1) */
    FIO_PHASE_PAPER_ELLIPSE = 4, /* Section 4, eq. (nrphase): h = p0 sqrt(r1^2 xi1^2 + r2^2 xi2^2),
                                    r1 = (2+sin 4pi x1)(2+sin 4pi x2)/9, r2 = (2+cos 4pi x1)(2+cos 4pi x2)/9 */
    FIO_PHASE_PAPER_CIRCLE = 5   /* eq. (circlerad): h = p0 r(x)|xi|, r = (3+sin 4pi x1)(3+sin 4pi x2)/16 */
};
typedef struct {
    int kind;
    double p[8];
} fio_phase;

/* Amplitude a(x, xi).  FIO_AMP_ONE: a = 1 (the Egorov form, Section 3).
 * FIO_AMP_BESSEL: the amplitude of the integration along ellipses (Section 4,
 * eq. (ellipses_amp), '+' sign), a = (1/4pi)(J0(2 pi rho) + i Y0(2 pi rho))
 * exp(-2 pi i rho) with rho = h(x, xi), for phases with h >= 0 (kinds 1-5 with
 * p0 >= 0, and |p1| <= 1 for kind 3; FIO_EINVAL otherwise); a(x, 0) = 0, since
 * Y0 is singular at 0 and the paper states no value there.  The amplitude is
 * folded into the separated kernel a exp(2 pi i Phi_ell) of every wedge, as
 * Section 4 describes.  Plans with FIO_AMP_BESSEL do not use a learned
 * network.  Other kinds give FIO_ENOTSUP. */
enum { FIO_AMP_ONE = 0, FIO_AMP_BESSEL = 1 };
typedef struct {
    int kind;
    double p[4];
} fio_amplitude;

enum { FIO_F32 = 0, FIO_F64 = 1 };
enum { FIO_PART_EQUIANGULAR = 0, FIO_PART_CORONAE = 1 };
/* Factor modes.  STORED keeps gamma^x for every grid point (N^2 q complex per
 * wedge); REGEN keeps only the compressed factors of eq. (probnewfac), the
 * sampled columns C and Z = V S^-1 (reduced to about rank-many columns C' by
 * an interpolative decomposition, A(:, C) ~ A(:, C') W, Z' = W Z, where the
 * s x s estimate accepts it), and the apply recomputes
 * gamma^x(x) = A(x, C') Z' from the residual phase (Section 3.2, the
 * storage-compressed form): far less memory, more arithmetic per apply, and
 * available while the padded rank is at most 16 (FP32) or 8 (FP64); FP32
 * plans regenerate gamma^x in FP32 (phases reduced in FP64) and take the
 * amplitude a = 1 only (FIO_ENOTSUP otherwise);
 * LEARNED takes gamma^x from a trained network; TAYLOR builds both factors by
 * the deterministic preprocessing of Section 3.1 (polar Taylor expansion of
 * the residual phase, truncated exponential series, QR and SVD compression
 * of the products; FP64 on the GPU with rocBLAS), stored like STORED, for
 * the amplitude a = 1 only (FIO_ENOTSUP otherwise); FIO_EACCURACY where a
 * wedge reaches past the polar series' radius of convergence (the nearest
 * complex singularity of the residual phase in the angle, about 0.11 rad for
 * the paper's ellipse family) or the series needs more than 31 orders: more
 * wedges then help.  Its plans are not written to plan files (FIO_ENOTSUP). */
enum {
    FIO_FACTORS_AUTO = 0,
    FIO_FACTORS_STORED = 1,
    FIO_FACTORS_REGEN = 2,
    FIO_FACTORS_LEARNED = 3,
    FIO_FACTORS_TAYLOR = 4
};

/* Plan options.  Start from fio_default_options(); zero means "automatic" where noted. */
typedef struct {
    int precision;          /* FIO_F32 (default): FP32 data, FFT and combine, FP64 phase and points;
                               FIO_F64: FP64 throughout */
    int partition;          /* FIO_PART_EQUIANGULAR (Section 1.3) or FIO_PART_CORONAE (dyadic rings) */
    int n_wedges;           /* equiangular wedge count L; 0 = automatic: the network's L when a learned
                               network of the same N is given, else L ~ sqrt(N) (Section 1.3) raised for
                               strong phases: the multiple of 8 at least 8 ceil(sqrt(N) / 8) and
                               pi sqrt(S N / (1.5 sqrt 2)), S = max |grad_xi h| of the family */
    int factor_mode;        /* FIO_FACTORS_AUTO / STORED / REGEN (randomized separation) / LEARNED (network) /
                               TAYLOR (deterministic expansion) */
    unsigned long long seed;/* seed of the column/row sampling of the separation */
    int max_batch;          /* right-hand sides processed per pass of the workspace (default 8) */
    double sep_tol_frac;    /* separation threshold = tol * sep_tol_frac (default 0.25) */
    double nufft_tol_frac;  /* NUFFT kernel tolerance = tol * nufft_tol_frac (default 0.1) */
    double sigma;           /* NUFFT oversampling factor; 0 = 2.0 */
    int kernel_width;       /* NUFFT kernel width w in fine cells; 0 = from the tolerance */
    int r0;                 /* initial column/row sample count of the separation; 0 = 32 */
    int verify_samples;     /* s of the s x s separation-error estimate (Section 4); 0 = 200 */
    const void *learned;    /* fio_learned_t handle for FIO_FACTORS_LEARNED / AUTO, or NULL */
    double learned_scale;   /* phase-scale input of the network (the family's p0) */
} fio_options;

typedef struct {
    int N, L, precision, factor_mode, kernel_width, max_rank, min_rank, fallback;
    double sigma, tol, plan_ms, max_sep_error;
    long long fine_cells;      /* sum over wedges of n1*n2 */
    long long box_cells;       /* sum over wedges of B1*B2 */
    long long factor_bytes;    /* device bytes of stored factors */
    long long workspace_bytes; /* device bytes of the per-batch workspace */
    long long compressed_bytes;/* bytes of the compressed factors (V S^-1 and U_R^+, eq. (probnewfac)) */
    double learned_sep_error;  /* largest separation-error estimate of the learned attempt (0: none) */
    double learned_ms;         /* time of the learned attempt: inference, refit and estimate */
} fio_plan_info_t;

typedef struct {
    double theta;        /* centre angle of the wedge */
    int members;         /* |W_ell| */
    int rank;            /* q_ell, the separation rank */
    int samples;         /* r, the accepted column/row sample count */
    int M[4];            /* integer shear, row-major: xi' = M xi - xi_c (Section 3.4) */
    int xi_c[2];         /* translation */
    int box[2];          /* B1, B2: extent of the sheared, centred box */
    int lo[2];           /* centred frequency of box index 0 in each axis */
    int fine[2];         /* n1, n2: oversampled FFT grid */
    double sep_error;    /* estimated relative separation error on a random s x s submatrix */
} fio_wedge_info_t;

void fio_default_options(fio_options *opt);

/* Build a plan (Section 3.2 preprocessing: partition, shears, NUFFT set-up,
 * randomized separation with adaptive r, factor storage).  tol is the target
 * relative l2 error of the apply, at least 5e-7 in either precision (the
 * separation reads singular values off the FP64 Gram matrix of the sampled
 * columns), else FIO_ENOTSUP.  FIO_EACCURACY if a wedge's separation error
 * estimate stays above tol after the verification retries.  On success *out
 * owns device memory, among it the interpolation window of every 16 x 16
 * output tile on every wedge (32 bytes each), recorded once here so that the
 * applies read it. */
fio_status fio_plan(int N, const fio_phase *phase, const fio_amplitude *amp, double tol, fio_plan_t *out);
fio_status fio_plan_ex(int N, const fio_phase *phase, const fio_amplitude *amp, double tol,
                       const fio_options *opt /* nullable */, fio_plan_t *out);

/* Plan files.  fio_plan_save writes the plan's build inputs (N, phase, tol,
 * options) and, per wedge, the compressed factors of its randomized
 * separation (Section 3.2, eq. (probnewfac): sampled columns and rows,
 * Z = V S^-1, U_[R]^+, rank and error estimate) to a little-endian binary file
 * with a checksum; the caller owns the path.  fio_plan_load rebuilds the
 * geometry, checks it against the file and evaluates the factors on the
 * current device, skipping the sampling and the eigen-solves: the loaded plan
 * applies bit for bit like the saved one and is owned by the caller (release
 * with fio_destroy).  FIO_ENOTSUP for a plan with learned factors (save its
 * network with fio_learned_save instead); FIO_EINVAL for an unreadable,
 * truncated or corrupted file, or one whose geometry this library does not
 * reproduce. */
fio_status fio_plan_save(fio_plan_t plan, const char *path);
fio_status fio_plan_load(const char *path, fio_plan_t *out);

/* u = L fhat for one right-hand side (Section 3.4, eq. (dfioalgo)). */
fio_status fio_apply(fio_plan_t plan, const void *fhat, void *u, void *stream);

/* B right-hand sides, fhat and u holding B arrays each; the factors, warped
 * points and kernel weights are shared across the batch. */
fio_status fio_apply_batch(fio_plan_t plan, int B, const void *fhat, void *u, void *stream);

/* The adjoint (Section 3.5): the Fourier coefficients of L*g,
 *     hhat(xi) = (1/N) sum_{y in X} conj(a(y, xi)) exp(-2 pi i Phi(y, xi)) g(y),  xi in Omega,
 * for g on the grid X (row-major, like u) and hhat centred (like fhat): the
 * conjugate transpose of the map fio_apply computes, so that
 * <L fhat, g> = <fhat, L* g>.  It runs the algorithm of Section 3.5 with the
 * plan's wedges, separated factors, grids and kernel (type-1 NUFFT: spreading
 * of conj(gamma^x) g onto each wedge's oversampled grid, the transposed FFT
 * stages, and the sum over ranks with conj(gamma^xi)); the computed map is the
 * exact adjoint of the computed forward map up to rounding.  An inverse 2-D
 * DFT of hhat gives (L*g)(x).  It uses the plan's workspace, so a plan runs
 * one forward or adjoint apply at a time.  B right-hand sides are back to
 * back, as in fio_apply_batch.  The first adjoint call on a plan also lists,
 * for every 4 x 8 cell strip of each wedge's grid, the grid points whose
 * stencils touch it, in point order (about 12 bytes per grid point and wedge
 * of device memory at kernel width 5, owned by the plan); that call
 * synchronises the device.  The spreading sums every cell in list order;
 * only where a wedge's transformed rows are split into chunks of ranks are
 * the chunks added with floating-point atomics, so the last bits of such
 * plans can differ between runs. */
fio_status fio_apply_adjoint(fio_plan_t plan, const void *g, void *hhat, void *stream);
fio_status fio_apply_adjoint_batch(fio_plan_t plan, int B, const void *g, void *hhat, void *stream);

/* fio_apply_batch for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * It calls no allocating routine: the row-stage output and the oversampled
 * grids, which fio_apply_batch keeps in the plan's workspace, live in a fixed
 * 128 MiB device array of the library instead (one per device, held until
 * the process ends).  Same kernels and results as fio_apply_batch, bit for
 * bit.  Right-hand sides are processed in as many passes as the array needs;
 * FIO_EINVAL if one right-hand side does not fit (about N <= 256 at tol 1e-4
 * fits).  Every call on a device shares that device's array: calls that
 * overlap on one device (two streams, two threads) race and must not be
 * issued.  The plan's own workspace is not touched. */
fio_status fio_apply_batch_noalloc(fio_plan_t plan, int B, const void *fhat, void *u, void *stream);

/* n instances of possibly different N (each its own plan, all of one
 * precision), instance i with B[i] right-hand sides at fhat[i] -> u[i] (host
 * arrays of device pointers).  All instances, wedges and right-hand sides run
 * in one launch of each stage; the launch sequence is captured into a HIP
 * graph that is replayed while the plans and batch sizes stay the same (new
 * pointers refresh its argument table).  Instances of different kernel
 * widths share the interpolation launch of the widest; its windows (32 bytes
 * per output tile and wedge of every instance) are recorded when the graph is
 * built and held with it.  Instances run one after another instead when their
 * factor modes differ, B[i] exceeds plan i's max_batch, or a plan appears more
 * than once in the list (its one workspace cannot hold two instances at
 * once). */
fio_status fio_apply_multi(int n, const fio_plan_t *plans, const void *const *fhat, void *const *u,
                           const int *B, void *stream);

/* Partial operator sum_{l0 <= ell < l1} L_ell (Section 1.3), for per-wedge checks. */
fio_status fio_apply_wedges(fio_plan_t plan, int l0, int l1, int B, const void *fhat, void *u, void *stream);

fio_status fio_plan_info(fio_plan_t plan, fio_plan_info_t *out);
fio_status fio_wedge_info(fio_plan_t plan, int ell, fio_wedge_info_t *out);

/* Host copy of the wedge id of every frequency (N*N int32, centred layout). */
fio_status fio_wedge_map(fio_plan_t plan, int *ids_out);

/* Separated factors of wedge ell evaluated in FP64 from the plan's compressed
 * form (eq. (probnewfac)): gx[i*q + t] = gamma^x_{ell t}(x_i) for the nx flat
 * grid indices xidx[i]; gxi[j*q + t] = gamma^xi_{ell t}(xi_j) for the nxi flat
 * centred indices xiidx[j] (which must lie in W_ell).  Host arrays of
 * complex double; q from fio_wedge_info.  Either side may be skipped with n = 0. */
fio_status fio_wedge_factors(fio_plan_t plan, int ell, int nx, const long long *xidx, double *gx,
                             int nxi, const long long *xiidx, double *gxi);

/* Warped points y = grad_xi Phi(x, xi_hat_ell) (FP64, computed by the same
 * device code the apply uses) for nx flat grid indices: y[2i], y[2i+1]. */
fio_status fio_wedge_warp(fio_plan_t plan, int ell, int nx, const long long *xidx, double *y);

/* Per-stage timing with HIP events recorded on the apply stream around each
 * kernel launch (stage 0: window + row FFT, 1: column FFT, 2: interpolate +
 * combine).  fio_profile(plan, 1) starts recording (and clears the totals);
 * fio_profile_read waits for the recorded events and returns, per stage, the
 * summed milliseconds and the number of launches.  Profiling adds one event
 * pair per launch; it is off by default. */
fio_status fio_profile(fio_plan_t plan, int on);
fio_status fio_profile_read(fio_plan_t plan, double ms[3], long long launches[3]);

fio_status fio_destroy(fio_plan_t plan);

const char *fio_last_error(void);

/* Host linear algebra of the plan, exported for CPU tests (no device use):
 * Hermitian eigen-decomposition of an n x n complex double matrix (row-major,
 * interleaved) by Householder tridiagonalisation and implicit QL; w: n
 * eigenvalues in descending order, V: n x n eigenvectors as columns
 * (row-major). */
fio_status fio_host_eigh(int n, const double *A, double *w, double *V);
/* Column interpolative decomposition of an m x n complex double matrix A
 * (row-major, interleaved) by Householder QR with column pivoting, stopped
 * at a remaining column norm of tol times the first pivot's (the reduction
 * of FIO_FACTORS_REGEN's columns).  *k receives the number of kept columns;
 * perm (n) the column order, kept columns first; T (k x (n - k) complex,
 * row-major; room for n x n) with A(:, perm[k..n)) ~ A(:, perm[0..k)) T.
 * FIO_EINVAL on bad sizes or null pointers. */
fio_status fio_host_column_id(int m, int n, const double *A, double tol, int *k, int *perm, double *T);

/* Relative l2 error (the Section 4 estimator) of a computed u = L fhat at
 * nsamples grid points drawn from `seed`, against an FP64 direct summation of
 * eq. (dfio) on the device.  fhat, u: device arrays of the plan's precision
 * (one right-hand side).  Synchronises the stream. */
fio_status fio_probe_error(fio_plan_t plan, const void *fhat, const void *u, int nsamples, unsigned long long seed,
                           double *err, void *stream);

/* Plain device-to-device copy of `bytes` (a multiple of 16; both pointers
 * 16-byte aligned, device memory, non-overlapping) as one kernel launch on
 * `stream`, asynchronous.  It is a measurement aid: its event time gives the
 * achievable HBM bandwidth and its hardware byte counters calibrate those of
 * the apply kernels.  FIO_EINVAL on a null or misaligned argument. */
fio_status fio_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Autotuner.  Builds candidate plans over the wedge count (L0 - 8 .. L0 + 16),
 * the oversampling factor (1.5, 1.75, 2, 2.5), the split of tol between
 * separation and NUFFT and the kernel width (the bound's and one below),
 * times an apply of B right-hand sides with HIP events and probes its error
 * at 256 points with fio_probe_error; *best is the fastest candidate whose
 * error is at most 0.8 tol.  If the environment variable FIO_TUNE_CACHE names a file, a
 * cached choice for the same problem is returned without tuning and new
 * choices are appended.  Copy best's fields into fio_options to use them. */
typedef struct {
    int n_wedges;
    double sigma;
    int kernel_width;
    double sep_tol_frac, nufft_tol_frac;
    double ms_per_rhs;   /* measured apply time per right-hand side */
    double error;        /* probed relative l2 error */
} fio_tune_result_t;
fio_status fio_autotune(int N, const fio_phase *phase, const fio_amplitude *amp, double tol,
                        const fio_options *base /* nullable */, int B, fio_tune_result_t *tried, int max_tried,
                        int *ntried, fio_tune_result_t *best);

/* ---------------------------------------------------------------------------
 * Learned spatial factors.  A network maps (x1, x2, theta_ell, s) through a
 * fixed periodic feature map (16 inputs), three hidden layers of width 128
 * (tanh form of GELU) and 32 outputs to 16 complex spatial factors alpha_t(x)
 * of wedge ell at phase scale s (the family's p0).  Weights are FP32 masters
 * fed to the BF16 matrix cores with FP32 accumulation; training and inference
 * run on the device that is current at creation.  Its targets are the
 * factors of the randomized separation (Section 3.2) with one column sample
 * per wedge shared by all training scales: alpha*_s(x) = A_s(x, C) V / s1,
 * V the leading 16 eigenvectors of the Gram matrix of A_s(:, C) summed over
 * the scales.  A plan built with opt.learned = this network (factor_mode
 * AUTO or LEARNED, equiangular wedges, FP32, same N, wedge count and phase
 * kind) takes gamma^x from the network and refits gamma^xi = alpha_[R]^+ A_[R]
 * on sampled rows; if an s x s estimate of the separation error exceeds half
 * the tolerance, AUTO falls back to the exact separation (fio_plan_info's
 * fallback flag) and LEARNED fails with FIO_EACCURACY.
 * ------------------------------------------------------------------------- */
fio_status fio_learned_create(int N, const fio_phase *family, int n_wedges /* 0 = default L */,
                              unsigned long long seed, fio_learned_t *out);
/* Training data: x_samples grid points per (scale, wedge), r_cols sampled columns per wedge. */
fio_status fio_learned_generate(fio_learned_t m, int nscales, const double *scales, int x_samples, int r_cols);
/* Adam on minibatches of `batch` samples (a multiple of 64), learning rate
 * decaying from lr to lr_final on a cosine; *final_loss = last minibatch loss. */
fio_status fio_learned_train(fio_learned_t m, int steps, int batch, double lr, double lr_final, double *final_loss);
/* Mean loss over the current training data (e.g. generated for held-out scales). */
fio_status fio_learned_eval(fio_learned_t m, double *loss);
/* Read (get = 1) or write (get = 0) the FP32 parameters: W1, b1, ..., W4, b4,
 * W row-major [in][out]; n must equal fio_learned_param_count(). */
fio_status fio_learned_params(fio_learned_t m, int get, float *params, int n);
int fio_learned_param_count(void);
/* Forward pass on n feature rows (host arrays, n x 16 in, n x 32 out). */
fio_status fio_learned_forward(fio_learned_t m, int n, const float *feat, float *out);
/* One backward pass of the mean squared error on n rows (n a multiple of 64):
 * flat gradients in the parameter order (no update) and the loss. */
fio_status fio_learned_grads(fio_learned_t m, int n, const float *feat, const float *target, float *grads,
                             double *loss);
/* Introspection of the training targets (for checks against a CPU model).
 * fio_learned_basis: host copy of wedge ell's column sample C (cols[2c],
 * cols[2c+1] = centred frequency (k1, k2) of column c), of the joint right
 * singular vectors V (r x 16 complex, row-major, interleaved) and of s1, the
 * leading joint singular value per scale (sqrt of the Gram matrix's largest
 * eigenvalue over the scale count); *r = column count.  cap is the capacity
 * of cols (2 cap doubles) and V (32 cap doubles); FIO_EINVAL if r > cap or
 * no data was generated.
 * fio_learned_targets: the targets alpha*_s(x) = A_s(x, C) V sqrt(N^2) / s1
 * (the residual kernel exp(2 pi i Phi_ell) of Section 3.2 at scale s) at nx
 * given flat grid indices, out[i*32 + 2t], out[i*32 + 2t + 1] = re, im of
 * factor t, computed by the kernel that generates the training data. */
fio_status fio_learned_basis(fio_learned_t m, int ell, int cap, int *r, double *cols, double *V, double *s1);
fio_status fio_learned_targets(fio_learned_t m, int ell, double scale, int nx, const long long *xidx, float *out);
/* One Adam update (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step
 * count kept by the network and reset by fio_learned_params) of the FP32
 * parameters with the given flat gradients (host, parameter order), by the
 * kernel the training loop uses. */
fio_status fio_learned_adam_step(fio_learned_t m, const float *grads, double lr);
fio_status fio_learned_save(fio_learned_t m, const char *path);
fio_status fio_learned_load(const char *path, fio_learned_t *out);
fio_status fio_learned_destroy(fio_learned_t m);

/* Library version string. */
const char *fio_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FIO_H */
