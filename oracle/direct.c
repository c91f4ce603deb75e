/*
 * Oracle -- TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link,
 * load or call this file; it exists so that tests, the smoke check and the
 * CPU baseline of the benchmark can compare against a plain, slow, obviously
 * correct computation.  It shares no code with the HIP library.
 *
 * Plain FP64 direct summation of the discrete Fourier integral operator of
 * Section 1.2, eq. (dfio):
 *
 *     (Lf)(x) = (1/N) sum_{xi in Omega} a(x,xi) exp(2 pi i Phi(x,xi)) fhat(xi),
 *
 * with X = {(n1/N, n2/N)}, Omega = [-N/2, N/2)^2, a = 1 (the Egorov form of
 * Section 3, eq. (Egorov)) or the Bessel amplitude of Section 4 (see
 * oracle_amp), and Phi(x,xi) = x.xi + h(x,xi) with h
 * homogeneous of degree one in xi.  The phase families are:
 *   0 linear shift   h = p0 xi1 + p1 xi2               (exact translation)
 *   1 wave           h = p0 |xi|                       (Section 1, Phi_pm = x.xi +- c|xi|t)
 *   2 c1/c2 ellipse  h = p0 sqrt(c1^2 xi1^2 + c2^2 xi2^2),
 *                    c1 = (2 + sin 2pi x1 sin 2pi x2)/16, c2 = (2 + cos 2pi x1 cos 2pi x2)/16
 *   3 radial         h = rho(x)|xi|, rho = p0 (1 + p1 sin 2pi x1)
 *   4 paper ellipse  h = p0 sqrt(r1^2 xi1^2 + r2^2 xi2^2)  (Section 4, eq. (nrphase)),
 *                    r1 = (2+sin 4pi x1)(2+sin 4pi x2)/9, r2 = (2+cos 4pi x1)(2+cos 4pi x2)/9
 *   5 paper circle   h = p0 r(x)|xi|, r = (3+sin 4pi x1)(3+sin 4pi x2)/16  (eq. (circlerad))
 *
 * Arithmetic: x.xi mod 1 is formed exactly in integers ((n1 k1 + n2 k2) mod N)/N;
 * h is FP64; the total phase is reduced by its nearest integer before
 * sin/cos(2 pi r); accumulation is FP64, summed per frequency row first.
 *
 * ORACLE_PLANT (tests only): compiling with -DORACLE_PLANT=1..6 plants a
 * known mistake (flipped sign of h / dropped 1/N / swapped x1, x2 in h /
 * sin and cos exchanged in c1, c2 / 2 pi for 4 pi in r1, r2 / the adjoint
 * without the conjugation) so that a test can show the pins catch it.  The
 * default build plants nothing.
 */
#include <math.h>
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static const double TWO_PI = 6.283185307179586476925286766559;

/* h(x, xi) for one family (see header). */
static double oracle_h(int kind, const double *p, double x1, double x2, double k1, double k2)
{
    switch (kind) {
    case 0:
        return p[0] * k1 + p[1] * k2;
    case 1:
        return p[0] * sqrt(k1 * k1 + k2 * k2);
    case 2: {
#if defined(ORACLE_PLANT) && ORACLE_PLANT == 4
        double c1 = (2.0 + cos(TWO_PI * x1) * cos(TWO_PI * x2)) / 16.0;
        double c2 = (2.0 + sin(TWO_PI * x1) * sin(TWO_PI * x2)) / 16.0;
#else
        double c1 = (2.0 + sin(TWO_PI * x1) * sin(TWO_PI * x2)) / 16.0;
        double c2 = (2.0 + cos(TWO_PI * x1) * cos(TWO_PI * x2)) / 16.0;
#endif
        return p[0] * sqrt(c1 * c1 * k1 * k1 + c2 * c2 * k2 * k2);
    }
    case 3: {
        double rho = p[0] * (1.0 + p[1] * sin(TWO_PI * x1));
        return rho * sqrt(k1 * k1 + k2 * k2);
    }
    case 4: {
#if defined(ORACLE_PLANT) && ORACLE_PLANT == 5
        double r1 = (2.0 + sin(TWO_PI * x1)) * (2.0 + sin(TWO_PI * x2)) / 9.0;
        double r2 = (2.0 + cos(TWO_PI * x1)) * (2.0 + cos(TWO_PI * x2)) / 9.0;
#else
        double r1 = (2.0 + sin(2.0 * TWO_PI * x1)) * (2.0 + sin(2.0 * TWO_PI * x2)) / 9.0;
        double r2 = (2.0 + cos(2.0 * TWO_PI * x1)) * (2.0 + cos(2.0 * TWO_PI * x2)) / 9.0;
#endif
        return p[0] * sqrt(r1 * r1 * k1 * k1 + r2 * r2 * k2 * k2);
    }
    case 5: {
        double r = (3.0 + sin(2.0 * TWO_PI * x1)) * (3.0 + sin(2.0 * TWO_PI * x2)) / 16.0;
        return p[0] * r * sqrt(k1 * k1 + k2 * k2);
    }
    default:
        return NAN;
    }
}

/*
 * Amplitudes a(x, xi).  0: a = 1 (the Egorov form).  1: the Bessel amplitude
 * of the integration along ellipses (Section 4, eq. (ellipses_amp), the '+'
 * sign), a = (1/4pi) (J0(2 pi rho) + i Y0(2 pi rho)) exp(-2 pi i rho) with
 * rho = h(x, xi) >= 0, taken as 0 at xi = 0, where Y0 is singular and the
 * paper states no value.  J0 and Y0 are the C library's.
 */
static void oracle_amp(int amp, double hv, double k1, double k2, double *ar, double *ai)
{
    if (amp == 0) {
        *ar = 1.0;
        *ai = 0.0;
        return;
    }
    if (k1 == 0.0 && k2 == 0.0) {
        *ar = *ai = 0.0;
        return;
    }
    const double z = TWO_PI * hv;
    const double jr = j0(z), yi = y0(z);
    const double r = hv - rint(hv);
    const double c = cos(TWO_PI * r), sn = -sin(TWO_PI * r);
    const double s4 = 1.0 / (2.0 * TWO_PI);
    *ar = s4 * (jr * c - yi * sn);
    *ai = s4 * (jr * sn + yi * c);
}

/* a only, for tests of the amplitude: out[2i], out[2i+1] = a(x_i, xi_i). */
void oracle_amp_batch(int kind, const double *p, int amp, int n, const double *x1, const double *x2,
                      const double *k1, const double *k2, double *out)
{
    for (int i = 0; i < n; ++i)
        oracle_amp(amp, oracle_h(kind, p, x1[i], x2[i], k1[i], k2[i]), k1[i], k2[i], out + 2 * i, out + 2 * i + 1);
}

/* h only, for tests of the phase families: out[i] = h(x_i, xi_i). */
void oracle_h_batch(int kind, const double *p, int n, const double *x1, const double *x2,
                    const double *k1, const double *k2, double *out)
{
    for (int i = 0; i < n; ++i)
        out[i] = oracle_h(kind, p, x1[i], x2[i], k1[i], k2[i]);
}

/*
 * u[s*nrhs + b] = (1/N) sum_{xi in Omega} exp(2 pi i Phi(x_s, xi)) fhat_b(xi)
 *
 *   xidx  : ns flat grid indices n1*N + n2
 *   fhat  : nrhs arrays of N*N complex (interleaved re, im), centred layout
 *           index (k1 + N/2)*N + (k2 + N/2)
 *   member: optional N*N int array (centred layout) and wedge id `only`;
 *           if member != NULL, only xi with member[xi] == only are summed
 *           (the wedge-restricted operator L_ell of Section 1.3)
 *   u     : ns*nrhs complex (interleaved) output
 * Returns 0, or -1 on bad arguments.
 */
int oracle_direct_amp(int N, int kind, const double *p, int amp, int ns, const int64_t *xidx, int nrhs,
                      const double *fhat, const int32_t *member, int only, double *u, int nthreads)
{
    if (N <= 0 || (N & 1) || ns < 0 || nrhs <= 0 || nrhs > 64)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const int h = N / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < ns; ++s) {
        const int64_t n1 = xidx[s] / N, n2 = xidx[s] % N;
        const double x1 = (double)n1 / N, x2 = (double)n2 / N;
        double acc_re[64], acc_im[64];
        for (int b = 0; b < nrhs; ++b)
            acc_re[b] = acc_im[b] = 0.0;
        for (int k1 = -h; k1 < h; ++k1) {
            double row_re[64], row_im[64];
            for (int b = 0; b < nrhs; ++b)
                row_re[b] = row_im[b] = 0.0;
            for (int k2 = -h; k2 < h; ++k2) {
                const int64_t cell = (int64_t)(k1 + h) * N + (k2 + h);
                if (member && member[cell] != only)
                    continue;
                /* x.xi mod 1 exactly: ((n1 k1 + n2 k2) mod N) / N */
                int64_t ip = (n1 * k1 + n2 * k2) % N;
                if (ip < 0)
                    ip += N;
#if defined(ORACLE_PLANT) && ORACLE_PLANT == 3
                const double hv = oracle_h(kind, p, x2, x1, (double)k1, (double)k2);
#else
                const double hv = oracle_h(kind, p, x1, x2, (double)k1, (double)k2);
#endif
#if defined(ORACLE_PLANT) && ORACLE_PLANT == 1
                double ph = (double)ip / N - hv;
#else
                double ph = (double)ip / N + hv;
#endif
                double r = ph - rint(ph);
                double c = cos(TWO_PI * r), sn = sin(TWO_PI * r);
                if (amp) {
                    double ar, ai;
                    oracle_amp(amp, hv, (double)k1, (double)k2, &ar, &ai);
                    const double cr = c * ar - sn * ai, ci = c * ai + sn * ar;
                    c = cr;
                    sn = ci;
                }
                for (int b = 0; b < nrhs; ++b) {
                    const double *f = fhat + 2 * ((int64_t)b * N * N + cell);
                    row_re[b] += c * f[0] - sn * f[1];
                    row_im[b] += c * f[1] + sn * f[0];
                }
            }
            for (int b = 0; b < nrhs; ++b) {
                acc_re[b] += row_re[b];
                acc_im[b] += row_im[b];
            }
        }
#if defined(ORACLE_PLANT) && ORACLE_PLANT == 2
        const double scale = 1.0;
#else
        const double scale = 1.0 / N;
#endif
        for (int b = 0; b < nrhs; ++b) {
            u[2 * ((int64_t)s * nrhs + b)] = acc_re[b] * scale;
            u[2 * ((int64_t)s * nrhs + b) + 1] = acc_im[b] * scale;
        }
    }
    return 0;
}

/* The Egorov form a = 1. */
int oracle_direct(int N, int kind, const double *p, int ns, const int64_t *xidx, int nrhs, const double *fhat,
                  const int32_t *member, int only, double *u, int nthreads)
{
    return oracle_direct_amp(N, kind, p, 0, ns, xidx, nrhs, fhat, member, only, u, nthreads);
}

/*
 * Adjoint (Section 3.5): the Fourier coefficients of L*g,
 *
 *   hhat[s*nrhs + b] = (1/N) sum_{y in X} exp(-2 pi i Phi(y, xi_s)) g_b(y),
 *
 * the conjugate transpose of the operator above as a map from fhat on Omega
 * to u on X.
 *   xiidx : ns flat centred frequency indices (k1 + N/2)*N + (k2 + N/2)
 *   g     : nrhs arrays of N*N complex (interleaved), row-major n1*N + n2
 *   hhat  : ns*nrhs complex (interleaved) output
 * Same arithmetic as oracle_direct: y.xi mod 1 in integers, h in FP64,
 * reduction by the nearest integer, FP64 accumulation summed per row of y.
 * Returns 0, or -1 on bad arguments.
 */
int oracle_direct_adjoint_amp(int N, int kind, const double *p, int amp, int ns, const int64_t *xiidx, int nrhs,
                              const double *g, double *hhat, int nthreads)
{
    if (N <= 0 || (N & 1) || ns < 0 || nrhs <= 0 || nrhs > 64)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const int h = N / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < ns; ++s) {
        const int64_t k1 = xiidx[s] / N - h, k2 = xiidx[s] % N - h;
        double acc_re[64], acc_im[64];
        for (int b = 0; b < nrhs; ++b)
            acc_re[b] = acc_im[b] = 0.0;
        for (int n1 = 0; n1 < N; ++n1) {
            double row_re[64], row_im[64];
            for (int b = 0; b < nrhs; ++b)
                row_re[b] = row_im[b] = 0.0;
            const double x1 = (double)n1 / N;
            for (int n2 = 0; n2 < N; ++n2) {
                const double x2 = (double)n2 / N;
                int64_t ip = ((int64_t)n1 * k1 + (int64_t)n2 * k2) % N;
                if (ip < 0)
                    ip += N;
                const double hv = oracle_h(kind, p, x1, x2, (double)k1, (double)k2);
                double ph = (double)ip / N + hv;
#if defined(ORACLE_PLANT) && ORACLE_PLANT == 6
                ph = -ph;
#endif
                double r = ph - rint(ph);
                /* conj(a) exp(-2 pi i r) */
                double c = cos(TWO_PI * r), sn = -sin(TWO_PI * r);
                if (amp) {
                    double ar, ai;
                    oracle_amp(amp, hv, (double)k1, (double)k2, &ar, &ai);
                    const double cr = c * ar + sn * ai, ci = sn * ar - c * ai;
                    c = cr;
                    sn = ci;
                }
                const int64_t cell = (int64_t)n1 * N + n2;
                for (int b = 0; b < nrhs; ++b) {
                    const double *v = g + 2 * ((int64_t)b * N * N + cell);
                    row_re[b] += c * v[0] - sn * v[1];
                    row_im[b] += c * v[1] + sn * v[0];
                }
            }
            for (int b = 0; b < nrhs; ++b) {
                acc_re[b] += row_re[b];
                acc_im[b] += row_im[b];
            }
        }
        for (int b = 0; b < nrhs; ++b) {
            hhat[2 * ((int64_t)s * nrhs + b)] = acc_re[b] / N;
            hhat[2 * ((int64_t)s * nrhs + b) + 1] = acc_im[b] / N;
        }
    }
    return 0;
}

int oracle_direct_adjoint(int N, int kind, const double *p, int ns, const int64_t *xiidx, int nrhs, const double *g,
                          double *hhat, int nthreads)
{
    return oracle_direct_adjoint_amp(N, kind, p, 0, ns, xiidx, nrhs, g, hhat, nthreads);
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
