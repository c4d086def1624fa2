/*
 * fgl_oracle.c -- plain FP64 CPU oracle for the batched Gaussian
 * log-likelihood of the region-based foreground model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path links, loads or
 * calls this file: only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header, table or constant with the HIP
 * library; it is written from the paper's definitions alone, slowly and in
 * the order the definitions are stated, so it can be checked by eye.
 *
 * What it computes, for every parameter row b (Tutt et al.):
 *
 *   g(nu)      = exp(-(nu - nu21)^2 / (2 w^2))               Eq. t21model
 *   T_FG       = sum_i K[i,nu,t] (nu/nu_ref)^(-beta_i) + T_CMB
 *                                        Eq. fast_forward_model, with the
 *                amplitude masks collapsed to one (alpha = 1), as the paper
 *                fits spectral-index masks only (end of Sec. 2.2)
 *   M(nu,t)    = T_FG(nu,t) + A g(nu)          definition after Eq. likelihood
 *   lnL        = -1/2 sum_{nu,t} [ ln(2 pi sigma^2) + (D - M)^2 / sigma^2 ]
 *                                                            Eq. likelihood
 *
 * Parameter row layout: [beta_0 .. beta_{N-1}, A, nu21, w, sigma]
 * (the region indices, the three 21-cm parameters of Eq. t21model and the
 * noise level of Eq. likelihood; sigma is linear, in K).  With flag bit 0
 * (no 21-cm term) the row is [beta_0 .. beta_{N-1}, sigma].
 *
 * A row with sigma <= 0, w <= 0, any non-finite entry, or a spectral index
 * outside [-64, 64] gets lnL = -inf.  The paper does not define these rows;
 * they have zero prior mass (its spectral-index prior spans 2.458-3.146), and
 * the index bound keeps every power of a frequency ratio within 2^+-8 inside
 * the double range.
 *
 * All arithmetic is IEEE double.  Powers use pow(); the region sum runs in
 * ascending i; the chi-square is summed over (nu, t) in row-major order with
 * Neumaier's compensated summation.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_NO_21CM 1u

/* Compensated (Neumaier) accumulator. */
typedef struct { double s, c; } neumaier_t;

static void nm_add(neumaier_t *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static int row_valid(const double *th, int P, int N, unsigned flags)
{
    for (int k = 0; k < P; ++k)
        if (!isfinite(th[k])) return 0;
    for (int i = 0; i < N; ++i)
        if (fabs(th[i]) > 64.0) return 0;
    double sigma = th[P - 1];
    if (!(sigma > 0.0)) return 0;
    if (!(flags & ORACLE_NO_21CM)) {
        double w = th[N + 2];
        if (!(w > 0.0)) return 0;
    }
    return 1;
}

/* Model M(nu, t) of one parameter row into m[F*T].  Returns 0, or -1 when
 * the row is invalid (m is then left untouched). */
int oracle_model(const float *K, const double *freqs, double nu_ref,
                 double t_cmb, int N, int F, int T, unsigned flags,
                 const double *theta_row, double *m)
{
    int P = (flags & ORACLE_NO_21CM) ? N + 1 : N + 4;
    if (!row_valid(theta_row, P, N, flags)) return -1;
    const double *beta = theta_row;
    double *powv = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    if (!powv) return -2;
    for (int f = 0; f < F; ++f) {
        double nu = freqs[f];
        double ratio = nu / nu_ref;
        for (int i = 0; i < N; ++i)
            powv[i] = pow(ratio, -beta[i]);          /* (nu/nu_ref)^(-beta_i) */
        double sig21 = 0.0;
        if (!(flags & ORACLE_NO_21CM)) {
            double A = theta_row[N], nu21 = theta_row[N + 1], w = theta_row[N + 2];
            double dv = nu - nu21;
            sig21 = A * exp(-(dv * dv) / (2.0 * w * w));
        }
        double *row = m + (size_t)f * T;
        for (int t = 0; t < T; ++t) row[t] = 0.0;
        for (int i = 0; i < N; ++i) {                 /* ascending i */
            const float *Ki = K + ((size_t)i * F + f) * T;
            for (int t = 0; t < T; ++t)
                row[t] += (double)Ki[t] * powv[i];
        }
        for (int t = 0; t < T; ++t)
            row[t] = row[t] + t_cmb + sig21;
    }
    free(powv);
    return 0;
}

/* lnL of one row, given the data D[F*T]; scratch m[F*T]. */
static double loglike_row(const float *K, const double *freqs,
                          const double *D, double nu_ref, double t_cmb,
                          int N, int F, int T, unsigned flags,
                          const double *theta_row, double *m)
{
    int P = (flags & ORACLE_NO_21CM) ? N + 1 : N + 4;
    if (oracle_model(K, freqs, nu_ref, t_cmb, N, F, T, flags, theta_row, m) != 0)
        return -INFINITY;
    double sigma = theta_row[P - 1];
    neumaier_t chi2 = {0.0, 0.0};
    for (size_t k = 0; k < (size_t)F * T; ++k) {
        double r = D[k] - m[k];
        nm_add(&chi2, r * r);
    }
    double s2 = sigma * sigma;
    double n = (double)F * (double)T;
    return -0.5 * (chi2.s + chi2.c) / s2 - 0.5 * n * log(2.0 * M_PI * s2);
}

/* lnL for B rows of theta[B][P] into out[B].  nthreads <= 0 uses the
 * OpenMP default; 1 runs serially.  Returns 0, or -1 on bad sizes. */
int oracle_loglike(const float *K, const double *freqs, const double *D,
                   double nu_ref, double t_cmb, int N, int F, int T,
                   unsigned flags, const double *theta, int B, double *out,
                   int nthreads)
{
    if (N < 0 || F <= 0 || T <= 0 || B < 0) return -1;
    int P = (flags & ORACLE_NO_21CM) ? N + 1 : N + 4;
    int fail = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double *m = (double *)malloc(sizeof(double) * (size_t)F * T);
        if (!m) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (int b = 0; b < B; ++b)
                out[b] = loglike_row(K, freqs, D, nu_ref, t_cmb, N, F, T,
                                     flags, theta + (size_t)b * P, m);
            free(m);
        }
    }
    return fail ? -2 : 0;
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
