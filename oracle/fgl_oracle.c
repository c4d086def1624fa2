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
 *   T_FG       = sum_i sum_j alpha_i K[i,j,nu,t] (nu/nu_ref)^(-beta_j) + T_CMB
 *                                                  Eq. fast_forward_model
 *   M(nu,t)    = T_FG(nu,t) + A g(nu)          definition after Eq. likelihood
 *   lnL        = -1/2 sum_{nu,t} [ ln(2 pi sigma^2) + (D - M)^2 / sigma^2 ]
 *                                                            Eq. likelihood
 *
 * Two parameterisations of the masks (Sec. 2.2):
 *
 *  - spectral-index masks only (the paper's fits, end of Sec. 2.2): one
 *    amplitude mask with alpha = 1, K[j,nu,t] for j < N, and the row
 *    [beta_0 .. beta_{N-1}, A, nu21, w, sigma];
 *  - n_alpha amplitude masks crossed with n_beta spectral-index masks:
 *    K[i,j,nu,t] at K + ((i n_beta + j) F + nu) T, and the row
 *    [beta_0 .. beta_{n_beta-1}, alpha_0 .. alpha_{n_alpha-1}, A, nu21, w,
 *    sigma].
 *
 * The three 21-cm parameters are those of Eq. t21model and sigma is the
 * noise level of Eq. likelihood (linear, in K).  With flag bit 0 (no 21-cm
 * term) they are left out and the row ends with sigma alone.
 *
 * A row with sigma <= 0, w <= 0, any non-finite entry, a spectral index
 * outside [-64, 64] or an amplitude scale outside [2^-32, 2^32] gets
 * lnL = -inf.  The paper does not define these rows; they have zero prior
 * mass (its spectral-index prior spans 2.458-3.146; alpha is a gain
 * correction near one), and the bounds keep every term inside the double
 * range.
 *
 * All arithmetic is IEEE double.  Powers use pow(); the region sum runs in
 * ascending (i, j), each term formed as (alpha_i K) times the power; the
 * chi-square is summed over (nu, t) in row-major order with Neumaier's
 * compensated summation.
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

/* Parameter count of a row. */
static int n_params(int NA, int NB, unsigned flags)
{
    return NB + NA + ((flags & ORACLE_NO_21CM) ? 1 : 4);
}

static int row_valid(const double *th, int P, int NA, int NB, unsigned flags)
{
    for (int k = 0; k < P; ++k)
        if (!isfinite(th[k])) return 0;
    for (int j = 0; j < NB; ++j)
        if (fabs(th[j]) > 64.0) return 0;
    for (int i = 0; i < NA; ++i) {
        double a = th[NB + i];
        if (!(a >= 0x1p-32 && a <= 0x1p32)) return 0;
    }
    double sigma = th[P - 1];
    if (!(sigma > 0.0)) return 0;
    if (!(flags & ORACLE_NO_21CM)) {
        double w = th[P - 2];
        if (!(w > 0.0)) return 0;
    }
    return 1;
}

/* Model M(nu, t) of one parameter row into m[F*T], with NA amplitude masks
 * (NA = 0: none, alpha = 1) and NB spectral-index masks.  Returns 0, or -1
 * when the row is invalid (m is then left untouched). */
int oracle_model_masks(const float *K, const double *freqs, double nu_ref,
                       double t_cmb, int NA, int NB, int F, int T,
                       unsigned flags, const double *theta_row, double *m)
{
    int P = n_params(NA, NB, flags);
    if (!row_valid(theta_row, P, NA, NB, flags)) return -1;
    const double *beta = theta_row;              /* beta_j, j < NB */
    const double *alpha = theta_row + NB;        /* alpha_i, i < NA */
    int n_amp = NA > 0 ? NA : 1;                 /* amplitude masks */
    double *powv = (double *)malloc(sizeof(double) * (size_t)(NB > 0 ? NB : 1));
    if (!powv) return -2;
    for (int f = 0; f < F; ++f) {
        double nu = freqs[f];
        double ratio = nu / nu_ref;
        for (int j = 0; j < NB; ++j)
            powv[j] = pow(ratio, -beta[j]);          /* (nu/nu_ref)^(-beta_j) */
        double sig21 = 0.0;
        if (!(flags & ORACLE_NO_21CM)) {
            double A = theta_row[P - 4], nu21 = theta_row[P - 3], w = theta_row[P - 2];
            double dv = nu - nu21;
            sig21 = A * exp(-(dv * dv) / (2.0 * w * w));
        }
        double *row = m + (size_t)f * T;
        for (int t = 0; t < T; ++t) row[t] = 0.0;
        for (int i = 0; i < n_amp; ++i) {             /* ascending (i, j) */
            double a = NA > 0 ? alpha[i] : 1.0;
            for (int j = 0; j < NB; ++j) {
                const float *Kij = K + (((size_t)i * NB + j) * F + f) * T;
                for (int t = 0; t < T; ++t)
                    row[t] += (a * (double)Kij[t]) * powv[j];
            }
        }
        for (int t = 0; t < T; ++t)
            row[t] = row[t] + t_cmb + sig21;
    }
    free(powv);
    return 0;
}

/* The spectral-index-only model: N masks, alpha = 1. */
int oracle_model(const float *K, const double *freqs, double nu_ref,
                 double t_cmb, int N, int F, int T, unsigned flags,
                 const double *theta_row, double *m)
{
    return oracle_model_masks(K, freqs, nu_ref, t_cmb, 0, N, F, T, flags,
                              theta_row, m);
}

/* lnL of one row, given the data D[F*T]; scratch m[F*T]. */
static double loglike_row(const float *K, const double *freqs,
                          const double *D, double nu_ref, double t_cmb,
                          int NA, int NB, int F, int T, unsigned flags,
                          const double *theta_row, double *m)
{
    int P = n_params(NA, NB, flags);
    if (oracle_model_masks(K, freqs, nu_ref, t_cmb, NA, NB, F, T, flags,
                           theta_row, m) != 0)
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

/* lnL for B rows of theta[B][P] into out[B] (masks as in
 * oracle_model_masks).  nthreads <= 0 uses the OpenMP default; 1 runs
 * serially.  Returns 0, or -1 on bad sizes. */
int oracle_loglike_masks(const float *K, const double *freqs, const double *D,
                         double nu_ref, double t_cmb, int NA, int NB, int F,
                         int T, unsigned flags, const double *theta, int B,
                         double *out, int nthreads)
{
    if (NA < 0 || NB < 0 || F <= 0 || T <= 0 || B < 0) return -1;
    int P = n_params(NA, NB, flags);
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
                out[b] = loglike_row(K, freqs, D, nu_ref, t_cmb, NA, NB, F, T,
                                     flags, theta + (size_t)b * P, m);
            free(m);
        }
    }
    return fail ? -2 : 0;
}

/* The spectral-index-only likelihood: N masks, alpha = 1. */
int oracle_loglike(const float *K, const double *freqs, const double *D,
                   double nu_ref, double t_cmb, int N, int F, int T,
                   unsigned flags, const double *theta, int B, double *out,
                   int nthreads)
{
    return oracle_loglike_masks(K, freqs, D, nu_ref, t_cmb, 0, N, F, T, flags,
                                theta, B, out, nthreads);
}

/* Gradient of lnL of one row with respect to the row's parameters, into
 * g[P]; returns lnL (-inf for an invalid row, whose g is all NaN).  The
 * chain rule through Eq. likelihood, Eq. fast_forward_model and
 * Eq. t21model, with r = D - M and the sums over (nu, t):
 *
 *   dlnL/dtheta   = (1/sigma^2) sum r dM/dtheta       (theta other than sigma)
 *   dM/dbeta_j    = -ln(nu/nu_ref) sum_i alpha_i K_ij (nu/nu_ref)^(-beta_j)
 *   dM/dalpha_i   = sum_j K_ij (nu/nu_ref)^(-beta_j)
 *   dM/dA         = g(nu)
 *   dM/dnu21      = A g(nu) (nu - nu21) / w^2
 *   dM/dw         = A g(nu) (nu - nu21)^2 / w^3
 *   dlnL/dsigma   = chi2 / sigma^3 - F T / sigma
 *
 * Every sum over (nu, t) is compensated (Neumaier). */
double oracle_grad_masks(const float *K, const double *freqs, const double *D,
                         double nu_ref, double t_cmb, int NA, int NB, int F,
                         int T, unsigned flags, const double *theta_row,
                         double *g, double *m)
{
    int P = n_params(NA, NB, flags);
    if (oracle_model_masks(K, freqs, nu_ref, t_cmb, NA, NB, F, T, flags,
                           theta_row, m) != 0) {
        for (int k = 0; k < P; ++k) g[k] = NAN;
        return -INFINITY;
    }
    const double *beta = theta_row, *alpha = theta_row + NB;
    int n_amp = NA > 0 ? NA : 1;
    int no21 = (flags & ORACLE_NO_21CM) != 0;
    double sigma = theta_row[P - 1];
    neumaier_t *acc = (neumaier_t *)calloc((size_t)P, sizeof(neumaier_t));
    if (!acc) return NAN;
    neumaier_t chi2 = {0.0, 0.0};
    for (int f = 0; f < F; ++f) {
        double nu = freqs[f];
        double lr = log(nu / nu_ref);
        double dnu = 0.0, w = 1.0, A = 0.0, gnu = 0.0;
        if (!no21) {
            A = theta_row[P - 4];
            double nu21 = theta_row[P - 3];
            w = theta_row[P - 2];
            dnu = nu - nu21;
            gnu = exp(-(dnu * dnu) / (2.0 * (w * w)));
        }
        for (int t = 0; t < T; ++t) {
            double r = D[(size_t)f * T + t] - m[(size_t)f * T + t];
            nm_add(&chi2, r * r);
            for (int i = 0; i < n_amp; ++i) {
                double amp = NA > 0 ? alpha[i] : 1.0;
                for (int j = 0; j < NB; ++j) {
                    double kp = (double)K[(((size_t)i * NB + j) * F + f) * T + t]
                                * pow(nu / nu_ref, -beta[j]);
                    nm_add(&acc[j], r * (-lr * amp * kp));       /* beta_j */
                    if (NA > 0) nm_add(&acc[NB + i], r * kp);  /* alpha_i */
                }
            }
            if (!no21) {
                nm_add(&acc[P - 4], r * gnu);
                nm_add(&acc[P - 3], r * (A * gnu * dnu / (w * w)));
                nm_add(&acc[P - 2], r * (A * gnu * dnu * dnu / (w * w * w)));
            }
        }
    }
    double var = sigma * sigma;
    for (int k = 0; k < P - 1; ++k) g[k] = (acc[k].s + acc[k].c) / var;
    double c2 = chi2.s + chi2.c;
    double n = (double)F * (double)T;
    g[P - 1] = c2 / (var * sigma) - n / sigma;
    free(acc);
    return -0.5 * c2 / var - 0.5 * n * log(2.0 * M_PI * var);
}

/* lnL and its gradient for B rows: out[B], grad[B][P]. */
int oracle_grad_batch_masks(const float *K, const double *freqs,
                            const double *D, double nu_ref, double t_cmb,
                            int NA, int NB, int F, int T, unsigned flags,
                            const double *theta, int B, double *out,
                            double *grad, int nthreads)
{
    if (NA < 0 || NB < 0 || F <= 0 || T <= 0 || B < 0) return -1;
    int P = n_params(NA, NB, flags);
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
                out[b] = oracle_grad_masks(K, freqs, D, nu_ref, t_cmb, NA, NB, F, T,
                                           flags, theta + (size_t)b * P,
                                           grad + (size_t)b * P, m);
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
