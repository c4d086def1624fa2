/*
 * fgl.h -- C-ABI of the batched Gaussian log-likelihood of the region-based
 * global-21-cm foreground model (Tutt et al., "Optimising Foreground
 * Modelling for Global 21cm Cosmology with GPU-Accelerated Nested
 * Sampling"), on one AMD Instinct MI355X (gfx950).
 *
 * The operation (Sec. 2.2, Eq. fast_forward_model with the amplitude masks
 * collapsed to alpha = 1 as the paper fits spectral-index masks only;
 * Sec. 2.1, Eq. t21model; Sec. 2.3.1, Eq. likelihood): for every parameter
 * row b,
 *
 *   M[b,nu,t] = sum_i K[i,nu,t] (nu/nu_ref)^(-beta_bi) + T_CMB
 *               + A_b exp(-(nu - nu21_b)^2 / (2 w_b^2))
 *   lnL_b     = -1/2 sum_{nu,t} [ ln(2 pi sigma_b^2) + (D[nu,t] - M[b,nu,t])^2 / sigma_b^2 ]
 *
 * K[i,nu,t] are the chromatic response functions of the regions
 * (Eq. chromatic_function), precomputed by the caller; D is the observed
 * antenna temperature on the channel-time grid.
 *
 * Parameter rows (theta) are FP64, row-major [B][P]:
 *   [beta_0 .. beta_{N-1}, A (K, signed), nu21 (MHz), w = sigma_21 (MHz), sigma (K)]
 * with P = N + 4; with FGL_NO_21CM the row is [beta_0 .. beta_{N-1}, sigma],
 * P = N + 1.  (Table priors lists these parameters; sigma is linear.)
 *
 * Row validity: a row with a non-finite entry, sigma <= 0, w <= 0 (with the
 * 21-cm term) or |beta_i| > 64 yields lnL = -inf.  This does not fail the
 * call.
 *
 * Precision modes:
 *   FGL_PREC_MIXED  the region sum as exact 8-bit integer slices of the
 *                   powers and of the model's matrix on the matrix cores
 *                   (int32 sums), the residual and the chi-square in FP64.
 *                   Agrees with an FP64 evaluation within
 *                   |dlnL| <= 1e-6 |lnL| + 1e-3.  Two forms give that same
 *                   quantity (fgl_mixed_form): the direct form evaluates
 *                   M on the T time bins; the projected form, used when
 *                   T >= N + 1, N <= 96 and it needs fewer 32-row tiles,
 *                   evaluates the time sum of each channel exactly in an
 *                   orthonormal basis of the channel's centred responses
 *                   (N + 1 rows instead of T).  Small models are
 *                   evaluated per row in FP64 on the vector units instead
 *                   (FGL_FORM_THIN): N <= 32, T <= 64 and a measured cost
 *                   model of the two kernels favours it (S = N rounded up to
 *                   4, 8, 12, 16, 24 or 32; thin when
 *                   (S T + 12 S + 2 T) c(S) <= 650 for T <= 32 or 580
 *                   above, with c(24) = 1.17, c(32) = 0.90, c(12) = 0.97,
 *                   else 1: e.g. N <= 32 at T <= 8, N <= 16 at T <= 24,
 *                   N <= 8 at T <= 46; the paper's time-integrated fits
 *                   have T = 1).
 *                   There the matrix tiles would be mostly padding, and FP64
 *                   meets the bound exactly.  FGL_MIXED_DIRECT keeps the
 *                   digit kernel's direct form for them.
 *   FGL_PREC_FP32   the model in FP32, residual and chi-square in FP64.
 *   FGL_PREC_FP64   everything in FP64 (per row on the vector units for the
 *                   small models described above).
 *
 * Errors: every call returns an FGL_* status; fgl_last_error() gives a
 * message for the calling thread's last failure.  Nothing is ever printed.
 *
 * Determinism: the same model, rows and mode give bitwise-identical
 * results, whatever else runs on the device at the same time.
 *
 * Threads: calls on different models may run concurrently.  Calls on one
 * model are serialised by the library (host-pointer entry points) or must be
 * ordered by the caller's stream (device entry point).
 */
#ifndef FGL_H
#define FGL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fgl_model fgl_model;   /* opaque, library-owned */
typedef struct fgl_server fgl_server; /* opaque, library-owned */

enum {
  FGL_OK = 0,
  FGL_EINVAL = -1,  /* bad argument (the message says which) */
  FGL_ENOMEM = -2,  /* device or host allocation failed */
  FGL_EBUSY = -3,   /* object still has requests in flight */
  FGL_EDEVICE = -4, /* HIP runtime error */
  FGL_EAGAIN = -5,  /* not yet: retry later (serving admission) */
  FGL_ECANCELED = -6, /* serving: the request was cancelled while queued */
  FGL_ETIMEDOUT = -7  /* serving: the request waited in the queue past the limit */
};

enum { FGL_PREC_MIXED = 0, FGL_PREC_FP32 = 1, FGL_PREC_FP64 = 2 };

#define FGL_NO_21CM 1u      /* model without the 21-cm term: P = N + 1 */
#define FGL_MIXED_DIRECT 2u /* mixed precision: always use the direct form */
/* plain FP32 and FP64 precisions in the projected form where the model has
 * it (fgl_mixed_form is FGL_FORM_PROJECTED): the time sum of each channel in
 * the orthonormal basis, with FP32 (or FP64) rows and powers, residual and
 * chi-square in FP64.  Without the flag they evaluate M on the T time bins,
 * the paper's formulation. */
#define FGL_PLAIN_PROJECTED 4u

/* Forms of the mixed-precision evaluation (fgl_mixed_form). */
enum { FGL_FORM_DIRECT = 0, FGL_FORM_PROJECTED = 1, FGL_FORM_THIN = 2 };

/*
 * Create a model: the fixed inputs of the likelihood (Sec. 2.2 precomputes
 * K once per observation; Eq. likelihood's D is fixed per fit).
 *   K      host, FP32 [N][F][T], row-major; finite.
 *   freqs  host, FP64 [F], channel frequencies in MHz, finite, > 0, with
 *          2^-8 <= freqs/nu_ref <= 2^8.
 *   data   host, FP64 [F][T], antenna temperature D in K, finite.
 *   nu_ref reference frequency of the power laws (MHz, > 0).
 *   N      regions, 1..128;  F channels >= 1;  T time bins >= 1.
 *   t_cmb  CMB temperature added to the model (K), finite.
 *   flags  0, or any of FGL_NO_21CM, FGL_MIXED_DIRECT (keep the direct
 *          form of the mixed evaluation even where the projected one is
 *          shorter) and FGL_PLAIN_PROJECTED (the plain precisions take the
 *          projected form too, where the model has it).
 * The library copies everything to the device and re-lays it out for its
 * kernels; the caller may free its arrays on return.  *out receives the
 * model, owned by the library until fgl_model_destroy.
 * Returns FGL_OK, FGL_EINVAL, FGL_ENOMEM or FGL_EDEVICE.
 */
int fgl_model_create(const float* K, const double* freqs, const double* data,
                     double nu_ref, int N, int F, int T, double t_cmb,
                     unsigned flags, fgl_model** out);

/*
 * Create a model with amplitude masks crossed with spectral-index masks
 * (Sec. 2.2, Eq. fast_forward_model with its amplitude scales; the paper
 * fits spectral-index masks only and leaves amplitude masks to later work):
 *
 *   M[b,nu,t] = sum_i sum_j alpha_bi K[i,j,nu,t] (nu/nu_ref)^(-beta_bj)
 *               + T_CMB + A_b exp(-(nu - nu21_b)^2 / (2 w_b^2))
 *
 *   K        host, FP32 [n_alpha][n_beta][F][T], row-major; finite.  Entry
 *            (i, j) is the response of the overlap of amplitude mask i with
 *            spectral-index mask j (Eq. chromatic_function); an empty
 *            overlap has K = 0.
 *   n_alpha  amplitude masks >= 1;  n_beta  spectral-index masks >= 1;
 *            n_alpha * n_beta <= 128 regions.
 *   The other arguments are those of fgl_model_create.
 * Parameter rows: [beta_0 .. beta_{n_beta-1}, alpha_0 .. alpha_{n_alpha-1},
 * A, nu21, w, sigma], P = n_beta + n_alpha + 4 (n_beta + n_alpha + 1 with
 * FGL_NO_21CM).  A row with an amplitude scale outside [2^-32, 2^32] (zero
 * and negative scales included: alpha is a gain correction) yields
 * lnL = -inf, besides the rows described above.  Every other entry point,
 * precision mode and accuracy statement applies unchanged; the projected
 * form is chosen on N = n_alpha * n_beta.
 * Returns FGL_OK, FGL_EINVAL, FGL_ENOMEM or FGL_EDEVICE.
 */
int fgl_model_create_masks(const float* K, const double* freqs,
                           const double* data, double nu_ref, int n_alpha,
                           int n_beta, int F, int T, double t_cmb,
                           unsigned flags, fgl_model** out);

/* Parameters per row (N + 4, or N + 1 with FGL_NO_21CM; with amplitude
 * masks n_beta + n_alpha + 4 or + 1); -1 for NULL. */
int fgl_model_nparams(const fgl_model* m);

/* Form of the model's mixed-precision evaluation: FGL_FORM_DIRECT,
 * FGL_FORM_PROJECTED or FGL_FORM_THIN (fixed at creation); FGL_EINVAL for
 * NULL. */
int fgl_mixed_form(const fgl_model* m);

/*
 * lnL for B rows (Eq. likelihood).
 *   theta  host, FP64 [B][P] (layout above), read during the call only.
 *   B      rows, 0..2^26 (B = 0 is a no-op); the same bound holds for every
 *          entry point that takes B.
 *   out    host, FP64 [B], written on success.
 *   prec   FGL_PREC_MIXED, FGL_PREC_FP32 or FGL_PREC_FP64.
 * Synchronous: returns when out is written.  Returns FGL_OK, FGL_EINVAL,
 * FGL_ENOMEM, FGL_EBUSY (model being destroyed) or FGL_EDEVICE.
 */
int fgl_loglike_batch(fgl_model* m, const double* theta, int B,
                      double* out_logL, int prec);

/*
 * Same as fgl_loglike_batch with device memory, enqueued on a caller stream.
 *   d_theta  device, FP64 [B][P];  d_out  device, FP64 [B].
 *   hip_stream  hipStream_t (NULL = the legacy default stream).
 * Asynchronous: returns after enqueueing; d_out is valid once the stream
 * reaches this point.  d_theta must stay valid until then.  The model's
 * per-stream workspace is reused by the next call on the same stream.
 * With FGL_DEVICE_GRAPHS=1 in the environment when the model is created, a
 * call seen before (same precision, B, tile, buffers and stream) is
 * replayed from a captured hipGraph, with bitwise the same results; by
 * default the kernels are launched directly, which costs the host less here.
 */
int fgl_loglike_batch_device(fgl_model* m, const double* d_theta, int B,
                             double* d_out, int prec, void* hip_stream);

/*
 * fgl_loglike_batch_device for callers that cannot allocate device memory:
 * code under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It allocates nothing: the call's workspace (transposed
 * spectral indices, row records, chi-square partials) lives in one 64 MiB
 * array per GPU, held from the first call on that GPU to the end of the
 * process.  Same arguments, kernels and results (bitwise) as
 * fgl_loglike_batch_device; the tile is the tuned one if fgl_tune ran for
 * this batch size, else the default (no tuning, no kernel timing here).
 * Every call on one GPU shares the array: calls that overlap on one GPU,
 * on any model or stream, race, so the caller orders them (one stream, or
 * events).  Nothing in the array has to start at zero.
 * Returns FGL_OK; FGL_EINVAL for the arguments fgl_loglike_batch_device
 * refuses and for a batch whose workspace exceeds 64 MiB (the message gives
 * the model's largest batch: about 70,000 rows of the N=32, F=301 model);
 * FGL_EAGAIN if a server evicted the model (an allocating call makes it
 * resident again); FGL_EBUSY; FGL_EDEVICE.
 */
int fgl_loglike_batch_device_noalloc(fgl_model* m, const double* d_theta, int B,
                                     double* d_out, int prec, void* hip_stream);

/*
 * lnL and its gradient d lnL / d theta for B rows (the chain rule through
 * Eq. likelihood, Eq. fast_forward_model and Eq. t21model; the paper's
 * pipeline is differentiable, Sec. 3).  Entries follow the row layout:
 *   d/dbeta_j  = (1/sigma^2) sum_{nu,t} r (-ln(nu/nu_ref)) sum_i alpha_i K_ij P_j
 *   d/dalpha_i = (1/sigma^2) sum_{nu,t} r sum_j K_ij P_j   (crossed masks)
 *   d/dA, d/dnu21, d/dw through g(nu) = exp(-(nu-nu21)^2/(2 w^2))
 *   d/dsigma   = chi2/sigma^3 - F T/sigma
 * with r = D - M and P_j = (nu/nu_ref)^(-beta_j).
 *   theta  host, FP64 [B][P], read during the call only.
 *   out    host, FP64 [B]: lnL, as fgl_loglike_batch with FGL_PREC_FP64
 *          up to rounding.
 *   grad   host, FP64 [B][P].
 *   prec   FGL_PREC_FP64 (the only mode with a gradient; others give
 *          FGL_EINVAL).
 * Invalid rows get lnL = -inf and a NaN gradient.  Synchronous.  Returns
 * FGL_OK, FGL_EINVAL, FGL_ENOMEM, FGL_EBUSY or FGL_EDEVICE.
 */
int fgl_loglike_grad_batch(fgl_model* m, const double* theta, int B,
                           double* out_logL, double* grad, int prec);

/* Same with device memory (d_grad: FP64 [B][P]), enqueued on hip_stream as
 * fgl_loglike_batch_device.  The kernel timing counters cover the gradient
 * kernel of these calls too. */
int fgl_loglike_grad_batch_device(fgl_model* m, const double* d_theta, int B,
                                  double* d_out, double* d_grad, int prec,
                                  void* hip_stream);

/*
 * Tile configuration used for (model, B, prec): waves per workgroup,
 * channels per workgroup and the waves per SIMD the kernel variant is
 * compiled for, as chosen by the autotuner (measuring on first use when
 * FGL_TUNE=1 or fgl_tune was called).  Any output pointer may be NULL.
 * The tile never changes results.  Returns FGL_OK.
 */
int fgl_get_tile(fgl_model* m, int B, int prec, int* waves, int* chans,
                 int* occupancy);

/* Measure the candidate tiles for (model, B, prec) now and keep the
 * fastest for later calls, and in the tuner cache.  Synchronous; uses the
 * device. */
int fgl_tune(fgl_model* m, int B, int prec);

/*
 * The tuner cache: the tiles fgl_tune (or FGL_TUNE=1) measured, by device
 * architecture, kernel family, model shape (N, n_alpha, F, T) and form,
 * and batch bucket (B rounded up to a power of two >= 256), shared by all
 * models of the process.  A model without a tile of its own for a call uses
 * the cached one when it is still a candidate for it, else the default.
 * path: a file of one JSON object per line,
 *   {"arch":"gfx950","kind":0,"N":32,...,"bucket":16384,"waves":8,"fc":8,"occ":3}
 * whose entries are loaded now (a missing file is an empty cache) and which
 * is rewritten after every tuning; NULL stops writing.  The environment
 * variable FGL_TUNE_CACHE names such a file for the process when this is
 * never called.  Tiles never change results.  Returns FGL_OK.
 */
int fgl_tune_cache(const char* path);

/* Force the tile for (model, B's size class, prec); FGL_EINVAL unless it is
 * one of the tuner's candidates for this model.  Results are unchanged. */
int fgl_set_tile(fgl_model* m, int B, int prec, int waves, int chans,
                 int occupancy);

/* Device bytes held by the model (its resident inputs, not workspaces). */
size_t fgl_model_bytes(const fgl_model* m);

/*
 * Kernel timing (instrumentation for benchmarks and roofline reports).
 * fgl_kernel_timing(m, n) with n >= 1 resets the counters and, from then on,
 * records a HIP event pair around the likelihood kernel of every n-th call
 * on m (n = 1: every call), on the stream that kernel runs on (graph replay
 * is bypassed meanwhile).  The events carry no system-scope fence; each pair
 * still adds a few microseconds to its call, which n > 1 spreads over n
 * calls.  fgl_kernel_timing(m, 0) stops recording; n < 0 is FGL_EINVAL.
 * fgl_kernel_time waits for the recorded kernels and returns their summed
 * duration (ms) and count.
 */
int fgl_kernel_timing(fgl_model* m, int enable);
int fgl_kernel_time(fgl_model* m, double* total_ms, int64_t* launches);

/* Destroy a model.  Returns FGL_EBUSY, freeing nothing, while a call or a
 * served request on it is in flight; never blocks. */
int fgl_model_destroy(fgl_model* m);

/*
 * Serving (continuous batching of likelihood requests from many concurrent
 * samplers, Sec. 3.1.2: each nested-sampling iteration submits the rows of
 * its parallel slice chains).
 *   hbm_budget_bytes  device bytes the server may keep resident for the
 *                     models of admitted requests (0 = no limit, unless
 *                     FGL_HBM_BUDGET_MB is set: then that many MiB).
 *   max_inflight      requests on the device at once (>= 1).
 * A request is admitted when its model is resident or can be made resident
 * within the budget (idle models are evicted least-recently-used first) and
 * a slot is free; otherwise it waits in arrival order.  Admitted requests
 * run on several streams so that their work overlaps on the device.
 */
int fgl_serve_create(size_t hbm_budget_bytes, int max_inflight,
                     fgl_server** out);

/*
 * Submit B rows (1..2^26) of theta (host) for model m; out_logL (host, [B]) is
 * written before the request is reported done.  theta and out_logL must
 * stay valid until fgl_serve_poll reports done.  *ticket identifies the
 * request.  Returns FGL_OK, FGL_EINVAL, or FGL_EAGAIN when the model alone
 * exceeds the budget.
 */
int fgl_serve_submit(fgl_server* s, fgl_model* m, const double* theta, int B,
                     double* out_logL, int prec, uint64_t* ticket);

/*
 * Launches shared by models (Sec. 3.1.2: many samplers' likelihood calls on
 * one device): with max_models_per_launch > 1, the groups of up to that many
 * waiting models whose likelihood kernel is the same compiled variant join
 * one launch of the row-preparation, likelihood and finalize kernels, each
 * workgroup finding its model in a descriptor table; every row's result is
 * bitwise the one it gets alone.  The shareable variants are those the
 * default tiles of models without amplitude masks use (the mixed kernel
 * with 8-wave workgroups and at most 64 regions, in either form, and the
 * small-model FP64 kernel); other requests launch per model.  1 (the
 * default, or FGL_SERVE_SHARE at creation) launches per model.
 * max_models_per_launch in 1..16.  Returns FGL_OK or FGL_EINVAL.
 */
int fgl_serve_set_sharing(fgl_server* s, int max_models_per_launch);

/* Launch counters of a server: all launches, shared ones (more than one
 * model) and the model groups those carried.  Any pointer may be NULL. */
int fgl_serve_stats(fgl_server* s, uint64_t* launches, uint64_t* shared_launches,
                    uint64_t* shared_groups);

/*
 * Poll a ticket: *done = 1 when out_logL is written (then *latency_us is the
 * submit-to-completion time), else 0.  A done ticket is retired by the poll
 * that reports it; polling it again returns FGL_EINVAL.  A request that
 * failed on the device, was cancelled or timed out reports done with its
 * status (FGL_EDEVICE, FGL_ECANCELED, FGL_ETIMEDOUT) as the return value.
 */
int fgl_serve_poll(fgl_server* s, uint64_t ticket, int* done,
                   double* latency_us);

/*
 * Cancel a request that is still queued: it is reported done by the next
 * poll, with FGL_ECANCELED and out_logL unwritten (theta and out_logL may be
 * released after that poll).  Returns FGL_OK; FGL_EBUSY when the request is
 * already launched or complete (it completes normally); FGL_EINVAL for an
 * unknown or retired ticket.
 */
int fgl_serve_cancel(fgl_server* s, uint64_t ticket);

/*
 * Wait limit of queued requests: a request still queued max_wait_us after
 * its submission (held or waiting for a slot or for HBM budget) is reported
 * done with FGL_ETIMEDOUT and out_logL unwritten; launched requests always
 * complete.  0 (the default) sets no limit.  Returns FGL_OK or FGL_EINVAL
 * (negative or non-finite).
 */
int fgl_serve_set_timeout(fgl_server* s, double max_wait_us);

/* Block until every submitted request is done (completions stay pollable).
 * FGL_EAGAIN, without waiting for the queue, while the server is held with
 * requests queued (launches in flight are still waited for). */
int fgl_serve_drain(fgl_server* s);

/*
 * Hold (hold != 0) or release (0) admission.  While held, submitted requests
 * only queue; launches already in flight complete.  On release the scheduler
 * plans the whole queue at once, so that a batch submitted together (the
 * requests of many samplers at one iteration) is merged per model and, with
 * sharing on, joined across models of one kernel variant as far as the
 * slots allow.  Returns FGL_OK or FGL_EINVAL.
 */
int fgl_serve_hold(fgl_server* s, int hold);

/* Destroy the server: FGL_EBUSY while requests are pending or in flight. */
int fgl_serve_destroy(fgl_server* s);

/*
 * Slice-sampling chains on the device (the replacement step of batched
 * nested sampling, Sec. 3.1.2 and Sec. 3.1.3).  Sampler coordinates are the
 * parameter row with its last entry (sigma) replaced by log sigma; the prior
 * is uniform over the box [lo, hi] in those coordinates.
 *
 * fgl_chains_create: an engine for model m with room for max_chains chains
 *   (1..2^26);
 *   lo, hi host [P] (finite, lo < hi), copied; seed keys the chains' Philox
 *   random streams.  The model cannot be destroyed while the engine exists
 *   (fgl_model_destroy returns FGL_EBUSY).
 * fgl_chains_run: n chains start at x0 (host [n][P], inside the box) with
 *   lnL l0 (host [n]) and each takes `steps` hit-and-run slice steps under
 *   lnL > lstar, directions drawn in the geometry of chol (host [P][P],
 *   row-major lower-triangular factor of the live points' covariance), the
 *   likelihood evaluated in precision prec.  x_out, l_out (host [n][P], [n])
 *   receive the end points and their lnL; *evals (optional) the number of
 *   in-box proposals evaluated, *rounds (optional) the batched rounds run.
 *   Synchronous.  FGL_EAGAIN if chains did not finish within a generous
 *   bound of rounds (a likelihood that is nowhere above lstar near a start).
 * fgl_chains_destroy: releases the engine.
 */
typedef struct fgl_chains fgl_chains;  /* opaque, library-owned */
int fgl_chains_create(fgl_model* m, int max_chains, const double* lo,
                      const double* hi, uint64_t seed, fgl_chains** out);
int fgl_chains_run(fgl_chains* c, const double* x0, const double* l0, int n,
                   double lstar, const double* chol, int steps, int prec,
                   double* x_out, double* l_out, int64_t* evals,
                   int64_t* rounds);
int fgl_chains_destroy(fgl_chains* c);

/*
 * The chains' random numbers, for reproducing or checking their draws:
 * out[4j..4j+3] = Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011:
 * ten rounds, multipliers 0xD2511F53 and 0xCD9E8D57, Weyl key increments
 * 0x9E3779B9 and 0xBB67AE85) of the counter block ctr[4j..4j+3] under the
 * key (k0, k1), computed by the device function the chains use.  A chain
 * engine created with seed s draws with k0 = s mod 2^32, k1 = s / 2^32, and
 * its chain i's draw number c is the block (c mod 2^32, c / 2^32, i,
 * 0x5eed5eed); a uniform is the top 53 bits of the 64-bit word (w0 2^32 +
 * w1), or of (w2 2^32 + w3), times 2^-53.  ctr and out are host uint32
 * arrays [4n], n in 1..2^24.  Synchronous.  Returns FGL_OK, FGL_EINVAL,
 * FGL_ENOMEM or FGL_EDEVICE.
 */
int fgl_chains_philox(const uint32_t* ctr, int n, uint32_t k0, uint32_t k1,
                      uint32_t* out);

/*
 * Profiling ranges: with FGL_ROCTX=1 in the environment when the library is
 * first used, the likelihood, gradient, tuning, serving-launch, chain, sky
 * and noise calls push a roctx range (named for the call, with its main
 * sizes) for rocprofv3 --marker-trace.  The roctx library is loaded at run
 * time; without it, or without the variable, the ranges cost one branch.
 */

/* Message of the calling thread's last failure ("" if none). */
const char* fgl_last_error(void);

/*
 * Region construction and chromatic response functions (Sec. 4; Eq.
 * chromatic_function), upstream of the likelihood: they produce the K a
 * model is created from.
 *
 * The sky is an equirectangular grid of nlat rings (declination) by nlon
 * columns (right ascension); pixel (r, c) has solid angle 4 pi omega[r].
 * Sky-frame maps are indexed (ring, ra); the beam and horizon are fixed to
 * the antenna and indexed (ring, hour angle).  At LST step t the sky pixel
 * (r, c) sits at the antenna pixel (r, (c - s_t) mod nlon); shifts[t] = s_t.
 */
typedef struct fgl_sky fgl_sky;       /* opaque, library-owned */

enum { FGL_WEIGHT_HORIZON = 0, FGL_WEIGHT_SKY = 1, FGL_WEIGHT_BEAM = 2 };
enum { FGL_PARTITION_HIERARCHICAL = 0, FGL_PARTITION_RECURSIVE = 1 };

/*
 * Copy a sky to the device.
 *   omega    host FP64 [nlat], pixel solid angle / (4 pi) of each ring, > 0.
 *   t_ex     host FP64 [nlat][nlon], T_base - T_CMB at nu0 (K), sky frame.
 *   beta     host FP64 [nlat][nlon], spectral index (Eq. spectralindexmap),
 *            |beta| <= 64, sky frame.
 *   beam     host FP32 [F][nlat][nlon], D(nu), antenna frame.
 *   horizon  host uint8 [nlat][nlon], H (0 or non-zero), antenna frame.
 *   freqs    host FP64 [F] (MHz, > 0); nu0 reference frequency (MHz, > 0);
 *   t_cmb    CMB temperature (K).
 * All inputs are copied; returns FGL_OK, FGL_EINVAL, FGL_ENOMEM, FGL_EDEVICE.
 */
int fgl_sky_create(int nlat, int nlon, int F, const double* omega,
                   const double* t_ex, const double* beta, const float* beam,
                   const uint8_t* horizon, const double* freqs, double nu0,
                   double t_cmb, fgl_sky** out);

/*
 * Importance of every sky pixel for one of the three weightings of
 * Sec. 4.2 (horizon: H; sky: T_sky H; beam: T_sky D H, with
 * T_sky = t_ex (nu/nu0)^(-beta) + T_CMB, Eq. skyapproximation), each
 * normalised to integrate to one over the sphere per (nu, t):
 *   importance[q] = sum_{nu, t} omega(q) W(p_t(q), nu, t)   (host FP64
 *   [nlat][nlon]), the per-pixel weights of Eq. weighted_cdf.
 * shifts: host int32 [T], each in [0, nlon).  FGL_EINVAL when a weight
 * integrates to zero at some (nu, t).  Synchronous.
 */
int fgl_sky_importance(fgl_sky* s, const int32_t* shifts, int T, int scheme,
                       double* importance);

/*
 * Partition the spectral-index range on the importance-weighted CDF of n
 * pixels (Eq. weighted_cdf) into n_regions regions by Alg. method1
 * (FGL_PARTITION_HIERARCHICAL) or Alg. method2 (FGL_PARTITION_RECURSIVE).
 * edges (host FP64 [n_regions + 1]) receives the non-decreasing edges; region
 * j holds e_j <= beta < e_{j+1} (the last is closed).  C is the cumulative
 * weight of the pixels in ascending beta (stable), divided by its total;
 * C^{-1}(c) is the smallest pixel beta with C >= c; a region's mass is the
 * increase of C across it; ties go to the lowest region.  Host only.
 */
int fgl_partition(const double* beta, const double* weight, int n,
                  int n_regions, int method, double* edges);

/*
 * Chromatic response functions of the regions given by edges (Eq.
 * chromatic_function, one amplitude mask):
 *   K[j][nu][t] = sum_{q: region(q) = j} omega(q) t_ex(q) D(nu, p_t(q))
 * in FP64 (host [n_regions][F][T]); pixels outside [e_0, e_N] belong to no
 * region.  n_regions in 1..1024 (within one workgroup's LDS).  Synchronous;
 * fgl_sky_kernel_ms then gives the correlation kernel's duration.
 */
int fgl_sky_chromatic(fgl_sky* s, const double* edges, int n_regions,
                      const int32_t* shifts, int T, double* K);
int fgl_sky_kernel_ms(const fgl_sky* s, double* ms);
int fgl_sky_destroy(fgl_sky* s);

/* ---- Residual-likelihood reference distribution (accuracy criterion) ----
 * Sec. 5 classifies a fit as consistent with noise when its median
 * posterior lnL is not in the lower q_threshold tail of the likelihood over
 * data sets that the model describes exactly up to realisations of the
 * assumed noise (uncorrelated Gaussian).  For data = M(theta) + e the
 * residual at theta is e, so Eq. likelihood at theta is
 *   lnl[r] = -sum_{k<n} e_rk^2 / (2 sigma_like^2) - (n/2) ln(2 pi sigma_like^2)
 * with e_rk = sigma_noise z_rk and n = F T residuals per data set.
 */

/*
 * lnL of R noise-only data sets (FP64 host [R]).  The standard normals z_rk
 * are fixed by (seed, r, k): under key (seed low 32 bits, seed high 32 bits),
 * block b of stream s is Philox4x32-10 (Salmon et al., SC 2011) of counter
 * (b, r, s, 0x6e6f6973); normals 2j and 2j+1 are the Box-Muller pair of
 * u1 = (w + 1) 2^-32 and u2 = v 2^-32, w and v the 32-bit word j % 4 of
 * block j / 4 of streams 0 and 1: z = sqrt(-2 ln u1) (cos 2 pi u2,
 * sin 2 pi u2).
 * n in 1..2^31; R in 1..2^23; n R <= 2^40 (a call runs at most a few
 * seconds); sigma_noise finite >= 0; sigma_like finite > 0.  kernel_ms (may
 * be NULL) receives the kernel's duration.
 * Synchronous.  Returns FGL_OK, FGL_EINVAL, FGL_ENOMEM or FGL_EDEVICE.
 */
int fgl_noise_loglike(int64_t n, int R, double sigma_noise, double sigma_like,
                      uint64_t seed, double* lnl, double* kernel_ms);

/*
 * q[i] = #{r < R : lnl_noise[r] <= lbar[i]} / R (host FP64 arrays
 * lnl_noise [R], lbar [nb], q [nb]): the fraction of the reference
 * distribution at or below each fit's median lnL (a NaN on either side
 * never counts).  R >= 1, nb in 1..2^23.  Computed on the device.  Synchronous.  Returns FGL_OK, FGL_EINVAL,
 * FGL_ENOMEM or FGL_EDEVICE.
 */
int fgl_noise_quantile(const double* lnl_noise, int R, const double* lbar,
                       int nb, double* q);

#ifdef __cplusplus
}
#endif

#endif /* FGL_H */
