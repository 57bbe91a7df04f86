/*
 * ftp.h -- C ABI of the MI355X (gfx950) fast template periodogram library.
 *
 * The method is Hoffman, Vanderplas, Hartman & Bakos, "A Fast Template
 * Periodogram" (arXiv:2101.12348).  Given observations S = {(t_i, y_i,
 * sigma_i)} and a template fixed by its truncated Fourier coefficients
 * M(x) = sum_{n=1..H} c_n cos(n x) + s_n sin(n x) (Section 2), the library
 * fits y ~ theta_1 M(w t - theta_2) + theta_3 at every trial frequency
 * f_j = j df, j = 1..n_f (w = 2 pi f_j) and returns the periodogram
 * P = (chi2_0 - chi2)/chi2_0 (Section 1, Eq. lsp; Section 2:
 * P = YM^2/(YY MM)) with the best theta_2, theta_1 and theta_3.
 *
 * Conventions shared by every entry point:
 *  - Return value: 0 on success, a negative FTP_E_* code otherwise.  Host-
 *    detectable problems are reported synchronously; nothing is enqueued then.
 *  - "device" pointers are HIP device allocations (e.g. torch tensors on
 *    cuda:0); "host" pointers are ordinary host memory.  The caller owns every
 *    array it passes; the library never frees them.
 *  - stream: a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is enqueued asynchronously on it; outputs are valid once
 *    that stream has completed the call's work.
 *  - Data-dependent problems found on the device (NaN/Inf in inputs,
 *    sigma < 0, mixed zero and non-zero sigma, Var(y) = 0) make every
 *    frequency of that lightcurve report FTP_ST_BAD_LC in `status` with
 *    P = 0; per-frequency conditions use the other FTP_ST_* codes.
 *  - theta_2 (phase) is reported in [0, 2 pi) relative to t = 0 as given.
 *  - A plan must not be used from two host threads at once, and calls on one
 *    plan must not overlap on different streams (the plan's scratch is
 *    reused in stream order).
 */
#ifndef FTP_H
#define FTP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define FTP_OK 0
#define FTP_E_NULL -1          /* a required pointer is NULL */
#define FTP_E_H -2             /* H < 1, H > FTP_MAX_H, or all c = s = 0 */
#define FTP_E_NOBS -3          /* n_obs < 3 (or a ragged batch segment < 3) */
#define FTP_E_DF -4            /* df <= 0 or not finite */
#define FTP_E_NF -5            /* n_f < 1 */
#define FTP_E_OFFSETS -6       /* obs_off / freq_off not monotone or not starting at 0 */
#define FTP_E_SIZE -7          /* a size overflows the library's limits */
#define FTP_E_HIP -8           /* a HIP runtime call failed (see ftp_last_error) */
#define FTP_E_OPTION -9        /* an option value is invalid */
#define FTP_E_NO_MODEL -10     /* learned solver requested but no network loaded */
#define FTP_E_IO -11           /* a file could not be read or written (tuning cache) */

/* per-frequency status values (uint8) */
#define FTP_ST_OK 0
#define FTP_ST_DEGENERATE 1    /* MM ~ 0 at every candidate (all phases coincide): P = 0 */
#define FTP_ST_CONSTANT 2      /* the phase polynomial vanishes: P does not depend on theta_2 */
#define FTP_ST_NO_CONVERGE 3   /* companion QR hit its iteration limit */
#define FTP_ST_BAD_LC 4        /* the lightcurve was rejected (see above) */
#define FTP_ST_FALLBACK 8      /* bit: the solver's first method did not settle the frequency
                                  (learned / uniform: Newton roots not confirmed by the Sturm
                                  count; the roots came from Aberth or the companion solve) */
#define FTP_ST_FALLBACK_QR 16  /* bit: the roots came from the companion solve after the
                                  Aberth iteration did not converge (learned / uniform / Aberth) */

#define FTP_MAX_H 15   /* D = 6H - 2 <= 88: up to two companion rows and two coefficients per lane */

/* precision of the NFFT stage (spreading, FFT, sums); assembly, roots and
 * scoring are always FP64 */
#define FTP_FP32_SUMS 0
#define FTP_FP64 1

/* root solver */
#define FTP_SOLVER_PLAIN 0     /* companion-matrix eigenvalues (Section 2) */
#define FTP_SOLVER_LEARNED 1   /* per frequency a Sturm count of the real-phase roots, then Newton
                                  from evenly spaced starts (min(32, 6H - 2) for H <= 10, 4H for
                                  H >= 11); the frequencies whose roots do not reach the count get a
                                  second Newton round from the network's 2H seeds plus evenly spaced
                                  starts (with FTP_FLAG_SEEDS_ALL the seeds enter every frequency's
                                  first round); what is still unconfirmed goes to Aberth (H <= 11),
                                  then to the companion solve */
#define FTP_SOLVER_UNIFORM 2   /* as LEARNED without the network (ablation): the second round starts
                                  from evenly spaced phases only */
#define FTP_SOLVER_ABERTH 3    /* Aberth-Ehrlich iteration on every frequency; companion solve
                                  where it does not converge (H <= 11: one root per lane; larger H
                                  is refused with FTP_E_OPTION) */

/* option flags */
#define FTP_FLAG_FORCE_FALLBACK 1u  /* learned / uniform / Aberth solvers: send every frequency to
                                       the companion solve */
#define FTP_FLAG_TIME_STAGES 2u     /* record HIP events around the NFFT and per-frequency stages
                                       (read back by ftp_last_stats) */
#define FTP_FLAG_SEEDS_ALL 16u      /* learned solver: network seeds in every frequency's first
                                       Newton round (2H seeds + evenly spaced starts), not only in
                                       the second round of the frequencies the first left */
#define FTP_FLAG_2H_STARTS 32u      /* learned / uniform (H <= 10): the first Newton round starts from
                                       2H phases only (with FTP_FLAG_SEEDS_ALL the network's seeds,
                                       else evenly spaced), for comparing the two at equal starts */
#define FTP_FLAG_POSITIVE_AMP 8u    /* fit constrained to theta_1 > 0 (Section 2.1): the best
                                       candidate with YM > 0 (P = YM^2/(YY MM) vanishes on YM = 0,
                                       so the constrained maximum is one of the same stationary
                                       points); none: P = 0, theta_1 = 0, theta_3 = ybar,
                                       theta_2 = 0 */

typedef struct ftp_plan ftp_plan;

typedef struct {
  int precision;        /* FTP_FP32_SUMS (default) or FTP_FP64 */
  int solver;           /* FTP_SOLVER_* (default PLAIN) */
  double nfft_R;        /* minimum grid oversampling; 0 = 2.0 */
  int nfft_msp;         /* Gaussian half-width in cells; 0 = 7 (FP32) / 12 (FP64) */
  int solve_waves;      /* persistent solve grid in waves; 0 = autotuned default */
  unsigned flags;       /* FTP_FLAG_* */
} ftp_options;

typedef struct {
  uint64_t n_pairs;        /* frequencies solved by the last call */
  uint64_t n_fallback;     /* learned / uniform: frequencies whose Newton roots the Sturm
                              count did not confirm (solved by the Aberth tier) */
  uint64_t n_fallback_qr;  /* frequencies left to the companion solve by the Aberth tier */
  uint64_t qr_sweeps;      /* Francis double-shift sweeps performed */
  uint64_t newton_iters;   /* Newton iterations performed (learned path) */
  uint64_t roots_found;    /* distinct real roots accepted (learned path) */
  uint64_t aberth_iters;   /* Aberth sweeps, summed over the frequencies it solved */
  double ms_nfft;          /* device time of the NFFT stage (ms, 0 if not timed) */
  double ms_solve;         /* device time of the per-frequency stage (ms) */
  double ms_roots;         /* of which in the root-finding kernels (ms) */
  double ms_mlp;           /* learned: features + network forward (ms) */
  double ms_verify;        /* learned: Newton + Sturm verification (ms) */
  double ms_aberth;        /* learned / uniform / Aberth: the Aberth kernel (ms) */
  double ms_fallback;      /* learned / uniform / Aberth: companion solve of what is left (ms) */
  double ms_spread;        /* of the NFFT stage: the spreading kernel (ms) */
  double ms_fft;           /* of the NFFT stage: the FFT passes (ms) */
  double ms_retry;         /* learned / uniform: the second Newton round (ms) */
  uint64_t n_fallback_aberth;   /* learned / uniform: frequencies the second Newton round
                                   left to the Aberth tier */
} ftp_stats;

/* Launch shapes of the per-frequency kernels, in wavefronts per compute
 * unit (1..256), and the implementation of the network's forward pass.  They change timing only: every frequency is computed by one
 * wavefront whatever the grid, so results are identical for every setting.
 * The companion-QR and Aberth kernels, whose work per frequency varies with
 * their iteration counts, take frequencies from a work queue; assembly,
 * Newton + Sturm and scoring stride over them. */
typedef struct {
  int assemble_wpc;     /* assembly (and network features) */
  int newton_wpc;       /* Newton + Sturm (learned / uniform) */
  int aberth_wpc;       /* Aberth */
  int qr_wpc;           /* companion QR */
  int score_wpc;        /* scoring */
  int mlp_fused;        /* learned: 1 = one kernel for the four network layers (LDS-staged
                           weights, activations kept per wavefront), 0 = four GEMM
                           launches; identical results */
  int newton_occ;       /* Newton + Sturm (H <= 10): the build compiled for 4, 5 or 6
                           resident wavefronts per SIMD (fewer registers per lane at more) */
} ftp_tuning;

#define FTP_TUNE_FORCE 1u   /* ftp_autotune: measure even if the cache holds an entry */

/* Fill `opt` with the defaults.  Returns FTP_E_NULL if opt is NULL. */
int ftp_options_default(ftp_options* opt);

/*
 * Create a plan for one template (Section 2: c_n, s_n, n = 1..H; host arrays
 * of length H, copied).  `opt` may be NULL (defaults).  *out receives the plan.
 * Errors: FTP_E_NULL, FTP_E_H, FTP_E_OPTION, FTP_E_HIP.
 */
int ftp_plan_create(ftp_plan** out, int H, const double* c, const double* s, const ftp_options* opt);

/*
 * Create a plan for the shared-phase multi-band model (Appendix A): one
 * template per band, c and s host arrays of n_band x H values, band-major
 * (band k's c_n at c[k H + n - 1]); a band with fewer harmonics is padded
 * with zeros, a band whose template is all zero is allowed as long as one
 * band's is not.  1 <= n_band <= 16.  Such a plan serves only
 * ftp_periodogram_shared_phase (ftp_last_stats, tuning and destroy as any
 * plan); the other periodogram calls return FTP_E_OPTION on it.
 * Errors: FTP_E_NULL, FTP_E_H, FTP_E_OPTION (n_band out of range), FTP_E_HIP.
 */
int ftp_plan_create_bands(ftp_plan** out, int n_band, int H, const double* c, const double* s,
                          const ftp_options* opt);

/* Release a plan and its device scratch (synchronises the device). */
int ftp_plan_destroy(ftp_plan* plan);

/*
 * Template periodogram of one lightcurve (Section 2).
 *   t, y, sigma : device, n_obs FP64 each; t in any order; sigma >= 0
 *                 (all zero = uniform weights, Section 2).
 *   df, n_f     : trial frequencies f_j = j df, j = 1..n_f (Section 1 grid).
 *   power, phase, amp, offset : device, n_f FP64 each (P, theta_2, theta_1,
 *                 theta_3 of Section 2).  status: device, n_f uint8, may be NULL.
 * Errors: FTP_E_NULL, FTP_E_NOBS, FTP_E_DF, FTP_E_NF, FTP_E_SIZE, FTP_E_HIP.
 */
int ftp_periodogram(ftp_plan* plan, const double* t, const double* y, const double* sigma, int64_t n_obs,
                    double df, int64_t n_f, double* power, double* phase, double* amp, double* offset,
                    uint8_t* status, void* stream);

/*
 * Ragged batch of n_lc lightcurves sharing the plan's template.
 *   obs_off  : host, n_lc + 1 prefix offsets into t/y/sigma (obs_off[0] = 0).
 *   t, y, sigma : device, obs_off[n_lc] FP64 each.
 *   df       : host, n_lc frequency spacings.
 *   freq_off : host, n_lc + 1 prefix offsets into the outputs; lightcurve b
 *              has n_f = freq_off[b+1] - freq_off[b] frequencies j = 1..n_f.
 *   power, phase, amp, offset : device, freq_off[n_lc] FP64 each; status as above.
 * Errors: as ftp_periodogram, plus FTP_E_OFFSETS.
 */
int ftp_periodogram_batch(ftp_plan* plan, int64_t n_lc, const int64_t* obs_off, const double* t,
                          const double* y, const double* sigma, const double* df, const int64_t* freq_off,
                          double* power, double* phase, double* amp, double* offset, uint8_t* status,
                          void* stream);

/*
 * Multi-phase multi-band periodogram (Section 2.2, Eq. multibandmultiphase):
 * n_band bands of one object, each with its own phase, amplitude and offset,
 * the plan's template for all of them, on the common grid f_j = j df,
 * j = 1..n_f:  power[j] = sum_k chi2_0,k P_k[j] / sum_k chi2_0,k with
 * chi2_0,k = sum over band k of (y - ybar_k)^2 / sigma^2 (unit weights when
 * every sigma of the band is 0).  Runs the bands as a ragged batch.
 *   obs_off : host, n_band + 1 offsets of the bands in t, y, sigma (device).
 *   power   : device, n_f FP64.
 *   band_power (nullable): device, n_band x n_f FP64, the band periodograms.
 *   chi2_0  (nullable): device, n_band FP64 (0 for a rejected band, which
 *             then does not count; all rejected: power = 0).
 * Errors: as ftp_periodogram_batch.  Plan scratch grows to n_band n_f
 * records of 33 bytes.
 */
int ftp_periodogram_multiband(ftp_plan* plan, int64_t n_band, const int64_t* obs_off, const double* t,
                              const double* y, const double* sigma, double df, int64_t n_f, double* power,
                              double* band_power, double* chi2_0, void* stream);

/*
 * Shared-phase multi-band periodogram (Appendix A) of one object observed in
 * the plan's n_band bands: band k's observations are t, y, sigma[obs_off[k]
 * .. obs_off[k+1]) (device arrays; obs_off on the host, n_band + 1 entries,
 * obs_off[0] = 0, every band non-empty).  The bands share amplitude theta_1,
 * phase theta_2 and offset theta_3; band k's data are modelled as
 * theta_1 M_k(omega t - theta_2) + theta_3 + offsets[k] with fixed offsets
 * (host, n_band values; NULL = all zero), subtracted before anything else.
 * Weights sigma^-2 are normalised over all observations (all sigma zero in
 * every band: unit weights); ybar and YY = chi^2_0 are those of all bands
 * together.  Per frequency j df, j = 1..n_f, the sums of every band give
 * MM = psi^2H MMhat - (psi^H Mbar)^2 and YM = sum w y psi^H M - ybar psi^H Mbar,
 * whose polynomial (Eq. finalpoly) is solved and scored exactly as in the
 * single-band call; outputs as ftp_periodogram (device, n_f each): power,
 * phase (theta_2), amp (theta_1), offset (theta_3, the common offset before
 * the band offsets are added back), status.  FTP_FLAG_POSITIVE_AMP applies.
 * All bands' grids are resident together (no chunking).
 * Errors: FTP_E_NULL, FTP_E_OPTION (not a bands plan, non-finite offset),
 * FTP_E_OFFSETS, FTP_E_NOBS (an empty band), FTP_E_DF, FTP_E_NF, FTP_E_SIZE,
 * FTP_E_NO_MODEL, FTP_E_HIP.  Mixed unit and sigma weights across bands, or
 * non-finite input, give status FTP_ST_BAD_LC for every frequency.
 */
int ftp_periodogram_shared_phase(ftp_plan* plan, const int64_t* obs_off, const double* t, const double* y,
                                 const double* sigma, const double* offsets, double df, int64_t n_f,
                                 double* power, double* phase, double* amp, double* offset, uint8_t* status,
                                 void* stream);

/*
 * NFFT stage alone (for checking the sums): writes, per frequency j = 1..n_f,
 * 3H complex FP64 values to `sums` (device, n_f * 6H doubles, interleaved
 * re/im): Z_w(k j), k = 1..2H, then Z_y(k j), k = 1..H, where
 *   Z_w(m) = sum_i w_i exp(2 pi i m df (t_i - t_ref)),
 *   Z_y(m) = sum_i w_i (y_i - ybar) exp(2 pi i m df (t_i - t_ref))
 * (the raw sums behind Eqs. CCdef-YSdef).  `lc_stats` (device, 4 doubles)
 * receives t_ref, ybar, YY = chi2_0 and the lightcurve status bits.
 * Errors: as ftp_periodogram.
 */
int ftp_nfft_sums(ftp_plan* plan, const double* t, const double* y, const double* sigma, int64_t n_obs,
                  double df, int64_t n_f, double* sums, double* lc_stats, void* stream);

/*
 * Per-frequency stage alone, from given sums in the layout ftp_nfft_sums
 * writes (device `sums`), with t_ref, ybar and YY given on the host
 * (`lc_stats`, 3 doubles).  Outputs as ftp_periodogram.
 * Errors: FTP_E_NULL, FTP_E_DF, FTP_E_NF, FTP_E_HIP.
 */
int ftp_solve_sums(ftp_plan* plan, const double* sums, const double* lc_stats, double df, int64_t n_f,
                   double* power, double* phase, double* amp, double* offset, uint8_t* status,
                   void* stream);

/*
 * ftp_solve_sums without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, outputs and errors as ftp_solve_sums, on a
 * plan created beforehand (ftp_plan_create allocates; this call does not).
 * Solvers: plain, uniform and Aberth; FTP_E_OPTION for the learned solver
 * (its network buffers are the plan's) and for a bands plan.
 * Scratch: a fixed 64 MiB device array inside the library, one per GPU, held
 * until the process ends; frequencies are processed in chunks that fit it, so
 * n_f is not limited by it (FTP_E_SIZE only if one frequency's record would not
 * fit).  Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams, or host threads without ordering) race and must not
 * be made.  No statistics are kept and FTP_FLAG_TIME_STAGES is ignored.
 */
int ftp_solve_sums_noalloc(ftp_plan* plan, const double* sums, const double* lc_stats, double df, int64_t n_f,
                           double* power, double* phase, double* amp, double* offset, uint8_t* status,
                           void* stream);

/*
 * Root counts of the per-frequency phase polynomials (a check of the count
 * the learned and uniform solvers rely on), from given sums in the layout
 * ftp_nfft_sums writes (device `sums`; t_ref, ybar, YY on the host in
 * `lc_stats`, 3 doubles).  Per frequency j = 1..n_f (device int32 arrays of
 * n_f values):
 *   sturm_count[j-1]    : distinct real roots of R(theta) (the real-phase
 *                         solutions of Eq. theta2cond, Section 2) from the
 *                         Sturm sequence of the solvers' Cayley polynomial, as
 *                         the learned / uniform solvers compute it; -1000 - n
 *                         when the sequence fails its conditioning test (the
 *                         solvers then fall back; n is the count the sequence
 *                         reached regardless, a diagnostic), -2 for a frequency
 *                         the solvers skip (P constant in theta_2);
 *   companion_real[j-1] : real eigenvalues of that polynomial's companion
 *                         matrix by the plain solver's QR (the unit-circle roots
 *                         psi of Eq. finalpoly); -1 if the QR did not converge,
 *                         -2 as above.
 * Errors: FTP_E_NULL, FTP_E_DF, FTP_E_NF, FTP_E_OPTION (bands plan, invalid
 * lc_stats), FTP_E_HIP.
 */
int ftp_root_counts(ftp_plan* plan, const double* sums, const double* lc_stats, double df, int64_t n_f,
                    int32_t* sturm_count, int32_t* companion_real, void* stream);

/*
 * Load the root-proposal network (learned solver): `weights` is a host FP32
 * array of n_floats values in the order W1, b1, W2, b2, W3, b3, W4, b4 with
 * W stored (out, in) row-major; sizes d_in = 2(6H-1), width, d_out = 4H.
 * Errors: FTP_E_NULL, FTP_E_SIZE (n_floats does not match), FTP_E_HIP.
 */
int ftp_plan_load_mlp(ftp_plan* plan, const float* weights, int64_t n_floats, int width);

/* ------------------------------------------------------------------
 * Root-proposal network (learned solver; a project addition to the method).
 * An MLP d_in -> W -> W -> W -> d_out with ReLU, bf16 weights and activations
 * and FP32 accumulation on the matrix cores; parameters W1, b1, ..., W4, b4
 * with W stored (out, in) row-major: n = d_in W + W + 2 (W^2 + W) + d_out W +
 * d_out.  For a plan with H harmonics d_in = 2 (6H - 1) (the normalised
 * coefficients p_k, k = 0..6H-2, of Eq. finalpoly as (Re, Im) pairs, rotated so
 * that the first trig coefficient of R(theta) is real) and d_out = 4H (2H seed
 * directions (u, v); seed = atan2(v, u) in that rotated frame).
 * Inputs X are bf16 bit patterns (uint16), row-major B x d_in, device.
 * Training labels: up to R real-root phases per sample in the same frame
 * (device B x R floats) and their counts (device B ints).  Loss: Chamfer
 * distance on the circle between seed vectors and root unit vectors,
 *   L = mean_b [ (1/n_b) sum_j min_k |e_k - r_j|^2 + lam (1/K) sum_k min_j |e_k - r_j|^2 ].
 * ------------------------------------------------------------------ */
typedef struct ftp_mlp ftp_mlp;

/* Create a network; weights: host FP32 array of n values, or NULL for
 * He-uniform weights and zero biases drawn from `seed`.
 * Errors: FTP_E_NULL, FTP_E_SIZE (dimensions out of range), FTP_E_HIP. */
int ftp_mlp_create(ftp_mlp** out, int d_in, int width, int d_out, const float* weights, uint64_t seed);
int ftp_mlp_destroy(ftp_mlp* net);
int ftp_mlp_num_params(const ftp_mlp* net, int64_t* n);
/* FP32 master weights to host (synchronises the device). */
int ftp_mlp_get_weights(ftp_mlp* net, float* host, int64_t n);
/* out (device, B x d_out FP32) = network(X). */
int ftp_mlp_forward(ftp_mlp* net, const uint16_t* X, int64_t B, float* out, void* stream);
/* Per-sample loss (device B floats, nullable) and the loss gradient w.r.t.
 * every parameter (device n floats, nullable), without updating. */
int ftp_mlp_loss_grad(ftp_mlp* net, const uint16_t* X, int64_t B, const float* roots, const int* nroots, int R,
                      float lam, float* loss, float* grads, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 masters with
 * learning rate lr; the bf16 copies follow.  loss: as above. */
int ftp_mlp_train_step(ftp_mlp* net, const uint16_t* X, int64_t B, const float* roots, const int* nroots, int R,
                       float lam, float lr, float* loss, void* stream);
/* Training samples from one lightcurve: runs the periodogram with the
 * companion solve and writes, per frequency j = 1..n_f, the network features
 * (X, device n_f x 2(6H-1) bf16) and the real roots of the phase polynomial in
 * the feature frame (roots, device n_f x R; nroots, device n_f, capped at R). */
int ftp_learned_dataset(ftp_plan* plan, const double* t, const double* y, const double* sigma, int64_t n_obs,
                        double df, int64_t n_f, uint16_t* X, float* roots, int* nroots, int R, void* stream);

/* Current launch shapes of the plan (until set or tuned: assembly, Newton and
 * scoring 256 waves per CU, Aberth and QR 16, four GEMM launches for the
 * network, the Newton kernel built for 5 waves per SIMD). */
int ftp_plan_get_tuning(const ftp_plan* plan, ftp_tuning* out);

/* Set the launch shapes.  FTP_E_OPTION if a shape is outside 1..256,
 * mlp_fused is not 0 or 1 or newton_occ is not 4, 5 or 6. */
int ftp_plan_set_tuning(ftp_plan* plan, const ftp_tuning* tuning);

/*
 * Autotuner of the launch shapes (the schedule of the ragged-batch path): on
 * the given lightcurve (same arguments as ftp_periodogram; device arrays),
 * each shape that matters for the plan's solver is swept over 4..256 waves per
 * compute unit (and, for the learned solver, both network implementations; for
 * the Sturm-verified Newton solvers, both register budgets of its kernel),
 * one at a time, keeping the fastest whole periodogram call
 * (best of two, HIP events on `stream`).  The result is applied to the plan
 * and written to *out.
 * cache_path (nullable): a text file of "key assemble newton aberth qr score
 * mlp_fused newton_occ" lines (a line without newton_occ reads as 4); the key (ftp_plan_tune_key) names the device, its compute units, H,
 * precision, solver and a bucket of n_f.  An entry found there is applied without measuring
 * (unless flags has FTP_TUNE_FORCE); a measured result is stored there.
 * Returns 1 when the cache supplied the shapes, 0 when they were measured, or
 * an error (FTP_E_*; the plan's shapes are then unchanged).  Allocates
 * scratch outputs of n_f frequencies; synchronises `stream`; the timing calls
 * count in the ftp_last_stats window like any other call.
 */
int ftp_autotune(ftp_plan* plan, const double* t, const double* y, const double* sigma, int64_t n_obs, double df,
                 int64_t n_f, const char* cache_path, unsigned flags, ftp_tuning* out, void* stream);

/* Cache key of the plan for periodograms of n_f frequencies
 * ("<arch>/<CUs>cu/H<H>/p<precision>/s<solver>/nf<b>", b even with 2^b <= n_f
 * < 2^(b+2), clamped to 10..24: launch shapes depend on the work per launch)
 * into buf (len bytes, NUL terminated).  FTP_E_NF if n_f < 1, FTP_E_SIZE if
 * it does not fit. */
int ftp_plan_tune_key(const ftp_plan* plan, int64_t n_f, char* buf, int len);

/* Tuning-cache file access (host only, no device use).  lookup: 1 and *out
 * filled when `key` has a well-formed entry, 0 when it has none (or the file
 * does not exist); store: replaces or appends the entry, rewriting the file
 * through a temporary and a rename.  Errors: FTP_E_NULL, FTP_E_OPTION (empty
 * key, white space in it, a shape outside 1..256 or mlp_fused not 0 / 1),
 * FTP_E_IO. */
int ftp_tune_cache_lookup(const char* path, const char* key, ftp_tuning* out);
int ftp_tune_cache_store(const char* path, const char* key, const ftp_tuning* tuning);

/* Statistics accumulated over the plan's calls since the previous
 * ftp_last_stats (or plan creation); resets the accumulation.  Synchronises
 * `stream`, which must be the stream the calls were made on. */
int ftp_last_stats(ftp_plan* plan, ftp_stats* out, void* stream);

/* Human-readable text for an FTP_E_* or FTP_ST_* code. */
const char* ftp_status_string(int code);

/* Text of the last HIP error seen by the library (thread-local). */
const char* ftp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FTP_H */
