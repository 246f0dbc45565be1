/*
 * lasp.h -- C ABI of the MI355X grouped full-spectrum fitting library.
 *
 * The library fits, for N spectra at once, the model of the paper's
 * LASP-Adam-GPU method (arXiv 2512.24840, Section 2.2):
 *   Eq. 1  model spectrum from a polynomial interpolator, F' = Phi(theta) B
 *   Eq. 5  Gaussian velocity shift and broadening, F'' = F' (x) G(mu, sigma)
 *   Eq. 6  multiplicative polynomial continuum fitted by weighted least squares
 *   Eq. 7  residual, and Eq. 9 objective read per spectrum as chi2 / n_eff
 *   stage 8 Adam on the five parameters normalised to [-1, 1]
 *   stage 9 parameter covariance by linear error propagation
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers (HIP global memory) unless marked
 *    HOST.  They are owned by the caller, C-contiguous, row-major.  The
 *    library reads and writes them only from work it enqueues on
 *    opts->stream and never keeps them past that work.
 *  - Calls are stream ordered: they return once the work is enqueued (after
 *    host-side validation); results are valid after the stream is
 *    synchronised.  Internal scratch memory (per device and stream) is cached
 *    between calls and returned by lasp_release().  Two calls that overlap on
 *    the same stream are ordered; calls on different streams use separate
 *    scratch.
 *  - Parameters, physical units: (Teff [K], log g [dex], [Fe/H] [dex],
 *    RV [km/s], sigma [km/s]).  Normalised parameters u in [-1, 1]:
 *    u_t = 2 (theta_t - lo_t) / (hi_t - lo_t) - 1 with theta = (log10 Teff,
 *    log g, [Fe/H], RV, sigma) and the box opts->box_lo / box_hi.  The fit
 *    does not clamp u to the box.
 *  - Return value: LASP_OK (0) or a negative LASP_E_* code; the message of
 *    the last failure on the calling thread is lasp_last_error().  No entry
 *    point aborts or throws.
 */
#ifndef LASP_H
#define LASP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LASP_OK 0
#define LASP_E_ARG (-1)         /* null pointer, bad dimension or option */
#define LASP_E_GRID (-2)        /* wave_grid not uniform in log10(lambda) */
#define LASP_E_DEVICE (-3)      /* HIP runtime or launch error */
#define LASP_E_NOMEM (-4)       /* device allocation failed */
#define LASP_E_UNSUPPORTED (-5) /* shape/precision without a compiled kernel */

/* Per-spectrum status bits (opts->status).  One spectrum's status never
 * changes another spectrum's results.
 *  Input bits, from obs and ivar: NONFINITE_INPUT, NO_DATA.
 *  Evaluation bits, at the parameters the call returns (lasp_fit_group,
 *  lasp_pool_finish) or evaluates (lasp_forward); a condition met only at
 *  intermediate points of a fit is not reported: SINGULAR, CONT_NONPOS,
 *  OUT_OF_BOX, SIGMA_FLOOR.  CONT_NONPOS is the failed-fit test of the
 *  paper's Section 4.2 (a nonpositive multiplicative correction P(x) b,
 *  Step 5 of Section 2.2).
 *  Course-of-fit bits: STOP_FLAT, STOP_RISING, NOT_CONVERGED, POLISH_LIMIT. */
#define LASP_ST_NONFINITE_INPUT 0x01u /* some obs/ivar not finite: pixel weight set to 0 */
#define LASP_ST_NO_DATA 0x02u         /* n_eff <= 5 + degree + 1 */
#define LASP_ST_SINGULAR 0x04u        /* continuum normal equations (or, with a covariance
                                         requested, its Schur complement) not positive definite */
#define LASP_ST_CONT_NONPOS 0x08u     /* fitted continuum P(x) b <= 0 at some pixel */
#define LASP_ST_OUT_OF_BOX 0x10u      /* |u_t| > 1.5 (or not finite) for some parameter */
#define LASP_ST_SIGMA_FLOOR 0x20u     /* broadening width at the 0.1 px floor in some arm
                                         (d chi2 / d sigma is 0 there) */
#define LASP_ST_STOP_FLAT 0x40u       /* stopped: loss changed < stop_tol over the window */
#define LASP_ST_STOP_RISING 0x80u     /* stopped: loss rose at every step of the window */
#define LASP_ST_NOT_CONVERGED 0x100u  /* stopping rules on, step limit reached first */
#define LASP_ST_POLISH_LIMIT 0x200u   /* polish reached polish_iters before its stopping test */

#define LASP_PREC_FP32 0   /* FP32 interpolator contraction */
#define LASP_PREC_BF16X3 1 /* BF16 hi/lo split contraction, FP32 accumulate */

#define LASP_N_BASIS 20 /* monomials of total degree <= 3 in (u1, u2, u3) */
#define LASP_MAX_CLASSES 3 /* emulator temperature classes (cool, warm, hot) */
#define LASP_N_PAR 5
#define LASP_MAX_ARMS 4

/*
 * Options.  Fill with lasp_default_opts() and override.
 *  n_spec, n_pix   number of spectra B and pixels P per spectrum.
 *  n_basis         must be LASP_N_BASIS * n_classes; basis row k multiplies monomial k of
 *                  (u1, u2, u3) in graded lexicographic order:
 *                  1, u1, u2, u3, u1^2, u1u2, u1u3, u2^2, u2u3, u3^2, u1^3,
 *                  u1^2u2, u1^2u3, u1u2^2, u1u2u3, u1u3^2, u2^3, u2^2u3,
 *                  u2u3^2, u3^3.
 *  margin          M: the basis covers P + 2M pixels, column c <-> pixel c-M.
 *  degree          continuum degree D; compiled: 4, 6, 8, 10.
 *  precision       LASP_PREC_FP32 or LASP_PREC_BF16X3.
 *  box_lo, box_hi  normalisation box (see above).
 *  lr, beta1, beta2, eps   Adam hyper-parameters (torch.optim.Adam form).
 *  weight_quantile flux quantile used as the per-spectrum weight w of Eq. 6
 *                  (Section 3.3: 0.5); <= 0 uses w = 1.  The objective is
 *                  invariant to w; it only conditions the arithmetic.
 *  n_arms, arm_start, arm_sigma_kms   optional spectrograph arms: pixel j in
 *                  arm a is broadened by sqrt(sigma^2 + arm_sigma_kms[a]^2).
 *                  n_arms = 0: one arm, no instrumental term.
 *  stream          hipStream_t to enqueue on (NULL: the null stream).
 *  status          optional device uint32 [n_spec]: LASP_ST_* bits.
 *  out_chi2        optional device double [n_spec]: chi2 at the returned
 *                  parameters (weights ivar, data obs).
 *  stop_window, stop_tol   per-spectrum stopping rules of Section 2.2 stage 8
 *                  (0 = off: every fit takes n_steps steps).  With loss
 *                  ell_t = sqrt(chi2 / n_eff) after t steps, a fit stops after
 *                  t steps when t >= W and |ell_{t-W} - ell_t| < stop_tol
 *                  (LASP_ST_STOP_FLAT), or when the loss rose at each of the
 *                  last W steps (LASP_ST_STOP_RISING); otherwise after n_steps
 *                  (LASP_ST_NOT_CONVERGED).  W = stop_window <= 4096; the
 *                  paper's window is 50 and its threshold 1e-5.  A stopped
 *                  fit takes no further steps; the others are not affected.
 *                  With the rules on, lasp_fit_group lists the fits still
 *                  stepping every 16 steps so that the step kernels cover
 *                  only those, and waits on its stream (for the list length
 *                  of 16 steps earlier) so that it stops enqueuing steps
 *                  once every fit has stopped: the call then returns about
 *                  16 steps before the stream finishes instead of at once.
 *  out_steps       optional device int32 [n_spec]: Adam steps each fit took.
 *  polish_iters    after the Adam steps, up to this many Levenberg-Marquardt
 *                  iterations per spectrum (0 = none): damped Gauss-Newton
 *                  steps on the residual with the continuum profiled out,
 *                  (S + lambda diag S) du = Ju^T W e, kept when chi2 falls;
 *                  a spectrum stops when the predicted chi2 decrease of its
 *                  next step du^T q is below 1e-6, when an accepted step
 *                  lowers chi2 by less than 1e-10 relative or moves u by
 *                  less than 1e-7, or when lambda exceeds 1e10
 *                  (LASP_ST_POLISH_LIMIT if the iteration limit came first).  The paper proposes adding curvature
 *                  information to its Adam stage (Section 4.5); n_steps = 0
 *                  with polish_iters > 0 is a plain LM fit.  Every 4
 *                  iterations the number of spectra still iterating is
 *                  counted on the device; once a count reads 0 the call
 *                  stops enqueuing iterations (it waits on its stream for
 *                  the count of 4 iterations earlier), which changes no
 *                  result: a stopped spectrum's iterations do nothing.
 *  clean_every, clean_max  the Clean strategy of Section 2.2 (steps 6 and 8):
 *                  after every clean_every Adam steps (at most clean_max
 *                  times; the paper's 30 and 11) the model at the current
 *                  parameters gives each spectrum's residual, the three-step
 *                  clipping of lasp_clean_mask (f_shift 0.5 at the first
 *                  update, 0.2 after) gives its mask, and clipped pixels get
 *                  zero weight until the next update.  0 = No Clean.
 *  out_mask        optional device uint8 [n_spec][n_pix]: the last Clean
 *                  mask (1 kept, 0 clipped; all 1 if no update ran).
 *  n_classes       1, or 3: the interpolator of Eq. 1 over the five Teff
 *                  regimes of the emulator, with one set of 20 coefficient
 *                  spectra per temperature class (cool, warm, hot; basis rows
 *                  20 q .. 20 q + 19 for class q).  At T = 10^(log10 Teff)
 *                  with a = clamp((T - e0) / (e1 - e0)) and
 *                  b = clamp((T - e2) / (e3 - e2)) the classes weigh 1 - a,
 *                  a (1 - b) and a b: one class inside the regimes T <= e0,
 *                  e1 <= T <= e2 and T >= e3, a linear blend in Teff across
 *                  (e0, e1) and (e2, e3).  BF16X3 supports one class only.
 *  class_edges     e0 < e1 < e2 < e3 in K (default 4000, 4550, 7000, 9000).
 *  step_graph      1 (default): lasp_fit_group enqueues its Adam steps as
 *                  replays of one HIP graph of 25 steps when no stopping
 *                  rules, no Clean and one emulator class are asked for
 *                  (the steps then launch the same kernels with the same
 *                  arguments) and n_spec <= 4096 (larger groups launch
 *                  long kernels); the graph is captured on first use and kept
 *                  with the call's cached device scratch until the
 *                  geometry, the buffers or the Adam settings change, and
 *                  the results are those of launching each step's kernels
 *                  (0).  Kernel timing (lasp_profile_enable) launches
 *                  them one by one.
 */
typedef struct lasp_opts {
  int32_t n_spec;
  int32_t n_pix;
  int32_t n_basis;
  int32_t margin;
  int32_t degree;
  int32_t precision;
  double box_lo[LASP_N_PAR];
  double box_hi[LASP_N_PAR];
  float lr, beta1, beta2, eps;
  float weight_quantile;
  int32_t n_arms;
  int32_t arm_start[LASP_MAX_ARMS];
  float arm_sigma_kms[LASP_MAX_ARMS];
  void *stream;
  uint32_t *status;
  double *out_chi2;
  int32_t stop_window;
  float stop_tol;
  int32_t *out_steps;
  int32_t polish_iters;
  int32_t clean_every;
  int32_t clean_max;
  uint8_t *out_mask;
  int32_t n_classes;
  double class_edges[4];
  int32_t step_graph;
} lasp_opts;

/* Defaults: n_basis 20, margin 64, degree 10, FP32, box
 * lo = (log10 4000, 1, -2.5, -300, 50), hi = (log10 8000, 5, 0.5, 300, 150),
 * lr 1e-2, betas (0.9, 0.999), eps 1e-8, weight_quantile 0.5, no arms,
 * null stream, no status/chi2 outputs, stopping rules off (stop_window 0,
 * stop_tol 1e-5), no out_steps, no polish, No Clean (clean_every 0,
 * clean_max 11), no out_mask, one emulator class (class_edges 4000, 4550,
 * 7000, 9000 K).  n_spec and n_pix are set to 0. */
void lasp_default_opts(lasp_opts *opts);

/*
 * Grouped fit (Section 2.2, stages 2-9): n_steps Adam steps on every
 * spectrum's chi2 / n_eff, then optionally the covariance.
 *   obs          [B][P] float   observed flux (any scale)
 *   ivar         [B][P] float   inverse variance; <= 0 or non-finite masks a pixel
 *   wave_grid    HOST [P] double  pixel wavelengths (A); must be uniform in
 *                log10 to 1e-6 of the step, else LASP_E_GRID
 *   basis        [20 n_classes][P+2M] float interpolator coefficient spectra
 *   init_params  [B][5] float   start, physical units
 *   out_params   [B][5] float   result, physical units (may alias init_params)
 *   out_cov      [B][5][5] double covariance in physical units, or NULL
 *   n_steps      >= 0 Adam steps
 * Returns LASP_OK or a LASP_E_* code.
 */
int lasp_fit_group(const float *obs, const float *ivar, const double *wave_grid,
                   const float *basis, const float *init_params, float *out_params,
                   double *out_cov, int32_t n_steps, const lasp_opts *opts);

/*
 * Model at fixed normalised parameters (one forward pass and its adjoint).
 *   u         [B][5] float normalised parameters
 *   out_model [B][P] float  C (.) F'' in the units of obs, or NULL
 *   out_chi2  [B] double    chi2 = sum_j W_j (o_j - C_j F''_j)^2 (required)
 *   out_J     [B] float     objective J = chi2 / n_eff (0 when n_eff = 0), or NULL
 *   out_neff  [B] int32     pixels with positive weight, or NULL
 *   out_grad  [B][5] float  dJ/du with the continuum held at its least-squares
 *             value (envelope theorem), or NULL
 *   out_jac   [B][5][P] float d model / d u at fixed continuum, or NULL
 *   out_cov   [B][5][5] double covariance at u in physical units
 *             (Section 2.2 stage 9), or NULL
 * Other arguments as in lasp_fit_group (opts->out_chi2 is ignored).
 */
int lasp_forward(const float *obs, const float *ivar, const double *wave_grid,
                 const float *basis, const float *u, float *out_model, double *out_chi2,
                 float *out_J, int32_t *out_neff, float *out_grad, float *out_jac,
                 double *out_cov, const lasp_opts *opts);

/*
 * lasp_forward without allocation: the same evaluation and outputs as
 * lasp_forward (same arguments, same kernels, bitwise the same results), for
 * callers that cannot allocate device memory -- code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  It calls no
 * hipMalloc, hipFree or allocating library routine: its scratch (F', F-bar',
 * the per-spectrum state and the padded basis) lives in one fixed device
 * array of 64 MiB per device (LASP_NOALLOC_SCRATCH_BYTES), held from the
 * library's first kernel launch on a device until the process ends.  The
 * caller still passes every input and output.
 *  - Sizes: the call returns LASP_E_NOMEM, enqueuing nothing, when B spectra
 *    of the shape need more than the array; at 3,900 pixels, margin 64, that
 *    is about 980 spectra (about 570 with out_jac or out_cov).
 *  - Every call on one device shares that device's array and clears the part
 *    it uses (with a fill kernel) before using it; calls that overlap on one
 *    device, on different streams or host threads, race and give undefined
 *    results.  Calls on one stream are ordered and safe.
 */
#define LASP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int lasp_forward_noalloc(const float *obs, const float *ivar, const double *wave_grid,
                         const float *basis, const float *u, float *out_model, double *out_chi2,
                         float *out_J, int32_t *out_neff, float *out_grad, float *out_jac,
                         double *out_cov, const lasp_opts *opts);

/*
 * Clean outlier mask (Section 2.2, step 6) of each spectrum from its
 * residual eps = obs - model, in three steps:
 *   B  |eps_j| - f_shift G_j > k sigma, with G_j = max |model_j - model_{j+-1}|
 *      and k = 3, relaxed to 4, 5, 7 while more than 3 % of the valid
 *      pixels would be clipped;
 *   C  a neighbour of a B outlier with |eps| - f_shift G > 2 sigma;
 *   D  a neighbour j' of an outlier j with eps_j eps_j' > 0,
 *      |eps_j'| <= |eps_j| and |eps_j'| - f_shift G_j' > sigma', repeated
 *      until it does not change (at most 20 passes).
 * sigma is the sample standard deviation of eps over the valid pixels
 * (finite obs and ivar, ivar > 0) and sigma' over those kept by B and C.
 * Only valid pixels are clipped or seed a neighbour test.
 *   obs, ivar, model  [B][P] float (device)
 *   keep              [B][P] uint8 (device): 1 kept (or invalid), 0 clipped
 *   n_masked          optional [B] int32 (device): clipped valid pixels
 * Uses opts->n_spec, n_pix, margin (for the pixel layout) and stream.
 */
int lasp_clean_mask(const float *obs, const float *ivar, const float *model, float f_shift,
                    uint8_t *keep, int32_t *n_masked, const double *wave_grid,
                    const lasp_opts *opts);

/*
 * Flux-conserving resampling (Section 2.2, step 3, Eqs. 2-4) of n_rows
 * spectra from a linear wavelength grid onto a grid uniform in log10.
 * Source row r holds the flux of bins centred at lam0 + i dlam (i < n_src,
 * width dlam); target pixel j of n_out has edges 10^(lg0 + (j -+ 1/2) dlog10).
 * out[r][j] is the integral of the piecewise-constant source over target
 * bin j divided by the bin's width: the difference quotient of the
 * cumulative integral (Eq. 2) interpolated linearly at the edges (Eq. 3),
 * Eq. 4.  The result is linear in the source and independent of the fitted
 * parameters, so a basis is resampled once (each of its rows is a spectrum).
 *   src      device float [n_rows][ld_src], ld_src >= n_src
 *   out      device float [n_rows][ld_out], ld_out >= n_out (not aliasing src)
 *   stream   hipStream_t (NULL: the null stream); the call is asynchronous.
 * The arithmetic is FP64; out is rounded to FP32.  Returns LASP_E_GRID if a
 * target edge falls outside the source range [lam0 - dlam/2,
 * lam0 + (n_src - 1/2) dlam], LASP_E_ARG for other invalid arguments.
 */
int lasp_resample(const float *src, int32_t n_rows, int32_t n_src, int64_t ld_src, double lam0,
                  double dlam, float *out, int32_t n_out, int64_t ld_out, double lg0,
                  double dlog10, void *stream);

/*
 * Kernel timing for benchmarks.  lasp_profile_enable(mask) clears the
 * counters and, for every kernel class whose bit (1 << LASP_K_*) is set in
 * mask, brackets each later launch with a pair of hipEvents recorded on the
 * launch's stream (mask 0 switches timing off).  lasp_profile_read waits for
 * the recorded events and returns, per class, the summed kernel time in ms
 * and the number of launches (arrays of n <= LASP_NK entries, host memory).
 * Timing adds two event records per bracketed launch.  Not thread safe:
 * use from one host thread.
 */
#define LASP_K_PREPARE 0
#define LASP_K_INTERP_FWD 1
#define LASP_K_FUSED 2
#define LASP_K_INTERP_BWD 3
#define LASP_K_COV 4
#define LASP_K_FINALIZE 5
#define LASP_NK 6
int lasp_profile_enable(uint32_t mask);
int lasp_profile_read(double *total_ms, int64_t *launches, int32_t n);

/*
 * Resident slot pools for continuous batching (serving).  A pool holds up to
 * opts->n_spec fits of one spectral shape (opts: n_pix, margin, degree, arms,
 * precision, box, Adam settings; the grid and basis are copied at creation)
 * on the current device, with per-slot Adam state (u, m, v, step count) kept
 * in device memory between calls.  All work is enqueued on opts->stream.
 *   lasp_pool_slot_bytes  device bytes one slot occupies (for admission by
 *                         memory footprint); 0 if opts are invalid.
 *   lasp_pool_create      allocates the pool (LASP_E_NOMEM if it does not fit).
 *   lasp_pool_load        prepares `count` spectra (obs, ivar [count][P],
 *                         init_params [count][5], device) into slots
 *                         [slot0, slot0 + count) and sets their step target
 *                         to n_steps; their step counts restart at 0.
 *   lasp_pool_step        advances every slot in [0, slot_end) whose step
 *                         count is below its target by up to k Adam steps
 *                         (Section 2.2 stages 2-8); other slots are untouched.
 *                         With opts->stop_window > 0 a slot also stops when a
 *                         stopping rule holds (its target becomes its count).
 *   lasp_pool_progress    writes, for slots [slot0, slot0 + count), the Adam
 *                         steps taken (steps [count], device int32) and 1 if
 *                         the slot has stopped, else 0 (done [count], device
 *                         int32); either pointer may be NULL.
 *   lasp_pool_finish      evaluates slots [slot0, slot0 + count) at their
 *                         current parameters and writes out_params [count][5]
 *                         (physical units), optional out_cov [count][5][5],
 *                         status [count] and chi2 [count] (device).
 *   lasp_pool_destroy     waits for the pool's stream and frees it.
 * Slots are independent: a fit's result does not depend on which other
 * slots are occupied.  Calls on one pool must come from one host thread.
 */
typedef struct lasp_pool lasp_pool;
size_t lasp_pool_slot_bytes(const lasp_opts *opts, const double *wave_grid);
int lasp_pool_create(const double *wave_grid, const float *basis, const lasp_opts *opts,
                     lasp_pool **out);
int lasp_pool_load(lasp_pool *pool, int32_t slot0, int32_t count, const float *obs,
                   const float *ivar, const float *init_params, int32_t n_steps);
int lasp_pool_step(lasp_pool *pool, int32_t slot_end, int32_t k);
int lasp_pool_progress(lasp_pool *pool, int32_t slot0, int32_t count, int32_t *steps,
                       int32_t *done);
int lasp_pool_finish(lasp_pool *pool, int32_t slot0, int32_t count, float *out_params,
                     double *out_cov, uint32_t *status, double *chi2);
int lasp_pool_destroy(lasp_pool *pool);

/*
 * Pool capacity and footprint.
 *   lasp_pool_resize    makes the pool hold `capacity` slots, keeping the
 *                       state of slots [0, keep) (keep <= both capacities);
 *                       slots past `keep` become idle.  Enqueued on the pool's
 *                       stream; returns after that stream has finished every
 *                       earlier step (the old buffers are then freed).
 *                       LASP_E_NOMEM leaves the pool as it was.
 *   lasp_pool_bytes     device bytes the pool holds now (capacity x slot
 *                       bytes + its basis copies).
 *   lasp_pool_capacity  slots the pool holds now.
 */
int lasp_pool_resize(lasp_pool *pool, int32_t capacity, int32_t keep);
size_t lasp_pool_bytes(const lasp_pool *pool);
int32_t lasp_pool_capacity(const lasp_pool *pool);

/*
 * Fit server: continuous batching of fit requests over slot pools under one
 * device-wide HBM budget (the serving pattern of grouped fitting, Section 2.2
 * stages 2-9 per request; group sizes as in the paper's Section 4.1 and
 * Table 2, shapes as in its Section 4.4).
 *
 * A server owns one slot pool per spectral shape (lasp_server_add_shape:
 * pixel grid, basis, arms, continuum degree, precision, Adam settings and
 * optional stopping rules, as lasp_opts of lasp_pool_create; opts->n_spec
 * and opts->stream are ignored) and a worker thread on the device that was
 * current at lasp_server_create.  A request is a group of `count` spectra of
 * one shape (obs, ivar [count][P], init_params [count][5], device).
 *  - Admission by HBM footprint: the pools together hold at most
 *    hbm_budget bytes (lasp_pool_bytes summed over shapes).  A request is
 *    admitted, in arrival order within its shape, when a contiguous range of
 *    `count` free slots exists in its shape's pool, or when the pool can grow
 *    to provide one within the budget; a pool gives capacity back (shrinks to
 *    its occupied prefix) when another shape's request waits for bytes.
 *    Pools grow and shrink in multiples of capacity_quantum slots (live
 *    fits are copied, never restarted).
 *  - Continuous batching: every tick, each shape with resident fits gets one
 *    launch sequence of up to steps_per_tick Adam steps covering all of its
 *    resident fits (per-fit Adam state stays on the device); the shapes run
 *    on streams of their own and overlap on the device.  A fit's arithmetic
 *    does not depend on which other fits are resident: a request's results
 *    are the same alone and in any mix.
 *  - A request finishes after n_steps Adam steps or, with the shape's
 *    stopping rules on, once every one of its fits has stopped; it is then
 *    evaluated (lasp_pool_finish) into the caller's output arrays and
 *    reported by lasp_server_poll once that work has completed on the
 *    device.
 *
 * lasp_server_default_opts  hbm_budget 0 (= three quarters of the device's
 *                         free memory at creation), n_steps 500,
 *                         steps_per_tick 25, want_cov 0,
 *                         capacity_quantum 1024.
 * lasp_server_create      starts the server (no shapes yet).
 * lasp_server_add_shape   adds a shape before the first submit; its id is
 *                         0, 1, ... in order (at most LASP_SERVER_MAX_SHAPES).
 *                         LASP_E_NOMEM if its first quantum of slots does not
 *                         fit the budget.
 * lasp_server_submit      queues a request.  Inputs and outputs are device
 *                         arrays owned by the caller that must stay valid
 *                         until the request is reported done; the inputs
 *                         must be ready when submit is called (their
 *                         producing work finished).  Outputs: out_params
 *                         [count][5] float (physical units, required),
 *                         out_cov [count][5][5] double (used when want_cov),
 *                         out_status [count] uint32 (LASP_ST_* bits) and
 *                         out_chi2 [count] double (either may be NULL).
 *                         LASP_E_NOMEM if the request could never fit the
 *                         budget.  *request_id receives its id (0, 1, ...).
 * lasp_server_poll        moves up to max_done finished requests into
 *                         done[] (HOST array) and sets *n_done; waits up to
 *                         timeout_ms for the first one (0: does not wait).
 *                         Times are seconds on the server's steady clock,
 *                         from lasp_server_create.
 * lasp_server_stats       counters and the current footprint (HOST struct).
 * lasp_server_destroy     stops the worker, waits for the device work it
 *                         enqueued and frees the pools; requests not yet
 *                         reported are abandoned (their outputs undefined).
 * A failure on the worker thread (a HIP error) stops the server: later
 * submit, poll and stats calls return its code, and lasp_last_error() its
 * message.  All calls are thread safe.
 */
#define LASP_SERVER_MAX_SHAPES 8
typedef struct lasp_server lasp_server;
typedef struct lasp_server_opts {
  size_t hbm_budget;
  int32_t n_steps;
  int32_t steps_per_tick;
  int32_t want_cov;
  int32_t capacity_quantum;
} lasp_server_opts;
typedef struct lasp_request_info {
  int64_t id;
  int32_t shape;
  int32_t count;
  int32_t max_steps;  /* Adam steps the request's launches covered (each of
                         its fits took at most this many) */
  int32_t stopped;    /* 1: finished by the stopping rules before n_steps */
  double t_submit, t_admit, t_done;
} lasp_request_info;
typedef struct lasp_server_counters {
  size_t hbm_budget;
  size_t hbm_in_use;  /* bytes the pools hold now */
  int64_t submitted, completed, ticks, resizes;
  int32_t queued, active, finishing;
  int32_t n_shapes;
  int32_t capacity[LASP_SERVER_MAX_SHAPES];
  int32_t used_slots[LASP_SERVER_MAX_SHAPES];
} lasp_server_counters;
void lasp_server_default_opts(lasp_server_opts *opts);
int lasp_server_create(const lasp_server_opts *opts, lasp_server **out);
int lasp_server_add_shape(lasp_server *server, const double *wave_grid, const float *basis,
                          const lasp_opts *opts, int32_t *shape_id);
int lasp_server_submit(lasp_server *server, int32_t shape, int32_t count, const float *obs,
                       const float *ivar, const float *init_params, float *out_params,
                       double *out_cov, uint32_t *out_status, double *out_chi2,
                       int64_t *request_id);
int lasp_server_poll(lasp_server *server, lasp_request_info *done, int32_t max_done,
                     int32_t timeout_ms, int32_t *n_done);
int lasp_server_stats(lasp_server *server, lasp_server_counters *stats);
int lasp_server_destroy(lasp_server *server);

/* Message describing the last failure on the calling thread ("" if none). */
const char *lasp_last_error(void);

/* Frees all cached device scratch memory on every device. */
void lasp_release(void);

#ifdef __cplusplus
}
#endif

#endif /* LASP_H */
