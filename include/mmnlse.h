/*
 * mmnlse.h -- RK4IP propagation of coupled multimode nonlinear Schroedinger
 * equations on one AMD Instinct MI355X (gfx950).
 *
 * The library advances a field A[M][T] (M modes, T time samples per mode)
 * along a fiber with the fourth-order Runge-Kutta method in the interaction
 * picture, Eq. (6a-f) of Brehler, Schirwon, Krummrich, Goeddeke,
 * "Simulation of Nonlinear Signal Propagation in Multimode Fibers on
 * Multi-GPU Systems" (Section 3.2), with:
 *
 *   linear part (Eq. 1, operator L): -alpha_p/2 + i sum_n beta_{n,p} (-w)^n / n!
 *       applied per mode in the frequency domain (Section 3.1);
 *   Kerr part: N_p = i gamma sum_{l,m,n} S_plmn A_l A_m conj(A_n), the
 *       general multimode form the paper cites in Section 2 (for M = 1 it is
 *       the paper's gamma |A|^2 A), or, with MMNLSE_KERR_MANAKOV, the
 *       paper's own operator of Eq. (1), N_a = i gamma (sum_b kappa_ab
 *       |A_b|^2) A_a.
 *
 * Also: the two split-step variants of Section 3.1 for comparison
 * (mmnlse_method), fiber spans with loss-compensating amplifiers
 * (mmnlse_config.span_km, Section 5), an adaptive step size from the
 * step-doubling estimate, and a continuous-batching server.
 *
 * Conventions
 *   - Units: t in ps, z in km, power in W, beta_n in ps^n/km, gamma in 1/(W km).
 *   - Fields are complex, interleaved (re, im), row-major [M][T]: each mode's
 *     T samples are contiguous (the paper's row-major signal matrix,
 *     Section 4).  T must be a power of two, 64 <= T <= 2^20.
 *   - Forward transform kernel exp(-i w t); w = 2 pi fftfreq(T, dt) with the
 *     Nyquist bin negative.
 *   - Eq. (6b) is read as k1 = exp(h/2 L)[h N(A(z))].
 *   - Device pointers must belong to the handle's device and are used in
 *     stream order on the handle's stream.  The caller owns every pointer it
 *     passes; nothing is retained after a call returns.
 *   - Every function returns an mmnlse_status and never throws.  On error
 *     mmnlse_last_error() describes the failure (thread-local string, valid
 *     until the next call on the same thread).  A failed call leaves the
 *     handle usable, except after MMNLSE_E_DEVICE.
 *   - One handle must not be used from two host threads at once.
 */
#ifndef MMNLSE_H
#define MMNLSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MMNLSE_OK = 0,
  MMNLSE_E_INVALID = 1,     /* bad argument or configuration */
  MMNLSE_E_NOMEM = 2,       /* device or host allocation failed, or budget exceeded */
  MMNLSE_E_DEVICE = 3,      /* HIP runtime error */
  MMNLSE_E_NONFINITE = 4,   /* NaN or Inf found in an input or result */
  MMNLSE_E_BUSY = 5,        /* request not finished yet (serving) */
  MMNLSE_E_UNSUPPORTED = 6, /* valid request the library does not implement */
  MMNLSE_E_STEP = 7         /* adaptive stepping could not reach the end (step below
                               h_min, or max_trials used up) */
} mmnlse_status;

/* Arithmetic of the Kerr contraction; FFTs and field storage are FP32 in both. */
typedef enum {
  MMNLSE_FP32 = 0,        /* FP32 products, FP32 accumulation */
  MMNLSE_SPLIT_BF16 = 1,  /* S and A_l A_m split into bf16 hi + lo; hi*hi + hi*lo + lo*hi
                             on matrix cores with FP32 accumulation (needs a symmetric S) */
  MMNLSE_SPLIT_BF16_S = 2 /* S split into bf16 hi + lo, A_l A_m rounded to bf16 (nearest
                             even); hi*B + lo*B, two matrix-core products instead of three,
                             FP32 accumulation (needs a symmetric S).  The rounding of the
                             products dominates its error, which grows like sqrt(steps) */
} mmnlse_precision;

typedef enum { MMNLSE_C64 = 0, MMNLSE_C128 = 1 } mmnlse_dtype;

/* Stepping method.  RK4IP is the paper's method, Eq. (6a-f); SSFM_RK4 is the
 * symmetric split-step of Eq. (4) with the nonlinear part integrated over h
 * by classical RK4 (the paper's "SSFM-RK4" variant, Section 3.1): half a
 * linear step, four Kerr evaluations, half a linear step (consecutive half
 * steps inside one call are applied as one full step).  SSFM_AGRAWAL
 * (MMNLSE_KERR_MANAKOV plans only) is the same split-step with the
 * nonlinear integral taken by the trapezoidal rule (the paper's
 * "SSFM-Agrawal", Section 3.1): for the Manakov operator the nonlinear step
 * is the phase rotation exp(i gamma h/2 kappa (|A(z)|^2 + |A(z+h)|^2)), with
 * A(z+h) first replaced by A(z) and then by the field the first pass
 * reached (two passes; three half-step propagators per step). */
typedef enum { MMNLSE_RK4IP = 0, MMNLSE_SSFM_RK4 = 1, MMNLSE_SSFM_AGRAWAL = 2 } mmnlse_method;

/* S is symmetric in (l,m) and in (p,n): S_plmn == S_pmln == S_nlmp (checked to
 * 1e-6 relative at create).  Enables the packed contraction over the
 * P = M(M+1)/2 pairs.  Every tensor symmetric under all index permutations
 * qualifies. */
#define MMNLSE_S_SYMMETRIC 0x1u
/* Force the unpacked per-sample Kerr kernel (any S). */
#define MMNLSE_KERR_GENERIC 0x2u
/* Use the paper's own nonlinear operator of Eq. (1) (Manakov / XPM form)
 * instead of the tensor form: N_a = i gamma (sum_b kappa_ab |A_b|^2) A_a with
 * the real [M][M] matrix `kappa` (kappa_aa intramodal, kappa_ab intermodal
 * coefficients; rows are spatial and polarization modes).  S is ignored and
 * may be NULL.  FP32 only. */
#define MMNLSE_KERR_MANAKOV 0x4u

typedef struct {
  int32_t M;             /* modes (rows), 1 <= M <= 256 */
  int32_t T;             /* samples per mode, power of two, 64 <= T <= 2^20 */
  double dt_ps;          /* sample spacing in ps, > 0 */
  int32_t n_beta;        /* number of Taylor coefficients beta_0..beta_{n_beta-1}, 0..8 */
  const double *beta;    /* [M][n_beta] host array, ps^n/km; copied at create */
  const double *alpha;   /* [M] host array, power attenuation in 1/km, or NULL for 0 */
  const float *S;        /* [M][M][M][M] host array, index order (p,l,m,n); copied
                            (may be NULL with MMNLSE_KERR_MANAKOV) */
  double gamma;          /* nonlinear coefficient, 1/(W km) */
  double h_km;           /* step size, > 0 */
  double L_km;           /* fiber length; L/h must be an integer within 1e-9 relative */
  int32_t precision;     /* mmnlse_precision */
  uint32_t flags;        /* MMNLSE_S_SYMMETRIC | MMNLSE_KERR_GENERIC | MMNLSE_KERR_MANAKOV */
  const float *kappa;    /* [M][M] host array (row a, column b), used with
                            MMNLSE_KERR_MANAKOV, else ignored; copied */
  int32_t method;        /* mmnlse_method (0 = RK4IP) */
  int32_t diag_every;    /* mmnlse_propagate: FP64 diagnostics every this many steps
                            (power drift; for RK4IP also the step-doubling local-error
                            estimate), 0 = only power at the end; >= 0 */
  double span_km;        /* fiber span between amplifiers (Section 5: two 80 km spans with
                            the loss compensated after each), 0 = one unamplified fiber of
                            length L.  When > 0, span/h and L/span must be integers within
                            1e-9 relative; after every span mmnlse_propagate (and the
                            server) multiplies mode p by exp(alpha_p span / 2), the
                            noiseless flat-gain amplifier that restores the span's loss */
} mmnlse_config;

typedef struct {
  double power_in;       /* dt * sum |A_in|^2 in W ps, FP64 reduction on the device */
  double power_out;      /* same for the result */
  double seconds;        /* wall time of the step loop (host clock, synchronised),
                            diagnostics included */
  int64_t steps;         /* RK4IP steps taken */
  double power_drift_max; /* max |P(z)/P(0) - 1| over the diagnostic points (diag_every > 0) */
  double local_err_max;  /* max over the points of delta/15, delta the step-doubling estimate
                            of mmnlse_step_doubling from the state there (RK4IP plans) */
  int64_t diag_points;   /* diagnostic points taken (0 when diag_every == 0) */
} mmnlse_stats;

typedef struct mmnlse_ctx *mmnlse_t;

/* Device fields.  Every device pointer to a complex64 field [M][T] passed to
 * the calls below must be 16-byte aligned (hipMalloc and torch allocations
 * are): the transforms move two samples per access.  A misaligned pointer is
 * E_INVALID. */

/* Create a propagation plan on the current HIP device.
 * Copies beta, alpha and S to the device, tabulates exp(h/2 L) per mode and
 * bin in FP64 on the device (stored as FP32 hi + lo), the FFT twiddles
 * likewise on the host, and the
 * Kerr tensor in the layout of the selected kernel.  Allocates three field
 * buffers of M*T complex64 as workspace.  `stream` is a hipStream_t (NULL =
 * the default stream); the handle does not own it.  Synchronises the stream
 * before returning.
 * Errors: E_INVALID (sizes, L/h, symmetry flag not satisfied, split precision
 * without MMNLSE_S_SYMMETRIC), E_NOMEM (device or host memory; when the
 * environment variable MMNLSE_HOST_BYTES_LIMIT is set, set-ups whose host
 * tables would exceed that many bytes are refused before any device call),
 * E_DEVICE.  Never throws.
 * Environment variables read here select among equivalent schedules, for
 * measurement and tests (results stay within the stated tolerances, and
 * are bit-identical where noted):
 *   MMNLSE_FORCE_FOUR_STEP=1|0  four-step transform from T >= 1024 / single
 *                               pass up to T = 16384
 *   MMNLSE_KERR_PATH=0|1|2      FP32 Kerr kernel: small-M registers (M <= 8),
 *                               tiled generic, matrix cores (symmetric S)
 *   MMNLSE_MFMA_RT=2|4          row tiles per pass of the per-pass kernel
 *   MMNLSE_GROUP_KERNEL=0|1     never / always the matrix-core kernel that
 *                               forms B once per workgroup (default: dense
 *                               tensors only)
 *   MMNLSE_SOLO=0|1             one-mode fields: never / up to T = 4096 whole
 *                               steps in one workgroup (default T <= 2048;
 *                               bit-identical to the launched schedule)
 *   MMNLSE_GRAPH=0              no step-graph replay (read at each call;
 *                               bit-identical)
 *   MMNLSE_HOST_BYTES_LIMIT=n   see E_NOMEM above */
mmnlse_status mmnlse_create(const mmnlse_config *cfg, void *stream, mmnlse_t *out);

/* Release everything create allocated.  NULL is accepted. */
mmnlse_status mmnlse_destroy(mmnlse_t h);

/* Thread-local description of the last error on this thread ("" if none). */
const char *mmnlse_last_error(void);

/* Propagate over the configured length, L/h RK4IP steps (Eq. 6a-f).
 * With cfg->span_km > 0 the amplifier of mmnlse_amplify acts after every
 * span (span/h steps), the last one included.
 * With cfg->diag_every = k > 0 the steps run in chunks of k (bit-identical to
 * one run) and after each chunk the FP64 power and, for RK4IP plans, the
 * step-doubling estimate are taken from the state (see mmnlse_stats).
 * A_in, A_out: [M][T] complex of type `dtype` (mmnlse_dtype); host pointers
 * when on_device == 0 (the call then copies, runs and synchronises), device
 * pointers when on_device != 0 (still synchronises before returning, so
 * that `st` is filled).  A_out may equal A_in.  complex128 data is rounded
 * to complex64 on the device before the first step.  `st` may be NULL.
 * Errors: E_INVALID, E_NONFINITE (non-finite input or result power),
 * E_DEVICE. */
mmnlse_status mmnlse_propagate(mmnlse_t h, const void *A_in, void *A_out, int32_t dtype,
                               int32_t on_device, mmnlse_stats *st);

/* Advance a device-resident complex64 field A[M][T] in place by n_steps
 * RK4IP steps of size h (n_steps >= 0), asynchronously on the handle's
 * stream.  This is the hot path with no host transfer and no host sync.
 * For fields of at most 2^20 samples (M*T), where a step is a few short
 * kernels, the middle steps of calls with n_steps >= 18 run as replays of a
 * HIP graph of 16 steps, captured by the first call that passes a given A
 * (on an internal stream; replayed on the handle's stream) -- the same
 * kernels in the same order, so the result is bit-identical to the eager
 * schedule.  The environment variable MMNLSE_GRAPH=0 disables this.
 * Every call starts afresh from A: for RK4IP and SSFM-RK4 plans the result
 * of several calls is bit-identical to one call over their steps; an
 * SSFM-Agrawal plan on the four-step transform computes the first half step
 * of a call's first step by itself (within a call, and within
 * mmnlse_propagate and the server, it comes from the previous step's dual
 * transform), so split calls differ from one call at FP32 rounding level.
 * Errors: E_INVALID, E_DEVICE (launch failure). */
mmnlse_status mmnlse_advance(mmnlse_t h, void *A, int64_t n_steps);

/* The amplifier at the end of a span (Section 5): multiplies row p of the
 * device complex64 field A[M][T] in place by exp(alpha_p span_km / 2), flat in
 * frequency, which restores the power the span's attenuation took.  For
 * composing mmnlse_advance calls span by span (mmnlse_advance itself never
 * amplifies).  Asynchronous.  Errors: E_INVALID (null argument, or the plan
 * has span_km == 0), E_DEVICE. */
mmnlse_status mmnlse_amplify(mmnlse_t h, void *A);

/* One application of the half-step linear propagator exp(h/2 L) (the
 * operator of Eq. 6a) to every row: Y = IFFT(exp(h/2 L) * FFT(X)).
 * X, Y: device complex64 [M][T]; Y may equal X.  Asynchronous. */
mmnlse_status mmnlse_linear_half_step(mmnlse_t h, const void *X, void *Y);

/* The Kerr increment Y = h * N(X), N_p = i gamma sum S_plmn X_l X_m conj(X_n)
 * (the bracketed terms of Eq. 6b-e), with the handle's tensor and precision.
 * X, Y: device complex64 [M][T]; Y must not overlap X.  Asynchronous. */
mmnlse_status mmnlse_kerr(mmnlse_t h, const void *X, void *Y);

/* FP64 reduction of dt * sum_p sum_t |X_p(t)|^2 for a device complex64
 * field; synchronises and writes *out (host).  Total power is conserved by
 * Eq. (1) for alpha = 0 and a tensor with S_plmn == S_lpnm. */
mmnlse_status mmnlse_power(mmnlse_t h, const void *X, double *out);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, serving loops and harnesses that forbid hipMalloc): the power of
 * mmnlse_power without a handle and without any allocation or host sync.
 * X: device complex64 array of n values (a field [M][T] has n = M*T) on the
 * current device, 8-byte aligned; dt_ps: sample spacing (finite, > 0);
 * out: device pointer to one double, 8-byte aligned, that receives
 * dt_ps * sum |X|^2 computed in FP64.  Asynchronous on `stream` (a
 * hipStream_t, NULL = the default stream).  For the same n and dt the value
 * is bit-identical to mmnlse_power's (same blocks, same summation order).
 * Scratch: a fixed device array of 1024 FP64 partial pairs (16 KiB) in the
 * library, one per device, whose address is looked up on the first call on
 * each device and which each device holds until the process ends.  Every
 * call writes all the partials it reads, so nothing needs clearing, but all
 * calls on one device share the array: calls that overlap on one device
 * (several streams or threads) race and must be serialised by the caller.
 * The partial count is n/4096 clamped to 1..1024, so every n up to
 * MMNLSE_NOALLOC_MAX_VALUES fits the scratch.
 * Errors: E_INVALID (null or misaligned pointer, n outside
 * 1..MMNLSE_NOALLOC_MAX_VALUES, bad dt_ps; checked before any device call),
 * E_DEVICE (no current device, symbol lookup or launch failure). */
#define MMNLSE_NOALLOC_MAX_VALUES ((int64_t)1 << 40)
mmnlse_status mmnlse_power_noalloc(const void *X, int64_t n, double dt_ps, double *out, void *stream);

/* Step-doubling local error estimate (Richardson), RK4IP plans only
 * (E_UNSUPPORTED otherwise): from device field X,
 * takes two RK4IP steps of h and one step of 2h, and writes
 * delta = ||fine - coarse|| / ||fine|| computed in FP64 to *delta (host).
 * The error of the fine result is about delta/15 (fourth order, Section
 * 3.2).  X is not modified.  Synchronises. */
mmnlse_status mmnlse_step_doubling(mmnlse_t h, const void *X, double *delta);

/* Adaptive step size driven by the step-doubling estimate.  The paper uses
 * fixed steps; the control is the textbook step-doubling scheme for
 * Runge-Kutta methods, with the exponent 1/5 from the fifth-order local
 * error of RK4IP (Section 3.2):
 *   a trial of size h from position z takes one RK4IP step of h and two of
 *   h/2 from the same state and computes delta = ||fine - coarse|| / ||fine||
 *   (FP64 reduction; 0 for an all-zero field); it is accepted when
 *   delta <= tol, and then the state becomes the fine result and z += h;
 *   the next trial is h * clamp(0.9 (tol/delta)^(1/5), 0.5, 2) (2 when
 *   delta == 0, 0.5 when delta is not finite), at most h_max, cut to the
 *   distance left.  The propagation ends when less than 1e-12 of the length
 *   is left.
 * The plan's own h, L and tables are not used or changed; the propagator
 * tables for each new trial step are built on the device. */
typedef struct {
  double length_km;   /* distance to propagate, > 0 */
  double tol;         /* acceptance bound on delta, > 0 */
  double h_init_km;   /* first trial step, > 0 */
  double h_min_km;    /* a trial step below this fails with E_STEP (0 = no bound) */
  double h_max_km;    /* largest trial step (0 = no bound) */
  int64_t max_trials; /* bound on the number of trials, > 0 */
} mmnlse_adaptive_config;

typedef struct {
  double z_km;        /* position at the start of the trial */
  double h_km;        /* trial step */
  double delta;       /* ||fine - coarse|| / ||fine|| */
  int32_t accepted;   /* 1 if the fine result was kept */
  int32_t reserved;
} mmnlse_trial;

typedef struct {
  double z_km;        /* distance covered (the length on success) */
  double h_next_km;   /* step the controller would try next */
  int64_t accepted, rejected, trials;
  double seconds;     /* host wall time of the call */
} mmnlse_adaptive_result;

/* Propagate the device-resident complex64 field A[M][T] in place over
 * ac->length_km with adaptive steps (RK4IP plans only, else E_UNSUPPORTED).
 * The first min(trials, log_cap) trials are written to `log` (host array,
 * may be NULL when log_cap == 0); `res` (host) is always filled.
 * Synchronises once per trial to read delta.  On E_STEP, A holds the state
 * at res->z_km.  Allocates on first use two more tables and two fields of
 * M*T (kept until destroy).  Errors: E_INVALID, E_NOMEM, E_STEP, E_DEVICE. */
mmnlse_status mmnlse_propagate_adaptive(mmnlse_t h, void *A, const mmnlse_adaptive_config *ac,
                                        mmnlse_trial *log, int64_t log_cap,
                                        mmnlse_adaptive_result *res);

/* Measurement: run n_steps exactly like mmnlse_advance, with a HIP event
 * pair recorded on the handle's stream around every kernel-class launch,
 * synchronise, and report the summed device time per class in
 * ms[0] (Kerr launches) and ms[1] (linear half-step applications; a
 * four-step transform is three kernels timed as one application), with the
 * launch counts in counts[0], counts[1] and the number of Kerr evaluations
 * h N(.) in counts[2].  A one-mode RK4IP plan with 64 <= T <= 2048 (4096
 * with MMNLSE_SOLO=1 in the environment at create) runs all steps of a call
 * in one launch of one workgroup; that launch is reported
 * under ms[0] / counts[0] with no linear launches.  A is advanced in place.
 * Errors: E_INVALID, E_DEVICE. */
mmnlse_status mmnlse_profile(mmnlse_t h, void *A, int64_t n_steps, double *ms, int64_t *counts);

/* Wait for all work queued on the handle's stream. */
mmnlse_status mmnlse_synchronize(mmnlse_t h);

/* Bytes of device memory the handle holds (workspace, tables, tensor). */
mmnlse_status mmnlse_footprint(const mmnlse_t h, size_t *bytes);

/* Work of one Kerr evaluation per time sample on the matrix-core path
 * (E_UNSUPPORTED for the other paths), as counts of packed tensor entries:
 * entries[0] = P*P (P = M(M+1)/2, the dense packed contraction),
 * entries[1] = entries in the blocks the kernel multiplies (32 row slots by
 * one k-step, kept when they hold a nonzero entry; padding included),
 * entries[2] = nonzero entries.  Each entry costs 4 flops per sample (a real
 * multiply-add on the real and on the imaginary part of B_q).  Host array
 * of 3 doubles. */
mmnlse_status mmnlse_kerr_work(const mmnlse_t h, double *entries);

/* Host-only dry run of the matrix-core contraction plan for S (no device is
 * touched): the packed form Sp[(p,n)][(l,m)] = w S[p,l,m,n] (w = 2 for
 * l < m) of a tensor symmetric in (l,m) and in (p,n), over P = M(M+1)/2
 * pairs, with the column order, the row tiles and the blocks (32 row slots
 * x one k-step of 8 columns FP32 / 16 split) that mmnlse_create would use.
 * counts (host, 7 ints, required): P, Ppad (column positions: at least P,
 * a multiple of 32), number of passes, length of the k-list array, k-step
 * width in columns, largest number of row tiles per pass, number of row
 * tiles.  The arrays may be NULL; when given they must hold: perm [Ppad]
 * (natural pair index, in the order l <= m row-major, at each column
 * position, -1 for a zero padding column; every pair appears once), rows
 * [32 * row tiles] (natural pair index in each row slot, -1 for a zero
 * padding row; every pair appears once), passes [4 * number of passes]
 * (first row tile, row tiles, offset into klist, count), klist [length]
 * (k-steps each pass multiplies; a block outside every list is entirely
 * zero), entries [3] (as mmnlse_kerr_work).  Call once with NULL arrays to
 * get the sizes.  Errors: E_INVALID, E_NOMEM. */
mmnlse_status mmnlse_kerr_plan(const float *S, int32_t M, int32_t precision, int32_t *counts, int32_t *perm,
                               int32_t *rows, int32_t *passes, int32_t *klist, double *entries);

/* Kernel used for the Kerr term: 0 = per-sample register kernel (M <= 8),
 * 1 = generic LDS kernel (any S), 2 = packed matrix-core contraction,
 * 3 = Manakov / XPM form of Eq. (1). */
mmnlse_status mmnlse_kerr_path(const mmnlse_t h, int32_t *path);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of propagation requests on one device.
 *
 * A planner thread admits queued requests in arrival order while the summed
 * device footprint of the admitted ones stays within the budget (and at most
 * max_active are resident), and sets each one up (plan, field upload, input
 * power) on a stream of its own.  A worker thread keeps every admitted field
 * and its plan resident on the device and advances each request in ticks of
 * up to steps_per_tick RK4IP steps on one of n_streams HIP streams, so that
 * the kernels of different requests overlap on the device; each request's
 * next tick is launched as soon as its previous one has completed (an event
 * per request), independently of the other requests.  A request that has
 * taken its L/h steps is copied back and retired, which frees its memory
 * for the next admission.  A request advanced in ticks does exactly the
 * arithmetic of one mmnlse_propagate call, so its result is bit-identical
 * alone and in any mix.
 * ------------------------------------------------------------------------ */
typedef struct {
  size_t mem_budget_bytes;  /* device bytes the admitted requests may hold together;
                               0 = 80 % of the free device memory at create */
  int32_t max_active;       /* requests resident at once; 0 = 32 */
  int32_t n_streams;        /* HIP streams (default priority) requests are spread over; 0 = 4 */
  int32_t steps_per_tick;   /* RK4IP steps per tick of a request; 0 = 8 */
} mmnlse_server_config;

typedef struct {
  int64_t submitted, completed, failed;
  int32_t queued, active;
  size_t admitted_bytes;       /* footprint of the requests resident now */
  size_t peak_admitted_bytes;  /* largest admitted footprint seen */
  int64_t rounds;              /* ticks launched (over all requests) */
} mmnlse_server_counters;

typedef struct mmnlse_server *mmnlse_server_t;

/* Start a server (and its planner and worker threads) on the current HIP device.
 * Errors: E_INVALID, E_NOMEM, E_DEVICE. */
mmnlse_status mmnlse_server_create(const mmnlse_server_config *cfg, mmnlse_server_t *out);

/* Queue one propagation of the configuration `cfg` (validated like
 * mmnlse_create; its arrays are copied) from the host field A_in
 * ([M][T] of type `dtype`, copied).  *ticket identifies the request.
 * Thread-safe.  Errors: E_INVALID; E_NOMEM when the request alone exceeds
 * the memory budget. */
mmnlse_status mmnlse_server_submit(mmnlse_server_t s, const mmnlse_config *cfg, const void *A_in,
                                   int32_t dtype, uint64_t *ticket);

/* Non-blocking: E_BUSY while the request is queued or running.  Once it is
 * done, copies the result (type as submitted) to the host buffer A_out,
 * fills st (may be NULL) and *latency_s (submit to result on the host, may
 * be NULL), releases the ticket and returns the request's own status (OK,
 * or e.g. E_NONFINITE / E_DEVICE with mmnlse_last_error set).  Thread-safe.
 * E_INVALID for an unknown ticket. */
mmnlse_status mmnlse_server_poll(mmnlse_server_t s, uint64_t ticket, void *A_out, mmnlse_stats *st,
                                 double *latency_s);

/* As mmnlse_server_poll, but blocks until the request is done. */
mmnlse_status mmnlse_server_wait(mmnlse_server_t s, uint64_t ticket, void *A_out, mmnlse_stats *st,
                                 double *latency_s);

/* Counters of the scheduler.  Thread-safe. */
mmnlse_status mmnlse_server_stats(mmnlse_server_t s, mmnlse_server_counters *out);

/* Stop the worker after the resident requests finish; queued requests that
 * were never admitted are dropped.  Frees everything.  NULL is accepted. */
mmnlse_status mmnlse_server_destroy(mmnlse_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* MMNLSE_H */
