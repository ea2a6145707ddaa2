/*
 * few.h -- C ABI of libfew, an MI355X (gfx950) implementation of the
 * interpolated harmonic-mode summation of Katz, Chua, Speri, Warburton and
 * Hughes, "Fast extreme-mass-ratio-inspiral waveforms" (arXiv:2104.04582).
 *
 * The library computes, on a dense grid t_j = t_start + j dt (j < n_samples,
 * evaluated in binary64 exactly as written),
 *
 *   h(t_j) = scale * sum_{listed (l,m,n)} [ A_lmn(t_j) -2Y_lm(theta, phi) e^{-i psi}
 *            + [m > 0] (-1)^l conj(A_lmn(t_j)) -2Y_{l,-m}(theta, phi) e^{+i psi} ],
 *   psi = m Phi_phi(t_j) + n Phi_r(t_j)
 *
 * i.e. the Schwarzschild-eccentric sum of Eq. (10) (Sec. IV) with the
 * negative-m modes supplied by the amplitude symmetry of Eq. (9) (k = 0):
 * A_{l,-m,-n} = (-1)^l conj(A_lmn).  The output is h = h_plus - i h_cross
 * (Sec. II), so Re h = h_plus and Im h = -h_cross.  `scale` is the mu/d_L
 * prefactor of Eq. (10).
 *
 * A_lmn(t), Phi_phi(t) and Phi_r(t) are not-a-knot cubic splines through their
 * values on one shared sparse knot grid (Sec. III C, "Interpolated
 * Summation"); the real and imaginary parts of each amplitude are splined
 * separately (equivalent to a complex spline by linearity).
 *
 * Conventions
 *  - List only modes with 0 <= m <= l, l >= 2; the m < 0 partners are implied
 *    (Sec. III C).  m = 0 modes are summed once and never mirrored.
 *  - Initial phases are part of Phi_phi[0] and Phi_r[0].
 *  - Interval rule: sample t_j uses the cubic of the largest knot interval i
 *    (0 <= i <= K-2) with t_i <= t_j; the last interval is closed at t_{K-1}.
 *  - -2Y_lm follows the standard spin-weighted convention fixed by
 *    -2Y_22 = sqrt(5/(64 pi)) (1 + cos theta)^2 e^{2 i phi}.
 *
 * Memory and ownership
 *  - "host" pointers are read before the call returns.
 *  - "device" pointers are HIP device memory of the plan's device (for example
 *    torch tensors).  Inputs must stay alive and unmodified, and outputs must
 *    not be read, until the work has completed: for the synchronous calls,
 *    until the plan's stream passes the enqueued work; for few_submit, until
 *    few_poll returns something other than FEW_PENDING.
 *  - The library owns plan scratch, few_spline objects and request state,
 *    all carved from one device arena of hbm_budget_bytes per plan, and a
 *    little pinned host memory per plan: the upload staging buffers and, per
 *    stream the plan launches on, a 2 KiB array in which the matrix-core
 *    summation's workgroups report their times (the plan splits later
 *    launches' samples between the GPU's XCDs by them; results do not depend
 *    on the split).
 *
 * Errors
 *  - Every function returns a few_status.  Argument, knot and mode errors are
 *    detected on the host before anything is enqueued.  No C++ exception
 *    crosses this interface.  few_last_error() returns the calling thread's
 *    last message.
 *
 * Threading
 *  - few_submit / few_poll / few_wait are thread-safe.  The synchronous calls
 *    (few_spline_fit, few_mode_sum) take one plan per thread.
 */
#ifndef FEW_H
#define FEW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FEW_OK = 0,
    FEW_PENDING = 1,
    FEW_E_ARG = -1,        /* null pointer, dt <= 0, n_samples <= 0, NaN/Inf */
    FEW_E_KNOTS = -2,      /* K < 4, K > max_knots, knots not strictly increasing */
    FEW_E_MODES = -3,      /* M < 1, M > max_modes, l < 2, l > 30, m < 0, m > l, |n| > 1000 */
    FEW_E_RANGE = -4,      /* samples outside [t_0, t_{K-1}] */
    FEW_E_TOO_LARGE = -5,  /* request footprint exceeds the whole plan budget */
    FEW_E_NOMEM = -6,      /* arena or host allocation failed */
    FEW_E_HIP = -7,        /* a HIP runtime call failed */
    FEW_E_STATE = -8       /* bad handle, unknown ticket, plan being destroyed */
} few_status;

typedef enum {
    FEW_FP64 = 0,   /* every step in binary64 (phases in double-double) */
    FEW_MIXED = 1   /* binary64 spline solve, phases and mod-2pi reduction;
                       binary32 amplitude evaluation, harmonics and products,
                       compensated binary32 accumulation; complex64 output */
} few_precision;

enum {
    FEW_FLAG_TIMING = 1,      /* record HIP events around every kernel launch */
    FEW_FLAG_TIMING_SUM = 2,  /* record them around summation launches only: each event pair
                                 delays the launch after it by several microseconds, so this
                                 keeps the other stages back to back while the dominant
                                 kernel is timed */
    FEW_FLAG_VECTOR_ONLY = 4, /* FEW_MIXED: never use the matrix-core summation (fp16 hi/lo
                                 operands on the MFMA units, fp32 accumulation); every sum
                                 runs on the vector units in binary32 with Kahan-compensated
                                 accumulation */
    FEW_FLAG_TIMING_SPARSE = 16, /* with FEW_FLAG_TIMING_SUM: events around every 8th
                                   summation launch only (the first, the ninth, ... counted
                                   from plan creation or the last few_plan_timing reset), so
                                   the instrumentation delays one step in eight */
    FEW_FLAG_SELECT_SORTED = 8 /* few_mode_select: sort every knot and sum sequentially; by
                                 default a knot is decided from sums with a proven error
                                 bound and sorted only when a comparison falls within it
                                 (the result is the same either way) */
};

typedef struct few_plan_s *few_plan;
typedef struct few_spline_s *few_spline;

typedef struct {
    int32_t device;            /* HIP device ordinal */
    void *stream;              /* hipStream_t for the synchronous calls (borrowed; NULL = null stream) */
    int32_t precision;         /* few_precision */
    int32_t max_knots;         /* <= 1024; 0 -> 1024 */
    int32_t max_modes;         /* 0 -> 65536 */
    int32_t max_inflight;      /* served path: concurrent batch streams, 1..8; 0 -> 2 */
    uint64_t hbm_budget_bytes; /* device arena per plan; 0 -> 2 GiB */
    int32_t flags;             /* FEW_FLAG_* */
} few_plan_desc;

/* One served waveform request: the few_spline_fit arguments followed by the
 * few_mode_sum arguments (same meaning, layout and ownership). */
typedef struct {
    int32_t n_knots;
    const double *t_knots;     /* host [K] */
    const double *phi_phi;     /* device [K] */
    const double *phi_r;       /* device [K] */
    int32_t n_modes;
    const int32_t *lmn;        /* host [M][3] */
    const double *amp;         /* device [K][M][2], knot-major (re, im) */
    double theta, phi, scale, t_start, dt;
    int64_t n_samples;
    void *out;                 /* device complex128 (FEW_FP64) / complex64 (FEW_MIXED) [n_samples] */
} few_request;

/* Per-plan kernel timing (FEW_FLAG_TIMING), milliseconds summed over launches. */
typedef struct {
    double spline_ms;  int64_t spline_launches;
    double prepare_ms; int64_t prepare_launches;
    double sum_ms;     int64_t sum_launches;
} few_timing;

/* Create a plan on `desc->device`: validates the descriptor and reserves the
 * device arena.  *out is set only on FEW_OK. */
int32_t few_plan_create(const few_plan_desc *desc, few_plan *out);

/* Drain in-flight work on every plan stream and release the plan, its arena
 * and every few_spline made from it.  Outstanding tickets become invalid. */
int32_t few_plan_destroy(few_plan plan);

/*
 * Spline stage (Sec. III C): fit not-a-knot cubic splines to Phi_phi, Phi_r
 * and the real and imaginary part of every listed amplitude, all on the knot
 * grid t_knots, and keep the coefficients resident in the plan arena.
 *   K        number of knots, 4 <= K <= max_knots
 *   t_knots  host [K], strictly increasing
 *   phi_phi  device [K]  azimuthal phase at the knots (radians)
 *   phi_r    device [K]  radial phase at the knots (radians)
 *   M        number of listed modes, 1 <= M <= max_modes
 *   lmn      host [M][3] int32 (l, m, n), 2 <= l <= 30, 0 <= m <= l, |n| <= 1000
 *   amp      device [K][M][2] float64, knot-major: amp[(i*M + k)*2 + 0/1] is
 *            Re/Im A of mode k at knot i (the amplitude module's 2-D layout, Sec. III B)
 * Enqueued on the plan stream; *out is a library-owned handle.
 */
int32_t few_spline_fit(few_plan plan, int32_t K, const double *t_knots,
                       const double *phi_phi, const double *phi_r,
                       int32_t M, const int32_t *lmn, const double *amp,
                       few_spline *out);

/*
 * Generic-Kerr spherical-projected sum (Sec. VII, spherical projection of the
 * spheroidal harmonics): modes (l, m, k, n) with phase
 * m Phi_phi + k Phi_theta + n Phi_r, and the amplitude symmetry of Eq. (9)
 * with general k, A_{l,-m,-k,-n} = (-1)^{l+k} conj(A_lmkn).  Same as
 * few_spline_fit plus:
 *   phi_theta  device [K]    polar orbital phase at the knots
 *   lmkn       host [M][4]   (l, m, k, n); 2 <= l <= 30, 0 <= m <= l,
 *                            |k| <= 30, |n| <= 1000 (FEW_E_MODES otherwise);
 *                            m = 0 modes are not mirrored
 * The resulting spline is summed by few_mode_sum like any other.  The batched
 * and served entry points take (l, m, n) requests only.
 */
int32_t few_spline_fit_kerr(few_plan plan, int32_t K, const double *t_knots,
                            const double *phi_phi, const double *phi_theta,
                            const double *phi_r, int32_t M, const int32_t *lmkn,
                            const double *amp, few_spline *out);

/* Release a spline's arena memory.  Safe while work using the spline is still
 * queued on the plan stream: the block returns to the arena only once the work
 * enqueued there before this call has completed (an event recorded now), so
 * neither synchronous calls nor served batches on the library's own streams
 * receive it earlier. */
int32_t few_spline_free(few_spline spline);

/*
 * Copy a fitted spline's coefficients into device memory `dst` (plan stream):
 *   which = 0: amplitudes, float64 [K-1][M][4][2]: coefficient of x^p (x = t - t_i)
 *              of Re/Im A_k on interval i at dst[((i*M + k)*4 + p)*2 + re/im].
 *   which = 1: phases, float64 [K-1][P][4][2]: coefficient p of Phi_phi (0) /
 *              Phi_r (1) / Phi_theta (2, generic-Kerr splines; P = 3, else 2)
 *              as a double-double (hi, lo); p = 0 holds the knot value reduced
 *              to [-pi, pi) (adding 2 pi k leaves e^{-i psi} unchanged).
 */
int32_t few_spline_coefs(few_spline spline, int32_t which, void *dst);

/*
 * Summation stage (Sec. III C and Eqs. (9)-(10)): evaluate the splines on
 * t_j = t_start + j dt, j < n_samples, combine each listed mode and its
 * mirror with -2Y_lm(theta, phi), sum over modes and write
 *   out[j] = h(t_j) = h_plus - i h_cross
 * as interleaved complex128 (FEW_FP64) or complex64 (FEW_MIXED) device memory.
 * Requires t_0 <= t_start and t_start + (n_samples-1) dt <= t_{K-1}.
 * Enqueued on the plan stream; returns before the kernels finish.
 */
int32_t few_mode_sum(few_plan plan, few_spline spline, double theta, double phi,
                     double scale, double t_start, double dt, int64_t n_samples,
                     void *out);

/*
 * Detector-frame waveform (Sec. II frame conventions): the sum of few_mode_sum
 * viewed from sky position (theta_S, phi_S) for a spin direction
 * (theta_K, phi_K), both in the solar-system-barycentre frame, written in the
 * barycentre polarisation basis.  The source-frame viewing angles are
 * theta = arccos(-R.S), phi = -pi/2 (R, S: unit vectors of the two
 * directions); the pi/2 alignment of the polarisation bases flips the sign of
 * h and the rotation through the polarisation angle psi (tan psi = [cos
 * theta_S sin theta_K cos(phi_S - phi_K) - sin theta_S cos theta_K] /
 * [sin theta_K sin(phi_S - phi_K)]) multiplies it by e^{-2 i psi}:
 *   out[j] = -e^{-2 i psi} h(t_j; theta, phi)
 * The constant factor is applied to the folded coefficients, so this costs the
 * same as few_mode_sum.  R parallel to S leaves psi undefined (factor -1).
 */
int32_t few_mode_sum_ssb(few_plan plan, few_spline spline, double theta_S, double phi_S,
                         double theta_K, double phi_K, double scale, double t_start,
                         double dt, int64_t n_samples, void *out);

/*
 * Fused inner products (Sec. VI): the same summation as few_mode_sum, but
 * instead of writing h it forms, with a unit PSD (by Parseval the one-sided
 * noise-weighted integral over both polarisations equals this time sum),
 *   out2[0] = <d|h> = 2 dt sum_j Re(conj(d_j) h_j)
 *   out2[1] = <h|h> = 2 dt sum_j |h_j|^2
 * d: device [n_samples] complex data in the plan's output type (complex64 for
 * FEW_MIXED, complex128 for FEW_FP64).  out2: device float64 [2].  Products
 * and sums are binary64, added per tile and then in a fixed order, so results
 * are reproducible.  h is never written; the plan keeps one partial-sum
 * buffer (16 B per tile) in its arena.  Enqueued on the plan stream.
 */
int32_t few_inner_product(few_plan plan, few_spline spline, double theta, double phi,
                          double scale, double t_start, double dt, int64_t n_samples,
                          const void *data, double *out2);

/*
 * Allocation-free variant of few_inner_product, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and kernels (the
 * results equal few_inner_product's bit for bit), but the per-tile partial
 * sums go to a static device array of 131072 entries (2 MiB, one per GPU,
 * held until the process ends) instead of a buffer grown in the plan arena,
 * and no events are recorded (timing flags are ignored).  The call makes no
 * hipMalloc, hipFree or other allocating call; the array's device address is
 * looked up once per device by few_plan_create.  Every tile slot the launch
 * uses is written before it is read, so nothing needs clearing between calls.
 *   Limit: the launch's tile slots must fit the array (about 16 million
 *   samples in binary64, 130 million in binary32, at 100 knots); larger
 *   calls return FEW_E_TOO_LARGE before anything is enqueued.
 *   Concurrency: every call on one GPU shares that GPU's array, so calls that
 *   overlap on the device (other plans, streams or threads) race; serialise
 *   them, for example by issuing them on one stream.
 */
int32_t few_inner_product_noalloc(few_plan plan, few_spline spline, double theta, double phi,
                                  double scale, double t_start, double dt, int64_t n_samples,
                                  const void *data, double *out2);

/*
 * Mode selector (Sec. III D): choose the modes that carry all but a fraction
 * eps of the power at some knot.  At every knot k the power of mode j is
 * |A_j(t_k)|^2 = re*re + im*im (binary64, no fused multiply-add); modes are
 * ordered by decreasing power (ties by increasing index), their powers summed
 * sequentially in that order, and the shortest prefix whose sum reaches
 * (1 - eps) of the knot's total is kept (at least the top mode).
 *   K, M   knots and listed modes, K >= 1, 1 <= M <= 4096
 *   amp    device [K][M][2] float64, the same knot-major layout as few_spline_fit
 *   eps    in [0, 1)
 *   keep   device [M] int32: 1 if the mode is kept at any knot (the union), else 0
 * Enqueued on the plan stream.  The result depends only on the inputs (no
 * order of floating-point reduction is left open): every knot is decided
 * either from sums whose error bound keeps each comparison on the same side
 * as that of the sequential sums, or, when a comparison lies within the
 * bound (or FEW_FLAG_SELECT_SORTED is set), from the sequential sums
 * themselves.
 */
int32_t few_mode_select(few_plan plan, int32_t K, int32_t M, const double *amp, double eps,
                        int32_t *keep);

/*
 * Batched path: fit and sum n independent requests (each as few_spline_fit +
 * few_mode_sum, Sec. III C) in one batched launch on the plan stream: one fit
 * kernel, one prepare/fold pair and one persistent summation kernel whose
 * waves pull tiles of every request from a shared counter.  Results are
 * bitwise identical to n separate calls.  Returns before the kernels finish;
 * request inputs and outputs follow the synchronous-call ownership rule.
 */
int32_t few_batch(few_plan plan, int32_t n, const few_request *reqs);

/*
 * Served path: queue one request (spline fit + summation) for continuous
 * batching.  A host scheduler thread admits queued requests in arrival order
 * while their arena footprint fits the plan budget, packs the admitted ones
 * into one batched launch on one of max_inflight library-owned streams, and
 * retires them when that launch completes.  Each result is bitwise identical
 * to the same request run alone.  While launches are in flight the scheduler
 * polls their completion back to back, so it keeps one host core busy; it
 * sleeps when nothing is queued or running.
 * Ordering: few_submit records an event on the plan stream and the request's
 * launch waits for it, so work the caller enqueued on the plan stream before
 * the call (writing phi_phi, phi_r, amp; last reads of out) completes first.
 * Work on other streams must be ordered before the call by the caller.
 * Errors: FEW_E_TOO_LARGE at submit if the request can never fit the budget;
 * few_poll returns FEW_E_NOMEM if, with none of the plan's served work in
 * flight, the arena still cannot hold the request because synchronous-path
 * splines or buffers occupy it.
 */
int32_t few_submit(few_plan plan, const few_request *req, uint64_t *ticket);

/* FEW_PENDING while queued or running; FEW_OK once `out` holds the result
 * (the ticket is then retired); or the request's asynchronous error. */
int32_t few_poll(few_plan plan, uint64_t ticket);

/* Block until the ticket is no longer pending; returns what few_poll would. */
int32_t few_wait(few_plan plan, uint64_t ticket);

/*
 * Request log of the server (few_submit): with a path, the scheduler appends
 * one JSON line per request when it retires -- ticket, status, knots, modes,
 * samples, path ("mfma", "vector" or "fp64"), batch number and size, and the
 * times in microseconds since plan creation (host steady clock) at which it
 * arrived (few_submit), was admitted into a batch and was seen complete
 * (admit_us is -1 for a request that was never admitted).  The file is
 * opened for appending and flushed after every retired batch; NULL closes
 * it.  Returns FEW_E_ARG if the file cannot be opened.
 */
int32_t few_plan_log(few_plan plan, const char *path);

/* Kernel times recorded so far (FEW_FLAG_TIMING), after synchronising the
 * plan stream; reset != 0 clears the counters (and restarts the count of
 * FEW_FLAG_TIMING_SPARSE, so the next summation launch is timed). */
int32_t few_plan_timing(few_plan plan, few_timing *out, int32_t reset);

/* The calling thread's last error message ("" if none). */
const char *few_last_error(void);

/* ---- Host-side helpers (no device work; usable without a GPU) ---------- */

/*
 * Term layout used by the summation kernel.  For fixed theta and phi the l-sum
 * of Eq. (10) folds into one complex cubic per signed (m, n):
 *   C_{m,n}  = sum_l -2Y_lm A_lmn                  (listed modes, m >= 0)
 *   C_{-m,-n} = sum_l (-1)^l -2Y_{l,-m} conj(A_lmn)  (mirrors, m > 0)
 * so h = sum_{m,n} C_{m,n}(t) e^{-i(m Phi_phi + n Phi_r)}.  Terms are grouped
 * into segments of one signed m and a contiguous n range (gaps of at most
 * `max_gap` zero terms are filled).  Writes up to cap_* entries:
 *   segs[4*s + 0..3] = (m, n_lo, length, first term index)
 *   term_ptr[n_terms + 1], term_src[2*e + 0/1] = (mode index,
 *     l | m << 8 | mirror << 16 | 64 << 17)
 * and the counts.  Returns FEW_E_ARG if a capacity is too small.
 */
int32_t few_host_terms(int32_t M, const int32_t *lmn, int32_t max_gap,
                       int32_t cap_segs, int32_t *segs, int32_t *n_segs,
                       int32_t cap_terms, int32_t *term_ptr, int32_t *n_terms,
                       int32_t cap_src, int32_t *term_src, int32_t *n_src);

/*
 * The same for generic-Kerr modes lmkn [M][4] = (l, m, k, n): one complex cubic
 * per signed (m, k, n), mirrors weighted by (-1)^{l+k} -2Y_{l,-m}; segments of
 * one signed (m, k) with contiguous n, in (m, k, n) order;
 *   segs[4*s + 0] = m + 256 k
 *   term_src[2*e + 1] = l | m << 8 | mirror << 16 | (k + 64) << 17
 * (few_host_terms writes the same fields with k = 0).
 */
int32_t few_host_terms_kerr(int32_t M, const int32_t *lmkn, int32_t max_gap,
                            int32_t cap_segs, int32_t *segs, int32_t *n_segs,
                            int32_t cap_terms, int32_t *term_ptr, int32_t *n_terms,
                            int32_t cap_src, int32_t *term_src, int32_t *n_src);

/*
 * First sample of each knot interval: starts[i] = min{ j in [0, n] :
 * t_start + j dt >= t_knots[i] } for 1 <= i <= K-2 (binary64 sample times),
 * starts[0] = 0 and starts[K-1] = n.  The device computes the same starts.
 */
int32_t few_host_interval_starts(int32_t K, const double *t_knots, double t_start,
                                 double dt, int64_t n, int64_t *starts);

/* Detector-frame quantities of few_mode_sum_ssb: out4 = (theta, phi, Re, Im)
 * of the source viewing angles and the factor -e^{-2 i psi}.  FEW_E_ARG for
 * non-finite angles. */
int32_t few_host_frame(double theta_S, double phi_S, double theta_K, double phi_K,
                       double *out4);

/* Arena bytes a served request of this shape reserves (precision of the plan
 * descriptor `precision`), or 0 for invalid shapes. */
uint64_t few_host_request_bytes(int32_t precision, int32_t K, int32_t M,
                                int32_t n_terms);

/*
 * Matrix-core summation of FEW_MIXED plans (a contraction of the folded
 * coefficients of Eq. (10) with powers of e^{-i Phi_r}, Sec. III C, on fp16
 * hi/lo operands with fp32 accumulation).  few_host_mfma_path returns 1 if a
 * binary32 request with this (l, m, n) mode list is summed on the matrix
 * cores (unless the plan sets FEW_FLAG_VECTOR_ONLY), 0 if on the vector
 * units, or a negative few_status for an invalid list.  few_host_mfma_shape
 * writes the launch shape: out8 = (waves per workgroup, 16-sample tiles per
 * wave, 16-row tiles, 32-column steps per sign of n, MFMA instructions per
 * tile and round, largest |n| + 1, largest number of signed m values,
 * smallest number of folded terms).  Each workgroup (one per compute unit)
 * takes a contiguous share of the samples; the shares of the GPU's eight XCDs
 * are weighted by the rule of few_host_xcd_split_step.
 */
int32_t few_host_mfma_path(int32_t M, const int32_t *lmn);
void few_host_mfma_shape(int32_t *out8);

/*
 * The XCD split of the matrix-core summation (a performance rule; results do
 * not depend on it): from the weights w_prev[8] a launch gave the samples of
 * XCD x (workgroup b runs on XCD b mod 8; the weights have mean 1) and the
 * time its slowest workgroup on each XCD took, times[8], the plan's next
 * launch uses w_next[x] = w_prev[x] (1 + (T / times[x] - 1) / 2), T the mean
 * of the times, renormalised to mean 1 and clamped to [1/2, 2]: half a step
 * towards equal finishing times.  FEW_E_ARG for a null pointer or a time or
 * weight that is not finite and > 0.
 */
int32_t few_host_xcd_split_step(const double *w_prev, const double *times, double *w_next);

#ifdef __cplusplus
}
#endif

#endif /* FEW_H */
