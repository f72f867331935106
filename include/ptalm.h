/*
 * ptalm.h -- C ABI of the MI355X (gfx950) library for the direct
 * point-to-harmonic transform of Baleato Lizancos & White, "Harmonic analysis of
 * discrete tracers of large-scale structure" (arXiv:2312.12285).
 *
 * Conventions shared by every entry point
 *  - a_lm arrays hold 2*T doubles, (re, im) interleaved, in healpy order:
 *      index(l, m) = m*(2*lmax+1-m)/2 + l,  0 <= m <= l <= lmax,
 *      T = (lmax+1)(lmax+2)/2.
 *    Only m >= 0 is stored; a_{l,-m} = (-1)^m conj(a_lm) for real weights
 *    (Sec. 2.2, the symmetry stated after eq. alm_def).
 *  - Y_lm is orthonormal on the unit sphere with the Condon-Shortley phase
 *    (Sec. 2.2 normalisation N_lm; App. A.1 sectoral recurrence sign).
 *  - Buffers are DEVICE pointers on the current HIP device unless a comment
 *    says otherwise.  The caller owns every buffer it passes; the library keeps
 *    no pointer after the work it enqueued has finished.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls are
 *    asynchronous: outputs are valid once the stream has reached the call's
 *    work.  Outputs are overwritten, never accumulated into.
 *  - Errors: arguments are validated synchronously before anything is
 *    enqueued; on PTALM_EINVAL no output is touched.  PTALM_EDEVICE reports a
 *    HIP error (a launch failure, or an error left by earlier work that
 *    surfaced here).  ptalm_last_error() returns a message for the calling
 *    thread.  No C++ exception crosses this boundary.
 *  - Thread safety: concurrent calls from different host threads on different
 *    streams are safe (each call allocates its own scratch, stream-ordered).
 *  - Results are deterministic: for a given (n, lmax, options, device) every
 *    reduction is done in a fixed order, so repeated calls are bitwise equal.
 */
#ifndef PTALM_H
#define PTALM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PTALM_OK = 0,
    PTALM_EINVAL = -1,   /* bad argument; nothing enqueued, outputs untouched   */
    PTALM_ENOMEM = -2,   /* device allocation of scratch or tables failed        */
    PTALM_EDEVICE = -3,  /* HIP runtime error                                    */
    PTALM_EBUSY = -4,    /* not now: server budget full, or tables not prepared under capture */
    PTALM_ENOTSUP = -5   /* option combination not implemented                   */
} ptalm_status;

/* Largest lmax accepted; keeps T < 2^31 and every index in 32 bits. */
#define PTALM_LMAX_MAX 16383

/* T = (lmax+1)(lmax+2)/2 for 0 <= lmax <= PTALM_LMAX_MAX, else 0. Host only. */
int64_t ptalm_alm_size(int lmax);

/* healpy index of (l, m), or -1 unless 0 <= m <= l <= lmax <= PTALM_LMAX_MAX. Host only. */
int64_t ptalm_alm_index(int lmax, int l, int m);

/*
 * a_lm = sum_{i<n} w_i Y*_lm(theta_i, phi_i) for 0 <= m <= l <= lmax
 * (eq. alm_def, Sec. 2.2), in FP64.
 *   theta, phi, w : n doubles each (structure of arrays).  theta in [0, pi] is
 *                   a precondition (not checked per element); phi any finite
 *                   value; weights any finite values, negative allowed.
 *   alm           : 2*T doubles, output.
 * n = 0 writes an all-zero a_lm.  Terms whose |Pbar_l^m| stays below about
 * 2^-1000 (points near the poles at large m) contribute nothing; such terms
 * cannot change an FP64 result.
 * PTALM_EINVAL: n < 0, lmax out of range, a NULL pointer with n > 0, alm NULL.
 */
int ptalm_alm_from_points(const double *theta, const double *phi, const double *w,
                          int64_t n, int lmax, double *alm, void *stream);

/* Arithmetic of the transform. */
typedef enum {
    PTALM_FP64 = 0,   /* recurrence, products and sums in FP64                                  */
    PTALM_MIXED = 1,  /* FP64 recurrence; FP32 products, per-lane sums and cross-lane reduction;
                         FP64 trig, seed exponent, phase and block partials                     */
    PTALM_FP32 = 2,   /* FP32 recurrence and products; FP64 trig, seed exponent, phase and block
                         partials.  An FP32 recurrence carries x = cos(theta) to 2^-24, which
                         costs ~l * 2^-24 relative per value at degree l                        */
    PTALM_BF16X3 = 3  /* multi-weight only (n_weights 16 or 32): FP64 recurrence; the sum over
                         points as a matrix product on the matrix cores with bf16 hi+lo split
                         operands, three products (hi.hi + hi.lo + lo.hi), FP32 accumulation,
                         FP64 final sum: ~1e-5 relative per product                             */
} ptalm_precision;

/* Options of ptalm_alm_from_points_ex.  Zero-initialise, then set fields;
 * 0 in a tile field means "use the tuned/default value". */
typedef struct ptalm_opts {
    int precision;     /* ptalm_precision                                          */
    int n_weights;     /* >= 1: w holds n_weights rows of n (row-major); alm holds
                          n_weights blocks of 2*T doubles.  Positions are shared. */
    int points_per_lane;  /* kernel variant: points held per lane (0 = tuned)     */
    int l_block;          /* kernel variant: l values per register block (0 = tuned) */
    int n_slices;      /* point slices = partial results reduced in the second pass (0 = auto) */
    int m_ranges;      /* contiguous m ranges, one work item per (slice, range) (0 = auto)    */
    int reduction;     /* cross-lane reduction variant: 0 = tuned default, else
                          1 + (register butterfly stage ? 1 : 0) + (pipelined ? 2 : 0)     */
    int timing;        /* != 0: record HIP events around the transform kernel(s) on `stream`;
                          read them with ptalm_last_timing()                               */
} ptalm_opts;

/*
 * Extended transform: precision and multi-weight batches (several weight
 * vectors sharing one position set).  With workspace != NULL the call uses
 * that buffer for its scratch (device memory of the calling device from
 * hipMalloc or hipMallocAsync, 256-byte aligned, ws_bytes >=
 * ptalm_workspace_bytes(...); the split-bf16 form adds into it with device
 * float atomics, which host-coherent memory need not support) and allocates
 * nothing, which allows capture into a HIP graph; with NULL it allocates
 * stream-ordered scratch itself.
 * PTALM_EINVAL as above, or opts fields out of range, or a workspace that is
 * too small or misaligned.
 * PTALM_ENOTSUP if the (precision, n_weights, tile) combination has no kernel.
 */
int ptalm_alm_from_points_ex(const double *theta, const double *phi, const double *w,
                             int64_t n, int lmax, double *alm, const ptalm_opts *opts,
                             void *workspace, size_t ws_bytes, void *stream);

/* Scratch bytes ptalm_alm_from_points_ex needs for these arguments (0 on bad
 * arguments). Host only. */
size_t ptalm_workspace_bytes(int64_t n, int lmax, const ptalm_opts *opts);

/*
 * Pseudo-spectrum C_l = (2l+1)^-1 sum_{m=-l..l} |a_lm|^2 (eq. pseudoCl), the m<0
 * half by the symmetry a_{l,-m} = (-1)^m conj(a_lm).
 *   alm : 2*T doubles (input);  cl : lmax+1 doubles (output).
 * PTALM_EINVAL as above, or cl overlapping alm.
 */
int ptalm_cl_from_alm(const double *alm, int lmax, double *cl, void *stream);

/*
 * Cross spectrum C^AB_l = (2l+1)^-1 sum_{m=-l..l} Re(a_lm conj(b_lm)), the
 * generalisation of eq. pseudoCl to two fields (Sec. 1, Sec. 4).
 *   alm1, alm2 : 2*T doubles each (alm1 == alm2 gives the auto-spectrum);
 *   cl : lmax+1 doubles.  PTALM_EINVAL as above, or cl overlapping an input.
 */
int ptalm_cross_cl(const double *alm1, const double *alm2, int lmax, double *cl, void *stream);

/* y <- y + alpha * x over 2*T doubles (x, y device; alpha host).  x == y is allowed;
 * PTALM_EINVAL for other overlaps of x and y. */
int ptalm_alm_axpy(double alpha, const double *x, double *y, int lmax, void *stream);

/*
 * FKP field of Sec. 2.3: alpha = a_00(data) / a_00(randoms), which normalises
 * the randoms so that alpha*a_00(randoms) = a_00(data), then
 *   delta  = a(data) - alpha * a(randoms)     (the transform of n_g - alpha n_r, Sec. 1)
 *   window = alpha * a(randoms)               (w_lm of eq. wldef; C_l of it is W_l)
 * alpha is written to the device double *alpha_out (may be NULL).  No host
 * synchronisation.  delta or window may be NULL to skip that output.  Outputs
 * must not overlap the inputs (PTALM_EINVAL if a pointer is equal to one).
 * Randoms whose weights sum to zero give a non-finite alpha.
 */
int ptalm_fkp_fields(const double *alm_data, const double *alm_randoms, int lmax,
                     double *delta, double *window, double *alpha_out, void *stream);

/* ------------------------------------------------------------------------
 * Mode coupling and bandpowers (Sec. 2.1 eq. chat, eq. mode_coupling,
 * eq. expectation_value; 3j symbols of App. B).  Device pointers, async on
 * `stream`.
 * ------------------------------------------------------------------------ */

/* Shot noise of a weighted point set: out[0] = a^2 sum_i w_i^2 / (4 pi) with
 * a = alpha[0] (device) or 1 if alpha is NULL; for the window of scaled
 * randoms (the footnote to eq. wldef).  Fixed summation order (per-block
 * partial sums, then their sum in block order).  Allocates stream-ordered
 * scratch. */
int ptalm_window_shot_noise(const double *w, int64_t n, const double *alpha, double *out, void *stream);

/* Mode-coupling matrix
 *   M[l][l'] = (2l'+1)/(4 pi) sum_lambda (2 lambda+1) (l l' lambda; 0 0 0)^2 W_lambda   (eq. chat)
 *   Wl    : lmax_w+1 doubles, the window spectrum W_lambda (eq. wldef; lambda > lmax_w
 *           counts as 0; W up to 2 lmax gives the complete matrix);
 *   shot  : NULL, or one device double subtracted from every W_lambda first;
 *   M     : (lmax+1)^2 doubles, row-major in l (output).
 * FP64.  With J = (l + l' + lambda)/2 and a(n) = binom(2n, n)/4^n the 3j square
 * is a(J-l) a(J-l') a(J-lambda) / ((2J+1) a(J)); the matrix is computed as a
 * triangular matrix product on the matrix cores from tables of a(n) (the same
 * values the App. B recurrence gives).  Allocates stream-ordered scratch.  The
 * tables that depend on lmax only (a(n) and 1/((2J+1) a(J)), about 3 lmax
 * doubles) are kept per (device, lmax) for the rest of the process: the first
 * call for an lmax outside stream capture allocates them and waits for them once
 * (a synchronisation of `stream`); under capture an lmax not seen before
 * computes them into the call's scratch instead, so the call stays capturable.
 * PTALM_EINVAL on bad sizes or NULL pointers. */
int ptalm_coupling_matrix(const double *Wl, int lmax_w, const double *shot, int lmax, double *M, void *stream);

/* Number of complete bins [lmin + b delta_l, lmin + (b+1) delta_l) within lmax (0 if none). Host only. */
int ptalm_bandpower_count(int lmax, int lmin, int delta_l);

/* Bandpowers of a pseudo-spectrum cl_hat[0..lmax] with theta_b^l = 1/delta_l on
 * those bins (Sec. 2.1):
 *   mode 0, mode-decoupled (eq. mode_coupling): cb = Mbb^-1 theta cl_hat with
 *     Mbb[b][b'] = sum_{l in b} sum_{l' in b'} theta_b^l M[l][l'], and
 *     window = Mbb^-1 theta M (eq. expectation_value), by LU factorisation of
 *     Mbb with partial pivoting and forward/back substitution in FP64 (a
 *     singular Mbb, from bins too narrow for the mask, gives non-finite output);
 *   mode 1, normalised: cb = N theta cl_hat, window = N theta M with
 *     1/N = sum_l (2l+1) W_l / (4 pi) (needs Wl, lmax_w).
 * cb: nb doubles, window: nb x (lmax+1) doubles row-major (may be NULL).
 * Allocates stream-ordered scratch.  PTALM_EINVAL: no complete bin, more than
 * 1024 bins, bad mode, NULL inputs. */
int ptalm_bandpowers(const double *cl_hat, const double *M, const double *Wl, int lmax_w, int lmax, int lmin,
                     int delta_l, int mode, double *cb, double *window, void *stream);

/* ------------------------------------------------------------------------
 * Interpolated transform (App. A.2): cubic Hermite splines of y_lm(x) and
 * y'_lm(x) on a node grid instead of the per-point recurrence.
 * ------------------------------------------------------------------------ */

#define PTALM_SPLINE_NODES_MAX 65536
/* Largest point count of the interpolated transform: points are counted per interval
 * in 32-bit counters. */
#define PTALM_SPLINE_N_MAX 4294967295LL

/* a_lm ~= sum_i w_i Y*_lm(theta_i, phi_i) by the interpolated transform of
 * App. A.2, same arguments and output layout as ptalm_alm_from_points:
 *   n_nodes   : spline nodes, uniform in theta over [theta_cut, pi - theta_cut]
 *               (x_j = cos(pi - theta_cut - j h), ascending in x);
 *   theta_cut : points with theta < theta_cut or theta > pi - theta_cut (the
 *               polar caps) take the exact sum instead of the spline; in (0, pi/2).
 * Per interval [x_j, x_{j+1}) and order m the points are summed into the
 * binned weights v_ja^(m) = sum w e^{-i m phi} c_a(t) (the Hermite basis of
 * App. A.2, with the (x_{j+1} - x_j) factors on the derivative terms), and
 * a_lm = sum_j [v_j0 y(x_j) + v_j1 dx_j y'(x_j) + v_j2 y(x_{j+1}) + v_j3 dx_j y'(x_{j+1})]
 * with y' from the derivative relation of App. A.1.  Approximate: the error
 * falls like (l h)^4 with the node spacing h in theta.  FP64 throughout.
 * The points are put in interval order by a stable counting sort (inside an
 * interval they keep their input order), so repeated calls give the same bits.
 * Scratch: ptalm_spline_workspace_bytes(n, lmax, n_nodes) bytes (about 88 B per
 * point, plus (lmax+1) x n_nodes x 112 B, plus about 270 B per (l, m)); with
 * workspace != NULL (device, 256-byte aligned, ws_bytes at least that) the call
 * uses it and allocates nothing, else it allocates stream-ordered scratch.  The
 * call never synchronizes: the number of polar points stays on the device.  It
 * can be captured into a HIP graph when given a workspace after
 * ptalm_prepare_spline_call(n, lmax, n_nodes) (else PTALM_EINVAL without a
 * workspace, PTALM_EBUSY when not prepared).  opts: NULL, or opts->timing != 0
 * to record HIP events around the binning kernel (the dominant one) on
 * `stream`, read with ptalm_last_timing() (not under capture); the other fields
 * are not used.  PTALM_EINVAL on bad sizes or pointers, a small or misaligned
 * workspace, or n > PTALM_SPLINE_N_MAX. */
int ptalm_alm_from_points_spline(const double *theta, const double *phi, const double *w, int64_t n, int lmax,
                                 int n_nodes, double theta_cut, double *alm, const ptalm_opts *opts,
                                 void *workspace, size_t ws_bytes, void *stream);

/* Scratch bytes of ptalm_alm_from_points_spline for these sizes (0 on bad
 * arguments).  Host only. */
size_t ptalm_spline_workspace_bytes(int64_t n, int lmax, int n_nodes);

/* Builds, on the current device, the tables a later
 * ptalm_alm_from_points_spline(n, lmax, n_nodes, ...) call needs (direct-sum
 * coefficient tables for the polar caps, the m-range tables of the node sum
 * and of the polar sum), so that the call can be captured.  Host only. */
int ptalm_prepare_spline_call(int64_t n, int lmax, int n_nodes);

/*
 * Spin-weighted transform for shear (spin +-2 harmonics in place of Y_lm, the
 * generalisation the paper notes at the end of Sec. 4).  For a catalog with
 * weights w and shear components (g1, g2) it forms
 *     _{+2}a_lm = sum_i w_i (g1_i + i g2_i) _{+2}Y*_lm(theta_i, phi_i),
 *     _{-2}a_lm = sum_i w_i (g1_i - i g2_i) _{-2}Y*_lm(theta_i, phi_i),
 * and writes the E and B modes
 *     alm_E = -(_{+2}a + _{-2}a) / 2,   alm_B = i (_{+2}a - _{-2}a) / 2
 * with _sY_lm(theta, phi) = (-1)^m sqrt((2l+1)/4pi) d^l_{m,-s}(theta) e^{i m phi}
 * (Wigner d; the convention of Goldberg et al. 1967 and healpy's E/B signs).
 * theta, phi, w, g1, g2: device, n doubles each (structure of arrays).
 * alm_E, alm_B: device, 2*T doubles each, healpy order (complex interleaved),
 * written completely (0 for l < 2).  FP64 throughout.
 * opts: NULL for defaults; honours points_per_lane, l_block (a compiled
 * spin variant), n_slices, m_ranges, timing (ptalm_last_timing then reads
 * the spin kernel's device time) and reduction (0: the default form, 1: both
 * spins in one wavefront, 4 reals reduced per l; 2: one spin per wavefront,
 * 2 reals per l, twice the wavefronts; else PTALM_EINVAL); precision must be
 * PTALM_FP64 and n_weights 0 or 1 (else PTALM_ENOTSUP).  Allocates and frees stream-ordered scratch of
 * ptalm_shear_workspace_bytes(n, lmax, opts) bytes; builds the spin tables for
 * lmax on first use (synchronously).  Deterministic: the same inputs give the
 * same bits.  PTALM_EINVAL on bad sizes or pointers.
 */
int ptalm_shear_alm_from_points(const double *theta, const double *phi, const double *w, const double *g1,
                                const double *g2, int64_t n, int lmax, double *alm_E, double *alm_B,
                                const ptalm_opts *opts, void *stream);

/* Scratch bytes of ptalm_shear_alm_from_points for these arguments (0 on bad
 * arguments).  Host only. */
size_t ptalm_shear_workspace_bytes(int64_t n, int lmax, const ptalm_opts *opts);

/* Device time of the transform kernel(s) of the last ptalm_alm_from_points_ex
 * or ptalm_shear_alm_from_points call made on this thread with opts->timing
 * set: from just before the first transform kernel to just after the last
 * one, on that call's stream (for ptalm_alm_from_points_spline: its binning
 * kernel).  Blocks
 * until that work has finished.  PTALM_EINVAL if no timed call was made.
 * Host only. */
int ptalm_last_timing(double *transform_ms);

/* Builds, on the current device, the coefficient tables the transform uses for
 * this lmax (normally built on first use, synchronously).  Lets a caller keep
 * that one-off cost out of a timed region or a latency-sensitive loop.  Also the
 * set-up of ptalm_alm_from_points_noalloc for this lmax (its m-range table and
 * the address of its static scratch on this device). */
int ptalm_prepare(int lmax);

/*
 * No-allocation form of ptalm_alm_from_points, for callers that cannot
 * allocate device memory at call time: code being captured into a HIP graph,
 * tight serving loops, hosts that forbid allocation after set-up.  Same
 * arguments, result and FP64 arithmetic as ptalm_alm_from_points (eq. alm_def);
 * the per-slice partial sums go to a static device array of
 * PTALM_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends, so the call allocates nothing and synchronizes
 * nothing.  Set-up: ptalm_prepare(lmax) must have been called on the current
 * device for this lmax (it builds the tables and looks up the array's address);
 * otherwise PTALM_EBUSY.  Limits: lmax <= PTALM_NOALLOC_LMAX_MAX (one slice of
 * partials, 16*T bytes, must fit the array), else PTALM_EINVAL.  Every call on
 * one device shares that device's array: calls that overlap in time on one
 * device (different streams without ordering between them) race and give wrong
 * results; order them on one stream or synchronize in between.
 */
#define PTALM_NOALLOC_SCRATCH_BYTES (128u << 20)
#define PTALM_NOALLOC_LMAX_MAX 4094
int ptalm_alm_from_points_noalloc(const double *theta, const double *phi, const double *w,
                                  int64_t n, int lmax, double *alm, void *stream);

/* Builds everything the call ptalm_alm_from_points_ex(n, lmax, opts, ...)
 * would build on first use (coefficient tables, m-range table), so that the
 * call can afterwards be captured into a HIP graph: under stream capture the
 * transform allocates and synchronizes nothing, needs a caller workspace and
 * returns PTALM_EBUSY if the tables were not prepared.  Host only. */
int ptalm_prepare_call(int64_t n, int lmax, const ptalm_opts *opts);

/* Autotuner.  Times, on `stream` with HIP events, one call of every compiled
 * kernel variant of `precision` (points per lane x l-block x reduction for the
 * vector forms; point slices for PTALM_BF16X3) on the given points (device
 * pointers as in ptalm_alm_from_points_ex; a few 1e5 points are a good
 * sample), and writes the fastest options to *best.  The choice is also kept
 * per (device, precision, n_weights, lmax) and used for every option left at
 * 0 in later calls.  Synchronizes `stream`; allocates and frees stream-ordered
 * scratch.  PTALM_EINVAL on bad arguments or under stream capture. */
int ptalm_autotune(const double *theta, const double *phi, const double *w, int64_t n, int lmax,
                   int precision, int n_weights, ptalm_opts *best, void *stream);

/* ------------------------------------------------------------------------
 * Request server: continuous batching of transforms on one device (host API).
 *
 * A server owns an arena of device memory (the scratch budget) and `slots`
 * HIP streams.  A scheduler thread admits submitted requests into the arena
 * (their scratch footprint, ptalm_workspace_bytes of their call) in arrival
 * order, letting later requests that fit pass one that does not until it has
 * waited 30 s.  Each admitted request runs as work items: launches of its
 * transform over consecutive groups of its point slices (about 2e11 terms
 * each), then one finishing launch (the second pass and the spectrum).  Items
 * go to free slots, the request with the least remaining work first, so small
 * requests do not wait behind large ones; requests waiting longer than 30 s
 * go before all others (oldest first), so none starves under overload; items
 * of different requests run concurrently on the device.  Each request uses the work plan of the same call made alone and
 * its chunks compute exactly that call's slice partials, so its a_lm are
 * bitwise those of the solo call.
 * The catalog and output buffers are device memory owned by the caller: the
 * inputs must be complete before ptalm_server_submit and stay valid, and the
 * outputs untouched, until the request completes.
 * ------------------------------------------------------------------------ */
typedef struct ptalm_server ptalm_server;

typedef struct ptalm_request {
    const double *theta, *phi, *w;   /* device, n doubles each                        */
    int64_t n;
    int lmax;
    int precision;                   /* PTALM_FP64, PTALM_MIXED or PTALM_FP32          */
    double *alm;                     /* device, 2*T doubles: a_lm (output)            */
    double *cl;                      /* device, lmax+1 doubles: C_l (output), or NULL */
} ptalm_request;

typedef struct ptalm_request_stats {
    int status;                /* PTALM_OK or the error of the request                 */
    int slot;                  /* stream slot of its first work item                   */
    size_t footprint_bytes;    /* arena bytes held from admission to completion        */
    double submit_s, admit_s, done_s;   /* steady (CLOCK_MONOTONIC) clock, seconds:
                                           submission, admission, completion seen      */
} ptalm_request_stats;

typedef struct ptalm_server_state {
    size_t arena_bytes, arena_in_use;
    int slots, running;        /* running: requests admitted and not yet complete   */
    int64_t waiting;           /* waiting: submitted requests not yet admitted       */
} ptalm_server_state;

/* Creates a server on `device` with an arena of arena_bytes (allocated now)
 * and 1..64 slots.  PTALM_EINVAL bad arguments; PTALM_ENOMEM arena. */
int ptalm_server_create(int device, size_t arena_bytes, int slots, ptalm_server **out);

/* Queues a request and returns at once with its ticket.  PTALM_EINVAL bad
 * request; PTALM_EBUSY its footprint exceeds the whole arena (never admitted). */
int ptalm_server_submit(ptalm_server *s, const ptalm_request *req, int64_t *ticket);

/* *done = 1 once the request has completed; then *stats is filled, the ticket
 * is retired and the request's status is returned. */
int ptalm_server_poll(ptalm_server *s, int64_t ticket, int *done, ptalm_request_stats *stats);

/* Blocks until the request completes; fills *stats (may be NULL), retires the
 * ticket and returns the request's status.  One wait or final poll per ticket. */
int ptalm_server_wait(ptalm_server *s, int64_t ticket, ptalm_request_stats *stats);

/* Arena use, running and waiting requests right now. */
int ptalm_server_query(ptalm_server *s, ptalm_server_state *state);

/* Completes every queued and running request, then frees the server. */
int ptalm_server_destroy(ptalm_server *s);

/* Message of the last failed server call (or failed request) on this thread. */
const char *ptalm_server_last_error(void);

/* Message of the last failed call on this thread ("" if none). Host only. */
const char *ptalm_last_error(void);

/* Frees the per-device tables cached by earlier calls (coefficients per lmax,
 * the lmax-only tables of the mode coupling) and forgets the autotuner's
 * choices.  PTALM_EDEVICE with the first failed free's message, else PTALM_OK.
 * Call only when no work of this library is pending on the current device. */
int ptalm_release_cache(void);

#ifdef __cplusplus
}
#endif
#endif /* PTALM_H */
