/*
 * qc.h - C-ABI of libqc, an MI355X (gfx950) implementation of the
 * per-solution-interval Jones-chain gain solver of Kenyon et al.,
 * "Africanus II. QuartiCal: calibrating radio interferometer data at scale
 * using Numba and Dask" (arXiv 2412.10072).
 *
 * The method (Section 2 and Algorithm 1 of the paper): for every solution
 * interval of one chain term, form the corrupted model
 *     V_pq = sum_d C_{p,d} M_{pq,d} C_{q,d}^H            (eq. baselinemodel)
 * with C a product of 2x2 Jones terms (eq. joneschain), the residual
 * r = d - v (eq. baselineresidual), reduce the per-antenna "AllJones" blocks
 * J^H W J and J^H W r over every row and channel of the interval
 * (eq. jhj_entry_simplified, eq. jhr_entry_simplified; eq. jhj_case2 /
 * eq. jhwr_case2 for delay terms), solve the small per-antenna systems and
 * update the gains (eq. update), and iterate to convergence.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array pointer is a DEVICE pointer owned by the caller.  The library
 *   never frees or retains it beyond the enqueued work.
 * - 2x2 matrices are stored row-major as 4 correlations XX, XY, YX, YY
 *   (eq. gvec, eq. jones).  complex64 = 2 x float (re, im), complex128 =
 *   2 x double.
 * - Rows are ordered by time (row_time non-decreasing); every term's t_map
 *   and f_map are non-decreasing, so each solution interval is a contiguous
 *   block of rows x a contiguous block of channels.  Violations are reported
 *   as QC_E_ARG / QC_E_RANGE before any solve work is enqueued.
 * - Errors: no exception crosses the ABI.  A non-OK status leaves a message
 *   in qc_last_error(ctx).  Non-convergence is not an error (stats.converged
 *   = 0); a singular or empty per-antenna block is not an error (its
 *   gain_flags entry is set to 1 and its update is zero).  A non-finite value
 *   in an unflagged sample is latched on the device and returned by
 *   qc_ctx_sync as QC_E_NONFINITE.
 * - Work is enqueued on `stream` (NULL = the null stream).  The argument
 *   checks that need device data (row_time order, antenna and map ranges)
 *   run first on the same stream and are waited for, so a call that returns
 *   QC_OK has passed them.  The solve itself is asynchronous.
 */
#ifndef QC_H
#define QC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qc_status;
#define QC_OK           0
#define QC_E_ARG       -1   /* bad argument (null pointer, bad enum, bad size, unsorted rows) */
#define QC_E_RANGE     -2   /* antenna / time / map index out of range                        */
#define QC_E_NONFINITE -3   /* non-finite value in an unflagged sample (latched)              */
#define QC_E_DEVICE    -4   /* HIP runtime error                                              */
#define QC_E_NOMEM     -5   /* device allocation failed                                       */
#define QC_E_UNSUPPORTED -6 /* valid input outside what the library implements (message says) */

#define QC_MAX_TERMS 8      /* chain length limit                                   */
#define QC_MAX_DIR   8      /* model directions limit                               */
#define QC_MAX_GDIR  4      /* gain directions of one term                          */
#define QC_MAX_ANT   256    /* antennas                                             */

typedef enum { QC_C64 = 0, QC_C128 = 1 } qc_dtype;          /* storage of data/model */
typedef enum { QC_PREC_FP64 = 0, QC_PREC_MIXED = 1 } qc_prec;
/* QC_PREC_FP64 : every product, sum and solve in FP64 (complex64 inputs are
 *                upcast exactly).
 * QC_PREC_MIXED: complex64 products and residuals, FP32 accumulation with
 *                compensated (Kahan) sums of the per-antenna blocks, FP64
 *                block solve, update and convergence test.  Needs QC_C64.   */

typedef enum {
  QC_TERM_DIAGONAL = 0, QC_TERM_COMPLEX2X2 = 1, QC_TERM_DELAY = 2, QC_TERM_PHASE = 3, QC_TERM_AMPLITUDE = 4,
  QC_TERM_DELAY_OFFSET = 5, QC_TERM_POINTING = 6
} qc_term_type;
/* DIAGONAL  : unknowns XX, YY of the gain (XY = YX = 0).
 * COMPLEX2X2: all four entries.
 * DELAY     : real parameters tau_X, tau_Y (seconds); the Jones matrix is
 *             diag(exp(2 pi i nu tau_X), exp(2 pi i nu tau_Y)) at channel
 *             frequency nu (the paper's second parameterisation scenario,
 *             eq. jhj_case2, with a delay as the coarse parameter).
 * PHASE     : real parameters phi_X, phi_Y (radians), Jones matrix
 *             diag(exp(i phi_X), exp(i phi_Y)) (phase-only gain; the paper's
 *             first parameterisation scenario, eq. jhj_case1 / jhwr_case1).
 * AMPLITUDE : real parameters a_X, a_Y, Jones matrix diag(a_X, a_Y)
 *             (amplitude-only gain, same scenario).
 * DELAY_OFFSET: real parameters phi0 (radians) and tau (seconds) per hand,
 *             Jones matrix diag(exp(i (phi0_X + 2 pi nu tau_X)),
 *             exp(i (phi0_Y + 2 pi nu tau_Y))) (residual delays with phase
 *             offsets, the K term of the paper's experiments); per hand a real
 *             2x2 block whose pivots are tested against their own diagonal
 *             entries (the two unknowns differ in scale by (2 pi nu)^2).  Not
 *             with QC_DAMP_LM.
 * POINTING  : the paper's third parameterisation scenario (eq. jhj_case3,
 *             eq. jhwr_case3): one real parameter pair per antenna, its
 *             pointing offset (dl, dm) in direction cosines, whose effect
 *             differs by direction: the Jones matrix at model direction d is
 *             b I with the Gaussian beam b = exp(-4 ln 2 ((l_d - dl)^2 +
 *             (m_d - dm)^2) (nu / (beam_fwhm beam_freq))^2), (l_d, m_d) =
 *             dir_lm[d], both hands alike.  n_gdir = 1 and d_map all zero
 *             (the parameter is shared by every direction); one real 2x2
 *             block per (interval, antenna) from the Jacobian summed over
 *             directions.  Solved by a schedule of its own (interval rows cut
 *             into parts, FP64 sums per part, one host wait per iteration);
 *             convergence measures the step in beam widths at the top of the
 *             interval's band, |alpha Delta| nu_max / (beam_fwhm beam_freq).
 *             Not with QC_DAMP_LM or qc_solve_batch; it differs by direction,
 *             so CORRECT and corrected weights refuse a chain holding it.
 * DELAY, PHASE, AMPLITUDE, DELAY_OFFSET and POINTING terms keep their
 * parameters in qc_term.params; the blocks of the first four are real 2x2
 * (one per hand, decoupled) unless the chain left of them needs full blocks
 * (see qc_solve_interval). */

typedef enum { QC_DAMP_FULL = 0, QC_DAMP_HALF = 1, QC_DAMP_ALTERNATE = 2, QC_DAMP_AUTO = 3,
               QC_DAMP_LM = 4 } qc_damping;
/* Step length alpha_k of x <- x + alpha_k * Delta (the paper leaves the step
 * open, noting that Levenberg-Marquardt is a trivial extension):
 * FULL alpha = 1; HALF alpha = 1/2; ALTERNATE alpha = 1 on odd, 1/2 on even
 * updates; AUTO = FULL for delay, phase and delay-offset terms, ALTERNATE for
 * pointing terms, HALF for other direction-dependent terms, ALTERNATE
 * otherwise.
 * LM: Levenberg-Marquardt with the gain-ratio strategy of Madsen et al.
 * (2004): one damping mu per interval (1e-3 of the largest diagonal block
 * entry at first), every block solves (H + mu I) Delta = b and the full step
 * is attempted; the next pass judges it by rho = (chi^2 before - after) /
 * (sum over blocks of Re(Delta^H b) + mu |Delta|^2): rho > 0 accepts it (mu
 * *= max(1/3, 1 - (2 rho - 1)^3)), otherwise the last accepted gains return
 * (mu *= nu, nu doubles, starting at 2) and the blocks are formed again there.
 * Every attempt counts as an iteration and the last one is judged (one more
 * pass), so the result is the last accepted gains unless the interval
 * converged.  On the split schedule the interval's damping state and last
 * accepted gains live in context memory and a rejected attempt costs one more
 * pass; batched solves run it in every problem.                             */

typedef enum { QC_CORRUPT = 0, QC_CORRECT = 1 } qc_apply_mode;

typedef struct qc_ctx qc_ctx;   /* opaque: device, scratch, latched device error */

/* Create a context on HIP device `device`.  One context per host thread. */
qc_status   qc_ctx_create(int32_t device, qc_ctx** out);
/* Destroy a context and free its scratch memory. */
qc_status   qc_ctx_destroy(qc_ctx* ctx);
/* Wait for the last stream used by ctx; returns a latched device error
 * (QC_E_NONFINITE / QC_E_RANGE) and clears it. */
qc_status   qc_ctx_sync(qc_ctx* ctx);
/* Message for the last non-OK status of ctx; valid until the next call. */
const char* qc_last_error(const qc_ctx* ctx);
/* Duration in milliseconds of the timed kernels of the last call through ctx
 * that launched any, measured with HIP events on the launch stream (waits for
 * them): a solve's solve kernel alone; for qc_mad_flag, qc_robust_weights,
 * qc_predict_dft, qc_apply_gains, qc_residual and qc_corrected_weights their
 * kernels after the argument checks.  Negative if none. */
double      qc_last_kernel_ms(qc_ctx* ctx);

/* Launch shape of the per-interval solve used by qc_solve_interval,
 * qc_solve_chain: waves per workgroup (1, 2, 4, 8; 0 = 4) and rows per
 * wavefront step (1, 2, 4; 0 = 4 rows of 16 lanes).
 * Multi-row steps apply to single-term, single-direction chains only.
 * rows_per_step 8 sets the split schedule of one-channel intervals (a
 * bandpass per channel on a diagonal chain) to steps of 8 rows x 8 channels
 * instead of 4 rows x 16 channels, and leaves the other kernels at their
 * default. */
qc_status   qc_ctx_set_tile(qc_ctx* ctx, int32_t waves, int32_t rows_per_step);
/* Schedule of qc_solve_interval: parts = 0 chooses automatically (a term with
 * fewer intervals than four times the compute units, of >= 2^18 samples on
 * average, is split into about 32 workgroups per compute unit; not with a
 * chisq_ref), 1 never splits (one workgroup runs each interval to the end),
 * > 1 cuts every interval's rows into that many parts streamed by separate
 * workgroups whose FP64 blocks are summed in a fixed order before each update
 * (the host then waits on the device once per iteration). */
qc_status   qc_ctx_set_split(qc_ctx* ctx, int32_t parts);
/* Parts per interval of the last qc_solve_interval (1 = not split). */
int32_t     qc_ctx_last_split(const qc_ctx* ctx);

/* One visibility set (paper Section 2.2; data model of Section 4.1). */
typedef struct {
  int64_t n_row;
  int32_t n_chan, n_dir, n_ant, n_time, n_wcorr;  /* n_wcorr in {1, 4}        */
  qc_dtype dtype;
  const void*    data;      /* [n_row][n_chan][4]          complex            */
  const void*    model;     /* [n_row][n_chan][n_dir][4]   complex            */
  const void*    weight;    /* [n_row][n_chan][n_wcorr]    float (C64) / double (C128) */
  const uint8_t* flag;      /* [n_row][n_chan]             nonzero = flagged  */
  const int32_t* ant1;      /* [n_row] p                                      */
  const int32_t* ant2;      /* [n_row] q (rows with p == q are ignored)       */
  const int32_t* row_time;  /* [n_row] time index in [0, n_time), non-decreasing */
  const double*  chan_freq; /* [n_chan] Hz                                    */
} qc_vis;

/* One term of the Jones chain with its own solution intervals (paper
 * Section 4.3: data-to-gain mappings; gain layout of Section 4.4). */
typedef struct {
  qc_term_type type;
  int32_t direction_dependent;  /* informs QC_DAMP_AUTO only; d_map decides the sharing */
  int32_t n_gt, n_gf, n_gdir;
  const int32_t* t_map;     /* [n_time] -> [0, n_gt), non-decreasing          */
  const int32_t* f_map;     /* [n_chan] -> [0, n_gf), non-decreasing          */
  const int32_t* d_map;     /* [n_dir]  -> [0, n_gdir)                        */
  void*   gains;            /* [n_gt][n_gf][n_ant][n_gdir][4] complex128, in/out (DIAGONAL, COMPLEX2X2) */
  double* params;           /* [n_gt][n_gf][n_ant][n_gdir][2] in/out: tau_X, tau_Y in s (DELAY),
                               phi_X, phi_Y in rad (PHASE), a_X, a_Y (AMPLITUDE);
                               [..][4] phi0_X, tau_X, phi0_Y, tau_Y (DELAY_OFFSET);
                               [..][2] dl, dm (POINTING, n_gdir = 1) */
  int8_t* gain_flags;       /* [n_gt][n_gf][n_ant][n_gdir] out (may be NULL for fixed terms) */
  const double* dir_lm;     /* POINTING: [n_dir][2] (l, m) of each model direction (device); else unused */
  double beam_fwhm;         /* POINTING: full width at half maximum of the beam (rad) at beam_freq */
  double beam_freq;         /* POINTING: Hz */
} qc_term;

typedef struct {
  double     tol;           /* stop when the step ratio <= tol (negative: never) */
  int32_t    max_iter;      /* updates per interval; 0 = evaluate chi^2 only     */
  qc_prec    prec;
  qc_damping damping;
  void*      stream;        /* hipStream_t or NULL                               */
  const double* chisq_ref;  /* NULL, or per interval of the active term [n_gt][n_gf]:
                               an interval whose chi^2 at the starting gains exceeds
                               its entry restarts once from unit gains (warm-start
                               fallback; the reference is chi^2 at unit gains) */
} qc_solve_opts;

/* Per interval of the active term, [n_gt][n_gf]; any pointer may be NULL. */
typedef struct {
  int32_t* iters;           /* number of applied updates                         */
  uint8_t* converged;       /* 1 if the step ratio reached tol                    */
  double*  chisq_first;     /* sum w |r|^2 at the initial gains                   */
  double*  chisq_last;      /* sum w |r|^2 at the gains before the last update    */
  uint8_t* restarted;       /* 1 if the chisq_ref fallback restarted the interval */
} qc_solve_stats;

/*
 * Solve term `active` of `chain` (chain order = array order, C = G_0 G_1 ...,
 * eq. joneschain) over all of its solution intervals, each independently
 * (Section 2.3, last paragraph), with the other terms fixed (Section 4.3).
 * Algorithm 1 per interval:
 *   repeat: accumulate JHJ and JHr per (antenna, gain direction) over the
 *   interval's unflagged cross-correlation samples, conjugate baselines
 *   folded in (eq. jhj_entry_simplified, eq. jhr_entry_simplified);
 *   Delta = JHJ^-1 JHr by FP64 Cholesky; x <- x + alpha_k Delta;
 *   stop when ||alpha_k Delta||_2 / ||x||_2 <= tol over the unflagged blocks
 *   (delay: max over blocks of 2 pi nu_max |alpha_k Delta tau| <= tol) or
 *   after max_iter updates.
 * A block whose Cholesky pivot is <= 1e-12 of its largest diagonal entry (or
 * that has no data) gets Delta = 0 and gain_flags = 1.
 * The active term's gains/params are overwritten in place.
 * Any term may sit left of the active one (eq. jonesfactor): the Jacobian
 * block of antenna p is K = sum_d C<_{p,d} (x) (C>_{p,d} M_d C_{q,d}^H)^T over
 * the directions sharing the gain (eq. g_derivative_dd / _di).  When that left
 * product is diagonal and shared by every direction, or every term of the
 * chain is diagonal (diagonal Jones matrices commute), the block splits by gain
 * row (two 2x2 blocks for COMPLEX2X2, decoupled hands otherwise); else the
 * solver forms the full block over all unknowns of the antenna (4x4 Hermitian
 * for COMPLEX2X2, 2x2 for DIAGONAL, real 2x2 for DELAY / PHASE / AMPLITUDE,
 * real 4x4 for DELAY_OFFSET, whose pivots are then each tested against their
 * own diagonal entry), one row per wavefront step.
 */
qc_status qc_solve_interval(qc_ctx* ctx, const qc_vis* vis, qc_term* chain, int32_t n_term,
                            int32_t active, const qc_solve_opts* opts, qc_solve_stats* stats);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as qc_solve_interval, with the same arguments, results and errors,
 * that calls no hipMalloc, hipFree or allocating library routine.  Its device
 * scratch (row positions of every time, the row and channel ranges of the
 * active term's intervals) lives in a fixed array of QC_STATIC_SCRATCH_BYTES
 * per device, held until the process ends; a solve needing more, i.e.
 * 256-byte-aligned blocks of 8 (n_time + 1), 16 n_gt, 8 n_gt and 8 n_gf bytes
 * summing past it, returns QC_E_UNSUPPORTED before any work is enqueued.
 * Always the fused schedule (one workgroup runs each interval to the end,
 * whatever qc_ctx_set_split says), without the fixed-factor table of diagonal
 * chains (those factors are formed per sample); an active POINTING term is
 * QC_E_UNSUPPORTED.  Every call on a device shares that device's array and
 * overwrites what it needs before reading it: calls that overlap on one device
 * (other streams, other host threads, other contexts) race and must not.
 */
#define QC_STATIC_SCRATCH_BYTES (4 * 1024 * 1024)
qc_status qc_solve_interval_static(qc_ctx* ctx, const qc_vis* vis, qc_term* chain, int32_t n_term,
                                   int32_t active, const qc_solve_opts* opts, qc_solve_stats* stats);

/*
 * Chain / epoch driver (Section 4.3): for n_epoch passes over the chain, solve
 * every term in array order with qc_solve_interval, the others fixed.
 * stats: NULL or an array of n_epoch * n_term entries ([epoch][term]).
 */
qc_status qc_solve_chain(qc_ctx* ctx, const qc_vis* vis, qc_term* chain, int32_t n_term, int32_t n_epoch,
                         const qc_solve_opts* opts, qc_solve_stats* stats);

/*
 * Chain / epoch driver with robust reweighting between epochs (Section 4.3,
 * solver features): as qc_solve_chain, and after every epoch but the last
 * the residual of the whole chain is formed into resid_work ([n_row][n_chan][4],
 * the data dtype) and the next epoch's weights into weight_work (the layout
 * and type of vis->weight) by qc_robust_weights from the prior weights
 * vis->weight and nu.  The work arrays are device memory owned by the caller
 * (unused, and may be NULL, when n_epoch <= 1); vis is not modified.
 */
qc_status qc_solve_chain_robust(qc_ctx* ctx, const qc_vis* vis, qc_term* chain, int32_t n_term, int32_t n_epoch,
                                const qc_solve_opts* opts, double nu, void* resid_work, void* weight_work,
                                qc_solve_stats* stats);

/*
 * Initial delay estimate (Section 4.3, "Initial estimates"): for every
 * interval of the DELAY (or DELAY_OFFSET) term k_term and every antenna a != ref_ant, per hand
 * (X: XX, Y: YY), y(nu) = sum over the interval's unflagged samples of the
 * baselines (ref, a) and (a, ref) of w D conj(M) (oriented so y ~
 * exp(2 pi i nu (tau_a - tau_ref)), M summed over directions); tau_a is the
 * first maximum of |sum_nu y(nu) exp(-2 pi i nu tau)|^2 on the grid
 * tau_k = k / (N dnu), k = -N/2..N/2-1, dnu the mean channel spacing of the
 * interval, N the smallest power of two >= 8 x its channels.  FP64.
 * Evenly spaced channels (to 1e-9 of their spacing, increasing or
 * decreasing) in intervals of at most 1024 channels take eight length-N/8
 * FFTs per hand; others the direct sum over channels (both give the grid
 * values to rounding).  Writes k_term->params for every gain direction
 * (DELAY_OFFSET terms: tau, with phi0 = 0); ref_ant gets 0.
 * QC_E_UNSUPPORTED if an interval has more than 1823 channels.
 */
qc_status qc_delay_init(qc_ctx* ctx, const qc_vis* vis, qc_term* k_term, int32_t ref_ant, void* stream);

/*
 * Visibility outputs (Section 4.4).  For every (row, channel), flagged
 * samples and autocorrelations included:
 *   CORRUPT: out = sum_{d in mask} C_{p,d} M_d C_{q,d}^H
 *   CORRECT: out = C_p^-1 D C_q^-H  (direction 0 of a chain whose every term
 *            maps all directions to one gain and that holds no POINTING term,
 *            QC_E_ARG otherwise; 0 where C_p or C_q is singular)
 * dir_mask: [n_dir] uint8 host array, NULL = all directions.
 * out: [n_row][n_chan][4] device array of the data dtype.  Arithmetic is in
 * the data precision (complex64 -> FP32, complex128 -> FP64).
 */
qc_status qc_apply_gains(qc_ctx* ctx, const qc_vis* vis, const qc_term* chain, int32_t n_term,
                         qc_apply_mode mode, const uint8_t* dir_mask, void* out, void* stream);

/* Residual r = D - sum_{d in mask} C_{p,d} M_d C_{q,d}^H (eq. baselineresidual);
 * a mask that drops directions peels them.  Same layout and precision rules as
 * qc_apply_gains. */
qc_status qc_residual(qc_ctx* ctx, const qc_vis* vis, const qc_term* chain, int32_t n_term,
                      const uint8_t* dir_mask, void* out, void* stream);

/* Gain solutions interpolated onto another time/frequency grid (paper
 * Section 4.4: gains of a previous run applied up- or downsampled, and
 * interpolated from one field to another for 1GC / transfer calibration).
 * src and dst are terms of the same type and n_gdir over n_ant antennas;
 * t_src [src->n_gt] and f_src [src->n_gf] (device, strictly increasing) are
 * the times (s) and frequencies (Hz) of src's solution points, t_dst
 * [dst->n_gt] and f_dst [dst->n_gf] (device) those wanted.  Per axis a
 * target point between source points i and i + 1 takes u = (x - x_i) /
 * (x_{i+1} - x_i); outside the source range the nearest end point.
 * Bilinear: amplitudes of the gain entries linearly, their phases relative to
 * the lower-left neighbour on the shortest arc linearly (then added to its
 * phase); DELAY/PHASE/AMPLITUDE terms interpolate their params linearly.
 * A target point with a flagged contributing neighbour (src->gain_flags, may
 * be NULL) is flagged in dst->gain_flags (may be NULL) and gets the identity
 * (zero params).  Writes dst->gains or dst->params.  FP64.  Reads the
 * coordinates back to check them (waits for `stream` once). */
qc_status qc_interp_term(qc_ctx* ctx, const qc_term* src, const double* t_src, const double* f_src,
                         qc_term* dst, const double* t_dst, const double* f_dst, int32_t n_ant, void* stream);

/* Weights of the corrected data C_p^-1 D C_q^-H (paper Section 4.4: corrected
 * weights as an output): w |c_p,i|^2 |c_q,j|^2 per correlation (i, j) in the
 * order XX, XY, YX, YY, c the diagonal of the chain's Jones matrix (the
 * off-diagonal terms of a full 2x2 chain are left out); with one weight per
 * sample (n_wcorr = 1) the mean of the four factors.  The chain must be
 * direction independent, without a POINTING term (QC_E_ARG otherwise).  weight_out: device, the layout
 * and type of vis->weight (may equal it).  Every (row, channel). */
qc_status qc_corrected_weights(qc_ctx* ctx, const qc_vis* vis, const qc_term* chain, int32_t n_term,
                               void* weight_out, void* stream);

/* Robust reweighting (paper Section 4.3, solver features: reweighting between
 * epochs after Sob et al. 2020, against overfitting RFI and unmodelled
 * emission), the expectation step of a complex Student's t noise model with
 * nu > 0 degrees of freedom: a weight w0 of vis->weight shared by D complex
 * correlations (D = 1 for n_wcorr = 4, D = 4 for n_wcorr = 1) with residuals
 * r_k becomes
 *   w = w0 (nu + D) / (nu + w0 sum_k |r_k|^2 / s2),
 * s2 the mean of w0 |r|^2 over every complex residual value of the unflagged
 * cross-correlation samples with a finite residual; other samples (and all
 * samples if there is none) keep w0.  FP64 arithmetic, fixed-order sums.
 * resid: device [n_row][n_chan][4] of the data dtype (qc_residual's output);
 * weight_out: device, the layout and type of vis->weight (may equal it);
 * s2_out: host, may be NULL (the call then does not wait), NaN if undefined. */
qc_status qc_robust_weights(qc_ctx* ctx, const qc_vis* vis, const void* resid, double nu, void* weight_out,
                            double* s2_out, void* stream);

/* Outlier flags from residual visibilities by the median absolute deviation
 * (paper Section 4.7, "Additional Features": with a near-complete model the
 * residuals are Gaussian and outliers are taken to be RFI).
 *   resid    : device [n_row][n_chan][4], same dtype as vis->data (the output
 *              of qc_residual); vis supplies weights, flags and antennas.
 * Per unflagged cross-correlation sample s = sum_k w_k |R_k|^2 (in the
 * residual's precision, one rounding per operation in a fixed order); per
 * group (QC_MAD_GLOBAL: every such sample; QC_MAD_BASELINE: every unordered
 * antenna pair) m = lower median of s, d = lower median of |s - m| (the
 * lower median of N values is the one of rank floor((N - 1) / 2)).  A sample
 * is flagged when s > m + k d (float64); a group with d = 0 flags nothing;
 * non-finite s take no part.  flag_out[r][c] (device, may equal vis->flag)
 * receives the input flag where it is set, else 1 for a new outlier, else 0.
 * stats (device, may be NULL): [n_groups][2] double (m, d); n_groups = 1 for
 * QC_MAD_GLOBAL, n_ant (n_ant - 1) / 2 for QC_MAD_BASELINE with the pair
 * (p, q), p < q, at p n_ant - p (p + 1) / 2 + q - p - 1.  n_flagged (host,
 * may be NULL) receives the number of new flags (the call then waits).
 * k must be finite and >= 0.  Scratch memory is owned by ctx. */
typedef enum { QC_MAD_GLOBAL = 0, QC_MAD_BASELINE = 1 } qc_mad_mode;
qc_status qc_mad_flag(qc_ctx* ctx, const qc_vis* vis, const void* resid, qc_mad_mode mode, double k,
                      uint8_t* flag_out, double* stats, int64_t* n_flagged, void* stream);

/*
 * Model visibilities predicted from a list of point components by a direct
 * Fourier sum (paper Section 4.7, "Additional Features": component models
 * predicted on the fly with the DFT; the predicted visibility M of
 * eq. baselinemodel).  For every row r, channel nu and direction d:
 *   M[r][nu][d] = sum over the components c with dir[c] = d of
 *                 B_c (nu / nu0_c)^alpha_c exp(-2 pi i nu (u l + v m + w (n - 1)) / c0)
 * with (u, v, w) = uvw[r] in metres, n = sqrt(1 - l^2 - m^2), c0 the speed of
 * light in vacuum, and the linear-feed brightness in the order (XX, XY, YX, YY)
 *   B = (I + Q, U + iV, U - iV, I - Q)   (no factor 1/2).
 * A direction without components predicts zero.
 * Components of one direction are summed in their order in the arrays.
 */
typedef struct {
  int64_t n_comp;
  const double*  lm;        /* [n_comp][2] direction cosines, l^2 + m^2 < 1        */
  const double*  stokes;    /* [n_comp][4] I, Q, U, V in Jy at ref_freq            */
  const double*  spi;       /* [n_comp] spectral index alpha                       */
  const double*  ref_freq;  /* [n_comp] reference frequency nu0 > 0, Hz            */
  const int32_t* dir;       /* [n_comp] model direction in [0, n_dir)              */
} qc_sky;
/* uvw [n_row][3] double, chan_freq [n_chan] double, every qc_sky array and
 * model_out [n_row][n_chan][n_dir][4] (complex64 for QC_C64, complex128 for
 * QC_C128, the layout of qc_vis.model) are device memory; model_out is
 * overwritten.  QC_C128: FP64 throughout.  QC_C64: the phase in turns is
 * formed and reduced to [-1/2, 1/2] in FP64, then the phasor, the spectral
 * factor and the sums are FP32.  The call reads the component directions back
 * to the host (it waits for `stream` once) to order the sums; QC_E_RANGE for a
 * direction outside [0, n_dir), QC_E_ARG for l^2 + m^2 >= 1 or nu0 <= 0 (both
 * found on the device, reported by this call, which then waits again).
 * Scratch memory is owned by ctx. */
qc_status qc_predict_dft(qc_ctx* ctx, const double* uvw, int64_t n_row, const double* chan_freq, int32_t n_chan,
                         const qc_sky* sky, int32_t n_dir, qc_dtype dtype, void* model_out, void* stream);

/*
 * The solve and outputs with the model predicted inside their passes (paper
 * Section 4.7, "Additional Features": component models predicted with the
 * DFT, here on the fly): every pass evaluates, per sample and model direction,
 * the direct Fourier sum of qc_predict_dft from the sky's components instead
 * of reading vis->model, which is not read and may be NULL (vis->n_dir gives
 * the directions; component directions must lie in [0, n_dir)).  uvw
 * [n_row][3] double (device, metres) are the rows' baseline coordinates.
 * The phase in turns is formed and reduced to [-1/2, 1/2] in FP64; the
 * phasor and the sums are in the solve's arithmetic (FP32 in MIXED, as
 * qc_predict_dft's complex64 output; FP64 otherwise).  Otherwise the calls
 * take the arguments and give the results of qc_solve_interval and
 * qc_residual / qc_apply_gains(CORRUPT).  The solve takes a single term with
 * one direction, or a chain whose terms are all DIAGONAL / DELAY / PHASE /
 * AMPLITUDE / DELAY_OFFSET / POINTING, with an active term that is not
 * POINTING and damping other than LM (QC_E_UNSUPPORTED otherwise); the
 * outputs take any chain.  The sky is checked and ordered as in
 * qc_predict_dft (the call waits for `stream` once to read it).
 */
qc_status qc_solve_interval_sky(qc_ctx* ctx, const qc_vis* vis, const qc_sky* sky, const double* uvw,
                                qc_term* chain, int32_t n_term, int32_t active, const qc_solve_opts* opts,
                                qc_solve_stats* stats);
qc_status qc_residual_sky(qc_ctx* ctx, const qc_vis* vis, const qc_sky* sky, const double* uvw,
                          const qc_term* chain, int32_t n_term, const uint8_t* dir_mask, void* out, void* stream);
qc_status qc_corrupt_sky(qc_ctx* ctx, const qc_vis* vis, const qc_sky* sky, const double* uvw,
                         const qc_term* chain, int32_t n_term, const uint8_t* dir_mask, void* out, void* stream);

/*
 * Learned warm start (a two-layer MLP from interval features to initial
 * diagonal gains), all FP32 unless stated.  Parameters are one flat array
 * [W1 (n_hid x n_in) | b1 (n_hid) | W2 (n_out x n_hid) | b2 (n_out)],
 * row-major; y = W2 relu(W1 x + b1) + b2.
 */
/* Interval features of `layout`'s solution intervals: per antenna a and
 * correlation k, rho_{a,k} = sum w_k D_k conj(M_k) / (sum w_k |M_k|^2 + 1e-12)
 * over the interval's unflagged samples, conjugate baselines folded in (D^H,
 * M^H, weights permuted by P), M summed over directions.
 * feat: [n_gt*n_gf][n_ant*8] float, layout [antenna][corr][re, im].
 * chisq_unit: NULL or [n_gt*n_gf] double, sum w |D - M|^2 (chi^2 at unit gains).
 * ref_ant >= 0: every ratio is rotated, per correlation, by the phase of that
 * antenna's, rho_a conj(rho_ref) / |rho_ref| (the gauge of the targets);
 * ref_ant < 0: raw ratios. */
qc_status qc_ws_features(qc_ctx* ctx, const qc_vis* vis, const qc_term* layout, float* feat,
                         double* chisq_unit, int32_t ref_ant, void* stream);
/* Forward pass of a batch: pre [batch][n_hid] = W1 x + b1, y [batch][n_out]. */
qc_status qc_mlp_forward(qc_ctx* ctx, const float* params, const float* x, int32_t batch, int32_t n_in,
                         int32_t n_hid, int32_t n_out, float* y, float* pre, void* stream);
/* Gradient of sum(dy * y) with respect to the parameters (grad has the
 * parameters' layout); needs the forward pass's pre-activations. */
qc_status qc_mlp_backward(qc_ctx* ctx, const float* params, const float* x, const float* pre, const float* dy,
                          int32_t batch, int32_t n_in, int32_t n_hid, int32_t n_out, float* grad, void* stream);
/* Adam (Kingma & Ba) with bias correction; step counts from 1. */
qc_status qc_adam_step(qc_ctx* ctx, float* params, const float* grad, float* m, float* v, int32_t n, float lr,
                       float b1, float b2, float eps, int32_t step, void* stream);
/* Mean squared error over n values: dy = 2 (y - t) / n; loss (device, 1 float, may be NULL). */
qc_status qc_mse_grad(qc_ctx* ctx, const float* y, const float* t, int32_t n, float* dy, float* loss, void* stream);
/* Diagonal gains [n_int][n_ant][1][4] complex128 from y [n_int][n_ant][hand][re, im]. */
qc_status qc_ws_gains(qc_ctx* ctx, const float* y, int32_t n_int, int32_t n_ant, void* gains, void* stream);
/* Regression targets from solved diagonal gains [n_int][n_ant][1][4] complex128:
 * per interval and hand, g_a conj(g_ref) / |g_ref| (the free phase gauge fixed at
 * ref_ant), written as y [n_int][n_ant][hand][re, im] float. */
qc_status qc_ws_labels(qc_ctx* ctx, const void* gains, int32_t n_int, int32_t n_ant, int32_t ref_ant, float* y,
                       void* stream);

/*
 * Batched solve of many independent problems of uneven size (row counts,
 * antennas, channels, term types) in one graph launch.  Solution intervals
 * are independent (Section 2.3), so the intervals of all problems form one
 * pool of work: a persistent kernel per size bucket pulls intervals from a
 * device queue (largest first) and runs the same per-interval solve as
 * qc_solve_interval.  Each problem is a single-term chain: DIAGONAL or
 * COMPLEX2X2, one model direction, one gain direction (QC_E_UNSUPPORTED
 * otherwise).  Every problem must share the data dtype; opts apply to all.
 * The plan holds the problems' device pointers: they must stay valid until
 * qc_batch_destroy.  Gains are overwritten in place on every run.
 */
typedef struct {
  qc_vis vis;
  qc_term term;             /* the solved term (its gains/gain_flags are in/out) */
  qc_solve_stats stats;     /* per interval of the term; pointers may be NULL */
  const double* chisq_ref;  /* NULL, or per interval of the term [n_gt][n_gf]: the
                               warm-start fallback of qc_solve_opts.chisq_ref for
                               this problem (opts.chisq_ref itself is ignored here) */
} qc_problem;

#define QC_BATCH_BUCKETS 6  /* channel width (<=16, <=32, wider) x size (< 65536 samples, larger) */

typedef struct qc_batch qc_batch;
/* Validate every problem, build the work items and capture the graph. */
qc_status qc_batch_create(qc_ctx* ctx, const qc_problem* problems, int32_t n_problem,
                          const qc_solve_opts* opts, qc_batch** out);
/* Autotuner: for every bucket, time each (waves per workgroup in {1,2,4,8},
 * rows per step in {1,2,4}) on the batch itself (best of `reps` runs, each
 * from the gains present at the call, which are restored afterwards), keep
 * the fastest and re-capture the graph.  Call it with the starting gains in
 * place: from converged gains every trial times only one or two updates. */
qc_status qc_batch_tune(qc_batch* batch, int32_t reps);
/* Launch the graph, ordered after earlier work on `stream`; later work on
 * `stream` waits for it. */
qc_status qc_batch_run(qc_batch* batch, void* stream);
/* Milliseconds of the last qc_batch_run (waits for it); negative on error. */
double    qc_batch_last_ms(qc_batch* batch);
/* Schedule per bucket (arrays of QC_BATCH_BUCKETS; any may be NULL):
 * work items, waves per workgroup, rows per step, tuned time (ms, < 0 if untuned). */
qc_status qc_batch_schedule(const qc_batch* batch, int32_t* items, int32_t* waves, int32_t* rows_per_step,
                            float* tuned_ms, int32_t n);
qc_status qc_batch_destroy(qc_batch* batch);
/* Learned warm start over a batch (the growth direction of the warm start;
 * no paper passage): the feature pass of qc_ws_features and the gain write
 * of qc_ws_gains for every interval of every problem, one launch each, on the
 * intervals the batch has already validated (no host wait).  Per-interval
 * arrays over the whole batch take the problems in order, the intervals of a
 * problem in its [n_gt][n_gf] order: interval (gt, gf) of problem i is row
 * n_0 + ... + n_{i-1} + gt * n_gf + gf, n_j = problem j's n_gt * n_gf;
 * qc_batch_n_intervals gives the total (-1 for a NULL batch).
 * qc_batch_ws_features: feat [rows][feat_stride] float (feat_stride >= 8 x
 * the largest antenna count; a problem with fewer antennas fills its first
 * 8 n_ant values), chisq_unit NULL or [rows] double (chi^2 at unit gains:
 * pass its row n_0 + ... + n_{i-1} as problem i's qc_problem.chisq_ref at
 * qc_batch_create for the unit-gain fallback), ref_ant as in qc_ws_features
 * (QC_E_ARG if outside a problem's antennas).
 * qc_batch_ws_gains: y [rows][y_stride] float, [antenna][hand][re, im] as
 * qc_ws_gains (y_stride >= 4 x the largest antenna count), written into every
 * problem's gains; every term must be DIAGONAL (QC_E_UNSUPPORTED otherwise).
 * All arrays are device memory; both are asynchronous on `stream`. */
int32_t   qc_batch_n_intervals(const qc_batch* batch);
qc_status qc_batch_ws_features(qc_batch* batch, float* feat, int32_t feat_stride, double* chisq_unit,
                               int32_t ref_ant, void* stream);
qc_status qc_batch_ws_gains(qc_batch* batch, const float* y, int32_t y_stride, void* stream);
/* create + run + wait + destroy */
qc_status qc_solve_batch(qc_ctx* ctx, const qc_problem* problems, int32_t n_problem, const qc_solve_opts* opts);

#ifdef __cplusplus
}
#endif
#endif /* QC_H */
