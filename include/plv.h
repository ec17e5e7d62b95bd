/*
 * plv.h -- C ABI of libplv: Phase Locking Value (PLV), imaginary PLV (iPLV)
 * and corrected imaginary PLV (ciPLV) of every pair of N signals on one AMD
 * MI355X (gfx950) GPU.
 *
 * Method (Bruna, Maestu, Pereda, "Phase Locking Value revisited"):
 *   Section II.A, Eq. 4:  each analytic-signal sample is normalised to a unit
 *                         phasor u = z / |z| (no angle, no exponential);
 *   Eqs. 5-7:             all pairs at once from one Hermitian product,
 *                         G = U U^H / T, G_ij = (1/T) sum_t u_i(t) conj(u_j(t));
 *   Eq. 2 / Eq. 7:        PLV_ij   = |G_ij|;
 *   Section II.C, Eq. 13: iPLV_ij  = |Im G_ij|;
 *   Eq. 14:               ciPLV_ij = |Im G_ij| / sqrt(1 - (Re G_ij)^2);
 *   Eq. 3:                for real input the analytic signal is formed first
 *                         (DFT-domain one-sided weights, optionally a
 *                         band-pass brick-wall mask).
 *
 * Conventions for every entry point:
 *   - Pointers inside plv_problem / plv_grad and the workspace are DEVICE
 *     pointers on the context's device.  Descriptor arrays (plv_problem,
 *     plv_grad, plv_band) and size outputs are HOST pointers.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Compute calls only enqueue work on it and return; results are ready
 *     when the stream has reached that point (plv_autotune alone waits for
 *     its trial runs).  Descriptor arrays may be freed as soon as the call
 *     returns.
 *   - Ownership: the caller allocates and owns every device buffer, including
 *     the workspace.  Compute entry points never allocate or free device
 *     memory.  plv_create allocates only host-side state.
 *   - Errors: arguments are checked on the host before anything is enqueued;
 *     on PLV_ERR_INVALID_ARG / PLV_ERR_WORKSPACE / PLV_ERR_UNSUPPORTED no
 *     output is touched.  PLV_ERR_DEVICE means a HIP call or launch failed
 *     (outputs undefined).  Faults inside kernels surface at the caller's next
 *     synchronisation.  plv_last_error() gives a message for the last failure
 *     on a context.  No C++ exception crosses the ABI.
 *   - Data: NaN/Inf in the input propagate to the affected outputs.  An exact
 *     zero sample z = 0 is not an error: its phasor is taken as 1 + 0i (the
 *     phase angle(0) = 0 of the per-pair formulation).
 *   - Outputs are full symmetric N x N matrices, row-major, with PLV = 1,
 *     iPLV = 0 and ciPLV = 0 on the diagonal; iPLV and ciPLV are absolute
 *     values (the signed parts are in G).  ciPLV is 0 where
 *     (1 - Re G)(1 + Re G) <= 0.
 *   - The normaliser is 1/T with T the true window length (t1 - t0), never a
 *     padded length.
 *   - A context may be used by one host thread at a time.
 */
#ifndef PLV_H
#define PLV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PLV_OK = 0,
    PLV_ERR_INVALID_ARG = 1, /* a pointer, size, enum or shape is invalid */
    PLV_ERR_WORKSPACE = 2,   /* workspace NULL, misaligned or smaller than required */
    PLV_ERR_DEVICE = 3,      /* a HIP runtime call or kernel launch failed */
    PLV_ERR_UNSUPPORTED = 4  /* a valid request that this build does not implement */
} plv_status;

/* Arithmetic of the Gram contraction (the phasor planes and the MFMA inputs).
 * Accumulation is FP32 inside a K-chunk of at most 16384 samples and FP64
 * across chunks for every mode except PLV_PREC_F64, which is FP64 throughout. */
typedef enum {
    PLV_PREC_F64 = 0,        /* FP64 input, FP64 phasors, FP64 MFMA; f64 / c128 outputs       */
    PLV_PREC_F32 = 1,        /* FP32 phasors, FP32 MFMA                                        */
    PLV_PREC_SPLIT_BF16 = 2, /* u = hi + lo in BF16; G ~ hi.hi^H + hi.lo^H + lo.hi^H, BF16 MFMA */
    PLV_PREC_BF16 = 3,       /* BF16 phasors, BF16 MFMA                                        */
    PLV_PREC_F16 = 4         /* FP16 phasors, FP16 MFMA                                        */
} plv_prec;

/* What `in` holds. */
typedef enum {
    PLV_INPUT_ANALYTIC = 0, /* interleaved complex analytic signal (c64; c128 for PLV_PREC_F64) */
    PLV_INPUT_REAL = 1      /* real band-limited signal (f32; f64 for PLV_PREC_F64)              */
} plv_input;

/* Which entry point a workspace is sized for. */
typedef enum {
    PLV_OP_FROM_ANALYTIC = 0,
    PLV_OP_FROM_REAL = 1,
    PLV_OP_BACKWARD_ANALYTIC = 2,
    PLV_OP_BACKWARD_REAL = 3,
    PLV_OP_COHERENCE = 4
} plv_op;

typedef struct plv_ctx plv_ctx;

/* One problem: N signals of one trial.  Several problems (uneven N and T) are
 * computed by one call, as the Appendix's per-trial loop does one trial at a
 * time. */
typedef struct {
    int64_t n;      /* signals, >= 1                                                  */
    int64_t t;      /* samples per signal held in `in`, >= 1                          */
    int64_t ld;     /* row stride of `in` in elements (complex elements for analytic
                       input), >= t                                                    */
    int64_t t0, t1; /* samples [t0, t1) enter the Gram, taken AFTER the analytic
                       signal is formed (trims padding).  t1 = 0 means t1 = t.
                       Requires 0 <= t0 < t1 <= t.                                     */
    const void *in; /* [n][ld] signals, device, 8-byte aligned (16 for c128)          */
    void *plv;      /* [nbands][n][n] outputs, device, or NULL when not wanted:       */
    void *iplv;     /*   f32 (f64 for PLV_PREC_F64), 4-byte aligned (8 for f64)       */
    void *ciplv;
    void *g;        /* [nbands][n][n] complex G = U U^H / T, interleaved (c64, or c128
                       for PLV_PREC_F64), or NULL.  Needed later by plv_backward.     */
} plv_problem;

/* Band of the analytic signal for real input, in Hz (Section II.A, Eq. 3).
 * fir_order = 0: a DFT-bin band, both edges included: weight 2 on the
 *   positive-frequency DFT bins k with f_lo <= k*fs/T <= f_hi (T = the full
 *   length t of the row), 0 on every other bin including DC and Nyquist.
 *   f_lo = f_hi = 0 selects the plain analytic signal (weights 1 at DC, 2 below
 *   Nyquist, 1 at Nyquist for even T, 0 above).
 * fir_order = L > 0 (even, <= PLV_FIR_MAX_ORDER, f_lo < f_hi <= fs/2): the
 *   forward-backward FIR band-pass the paper applies before the Hilbert
 *   transform (Section III; its design is not given there).  Taps: the ideal
 *   band-pass between f_lo and f_hi sampled at n = m - L/2, m = 0..L, times the
 *   Hamming window 0.54 - 0.46 cos(2 pi m / L), scaled to unit gain at
 *   (f_lo + f_hi) / 2.  Applied as the zero-phase gain |H|^2 on the row's DFT
 *   bins together with the plain one-sided weights, i.e. a circular
 *   convolution over the row with the taps and their reverse: it equals
 *   filtering forward then backward on every sample at least L from both ends
 *   of the row, so rows should carry at least L samples of real padding on
 *   each side, trimmed by [t0, t1). */
#define PLV_FIR_MAX_ORDER 16384
typedef struct {
    double f_lo, f_hi;
    int32_t fir_order; /* 0: DFT-bin band; L > 0: FIR band-pass of order L */
    int32_t reserved;  /* 0 */
} plv_band;

/* Upstream gradients for plv_backward: dL/d(output) as full [nbands][n][n]
 * matrices (same dtype as the outputs).  Entry (i,j) and (j,i) both feed pair
 * {i,j}; the diagonal is ignored.  NULL = zero. */
typedef struct {
    const void *dplv, *diplv, *dciplv;
    void *din; /* output: dL/d(in), same layout, ld and dtype as `in`; for
                  analytic input dL/dRe z + i dL/dIm z.  Samples outside [t0,t1)
                  get 0 for analytic input. */
} plv_grad;

/* ---------------------------------------------------------------- context */

/* Create a context bound to HIP device `device` (queries its compute-unit
 * count and kernel occupancy).  device = -1 creates a host-only context that
 * assumes an MI355X (256 CUs): it can size workspaces and validate arguments,
 * and compute calls on it return PLV_ERR_INVALID_ARG.  *ctx is NULL on failure. */
plv_status plv_create(plv_ctx **ctx, int device);
plv_status plv_destroy(plv_ctx *ctx);
const char *plv_status_str(plv_status s);
/* Message for the last failed call on `ctx` ("" if none); valid until the next call. */
const char *plv_last_error(const plv_ctx *ctx);
/* Library version as major*10000 + minor*100 + patch. */
int32_t plv_version(void);

/* ---------------------------------------------------------------- timing */

/* Stages of the path, as timed by plv_timing_read. */
typedef enum {
    PLV_STAGE_HILBERT = 0,   /* FFT analytic signal (+ normalisation when fused)  */
    PLV_STAGE_NORMALISE = 1, /* phasor normalisation of analytic input           */
    PLV_STAGE_GRAM = 2,      /* the Gram contraction on MFMA (all its launches)   */
    PLV_STAGE_EPILOGUE = 3,  /* chunk sum, metrics and mirrored store             */
    PLV_STAGE_BACKWARD = 4,  /* adjoint kernels of plv_backward                   */
    PLV_STAGE_STFT = 5,      /* windowed-segment DFT bins (plv_coherence_stft)   */
    PLV_NSTAGES = 8
} plv_stage;

typedef struct {
    double ms[PLV_NSTAGES];       /* summed GPU time per stage, milliseconds */
    int64_t calls[PLV_NSTAGES];   /* stage executions timed                  */
    int64_t launches[PLV_NSTAGES];/* kernel launches inside those stages     */
} plv_timing;

/* Enable (on != 0) or disable per-stage timing on `ctx`.  While enabled each
 * compute call records a HIP event pair on its stream around every stage
 * (the host-side cost is a few microseconds per stage). */
plv_status plv_timing_enable(plv_ctx *ctx, int32_t on);
/* Wait for the recorded events, add up their times into *out (host) and, if
 * reset != 0, forget them. */
plv_status plv_timing_read(plv_ctx *ctx, plv_timing *out, int32_t reset);
/* Per-call times of one stage: waits for the recorded (not yet reset) events
 * of `stage` and writes the duration of each recorded stage execution, in
 * call order, to ms[0..cap) (host, milliseconds) and its kernel launch count
 * to launches[0..cap) (host, may be NULL).  *count (host) receives the number
 * of recorded executions of the stage, which may exceed cap.  Nothing is
 * forgotten.  PLV_ERR_INVALID_ARG for a stage outside [0, PLV_NSTAGES), a
 * negative cap, or ms == NULL with cap > 0. */
plv_status plv_timing_list(plv_ctx *ctx, int32_t stage, double *ms, int32_t *launches, int64_t cap,
                           int64_t *count);

/* ------------------------------------------------------------- workspace */

/* Bytes of device workspace a call with these arguments needs (*bytes, host).
 * The workspace must be 256-byte aligned.  Its contents need no
 * initialisation and are garbage after the call. */
plv_status plv_workspace_size(const plv_ctx *ctx, plv_op op, plv_prec prec, const plv_problem *probs,
                              int64_t nprob, const plv_band *bands, int32_t nbands, size_t *bytes);

/* --------------------------------------------------------------- forward */

/* PLV, iPLV, ciPLV (and optionally G) of analytic signals (Eqs. 4-7, 13, 14).
 * Steps: phasor normalisation -> Gram on MFMA over K-chunks -> fixed-order
 * chunk sum + metric epilogue with mirrored store.  Outputs are [1][n][n]. */
plv_status plv_from_analytic(plv_ctx *ctx, plv_prec prec, const plv_problem *probs, int64_t nprob, void *ws,
                             size_t ws_bytes, void *stream);

/* The same from real signals: the analytic signal of every row is formed on
 * the GPU by FFT for each of the `nbands` bands (Eq. 3), trimmed to [t0, t1),
 * normalised and contracted.  Outputs are [nbands][n][n].  `bands` may be NULL
 * with nbands = 1 for the plain analytic signal.  fs > 0 is the sampling rate
 * in Hz used to place band edges (ignored when every band is plain).
 * A row's transforms are held in LDS: the FFT size M (t for a power-of-two
 * t >= 2, else the power of two >= 2t - 1) must be <= 8192 in every mode;
 * longer rows return PLV_ERR_UNSUPPORTED. */
plv_status plv_from_real(plv_ctx *ctx, plv_prec prec, const plv_problem *probs, int64_t nprob,
                         const plv_band *bands, int32_t nbands, double fs, void *ws, size_t ws_bytes,
                         void *stream);

/* Allocation-free variant of plv_from_analytic, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same computation, arguments and outputs
 * as plv_from_analytic with nprob = 1, but with no workspace argument: the
 * intermediate buffers (phasor planes, FP64 chunk partial sums) live in a
 * device array of PLV_NOALLOC_MAX_BYTES inside the library, one per GPU,
 * held until the process ends (its address on each device is looked up once,
 * in plv_create).  The call makes no hipMalloc / hipFree or other allocating
 * call and no host-to-device copy.  The caller still allocates and owns the
 * input and the outputs.
 *   Errors: PLV_ERR_UNSUPPORTED when nprob != 1 or when the problem needs more
 *   than PLV_NOALLOC_MAX_BYTES of scratch (the message gives the size needed;
 *   plv_workspace_size with PLV_OP_FROM_ANALYTIC returns the same figure);
 *   PLV_ERR_DEVICE when the library could not find its scratch array on this
 *   device; otherwise as plv_from_analytic.
 *   Concurrency: every call on one GPU uses that GPU's single scratch array,
 *   and the array keeps the previous call's contents (nothing in it needs to
 *   start at zero).  Calls on one stream are ordered and safe; calls whose
 *   work can overlap on one GPU (different streams, other host threads, other
 *   contexts on the same device) race on the array and give wrong results. */
#define PLV_NOALLOC_MAX_BYTES (64u << 20) /* 64 MiB per GPU */
plv_status plv_from_analytic_noalloc(plv_ctx *ctx, plv_prec prec, const plv_problem *probs, int64_t nprob,
                                     void *stream);

/* Coherency of complex rows (Section II.B, Eq. 12): Fourier coefficients of
 * one frequency over trials or windows, or analytic signals over time, given
 * exactly as for plv_from_analytic (interleaved c64; c128 for PLV_PREC_F64).
 *   C_ij = sum_s z_i(s) conj(z_j(s)) / sqrt(sum_s |z_i|^2 * sum_s |z_j|^2)
 * over the samples [t0, t1).  The problem's output fields are reused:
 * `plv` <- coherence |C|, `iplv` <- imaginary coherency |Im C|, `ciplv` <-
 * corrected imaginary coherency |Im C| / sqrt(1 - (Re C)^2) (radicand in FP64
 * as (1 - Re)(1 + Re), 0 where it is <= 0), `g` <- the complex coherency C.
 * The diagonal gets coherence 1, imaginary parts 0 and C_ii as computed; a
 * row that is zero over the window gets C = 0 with every other row.  Each
 * row is scaled by a power of two before the contraction (its largest
 * component into [0.5, 1)), which C does not see, so the 16-bit modes stay in
 * range.  Steps: row scale -> scaled planes -> Gram on MFMA -> fixed-order
 * chunk sums and the diagonal powers -> normalised epilogue with mirrored
 * store.  Outputs are [1][n][n]. */
plv_status plv_coherence(plv_ctx *ctx, plv_prec prec, const plv_problem *probs, int64_t nprob, void *ws,
                         size_t ws_bytes, void *stream);

/* Coherency of real signals over windowed segments (Section II.B, Eq. 12,
 * with the Fourier coefficients X_i(f, n) of segments n; Section III.B
 * computes coherence on Hamming-windowed segments with overlap).  Segment n
 * of a row covers samples t0 + n*hop + m, m = 0..seg-1, of its window
 * [t0, t1); there are S = floor((t1 - t0 - seg) / hop) + 1 >= 1 segments.
 * For every bin k = k_lo..k_hi of the segment length (frequency k*fs/seg):
 *   X_i(k, n) = sum_m w[m] x_i(t0 + n*hop + m) exp(-2 pi i k m / seg),
 *   C_ij(k)   = sum_n X_i(k,n) conj(X_j(k,n)) / sqrt(sum_n |X_i|^2 sum_n |X_j|^2),
 * and the outputs as plv_coherence gives them (`plv` <- coherence |C|,
 * `iplv` <- |Im C|, `ciplv` <- |Im C| / sqrt(1 - (Re C)^2), `g` <- C), one
 * [n][n] matrix per bin: outputs are [k_hi - k_lo + 1][n][n].  Windows are
 * symmetric: Hamming 0.54 - 0.46 cos(2 pi m / (seg - 1)), Hann
 * 0.5 - 0.5 cos(2 pi m / (seg - 1)), or rectangular.  `in` holds real rows
 * (f32; f64 for PLV_PREC_F64), 4-byte (8-byte) aligned; every problem of a
 * call uses the same segmentation.  Steps: twiddle and window tables ->
 * segment DFT bins (FP32; FP64 in PLV_PREC_F64) into the workspace -> the
 * coherency path of plv_coherence over the segments, all bins and problems
 * in one grouped launch.  Errors as for plv_coherence; PLV_ERR_INVALID_ARG
 * when the segmentation is out of range or a window holds no whole segment. */
typedef enum { PLV_WINDOW_HAMMING = 0, PLV_WINDOW_HANN = 1, PLV_WINDOW_RECT = 2 } plv_window;
#define PLV_STFT_MAX_SEG 4096
typedef struct {
    int32_t seg;      /* segment length, 2 <= seg <= PLV_STFT_MAX_SEG              */
    int32_t hop;      /* samples between segment starts, >= 1 (seg - overlap)      */
    int32_t k_lo;     /* DFT bins of a segment, 0 <= k_lo <= k_hi <= seg / 2;      */
    int32_t k_hi;     /*   at most 512 bins                                        */
    int32_t window;   /* plv_window                                                */
    int32_t reserved; /* 0                                                         */
} plv_stft;

plv_status plv_coherence_stft_workspace_size(const plv_ctx *ctx, plv_prec prec, const plv_problem *probs,
                                             int64_t nprob, const plv_stft *stft, size_t *bytes);
plv_status plv_coherence_stft(plv_ctx *ctx, plv_prec prec, const plv_problem *probs, int64_t nprob,
                              const plv_stft *stft, void *ws, size_t ws_bytes, void *stream);

/* Lachaux's time-resolved PLV across trials (Eq. 1; matrix form Eq. 8): for
 * every time point t of [t0, t1), the measures of the n signals with the
 * trials as the contracted axis,
 *   G_ij(t) = (1/ntr) sum_k u_i(t, k) conj(u_j(t, k)),  u = z / |z| (Eq. 4),
 * PLV(t) = |G(t)|, iPLV(t) = |Im G(t)|, ciPLV(t) as in plv_from_analytic.
 * Sample (trial k, signal i, time t) of the analytic signals is at
 * in + k*tstride + i*ld + t*sstride complex elements (c64; c128 for
 * PLV_PREC_F64), so trial-major [ntr][n][T] data (tstride = n*ld, sstride = 1)
 * and the signals x samples x trials layout (tstride = 1, sstride = ntr,
 * ld = T*ntr) are both accepted; reads coalesce best with sstride = 1.
 * Outputs are [t1 - t0][n][n] (g complex), NULL to skip.  Every time point
 * is one Gram problem of n rows and ntr samples; all of them run in one
 * grouped launch. */
typedef struct {
    int64_t n;        /* signals, >= 1                                          */
    int64_t ntr;      /* trials (the contracted axis), 1 <= ntr <= 2^17          */
    int64_t t;        /* time samples per signal and trial, >= 1                */
    int64_t ld;       /* stride between signals, complex elements, >= 1          */
    int64_t tstride;  /* stride between trials, complex elements, >= 1           */
    int64_t sstride;  /* stride between time samples, complex elements, >= 1     */
    int64_t t0, t1;   /* time points [t0, t1) get a matrix each; t1 = 0 means t */
    const void *in;
    void *plv, *iplv, *ciplv, *g;
} plv_trials;

plv_status plv_trials_workspace_size(const plv_ctx *ctx, plv_prec prec, const plv_trials *p, size_t *bytes);
plv_status plv_over_trials(plv_ctx *ctx, plv_prec prec, const plv_trials *p, void *ws, size_t ws_bytes,
                           void *stream);

/* -------------------------------------------------------------- autotune */

/* Measure the launch shape of a forward call on this device and keep the
 * fastest in `ctx`.  Not part of the paper: a tuning aid for the launch.
 *   One problem and one band: the K-chunk count.  The Gram sums over T
 *   (Eqs. 6-7) run as K-chunks, one work-group per (tile, chunk); the planner
 *   picks their number from a cost model, and this call replaces that choice
 *   by a measurement of the model's count and up to two exact splits on
 *   either side.  Every later plan on `ctx` with the same precision, row
 *   count and padded length uses the winner.
 *   Several problems or bands (one grouped launch, e.g. trials x bands of
 *   uneven size): the tile edge of each distinct row count n.  The Gram
 *   kernel has 128- and 64-wide output tiles (64 only in PLV_PREC_F64); for
 *   every n among the problems the call is run on the problems with that n
 *   alone, once per edge, and the faster edge is kept for row count n in
 *   every later forward plan on `ctx` (plv_tile_edge reports it).
 * Each candidate is run once untimed and three times between HIP events on
 * `stream` (the outputs are written as by the call itself); a candidate must
 * beat the best so far by more than 1% to replace it.  Query
 * plv_workspace_size again afterwards: the workspace depends on the choices.
 *   op: PLV_OP_FROM_ANALYTIC, PLV_OP_FROM_REAL or PLV_OP_COHERENCE; the other
 *     arguments exactly as for that call (bands/nbands/fs are read for
 *     PLV_OP_FROM_REAL only).  Candidates whose workspace exceeds ws_bytes are
 *     skipped.
 *   nchunk (host, may be NULL): the chunk count kept for a single problem, or
 *     0 for a grouped call.
 * Blocks the host until the trial runs have finished.  Argument errors as for
 * the compute call; PLV_ERR_DEVICE on a failed launch or event (the previous
 * choice is then kept). */
plv_status plv_autotune(plv_ctx *ctx, plv_op op, plv_prec prec, const plv_problem *probs, int64_t nprob,
                        const plv_band *bands, int32_t nbands, double fs, void *ws, size_t ws_bytes, void *stream,
                        int32_t *nchunk);

/* Tile edge (64 or 128) that a forward problem of n rows gets on `ctx` in
 * precision `prec`: the one plv_autotune measured or plv_set_tile_edge set,
 * else the planner's model (the edge with the smaller whole-tile MFMA work
 * over the upper triangle, the 64-wide tile's work weighted by 1/0.85).
 * ctx may be a host-only context or NULL (model only).  *bm is host. */
plv_status plv_tile_edge(const plv_ctx *ctx, plv_prec prec, int64_t n, int32_t *bm);
/* Set the tile edge of forward problems with n rows on `ctx` (bm = 64 or 128;
 * 64 only in PLV_PREC_F64), or return them to the model (bm = 0).  Host-only
 * bookkeeping; query plv_workspace_size afterwards. */
plv_status plv_set_tile_edge(plv_ctx *ctx, plv_prec prec, int64_t n, int32_t bm);

/* -------------------------------------------------------------- backward */

/* Gradient of a scalar loss with respect to the input, given dL/d(outputs).
 * Not in the paper; the adjoint of the forward map:
 *   Gbar from the metric derivatives; dL/dU = (Gbar + Gbar^H) U / T on MFMA;
 *   through u = z/|z|: zbar = i Im(conj(u) ubar) u / |z| (0 at z = 0);
 *   for real input through the analytic-signal map (a Hermitian operator):
 *   xbar = Re(IFFT(h .* FFT(zbar))).
 * Each problem must carry the complex G of the forward call in `g` (same
 * prec, bands, fs and window); the phasors are recomputed from `in`.
 * `kind` says what `in` holds; bands/nbands/fs as for plv_from_real (ignored
 * for analytic input). */
plv_status plv_backward(plv_ctx *ctx, plv_prec prec, plv_input kind, const plv_problem *probs,
                        const plv_grad *grads, int64_t nprob, const plv_band *bands, int32_t nbands, double fs,
                        void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PLV_H */
