/*
 * mf.h -- C ABI of libmf, an MI355X (gfx950) matched filter for compact-binary
 * inspiral searches.
 *
 * What it computes (arXiv:0906.4175, Sec. 1.1):
 *   Eq. (2)  S_n(f) = (4.49 f/f0)^-56 + 0.16 (f/f0)^-4.52 + 0.52 + 0.32 (f/f0)^2
 *   Eq. (1)  z(t)   = 4 int_0^inf conj(h_c(f)) s(f) / S_n(f) e^{2 pi i f t} df
 *            (conjugate on the template: the reading that makes z = x + i y
 *             with x, y the responses of h_c and h_s, h_c = -i h_s)
 *   Eq. (4)  sigma^2 = 4 int |h_c(f)|^2 / S_n(f) df
 *   Eq. (3)  rho(t) = |z(t)| / sigma, then its peak over t and a threshold count
 * with h_c the 2PN stationary-phase template with Newtonian amplitude that the
 * paper uses (Sec. 1.1), cut at f_low and at min(f_ISCO, Nyquist).
 *
 * Discretisation: N-point segments at sample rate fs, T = N/fs, df = 1/T,
 * one-sided bins k = 0..N/2 at f_k = k df; int df -> df * sum_k; the time
 * series is the unnormalised inverse DFT sum_k q_k e^{+2 pi i jk/N}.  The band
 * is k_lo = ceil(f_low T) .. k_hi = min(floor(f_ISCO T), N/2 - 1);
 * f_ISCO = 1/(6^{3/2} pi M), M = (m1+m2) G M_sun/c^3, G M_sun/c^3 =
 * 4.925490947641267e-6 s.  S_n carries no overall scale (S_0 = 1).
 *
 * Conventions for every call:
 *  - Pointers named *_dev are device pointers; *_host are host pointers.
 *    The caller owns every buffer.  The library calls no device allocator
 *    (mf_filter_noalloc works in a static device array of the library).
 *  - Complex arrays are interleaved (re, im) pairs: complex64 = 2 x float,
 *    complex128 = 2 x double.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Hot calls only
 *    enqueue work; setup calls may synchronise the stream.
 *  - Every call validates its arguments before enqueueing anything and returns
 *    an mf_status; on error nothing is enqueued and mf_last_error() holds a
 *    message (thread-local).  A HIP error of earlier asynchronous work can
 *    surface as MF_E_HIP on a later call.  Outputs are undefined after an
 *    error.  NaN/Inf inputs propagate to the affected outputs.
 */
#ifndef MF_H
#define MF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Same type as hipStream_t. */
typedef struct ihipStream_t* mf_stream_t;

typedef enum {
    MF_OK = 0,
    MF_E_ARG = -1,         /* null pointer, bad enum, bad count            */
    MF_E_SHAPE = -2,       /* N not a power of two in range, bad window     */
    MF_E_BAND = -3,        /* empty band (k_hi < k_lo) or f_low out of range */
    MF_E_HIP = -4,         /* HIP runtime error                             */
    MF_E_WORKSPACE = -5,   /* workspace too small                           */
    MF_E_UNSUPPORTED = -6  /* valid request the library does not implement  */
} mf_status;

typedef enum {
    MF_FP64 = 0,       /* plain path: data, phase, products, FFT, sigma in FP64   */
    MF_FP32_PH64 = 1,  /* FP32 data/products/FFT; SPA phase and sigma in FP64     */
    MF_FP32 = 2        /* FP32 throughout except sigma (precision study only)      */
} mf_precision;

typedef enum {
    MF_SIGMA_FP64 = 0,    /* sigma^2 accumulated in FP64                 */
    MF_SIGMA_COMP32 = 1   /* compensated (Kahan) FP32 accumulation        */
} mf_sigma_mode;

/* Segment grid: N = 2^m with 2^10 <= N <= 2^22, sample rate fs [Hz], low
 * frequency cutoff f_low [Hz] with 0 < f_low < fs/2, PSD knee f0 [Hz]
 * (150 for Eq. (2)). */
typedef struct {
    int64_t n;
    double fs;
    double f_low;
    double f0;
} mf_grid;

/* Per (template, segment) result.  rho is the maximum of |z_j|/sigma over the
 * search window, j its lowest index, n_above the number of window samples
 * with rho_j >= the threshold.  In the FP32 modes rho is computed from the
 * FP32 |z|^2 and the FP64 sigma. */
typedef struct {
    double rho;
    int32_t j;
    int32_t n_above;
} mf_peak;

/* One event (Sec. 3.3: triggers carry their SNR and chi^2): rho at sample j
 * of template t.  t = -1 marks a window without an event. */
typedef struct {
    double rho;
    int32_t j;
    int32_t t;
} mf_event;

/* Options of mf_filter.  A NULL options pointer means: no threshold count
 * (rho_threshold = +inf), window = the whole segment, no series. */
typedef struct {
    double rho_threshold;              /* count rho_j >= this (+inf: count none)        */
    int64_t j_begin, j_end;            /* search window [j_begin, j_end); j_end=0: N   */
    const int32_t* series_units_dev;   /* nullable: unit ids u = t*n_seg + s to store   */
    int32_t n_series;                  /* number of ids (rho_dev holds n_series x N)    */
} mf_filter_opts;

/* One template of a device bank (64 bytes, opaque to callers but fixed). */
typedef struct {
    double b1, b2, b3, b5;  /* SPA phase in cycles: sum_n b_n u^n, u = k^(-1/3)  */
    double c0;              /* constant phase in cycles                          */
    double sigma;           /* sqrt of Eq. (4) over the template's band          */
    int32_t k_lo, k_hi;     /* band                                              */
    float inv_sigma;        /* 1/sigma rounded to float                          */
    int32_t reserved;
} mf_bank_entry;

/* Thread-local message of the last failing call ("" if none). */
const char* mf_last_error(void);

/* Library version string. */
const char* mf_version(void);

/* Bytes of a device bank of n_tmpl templates (n_tmpl * sizeof(mf_bank_entry)). */
size_t mf_bank_bytes(int64_t n_tmpl);

/* Bytes of device workspace mf_filter needs for this request (0 on invalid
 * arguments, with mf_last_error set).  The bulk is one batch of
 * intermediates, min(n_tmpl * n_seg, units per batch) * N complex values: the
 * default plans batch about 8 GiB (1024 units at N = 2^20 in the FP32 modes),
 * so a large bank needs about 8 GiB plus N/2+1 complex weights per segment
 * (plus, with the persistent pass 1 of plan flag bit 5, one int32 work-order
 * entry per unit of a batch and a queue counter). */
size_t mf_filter_workspace_bytes(const mf_grid* grid, mf_precision prec,
                                 int64_t n_tmpl, int64_t n_seg);

/*
 * The launch plan mf_filter uses for this grid and precision (the built-in
 * default, or the plan installed by mf_set_plan): plan[0..7] = {N1, N2,
 * columns per pass-1 work-group, rows per pass-2 work-group, pass-1 threads,
 * pass-2 threads, units per batch, flags}.
 * flags bit 0: pass 1 of batch b and pass 2 of batch b-1 share a launch;
 * bit 1: the pass-2 stages exchange real and imaginary parts one after the
 * other through half the LDS (more work-groups per CU); bit 2 (with bit 1):
 * that exchange uses bank-conflict-free layouts (4096-point rows); bit 3:
 * pass 1 skips its first column stage for templates whose band lies below
 * row N1/16 (every such butterfly has one non-zero input); bit 4: pass 1
 * multiplies its output by the part of the four-step factor that the first
 * row stage of pass 2 would apply (a function of the row and of the block of
 * N2/R0 columns, R0 the first row radix), so that stage has no factor (needs
 * the pass-1 columns to divide N2/R0; not with bit 0); bit 5: pass 1 runs
 * as a persistent kernel (as many work-groups as stay resident) that takes
 * its tiles from a queue in the workspace, the units whose templates fill
 * the most band rows first (not with bit 0).  Bits 0-3 and 5 give bitwise the
 * same results; bit 4 moves one complex product from pass 2 to pass 1
 * (results agree to rounding).
 */
mf_status mf_filter_plan(const mf_grid* grid, mf_precision prec, int32_t plan[8]);

/*
 * Tuning support.  mf_plan_candidates writes up to `cap` candidate plans
 * (8 int32 each, same layout as mf_filter_plan, units = 0) for this N and
 * precision and returns how many exist (-1 on invalid arguments).
 * mf_set_plan installs a plan (units in [1, 4096]) for every later call with
 * this N and precision class (FP64 vs FP32 modes) in the process; NULL
 * restores the built-in default.  MF_E_UNSUPPORTED for a shape that is not
 * built.  Thread-safe.
 */
int32_t mf_plan_candidates(const mf_grid* grid, mf_precision prec, int32_t* plans, int32_t cap);
mf_status mf_set_plan(const mf_grid* grid, mf_precision prec, const int32_t plan[8]);

/*
 * mf_psd -- Eq. (2) on the one-sided bins (setup call).
 *   Sn_dev     [N/2+1] double, written: S_n(k df) for k_lo <= k <= N/2-1,
 *              +inf at the other bins (DC, below f_low, Nyquist), so that
 *              1/S_n = 0 there.
 *   prefix_dev nullable [N/2+1] double: P_k = sum_{k'<=k} f_k'^(-7/3) / S_n,k'
 *              (FP64 running sum; 4 df (P_khi - P_{klo-1}) is sigma^2).
 * Errors: MF_E_ARG (null grid/Sn_dev), MF_E_SHAPE (N), MF_E_BAND (f_low).
 */
mf_status mf_psd(const mf_grid* grid, double* Sn_dev, double* prefix_dev,
                 mf_stream_t stream);

/*
 * mf_psd_prefix -- the prefix array of mf_psd for a caller-supplied PSD
 * (setup call).  Any one-sided S_n array [N/2+1] can be passed to the other
 * calls in place of mf_psd's: they read it only on [k_lo, N/2-1] (bins
 * outside count as 1/S_n = 0, reading R3) and it must be finite and > 0
 * there (not checked on the device: a bad value propagates as NaN/inf into
 * sigma and rho).  This call writes P_k = sum_{1<=k'<=k, S finite}
 * f_k'^(-7/3) / S_n,k' for the chi^2 band edges.
 * Errors: MF_E_ARG, MF_E_SHAPE, MF_E_BAND, MF_E_HIP.
 */
mf_status mf_psd_prefix(const mf_grid* grid, const double* Sn_dev, double* prefix_dev,
                        mf_stream_t stream);

/*
 * mf_rfft_workspace_bytes / mf_rfft -- one-sided spectra of real time-domain
 * segments, s_k = dt sum_j x_j e^{-2 pi i jk/N} for k = 0..N/2 (the
 * discretisation of Eq. (1), reading R8; the paper's forward data FFTs,
 * Sec. 3.1).
 *   x_dev      [batch][N] real (double for MF_FP64, float otherwise).
 *   stilde_dev [batch][N/2+1] complex (complex128 / complex64), written: the
 *              layout mf_filter takes.
 *   N a power of two in [2^11, 2^23]; fs > 0 (dt = 1/fs).
 *   workspace  >= mf_rfft_workspace_bytes(n, prec, batch), 256-byte aligned.
 * Errors: MF_E_ARG, MF_E_SHAPE, MF_E_WORKSPACE, MF_E_HIP.
 */
size_t mf_rfft_workspace_bytes(int64_t n, mf_precision prec, int64_t batch);
mf_status mf_rfft(int64_t n, double fs, mf_precision prec, const void* x_dev, void* stilde_dev,
                  int64_t batch, void* workspace_dev, size_t workspace_bytes, mf_stream_t stream);

/*
 * mf_spa_bank -- 2PN stationary-phase templates (Sec. 1.1) and their norm
 * sigma (Eq. (4)) (setup call; synchronises `stream`).
 *   mc_host, eta_host [n_tmpl]: chirp mass [M_sun] > 0 and 0 < eta <= 1/4.
 *   Sn_dev     [N/2+1] double from mf_psd.
 *   prec       selects the materialised template's type (complex128 for
 *              MF_FP64, complex64 otherwise); the bank itself is FP64.
 *   sigma_mode FP64 or compensated-FP32 accumulation of sigma^2.
 *   bank_dev   mf_bank_bytes(n_tmpl) bytes, written.
 *   khi_host   nullable [n_tmpl] int32, written with k_hi.
 *   sigma_host nullable [n_tmpl] double, written with sigma.
 *   htilde_dev nullable [n_tmpl][N/2+1] complex: h_c(f_k) = f_k^(-7/6)
 *              exp(-i Psi(f_k)) in band, 0 outside (t_c = phi_c = 0).
 * Errors: MF_E_ARG (null pointers, mc <= 0, eta outside (0, 1/4]),
 *         MF_E_SHAPE, MF_E_BAND (a template whose band is empty; the message
 *         names its index), MF_E_HIP.
 */
mf_status mf_spa_bank(const mf_grid* grid, const double* mc_host, const double* eta_host,
                      int64_t n_tmpl, const double* Sn_dev, mf_precision prec,
                      mf_sigma_mode sigma_mode, void* bank_dev, int32_t* khi_host,
                      double* sigma_host, void* htilde_dev, mf_stream_t stream);

/*
 * mf_filter -- Eq. (1), (3) and the peak search for every (template, segment)
 * unit (hot call: asynchronous, no allocation, no synchronisation).
 *   bank_dev    from mf_spa_bank (same grid and Sn).
 *   stilde_dev  [n_seg][N/2+1] complex one-sided data spectra (complex128 for
 *               MF_FP64, complex64 otherwise), s_k = dt sum_j s_j e^{-2 pi i jk/N}.
 *   Sn_dev      [N/2+1] double from mf_psd.
 *   workspace   >= mf_filter_workspace_bytes(grid, prec, n_tmpl, n_seg) bytes,
 *               256-byte aligned.
 *   peaks_dev   [n_tmpl][n_seg] mf_peak, written.
 *   rho_dev     nullable; with opts->n_series > 0 it receives rho_j for the
 *               listed units, [n_series][N], float (FP32 modes) or double
 *               (MF_FP64).
 * Errors: MF_E_ARG, MF_E_SHAPE (bad window), MF_E_WORKSPACE, MF_E_HIP.
 */
mf_status mf_filter(const mf_grid* grid, const void* bank_dev, int64_t n_tmpl,
                    const void* stilde_dev, int64_t n_seg, const double* Sn_dev,
                    mf_precision prec, const mf_filter_opts* opts,
                    void* workspace_dev, size_t workspace_bytes,
                    mf_peak* peaks_dev, void* rho_dev, mf_stream_t stream);

/*
 * mf_filter_noalloc -- mf_filter for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as mf_filter, minus
 * the workspace: the call uses a static device array of
 * MF_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends, and calls no allocator.  The units per batch are
 * the plan's, lowered until one batch of intermediates fits the array (at
 * N = 2^20 in the FP32 modes, 63 units per batch for one segment), so the
 * results are bitwise those of mf_filter.
 *   stream  must belong to the current device (else MF_E_ARG).
 * Every call on a GPU shares that GPU's array: calls that overlap in time on
 * one GPU (different streams, host threads) race and their results are
 * undefined; calls ordered on one stream are safe.  The array keeps the last
 * call's contents; every value a call reads is written by that call first.
 * Errors: those of mf_filter; MF_E_WORKSPACE if one unit per batch plus the
 * per-segment weights and per-unit peak records exceed the array;
 * MF_E_HIP if the array's address cannot be looked up.
 */
#define MF_NOALLOC_SCRATCH_BYTES ((size_t)512 << 20)
mf_status mf_filter_noalloc(const mf_grid* grid, const void* bank_dev, int64_t n_tmpl,
                            const void* stilde_dev, int64_t n_seg, const double* Sn_dev,
                            mf_precision prec, const mf_filter_opts* opts,
                            mf_peak* peaks_dev, void* rho_dev, mf_stream_t stream);

/*
 * mf_ifft -- the unnormalised complex inverse DFT z_j = sum_k q_k e^{+2 pi i jk/N}
 * of `batch` contiguous N-point arrays, with the same two-pass kernels the
 * filter uses (diagnostic / test entry point).  q_dev and z_dev are
 * [batch][N] complex64 (MF_FP32*) or complex128 (MF_FP64) and may not
 * overlap.  workspace as for mf_ifft_workspace_bytes.
 */
size_t mf_ifft_workspace_bytes(int64_t n, mf_precision prec, int64_t batch);
mf_status mf_ifft(int64_t n, mf_precision prec, const void* q_dev, void* z_dev,
                  int64_t batch, void* workspace_dev, size_t workspace_bytes,
                  mf_stream_t stream);

/*
 * mf_snr_grad -- F = rho^2 = |Z|^2 / sigma^2 at continuous parameters and,
 * optionally, its gradient (hot call).
 *   theta_dev [n][3] double: chirp mass [M_sun], eta, t_c [s] per trigger.
 *   khi_dev   nullable [n] int32: frozen upper band edge per trigger (else
 *             computed from theta); the lower edge is k_lo of the grid.
 *   seg_dev   [n] int32 segment index of each trigger (0 <= seg < n_seg).
 *   Z = 4 df sum_{k in band} f_k^(-7/6) e^{+i Psi_k(theta)} s_k / S_k, i.e. z(t)
 *   of Eq. (1) at the continuous time t = t_c; sigma as in Eq. (4) over the
 *   same band.
 *   Z_dev     [n] complex128, written (kept for the backward pass).
 *   rho2_dev  [n] double, written with F.
 *   gbar_dev  nullable [n] double: if given, grad_dev [n][3] double receives
 *             gbar * dF/dtheta.
 * Errors: MF_E_ARG, MF_E_SHAPE, MF_E_BAND, MF_E_HIP.
 */
mf_status mf_snr_grad(const mf_grid* grid, const double* theta_dev, const int32_t* khi_dev,
                      const int32_t* seg_dev, int64_t n, const void* stilde_dev, int64_t n_seg,
                      const double* Sn_dev, mf_precision prec, double* Z_dev, double* rho2_dev,
                      const double* gbar_dev, double* grad_dev, mf_stream_t stream);

/*
 * mf_filter_events_workspace_bytes / mf_filter_events -- mf_filter with
 * thresholded, clustered events (Sec. 3.3; the paper gives no rule, this is
 * the library's): each series is cut into windows of W = 2^log2_window
 * samples.
 *  * Time clustering per (template, segment): a window's winner is its
 *    loudest sample with rho >= rho_threshold (lowest index on ties); it is an
 *    event unless the winner of an adjacent window lies within W samples of it
 *    with a larger rho (or an equal rho at a lower index).
 *  * Template clustering per segment: each window's loudest event across
 *    templates (ties: lowest template index), kept under the same rule.
 *   Arguments as for mf_filter (whole series, no window or series options),
 *   plus:
 *   rho_threshold   > 0; peaks_dev[].n_above counts samples at or above it.
 *   log2_window     4 <= log2_window <= min(16, log2 N).
 *   workspace       >= mf_filter_events_workspace_bytes(...), 256-byte aligned.
 *   unit_events_dev nullable [n_tmpl][n_seg][N/W] mf_event: time-clustered
 *                   events of every unit (t = -1 where none).
 *   seg_events_dev  [n_seg][N/W] mf_event, written: the segment events.
 * In MF_FP64 the window winner is decided on |z|^2 rounded down to 36
 * mantissa bits (relative 1.5e-11).
 * Errors: MF_E_ARG, MF_E_SHAPE, MF_E_WORKSPACE, MF_E_HIP.
 */
size_t mf_filter_events_workspace_bytes(const mf_grid* grid, mf_precision prec, int64_t n_tmpl,
                                        int64_t n_seg, int32_t log2_window);
mf_status mf_filter_events(const mf_grid* grid, const void* bank_dev, int64_t n_tmpl,
                           const void* stilde_dev, int64_t n_seg, const double* Sn_dev,
                           mf_precision prec, double rho_threshold, int32_t log2_window,
                           void* workspace_dev, size_t workspace_bytes, mf_peak* peaks_dev,
                           mf_event* unit_events_dev, mf_event* seg_events_dev, mf_stream_t stream);

/*
 * mf_chisq_events -- chi^2 of Eq. (5) and rho at listed events (hot call),
 * as mf_chisq but for event records instead of unit peaks.
 *   events_dev [n_seg][n_per_seg] mf_event (e.g. the seg_events_dev of
 *              mf_filter_events); row s belongs to segment s; entries with
 *              t < 0 are skipped (outputs 0).
 *   chisq_dev, rho_dev (nullable) [n_seg][n_per_seg] double, written.
 * Errors: MF_E_ARG, MF_E_SHAPE, MF_E_BAND, MF_E_HIP.
 */
mf_status mf_chisq_events(const mf_grid* grid, const void* bank_dev, int64_t n_tmpl,
                          const void* stilde_dev, int64_t n_seg, const double* Sn_dev,
                          const double* prefix_dev, mf_precision prec, int32_t p_bands,
                          const mf_event* events_dev, int64_t n_per_seg, double* chisq_dev,
                          double* rho_dev, mf_stream_t stream);

/*
 * mf_filter_chisq_workspace_bytes -- device workspace mf_filter_chisq needs:
 * the weighted data, the band table, and per unit of a batch the template x
 * weight product of the bands that are not transformed whole (at most
 * N/2 + p_bands (N2 + 16) values, N2 the plan's row length) and one
 * intermediate [N], plus peak partials.  0 for invalid arguments (no
 * band-mode plan, p_bands outside [2, 64]).
 */
size_t mf_filter_chisq_workspace_bytes(const mf_grid* grid, mf_precision prec, int64_t n_tmpl,
                                       int64_t n_seg, int32_t p_bands);

/* The launch plan of mf_filter_chisq for this grid and precision (layout of
 * mf_filter_plan; the last entry is 0).  Errors: MF_E_ARG, MF_E_SHAPE,
 * MF_E_UNSUPPORTED. */
mf_status mf_filter_chisq_plan(const mf_grid* grid, mf_precision prec, int32_t plan[8]);

/*
 * mf_set_band_plan -- installs a launch plan for mf_filter_chisq (tuning
 * support, host state only, thread-safe) for every later call with this N
 * and precision class (FP64 vs FP32 modes) in the process; NULL restores the
 * built-in default.  Layout of mf_filter_plan: plan[4] and plan[5] are the
 * pass-1 and pass-2 threads (plan[5] = B N2 / 16 selects radix-16 row stages,
 * B N2 / 8 radix 8, where built), plan[6] the units per batch in [1, 4096],
 * plan[7] must be 0.  The workspace size follows the installed plan.
 * Errors: MF_E_ARG (flags, units), MF_E_SHAPE, MF_E_UNSUPPORTED (shape not
 * built for this N and precision).
 */
mf_status mf_set_band_plan(const mf_grid* grid, mf_precision prec, const int32_t plan[8]);

/*
 * mf_filter_chisq -- the matched filter of mf_filter with the chi^2
 * time-frequency veto of Eq. (5) (Sec. 1.2) evaluated at EVERY time sample
 * (hot call: asynchronous, no allocation, no synchronisation).  The
 * template's band [k_lo, k_hi] is split into p_bands contiguous bands with
 * equal shares of sigma^2 (a bin belongs to the band in which the sum of
 * f^(-7/3)/S over the bins before it falls); z_l(t) is Eq. (1) restricted to
 * band l and
 *   chi^2(t) = p / sigma^2 sum_l |z_l(t) - z(t)/p|^2,  z = sum_l z_l.
 *   Arguments as for mf_filter, plus:
 *   prefix_dev     the prefix array written by mf_psd.
 *   p_bands        2 <= p <= 64.
 *   workspace      >= mf_filter_chisq_workspace_bytes(...), 256-byte aligned.
 *   peaks_dev      [n_tmpl][n_seg]: peak of rho = |z|/sigma (lowest index on
 *                  ties), threshold count, as mf_filter.
 *   chisq_dev      [n_tmpl][n_seg] double: chi^2 at each peak, written.
 *   rho_dev, chisq_series_dev  nullable; with opts->n_series > 0 both receive
 *                  [n_series][N] series (float for the FP32 modes, double for
 *                  MF_FP64) for the listed units.
 * Errors: MF_E_ARG, MF_E_SHAPE, MF_E_WORKSPACE, MF_E_UNSUPPORTED, MF_E_HIP.
 */
mf_status mf_filter_chisq(const mf_grid* grid, const void* bank_dev, int64_t n_tmpl,
                          const void* stilde_dev, int64_t n_seg, const double* Sn_dev,
                          const double* prefix_dev, mf_precision prec, int32_t p_bands,
                          const mf_filter_opts* opts, void* workspace_dev, size_t workspace_bytes,
                          mf_peak* peaks_dev, double* chisq_dev, void* rho_dev,
                          void* chisq_series_dev, mf_stream_t stream);

/*
 * mf_chisq -- the chi^2 veto of Eq. (5) (Sec. 1.2) at each unit's peak sample
 * (hot call).  The template's band [k_lo, k_hi] is split into p_bands
 * contiguous bands with equal shares of sigma^2 (a bin belongs to the band in
 * which the sum of f^(-7/3)/S over the bins before it falls), z_l(t) is Eq. (1)
 * restricted to band l, and
 *   chi^2(t) = p / sigma^2 sum_l |z_l(t) - z(t)/p|^2 ,
 * evaluated at t = peaks_dev[u].j * dt for every unit u = t*n_seg + s.
 *   bank_dev, stilde_dev, Sn_dev as for mf_filter; prefix_dev is the prefix
 *   array written by mf_psd; peaks_dev [n_tmpl][n_seg] from mf_filter.
 *   chisq_dev [n_tmpl][n_seg] double, written (NaN for an invalid peak index).
 *   rho_dev   nullable [n_tmpl][n_seg] double: |z(j)|/sigma at the same sample.
 *   2 <= p_bands <= 64.
 * Arithmetic: the SPA phase (plus the exactly reduced time shift j k / N) and
 * every band sum are FP64.  For MF_FP64 data the weight 4 df f^(-7/6) / S_n
 * and the rotor are FP64; for the FP32 modes they are FP32 (hardware square
 * root, reciprocal and sine/cosine of the reduced phase, as in mf_filter's
 * pass 1), which bounds chi^2 and rho at about 1e-6 relative to the FP64
 * evaluation.
 * Errors: MF_E_ARG, MF_E_SHAPE, MF_E_BAND, MF_E_HIP.
 */
mf_status mf_chisq(const mf_grid* grid, const void* bank_dev, int64_t n_tmpl, const void* stilde_dev, int64_t n_seg,
                   const double* Sn_dev, const double* prefix_dev, mf_precision prec, int32_t p_bands,
                   const mf_peak* peaks_dev, double* chisq_dev, double* rho_dev, mf_stream_t stream);

/*
 * mf_template_metric -- phase-maximised template-space metric at theta over
 * the band [k_lo, khi] (hot call).  With W_k = f_k^(-7/3)/S_k (= |h_k|^2/S_k,
 * the weight of Eq. (4)) and d_k = dPsi(f_k)/dtheta in radians,
 *   g_ij = <d_i d_j> - <d_i><d_j>,   <x> = sum_k W_k x_k / sum_k W_k,
 * so that near a maximum F(theta + delta) ~ F(theta) (1 - g_ij delta_i delta_j).
 *   theta_dev  [n][3] (M_c [M_sun], eta, t_c [s]);  khi_dev [n] int32 (required).
 *   metric_dev [n][6] double: (g_mm, g_me, g_mt, g_ee, g_et, g_tt).
 * Errors: MF_E_ARG, MF_E_SHAPE, MF_E_BAND, MF_E_HIP.
 */
mf_status mf_template_metric(const mf_grid* grid, const double* theta_dev, const int32_t* khi_dev, int64_t n,
                             const double* Sn_dev, double* metric_dev, mf_stream_t stream);

/*
 * Measurement hook (not part of the method).  With stride > 0, mf_filter
 * records a HIP event pair on its stream around every stride-th launch of its
 * transform kernels; mf_timing_read waits for the recorded events and returns
 * their summed duration [ms], the number of timed launches, and the
 * (template, segment) units whose pass 1 (template x weight product, column
 * transforms, intermediate store) and pass 2 (row transforms, |z| peak) those
 * launches processed; it then clears the record.  stride = 0 disables
 * recording.  Host state only; not thread-safe.
 */
mf_status mf_timing_enable(int32_t stride);
mf_status mf_timing_read(double* ms, int64_t* launches, int64_t* pass1_units, int64_t* pass2_units);
/* The same record split by launch kind: [0] pass-1 launches, [1] pass-2
 * launches, [2] pipelined steps (both roles).  mf_filter_chisq records its
 * band-mode passes the same way. */
mf_status mf_timing_read_split(double ms[3], int64_t launches[3], int64_t pass1_units[3],
                               int64_t pass2_units[3]);

/*
 * Calibration kernel (not part of the method): copies `bytes` (a non-zero
 * multiple of 16; both pointers 16-byte aligned, non-overlapping) from
 * src_dev to dst_dev with a plain streaming kernel.  Used to scale hardware
 * byte counters: it reads and writes exactly `bytes` each.
 */
mf_status mf_probe_copy(const void* src_dev, void* dst_dev, size_t bytes, mf_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* MF_H */
