/*
 * lloid.h -- C ABI of the MI355X (gfx950) LLOID filtering library.
 *
 * The library runs the filtering stage of the paper's pipeline on one GPU
 * (Sec. II.A and II.B): whitened strain is down-sampled to the rate of every
 * time slice, correlated with that slice's orthogonal basis filters,
 * multiplied by the slice's SVD coefficients (mixing matrix), up-sampled
 * and summed into one complex SNR series per template, and reduced on the
 * device to per-window SNR peaks; peaks with |SNR| >= threshold (4 by
 * default, Fig. 1 caption) are the triggers, and only they (not the SNR
 * series) come back to the host (Sec. II.B, last paragraph).  Each trigger
 * carries its phase, a sub-sample refinement of its peak and, for banks
 * given template autocorrelations, its signal-consistency value xi^2.  The
 * steps around the filter are here too: conditioning of raw strain (PSD,
 * whitening, gating; lloid_condition) and the coincidence of two detectors'
 * triggers (lloid_coincide).  Offline blocks go through lloid_filter /
 * lloid_filter_batch, live strides through the lloid_stream_* calls.
 *
 * Conventions shared by every call:
 *  - Every call returns lloid_status: LLOID_OK (0) or a negative error code.
 *    No C++ exception crosses this boundary.  lloid_last_error() returns a
 *    description of the last error raised on the calling thread.
 *  - Ownership: the caller owns every buffer passed in or out.  Inputs are
 *    copied (or fully consumed) before the call returns; the library owns
 *    its device state until the matching *_destroy call.
 *  - Pointers documented as "host or device" may point to host memory or to
 *    device memory of the context's GPU; the library finds out which.
 *  - Sample indices are full-rate samples; sample 0 is the first strain
 *    sample of an lloid_filter call or of a stream.
 *  - Strain is whitened data (unit variance per full-rate sample in the
 *    noise, as the filtering stage of Sec. II.A consumes it).  In the FP16
 *    and BF16 modes it is rounded to the operand type after multiplication
 *    by lloid_trigger_opts.strain_scale (exact power of two, default 1).
 *
 * Definitions (notation of the paper's method, Sec. II.A):
 *  f0 = full rate.  Template i has two real filters, row 2i (cos, Re z_i)
 *  and row 2i+1 (sin, Im z_i).  Slice s runs at rate r_s = f0 / D_s (D_s a
 *  power of two), starts J_s full-rate taps before coalescence (J_s a
 *  multiple of D_s), has N_s taps at rate r_s and L_s basis filters:
 *      o_s[l, k] = sum_{m < N_s} basis_s[l, m] x_s[k - J_s / D_s - m]
 *      y_s       = mixing_s o_s
 *  where x_s is the strain down-sampled to r_s by the zero-phase half-band
 *  stage d[k] = sum_{|n| <= 32} g[n] u[2k - n] applied log2(D_s) times,
 *      g[n] = 1/2 sinc(n/2) I0(10 sqrt(1 - (n/32)^2)) / I0(10),
 *  and the physical SNR is the up-sample-and-add cascade from the lowest
 *  rate up, w_k = (slices at rate f0/2^k) + up(w_{k+1}) with
 *      up(w)[n] = sum_j w[j] 2 g[n - 2j],
 *  Y = w_0, z_i[n] = Y_{2i}[n] + i Y_{2i+1}[n].  Strain is zero outside the
 *  data, so outputs near the ends see zero padding on both sides.
 *  Trigger window w covers samples [floor(w f0 a / b), floor((w+1) f0 a / b))
 *  for window length a/b seconds; its peak is the lowest sample attaining
 *  the maximum |z_i| in the window.
 */
#ifndef LLOID_H
#define LLOID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LLOID_OK = 0,
  LLOID_EINVAL = -1,  /* invalid argument (shape, rate, pointer, option) */
  LLOID_ENOMEM = -2,  /* device or host allocation failed */
  LLOID_EAGAIN = -3,  /* stream admission: not enough HBM budget now; the bank is queued */
  LLOID_ETRUNC = -4,  /* output buffer too small; the required count is returned */
  LLOID_EDEVICE = -5, /* a HIP runtime call failed */
  LLOID_EORDER = -6,  /* stream stride does not continue the previous one */
  LLOID_EDATA = -7    /* strain sample not finite once converted to FP32 and scaled */
} lloid_status;

typedef enum { LLOID_F64 = 0, LLOID_F32 = 1, LLOID_F16 = 2, LLOID_BF16 = 3 } lloid_dtype;

typedef struct lloid_ctx lloid_ctx;
typedef struct lloid_bank lloid_bank;
typedef struct lloid_stream lloid_stream;

/* One time slice of one SVD bank (Sec. II.A: the templates are split into
 * time slices, each with its own sample rate, and each slice is decomposed
 * by an SVD into orthogonal basis filters and SVD coefficients). */
typedef struct {
  int32_t rate_hz;       /* r_s; f0 / r_s is a power of two */
  int32_t n_taps;        /* N_s >= 1, taps at rate r_s */
  int64_t start_tap;     /* J_s >= 0, full-rate taps before coalescence, multiple of f0 / r_s */
  int32_t n_basis;       /* L_s, 1 <= L_s <= N_s */
  int32_t reserved;
  const double *basis;   /* host, [L_s][N_s] row-major; tap m sits J_s + m f0/r_s samples before coalescence */
  const double *mixing;  /* host, [2 n_templates][L_s] row-major; row 2i = cos (Re z_i), 2i+1 = sin (Im z_i) */
} lloid_slice;

typedef struct {
  int32_t full_rate_hz;  /* f0 */
  int32_t n_templates;   /* F >= 1 */
  int32_t n_slices;      /* S >= 1; every slice rate distinct from the others is not required */
  lloid_dtype compute;   /* operand type of both GEMMs: LLOID_F32, LLOID_F16 or LLOID_BF16;
                            accumulation is always FP32 */
  const lloid_slice *slices;
  int32_t autocorr_half; /* K, 0..512: lags of the signal-consistency value; 0 = not computed */
  int32_t reserved;
  const double *autocorr; /* host, [n_templates][2K + 1][2]: (Re, Im) of template i's normalised
                             complex autocorrelation R_i[k] at lag k = -K..K (index K + k; R_i[0] = 1);
                             NULL when K = 0 */
} lloid_bank_desc;

/* A trigger: the SNR peak of one template in one window with |z| >= threshold,
 * with its sub-sample refinement (Sec. III.C: the interpolation at the SNR
 * peak that the paper's port leaves out) and its signal-consistency value
 * (Sec. II.A: phase and xi^2 are computed for every trigger). */
typedef struct {
  int32_t bank;          /* bank index in a batched call / stream slot; 0 for lloid_filter */
  int32_t detector;      /* as passed by the caller */
  int32_t template_id;   /* i */
  float xi2;             /* sum_k |z_i[n*+k] - z_i[n*] R_i[k]|^2 / sum_k (2 - 2 |R_i[k]|^2) over the lags
                            k = -K..K with 0 <= n*+k < end of the data (1 on average in unit white
                            noise, 0 for a signal matching the template); 0 when the bank has K = 0 */
  int64_t window;        /* w */
  int64_t sample;        /* peak sample n* */
  float snr;             /* |z_i[n*]| */
  float phase;           /* atan2(Im z_i[n*], Re z_i[n*]) in (-pi, pi] */
  float snr_interp;      /* sub-sample peak: vertex of the parabola through |z_i| at n* - 1, n*, n* + 1 */
  float dt;              /* its offset from n* in samples, in [-1/2, 1/2] (0 when the triple is not
                            concave); the refined peak time is (sample + dt) / f0 */
} lloid_trigger;

typedef struct {
  int64_t window_num;    /* window length = window_num / window_den seconds, e.g. 1/10 */
  int64_t window_den;
  float threshold;       /* inclusive; 4.0 when the options pointer is NULL */
  float strain_scale;    /* power of two applied before rounding strain to FP16/BF16; 0 means 1 */
} lloid_trigger_opts;

/* Optional dense outputs of lloid_filter: the peak of every (template, window). */
typedef struct {
  float *snr;            /* [n_templates][n_windows], host or device, or NULL */
  int64_t *sample;       /* [n_templates][n_windows], host or device, or NULL */
  float *phase;          /* [n_templates][n_windows], host or device, or NULL */
  int64_t n_windows;     /* in: capacity per template; out: windows covering [0, n) */
} lloid_peaks;

/* Human-readable description of the last error on the calling thread. */
const char *lloid_last_error(void);

/* Library version string. */
const char *lloid_version(void);

/* Create a context on HIP device `device`.  `hip_stream` is the hipStream_t
 * every call of this context enqueues on (for example the caller's current
 * stream); NULL creates a private stream.  EDEVICE if the device is absent. */
lloid_status lloid_ctx_create(int device, void *hip_stream, lloid_ctx **out);
lloid_status lloid_ctx_destroy(lloid_ctx *ctx);

/* Stages of the filtering path, for per-stage device timing. */
typedef enum {
  LLOID_STAGE_INGEST = 0,    /* strain upload and conversion */
  LLOID_STAGE_DECIMATE = 1,  /* half-band decimation to every slice rate */
  LLOID_STAGE_FIR = 2,       /* basis-filter correlation, all slices */
  LLOID_STAGE_INTERP = 3,    /* interpolation of low-rate orthogonal SNR to f0 */
  LLOID_STAGE_MIX = 4,       /* mixing GEMM + complex SNR + window peaks */
  LLOID_STAGE_PHASE = 5,     /* phase, sub-sample peak and xi^2 at each trigger peak */
  LLOID_STAGE_TRIGGER = 6,   /* trigger compaction */
  LLOID_STAGE_D2H = 7,       /* results to the caller's buffers */
  LLOID_N_STAGES = 8
} lloid_stage;

/* Turn per-stage timing on (1) or off (0).  While on, every lloid_filter call
 * brackets each stage with HIP events on the context's stream and adds the
 * elapsed device time to the context's totals. */
lloid_status lloid_ctx_profile(lloid_ctx *ctx, int enable);

/* Totals since the last reset: ms[LLOID_N_STAGES] of device time and
 * calls[LLOID_N_STAGES] (host buffers, either may be NULL); reset != 0 clears
 * them afterwards. */
lloid_status lloid_ctx_stage_times(lloid_ctx *ctx, double *ms, int64_t *calls, int reset);

/* Upload one SVD bank (Sec. II.A "SVD bank").  Validates every slice (EINVAL
 * on a rate that is not f0 / 2^k with k <= 7, a start tap that is not a multiple of
 * f0 / r_s, L_s > N_s, a NULL array, autocorr_half outside 0..512 or a NULL
 * autocorr with K > 0, a non-finite autocorrelation value), scales each
 * slice's basis and the mixing matrices by exact powers of two, converts them
 * to the compute type, lays them out for the kernels, stores the
 * autocorrelations in FP32 and computes sigma^2 in FP64.  The descriptor and
 * its arrays are not referenced after the call returns. */
lloid_status lloid_bank_create(lloid_ctx *ctx, const lloid_bank_desc *desc, lloid_bank **out);

/* sigma2[i] = sum_s (1/D_s) sum_l (mixing_s[2i][l]^2 + mixing_s[2i+1][l]^2), the
 * squared full-rate norm of template i as the bank reconstructs it (cos plus
 * sin; equal to the expected |z_i|^2 in unit white noise), computed in FP64
 * on the device.  out: host, [n_templates]. */
lloid_status lloid_bank_sigma2(const lloid_bank *bank, double *out);

/* Shape of an uploaded bank. */
typedef struct {
  int32_t full_rate_hz;
  int32_t n_templates;
  int32_t n_slices;
  int32_t n_levels;      /* 1 + log2(f0 / lowest slice rate) */
  lloid_dtype compute;
  int32_t concat_k;      /* columns of the concatenated basis operand (sum of padded L_s) */
  int64_t device_bytes;  /* device memory held by the bank's arrays (not the workspace) */
} lloid_bank_info;

lloid_status lloid_bank_query(const lloid_bank *bank, lloid_bank_info *out);
lloid_status lloid_bank_destroy(lloid_bank *bank);

/* Filter one block of strain (offline mode: zero strain before sample 0 and
 * after sample n-1) and reduce it to triggers.
 *   strain: host or device, n samples of `strain_dtype` (F64 or F32).
 *   opts:   window and threshold; NULL means 1 s windows and threshold 4.
 *   trig:   host or device, capacity trig_cap; *n_trig receives the number
 *           of triggers.  If it exceeds trig_cap the first trig_cap (in
 *           template-major, window-minor order) are written and ETRUNC is
 *           returned with *n_trig = the required count.  Device memory and
 *           pinned host memory receive the records straight from the
 *           compaction kernel; pageable host memory through a staged copy.
 *   snr:    NULL, or host or device [n_templates][n][2] float receiving the
 *           complex SNR (Re, Im) of every template at every sample.
 *   peaks:  NULL, or dense per-(template, window) peak outputs.
 * Triggers are ordered by template, then window.  EDATA if a strain sample is
 * not finite; EINVAL if n is not in [1, 2^28] (longer blocks are split by
 * the caller).  Blocks until the results are in the caller's buffers. */
lloid_status lloid_filter(lloid_bank *bank, int32_t detector,
                          const void *strain, lloid_dtype strain_dtype, int64_t n,
                          const lloid_trigger_opts *opts,
                          lloid_trigger *trig, int64_t trig_cap, int64_t *n_trig,
                          float *snr, lloid_peaks *peaks);

/* Allocation-free form of lloid_filter, for callers that cannot allocate
 * device memory: code under HIP graph capture, serving loops and harnesses
 * that forbid hipMalloc.  Same arguments, results and errors as lloid_filter
 * (without the SNR-series output), bit-identical results.  Every device
 * buffer of the call comes from one static array per GPU of
 * LLOID_NOALLOC_SCRATCH_BYTES, part of the library's code object (held until
 * the process ends); windows are processed in chunks sized to fit it, and the
 * descriptor tables are staged in pageable host memory.  The call makes no
 * hipMalloc, hipHostMalloc or hipFree and records no profiling events.
 * ENOMEM, before any device work, when one window per chunk (the strain
 * levels, the peak tables, trig_cap trigger records and, for host strain, a
 * copy of it) does not fit the array.  Every call on one GPU, from any
 * context, shares that GPU's array: calls that overlap on one GPU race and
 * must be serialised by the caller.  The array keeps the last call's
 * contents; the call clears what it needs cleared. */
#define LLOID_NOALLOC_SCRATCH_BYTES (256ll << 20)
lloid_status lloid_filter_noalloc(lloid_bank *bank, int32_t detector,
                                  const void *strain, lloid_dtype strain_dtype, int64_t n,
                                  const lloid_trigger_opts *opts,
                                  lloid_trigger *trig, int64_t trig_cap, int64_t *n_trig,
                                  lloid_peaks *peaks);

/* Filter one block of strain of one detector with many SVD banks at once
 * (Sec. II.B: banks are stacked and filtered together).  The banks must share
 * the context, full rate and compute type; they may differ in every other
 * respect (templates, slices, rates, lengths).  Each stage of the path runs
 * as one launch over a descriptor table of all banks' work, longest work
 * first.  The strain is down-sampled once for all banks.
 *   banks:  n_banks bank handles; trigger records carry the bank's index in
 *           this array in their `bank` field.
 *   peaks:  NULL, or n_banks dense peak outputs (one per bank, as in
 *           lloid_filter).
 * Other arguments and errors are as for lloid_filter; triggers are ordered by
 * bank, then template, then window. */
lloid_status lloid_filter_batch(lloid_bank *const *banks, int32_t n_banks, int32_t detector,
                                const void *strain, lloid_dtype strain_dtype, int64_t n,
                                const lloid_trigger_opts *opts,
                                lloid_trigger *trig, int64_t trig_cap, int64_t *n_trig,
                                lloid_peaks *peaks);

/* ---- streaming (serving) ----
 * Sec. II.B (online, low-latency mode): strain arrives in strides per
 * detector; the down-sampled strain of every rate stays on the device as the
 * filters' history.  Every time all detectors hold enough strain to complete
 * trigger windows, one tick filters those windows for every admitted bank and
 * detector, one launch per stage for all of them, and queues the triggers for
 * lloid_stream_poll.  Banks ("requests") are admitted into slots while their
 * arrays plus their per-tick scratch fit the device-memory budget; later ones
 * wait in arrival order and are admitted when slots are removed.  A bank
 * reports the windows from its admission on; since the history is complete,
 * every result equals the one lloid_filter gives for the whole stream (bit for
 * bit).  After lloid_stream_flush (zero strain past the end, as lloid_filter
 * assumes) the stream emits its remaining windows and accepts no more strain.
 *
 * The work runs asynchronously: lloid_stream_push checks a stride and copies
 * it into a staging ring, then returns; a library thread uploads, converts
 * and decimates the strides in order on a second HIP stream and enqueues the
 * ticks on the context's stream without waiting for them, and another thread
 * queues each tick's triggers when its device work completes.  The upload of
 * the next stride and the host work of the next tick overlap the device work
 * of the current one.  Calls on one stream must not overlap (one producer
 * thread); lloid_stream_poll may wait for the work pushed before it. */
typedef struct {
  int32_t n_detectors;          /* 1..16 */
  int32_t min_rate_hz;          /* lowest slice rate an admitted bank may use */
  int32_t max_windows_per_tick; /* windows filtered by one tick at most; 0 means 8 */
  int32_t use_graph;            /* nonzero: each tick's device work (table upload, every stage,
                                   trigger count) runs as a captured HIP graph, replayed while the
                                   tick's shape (slots, windows, buffers) is unchanged and captured
                                   again when it changes; results are those of the direct launches */
  double max_filter_s;          /* longest slice span (J_s / f0 + N_s / r_s) an admitted bank may
                                   have, in seconds; sets the history kept; 0 means 66 */
  int64_t hbm_budget;           /* device bytes for admitted banks (arrays + per-tick scratch);
                                   0 means no limit */
  lloid_trigger_opts trig;      /* window length, threshold, strain scale */
  int32_t queue_strides;        /* staging entries of the stride ring (each holds up to
                                   max(f0, max_windows_per_tick window lengths + 1) samples):
                                   push waits while all hold strides not yet uploaded; 0 means 64 */
  int32_t reserved;
} lloid_stream_opts;

typedef struct {
  int64_t ticks;                /* ticks that filtered at least one bank */
  int64_t windows;              /* windows emitted (per detector) */
  int64_t triggers;             /* triggers queued so far */
  int64_t next_window;          /* first window not yet emitted */
  double latency_p50_ms;        /* push of the stride that completed a tick -> the tick's device
                                   work done and its triggers queued for poll (over the ticks since
                                   creation or the last lloid_stream_stats_reset) */
  double latency_p99_ms;
  double latency_max_ms;
  int32_t active_slots;
  int32_t queued_banks;
  int64_t bytes_in_use;         /* budget taken by active slots */
  int64_t graph_captures;       /* with use_graph: ticks that captured a new graph */
  int64_t graph_replays;        /* with use_graph: ticks that replayed the previous one */
  int64_t queued_strides;       /* pushed pieces not yet taken by the library thread */
  int64_t ticks_in_flight;      /* ticks enqueued on the device and not yet completed */
} lloid_stream_stats;

lloid_status lloid_stream_create(lloid_ctx *ctx, int32_t full_rate_hz, lloid_dtype compute,
                                 const lloid_stream_opts *opts, lloid_stream **out);
/* Admit a bank (same context, full rate and compute type as the stream).  The
 * bank must outlive its slot.  It joins at the stream's position after every
 * stride pushed so far (the call waits until the library thread has taken
 * them) and reports from the next window not yet enqueued
 * (lloid_stream_stats.next_window).  *slot receives the slot id, which trigger
 * records carry in their `bank` field.  EAGAIN: the bank is queued and becomes
 * active when enough budget frees up; ENOMEM: it can never fit the budget;
 * EINVAL: its filters are longer than the stream's history. */
lloid_status lloid_stream_admit(lloid_stream *s, lloid_bank *bank, int32_t *slot);
/* Remove an active or queued slot at the stream's position after every stride
 * pushed so far; queued banks are admitted as budget frees up.  Returns when
 * no tick in flight reads the bank any more (it may then be destroyed). */
lloid_status lloid_stream_remove(lloid_stream *s, int32_t slot);
/* Queue n samples (host or device, F64 or F32) of detector `detector`
 * starting at full-rate sample t0, which must continue the previous stride
 * (EORDER otherwise).  Non-blocking: the call checks every sample, copies the
 * stride into the staging ring and returns; it waits only while every ring
 * entry holds a stride not yet uploaded.  EDATA if a sample (scaled, in FP32)
 * is not finite: nothing of the stride is queued and the detector still
 * expects t0.  Errors of the asynchronous work are returned by the next call. */
lloid_status lloid_stream_push(lloid_stream *s, int32_t detector, int64_t t0, const void *data,
                               lloid_dtype dtype, int64_t n);
/* Move up to cap queued triggers (tick order; within a tick by slot,
 * detector, template, window) into out (host).  wait_ms = 0: return at once
 * with what is queued; > 0: first wait up to wait_ms milliseconds until every
 * stride pushed before the call is filtered; < 0: wait for that without a
 * limit. */
lloid_status lloid_stream_poll(lloid_stream *s, lloid_trigger *out, int64_t cap, int64_t *n_out, int32_t wait_ms);
/* Zero strain past the end of every detector (which must hold the same
 * number of samples); returns when every window is filtered and queued. */
lloid_status lloid_stream_flush(lloid_stream *s);
lloid_status lloid_stream_stats_get(const lloid_stream *s, lloid_stream_stats *out);
/* Clear the latency record and the tick, window, trigger and graph counts. */
lloid_status lloid_stream_stats_reset(lloid_stream *s);
/* Stops the library threads (strides not yet taken are dropped), waits for
 * the ticks in flight and frees the stream. */
lloid_status lloid_stream_destroy(lloid_stream *s);

/* ---- conditioning before the filter ----
 * Sec. II.A conditions the strain before filtering: a PSD estimate, whitening
 * with it, and gating of large deviations of the whitened data.  Segments of
 * L samples start every L/2 samples and carry a periodic Hann window
 * w[n] = sin^2(pi n / L) (w[n] + w[n + L/2] = 1).
 *   PSD:       the mean over the segments wholly inside the block of the
 *              one-sided periodogram c_f |DFT(w x_m)[f]|^2 / (f0 sum w^2),
 *              c_f = 2 except at f = 0 and L/2 (unit-variance white noise has
 *              S = 2 / f0); or the caller's PSD.
 *   whitening: every segment (data zero outside the block) is windowed,
 *              transformed, scaled by G[f] = 1 / sqrt(S[f] f0 / 2) (0 where
 *              S[f] <= 0), transformed back and overlap-added.
 *   gating:    every whitened sample above the threshold in magnitude zeroes
 *              the samples within gate_half_width of it. */
typedef struct {
  int32_t seg_len;         /* L: a power of two, 64..4096 */
  int32_t gate_half_width; /* >= 0 */
  float gate_threshold;    /* 0: no gating */
  int32_t reserved;
  const double *psd;       /* host, [L/2 + 1] one-sided PSD to whiten with; NULL: estimate it from
                              this block (which then needs n >= L) */
} lloid_condition_opts;

/* Condition one block of strain (host or device, F64 or F32, n >= 1 samples
 * at full_rate_hz) into out (n floats, host or device: the whitened and gated
 * strain, ready for lloid_filter).  psd_out: NULL or host [L/2 + 1], the PSD
 * used (the device estimates and applies it in FP32, a compensated mean over
 * the segments; a caller's PSD is rounded to FP32).  n_gated: NULL or the
 * number of samples zeroed by the gate.
 * EINVAL on a bad length, rate or option, a block shorter than one segment
 * without a PSD, or a non-finite PSD value; EDATA if a strain sample is not
 * finite.  Runs on the context's stream and returns when the results are in
 * the caller's buffers. */
lloid_status lloid_condition(lloid_ctx *ctx, int32_t full_rate_hz, const void *strain, lloid_dtype dtype, int64_t n,
                             const lloid_condition_opts *opts, float *out, double *psd_out, int64_t *n_gated);

/* ---- coincidence across detectors ----
 * A coincidence pairs the triggers of one template of one bank in two
 * detectors whose peak samples lie within the light travel time between the
 * detectors (Sec. II.A: the coincidence generator pairs triggers of the same
 * template within the light travel time; the non-coincident triggers of
 * times when several detectors observe are the background). */
typedef struct {
  int64_t a, b;          /* indices into the first and the second trigger list */
  int32_t bank;
  int32_t template_id;
  float snr_net;         /* network SNR sqrt(snr_a^2 + snr_b^2) */
  float dt;              /* (sample_b + dt_b) - (sample_a + dt_a): arrival difference in samples,
                            with each trigger's sub-sample refinement */
} lloid_coinc;

/* Every pair (i, j) with a[i].bank == b[j].bank, a[i].template_id ==
 * b[j].template_id and |a[i].sample - b[j].sample| <= max_dt (samples, for
 * example the light travel time times f0, rounded up), in order of i, then j.
 *   a, b:        trigger lists (host or device), each sorted by (bank,
 *                template_id, sample) as lloid_filter and lloid_filter_batch
 *                return one detector's triggers; n_a, n_b >= 0.
 *   out:         cap records (host or device); *n_out = number of pairs.
 *   background:  NULL, or n_a + n_b bytes (host or device): 1 for each trigger
 *                of a, then of b, that is in no pair, else 0.
 * EINVAL on a NULL list with a positive count, a list out of order or
 * max_dt < 0; ETRUNC when the pairs exceed cap (*n_out is then the number
 * needed; the first cap pairs are written).  Runs on the context's stream and
 * returns when the results are in the caller's buffers. */
lloid_status lloid_coincide(lloid_ctx *ctx, const lloid_trigger *a, int64_t n_a, const lloid_trigger *b,
                            int64_t n_b, int64_t max_dt, lloid_coinc *out, int64_t cap, int64_t *n_out,
                            uint8_t *background);

/* ---- tile shapes and their autotuning ----
 * The FIR and mixing kernels are compiled in a few tile shapes (variants:
 * FIR 0 .. LLOID_FIR_VARIANTS - 1, mixing 0 .. LLOID_MIX_VARIANTS - 1; 0 is
 * the default).  Every variant gives
 * bit-identical results (each output's sum over K runs in the same order);
 * only the speed differs with the banks' shapes.  A context starts with the
 * defaults, or the variants named by the environment variables
 * LLOID_FIR_VARIANT and LLOID_MIX_VARIANT. */
#define LLOID_FIR_VARIANTS 6
#define LLOID_MIX_VARIANTS 5

typedef struct {
  int32_t fir_variant;
  int32_t mix_variant;
  double ms;             /* fastest of four timed lloid_filter_batch calls after a warm-up */
} lloid_tune_result;

lloid_status lloid_ctx_set_tiles(lloid_ctx *ctx, int32_t fir_variant, int32_t mix_variant);
lloid_status lloid_ctx_get_tiles(const lloid_ctx *ctx, int32_t *fir_variant, int32_t *mix_variant);

/* Pick the tile variants for a set of banks: time lloid_filter_batch over
 * `seconds` (0 < seconds <= 4096) of synthetic unit-variance noise on the
 * device with every variant pair and keep the fastest on the context.
 *   cache_path: NULL, or a JSON file of earlier choices keyed by device
 *               architecture, operand type, the banks' shape (count, rows,
 *               concatenated K, longest filter, rate levels) and the block
 *               length (rounded up to a power of two; tune with the block
 *               length the filter calls will use).  A key
 *               found there is applied without timing (*n_results = 0); a
 *               new choice is added to the file.
 *   results:    host, cap entries receiving every timed pair; *n_results is
 *               the number timed.
 * EINVAL on a NULL argument, banks of another context, seconds out of range
 * or a cache file that cannot be written. */
lloid_status lloid_autotune(lloid_ctx *ctx, lloid_bank *const *banks, int32_t n_banks, double seconds,
                            const char *cache_path, lloid_tune_result *results, int32_t cap, int32_t *n_results);

/* Device bytes the filter calls of this context may use for the per-chunk
 * operands (the orthogonal SNR of every bank over a run of whole windows);
 * longer blocks are processed in several chunks.  Default 6 GiB. */
lloid_status lloid_ctx_set_chunk_bytes(lloid_ctx *ctx, int64_t bytes);

#ifdef __cplusplus
}
#endif

#endif /* LLOID_H */
