// Internal interfaces between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lloid.h"
#include "lloid_plan.h"

namespace lloid {

// GEMM tiling shared by the FIR and the mixing kernels (wave64, 4 waves).
constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kBK = 32;          // K chunk staged in LDS (FIR; the concatenated K is a multiple of 64)
constexpr int kLPad = 16;        // basis count padding inside the concatenated K
constexpr int kRowTile = 32;     // MFMA 32x32 tile

// FIR tiles of FP32 operands and of 16-bit variants 1 and 5: kFirWaves waves
// share 32 * kFirMT basis rows and split kFirWaves * 32 * kFirNT columns; the
// strain window of kFirKSup taps is staged in LDS at a time.
constexpr int kFirMT = 4, kFirNT = 2, kFirWaves = 8, kFirKSup = 1024;
// Mixing: waves arranged kMixWM x kMixWN, each 32 * kMixMT rows x 32 * kMixNT columns.
constexpr int kMixMT = 2, kMixNT = 4, kMixWM = 4, kMixWN = 2;
constexpr int kMixBM = 32 * kMixMT * kMixWM;
constexpr int kMixBN = 32 * kMixNT * kMixWN;

// Device-side description of one slice of a bank.
struct SliceDev {
  int rate = 0, dec = 1, level = 0;
  int64_t start_tap = 0;   // J_s (full rate)
  int n_taps = 0, n_basis = 0;
  int lp = 0;              // n_basis rounded up to kLPad (columns in the concatenated K)
  int lrows = 0;           // n_basis rounded up to kRowTile (rows of the FIR GEMM)
  int np = 0;              // n_taps rounded up to kBK
  int koff = 0;            // first column of this slice in the concatenated K
  float basis_scale = 1;   // power of two applied to the basis before rounding
  void *basis = nullptr;   // [lrows][np] compute type, taps reversed, zero padded
};

struct Workspace {
  void *base = nullptr;
  size_t bytes = 0;
};

// ---- descriptor tables: one launch per stage covers every job of a batch ----
// Work items of all jobs are numbered consecutively; job j owns items
// [item0_j, item0_{j+1}).  Jobs are laid out longest item first.

// FIR of one slice of one bank over output columns [k_lo, k_hi) at the slice rate.
struct FirJob {
  const void *basis;     // [rows][np] compute type, taps reversed
  const float *x;        // decimated strain of the slice's level, absolute index x_lo at x[0]
  void *out;             // column k goes to out[(k - out_lo) * ldo + col0 + l]
  int64_t x_lo, x_len, base, k_lo, k_hi, out_lo, item0;
  int rows, np, ldo, col0, col_limit, n_rtiles, n_ctiles, out_f32;
  int out_cm;            // channel-major output: out[l * ldo + (k - out_lo)]
  int pad;
};

// Interpolation of channel-major rows by R = 2 or 4 (one or two half-band x2
// stages as one composite filter) on MFMA: outputs n in [n_lo, n_hi) of the
// finer rate, computed in 32-sample tiles aligned to multiples of 32.  The
// source and a channel-major destination hold the low-rate buffer type
// (low_esz); a time-major destination is the mixing operand.
struct UpJob {
  const void *hf;        // MFMA fragments of the composite filter h_r (see interp_fragments)
  const void *src;       // channel-major [channels][ld_src], absolute column src_lo at column 0
  void *dst;             // dst_tm: dst[(n - dst_abs0) * ld_dst + col0 + c]; else dst[c * ld_dst + n - dst_abs0]
  int64_t src_lo, dst_abs0, n_lo, n_hi, n_first, item0;   // n_first: first tile start (multiple of 32)
  int64_t src_bytes;     // extent of src for the buffer resource
  int ld_src, ld_dst, col0, channels, r, dst_tm, n_ctiles, n_rtiles;
};

// Mixing + peaks of one bank over trigger windows [w0, w0 + nw).
struct MixJob {
  const void *mix;       // [rows][kld] compute type (columns past kcat are zeros)
  const void *ocat;      // [..][kld] compute type, absolute sample ocat_abs0 at row 0;
                         // columns past kcat are never read
  float *peak_snr;       // [F][ld_peak], column w - w_base
  int64_t *peak_n;
  float *peak_phase;
  float *peak_dt, *peak_si;   // sub-sample peak offset and value (triggers only)
  float *peak_xi;             // signal-consistency value (triggers only; banks with lags)
  float2 *peak_z;             // z at the peak (scaled), written with the phase; banks with lags
  const float *acorr;         // [n_templates][2 acorr_half + 1] (re, im) autocorrelation, or NULL
  float *snr;            // optional [F][snr_ld][2], column n - snr_abs0
  int64_t ocat_abs0, n_end, w0, nw, win_p, win_q, ld_peak, w_base, snr_ld, snr_abs0, item0, e0;
  int64_t x0;                 // first (job, window) item of this job in the signal-consistency launches
  int64_t ocat_end;           // absolute sample past the operand's last row
  int64_t *xi_key;            // listing slab [ld_peak][n_templates] of trigger keys (banks with lags)
  float inv_scale;
  int rows, kcat, n_templates, n_rtiles, acorr_half;
  int kld;                    // row pitch of mix and ocat (kcat rounded up to 64)
};

// One unit of the signal-consistency tiles: triggers first .. first + n - 1
// (n <= 64) of the listing of (job, window) item `item`.
struct XiUnit {
  int64_t item;
  int32_t first, n;
};

// Device scratch of the signal-consistency launches: the unit list and two
// counters (units listed, units taken).
struct XiWork {
  XiUnit *units = nullptr;
  int64_t cap = 0;
  int32_t *counters = nullptr;
};

// Trigger compaction over the peak table of one bank, windows [w_base, w_base + nw):
// dense [n_templates][nw] tables whose entries are numbered elem0, elem0 + 1, ...
// in the flat order of the batch.
struct TrigJob {
  const float *snr;
  const int64_t *peak_n;
  const float *phase, *dt, *si;
  const float *xi;                 // NULL: the bank computes no signal-consistency value
  int64_t w_base, nw, elem0;
  int n_templates, bank_id, detector, pad;
};

// Entries per trigger-compaction block, and the per-block count slots that
// n_elems entries need (the scan also keeps the total after them).
constexpr int kTrigPerBlock = 1024;
inline int64_t trig_blocks(int64_t n_elems) { return (n_elems + kTrigPerBlock - 1) / kTrigPerBlock; }

}  // namespace lloid

struct lloid_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  float *d_halfband = nullptr;  // device copy of g[n] (kHalfTaps floats)
  void *d_hfrag[3][2] = {};     // composite interpolation filters as MFMA fragments,
                                // [F32, F16, BF16 hi/lo split][R = 2, 4], in one
                                // allocation at d_hfrag[0][0]
  double halfband[lloid::kHalfTaps];
  int n_cu = 0;
  lloid::Workspace ws;          // grow-only device scratch of filter calls on this context
  void *static_scratch = nullptr;  // this device's static scratch array (lloid_filter_noalloc)
  void *pinned = nullptr;       // pinned host staging for descriptor tables
  size_t pinned_bytes = 0;
  int64_t chunk_budget = int64_t(6) << 30;  // device bytes of per-chunk operands
  int fir_variant = 0, mix_variant = 0;     // compiled tile shapes in use (lloid_ctx_set_tiles, lloid_autotune)
  bool profile = false;
  hipEvent_t ev[2 * LLOID_N_STAGES] = {};
  std::vector<hipEvent_t> cev;  // per chunk: start/end of the FIR, interpolation, mixing and phase stages
  double stage_ms[LLOID_N_STAGES] = {};
  int64_t stage_calls[LLOID_N_STAGES] = {};
};

struct lloid_bank {
  lloid_ctx *ctx = nullptr;
  int acorr_half = 0;       // K: lags of the signal-consistency value (0: none)
  float *acorr = nullptr;   // [n_templates][2K + 1] (re, im)
  int f0 = 0, n_templates = 0, n_levels = 1;
  lloid_dtype compute = LLOID_F16;
  std::vector<lloid::SliceDev> slices;
  int kcat = 0;             // concatenated K (multiple of kBK)
  int kld = 0;              // row pitch of mix and of the operand: kcat rounded up
                            // to 64 elements, so that operand rows start on 128-byte
                            // lines for 16-bit types
  int rows = 0;             // 2F rounded up to the mixing row tile
  float mix_scale = 1;      // power of two applied to the mixing matrix
  void *mix = nullptr;      // [rows][kld] compute type, zeros past kcat
  std::vector<double> sigma2;
  int64_t device_bytes = 0;
};

namespace lloid {

// ---- launch wrappers (lloid_kernels.hip) ----
hipError_t launch_convert(const void *src, lloid_dtype dt, int64_t n, float *dst, int64_t dst_lo,
                          int64_t dst_len, float scale, int *bad, hipStream_t s);
hipError_t launch_decimate(const float *u, int64_t u_lo, int64_t u_len, float *d, int64_t d_lo,
                           int64_t d_len, const float *g, hipStream_t s);
// Compiled tile-shape variants of the FIR and mixing kernels (0 = default);
// every variant gives bit-identical results (each output's K sum runs in the
// same order), only the speed differs.  Rows x columns per workgroup:
constexpr int kFirVariants = LLOID_FIR_VARIANTS, kMixVariants = LLOID_MIX_VARIANTS;
void fir_tile_shape(lloid_dtype t, int variant, int *bm, int *bn);
void mix_tile_shape(lloid_dtype t, int variant, int *bm, int *bn);
// One launch per stage over a device descriptor table (see the job structs).
hipError_t launch_fir_jobs(lloid_dtype t, int variant, const FirJob *jobs, int n_jobs, int64_t n_items,
                           hipStream_t s);
hipError_t launch_up_jobs(lloid_dtype t, const UpJob *jobs, int n_jobs, int64_t n_items, hipStream_t s);
// Work items of an interpolation job: four 32-channel x kUpCols-sample wave tasks each.
// Mixing and window peaks; then the phase at peaks with |z| >= phase_thr (0 for the others).
hipError_t launch_mix_jobs(lloid_dtype t, int variant, const MixJob *jobs, int n_jobs, int64_t n_items,
                           bool with_snr, hipStream_t s);
// White noise of unit variance (a counter-based hash of the sample index and
// seed, uniform on [-sqrt 3, sqrt 3]): synthetic strain for tuning runs.
hipError_t launch_noise(float *x, int64_t n, uint32_t seed, hipStream_t s);
hipError_t launch_peak_phase(lloid_dtype t, const MixJob *jobs, int n_jobs, int64_t n_entries, float phase_thr,
                             hipStream_t s);
// Signal-consistency value at the peaks with |z| >= thr of the jobs that carry
// autocorrelations; one workgroup per (job, window).
// n_windows: (job, window) items; kmax: largest kcat of a job with lags;
// acorr_max: largest n_templates * (2 acorr_half + 1) of those jobs;
// xw.cap >= sum over those jobs of nw * ceil(n_templates / 64)
hipError_t launch_xi2(lloid_dtype t, const MixJob *jobs, int n_jobs, int64_t n_windows, int kmax, int64_t acorr_max,
                      float thr, const XiWork &xw, int n_cu, hipStream_t s);
// Trigger compaction: counts, offsets and records (job-major, template, window);
// counts holds trig_blocks(n_elems) slots.
hipError_t launch_trigger_jobs(const TrigJob *jobs, int n_jobs, int64_t n_elems, float thr, int64_t *counts,
                               int64_t *total, int64_t cap, lloid_trigger *out, hipStream_t s);
// Conditioning of one block (float strain x[T]): PSD estimate into psd (when
// estimate; else psd holds the caller's), gain, whitened segments y, overlap-
// add into xw (or straight into out without gating), gating into out with
// the gated-sample count added to *count (mask zeroed by the caller).
constexpr int kCondMinLen = 64, kCondMaxLen = 4096;
hipError_t launch_condition(const float *x, int64_t T, int L, bool estimate, float f0, float *parts,
                            float *psd, float *gain, float *y, float *xw, float gate_thr, int gate_half,
                            uint8_t *mask, float *out, unsigned long long *count, hipStream_t s);
// Coincidences of two sorted trigger lists: per-trigger counts (na slots),
// their scan, pairs at the scanned offsets; *bad set when a list is out of order.
hipError_t launch_coincide(const lloid_trigger *a, int64_t na, const lloid_trigger *b, int64_t nb, int64_t max_dt,
                           int64_t *counts, int64_t *total, int *bad, int64_t cap, lloid_coinc *out, uint8_t *bg_a,
                           uint8_t *bg_b, hipStream_t s);
hipError_t launch_sigma2(const double *mix64, int n_templates, int lsum, const double *inv_dec_per_col,
                         double *out, hipStream_t s);
hipError_t launch_fill_u8(void *p, size_t bytes, hipStream_t s);
// ---- shared host helpers (lloid_host.cpp) ----
lloid_status fail(lloid_status st, const char *fmt, ...);


inline size_t dtype_size(lloid_dtype t) {
  switch (t) {
    case LLOID_F64: return 8;
    case LLOID_F32: return 4;
    case LLOID_F16: return 2;
    case LLOID_BF16: return 2;
  }
  return 0;
}

// Element size of the channel-major low-rate buffers (FIR outputs and
// intermediate interpolation hops): BF16 operands keep these in FP32, since
// two more roundings to an 8-bit significand would double the SNR error.
inline size_t low_esz(lloid_dtype t) { return t == LLOID_BF16 ? 4 : dtype_size(t); }

inline bool is_device_ptr(const void *p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// Address at which kernels can write the caller's buffer p: p itself for
// device memory, the device alias of pinned host memory, NULL for pageable
// host memory.
inline void *device_address(void *p) {
  hipPointerAttribute_t attr;
  if (!p || hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged) return p;
  if (attr.type == hipMemoryTypeHost && attr.devicePointer) return attr.devicePointer;
  return nullptr;
}


struct Carve {
  char *base;
  size_t off = 0;
  template <typename T> T *take(size_t count) {
    off = (size_t)round_up((int64_t)off, 256);
    T *r = (T *)(base + off);
    off += count * sizeof(T);
    return r;
  }
};

struct LevelView {
  const float *x;
  int64_t lo, len;
};

// Per (bank, detector) buffers of one chunk of windows.
struct BankBufs {
  void *ocat = nullptr;            // [chunk samples][kld]
  std::vector<std::vector<void *>> low;  // per slice at level > 0: FIR output, then each
                                         // interpolation hop's output except the last
  float *psnr = nullptr, *pphase = nullptr, *pdt = nullptr, *psi = nullptr, *pxi = nullptr;
  float2 *pz = nullptr;            // z at each peak, for the signal-consistency value
  int64_t *pkey = nullptr;         // trigger listing slab [ld_peak][F] (banks with lags)
  int64_t *pn = nullptr;
  int64_t ld_peak = 0, w_base = 0; // peak tables [F][ld_peak], column w - w_base
};

struct TileShapes {
  int fbm, fbn, mbm, mbn;
  TileShapes(lloid_dtype t, int fir_variant, int mix_variant) {
    fir_tile_shape(t, fir_variant, &fbm, &fbn);
    mix_tile_shape(t, mix_variant, &mbm, &mbn);
  }
};


struct StageItems {
  int64_t fir = 0, mix = 0, entries = 0;
  int64_t windows = 0;             // (job, window) pairs: workgroups of the signal-consistency launch
  bool xi2 = false;                // some mixing job carries autocorrelations
  int xi_kmax = 0;                 // largest kcat of such a job
  int64_t xi_acorr = 0;            // largest autocorrelation table of such a job (entries)
  int64_t xi_units = 0;            // signal-consistency units those jobs can list at most
  int64_t up[kMaxHops] = {};       // items of each interpolation hop
};

struct TabOffsets {
  size_t fir = 0, mix = 0, up[kMaxHops] = {};
  int n_fir = 0, n_mix = 0, n_up[kMaxHops] = {};
};

lloid_status ensure_ws(lloid_ctx *ctx, Workspace &ws, size_t bytes);
lloid_status ensure_pinned(lloid_ctx *ctx, void *&p, size_t &have, size_t bytes);
// Buffer resources address 32-bit byte offsets: a resource over the operand
// spans one trigger window plus its margins, and stays below kMaxBuffer bytes
// (the operand of a chunk itself is addressed with 64-bit pointers); the
// low-rate buffers of a chunk stay below kMaxBuffer bytes, level buffers below
// 2^30 bytes.
constexpr int64_t kMaxBuffer = (int64_t(1) << 31) - (int64_t(1) << 24);
constexpr int64_t kMaxBlock = int64_t(1) << 28;   // samples of one filter call
// t_len: operand rows of the chunk; win_len: samples of one trigger window
bool operands_fit(const lloid_bank *b, int64_t t_len, int64_t win_len);
// Composite interpolation filter of log2(R) cascaded half-band x2 stages
// (h_2[t] = 2 g[t], h_2R[t] = sum_m 2 g[m] h_R[t - R m]) laid out as MFMA B
// fragments: entry (ks, lane, j) holds h_R[lane % 32 - R kk + 32 R - 32] with
// kk = ks * KS + (lane / 32) * VEC + j.
void interp_fragments(const double *g, int R, int ks_elems, int vec, std::vector<double> &out);
// Entries of one fragment table (64 composite taps x 32 output samples); the
// BF16 split table holds the hi entries, then the lo entries.
constexpr int kInterpFragEntries = 2048;
// Append the FIR, interpolation and mixing jobs of bank b for output samples
// [t0, t1) (windows [wa, wb), data ending at n_end) to the tables.
void add_bank_jobs(const lloid_bank *b, const LevelView *lv, int64_t t0, int64_t t1, int64_t n_end, int64_t wa,
                   int64_t wb, const Windows &win, const BankBufs &bb, float inv_scale, float *snr, int64_t snr_ld,
                   const TileShapes &ts, std::vector<FirJob> &fj, std::vector<UpJob> *uj,
                   std::vector<MixJob> &mj);
// Sort longest-first and number the work items.
void number_jobs(std::vector<FirJob> &fj, std::vector<UpJob> *uj, std::vector<MixJob> &mj, StageItems &n);
// FIR, interpolation, mixing and phase launches over uploaded tables; ev:
// NULL, or 8 events bracketing those four stages.
constexpr int kChunkStages = 4;    // LLOID_STAGE_FIR .. LLOID_STAGE_PHASE
lloid_status launch_stages(lloid_ctx *ctx, lloid_dtype ct, const char *dtab, const TabOffsets &to,
                           const StageItems &n, bool with_snr, float phase_thr, float trig_thr, const XiWork &xw,
                           hipEvent_t *ev);
// Signal-consistency units that nw windows of a bank of F templates can list at most.
inline int64_t xi_unit_cap(int64_t nw, int F) { return nw * ceil_div(F, 64); }

// Samples of the mixing operand beyond each end of a chunk's outputs: one for
// the sub-sample refinement, K for the signal-consistency lags.
inline int64_t operand_margin(const lloid_bank *b) { return std::max(1, b->acorr_half); }

}  // namespace lloid

#define HIP_TRY(expr)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return lloid::fail(LLOID_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),     \
                         __FILE__, __LINE__);                                                      \
  } while (0)

#define ABI_GUARD_BEGIN try {
#define ABI_GUARD_END                                                     \
  }                                                                       \
  catch (const std::bad_alloc &) {                                        \
    return lloid::fail(LLOID_ENOMEM, "host allocation failed");           \
  }                                                                       \
  catch (const std::exception &ex) {                                      \
    return lloid::fail(LLOID_EINVAL, "internal error: %s", ex.what());    \
  }
