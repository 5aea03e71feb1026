// Internal interfaces between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lloid.h"

namespace lloid {

// Half-band resampler: g[n], |n| <= kHalfQ, zero at even n != 0.
constexpr int kHalfQ = 32;
constexpr int kHalfTaps = 2 * kHalfQ + 1;

// GEMM tiling shared by the FIR and the mixing kernels (wave64, 4 waves).
constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kBK = 32;          // K chunk staged in LDS
constexpr int kLPad = 16;        // basis count padding inside the concatenated K
constexpr int kRowTile = 32;     // MFMA 32x32 tile

// Tile shapes: rows per workgroup = 32 * MT, columns = 4 waves * 32 * NT.
constexpr int kFirMT = 2, kFirNT = 4;
constexpr int kMixMT = 2, kMixNT = 4;
constexpr int kFirBN = kWaves * 32 * kFirNT;
constexpr int kMixBN = kWaves * 32 * kMixNT;

struct Range {
  int64_t lo = 0, hi = 0;  // absolute indices [lo, hi)
  int64_t size() const { return hi > lo ? hi - lo : 0; }
};

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

}  // namespace lloid

struct lloid_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  float *d_halfband = nullptr;  // device copy of g[n] (kHalfTaps floats)
  double halfband[lloid::kHalfTaps];
  int n_cu = 0;
  bool profile = false;
  hipEvent_t ev[2 * LLOID_N_STAGES] = {};
  double stage_ms[LLOID_N_STAGES] = {};
  int64_t stage_calls[LLOID_N_STAGES] = {};
};

struct lloid_bank {
  lloid_ctx *ctx = nullptr;
  int f0 = 0, n_templates = 0, n_levels = 1;
  lloid_dtype compute = LLOID_F16;
  std::vector<lloid::SliceDev> slices;
  int kcat = 0;             // concatenated K (multiple of kBK)
  int rows = 0;             // 2F rounded up to the mixing row tile
  float mix_scale = 1;      // power of two applied to the mixing matrix
  void *mix = nullptr;      // [rows][kcat] compute type
  std::vector<double> sigma2;
  int64_t device_bytes = 0;
  lloid::Workspace ws;      // grow-only scratch reused by lloid_filter
};

namespace lloid {

// ---- launch wrappers (lloid_kernels.hip) ----
hipError_t launch_convert(const void *src, lloid_dtype dt, int64_t n, float *dst, int64_t dst_lo,
                          int64_t dst_len, float scale, int *bad, hipStream_t s);
hipError_t launch_decimate(const float *u, int64_t u_lo, int64_t u_len, float *d, int64_t d_lo,
                           int64_t d_len, const float *g, hipStream_t s);
// FIR: out[(k - out_lo) * ldo + col0 + l] = scale-free sum over taps, for k in [k_lo, k_hi).
hipError_t launch_fir(lloid_dtype t, const SliceDev &sl, const float *x, int64_t x_lo, int64_t x_len,
                      int64_t k_lo, int64_t k_hi, void *out, int64_t out_lo, int ldo, int col0,
                      int col_limit, hipStream_t s);
// One x2 interpolation stage: v[n] = sum_j w[j] 2 g[n - 2j] for n in [v_lo, v_lo + v_len);
// w is [w_len][ldw] (fp32 or compute type), v is [v_len][ldv] (fp32 or compute type).
hipError_t launch_interp(lloid_dtype in_t, const void *w, int64_t w_lo, int64_t w_len, int ldw,
                         lloid_dtype out_t, void *v, int64_t v_lo, int64_t v_len, int ldv, int col0,
                         int channels, const float *g, hipStream_t s);
// Mixing GEMM over the concatenated basis with the fused per-window peak epilogue.
struct PeakArgs {
  float *peak_snr;      // [F][n_windows]
  int64_t *peak_n;      // [F][n_windows]
  float *peak_phase;    // [F][n_windows]
  float *snr;           // optional [F][n][2]
  int64_t n_windows, win_p, win_q;  // window w starts at floor(w * win_p / win_q)
};
hipError_t launch_mix_peak(lloid_dtype t, const void *mix, int rows, int kcat, int n_templates,
                           const void *ocat, int64_t n, float inv_scale, const PeakArgs &pa,
                           hipStream_t s);
hipError_t launch_sigma2(const double *mix64, int n_templates, int lsum, const double *inv_dec_per_col,
                         double *out, hipStream_t s);
hipError_t launch_fill_u8(void *p, size_t bytes, hipStream_t s);
// Trigger compaction: counts, offsets and records (template-major, window-minor).
hipError_t launch_trigger_count(const float *peak_snr, int n_templates, int64_t n_windows, float thr,
                                int64_t *counts, hipStream_t s);
hipError_t launch_trigger_scan(int64_t *counts, int n_templates, int64_t *total, hipStream_t s);
hipError_t launch_trigger_write(const float *peak_snr, const int64_t *peak_n, const float *peak_phase,
                                int n_templates, int64_t n_windows, float thr, const int64_t *offsets,
                                int64_t cap, int32_t bank_id, int32_t detector, lloid_trigger *out,
                                hipStream_t s);

}  // namespace lloid
