// Host runtime and C ABI of the LLOID filtering library (see include/lloid.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lloid_internal.h"

using namespace lloid;

// ------------------------------------------------------------ error state

static thread_local std::string g_last_error;

lloid_status lloid::fail(lloid_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

extern "C" const char *lloid_last_error(void) { return g_last_error.c_str(); }
extern "C" const char *lloid_version(void) { return "lloid-gfx950 0.1"; }

// ------------------------------------------------------------ helpers

static bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
static int log2i(int64_t v) {
  int k = 0;
  while ((int64_t(1) << k) < v) ++k;
  return k;
}

// Modified Bessel function I0 by its power series sum_k ((x/2)^k / k!)^2.
static double bessel_i0(double x) {
  double term = 1.0, sum = 1.0, q = 0.25 * x * x;
  for (int k = 1; k < 200; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return sum;
}

// g[n] = 1/2 sinc(n/2) I0(beta sqrt(1 - (n/Q)^2)) / I0(beta), |n| <= Q, beta = 10.
static void halfband(double *g) {
  const double beta = 10.0, i0b = bessel_i0(beta);
  for (int n = -kHalfQ; n <= kHalfQ; ++n) {
    double s;
    if (n == 0) s = 1.0;
    else if (n % 2 == 0) s = 0.0;
    else s = std::sin(M_PI * n / 2.0) / (M_PI * n / 2.0);
    double r = (double)n / kHalfQ;
    g[n + kHalfQ] = 0.5 * s * bessel_i0(beta * std::sqrt(std::max(0.0, 1.0 - r * r))) / i0b;
  }
}

// Power of two p with max_abs * p in (1/2, 1].
static float pow2_scale(double max_abs) {
  if (!(max_abs > 0.0) || !std::isfinite(max_abs)) return 1.f;
  int e;
  std::frexp(max_abs, &e);  // max_abs = f 2^e, f in [1/2, 1)
  return (float)std::ldexp(1.0, -e);
}

// Device-side cast of an FP64 array to the compute type.
namespace lloid {
hipError_t launch_cast_f64(const double *src, lloid_dtype t, void *dst, int64_t n, hipStream_t s);
}

// ------------------------------------------------------------ static scratch
// Device memory of the allocation-free call (lloid_filter_noalloc): one array
// per GPU, part of the library's code object and held until the process ends.
// On the host this name is not a device address; host code only uses the
// address hipGetSymbolAddress returns with the device current, kept per device.
static __device__ __align__(256) unsigned char scratch[LLOID_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;   // indexed by device id
}  // namespace

// Address of `device`'s copy of the scratch array; the device must be current.
static lloid_status scratch_address(int device, void **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize((size_t)device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(LLOID_EDEVICE, "hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return LLOID_OK;
}

// ------------------------------------------------------------ context

extern "C" lloid_status lloid_ctx_create(int device, void *hip_stream, lloid_ctx **out) {
  ABI_GUARD_BEGIN
  if (!out) return fail(LLOID_EINVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return fail(LLOID_EDEVICE, "HIP device %d not available (%d visible)", device, count);
  HIP_TRY(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(LLOID_EDEVICE, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
  void *scr = nullptr;
  {
    const lloid_status r = scratch_address(device, &scr);
    if (r != LLOID_OK) return r;
  }
  lloid_ctx *c = new lloid_ctx();
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
  c->static_scratch = scr;
  // tile shapes: the defaults, or those named by LLOID_FIR_VARIANT / LLOID_MIX_VARIANT
  if (const char *v = getenv("LLOID_FIR_VARIANT")) c->fir_variant = std::min(std::max(atoi(v), 0), kFirVariants - 1);
  if (const char *v = getenv("LLOID_MIX_VARIANT")) c->mix_variant = std::min(std::max(atoi(v), 0), kMixVariants - 1);
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(LLOID_EDEVICE, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  halfband(c->halfband);
  float gf[kHalfTaps];
  for (int i = 0; i < kHalfTaps; ++i) gf[i] = (float)c->halfband[i];
  if (hipMalloc(&c->d_halfband, sizeof gf) != hipSuccess ||
      hipMemcpy(c->d_halfband, gf, sizeof gf, hipMemcpyHostToDevice) != hipSuccess) {
    lloid_ctx_destroy(c);
    return fail(LLOID_EDEVICE, "cannot upload resampler taps");
  }
  // composite interpolation filters as MFMA fragments: FP32 32x32x2 (KS 2,
  // one value per lane; the FP32 operand path), FP16 32x32x16 (KS 16, eight
  // values per lane) and, for the BF16 operand path (whose low-rate buffers
  // are FP32), the 32x32x16 layout split into BF16 hi and lo tables;
  // kInterpFragEntries entries each, built in FP64
  {
    constexpr size_t kEnt = kInterpFragEntries, kSlot = kEnt * 4;
    const lloid_dtype types[2] = {LLOID_F32, LLOID_F16};
    char *mem = nullptr;
    double *tmp = nullptr;
    bool ok = hipMalloc((void **)&mem, 6 * kSlot) == hipSuccess && hipMalloc((void **)&tmp, kEnt * 8) == hipSuccess;
    std::vector<double> frag;
    for (int ti = 0; ti < 2 && ok; ++ti)
      for (int ri = 0; ri < 2 && ok; ++ri) {
        const bool f32 = types[ti] == LLOID_F32;
        interp_fragments(c->halfband, ri == 0 ? 2 : 4, f32 ? 2 : 16, f32 ? 1 : 8, frag);
        c->d_hfrag[ti][ri] = mem + (ti * 2 + ri) * kSlot;
        ok = frag.size() == kEnt &&
             hipMemcpy(tmp, frag.data(), kEnt * 8, hipMemcpyHostToDevice) == hipSuccess &&
             launch_cast_f64(tmp, types[ti], c->d_hfrag[ti][ri], (int64_t)kEnt, c->stream) == hipSuccess &&
             hipStreamSynchronize(c->stream) == hipSuccess;
      }
    // BF16 split tables: the hi halves, then the lo halves
    for (int ri = 0; ri < 2 && ok; ++ri) {
      interp_fragments(c->halfband, ri == 0 ? 2 : 4, 16, 8, frag);
      std::vector<uint16_t> split(2 * kEnt);
      for (size_t q = 0; q < kEnt && q < frag.size(); ++q) bf16_split((float)frag[q], &split[q], &split[kEnt + q]);
      c->d_hfrag[2][ri] = mem + (4 + ri) * kSlot;
      ok = frag.size() == kEnt &&
           hipMemcpy(c->d_hfrag[2][ri], split.data(), split.size() * 2, hipMemcpyHostToDevice) == hipSuccess;
    }
    if (tmp) (void)hipFree(tmp);
    if (!ok) {
      if (mem) (void)hipFree(mem);
      c->d_hfrag[0][0] = nullptr;
      lloid_ctx_destroy(c);
      return fail(LLOID_EDEVICE, "cannot build the interpolation filters");
    }
  }
  *out = c;
  return LLOID_OK;
  ABI_GUARD_END
}

extern "C" lloid_status lloid_ctx_profile(lloid_ctx *ctx, int enable) {
  if (!ctx) return fail(LLOID_EINVAL, "NULL context");
  HIP_TRY(hipSetDevice(ctx->device));
  if (enable && !ctx->ev[0])
    for (auto &e : ctx->ev) HIP_TRY(hipEventCreate(&e));
  ctx->profile = enable != 0;
  return LLOID_OK;
}

extern "C" lloid_status lloid_ctx_stage_times(lloid_ctx *ctx, double *ms, int64_t *calls, int reset) {
  if (!ctx) return fail(LLOID_EINVAL, "NULL context");
  for (int i = 0; i < LLOID_N_STAGES; ++i) {
    if (ms) ms[i] = ctx->stage_ms[i];
    if (calls) calls[i] = ctx->stage_calls[i];
    if (reset) ctx->stage_ms[i] = 0.0, ctx->stage_calls[i] = 0;
  }
  return LLOID_OK;
}

extern "C" lloid_status lloid_ctx_destroy(lloid_ctx *ctx) {
  if (!ctx) return LLOID_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (auto &e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : ctx->cev) (void)hipEventDestroy(e);
  if (ctx->ws.base) (void)hipFree(ctx->ws.base);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->d_halfband) (void)hipFree(ctx->d_halfband);
  if (ctx->d_hfrag[0][0]) (void)hipFree(ctx->d_hfrag[0][0]);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return LLOID_OK;
}

// ------------------------------------------------------------ bank

static void free_bank_device(lloid_bank *b) {
  for (auto &s : b->slices)
    if (s.basis) (void)hipFree(s.basis), s.basis = nullptr;
  if (b->mix) (void)hipFree(b->mix), b->mix = nullptr;
  if (b->acorr) (void)hipFree(b->acorr), b->acorr = nullptr;
}

extern "C" lloid_status lloid_bank_destroy(lloid_bank *bank) {
  if (!bank) return LLOID_OK;
  (void)hipSetDevice(bank->ctx->device);
  (void)hipStreamSynchronize(bank->ctx->stream);
  free_bank_device(bank);
  delete bank;
  return LLOID_OK;
}

extern "C" lloid_status lloid_bank_create(lloid_ctx *ctx, const lloid_bank_desc *d, lloid_bank **out) {
  ABI_GUARD_BEGIN
  if (!ctx || !d || !out) return fail(LLOID_EINVAL, "NULL argument");
  *out = nullptr;
  if (d->full_rate_hz <= 0) return fail(LLOID_EINVAL, "full_rate_hz must be positive");
  if (d->n_templates <= 0) return fail(LLOID_EINVAL, "n_templates must be positive");
  if (d->n_slices <= 0 || !d->slices) return fail(LLOID_EINVAL, "a bank needs at least one slice");
  if (d->compute != LLOID_F32 && d->compute != LLOID_F16 && d->compute != LLOID_BF16)
    return fail(LLOID_EINVAL, "compute type must be F32, F16 or BF16");
  const int f0 = d->full_rate_hz, F = d->n_templates;
  for (int s = 0; s < d->n_slices; ++s) {
    const lloid_slice &sl = d->slices[s];
    if (sl.rate_hz <= 0 || f0 % sl.rate_hz || !is_pow2(f0 / sl.rate_hz))
      return fail(LLOID_EINVAL, "slice %d: rate %d Hz is not f0 / 2^k (f0 = %d)", s, sl.rate_hz, f0);
    const int dec = f0 / sl.rate_hz;
    if (dec > (1 << kMaxLevel))
      return fail(LLOID_EINVAL, "slice %d: rate %d Hz is below f0 / %d", s, sl.rate_hz, 1 << kMaxLevel);
    if (sl.start_tap < 0 || sl.start_tap % dec)
      return fail(LLOID_EINVAL, "slice %d: start tap %lld is not a non-negative multiple of %d", s,
                  (long long)sl.start_tap, dec);
    if (sl.n_taps <= 0) return fail(LLOID_EINVAL, "slice %d: n_taps must be positive", s);
    if (sl.n_basis <= 0 || sl.n_basis > sl.n_taps)
      return fail(LLOID_EINVAL, "slice %d: n_basis %d must be in [1, n_taps = %d]", s, sl.n_basis, sl.n_taps);
    if (!sl.basis || !sl.mixing) return fail(LLOID_EINVAL, "slice %d: NULL basis or mixing", s);
  }
  const int K = d->autocorr_half;
  if (K < 0 || K > kMaxAutocorrHalf)
    return fail(LLOID_EINVAL, "autocorr_half %d is outside [0, %d]", K, kMaxAutocorrHalf);
  if (K > 0 && !d->autocorr) return fail(LLOID_EINVAL, "NULL autocorr with autocorr_half %d", K);
  for (int64_t q = 0; K > 0 && q < (int64_t)F * (2 * K + 1) * 2; ++q)
    if (!std::isfinite(d->autocorr[q])) return fail(LLOID_EINVAL, "non-finite autocorrelation value");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;

  lloid_bank *b = new lloid_bank();
  b->ctx = ctx;
  b->f0 = f0;
  b->n_templates = F;
  b->compute = d->compute;
  b->rows = (int)round_up(2 * (int64_t)F, kMixBM);
  b->acorr_half = K;
  const size_t esz = dtype_size(d->compute);
  int koff = 0, lsum = 0;
  double max_mix = 0.0;
  for (int s = 0; s < d->n_slices; ++s) {
    const lloid_slice &in = d->slices[s];
    SliceDev sl;
    sl.rate = in.rate_hz;
    sl.dec = f0 / in.rate_hz;
    sl.level = log2i(sl.dec);
    sl.start_tap = in.start_tap;
    sl.n_taps = in.n_taps;
    sl.n_basis = in.n_basis;
    sl.lp = (int)round_up(in.n_basis, kLPad);
    sl.lrows = (int)round_up(in.n_basis, kRowTile);
    sl.np = (int)round_up(in.n_taps, kBK);
    lsum += in.n_basis;
    double mb = 0.0;
    for (int64_t i = 0; i < (int64_t)in.n_basis * in.n_taps; ++i) mb = std::max(mb, std::fabs(in.basis[i]));
    sl.basis_scale = pow2_scale(mb);
    for (int64_t i = 0; i < 2 * (int64_t)F * in.n_basis; ++i)
      max_mix = std::max(max_mix, std::fabs(in.mixing[i]) / sl.basis_scale);
    b->n_levels = std::max(b->n_levels, sl.level + 1);
    b->slices.push_back(sl);
  }
  // Column order of the concatenated K: the lower-rate slices first, then
  // the full-rate ones, so that the interpolation stage writes one run at the
  // start of every operand row and shares fewer 128-byte lines with the
  // FIR's columns (partly written lines slow its stores: 1.95 -> 2.77 TB/s
  // measured for the 1024-template bank's layout).  The slice last in that
  // order absorbs the padding of the concatenated K, so every column of the
  // operand is written by a FIR or an interpolation stage.
  std::vector<int> korder;
  for (int s = 0; s < d->n_slices; ++s)
    if (b->slices[s].level > 0) korder.push_back(s);
  for (int s = 0; s < d->n_slices; ++s)
    if (b->slices[s].level == 0) korder.push_back(s);
  for (int s : korder) {
    b->slices[s].koff = koff;
    koff += b->slices[s].lp;
  }
  b->kcat = (int)round_up(koff, kBK);
  b->kld = (int)round_up(b->kcat, 64);
  b->slices[korder.back()].lp += b->kcat - koff;
  for (auto &sl : b->slices) sl.lrows = (int)round_up(sl.lp, kRowTile);
  b->mix_scale = pow2_scale(max_mix);

  // Pack on the host in FP64, cast on the device.
  lloid_status status = LLOID_OK;
  double *dtmp = nullptr;
  size_t tmp_elems = (size_t)b->rows * b->kld;
  for (auto &sl : b->slices) tmp_elems = std::max(tmp_elems, (size_t)sl.lrows * sl.np);
  tmp_elems = std::max(tmp_elems, (size_t)2 * F * lsum + lsum + F);
  if (hipMalloc(&dtmp, tmp_elems * sizeof(double)) != hipSuccess) {
    delete b;
    return fail(LLOID_ENOMEM, "device allocation of %zu bytes failed", tmp_elems * sizeof(double));
  }
  std::vector<double> host;
  auto cleanup = [&](lloid_status stc) {
    (void)hipFree(dtmp);
    if (stc != LLOID_OK) {
      free_bank_device(b);
      delete b;
    }
    return stc;
  };
  for (int s = 0; s < d->n_slices && status == LLOID_OK; ++s) {
    const lloid_slice &in = d->slices[s];
    SliceDev &sl = b->slices[s];
    host.assign((size_t)sl.lrows * sl.np, 0.0);
    for (int l = 0; l < in.n_basis; ++l)
      for (int m = 0; m < in.n_taps; ++m)
        host[(size_t)l * sl.np + m] = in.basis[(size_t)l * in.n_taps + (in.n_taps - 1 - m)] * sl.basis_scale;
    if (hipMalloc(&sl.basis, host.size() * esz) != hipSuccess) return cleanup(fail(LLOID_ENOMEM, "basis alloc"));
    b->device_bytes += (int64_t)(host.size() * esz);
    if (hipMemcpyAsync(dtmp, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
        launch_cast_f64(dtmp, b->compute, sl.basis, (int64_t)host.size(), st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return cleanup(fail(LLOID_EDEVICE, "basis upload failed"));
  }
  host.assign((size_t)b->rows * b->kld, 0.0);
  for (int s = 0; s < d->n_slices; ++s) {
    const lloid_slice &in = d->slices[s];
    const SliceDev &sl = b->slices[s];
    const double f = b->mix_scale / sl.basis_scale;
    for (int r = 0; r < 2 * F; ++r)
      for (int l = 0; l < in.n_basis; ++l)
        host[(size_t)r * b->kld + sl.koff + l] = in.mixing[(size_t)r * in.n_basis + l] * f;
  }
  if (hipMalloc(&b->mix, host.size() * esz) != hipSuccess) return cleanup(fail(LLOID_ENOMEM, "mixing alloc"));
  b->device_bytes += (int64_t)(host.size() * esz);
  if (hipMemcpyAsync(dtmp, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
      launch_cast_f64(dtmp, b->compute, b->mix, (int64_t)host.size(), st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return cleanup(fail(LLOID_EDEVICE, "mixing upload failed"));

  // autocorrelations as FP32 (re, im) pairs, [F][2K + 1]
  if (K > 0) {
    const size_t na = (size_t)F * (2 * K + 1) * 2;
    std::vector<float> fa(na);
    for (size_t q = 0; q < na; ++q) fa[q] = (float)d->autocorr[q];
    if (hipMalloc(&b->acorr, na * sizeof(float)) != hipSuccess) return cleanup(fail(LLOID_ENOMEM, "autocorr alloc"));
    b->device_bytes += (int64_t)(na * sizeof(float));
    if (hipMemcpyAsync(b->acorr, fa.data(), na * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return cleanup(fail(LLOID_EDEVICE, "autocorr upload failed"));
  }

  // sigma^2 in FP64 from the unscaled mixing matrices
  host.assign((size_t)2 * F * lsum + lsum, 0.0);
  int c0 = 0;
  for (int s = 0; s < d->n_slices; ++s) {
    const lloid_slice &in = d->slices[s];
    for (int r = 0; r < 2 * F; ++r)
      for (int l = 0; l < in.n_basis; ++l) host[(size_t)r * lsum + c0 + l] = in.mixing[(size_t)r * in.n_basis + l];
    for (int l = 0; l < in.n_basis; ++l) host[(size_t)2 * F * lsum + c0 + l] = 1.0 / (f0 / in.rate_hz);
    c0 += in.n_basis;
  }
  double *d_m = dtmp, *d_inv = dtmp + (size_t)2 * F * lsum, *d_out = d_inv + lsum;
  b->sigma2.assign(F, 0.0);
  if (hipMemcpyAsync(dtmp, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
      launch_sigma2(d_m, F, lsum, d_inv, d_out, st) != hipSuccess ||
      hipMemcpyAsync(b->sigma2.data(), d_out, F * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return cleanup(fail(LLOID_EDEVICE, "sigma2 failed"));
  cleanup(LLOID_OK);
  *out = b;
  return LLOID_OK;
  ABI_GUARD_END
}

extern "C" lloid_status lloid_bank_sigma2(const lloid_bank *bank, double *out) {
  if (!bank || !out) return fail(LLOID_EINVAL, "NULL argument");
  std::memcpy(out, bank->sigma2.data(), bank->sigma2.size() * sizeof(double));
  return LLOID_OK;
}

extern "C" lloid_status lloid_bank_query(const lloid_bank *bank, lloid_bank_info *out) {
  if (!bank || !out) return fail(LLOID_EINVAL, "NULL argument");
  out->full_rate_hz = bank->f0;
  out->n_templates = bank->n_templates;
  out->n_slices = (int32_t)bank->slices.size();
  out->n_levels = bank->n_levels;
  out->compute = bank->compute;
  out->concat_k = bank->kcat;
  out->device_bytes = bank->device_bytes;
  return LLOID_OK;
}

// ------------------------------------------------------------ filter engine

lloid_status lloid::ensure_ws(lloid_ctx *ctx, Workspace &ws, size_t bytes) {
  if (ws.bytes >= bytes) return LLOID_OK;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (ws.base) (void)hipFree(ws.base);
  ws.base = nullptr;
  ws.bytes = 0;
  if (hipMalloc(&ws.base, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LLOID_ENOMEM, "workspace of %zu bytes does not fit on the device", bytes);
  }
  ws.bytes = bytes;
  return LLOID_OK;
}

lloid_status lloid::ensure_pinned(lloid_ctx *ctx, void *&p, size_t &have, size_t bytes) {
  if (have >= bytes) return LLOID_OK;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (p) (void)hipHostFree(p);
  p = nullptr;
  have = 0;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LLOID_ENOMEM, "pinned staging of %zu bytes failed", bytes);
  }
  have = bytes;
  return LLOID_OK;
}

bool lloid::operands_fit(const lloid_bank *b, int64_t t_len, int64_t win_len) {
  // a resource over the operand spans at most one window and its margins
  const int64_t span = std::min(t_len, win_len + 2 * operand_margin(b));
  if (span * b->kld * (int64_t)dtype_size(b->compute) > kMaxBuffer) return false;
  for (const auto &sl : b->slices)
    if (sl.level > 0)
      for (int64_t ld : low_ld(t_len, sl.level))
        if ((int64_t)sl.lp * ld * (int64_t)low_esz(b->compute) > kMaxBuffer) return false;
  return true;
}

void lloid::interp_fragments(const double *g, int R, int ks_elems, int vec, std::vector<double> &out) {
  // h_R on |t| <= 32 (R - 1), built by the recursion h_2R[t] = sum_m 2 g[m] h_R[t - R m]
  std::vector<double> h(2 * kHalfQ + 1);
  int half = kHalfQ;
  for (int t = -kHalfQ; t <= kHalfQ; ++t) h[t + kHalfQ] = 2.0 * g[t + kHalfQ];
  for (int r = 2; r < R; r *= 2) {
    const int nh = kHalfQ * (2 * r - 1);
    std::vector<double> h2(2 * nh + 1, 0.0);
    for (int m = -kHalfQ; m <= kHalfQ; ++m)
      for (int u = -half; u <= half; ++u) h2[r * m + u + nh] += 2.0 * g[m + kHalfQ] * h[u + half];
    h.swap(h2);
    half = nh;
  }
  const int nks = 64 / ks_elems;
  out.assign((size_t)nks * 64 * vec, 0.0);
  for (int ks = 0; ks < nks; ++ks)
    for (int lane = 0; lane < 64; ++lane)
      for (int j = 0; j < vec; ++j) {
        const int kk = ks * ks_elems + (lane / 32) * vec + j;
        const int t = lane % 32 - R * kk + 32 * R - 32;
        out[((size_t)ks * 64 + lane) * vec + j] = (t >= -half && t <= half) ? h[t + half] : 0.0;
      }
}

void lloid::add_bank_jobs(const lloid_bank *b, const LevelView *lv, int64_t t0, int64_t t1, int64_t n_end, int64_t wa,
                          int64_t wb, const Windows &win, const BankBufs &bb, float inv_scale, float *snr,
                          int64_t snr_ld, const TileShapes &ts, std::vector<FirJob> &fj, std::vector<UpJob> *uj,
                          std::vector<MixJob> &mj) {
  // the operand holds operand_margin(b) extra samples on each side: one for
  // the sub-sample refinement of peaks at the chunk's first and last samples,
  // K for the signal-consistency lags
  const int64_t mg = operand_margin(b);
  const int64_t e0 = t0 - mg, e1 = t1 + mg;
  const size_t lsz = low_esz(b->compute);
  // BF16 interpolates FP32 buffers with split-BF16 products
  const int ti = b->compute == LLOID_F16 ? 1 : b->compute == LLOID_BF16 ? 2 : 0;
  for (size_t s = 0; s < b->slices.size(); ++s) {
    const SliceDev &sl = b->slices[s];
    FirJob j{};
    j.basis = sl.basis;
    j.x = lv[sl.level].x;
    j.x_lo = lv[sl.level].lo;
    j.x_len = lv[sl.level].len;
    j.base = -(sl.start_tap / sl.dec + sl.n_taps - 1);
    j.rows = sl.lrows;
    j.np = sl.np;
    j.n_rtiles = (int)ceil_div(sl.lrows, ts.fbm);
    j.col_limit = sl.lp;
    if (sl.level == 0) {
      j.k_lo = e0;
      j.k_hi = e1;
      j.out = bb.ocat;
      j.out_lo = e0;
      j.ldo = b->kld;
      j.col0 = sl.koff;
    } else {
      // FIR at the slice rate into a channel-major buffer, then the hops up to f0
      const UpPlan p = up_plan(e0, e1, sl.level);
      const std::vector<int64_t> ld = low_ld(e1 - e0, sl.level);
      const int H = (int)p.r.size();
      j.k_lo = p.in[0].lo;
      j.k_hi = p.in[0].hi;
      j.out = bb.low[s][0];
      j.out_lo = p.in[0].lo;
      j.ldo = (int)ld[0];
      j.out_cm = 1;
      j.out_f32 = b->compute == LLOID_BF16;
      for (int h = 0; h < H; ++h) {
        UpJob q{};
        q.hf = b->ctx->d_hfrag[ti][p.r[h] == 2 ? 0 : 1];
        q.src = bb.low[s][h];
        q.src_lo = p.in[h].lo;
        q.ld_src = (int)ld[h];
        q.src_bytes = (int64_t)sl.lp * ld[h] * (int64_t)lsz;
        q.channels = sl.lp;
        q.r = p.r[h];
        q.n_lo = p.out[h].lo;
        q.n_hi = p.out[h].hi;
        q.n_first = floor_div(p.out[h].lo, 32) * 32;
        q.n_ctiles = (int)ceil_div(p.out[h].hi - q.n_first, kUpCols);
        q.n_rtiles = (int)ceil_div(sl.lp, 32);
        if (h + 1 == H) {
          q.dst = bb.ocat;
          q.dst_abs0 = e0;
          q.ld_dst = b->kld;
          q.col0 = sl.koff;
          q.dst_tm = 1;
        } else {
          q.dst = bb.low[s][h + 1];
          q.dst_abs0 = p.in[h + 1].lo;
          q.ld_dst = (int)ld[h + 1];
          q.dst_tm = 0;
        }
        uj[h].push_back(q);
      }
    }
    j.n_ctiles = (int)ceil_div(j.k_hi - j.k_lo, ts.fbn);
    fj.push_back(j);
  }
  MixJob m{};
  m.mix = b->mix;
  m.ocat = bb.ocat;
  m.peak_snr = bb.psnr;
  m.peak_n = bb.pn;
  m.peak_phase = bb.pphase;
  m.peak_dt = bb.pdt;
  m.peak_si = bb.psi;
  m.peak_xi = bb.pxi;
  m.peak_z = b->acorr ? bb.pz : nullptr;
  m.xi_key = b->acorr ? bb.pkey : nullptr;
  m.acorr = b->acorr;
  m.acorr_half = b->acorr_half;
  m.snr = snr;
  m.ocat_abs0 = e0;
  m.ocat_end = e1;
  m.snr_abs0 = t0;
  m.n_end = n_end;
  m.w0 = wa;
  m.nw = wb - wa;
  m.win_p = win.p;
  m.win_q = win.q;
  m.ld_peak = bb.ld_peak;
  m.w_base = bb.w_base;
  m.snr_ld = snr_ld;
  m.inv_scale = inv_scale;
  m.rows = b->rows;
  m.kcat = b->kcat;
  m.kld = b->kld;
  m.n_templates = b->n_templates;
  m.n_rtiles = (int)ceil_div(b->rows, ts.mbm);
  mj.push_back(m);
}

void lloid::number_jobs(std::vector<FirJob> &fj, std::vector<UpJob> *uj, std::vector<MixJob> &mj, StageItems &n) {
  // longest items first
  std::stable_sort(fj.begin(), fj.end(), [](const FirJob &a, const FirJob &b) { return a.np > b.np; });
  std::stable_sort(mj.begin(), mj.end(), [](const MixJob &a, const MixJob &b) { return a.kcat > b.kcat; });
  int64_t it = 0;
  for (auto &j : fj) j.item0 = it, it += (int64_t)j.n_rtiles * j.n_ctiles;
  n.fir = it;
  for (int h = 0; h < kMaxHops; ++h) {
    it = 0;
    // 8 runs (one per XCD) of ceil(tasks / 32) items of 4 tasks
    for (auto &q : uj[h]) q.item0 = it, it += 8 * ceil_div((int64_t)q.n_rtiles * q.n_ctiles, 32);
    n.up[h] = it;
  }
  it = 0;
  int64_t e = 0;
  for (auto &m : mj) {
    m.item0 = it;
    // windows in runs of 8 (one per XCD) per row tile; fewer than 8 windows
    // run window-major over the row tiles, padded to a multiple of 8
    it += m.nw >= 8 ? ceil_div(m.nw, 8) * 8 * m.n_rtiles : round_up(m.nw * m.n_rtiles, 8);
    m.e0 = e;
    e += (int64_t)m.n_templates * m.nw;
    m.x0 = n.windows;
    n.windows += m.nw;
    if (m.acorr) {
      n.xi2 = true;
      n.xi_kmax = std::max(n.xi_kmax, m.kcat);
      n.xi_acorr = std::max(n.xi_acorr, (int64_t)m.n_templates * (2 * m.acorr_half + 1));
      n.xi_units += xi_unit_cap(m.nw, m.n_templates);
    }
  }
  n.mix = it;
  n.entries = e;
}

lloid_status lloid::launch_stages(lloid_ctx *ctx, lloid_dtype ct, const char *dtab, const TabOffsets &to,
                                  const StageItems &n, bool with_snr, float phase_thr, float trig_thr,
                                  const XiWork &xw, hipEvent_t *ev) {
  hipStream_t st = ctx->stream;
  auto mark = [&](int stage, int end) -> hipError_t {
    return ev ? hipEventRecord(ev[2 * (stage - LLOID_STAGE_FIR) + end], st) : hipSuccess;
  };
  HIP_TRY(mark(LLOID_STAGE_FIR, 0));
  HIP_TRY(launch_fir_jobs(ct, ctx->fir_variant, (const FirJob *)(dtab + to.fir), to.n_fir, n.fir, st));
  HIP_TRY(mark(LLOID_STAGE_FIR, 1));
  HIP_TRY(mark(LLOID_STAGE_INTERP, 0));
  for (int h = 0; h < kMaxHops; ++h)
    HIP_TRY(launch_up_jobs(ct, (const UpJob *)(dtab + to.up[h]), to.n_up[h], n.up[h], st));
  HIP_TRY(mark(LLOID_STAGE_INTERP, 1));
  HIP_TRY(mark(LLOID_STAGE_MIX, 0));
  HIP_TRY(launch_mix_jobs(ct, ctx->mix_variant, (const MixJob *)(dtab + to.mix), to.n_mix, n.mix, with_snr, st));
  HIP_TRY(mark(LLOID_STAGE_MIX, 1));
  HIP_TRY(mark(LLOID_STAGE_PHASE, 0));
  HIP_TRY(launch_peak_phase(ct, (const MixJob *)(dtab + to.mix), to.n_mix, n.entries, phase_thr, st));
  if (n.xi2) {
    if (xw.cap < n.xi_units) return fail(LLOID_EINVAL, "signal-consistency unit list too small");
    HIP_TRY(launch_xi2(ct, (const MixJob *)(dtab + to.mix), to.n_mix, n.windows, n.xi_kmax, n.xi_acorr, trig_thr, xw,
                       ctx->n_cu, st));
  }
  HIP_TRY(mark(LLOID_STAGE_PHASE, 1));
  return LLOID_OK;
}
// Filter one block of strain of one detector with every bank of `banks`
// (same context, full rate and operand type) and compact the triggers.
// no_alloc: every device buffer comes from the context's static scratch
// (chunks of windows sized to fit it) and the descriptor tables are staged in
// pageable host memory: no device or pinned allocation, no profiling events.
static lloid_status filter_banks(lloid_bank *const *banks, int nb, int32_t detector, const void *strain,
                                 lloid_dtype sdt, int64_t n, const lloid_trigger_opts *opts, lloid_trigger *trig,
                                 int64_t trig_cap, int64_t *n_trig, float *snr, lloid_peaks *peaks,
                                 bool no_alloc = false) {
  if (!banks || nb <= 0 || !strain || !n_trig) return fail(LLOID_EINVAL, "NULL argument");
  for (int i = 0; i < nb; ++i)
    if (!banks[i]) return fail(LLOID_EINVAL, "bank %d is NULL", i);
  lloid_ctx *ctx = banks[0]->ctx;
  const int f0 = banks[0]->f0;
  const lloid_dtype ct = banks[0]->compute;
  for (int i = 1; i < nb; ++i) {
    if (banks[i]->ctx != ctx) return fail(LLOID_EINVAL, "banks of one batch must share a context");
    if (banks[i]->f0 != f0) return fail(LLOID_EINVAL, "banks of one batch must share the full rate");
    if (banks[i]->compute != ct) return fail(LLOID_EINVAL, "banks of one batch must share the compute type");
  }
  if (n <= 0) return fail(LLOID_EINVAL, "n must be positive");
  if (n > kMaxBlock) return fail(LLOID_EINVAL, "blocks longer than 2^28 samples must be split");
  if (sdt != LLOID_F64 && sdt != LLOID_F32) return fail(LLOID_EINVAL, "strain must be F64 or F32");
  if (trig_cap < 0 || (trig_cap > 0 && !trig)) return fail(LLOID_EINVAL, "bad trigger buffer");
  if (snr && nb != 1) return fail(LLOID_EINVAL, "the SNR series output needs a single bank");
  int64_t num = 1, den = 1;
  float thr = 4.f, sscale = 1.f;
  if (opts) {
    num = opts->window_num;
    den = opts->window_den;
    thr = opts->threshold;
    if (opts->strain_scale != 0.f) sscale = opts->strain_scale;
  }
  if (num <= 0 || den <= 0) return fail(LLOID_EINVAL, "window length must be positive");
  if ((int64_t)f0 * num < den) return fail(LLOID_EINVAL, "windows shorter than one sample");
  if (!(sscale > 0.f) || !std::isfinite(sscale)) return fail(LLOID_EINVAL, "strain_scale must be positive");
  {
    int e;
    if (std::frexp((double)sscale, &e) != 0.5) return fail(LLOID_EINVAL, "strain_scale must be a power of two");
  }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;

  Windows win{(int64_t)f0 * num, den};
  const int64_t W = win.count(n);
  if (peaks)
    for (int i = 0; i < nb; ++i)
      if ((peaks[i].snr || peaks[i].sample || peaks[i].phase) && peaks[i].n_windows < W) {
        peaks[i].n_windows = W;
        return fail(LLOID_ETRUNC, "peak table of bank %d needs %lld windows per template", i, (long long)W);
      }
  int n_levels = 1;
  for (int i = 0; i < nb; ++i) n_levels = std::max(n_levels, banks[i]->n_levels);
  std::vector<Range> sup(n_levels);
  sup[0] = {0, n};
  for (int k = 1; k < n_levels; ++k) sup[k] = halo_up(sup[k - 1]);

  // chunks of whole windows, sized so that every bank's operand fits the budget
  const size_t esz = dtype_size(ct);
  int64_t bytes_per_sample = 0;
  for (int i = 0; i < nb; ++i) {
    bytes_per_sample += banks[i]->kld * (int64_t)esz;
    for (const auto &sl : banks[i]->slices)
      if (sl.level > 0) {
        // low-rate buffers: one per hop input, at that hop's source rate
        const UpPlan p = up_plan(0, 1, sl.level);
        for (int lev : p.lev_in) bytes_per_sample += ((int64_t)sl.lp * (int64_t)low_esz(ct) >> lev) + 1;
      }
  }
  const int64_t win_len = ceil_div(win.p, win.q);
  int64_t wpc = std::max<int64_t>(1, ctx->chunk_budget / std::max<int64_t>(1, bytes_per_sample * win_len));
  wpc = std::min(wpc, W);
  // every buffer a kernel addresses through a buffer resource stays under 2 GiB
  for (int i = 0; i < nb; ++i)
    while (wpc > 1 &&
           !operands_fit(banks[i], std::min<int64_t>(n, win.start(wpc) + 1) + 2 * operand_margin(banks[i]), win_len))
      wpc = (wpc + 1) / 2;
  for (int i = 0; i < nb; ++i)
    if (!operands_fit(banks[i], std::min<int64_t>(n, win.start(wpc) + 1) + 2 * operand_margin(banks[i]), win_len))
      return fail(LLOID_EINVAL, "one trigger window of bank %d needs buffers over 2 GiB", i);
  const TileShapes ts(ct, ctx->fir_variant, ctx->mix_variant);

  // ---- workspace layout for chunks of wpc_ windows
  const bool host_strain = !is_device_ptr(strain);
  const bool host_snr = snr && !is_device_ptr(snr);
  int64_t total_rows = 0;
  for (int i = 0; i < nb; ++i) total_rows += banks[i]->n_templates;
  // a trigger buffer in device memory or pinned host memory takes the records
  // straight from the compaction kernel; otherwise they go through scratch
  lloid_trigger *direct_trig = trig_cap > 0 ? (lloid_trigger *)device_address(trig) : nullptr;
  const int64_t dev_cap = direct_trig ? trig_cap : std::min<int64_t>(trig_cap, total_rows * W);
  size_t n_fir = 0, n_up = 0;
  for (int i = 0; i < nb; ++i)
    for (const auto &sl : banks[i]->slices) {
      ++n_fir;
      if (sl.level > 0) n_up += up_plan(0, 1, sl.level).r.size();
    }
  auto table_bytes = [&](int64_t chunks) -> size_t {
    return (size_t)chunks * (n_fir * sizeof(FirJob) + n_up * sizeof(UpJob) + nb * sizeof(MixJob) +
                             64 * (3 + kMaxHops)) +
           nb * sizeof(TrigJob) + 256;
  };
  // signal-consistency units of the banks with lags over a chunk of wpc_ windows
  auto xi_cap = [&](int64_t wpc_) -> int64_t {
    int64_t c = 0;
    for (int i = 0; i < nb; ++i)
      if (banks[i]->acorr) c += xi_unit_cap(wpc_, banks[i]->n_templates);
    return c;
  };
  auto layout_bytes = [&](int64_t wpc_) -> size_t {
    const int64_t chunk_n_ = std::min<int64_t>(n, win.start(wpc_) + 1);
    size_t bytes = 0;
    auto add = [&](size_t cnt, size_t sz) { bytes = (size_t)round_up((int64_t)bytes, 256) + cnt * sz; };
    if (host_strain) add((size_t)n, dtype_size(sdt));
    for (int k = 0; k < n_levels; ++k) add((size_t)sup[k].size(), 4);
    for (int i = 0; i < nb; ++i) {
      const size_t tab = (size_t)banks[i]->n_templates * W;
      add(tab, 4);
      add(tab, 8);
      add(tab, 4);
      add(tab, 4);
      add(tab, 4);
      add(tab, 4);
      add(tab, 8);
      if (banks[i]->acorr) add(tab, 8);
      const int64_t ops = chunk_n_ + 2 * operand_margin(banks[i]);
      add((size_t)ops * banks[i]->kld, esz);
      for (const auto &sl : banks[i]->slices)
        if (sl.level > 0)
          for (int64_t ld : low_ld(ops, sl.level)) add((size_t)sl.lp * ld, low_esz(ct));
    }
    add((size_t)trig_blocks(total_rows * W) + 2, 8);
    add(1, 4);
    add((size_t)xi_cap(wpc_), sizeof(XiUnit));
    add(2, 4);
    if (!direct_trig) add((size_t)std::max<int64_t>(dev_cap, 1), sizeof(lloid_trigger));
    if (host_snr) add((size_t)n * 2 * banks[0]->n_templates, 4);
    add(table_bytes(ceil_div(W, wpc_)), 1);
    return bytes;
  };
  if (no_alloc) {
    // the largest chunk of windows whose buffers fit the static scratch
    const size_t cap = (size_t)LLOID_NOALLOC_SCRATCH_BYTES;
    const size_t need1 = layout_bytes(1);
    if (need1 > cap)
      return fail(LLOID_ENOMEM,
                  "this call needs %zu bytes of device scratch with one window per chunk; the static scratch "
                  "holds %zu (use lloid_filter, or a shorter block or fewer templates)",
                  need1, cap);
    int64_t lo = 1, hi = wpc;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (layout_bytes(mid) <= cap) lo = mid;
      else hi = mid - 1;
    }
    wpc = lo;
  }
  const int64_t n_chunks = ceil_div(W, wpc);
  const int64_t chunk_n = std::min<int64_t>(n, win.start(wpc) + 1);   // samples of the longest chunk
  const size_t tab_bytes = table_bytes(n_chunks);
  const size_t bytes = layout_bytes(wpc);
  std::vector<char> host_tab;   // pageable staging of the tables (no_alloc)
  void *ws_base = nullptr;
  if (no_alloc) {
    if (!ctx->static_scratch) return fail(LLOID_EDEVICE, "the context has no static scratch");
    ws_base = ctx->static_scratch;
    host_tab.resize(tab_bytes);
  } else {
    lloid_status rs = ensure_ws(ctx, ctx->ws, bytes);
    if (rs != LLOID_OK) return rs;
    rs = ensure_pinned(ctx, ctx->pinned, ctx->pinned_bytes, tab_bytes);
    if (rs != LLOID_OK) return rs;
    ws_base = ctx->ws.base;
  }
  const bool prof = ctx->profile && !no_alloc;

  Carve cv{(char *)ws_base};
  const void *d_strain = strain;
  void *strain_tmp = host_strain ? cv.take<char>((size_t)n * dtype_size(sdt)) : nullptr;
  std::vector<float *> xl(n_levels);
  std::vector<LevelView> lv(n_levels);
  for (int k = 0; k < n_levels; ++k) {
    xl[k] = cv.take<float>((size_t)sup[k].size());
    lv[k] = LevelView{xl[k], sup[k].lo, sup[k].size()};
  }
  std::vector<BankBufs> bw(nb);
  for (int i = 0; i < nb; ++i) {
    const size_t tab = (size_t)banks[i]->n_templates * W;
    bw[i].psnr = cv.take<float>(tab);
    bw[i].pn = cv.take<int64_t>(tab);
    bw[i].pphase = cv.take<float>(tab);
    bw[i].pdt = cv.take<float>(tab);
    bw[i].psi = cv.take<float>(tab);
    bw[i].pxi = cv.take<float>(tab);
    bw[i].pz = cv.take<float2>(tab);
    if (banks[i]->acorr) bw[i].pkey = cv.take<int64_t>(tab);
    bw[i].ld_peak = W;
    bw[i].w_base = 0;
    const int64_t ops = chunk_n + 2 * operand_margin(banks[i]);
    bw[i].ocat = cv.take<char>((size_t)ops * banks[i]->kld * esz);
    bw[i].low.assign(banks[i]->slices.size(), {});
    for (size_t s = 0; s < banks[i]->slices.size(); ++s) {
      const auto &sl = banks[i]->slices[s];
      if (sl.level > 0)
        for (int64_t ld : low_ld(ops, sl.level))
          bw[i].low[s].push_back(cv.take<char>((size_t)sl.lp * ld * low_esz(ct)));
    }
  }
  const int64_t n_blk = trig_blocks(total_rows * W);
  int64_t *counts = cv.take<int64_t>((size_t)n_blk + 2);
  int64_t *total = counts + n_blk;
  int *bad = cv.take<int>(1);
  XiWork xw;
  xw.cap = xi_cap(wpc);
  xw.units = cv.take<XiUnit>((size_t)xw.cap);
  xw.counters = cv.take<int32_t>(2);
  lloid_trigger *dtrig = direct_trig ? direct_trig : cv.take<lloid_trigger>((size_t)std::max<int64_t>(dev_cap, 1));
  float *dsnr = snr ? (host_snr ? cv.take<float>((size_t)n * 2 * banks[0]->n_templates) : snr) : nullptr;
  char *dtab = cv.take<char>(tab_bytes);

  // ---- descriptor tables of every chunk, uploaded in one copy
  struct Chunk {
    TabOffsets to;
    StageItems items;
  };
  std::vector<Chunk> chunks(n_chunks);
  char *htab = no_alloc ? host_tab.data() : (char *)ctx->pinned;
  size_t off = 0;
  auto put = [&](const void *src, size_t sz) -> size_t {
    off = (size_t)round_up((int64_t)off, 64);
    const size_t at = off;
    if (sz) std::memcpy(htab + off, src, sz);
    off += sz;
    return at;
  };
  for (int64_t c = 0; c < n_chunks; ++c) {
    const int64_t wa = c * wpc, wb = std::min(W, wa + wpc);
    const int64_t t0 = win.start(wa), t1 = std::min(n, win.start(wb));
    std::vector<FirJob> fj;
    std::vector<UpJob> uj[kMaxHops];
    std::vector<MixJob> mj;
    for (int i = 0; i < nb; ++i)
      add_bank_jobs(banks[i], lv.data(), t0, t1, n, wa, wb, win, bw[i], 1.f / (banks[i]->mix_scale * sscale),
                    (snr && i == 0) ? dsnr + t0 * 2 : nullptr, n, ts, fj, uj, mj);
    number_jobs(fj, uj, mj, chunks[c].items);
    TabOffsets &to = chunks[c].to;
    to.fir = put(fj.data(), fj.size() * sizeof(FirJob));
    for (int h = 0; h < kMaxHops; ++h) {
      to.up[h] = put(uj[h].data(), uj[h].size() * sizeof(UpJob));
      to.n_up[h] = (int)uj[h].size();
    }
    to.mix = put(mj.data(), mj.size() * sizeof(MixJob));
    to.n_fir = (int)fj.size();
    to.n_mix = (int)mj.size();
  }
  std::vector<TrigJob> tj(nb);
  {
    int64_t e = 0;
    for (int i = 0; i < nb; ++i) {
      tj[i] = TrigJob{bw[i].psnr, bw[i].pn, bw[i].pphase, bw[i].pdt, bw[i].psi,
                      banks[i]->acorr ? bw[i].pxi : nullptr, 0, W, e, banks[i]->n_templates, i, detector, 0};
      e += (int64_t)banks[i]->n_templates * W;
    }
  }
  const size_t trig_off = put(tj.data(), tj.size() * sizeof(TrigJob));

  // ---- launches
  auto mark = [&](int stage, int end) -> hipError_t {
    return prof ? hipEventRecord(ctx->ev[2 * stage + end], st) : hipSuccess;
  };
  HIP_TRY(mark(LLOID_STAGE_INGEST, 0));
  HIP_TRY(hipMemcpyAsync(dtab, htab, off, hipMemcpyHostToDevice, st));
  if (host_strain) {
    HIP_TRY(hipMemcpyAsync(strain_tmp, strain, (size_t)n * dtype_size(sdt), hipMemcpyHostToDevice, st));
    d_strain = strain_tmp;
  }
  HIP_TRY(launch_fill_u8(bad, sizeof(int), st));
  HIP_TRY(launch_convert(d_strain, sdt, n, xl[0], sup[0].lo, sup[0].size(), sscale, bad, st));
  HIP_TRY(mark(LLOID_STAGE_INGEST, 1));
  HIP_TRY(mark(LLOID_STAGE_DECIMATE, 0));
  for (int k = 1; k < n_levels; ++k)
    HIP_TRY(launch_decimate(xl[k - 1], sup[k - 1].lo, sup[k - 1].size(), xl[k], sup[k].lo, sup[k].size(),
                            ctx->d_halfband, st));
  HIP_TRY(mark(LLOID_STAGE_DECIMATE, 1));
  const float phase_thr = (peaks && peaks[0].phase) ? -1.f : thr;
  // every chunk's FIR, interpolation, mixing and phase stages get events of their own
  const size_t nev = (size_t)2 * kChunkStages * n_chunks;
  if (prof)
    while (ctx->cev.size() < nev) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      ctx->cev.push_back(e);
    }
  for (int64_t c = 0; c < n_chunks; ++c) {
    const lloid_status r2 = launch_stages(ctx, ct, dtab, chunks[c].to, chunks[c].items, snr != nullptr, phase_thr,
                                          thr, xw, prof ? &ctx->cev[(size_t)2 * kChunkStages * c] : nullptr);
    if (r2 != LLOID_OK) return r2;
  }
  HIP_TRY(mark(LLOID_STAGE_TRIGGER, 0));
  HIP_TRY(launch_trigger_jobs((const TrigJob *)(dtab + trig_off), nb, total_rows * W, thr, counts, total, dev_cap,
                              dtrig, st));
  HIP_TRY(mark(LLOID_STAGE_TRIGGER, 1));
  HIP_TRY(mark(LLOID_STAGE_D2H, 0));
  int64_t h_total = 0;
  int h_bad = 0;
  HIP_TRY(hipMemcpyAsync(&h_total, total, sizeof h_total, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&h_bad, bad, sizeof h_bad, hipMemcpyDeviceToHost, st));
  if (peaks)
    for (int i = 0; i < nb; ++i) {
      const size_t ld = (size_t)peaks[i].n_windows;   // the caller's rows may be wider than W
      const size_t F = (size_t)banks[i]->n_templates;
      if (peaks[i].snr) HIP_TRY(hipMemcpy2DAsync(peaks[i].snr, ld * 4, bw[i].psnr, W * 4, W * 4, F, hipMemcpyDefault, st));
      if (peaks[i].sample) HIP_TRY(hipMemcpy2DAsync(peaks[i].sample, ld * 8, bw[i].pn, W * 8, W * 8, F, hipMemcpyDefault, st));
      if (peaks[i].phase) HIP_TRY(hipMemcpy2DAsync(peaks[i].phase, ld * 4, bw[i].pphase, W * 4, W * 4, F, hipMemcpyDefault, st));
      peaks[i].n_windows = W;
    }
  if (host_snr)
    HIP_TRY(hipMemcpyAsync(snr, dsnr, (size_t)banks[0]->n_templates * n * 2 * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int64_t ncopy = direct_trig ? 0 : std::min(h_total, dev_cap);
  if (ncopy > 0) HIP_TRY(hipMemcpyAsync(trig, dtrig, (size_t)ncopy * sizeof(lloid_trigger), hipMemcpyDefault, st));
  HIP_TRY(mark(LLOID_STAGE_D2H, 1));
  if (ncopy > 0 || prof) HIP_TRY(hipStreamSynchronize(st));
  if (prof) {
    for (int i = 0; i < LLOID_N_STAGES; ++i) {
      float ms = 0.f;
      if (i >= LLOID_STAGE_FIR && i < LLOID_STAGE_FIR + kChunkStages) {
        for (int64_t c = 0; c < n_chunks; ++c) {
          float m = 0.f;
          const size_t k = (size_t)2 * (kChunkStages * c + i - LLOID_STAGE_FIR);
          HIP_TRY(hipEventElapsedTime(&m, ctx->cev[k], ctx->cev[k + 1]));
          ms += m;
        }
      } else {
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[2 * i], ctx->ev[2 * i + 1]));
      }
      ctx->stage_ms[i] += ms;
      ctx->stage_calls[i] += 1;
    }
  }
  *n_trig = h_total;
  if (h_bad) return fail(LLOID_EDATA, "strain holds a non-finite sample");
  if (h_total > trig_cap)
    return fail(LLOID_ETRUNC, "%lld triggers, buffer holds %lld", (long long)h_total, (long long)trig_cap);
  return LLOID_OK;
}

extern "C" lloid_status lloid_filter(lloid_bank *b, int32_t detector, const void *strain, lloid_dtype sdt, int64_t n,
                                     const lloid_trigger_opts *opts, lloid_trigger *trig, int64_t trig_cap,
                                     int64_t *n_trig, float *snr, lloid_peaks *peaks) {
  ABI_GUARD_BEGIN
  if (!b) return fail(LLOID_EINVAL, "NULL bank");
  return filter_banks(&b, 1, detector, strain, sdt, n, opts, trig, trig_cap, n_trig, snr, peaks);
  ABI_GUARD_END
}

extern "C" lloid_status lloid_filter_noalloc(lloid_bank *b, int32_t detector, const void *strain, lloid_dtype sdt,
                                             int64_t n, const lloid_trigger_opts *opts, lloid_trigger *trig,
                                             int64_t trig_cap, int64_t *n_trig, lloid_peaks *peaks) {
  ABI_GUARD_BEGIN
  if (!b) return fail(LLOID_EINVAL, "NULL bank");
  return filter_banks(&b, 1, detector, strain, sdt, n, opts, trig, trig_cap, n_trig, nullptr, peaks, true);
  ABI_GUARD_END
}

extern "C" lloid_status lloid_filter_batch(lloid_bank *const *banks, int32_t n_banks, int32_t detector,
                                           const void *strain, lloid_dtype sdt, int64_t n,
                                           const lloid_trigger_opts *opts, lloid_trigger *trig, int64_t trig_cap,
                                           int64_t *n_trig, lloid_peaks *peaks) {
  ABI_GUARD_BEGIN
  return filter_banks(banks, n_banks, detector, strain, sdt, n, opts, trig, trig_cap, n_trig, nullptr, peaks);
  ABI_GUARD_END
}

extern "C" lloid_status lloid_condition(lloid_ctx *ctx, int32_t full_rate_hz, const void *strain, lloid_dtype dtype,
                                       int64_t n, const lloid_condition_opts *opts, float *out, double *psd_out,
                                       int64_t *n_gated) {
  ABI_GUARD_BEGIN
  if (!ctx || !strain || !opts || !out) return fail(LLOID_EINVAL, "NULL argument");
  if (full_rate_hz <= 0) return fail(LLOID_EINVAL, "full_rate_hz must be positive");
  if (dtype != LLOID_F64 && dtype != LLOID_F32) return fail(LLOID_EINVAL, "strain must be F64 or F32");
  if (n < 1 || n > kMaxBlock) return fail(LLOID_EINVAL, "n must be in [1, 2^28]");
  const int L = opts->seg_len;
  if (L < kCondMinLen || L > kCondMaxLen || (L & (L - 1)))
    return fail(LLOID_EINVAL, "seg_len %d is not a power of two in [%d, %d]", L, kCondMinLen, kCondMaxLen);
  if (opts->gate_half_width < 0 || !(opts->gate_threshold >= 0.f) || !std::isfinite(opts->gate_threshold))
    return fail(LLOID_EINVAL, "bad gate options");
  const bool estimate = opts->psd == nullptr;
  if (estimate && n < L) return fail(LLOID_EINVAL, "a block of %lld samples is shorter than one segment", (long long)n);
  const int nf = L / 2 + 1;
  if (!estimate)
    for (int f = 0; f < nf; ++f)
      if (!std::isfinite(opts->psd[f])) return fail(LLOID_EINVAL, "non-finite PSD value at bin %d", f);
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const bool host_strain = !is_device_ptr(strain), host_out = !is_device_ptr(out);
  const bool gating = opts->gate_threshold > 0.f;
  const int64_t nseg_p = estimate ? (n - L) / (L / 2) + 1 : 0;
  const int64_t nseg_w = (2 * (n - 1)) / L + 2;
  size_t bytes = 0;
  auto add = [&](size_t cnt, size_t sz) { bytes = (size_t)round_up((int64_t)bytes, 256) + cnt * sz; };
  if (host_strain) add((size_t)n, dtype_size(dtype));
  add((size_t)n, 4);                       // float strain
  add((size_t)(nseg_p * nf), 4);           // periodograms
  add((size_t)nf, 4);                      // PSD (FP32 on the device)
  add((size_t)nf, 4);                      // gain
  add((size_t)(nseg_w * L), 4);            // whitened segments
  if (gating) add((size_t)n, 4), add((size_t)n, 1);
  if (host_out) add((size_t)n, 4);
  add(1, 8);
  add(1, sizeof(int));
  lloid_status rs = ensure_ws(ctx, ctx->ws, bytes);
  if (rs != LLOID_OK) return rs;
  Carve cv{(char *)ctx->ws.base};
  const void *d_strain = strain;
  if (host_strain) {
    char *p = cv.take<char>((size_t)n * dtype_size(dtype));
    HIP_TRY(hipMemcpyAsync(p, strain, (size_t)n * dtype_size(dtype), hipMemcpyHostToDevice, st));
    d_strain = p;
  }
  float *x = cv.take<float>((size_t)n);
  float *parts = cv.take<float>((size_t)(nseg_p * nf));
  float *psd = cv.take<float>((size_t)nf);
  float *gain = cv.take<float>((size_t)nf);
  float *y = cv.take<float>((size_t)(nseg_w * L));
  float *xw = gating ? cv.take<float>((size_t)n) : nullptr;
  uint8_t *mask = gating ? cv.take<uint8_t>((size_t)n) : nullptr;
  float *dout = host_out ? cv.take<float>((size_t)n) : out;
  unsigned long long *count = cv.take<unsigned long long>(1);
  int *bad = cv.take<int>(1);
  HIP_TRY(launch_fill_u8(bad, sizeof(int), st));
  HIP_TRY(launch_fill_u8(count, 8, st));
  if (gating) HIP_TRY(launch_fill_u8(mask, (size_t)n, st));
  std::vector<float> psd_h((size_t)nf);
  if (!estimate) {
    for (int f = 0; f < nf; ++f) psd_h[f] = (float)opts->psd[f];
    HIP_TRY(hipMemcpyAsync(psd, psd_h.data(), (size_t)nf * 4, hipMemcpyHostToDevice, st));
  }
  HIP_TRY(launch_convert(d_strain, dtype, n, x, 0, n, 1.f, bad, st));
  HIP_TRY(launch_condition(x, n, L, estimate, (float)full_rate_hz, parts, psd, gain, y, xw, opts->gate_threshold,
                           opts->gate_half_width, mask, dout, count, st));
  int h_bad = 0;
  unsigned long long h_count = 0;
  HIP_TRY(hipMemcpyAsync(&h_bad, bad, sizeof h_bad, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&h_count, count, sizeof h_count, hipMemcpyDeviceToHost, st));
  if (psd_out) HIP_TRY(hipMemcpyAsync(psd_h.data(), psd, (size_t)nf * 4, hipMemcpyDeviceToHost, st));
  if (host_out) HIP_TRY(hipMemcpyAsync(out, dout, (size_t)n * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (psd_out)
    for (int f = 0; f < nf; ++f) psd_out[f] = (double)psd_h[f];
  if (h_bad) return fail(LLOID_EDATA, "strain holds a non-finite sample");
  if (n_gated) *n_gated = (int64_t)h_count;
  return LLOID_OK;
  ABI_GUARD_END
}

extern "C" lloid_status lloid_coincide(lloid_ctx *ctx, const lloid_trigger *a, int64_t n_a, const lloid_trigger *b,
                                      int64_t n_b, int64_t max_dt, lloid_coinc *out, int64_t cap, int64_t *n_out,
                                      uint8_t *background) {
  ABI_GUARD_BEGIN
  if (!ctx || !n_out) return fail(LLOID_EINVAL, "NULL argument");
  if (n_a < 0 || n_b < 0 || cap < 0 || max_dt < 0) return fail(LLOID_EINVAL, "negative count, capacity or max_dt");
  if ((n_a > 0 && !a) || (n_b > 0 && !b)) return fail(LLOID_EINVAL, "NULL trigger list");
  if (cap > 0 && !out) return fail(LLOID_EINVAL, "NULL output with a positive capacity");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const bool host_a = n_a > 0 && !is_device_ptr(a), host_b = n_b > 0 && !is_device_ptr(b);
  const bool host_out = cap > 0 && !is_device_ptr(out);
  const bool host_bg = background && !is_device_ptr(background);
  size_t bytes = 0;
  auto add = [&](size_t cnt, size_t sz) { bytes = (size_t)round_up((int64_t)bytes, 256) + cnt * sz; };
  if (host_a) add((size_t)n_a, sizeof(lloid_trigger));
  if (host_b) add((size_t)n_b, sizeof(lloid_trigger));
  add((size_t)n_a + 2, 8);
  add(1, sizeof(int));
  if (host_out) add((size_t)cap, sizeof(lloid_coinc));
  if (host_bg) add((size_t)(n_a + n_b), 1);
  lloid_status rs = ensure_ws(ctx, ctx->ws, bytes);
  if (rs != LLOID_OK) return rs;
  Carve cv{(char *)ctx->ws.base};
  const lloid_trigger *da = a, *db = b;
  if (host_a) {
    lloid_trigger *p = cv.take<lloid_trigger>((size_t)n_a);
    HIP_TRY(hipMemcpyAsync(p, a, (size_t)n_a * sizeof(lloid_trigger), hipMemcpyHostToDevice, st));
    da = p;
  }
  if (host_b) {
    lloid_trigger *p = cv.take<lloid_trigger>((size_t)n_b);
    HIP_TRY(hipMemcpyAsync(p, b, (size_t)n_b * sizeof(lloid_trigger), hipMemcpyHostToDevice, st));
    db = p;
  }
  int64_t *counts = cv.take<int64_t>((size_t)n_a + 2);
  int64_t *total = counts + n_a;
  int *bad = cv.take<int>(1);
  lloid_coinc *dout = host_out ? cv.take<lloid_coinc>((size_t)cap) : out;
  uint8_t *dbg = host_bg ? cv.take<uint8_t>((size_t)(n_a + n_b)) : background;
  HIP_TRY(launch_fill_u8(bad, sizeof(int), st));
  HIP_TRY(launch_coincide(da, n_a, db, n_b, max_dt, counts, total, bad, cap, dout, dbg, dbg ? dbg + n_a : nullptr,
                          st));
  int64_t h_total = 0;
  int h_bad = 0;
  HIP_TRY(hipMemcpyAsync(&h_total, total, sizeof h_total, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&h_bad, bad, sizeof h_bad, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h_bad) return fail(LLOID_EINVAL, "a trigger list is not sorted by (bank, template_id, sample)");
  const int64_t ncopy = std::min(h_total, cap);
  if (host_out && ncopy > 0)
    HIP_TRY(hipMemcpyAsync(out, dout, (size_t)ncopy * sizeof(lloid_coinc), hipMemcpyDeviceToHost, st));
  if (host_bg && n_a + n_b > 0)
    HIP_TRY(hipMemcpyAsync(background, dbg, (size_t)(n_a + n_b), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *n_out = h_total;
  if (h_total > cap) return fail(LLOID_ETRUNC, "%lld coincidences, capacity %lld", (long long)h_total, (long long)cap);
  return LLOID_OK;
  ABI_GUARD_END
}

extern "C" lloid_status lloid_ctx_set_tiles(lloid_ctx *ctx, int32_t fir_variant, int32_t mix_variant) {
  if (!ctx) return fail(LLOID_EINVAL, "NULL context");
  if (fir_variant < 0 || fir_variant >= kFirVariants || mix_variant < 0 || mix_variant >= kMixVariants)
    return fail(LLOID_EINVAL, "tile variants must be in [0, %d) and [0, %d)", kFirVariants, kMixVariants);
  ctx->fir_variant = fir_variant;
  ctx->mix_variant = mix_variant;
  return LLOID_OK;
}

extern "C" lloid_status lloid_ctx_get_tiles(const lloid_ctx *ctx, int32_t *fir_variant, int32_t *mix_variant) {
  if (!ctx || !fir_variant || !mix_variant) return fail(LLOID_EINVAL, "NULL argument");
  *fir_variant = ctx->fir_variant;
  *mix_variant = ctx->mix_variant;
  return LLOID_OK;
}

// ---- autotuning of the tile shapes
namespace {

// Shape class of a bank set on this device: architecture, operand type, the
// sizes the tiles see (banks, rows, concatenated K, longest filter, levels)
// and the block length (samples, rounded up to a power of two): short blocks
// leave most of the GPU idle and can favour other tiles than long ones.
std::string tune_key(const lloid_ctx *ctx, lloid_bank *const *banks, int nb, int64_t n) {
  hipDeviceProp_t prop;
  std::string arch = "gfx";
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
  }
  int64_t rows = 0, kcat = 0, np = 0;
  int levels = 0;
  for (int i = 0; i < nb; ++i) {
    rows += banks[i]->rows;
    kcat += banks[i]->kcat;
    levels = std::max(levels, banks[i]->n_levels);
    for (const auto &sl : banks[i]->slices) np = std::max<int64_t>(np, sl.np);
  }
  int64_t block = 1;
  while (block < n) block <<= 1;
  static const char *names[] = {"f64", "f32", "f16", "bf16"};
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s/%s/banks%d/rows%lld/k%lld/taps%lld/levels%d/block%lld", arch.c_str(),
                names[banks[0]->compute], nb, (long long)rows, (long long)kcat, (long long)np, levels,
                (long long)block);
  return buf;
}

struct TuneEntry {
  std::string key;
  int fir = 0, mix = 0;
  double ms = 0;
};

// The cache is a JSON object with one line per shape class:
//   "key": {"fir": F, "mix": M, "ms": T},
std::vector<TuneEntry> read_tune_cache(const char *path) {
  std::vector<TuneEntry> out;
  FILE *f = path ? std::fopen(path, "r") : nullptr;
  if (!f) return out;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    const char *q0 = std::strchr(line, '"');
    const char *q1 = q0 ? std::strchr(q0 + 1, '"') : nullptr;
    if (!q1) continue;
    TuneEntry e;
    e.key.assign(q0 + 1, q1);
    if (std::sscanf(q1 + 1, ": {\"fir\": %d, \"mix\": %d, \"ms\": %lf", &e.fir, &e.mix, &e.ms) == 3 &&
        e.fir >= 0 && e.fir < kFirVariants && e.mix >= 0 && e.mix < kMixVariants)
      out.push_back(e);
  }
  std::fclose(f);
  return out;
}

bool write_tune_cache(const char *path, const std::vector<TuneEntry> &entries) {
  FILE *f = std::fopen(path, "w");
  if (!f) return false;
  std::fprintf(f, "{\n");
  for (size_t i = 0; i < entries.size(); ++i)
    std::fprintf(f, "\"%s\": {\"fir\": %d, \"mix\": %d, \"ms\": %.4f}%s\n", entries[i].key.c_str(), entries[i].fir,
                 entries[i].mix, entries[i].ms, i + 1 < entries.size() ? "," : "");
  std::fprintf(f, "}\n");
  return std::fclose(f) == 0;
}

}  // namespace

extern "C" lloid_status lloid_autotune(lloid_ctx *ctx, lloid_bank *const *banks, int32_t n_banks, double seconds,
                                      const char *cache_path, lloid_tune_result *results, int32_t cap,
                                      int32_t *n_results) {
  ABI_GUARD_BEGIN
  if (!ctx || !banks || n_banks <= 0 || !n_results) return fail(LLOID_EINVAL, "NULL argument or no banks");
  for (int i = 0; i < n_banks; ++i)
    if (!banks[i] || banks[i]->ctx != ctx) return fail(LLOID_EINVAL, "bank %d is NULL or of another context", i);
  if (!(seconds > 0) || seconds > 4096) return fail(LLOID_EINVAL, "seconds must be in (0, 4096]");
  if (cap < 0 || (cap > 0 && !results)) return fail(LLOID_EINVAL, "bad result buffer");
  *n_results = 0;
  const int64_t n = std::min<int64_t>(kMaxBlock, (int64_t)std::llround(seconds * banks[0]->f0));
  const std::string key = tune_key(ctx, banks, n_banks, n);
  std::vector<TuneEntry> cache = read_tune_cache(cache_path);
  for (const auto &e : cache)
    if (e.key == key) {
      ctx->fir_variant = e.fir;
      ctx->mix_variant = e.mix;
      return LLOID_OK;
    }
  HIP_TRY(hipSetDevice(ctx->device));
  float *x = nullptr;
  if (hipMalloc(&x, (size_t)n * sizeof(float)) != hipSuccess) return fail(LLOID_ENOMEM, "tuning strain");
  struct Free {
    float *p;
    ~Free() { (void)hipFree(p); }
  } guard{x};
  HIP_TRY(launch_noise(x, n, 0x2410164u, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  int64_t cap_t = 0;
  for (int i = 0; i < n_banks; ++i) cap_t += (int64_t)banks[i]->n_templates * (n / banks[0]->f0 + 2);
  std::vector<lloid_trigger> trig((size_t)cap_t);
  const int fir0 = ctx->fir_variant, mix0 = ctx->mix_variant;
  int best_f = fir0, best_m = mix0;
  double best_ms = 1e300;
  int32_t k = 0;
  for (int fv = 0; fv < kFirVariants; ++fv)
    for (int mv = 0; mv < kMixVariants; ++mv) {
      ctx->fir_variant = fv;
      ctx->mix_variant = mv;
      double ms = 1e300;
      for (int rep = 0; rep < 5; ++rep) {   // the first call warms up; the fastest of the others counts
        int64_t n_trig = 0;
        const auto t0 = std::chrono::steady_clock::now();
        const lloid_status st = lloid_filter_batch(banks, n_banks, 0, x, LLOID_F32, n, nullptr, trig.data(), cap_t,
                                                   &n_trig, nullptr);
        const auto t1 = std::chrono::steady_clock::now();
        if (st != LLOID_OK && st != LLOID_ETRUNC) {
          ctx->fir_variant = fir0;
          ctx->mix_variant = mix0;
          return st;
        }
        if (rep > 0) ms = std::min(ms, std::chrono::duration<double, std::milli>(t1 - t0).count());
      }
      if (k < cap) results[k] = lloid_tune_result{fv, mv, ms};
      ++k;
      if (ms < best_ms) best_ms = ms, best_f = fv, best_m = mv;
    }
  *n_results = k;
  ctx->fir_variant = best_f;
  ctx->mix_variant = best_m;
  if (cache_path) {
    cache.push_back(TuneEntry{key, best_f, best_m, best_ms});
    if (!write_tune_cache(cache_path, cache)) return fail(LLOID_EINVAL, "cannot write %s", cache_path);
  }
  return LLOID_OK;
  ABI_GUARD_END
}

extern "C" lloid_status lloid_ctx_set_chunk_bytes(lloid_ctx *ctx, int64_t bytes) {
  if (!ctx || bytes <= 0) return fail(LLOID_EINVAL, "bad argument");
  ctx->chunk_budget = bytes;
  return LLOID_OK;
}
