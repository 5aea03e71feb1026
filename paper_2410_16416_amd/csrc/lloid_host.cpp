// Host runtime and C ABI of the LLOID filtering library (see include/lloid.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lloid_internal.h"

using namespace lloid;

// ------------------------------------------------------------ error state

static thread_local std::string g_last_error;

static lloid_status fail(lloid_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(LLOID_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                                     \
  } while (0)

#define ABI_GUARD_BEGIN try {
#define ABI_GUARD_END                                                     \
  }                                                                       \
  catch (const std::bad_alloc &) {                                        \
    return fail(LLOID_ENOMEM, "host allocation failed");                  \
  }                                                                       \
  catch (const std::exception &ex) {                                      \
    return fail(LLOID_EINVAL, "internal error: %s", ex.what());           \
  }

extern "C" const char *lloid_last_error(void) { return g_last_error.c_str(); }
extern "C" const char *lloid_version(void) { return "lloid-gfx950 0.1"; }

// ------------------------------------------------------------ helpers

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
static int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
static int64_t ceil_div(int64_t a, int64_t b) { return -floor_div(-a, b); }
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

static bool is_device_ptr(const void *p) {
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

static size_t dtype_size(lloid_dtype t) {
  switch (t) {
    case LLOID_F64: return 8;
    case LLOID_F32: return 4;
    case LLOID_F16: return 2;
    case LLOID_BF16: return 2;
  }
  return 0;
}

// Device-side cast of an FP64 array to the compute type.
namespace lloid {
hipError_t launch_cast_f64(const double *src, lloid_dtype t, void *dst, int64_t n, hipStream_t s);
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
  lloid_ctx *c = new lloid_ctx();
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
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
  if (ctx->d_halfband) (void)hipFree(ctx->d_halfband);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return LLOID_OK;
}

// ------------------------------------------------------------ bank

static void free_bank_device(lloid_bank *b) {
  for (auto &s : b->slices)
    if (s.basis) (void)hipFree(s.basis), s.basis = nullptr;
  if (b->mix) (void)hipFree(b->mix), b->mix = nullptr;
  if (b->ws.base) (void)hipFree(b->ws.base), b->ws.base = nullptr, b->ws.bytes = 0;
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
    if (sl.start_tap < 0 || sl.start_tap % dec)
      return fail(LLOID_EINVAL, "slice %d: start tap %lld is not a non-negative multiple of %d", s,
                  (long long)sl.start_tap, dec);
    if (sl.n_taps <= 0) return fail(LLOID_EINVAL, "slice %d: n_taps must be positive", s);
    if (sl.n_basis <= 0 || sl.n_basis > sl.n_taps)
      return fail(LLOID_EINVAL, "slice %d: n_basis %d must be in [1, n_taps = %d]", s, sl.n_basis, sl.n_taps);
    if (!sl.basis || !sl.mixing) return fail(LLOID_EINVAL, "slice %d: NULL basis or mixing", s);
  }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;

  lloid_bank *b = new lloid_bank();
  b->ctx = ctx;
  b->f0 = f0;
  b->n_templates = F;
  b->compute = d->compute;
  b->rows = (int)round_up(2 * (int64_t)F, 32 * kMixMT);
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
    sl.koff = koff;
    koff += sl.lp;
    lsum += in.n_basis;
    double mb = 0.0;
    for (int64_t i = 0; i < (int64_t)in.n_basis * in.n_taps; ++i) mb = std::max(mb, std::fabs(in.basis[i]));
    sl.basis_scale = pow2_scale(mb);
    for (int64_t i = 0; i < 2 * (int64_t)F * in.n_basis; ++i)
      max_mix = std::max(max_mix, std::fabs(in.mixing[i]) / sl.basis_scale);
    b->n_levels = std::max(b->n_levels, sl.level + 1);
    b->slices.push_back(sl);
  }
  // the last slice absorbs the padding of the concatenated K, so every column
  // of the operand is written by a FIR or an interpolation stage
  b->kcat = (int)round_up(koff, kBK);
  b->slices.back().lp += b->kcat - koff;
  for (auto &sl : b->slices) sl.lrows = (int)round_up(sl.lp, kRowTile);
  b->mix_scale = pow2_scale(max_mix);

  // Pack on the host in FP64, cast on the device.
  lloid_status status = LLOID_OK;
  double *dtmp = nullptr;
  size_t tmp_elems = (size_t)b->rows * b->kcat;
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
  host.assign((size_t)b->rows * b->kcat, 0.0);
  for (int s = 0; s < d->n_slices; ++s) {
    const lloid_slice &in = d->slices[s];
    const SliceDev &sl = b->slices[s];
    const double f = b->mix_scale / sl.basis_scale;
    for (int r = 0; r < 2 * F; ++r)
      for (int l = 0; l < in.n_basis; ++l)
        host[(size_t)r * b->kcat + sl.koff + l] = in.mixing[(size_t)r * in.n_basis + l] * f;
  }
  if (hipMalloc(&b->mix, host.size() * esz) != hipSuccess) return cleanup(fail(LLOID_ENOMEM, "mixing alloc"));
  b->device_bytes += (int64_t)(host.size() * esz);
  if (hipMemcpyAsync(dtmp, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
      launch_cast_f64(dtmp, b->compute, b->mix, (int64_t)host.size(), st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return cleanup(fail(LLOID_EDEVICE, "mixing upload failed"));

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

// ------------------------------------------------------------ filter plan

namespace {

// Index ranges of one offline block of n full-rate samples.
struct Plan {
  int n_levels = 1;
  std::vector<Range> need;  // outputs needed at each level for Y on [0, n)
  std::vector<Range> sup;   // support of the decimated strain at each level
  int64_t n_windows = 0, win_p = 1, win_q = 1;
};

Plan make_plan(const lloid_bank *b, int64_t n, int64_t num, int64_t den) {
  Plan p;
  p.n_levels = b->n_levels;
  p.need.resize(p.n_levels);
  p.sup.resize(p.n_levels);
  p.need[0] = {0, n};
  p.sup[0] = {0, n};
  for (int k = 1; k < p.n_levels; ++k) {
    // interpolation reads w[j] with |n - 2j| <= Q; decimation reads u[2k - m], |m| <= Q
    p.need[k] = {ceil_div(p.need[k - 1].lo - kHalfQ, 2), floor_div(p.need[k - 1].hi - 1 + kHalfQ, 2) + 1};
    p.sup[k] = {ceil_div(p.sup[k - 1].lo - kHalfQ, 2), floor_div(p.sup[k - 1].hi - 1 + kHalfQ, 2) + 1};
  }
  p.win_p = (int64_t)b->f0 * num;
  p.win_q = den;
  // window of sample n-1: largest w with floor(w p / q) <= n - 1
  p.n_windows = ceil_div(n * p.win_q, p.win_p);
  return p;
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

}  // namespace

static lloid_status ensure_ws(lloid_bank *b, size_t bytes) {
  if (b->ws.bytes >= bytes) return LLOID_OK;
  HIP_TRY(hipStreamSynchronize(b->ctx->stream));
  if (b->ws.base) (void)hipFree(b->ws.base);
  b->ws.base = nullptr;
  b->ws.bytes = 0;
  if (hipMalloc(&b->ws.base, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LLOID_ENOMEM, "workspace of %zu bytes does not fit on the device", bytes);
  }
  b->ws.bytes = bytes;
  return LLOID_OK;
}

extern "C" lloid_status lloid_filter(lloid_bank *b, int32_t detector, const void *strain, lloid_dtype sdt, int64_t n,
                                     const lloid_trigger_opts *opts, lloid_trigger *trig, int64_t trig_cap,
                                     int64_t *n_trig, float *snr, lloid_peaks *peaks) {
  ABI_GUARD_BEGIN
  if (!b || !strain || !n_trig) return fail(LLOID_EINVAL, "NULL argument");
  if (n <= 0) return fail(LLOID_EINVAL, "n must be positive");
  if (sdt != LLOID_F64 && sdt != LLOID_F32) return fail(LLOID_EINVAL, "strain must be F64 or F32");
  if (trig_cap < 0 || (trig_cap > 0 && !trig)) return fail(LLOID_EINVAL, "bad trigger buffer");
  int64_t num = 1, den = 1;
  float thr = 4.f, sscale = 1.f;
  if (opts) {
    num = opts->window_num;
    den = opts->window_den;
    thr = opts->threshold;
    if (opts->strain_scale != 0.f) sscale = opts->strain_scale;
  }
  if (num <= 0 || den <= 0) return fail(LLOID_EINVAL, "window length must be positive");
  if ((int64_t)b->f0 * num < den) return fail(LLOID_EINVAL, "windows shorter than one sample");
  if (!(sscale > 0.f) || !std::isfinite(sscale)) return fail(LLOID_EINVAL, "strain_scale must be positive");
  {
    int e;
    if (std::frexp((double)sscale, &e) != 0.5) return fail(LLOID_EINVAL, "strain_scale must be a power of two");
  }

  lloid_ctx *ctx = b->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const Plan p = make_plan(b, n, num, den);
  if (peaks && peaks->n_windows < p.n_windows && (peaks->snr || peaks->sample || peaks->phase)) {
    int64_t need = p.n_windows;
    peaks->n_windows = need;
    return fail(LLOID_ETRUNC, "peak table needs %lld windows per template", (long long)need);
  }
  const int F = b->n_templates;
  const size_t esz = dtype_size(b->compute);
  const bool host_strain = !is_device_ptr(strain);
  const bool host_snr = snr && !is_device_ptr(snr);

  // workspace layout
  size_t bytes = 0;
  auto add = [&](size_t cnt, size_t sz) { bytes = (size_t)round_up((int64_t)bytes, 256) + cnt * sz; };
  if (host_strain) add((size_t)n, dtype_size(sdt));
  for (int k = 0; k < p.n_levels; ++k) add((size_t)p.sup[k].size(), 4);
  size_t pp_elems = 0;
  for (const auto &sl : b->slices)
    if (sl.level > 0) {
      add((size_t)p.need[sl.level].size() * sl.lp, 4);
      for (int k = 1; k < sl.level; ++k) pp_elems = std::max(pp_elems, (size_t)p.need[k].size() * sl.lp);
    }
  add(pp_elems, 4);
  add(pp_elems, 4);
  add((size_t)n * b->kcat, esz);
  const size_t table = (size_t)F * p.n_windows;
  add(table, 4);
  add(table, 8);
  add(table, 4);
  add((size_t)F + 2, 8);
  add(1, 4);
  const int64_t dev_cap = std::min<int64_t>(trig_cap, (int64_t)table);
  add((size_t)std::max<int64_t>(dev_cap, 1), sizeof(lloid_trigger));
  if (host_snr) add((size_t)F * n * 2, 4);
  lloid_status rs = ensure_ws(b, bytes);
  if (rs != LLOID_OK) return rs;

  Carve cv{(char *)b->ws.base};
  const void *d_strain = strain;
  if (ctx->profile) HIP_TRY(hipEventRecord(ctx->ev[2 * LLOID_STAGE_INGEST], st));
  if (host_strain) {
    void *tmp = cv.take<char>((size_t)n * dtype_size(sdt));
    HIP_TRY(hipMemcpyAsync(tmp, strain, (size_t)n * dtype_size(sdt), hipMemcpyHostToDevice, st));
    d_strain = tmp;
  }
  std::vector<float *> xl(p.n_levels);
  for (int k = 0; k < p.n_levels; ++k) xl[k] = cv.take<float>((size_t)p.sup[k].size());
  std::vector<float *> olow(b->slices.size(), nullptr);
  for (size_t s = 0; s < b->slices.size(); ++s)
    if (b->slices[s].level > 0) olow[s] = cv.take<float>((size_t)p.need[b->slices[s].level].size() * b->slices[s].lp);
  float *pp[2] = {cv.take<float>(pp_elems), cv.take<float>(pp_elems)};
  void *ocat = cv.take<char>((size_t)n * b->kcat * esz);
  PeakArgs pa;
  pa.peak_snr = cv.take<float>(table);
  pa.peak_n = cv.take<int64_t>(table);
  pa.peak_phase = cv.take<float>(table);
  int64_t *counts = cv.take<int64_t>((size_t)F + 2);
  int64_t *total = counts + F;
  int *bad = cv.take<int>(1);
  lloid_trigger *dtrig = cv.take<lloid_trigger>((size_t)std::max<int64_t>(dev_cap, 1));
  float *dsnr = snr ? (host_snr ? cv.take<float>((size_t)F * n * 2) : snr) : nullptr;
  pa.snr = dsnr;
  pa.n_windows = p.n_windows;
  pa.win_p = p.win_p;
  pa.win_q = p.win_q;

  auto mark = [&](int stage, int end) -> hipError_t {
    return ctx->profile ? hipEventRecord(ctx->ev[2 * stage + end], st) : hipSuccess;
  };
  // 1. strain -> FP32 at full rate, zero outside [0, n)
  HIP_TRY(launch_fill_u8(bad, sizeof(int), st));
  HIP_TRY(launch_convert(d_strain, sdt, n, xl[0], p.sup[0].lo, p.sup[0].size(), sscale, bad, st));
  HIP_TRY(mark(LLOID_STAGE_INGEST, 1));
  // 2. half-band decimation to every level
  HIP_TRY(mark(LLOID_STAGE_DECIMATE, 0));
  for (int k = 1; k < p.n_levels; ++k)
    HIP_TRY(launch_decimate(xl[k - 1], p.sup[k - 1].lo, p.sup[k - 1].size(), xl[k], p.sup[k].lo, p.sup[k].size(),
                            ctx->d_halfband, st));
  HIP_TRY(mark(LLOID_STAGE_DECIMATE, 1));
  // 3. FIR bank per slice
  HIP_TRY(mark(LLOID_STAGE_FIR, 0));
  for (size_t s = 0; s < b->slices.size(); ++s) {
    const SliceDev &sl = b->slices[s];
    const int k = sl.level;
    if (k == 0)
      HIP_TRY(launch_fir(b->compute, sl, xl[0], p.sup[0].lo, p.sup[0].size(), 0, n, ocat, 0, b->kcat, sl.koff, sl.lp,
                         st));
    else
      HIP_TRY(launch_fir(b->compute, sl, xl[k], p.sup[k].lo, p.sup[k].size(), p.need[k].lo, p.need[k].hi, olow[s],
                         p.need[k].lo, sl.lp, 0, sl.lp, st));
  }
  HIP_TRY(mark(LLOID_STAGE_FIR, 1));
  // 4. interpolation of the low-rate orthogonal SNR to f0, into the concatenated operand
  HIP_TRY(mark(LLOID_STAGE_INTERP, 0));
  for (size_t s = 0; s < b->slices.size(); ++s) {
    const SliceDev &sl = b->slices[s];
    const int k = sl.level;
    if (k == 0) continue;
    const float *src = olow[s];
    int64_t src_lo = p.need[k].lo, src_len = p.need[k].size();
    int which = 0;
    for (int j = k - 1; j >= 0; --j) {
      if (j == 0) {
        HIP_TRY(launch_interp(LLOID_F32, src, src_lo, src_len, sl.lp, b->compute, ocat, 0, n, b->kcat, sl.koff, sl.lp,
                              ctx->d_halfband, st));
      } else {
        float *dst = pp[which];
        HIP_TRY(launch_interp(LLOID_F32, src, src_lo, src_len, sl.lp, LLOID_F32, dst, p.need[j].lo, p.need[j].size(),
                              sl.lp, 0, sl.lp, ctx->d_halfband, st));
        src = dst;
        src_lo = p.need[j].lo;
        src_len = p.need[j].size();
        which ^= 1;
      }
    }
  }
  HIP_TRY(mark(LLOID_STAGE_INTERP, 1));
  // 5. mixing GEMM + complex SNR + per-window peaks
  const float inv_scale = 1.f / (b->mix_scale * sscale);
  HIP_TRY(mark(LLOID_STAGE_MIX, 0));
  HIP_TRY(launch_mix_peak(b->compute, b->mix, b->rows, b->kcat, F, ocat, n, inv_scale, pa, st));
  HIP_TRY(mark(LLOID_STAGE_MIX, 1));
  // 6. trigger compaction
  HIP_TRY(mark(LLOID_STAGE_TRIGGER, 0));
  HIP_TRY(launch_trigger_count(pa.peak_snr, F, p.n_windows, thr, counts, st));
  HIP_TRY(launch_trigger_scan(counts, F, total, st));
  HIP_TRY(launch_trigger_write(pa.peak_snr, pa.peak_n, pa.peak_phase, F, p.n_windows, thr, counts, dev_cap, 0,
                               detector, dtrig, st));
  HIP_TRY(mark(LLOID_STAGE_TRIGGER, 1));
  HIP_TRY(mark(LLOID_STAGE_D2H, 0));
  int64_t h_total = 0;
  int h_bad = 0;
  HIP_TRY(hipMemcpyAsync(&h_total, total, sizeof h_total, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&h_bad, bad, sizeof h_bad, hipMemcpyDeviceToHost, st));
  if (peaks) {
    if (peaks->snr) HIP_TRY(hipMemcpyAsync(peaks->snr, pa.peak_snr, table * 4, hipMemcpyDefault, st));
    if (peaks->sample) HIP_TRY(hipMemcpyAsync(peaks->sample, pa.peak_n, table * 8, hipMemcpyDefault, st));
    if (peaks->phase) HIP_TRY(hipMemcpyAsync(peaks->phase, pa.peak_phase, table * 4, hipMemcpyDefault, st));
    peaks->n_windows = p.n_windows;
  }
  if (host_snr) HIP_TRY(hipMemcpyAsync(snr, dsnr, (size_t)F * n * 2 * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int64_t ncopy = std::min(h_total, dev_cap);
  if (ncopy > 0) HIP_TRY(hipMemcpyAsync(trig, dtrig, (size_t)ncopy * sizeof(lloid_trigger), hipMemcpyDefault, st));
  HIP_TRY(mark(LLOID_STAGE_D2H, 1));
  HIP_TRY(hipStreamSynchronize(st));
  if (ctx->profile) {
    for (int i = 0; i < LLOID_N_STAGES; ++i) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[2 * i], ctx->ev[2 * i + 1]));
      ctx->stage_ms[i] += ms;
      ctx->stage_calls[i] += 1;
    }
  }
  *n_trig = h_total;
  if (h_bad) return fail(LLOID_EDATA, "strain holds a non-finite sample");
  if (h_total > trig_cap) return fail(LLOID_ETRUNC, "%lld triggers, buffer holds %lld", (long long)h_total,
                                      (long long)trig_cap);
  return LLOID_OK;
  ABI_GUARD_END
}
