// Streaming (serving) form of the filtering path: strides of strain arrive per
// detector, the down-sampled strain of every rate stays resident on the device
// as the filters' history, and every tick filters the newly complete trigger
// windows of every admitted bank and detector in one launch per stage
// (continuous batching).  Banks are admitted into slots while their arrays
// and per-tick scratch fit a device-memory budget; the others wait in a queue
// and are admitted as slots are removed.  A bank admitted mid-stream reports
// from the next window on and, because the strain history is complete, its
// results equal those of an offline run over the whole stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <vector>

#include "lloid_internal.h"

using namespace lloid;

namespace {

struct DetState {
  std::vector<float *> x;      // per level: device buffer of cap[k] floats
  std::vector<int64_t> lo;     // absolute index held in x[k][0]
  std::vector<int64_t> avail;  // computed frontier (exclusive) per level
  int64_t pushed = 0;          // full-rate samples received
};

struct Slot {
  lloid_bank *bank = nullptr;
  int32_t id = -1;
  int64_t bytes = 0;
  bool active = false;
};

}  // namespace

struct lloid_stream {
  lloid_ctx *ctx = nullptr;
  int f0 = 0, n_det = 1, n_levels = 1, max_w = 8;
  lloid_dtype ct = LLOID_F16;
  Windows win;
  float thr = 4.f, sscale = 1.f;
  int64_t budget = 0, used = 0;
  int64_t win_len = 1;
  std::vector<int64_t> hist, cap;  // per level: history kept, buffer capacity
  std::vector<DetState> det;
  std::vector<Slot> slots;         // index = slot id
  std::deque<int32_t> queue;       // slot ids waiting for admission
  int64_t w_next = 0;              // next window to emit
  int64_t n_end = -1;              // data end once flushed (-1 while streaming)
  int64_t push_max = 0;            // samples converted per internal push piece
  // device scratch for ticks and staging
  Workspace ws;
  void *pinned = nullptr;
  size_t pinned_bytes = 0;
  float *level_mem = nullptr;
  void *staging = nullptr;
  int *bad = nullptr;
  // captured tick (use_graph): replayed while the key (everything the
  // launches take as arguments or sizes) is unchanged
  bool use_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int64_t> graph_key;
  int64_t *hsmall = nullptr;       // pinned: [0] trigger count, [1] low 4 bytes: non-finite flag
  int64_t graph_captures = 0, graph_replays = 0;
  // results and statistics
  std::deque<lloid_trigger> out;
  std::vector<double> lat_ms;
  int64_t strides = 0, windows = 0, triggers = 0;
  std::chrono::steady_clock::time_point last_push;
};

namespace {

int64_t tick_samples(const lloid_stream *s) { return s->max_w * s->win_len + 1; }

// Samples at level k that a tick's operand margins (up to kMaxAutocorrHalf
// on each side) reach beyond the tick and the filter span.
int64_t margin_at(int k) { return ((2 * (int64_t)kMaxAutocorrHalf + 2) >> k) + 1; }

// device bytes one active bank needs beyond its own arrays: per-tick scratch of every detector
int64_t scratch_bytes(const lloid_stream *s, const lloid_bank *b) {
  const int64_t ts = tick_samples(s) + 2 * operand_margin(b);
  int64_t per = (int64_t)ts * b->kcat * (int64_t)dtype_size(b->compute);
  for (const auto &sl : b->slices)
    if (sl.level > 0)
      for (int64_t ld : low_ld(ts, sl.level)) per += (int64_t)sl.lp * ld * (int64_t)low_esz(b->compute) + 256;
  per += (int64_t)b->n_templates * s->max_w * (36 + (int64_t)sizeof(lloid_trigger)) + 4096;
  return per * s->n_det;
}

lloid_status check_bank(const lloid_stream *s, const lloid_bank *b) {
  if (!b) return fail(LLOID_EINVAL, "NULL bank");
  if (b->ctx != s->ctx) return fail(LLOID_EINVAL, "the bank belongs to another context");
  if (b->f0 != s->f0) return fail(LLOID_EINVAL, "the bank's full rate differs from the stream's");
  if (b->compute != s->ct) return fail(LLOID_EINVAL, "the bank's compute type differs from the stream's");
  if (b->n_levels > s->n_levels) return fail(LLOID_EINVAL, "the bank's lowest rate is below the stream's");
  if (!operands_fit(b, tick_samples(s) + 2 * operand_margin(b)))
    return fail(LLOID_EINVAL, "the bank's per-tick buffers exceed 2 GiB");
  for (const auto &sl : b->slices) {
    const int64_t span = sl.start_tap / sl.dec + sl.n_taps + 4 * kHalfQ;
    if (span > s->hist[sl.level]) return fail(LLOID_EINVAL, "a slice spans more than the stream's history");
  }
  return LLOID_OK;
}

// admit queued banks in arrival order while they fit the budget
void admit_queued(lloid_stream *s) {
  while (!s->queue.empty()) {
    Slot &q = s->slots[s->queue.front()];
    if (s->budget > 0 && s->used + q.bytes > s->budget) break;
    s->used += q.bytes;
    q.active = true;
    s->queue.pop_front();
  }
}

// Make room for `add` more samples at level k of detector d (keep the history).
lloid_status make_room(lloid_stream *s, DetState &d, int k, int64_t add) {
  const int64_t end = d.avail[k] + add;
  if (end - d.lo[k] <= s->cap[k]) return LLOID_OK;
  const int64_t keep_from =
      d.avail[k] - s->hist[k] - tick_samples(s) / (int64_t(1) << k) - 4 * kHalfQ - margin_at(k);
  const int64_t shift = keep_from - d.lo[k];
  const int64_t keep = d.avail[k] - keep_from;
  if (shift < keep || end - keep_from > s->cap[k])
    return fail(LLOID_EINVAL, "stream level buffer too small for this push");
  HIP_TRY(hipMemcpyAsync(d.x[k], d.x[k] + shift, (size_t)keep * 4, hipMemcpyDeviceToDevice, s->ctx->stream));
  d.lo[k] = keep_from;
  return LLOID_OK;
}

// Extend every level of detector d to the samples its inputs now allow.
lloid_status decimate_new(lloid_stream *s, DetState &d) {
  for (int k = 1; k < s->n_levels; ++k) {
    // sample i needs level k-1 up to 2i + Q
    const int64_t top = floor_div(d.avail[k - 1] - 1 - kHalfQ, 2) + 1;
    if (top <= d.avail[k]) continue;
    const lloid_status r = make_room(s, d, k, top - d.avail[k]);
    if (r != LLOID_OK) return r;
    HIP_TRY(launch_decimate(d.x[k - 1], d.lo[k - 1], d.avail[k - 1] - d.lo[k - 1], d.x[k] + (d.avail[k] - d.lo[k]),
                            d.avail[k], top - d.avail[k], s->ctx->d_halfband, s->ctx->stream));
    d.avail[k] = top;
  }
  return LLOID_OK;
}

// Largest window end wb (> w_next) whose outputs every active bank can compute now.
int64_t ready_until(const lloid_stream *s) {
  int64_t data_end = INT64_MAX;
  for (const auto &d : s->det) data_end = std::min(data_end, d.pushed);
  if (s->n_end >= 0) data_end = s->n_end;
  int64_t best = s->w_next;
  for (int64_t wb = s->w_next + 1; wb <= s->w_next + s->max_w; ++wb) {
    const int64_t t0 = s->win.start(s->w_next);
    int64_t t1 = s->win.start(wb);
    if (s->n_end >= 0) {
      if (t0 >= s->n_end) break;
      t1 = std::min(t1, s->n_end);
    } else if (t1 > data_end) {
      break;
    }
    bool ok = true;
    for (const auto &sl : s->slots) {
      if (!sl.active || !ok) continue;
      const int64_t mg = operand_margin(sl.bank);
      for (const auto &sd : sl.bank->slices) {
        // outputs [t0 - mg, t1 + mg): the peaks' sub-sample refinement and
        // signal-consistency lags read up to mg samples past t1
        const Range r = need_ranges(t0 - mg, t1 + mg, sd.level + 1)[sd.level];
        for (const auto &d : s->det)
          if (r.hi - sd.start_tap / sd.dec > d.avail[sd.level]) ok = false;
      }
    }
    if (!ok) break;
    best = wb;
    if (s->n_end >= 0 && t1 >= s->n_end) break;
  }
  return best;
}

// Filter windows [wa, wb) for every active bank and detector; triggers to the host queue.
lloid_status run_tick(lloid_stream *s, int64_t wa, int64_t wb) {
  lloid_ctx *ctx = s->ctx;
  hipStream_t st = ctx->stream;
  const int64_t t0 = s->win.start(wa);
  int64_t t1 = s->win.start(wb);
  const int64_t n_end = s->n_end >= 0 ? s->n_end : INT64_MAX / 4;
  t1 = std::min(t1, n_end);
  const int64_t nw = wb - wa;
  std::vector<int> act;
  for (size_t i = 0; i < s->slots.size(); ++i)
    if (s->slots[i].active) act.push_back((int)i);
  s->w_next = wb;
  s->windows += nw;
  if (act.empty()) return LLOID_OK;
  const TileShapes ts(s->ct, ctx->fir_variant, ctx->mix_variant);
  const size_t esz = dtype_size(s->ct);
  const int64_t tlen = t1 - t0;
  // scratch layout
  size_t bytes = 0;
  auto add = [&](size_t cnt, size_t sz) { bytes = (size_t)round_up((int64_t)bytes, 256) + cnt * sz; };
  int64_t rows = 0;
  size_t n_fir = 0, n_up = 0;
  for (int i : act) {
    const lloid_bank *b = s->slots[i].bank;
    for (int d = 0; d < s->n_det; ++d) {
      const int64_t ops = tlen + 2 * operand_margin(b);
      add((size_t)ops * b->kcat, esz);
      for (const auto &sl : b->slices) {
        ++n_fir;
        if (sl.level > 0)
          for (int64_t ld : low_ld(ops, sl.level)) add((size_t)sl.lp * ld, low_esz(s->ct)), ++n_up;
      }
      add((size_t)b->n_templates * nw, 4);
      add((size_t)b->n_templates * nw, 4);
      add((size_t)b->n_templates * nw, 8);
      add((size_t)b->n_templates * nw, 4);
      add((size_t)b->n_templates * nw, 4);
      add((size_t)b->n_templates * nw, 4);
      add((size_t)b->n_templates * nw, 8);
    }
    rows += (int64_t)b->n_templates * s->n_det;
  }
  add((size_t)trig_blocks(rows * nw) + 2, 8);
  add((size_t)rows * nw, sizeof(lloid_trigger));
  const size_t tab_bytes = n_fir * sizeof(FirJob) + n_up * sizeof(UpJob) +
                           act.size() * s->n_det * (sizeof(MixJob) + sizeof(TrigJob)) + 64 * (4 + kMaxHops);
  add(tab_bytes, 1);
  lloid_status rs = ensure_ws(ctx, s->ws, bytes);
  if (rs != LLOID_OK) return rs;
  rs = ensure_pinned(ctx, s->pinned, s->pinned_bytes, tab_bytes);
  if (rs != LLOID_OK) return rs;
  Carve cv{(char *)s->ws.base};
  std::vector<FirJob> fj;
  std::vector<UpJob> uj[kMaxHops];
  std::vector<MixJob> mj;
  std::vector<TrigJob> tj;
  int64_t row = 0;
  for (int i : act) {
    const lloid_bank *b = s->slots[i].bank;
    for (int d = 0; d < s->n_det; ++d) {
      BankBufs bb;
      const int64_t ops = tlen + 2 * operand_margin(b);
      bb.ocat = cv.take<char>((size_t)ops * b->kcat * esz);
      bb.low.assign(b->slices.size(), {});
      for (size_t k = 0; k < b->slices.size(); ++k)
        if (b->slices[k].level > 0)
          for (int64_t ld : low_ld(ops, b->slices[k].level))
            bb.low[k].push_back(cv.take<char>((size_t)b->slices[k].lp * ld * low_esz(s->ct)));
      bb.psnr = cv.take<float>((size_t)b->n_templates * nw);
      bb.pn = cv.take<int64_t>((size_t)b->n_templates * nw);
      bb.pphase = cv.take<float>((size_t)b->n_templates * nw);
      bb.pdt = cv.take<float>((size_t)b->n_templates * nw);
      bb.psi = cv.take<float>((size_t)b->n_templates * nw);
      bb.pxi = cv.take<float>((size_t)b->n_templates * nw);
      bb.pz = cv.take<float2>((size_t)b->n_templates * nw);
      bb.ld_peak = nw;
      bb.w_base = wa;
      std::vector<LevelView> lv(s->n_levels);
      const DetState &ds = s->det[d];
      for (int k = 0; k < s->n_levels; ++k) lv[k] = LevelView{ds.x[k], ds.lo[k], ds.avail[k] - ds.lo[k]};
      add_bank_jobs(b, lv.data(), t0, t1, n_end, wa, wb, s->win, bb, 1.f / (b->mix_scale * s->sscale), nullptr, 0, ts,
                    fj, uj, mj);
      tj.push_back(TrigJob{bb.psnr, bb.pn, bb.pphase, bb.pdt, bb.psi, b->acorr ? bb.pxi : nullptr, wa, nw, row * nw,
                           b->n_templates, s->slots[i].id, d, 0});
      row += b->n_templates;
    }
  }
  const int64_t n_blk = trig_blocks(rows * nw);
  int64_t *counts = cv.take<int64_t>((size_t)n_blk + 2);
  int64_t *total = counts + n_blk;
  const int64_t cap = rows * nw;
  lloid_trigger *dtrig = cv.take<lloid_trigger>((size_t)std::max<int64_t>(cap, 1));
  char *dtab = cv.take<char>(tab_bytes);
  StageItems items;
  number_jobs(fj, uj, mj, items);
  char *htab = (char *)s->pinned;
  size_t off = 0;
  auto put = [&](const void *src, size_t sz) -> size_t {
    off = (size_t)round_up((int64_t)off, 64);
    const size_t at = off;
    if (sz) std::memcpy(htab + off, src, sz);
    off += sz;
    return at;
  };
  TabOffsets to;
  to.fir = put(fj.data(), fj.size() * sizeof(FirJob));
  for (int h = 0; h < kMaxHops; ++h) {
    to.up[h] = put(uj[h].data(), uj[h].size() * sizeof(UpJob));
    to.n_up[h] = (int)uj[h].size();
  }
  to.mix = put(mj.data(), mj.size() * sizeof(MixJob));
  to.n_fir = (int)fj.size();
  to.n_mix = (int)mj.size();
  const size_t trig_off = put(tj.data(), tj.size() * sizeof(TrigJob));
  // the tick's device work: table upload, every stage, trigger count and the
  // two small results into pinned host memory
  auto enqueue = [&]() -> lloid_status {
    HIP_TRY(hipMemcpyAsync(dtab, htab, off, hipMemcpyHostToDevice, st));
    const lloid_status r = launch_stages(ctx, s->ct, dtab, to, items, false, s->thr, s->thr, nullptr);
    if (r != LLOID_OK) return r;
    HIP_TRY(launch_trigger_jobs((const TrigJob *)(dtab + trig_off), (int)tj.size(), rows * nw, s->thr, counts, total,
                                cap, dtrig, st));
    HIP_TRY(hipMemcpyAsync(s->hsmall, total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(s->hsmall + 1, s->bad, sizeof(int), hipMemcpyDeviceToHost, st));
    return LLOID_OK;
  };
  if (s->use_graph) {
    std::vector<int64_t> key = {(int64_t)(uintptr_t)dtab, (int64_t)(uintptr_t)htab, (int64_t)off, (int64_t)trig_off,
                                (int64_t)tj.size(), rows, cap, (int64_t)(uintptr_t)counts, (int64_t)(uintptr_t)dtrig,
                                items.fir, items.mix, items.entries, (int64_t)to.fir, (int64_t)to.mix, to.n_fir,
                                to.n_mix};
    key.push_back(items.xi2 ? 1 : 0);
    key.push_back(ctx->fir_variant * 16 + ctx->mix_variant);
    key.push_back(items.windows);
    for (int h = 0; h < kMaxHops; ++h) {
      key.push_back(items.up[h]);
      key.push_back((int64_t)to.up[h]);
      key.push_back(to.n_up[h]);
    }
    if (!s->exec || key != s->graph_key) {
      if (s->exec) (void)hipGraphExecDestroy(s->exec), s->exec = nullptr;
      if (s->graph) (void)hipGraphDestroy(s->graph), s->graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      const lloid_status r = enqueue();
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(st, &g);
      if (r != LLOID_OK) {
        if (ec == hipSuccess && g) (void)hipGraphDestroy(g);
        return r;
      }
      HIP_TRY(ec);
      s->graph = g;
      HIP_TRY(hipGraphInstantiate(&s->exec, g, nullptr, nullptr, 0));
      s->graph_key = key;
      ++s->graph_captures;
    } else {
      ++s->graph_replays;
    }
    HIP_TRY(hipGraphLaunch(s->exec, st));
  } else {
    rs = enqueue();
    if (rs != LLOID_OK) return rs;
  }
  HIP_TRY(hipStreamSynchronize(st));
  const int64_t h_total = s->hsmall[0];
  const int h_bad = *(const int *)(s->hsmall + 1);
  if (h_total > 0) {
    const size_t at = s->out.size();
    s->out.resize(at + (size_t)h_total);
    std::vector<lloid_trigger> tmp((size_t)h_total);
    HIP_TRY(hipMemcpyAsync(tmp.data(), dtrig, (size_t)h_total * sizeof(lloid_trigger), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::copy(tmp.begin(), tmp.end(), s->out.begin() + at);
  }
  s->triggers += h_total;
  s->strides += 1;
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - s->last_push).count();
  s->lat_ms.push_back(ms);
  if (h_bad) return fail(LLOID_EDATA, "strain holds a non-finite sample");
  return LLOID_OK;
}

lloid_status run_ready(lloid_stream *s) {
  for (;;) {
    const int64_t wb = ready_until(s);
    if (wb <= s->w_next) return LLOID_OK;
    admit_queued(s);
    const lloid_status r = run_tick(s, s->w_next, wb);
    if (r != LLOID_OK) return r;
  }
}

// Append n converted samples to level 0 of detector d and extend the other levels.
lloid_status append(lloid_stream *s, int d, const void *data, lloid_dtype dt, int64_t n, bool zeros) {
  DetState &ds = s->det[d];
  int64_t done = 0;
  while (done < n) {
    const int64_t m = std::min(n - done, s->push_max);
    lloid_status r = make_room(s, ds, 0, m);
    if (r != LLOID_OK) return r;
    float *dst = ds.x[0] + (ds.avail[0] - ds.lo[0]);
    if (zeros) {
      HIP_TRY(launch_fill_u8(dst, (size_t)m * 4, s->ctx->stream));
    } else {
      const size_t esz = dtype_size(dt);
      const char *src = (const char *)data + done * esz;
      const void *dsrc = src;
      if (!is_device_ptr(src)) {
        HIP_TRY(hipMemcpyAsync(s->staging, src, (size_t)m * esz, hipMemcpyHostToDevice, s->ctx->stream));
        dsrc = s->staging;
      }
      HIP_TRY(launch_convert(dsrc, dt, m, dst, 0, m, s->sscale, s->bad, s->ctx->stream));
    }
    ds.avail[0] += m;
    ds.pushed = ds.avail[0];
    r = decimate_new(s, ds);
    if (r != LLOID_OK) return r;
    done += m;
  }
  return LLOID_OK;
}

}  // namespace

extern "C" lloid_status lloid_stream_create(lloid_ctx *ctx, int32_t full_rate_hz, lloid_dtype compute,
                                            const lloid_stream_opts *opts, lloid_stream **out) {
  ABI_GUARD_BEGIN
  if (!ctx || !out || !opts) return fail(LLOID_EINVAL, "NULL argument");
  *out = nullptr;
  if (full_rate_hz <= 0) return fail(LLOID_EINVAL, "full rate must be positive");
  if (compute != LLOID_F32 && compute != LLOID_F16 && compute != LLOID_BF16)
    return fail(LLOID_EINVAL, "compute type must be F32, F16 or BF16");
  if (opts->n_detectors < 1 || opts->n_detectors > 16) return fail(LLOID_EINVAL, "1 to 16 detectors");
  if (opts->min_rate_hz <= 0 || full_rate_hz % opts->min_rate_hz || (full_rate_hz / opts->min_rate_hz) & ((full_rate_hz / opts->min_rate_hz) - 1))
    return fail(LLOID_EINVAL, "min_rate_hz must be the full rate over a power of two");
  const lloid_trigger_opts &t = opts->trig;
  if (t.window_num <= 0 || t.window_den <= 0 || (int64_t)full_rate_hz * t.window_num < t.window_den)
    return fail(LLOID_EINVAL, "bad window length");
  const float sscale = t.strain_scale != 0.f ? t.strain_scale : 1.f;
  {
    int e;
    if (!(sscale > 0.f) || std::frexp((double)sscale, &e) != 0.5)
      return fail(LLOID_EINVAL, "strain_scale must be a power of two");
  }
  HIP_TRY(hipSetDevice(ctx->device));
  lloid_stream *s = new lloid_stream();
  s->ctx = ctx;
  s->f0 = full_rate_hz;
  s->ct = compute;
  s->n_det = opts->n_detectors;
  s->win = Windows{(int64_t)full_rate_hz * t.window_num, t.window_den};
  s->win_len = ceil_div(s->win.p, s->win.q);
  s->thr = t.threshold;
  s->sscale = sscale;
  s->budget = opts->hbm_budget;
  s->max_w = opts->max_windows_per_tick > 0 ? opts->max_windows_per_tick : 8;
  s->use_graph = opts->use_graph != 0;
  int L = 1;
  while ((full_rate_hz >> (L - 1)) > opts->min_rate_hz) ++L;
  s->n_levels = L;
  const double span_s = opts->max_filter_s > 0 ? opts->max_filter_s : 66.0;
  s->push_max = std::max<int64_t>(tick_samples(s), full_rate_hz);
  s->hist.resize(L);
  s->cap.resize(L);
  size_t total = 0;
  for (int k = 0; k < L; ++k) {
    const int64_t rate = full_rate_hz >> k;
    s->hist[k] = (int64_t)std::ceil(span_s * rate) + 8 * kHalfQ;
    const int64_t tick_k = tick_samples(s) / (int64_t(1) << k) + 8 * kHalfQ + margin_at(k);
    const int64_t push_k = s->push_max / (int64_t(1) << k) + 8 * kHalfQ;
    s->cap[k] = 2 * (s->hist[k] + tick_k) + push_k;
    total += (size_t)s->cap[k];
  }
  const size_t lbytes = total * 4 * s->n_det;
  if (hipMalloc((void **)&s->level_mem, lbytes) != hipSuccess ||
      hipMalloc(&s->staging, (size_t)s->push_max * 8) != hipSuccess || hipMalloc((void **)&s->bad, 256) != hipSuccess ||
      hipHostMalloc((void **)&s->hsmall, 2 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    lloid_stream_destroy(s);
    return fail(LLOID_ENOMEM, "stream buffers do not fit on the device");
  }
  s->det.resize(s->n_det);
  float *p = s->level_mem;
  for (auto &d : s->det) {
    d.x.resize(L);
    d.lo.resize(L);
    d.avail.resize(L);
    int64_t sup_lo = 0;
    for (int k = 0; k < L; ++k) {
      d.x[k] = p;
      p += s->cap[k];
      if (k > 0) sup_lo = ceil_div(sup_lo - kHalfQ, 2);
      // before its support a level is exactly zero: the history starts as zeros
      d.lo[k] = sup_lo - s->hist[k] - 8 * kHalfQ - margin_at(k);
      d.avail[k] = sup_lo;
    }
  }
  if (launch_fill_u8(s->level_mem, lbytes, ctx->stream) != hipSuccess ||
      launch_fill_u8(s->bad, 4, ctx->stream) != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess) {
    lloid_stream_destroy(s);
    return fail(LLOID_EDEVICE, "stream initialisation failed");
  }
  *out = s;
  return LLOID_OK;
  ABI_GUARD_END
}

extern "C" lloid_status lloid_stream_admit(lloid_stream *s, lloid_bank *bank, int32_t *slot) {
  ABI_GUARD_BEGIN
  if (!s || !slot) return fail(LLOID_EINVAL, "NULL argument");
  lloid_status r = check_bank(s, bank);
  if (r != LLOID_OK) return r;
  Slot sl;
  sl.bank = bank;
  sl.id = (int32_t)s->slots.size();
  sl.bytes = bank->device_bytes + scratch_bytes(s, bank);
  if (s->budget > 0 && sl.bytes > s->budget) return fail(LLOID_ENOMEM, "the bank alone exceeds the stream's budget");
  s->slots.push_back(sl);
  s->queue.push_back(sl.id);
  admit_queued(s);
  *slot = sl.id;
  if (!s->slots[sl.id].active) return fail(LLOID_EAGAIN, "queued until device memory frees up");
  return LLOID_OK;
  ABI_GUARD_END
}

extern "C" lloid_status lloid_stream_remove(lloid_stream *s, int32_t slot) {
  ABI_GUARD_BEGIN
  if (!s || slot < 0 || slot >= (int32_t)s->slots.size() || !s->slots[slot].bank)
    return fail(LLOID_EINVAL, "no such slot");
  Slot &sl = s->slots[slot];
  if (sl.active) s->used -= sl.bytes;
  else s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), slot), s->queue.end());
  sl.active = false;
  sl.bank = nullptr;
  admit_queued(s);
  return LLOID_OK;
  ABI_GUARD_END
}

extern "C" lloid_status lloid_stream_push(lloid_stream *s, int32_t detector, int64_t t0, const void *data,
                                          lloid_dtype dt, int64_t n) {
  ABI_GUARD_BEGIN
  if (!s) return fail(LLOID_EINVAL, "NULL stream");
  if (detector < 0 || detector >= s->n_det) return fail(LLOID_EINVAL, "no such detector");
  if (s->n_end >= 0) return fail(LLOID_EORDER, "the stream was flushed");
  if (n < 0 || (n > 0 && !data)) return fail(LLOID_EINVAL, "bad stride");
  if (dt != LLOID_F64 && dt != LLOID_F32) return fail(LLOID_EINVAL, "strain must be F64 or F32");
  if (t0 != s->det[detector].pushed)
    return fail(LLOID_EORDER, "stride starts at %lld, expected %lld", (long long)t0, (long long)s->det[detector].pushed);
  s->last_push = std::chrono::steady_clock::now();
  HIP_TRY(hipSetDevice(s->ctx->device));
  lloid_status r = append(s, detector, data, dt, n, false);
  if (r != LLOID_OK) return r;
  return run_ready(s);
  ABI_GUARD_END
}

extern "C" lloid_status lloid_stream_flush(lloid_stream *s) {
  ABI_GUARD_BEGIN
  if (!s) return fail(LLOID_EINVAL, "NULL stream");
  if (s->n_end >= 0) return LLOID_OK;
  int64_t end = s->det[0].pushed;
  for (const auto &d : s->det)
    if (d.pushed != end) return fail(LLOID_EORDER, "detectors hold different amounts of strain");
  s->last_push = std::chrono::steady_clock::now();
  // zero strain past the end feeds the resamplers' look-ahead, as in lloid_filter
  const int64_t pad = (int64_t)(8 * kHalfQ) << s->n_levels;
  for (int d = 0; d < s->n_det; ++d) {
    lloid_status r = append(s, d, nullptr, LLOID_F32, pad, true);
    if (r != LLOID_OK) return r;
  }
  s->n_end = end;
  return run_ready(s);
  ABI_GUARD_END
}

extern "C" lloid_status lloid_stream_poll(lloid_stream *s, lloid_trigger *out, int64_t cap, int64_t *n_out) {
  if (!s || !n_out || cap < 0 || (cap > 0 && !out)) return fail(LLOID_EINVAL, "bad argument");
  const int64_t m = std::min<int64_t>(cap, (int64_t)s->out.size());
  std::copy(s->out.begin(), s->out.begin() + m, out);
  s->out.erase(s->out.begin(), s->out.begin() + m);
  *n_out = m;
  return LLOID_OK;
}

extern "C" lloid_status lloid_stream_stats_get(const lloid_stream *s, lloid_stream_stats *out) {
  if (!s || !out) return fail(LLOID_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof *out);
  out->ticks = s->strides;
  out->windows = s->windows;
  out->triggers = s->triggers;
  out->next_window = s->w_next;
  std::vector<double> v = s->lat_ms;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto q = [&](double f) { return v[std::min(v.size() - 1, (size_t)std::floor(f * (double)(v.size() - 1) + 0.5))]; };
    out->latency_p50_ms = q(0.50);
    out->latency_p99_ms = q(0.99);
    out->latency_max_ms = v.back();
  }
  for (const auto &sl : s->slots)
    if (sl.bank) (sl.active ? out->active_slots : out->queued_banks) += 1;
  out->bytes_in_use = s->used;
  out->graph_captures = s->graph_captures;
  out->graph_replays = s->graph_replays;
  return LLOID_OK;
}

extern "C" lloid_status lloid_stream_destroy(lloid_stream *s) {
  if (!s) return LLOID_OK;
  (void)hipSetDevice(s->ctx->device);
  (void)hipStreamSynchronize(s->ctx->stream);
  if (s->level_mem) (void)hipFree(s->level_mem);
  if (s->staging) (void)hipFree(s->staging);
  if (s->bad) (void)hipFree(s->bad);
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  if (s->hsmall) (void)hipHostFree(s->hsmall);
  if (s->ws.base) (void)hipFree(s->ws.base);
  if (s->pinned) (void)hipHostFree(s->pinned);
  delete s;
  return LLOID_OK;
}
