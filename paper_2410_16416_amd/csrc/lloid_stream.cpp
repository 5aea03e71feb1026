// Streaming (serving) form of the filtering path: strides of strain arrive per
// detector, the down-sampled strain of every rate stays resident on the device
// as the filters' history, and every tick filters the newly complete trigger
// windows of every admitted bank and detector in one launch per stage
// (continuous batching).  Banks are admitted into slots while their arrays
// and per-tick scratch fit a device-memory budget; the others wait in a queue
// and are admitted as slots are removed.  A bank admitted mid-stream reports
// from the next window on and, because the strain history is complete, its
// results equal those of an offline run over the whole stream.
//
// Threads and streams.  lloid_stream_push only checks a stride and copies it
// into a ring of staging slots (pinned host, or device for device strides),
// then returns.  A submitter thread takes the strides in order: it uploads,
// converts and decimates each on the ingest stream, and whenever whole
// windows are computable it builds the next tick's descriptor tables and
// enqueues the tick on the compute stream (the context's), behind an event
// of the ingest work it needs, without waiting for it.  A completer thread
// waits for each tick's completion event in order and publishes its triggers,
// which the trigger kernel writes straight into pinned host memory of the
// tick's ring entry.  So the ingest and table building of stride N + 1 overlap
// the device work of tick N.  Both streams have the default priority.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lloid_internal.h"

using namespace lloid;

namespace {

using Clock = std::chrono::steady_clock;

struct DetState {
  std::vector<float *> x;      // per level: device buffer of cap[k] floats
  std::vector<int64_t> lo;     // absolute index held in x[k][0]
  std::vector<int64_t> avail;  // computed frontier (exclusive) per level
  int64_t pushed = 0;          // full-rate samples ingested by the submitter
};

// One staging entry of the stride ring: a stride's samples on their way to
// the device (host strides in pinned memory, device strides already copied
// to device memory).
struct Staging {
  void *host = nullptr;        // pinned, push_max * 8 bytes
  void *dev = nullptr;         // device, push_max * 8 bytes
};

// A unit of work for the submitter, in push order.
struct Item {
  enum Kind { kStride, kFlush } kind = kStride;
  int det = 0;
  int64_t t0 = 0, n = 0;
  lloid_dtype dt = LLOID_F32;
  int ring = -1;               // staging entry
  bool on_device = false;      // samples in Staging::dev (else Staging::host)
  Clock::time_point pushed_at;
};

// Device and host resources of one tick in flight.
struct TickSlot {
  void *htab = nullptr;        // pinned descriptor tables
  size_t htab_bytes = 0;
  lloid_trigger *htrig = nullptr;  // pinned: the trigger kernel's output
  int64_t htrig_cap = 0;
  int64_t *hcount = nullptr;   // pinned: trigger count of the tick
  hipEvent_t done = nullptr;
  hipGraph_t graph = nullptr;  // use_graph: the captured tick of this entry
  hipGraphExec_t exec = nullptr;
  std::vector<int64_t> graph_key;
  // the tick in flight
  bool busy = false;
  uint64_t seq = 0;
  Clock::time_point ready_at;  // push of the stride that completed the tick
};

constexpr int kTickRing = 3;   // ticks in flight at most

}  // namespace

struct lloid_stream {
  lloid_ctx *ctx = nullptr;
  int f0 = 0, n_det = 1, n_levels = 1, max_w = 8;
  lloid_dtype ct = LLOID_F16;
  Windows win;
  float thr = 4.f, sscale = 1.f;
  int64_t win_len = 1;
  std::vector<int64_t> hist, cap;  // per level: history kept, buffer capacity
  std::vector<DetState> det;
  Admission adm;                   // slots: device-memory budget, arrival-order queue
  std::vector<lloid_bank *> bank_of;   // per slot id (NULL once removed)
  int64_t w_next = 0;              // next window to enqueue
  int64_t n_end = -1;              // data end once flushed (-1 while streaming)
  int64_t push_max = 0;            // samples per staging entry
  std::vector<int64_t> accepted;   // per detector: samples accepted by push
  bool flushed = false;            // lloid_stream_flush was called
  // device memory
  float *level_mem = nullptr;
  int *bad = nullptr;              // device flags: [0] the device-stride check in push, [32] the
                                   // submitter's conversions (never set: strides are checked first)
  float *check_buf = nullptr;      // device: converted copy of a device stride (check only)
  int *hbad = nullptr;             // pinned copy of the flag
  Workspace ws;                    // per-tick scratch + kTickRing device table areas
  size_t tab_area = 0;             // bytes of each device table area at the end of ws
  hipStream_t ingest = nullptr;    // uploads, conversion, decimation
  hipStream_t staging_stream = nullptr;  // device strides: copy and check in push
  hipEvent_t ingest_done = nullptr;
  // stride ring
  std::vector<Staging> ring;
  std::vector<int> ring_free;
  // ticks in flight
  TickSlot ticks[kTickRing];
  uint64_t seq_enqueued = 0, seq_completed = 0;
  std::deque<int> inflight;        // tick ring entries in enqueue order
  bool use_graph = false;
  int64_t graph_captures = 0, graph_replays = 0;
  // threads
  mutable std::mutex mu;
  std::condition_variable cv_sub;   // submitter: items or stop
  std::condition_variable cv_comp;  // completer: ticks in flight or stop
  std::condition_variable cv_done;  // callers: progress
  std::deque<Item> inbox;
  bool sub_busy = false;            // the submitter holds an item
  bool stop = false;
  std::thread submitter, completer;
  lloid_status error = LLOID_OK;    // first failure of a thread, returned by the next call
  std::string error_msg;
  // results and statistics
  std::deque<lloid_trigger> out;
  std::vector<double> lat_ms;
  int64_t ticks_run = 0, windows = 0, triggers = 0;
};

namespace {

int64_t tick_samples(const lloid_stream *s) { return s->max_w * s->win_len + 1; }

// Samples at level k that a tick's operand margins (up to kMaxAutocorrHalf
// on each side) reach beyond the tick and the filter span.
int64_t margin_at(int k) { return ((2 * (int64_t)kMaxAutocorrHalf + 2) >> k) + 1; }

// device bytes one active bank needs beyond its own arrays: per-tick scratch of every detector
int64_t scratch_bytes(const lloid_stream *s, const lloid_bank *b) {
  const int64_t ts = tick_samples(s) + 2 * operand_margin(b);
  int64_t per = (int64_t)ts * b->kld * (int64_t)dtype_size(b->compute);
  for (const auto &sl : b->slices)
    if (sl.level > 0)
      for (int64_t ld : low_ld(ts, sl.level)) per += (int64_t)sl.lp * ld * (int64_t)low_esz(b->compute) + 256;
  per += (int64_t)b->n_templates * s->max_w * 36 + 4096;
  return per * s->n_det;
}

lloid_status check_bank(const lloid_stream *s, const lloid_bank *b) {
  if (!b) return fail(LLOID_EINVAL, "NULL bank");
  if (b->ctx != s->ctx) return fail(LLOID_EINVAL, "the bank belongs to another context");
  if (b->f0 != s->f0) return fail(LLOID_EINVAL, "the bank's full rate differs from the stream's");
  if (b->compute != s->ct) return fail(LLOID_EINVAL, "the bank's compute type differs from the stream's");
  if (b->n_levels > s->n_levels) return fail(LLOID_EINVAL, "the bank's lowest rate is below the stream's");
  if (!operands_fit(b, tick_samples(s) + 2 * operand_margin(b), s->win_len))
    return fail(LLOID_EINVAL, "the bank's per-tick buffers exceed 2 GiB");
  for (const auto &sl : b->slices) {
    const int64_t span = sl.start_tap / sl.dec + sl.n_taps + 4 * kHalfQ;
    if (span > s->hist[sl.level]) return fail(LLOID_EINVAL, "a slice spans more than the stream's history");
  }
  return LLOID_OK;
}

// Record the first failure of a worker thread (lock held); later calls return it.
void set_error(lloid_stream *s, lloid_status st) {
  if (s->error == LLOID_OK) {
    s->error = st;
    s->error_msg = lloid_last_error();
  }
  s->cv_done.notify_all();
}

// The stored failure, raised on the calling thread (lock held).
lloid_status stored_error(const lloid_stream *s) {
  if (s->error == LLOID_OK) return LLOID_OK;
  return fail(s->error, "%s", s->error_msg.c_str());
}

// Wait (lock held) until the submitter has taken and processed every item
// queued so far.
void wait_submitted(lloid_stream *s, std::unique_lock<std::mutex> &lk) {
  s->cv_done.wait(lk, [&] { return (s->inbox.empty() && !s->sub_busy) || s->error != LLOID_OK; });
}

// Wait (lock held) until every tick enqueued so far has completed.
void wait_completed(lloid_stream *s, std::unique_lock<std::mutex> &lk) {
  const uint64_t target = s->seq_enqueued;
  s->cv_done.wait(lk, [&] { return s->seq_completed >= target || s->error != LLOID_OK; });
}

// ------------------------------------------------------------ submitter side
// The functions below run on the submitter thread only (they touch the level
// buffers and the tick ring without the lock, except where noted).

// Make room for `add` more samples at level k of detector d (keep the history).
// A shift moves data that ticks in flight may read: the ingest stream waits
// for the last enqueued tick first.
lloid_status make_room(lloid_stream *s, DetState &d, int k, int64_t add, const TickSlot *last) {
  const int64_t end = d.avail[k] + add;
  if (end - d.lo[k] <= s->cap[k]) return LLOID_OK;
  const int64_t keep_from =
      d.avail[k] - s->hist[k] - tick_samples(s) / (int64_t(1) << k) - 4 * kHalfQ - margin_at(k);
  const int64_t shift = keep_from - d.lo[k];
  const int64_t keep = d.avail[k] - keep_from;
  if (shift < keep || end - keep_from > s->cap[k])
    return fail(LLOID_EINVAL, "stream level buffer too small for this push");
  if (last) HIP_TRY(hipStreamWaitEvent(s->ingest, last->done, 0));
  HIP_TRY(hipMemcpyAsync(d.x[k], d.x[k] + shift, (size_t)keep * 4, hipMemcpyDeviceToDevice, s->ingest));
  d.lo[k] = keep_from;
  return LLOID_OK;
}

// Extend every level of detector d to the samples its inputs now allow.
lloid_status decimate_new(lloid_stream *s, DetState &d, const TickSlot *last) {
  for (int k = 1; k < s->n_levels; ++k) {
    // sample i needs level k-1 up to 2i + Q
    const int64_t top = floor_div(d.avail[k - 1] - 1 - kHalfQ, 2) + 1;
    if (top <= d.avail[k]) continue;
    const lloid_status r = make_room(s, d, k, top - d.avail[k], last);
    if (r != LLOID_OK) return r;
    HIP_TRY(launch_decimate(d.x[k - 1], d.lo[k - 1], d.avail[k - 1] - d.lo[k - 1], d.x[k] + (d.avail[k] - d.lo[k]),
                            d.avail[k], top - d.avail[k], s->ctx->d_halfband, s->ingest));
    d.avail[k] = top;
  }
  return LLOID_OK;
}

// Append n samples (a device buffer of type dt, or zeros when src is NULL) to
// level 0 of detector d and extend the other levels, on the ingest stream.
lloid_status ingest(lloid_stream *s, int d, const void *src, lloid_dtype dt, int64_t n, const TickSlot *last) {
  DetState &ds = s->det[d];
  lloid_status r = make_room(s, ds, 0, n, last);
  if (r != LLOID_OK) return r;
  float *dst = ds.x[0] + (ds.avail[0] - ds.lo[0]);
  if (!src) {
    HIP_TRY(launch_fill_u8(dst, (size_t)n * 4, s->ingest));
  } else {
    // checked finite at push time: the flag is not read here
    HIP_TRY(launch_convert(src, dt, n, dst, 0, n, s->sscale, s->bad + 32, s->ingest));
  }
  ds.avail[0] += n;
  ds.pushed = ds.avail[0];
  return decimate_new(s, ds, last);
}

// Largest window end wb (> w_next) whose outputs every active bank can compute
// now (submitter thread: the slot table does not change while it runs).
int64_t stream_ready_until(const lloid_stream *s) {
  ReadyState st;
  st.win = s->win;
  st.w_next = s->w_next;
  st.max_w = s->max_w;
  st.n_end = s->n_end;
  for (const auto &d : s->det) {
    st.pushed.push_back(d.pushed);
    st.avail.push_back(d.avail);
  }
  for (int32_t i = 0; i < s->adm.n_slots(); ++i)
    if (s->adm.active(i))
      for (const auto &sd : s->bank_of[i]->slices)
        st.slices.push_back(ReadySlice{sd.level, sd.start_tap / sd.dec, operand_margin(s->bank_of[i])});
  return ready_until(st);
}

lloid_status ensure_pinned_bytes(void *&p, size_t &have, size_t bytes) {
  if (have >= bytes) return LLOID_OK;
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

// Wait for a free tick ring entry (lock held by lk); returns its index.
int take_tick_slot(lloid_stream *s, std::unique_lock<std::mutex> &lk) {
  for (;;) {
    for (int i = 0; i < kTickRing; ++i)
      if (!s->ticks[i].busy) return i;
    s->cv_done.wait(lk);
    if (s->error != LLOID_OK) return -1;
  }
}

// Enqueue the tick of windows [wa, wb) for every active bank and detector on
// the compute stream; the completer publishes its triggers.
lloid_status enqueue_tick(lloid_stream *s, int64_t wa, int64_t wb, Clock::time_point ready_at) {
  lloid_ctx *ctx = s->ctx;
  hipStream_t st = ctx->stream;
  const int64_t t0 = s->win.start(wa);
  int64_t t1 = s->win.start(wb);
  const int64_t n_end = s->n_end >= 0 ? s->n_end : INT64_MAX / 4;
  t1 = std::min(t1, n_end);
  const int64_t nw = wb - wa;
  std::vector<int32_t> ids;
  std::vector<const lloid_bank *> bank_of;
  int ti = -1;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    for (int32_t i = 0; i < s->adm.n_slots(); ++i)
      if (s->adm.active(i)) ids.push_back(i), bank_of.push_back(s->bank_of[i]);
    s->w_next = wb;
    s->windows += nw;
    if (ids.empty()) {
      s->cv_done.notify_all();
      return LLOID_OK;
    }
    ti = take_tick_slot(s, lk);
    if (ti < 0) return stored_error(s);
  }
  TickSlot &tk = s->ticks[ti];
  const TileShapes ts(s->ct, ctx->fir_variant, ctx->mix_variant);
  const size_t esz = dtype_size(s->ct);
  const int64_t tlen = t1 - t0;
  // per-tick scratch layout, shared by the ticks (they run in order on one
  // stream), then kTickRing areas of device tables, one per ring entry
  size_t bytes = 0;
  auto add = [&](size_t cnt, size_t sz) { bytes = (size_t)round_up((int64_t)bytes, 256) + cnt * sz; };
  int64_t rows = 0, xi_cap = 0;
  size_t n_fir = 0, n_up = 0;
  for (const lloid_bank *b : bank_of) {
    for (int d = 0; d < s->n_det; ++d) {
      const int64_t ops = tlen + 2 * operand_margin(b);
      add((size_t)ops * b->kld, esz);
      for (const auto &sl : b->slices) {
        ++n_fir;
        if (sl.level > 0)
          for (int64_t ld : low_ld(ops, sl.level)) add((size_t)sl.lp * ld, low_esz(s->ct)), ++n_up;
      }
      for (int k = 0; k < 5; ++k) add((size_t)b->n_templates * nw, 4);
      add((size_t)b->n_templates * nw, 8);
      add((size_t)b->n_templates * nw, 8);
      if (b->acorr) {
        add((size_t)b->n_templates * nw, 8);
        xi_cap += xi_unit_cap(nw, b->n_templates);
      }
    }
    rows += (int64_t)b->n_templates * s->n_det;
  }
  add((size_t)trig_blocks(rows * nw) + 2, 8);
  add((size_t)xi_cap, sizeof(XiUnit));
  add(2, 4);
  const size_t tab_bytes = n_fir * sizeof(FirJob) + n_up * sizeof(UpJob) +
                           bank_of.size() * s->n_det * (sizeof(MixJob) + sizeof(TrigJob)) + 64 * (4 + kMaxHops);
  const size_t common = (size_t)round_up((int64_t)bytes, 256);
  const size_t area = (size_t)round_up((int64_t)std::max(tab_bytes, s->tab_area), 256);
  const size_t need = common + kTickRing * area;
  if (s->ws.bytes < need || area != s->tab_area) {
    // a new layout (or a new allocation) moves buffers that ticks in flight use
    std::unique_lock<std::mutex> lk(s->mu);
    wait_completed(s, lk);
    lk.unlock();
    const lloid_status r = ensure_ws(ctx, s->ws, need);
    if (r != LLOID_OK) return r;
    s->tab_area = area;
  }
  const size_t tab_base = s->ws.bytes - kTickRing * s->tab_area;
  lloid_status rs = ensure_pinned_bytes(tk.htab, tk.htab_bytes, tab_bytes);
  if (rs != LLOID_OK) return rs;
  const int64_t cap = rows * nw;
  if (tk.htrig_cap < cap) {
    if (tk.htrig) (void)hipHostFree(tk.htrig);
    tk.htrig = nullptr;
    tk.htrig_cap = 0;
    if (hipHostMalloc((void **)&tk.htrig, (size_t)std::max<int64_t>(cap, 1) * sizeof(lloid_trigger),
                      hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return fail(LLOID_ENOMEM, "pinned trigger buffer of %lld records failed", (long long)cap);
    }
    tk.htrig_cap = cap;
  }
  Carve cv{(char *)s->ws.base};
  std::vector<FirJob> fj;
  std::vector<UpJob> uj[kMaxHops];
  std::vector<MixJob> mj;
  std::vector<TrigJob> tj;
  int64_t row = 0;
  for (size_t a = 0; a < bank_of.size(); ++a) {
    const lloid_bank *b = bank_of[a];
    for (int d = 0; d < s->n_det; ++d) {
      BankBufs bb;
      const int64_t ops = tlen + 2 * operand_margin(b);
      bb.ocat = cv.take<char>((size_t)ops * b->kld * esz);
      bb.low.assign(b->slices.size(), {});
      for (size_t k = 0; k < b->slices.size(); ++k)
        if (b->slices[k].level > 0)
          for (int64_t ld : low_ld(ops, b->slices[k].level))
            bb.low[k].push_back(cv.take<char>((size_t)b->slices[k].lp * ld * low_esz(s->ct)));
      bb.psnr = cv.take<float>((size_t)b->n_templates * nw);
      bb.pphase = cv.take<float>((size_t)b->n_templates * nw);
      bb.pdt = cv.take<float>((size_t)b->n_templates * nw);
      bb.psi = cv.take<float>((size_t)b->n_templates * nw);
      bb.pxi = cv.take<float>((size_t)b->n_templates * nw);
      bb.pn = cv.take<int64_t>((size_t)b->n_templates * nw);
      bb.pz = cv.take<float2>((size_t)b->n_templates * nw);
      if (b->acorr) bb.pkey = cv.take<int64_t>((size_t)b->n_templates * nw);
      bb.ld_peak = nw;
      bb.w_base = wa;
      std::vector<LevelView> lv(s->n_levels);
      const DetState &ds = s->det[d];
      for (int k = 0; k < s->n_levels; ++k) lv[k] = LevelView{ds.x[k], ds.lo[k], ds.avail[k] - ds.lo[k]};
      add_bank_jobs(b, lv.data(), t0, t1, n_end, wa, wb, s->win, bb, 1.f / (b->mix_scale * s->sscale), nullptr, 0, ts,
                    fj, uj, mj);
      tj.push_back(TrigJob{bb.psnr, bb.pn, bb.pphase, bb.pdt, bb.psi, b->acorr ? bb.pxi : nullptr, wa, nw, row * nw,
                           b->n_templates, ids[a], d, 0});
      row += b->n_templates;
    }
  }
  const int64_t n_blk = trig_blocks(rows * nw);
  int64_t *counts = cv.take<int64_t>((size_t)n_blk + 2);
  int64_t *total = counts + n_blk;
  XiWork xw;
  xw.cap = xi_cap;
  xw.units = cv.take<XiUnit>((size_t)xi_cap);
  xw.counters = cv.take<int32_t>(2);
  char *dtab = (char *)s->ws.base + tab_base + (size_t)ti * s->tab_area;
  StageItems items;
  number_jobs(fj, uj, mj, items);
  char *htab = (char *)tk.htab;
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
  // the tick's device work: table upload, every stage, trigger records into
  // pinned host memory, the count into pinned host memory
  auto work = [&]() -> lloid_status {
    HIP_TRY(hipMemcpyAsync(dtab, htab, off, hipMemcpyHostToDevice, st));
    const lloid_status r = launch_stages(ctx, s->ct, dtab, to, items, false, s->thr, s->thr, xw, nullptr);
    if (r != LLOID_OK) return r;
    HIP_TRY(launch_trigger_jobs((const TrigJob *)(dtab + trig_off), (int)tj.size(), rows * nw, s->thr, counts, total,
                                cap, tk.htrig, st));
    HIP_TRY(hipMemcpyAsync(tk.hcount, total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    return LLOID_OK;
  };
  // the tick reads strain the ingest stream has written
  HIP_TRY(hipEventRecord(s->ingest_done, s->ingest));
  HIP_TRY(hipStreamWaitEvent(st, s->ingest_done, 0));
  if (s->use_graph) {
    std::vector<int64_t> key = {(int64_t)(uintptr_t)dtab, (int64_t)(uintptr_t)htab, (int64_t)off, (int64_t)trig_off,
                                (int64_t)tj.size(), rows, cap, (int64_t)(uintptr_t)counts,
                                (int64_t)(uintptr_t)tk.htrig, items.fir, items.mix, items.entries, (int64_t)to.fir,
                                (int64_t)to.mix, to.n_fir, to.n_mix};
    key.push_back(items.xi2 ? 1 : 0);
    key.push_back((int64_t)(uintptr_t)xw.units);
    key.push_back(xw.cap);
    key.push_back(ctx->fir_variant * 16 + ctx->mix_variant);
    key.push_back(items.windows);
    for (int h = 0; h < kMaxHops; ++h) {
      key.push_back(items.up[h]);
      key.push_back((int64_t)to.up[h]);
      key.push_back(to.n_up[h]);
    }
    if (!tk.exec || key != tk.graph_key) {
      if (tk.exec) (void)hipGraphExecDestroy(tk.exec), tk.exec = nullptr;
      if (tk.graph) (void)hipGraphDestroy(tk.graph), tk.graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      const lloid_status r = work();
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(st, &g);
      if (r != LLOID_OK) {
        if (ec == hipSuccess && g) (void)hipGraphDestroy(g);
        return r;
      }
      HIP_TRY(ec);
      tk.graph = g;
      HIP_TRY(hipGraphInstantiate(&tk.exec, g, nullptr, nullptr, 0));
      tk.graph_key = key;
      std::lock_guard<std::mutex> lk(s->mu);
      ++s->graph_captures;
    } else {
      std::lock_guard<std::mutex> lk(s->mu);
      ++s->graph_replays;
    }
    HIP_TRY(hipGraphLaunch(tk.exec, st));
  } else {
    rs = work();
    if (rs != LLOID_OK) return rs;
  }
  HIP_TRY(hipEventRecord(tk.done, st));
  {
    std::lock_guard<std::mutex> lk(s->mu);
    tk.busy = true;
    tk.seq = ++s->seq_enqueued;
    tk.ready_at = ready_at;
    s->inflight.push_back(ti);
  }
  s->cv_comp.notify_all();
  return LLOID_OK;
}

// The tick entry enqueued last (its event orders a level-buffer shift), or NULL.
const TickSlot *last_tick(lloid_stream *s) {
  std::lock_guard<std::mutex> lk(s->mu);
  return s->inflight.empty() ? nullptr : &s->ticks[s->inflight.back()];
}

// Process one item: ingest it, then enqueue every tick it makes ready.
lloid_status process(lloid_stream *s, const Item &it) {
  const TickSlot *last = last_tick(s);
  if (it.kind == Item::kFlush) {
    // zero strain past the end feeds the resamplers' look-ahead, as in lloid_filter
    const int64_t pad = (int64_t)(8 * kHalfQ) << s->n_levels;
    for (int d = 0; d < s->n_det; ++d) {
      int64_t done = 0;
      while (done < pad) {
        const int64_t m = std::min(pad - done, s->push_max);
        const lloid_status r = ingest(s, d, nullptr, LLOID_F32, m, last);
        if (r != LLOID_OK) return r;
        done += m;
      }
    }
    s->n_end = it.t0;
  } else {
    Staging &g = s->ring[it.ring];
    const size_t bytes = (size_t)it.n * dtype_size(it.dt);
    if (!it.on_device) HIP_TRY(hipMemcpyAsync(g.dev, g.host, bytes, hipMemcpyHostToDevice, s->ingest));
    const lloid_status r = ingest(s, it.det, g.dev, it.dt, it.n, last);
    if (r != LLOID_OK) return r;
  }
  for (;;) {
    const int64_t wb = stream_ready_until(s);
    if (wb <= s->w_next) break;
    const lloid_status r = enqueue_tick(s, s->w_next, wb, it.pushed_at);
    if (r != LLOID_OK) return r;
  }
  if (it.kind == Item::kStride) {
    // the staging entry is free once its upload and conversion are done
    HIP_TRY(hipStreamSynchronize(s->ingest));
  }
  return LLOID_OK;
}

void submitter_main(lloid_stream *s) {
  (void)hipSetDevice(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_sub.wait(lk, [&] { return s->stop || !s->inbox.empty(); });
    if (s->stop) break;
    Item it = s->inbox.front();
    s->inbox.pop_front();
    s->sub_busy = true;
    lk.unlock();
    const lloid_status r = s->error == LLOID_OK ? process(s, it) : s->error;
    lk.lock();
    if (it.kind == Item::kStride) s->ring_free.push_back(it.ring);
    if (r != LLOID_OK) set_error(s, r);
    s->sub_busy = false;
    s->cv_done.notify_all();
  }
}

// ------------------------------------------------------------ completer side

void completer_main(lloid_stream *s) {
  (void)hipSetDevice(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_comp.wait(lk, [&] { return !s->inflight.empty() || s->stop; });
    if (s->inflight.empty()) break;   // stop with nothing in flight
    TickSlot &tk = s->ticks[s->inflight.front()];
    lk.unlock();
    const hipError_t e = hipEventSynchronize(tk.done);
    const Clock::time_point now = Clock::now();
    lk.lock();
    if (e != hipSuccess) {
      set_error(s, fail(LLOID_EDEVICE, "a stream tick failed: %s", hipGetErrorString(e)));
    } else {
      const int64_t n = std::min(*tk.hcount, tk.htrig_cap);
      s->out.insert(s->out.end(), tk.htrig, tk.htrig + n);
      s->triggers += n;
      s->ticks_run += 1;
      s->lat_ms.push_back(std::chrono::duration<double, std::milli>(now - tk.ready_at).count());
    }
    s->seq_completed = tk.seq;
    tk.busy = false;
    s->inflight.pop_front();
    s->cv_done.notify_all();
  }
}

void free_stream(lloid_stream *s) {
  if (s->submitter.joinable() || s->completer.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv_sub.notify_all();
    if (s->submitter.joinable()) s->submitter.join();
    // the completer drains the ticks in flight before it ends
    s->cv_comp.notify_all();
    if (s->completer.joinable()) s->completer.join();
  }
  (void)hipSetDevice(s->ctx->device);
  if (s->ingest) (void)hipStreamSynchronize(s->ingest);
  (void)hipStreamSynchronize(s->ctx->stream);
  if (s->level_mem) (void)hipFree(s->level_mem);
  if (s->bad) (void)hipFree(s->bad);
  if (s->check_buf) (void)hipFree(s->check_buf);
  if (s->hbad) (void)hipHostFree(s->hbad);
  for (auto &g : s->ring) {
    if (g.host) (void)hipHostFree(g.host);
    if (g.dev) (void)hipFree(g.dev);
  }
  for (auto &tk : s->ticks) {
    if (tk.exec) (void)hipGraphExecDestroy(tk.exec);
    if (tk.graph) (void)hipGraphDestroy(tk.graph);
    if (tk.htab) (void)hipHostFree(tk.htab);
    if (tk.htrig) (void)hipHostFree(tk.htrig);
    if (tk.hcount) (void)hipHostFree(tk.hcount);
    if (tk.done) (void)hipEventDestroy(tk.done);
  }
  if (s->ingest_done) (void)hipEventDestroy(s->ingest_done);
  if (s->ws.base) (void)hipFree(s->ws.base);
  if (s->ingest) (void)hipStreamDestroy(s->ingest);
  if (s->staging_stream) (void)hipStreamDestroy(s->staging_stream);
  delete s;
}

// Is every sample of a host stride finite once scaled and rounded to FP32
// (the value the device computes with)?
template <typename T> bool host_finite(const T *p, int64_t n, float scale) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite((float)p[i] * scale)) return false;
  return true;
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
  if (opts->queue_strides < 0 || opts->queue_strides > 4096) return fail(LLOID_EINVAL, "queue_strides out of range");
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
  s->accepted.assign(s->n_det, 0);
  s->win = Windows{(int64_t)full_rate_hz * t.window_num, t.window_den};
  s->win_len = ceil_div(s->win.p, s->win.q);
  s->thr = t.threshold;
  s->sscale = sscale;
  s->adm = Admission(opts->hbm_budget);
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
  const int n_ring = opts->queue_strides > 0 ? opts->queue_strides : 64;
  const size_t lbytes = total * 4 * s->n_det;
  bool ok = hipMalloc((void **)&s->level_mem, lbytes) == hipSuccess &&
            hipMalloc((void **)&s->bad, 256) == hipSuccess &&
            hipMalloc((void **)&s->check_buf, (size_t)s->push_max * 4) == hipSuccess &&
            hipHostMalloc((void **)&s->hbad, 256, hipHostMallocDefault) == hipSuccess;
  s->ring.resize(n_ring);
  for (int i = 0; i < n_ring && ok; ++i) {
    ok = hipHostMalloc(&s->ring[i].host, (size_t)s->push_max * 8, hipHostMallocDefault) == hipSuccess &&
         hipMalloc(&s->ring[i].dev, (size_t)s->push_max * 8) == hipSuccess;
    s->ring_free.push_back(n_ring - 1 - i);
  }
  for (auto &tk : s->ticks)
    ok = ok && hipHostMalloc((void **)&tk.hcount, 64, hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&tk.done, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&s->ingest_done, hipEventDisableTiming) == hipSuccess &&
       hipStreamCreateWithFlags(&s->ingest, hipStreamNonBlocking) == hipSuccess &&
       hipStreamCreateWithFlags(&s->staging_stream, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_stream(s);
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
    free_stream(s);
    return fail(LLOID_EDEVICE, "stream initialisation failed");
  }
  s->submitter = std::thread(submitter_main, s);
  s->completer = std::thread(completer_main, s);
  *out = s;
  return LLOID_OK;
  ABI_GUARD_END
}

extern "C" lloid_status lloid_stream_admit(lloid_stream *s, lloid_bank *bank, int32_t *slot) {
  ABI_GUARD_BEGIN
  if (!s || !slot) return fail(LLOID_EINVAL, "NULL argument");
  lloid_status r = check_bank(s, bank);
  if (r != LLOID_OK) return r;
  std::unique_lock<std::mutex> lk(s->mu);
  // the bank joins at the stream's position after every stride pushed so far
  wait_submitted(s, lk);
  r = stored_error(s);
  if (r != LLOID_OK) return r;
  bool active = false;
  const int32_t id = s->adm.add(bank->device_bytes + scratch_bytes(s, bank), &active);
  if (id < 0) return fail(LLOID_ENOMEM, "the bank alone exceeds the stream's budget");
  s->bank_of.push_back(bank);
  *slot = id;
  if (!active) return fail(LLOID_EAGAIN, "queued until device memory frees up");
  return LLOID_OK;
  ABI_GUARD_END
}

extern "C" lloid_status lloid_stream_remove(lloid_stream *s, int32_t slot) {
  ABI_GUARD_BEGIN
  if (!s) return fail(LLOID_EINVAL, "NULL stream");
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->adm.present(slot)) return fail(LLOID_EINVAL, "no such slot");
  // the bank leaves at the stream's position after every stride pushed so far
  wait_submitted(s, lk);
  s->adm.remove(slot);   // queued banks that now fit become active
  s->bank_of[slot] = nullptr;
  // the caller may destroy the bank: no tick in flight may still read it
  wait_completed(s, lk);
  return stored_error(s);
  ABI_GUARD_END
}

extern "C" lloid_status lloid_stream_push(lloid_stream *s, int32_t detector, int64_t t0, const void *data,
                                          lloid_dtype dt, int64_t n) {
  ABI_GUARD_BEGIN
  if (!s) return fail(LLOID_EINVAL, "NULL stream");
  if (detector < 0 || detector >= s->n_det) return fail(LLOID_EINVAL, "no such detector");
  if (n < 0 || (n > 0 && !data)) return fail(LLOID_EINVAL, "bad stride");
  if (dt != LLOID_F64 && dt != LLOID_F32) return fail(LLOID_EINVAL, "strain must be F64 or F32");
  const Clock::time_point now = Clock::now();
  std::unique_lock<std::mutex> lk(s->mu);
  lloid_status r = stored_error(s);
  if (r != LLOID_OK) return r;
  if (s->flushed) return fail(LLOID_EORDER, "the stream was flushed");
  if (t0 != s->accepted[detector])
    return fail(LLOID_EORDER, "stride starts at %lld, expected %lld", (long long)t0,
                (long long)s->accepted[detector]);
  lk.unlock();
  HIP_TRY(hipSetDevice(s->ctx->device));
  const bool on_device = n > 0 && is_device_ptr(data);
  const size_t esz = dtype_size(dt);
  // check the whole stride before anything is queued: a non-finite sample
  // rejects it (EDATA) and the detector stays at t0
  if (n > 0 && !on_device) {
    const bool fin = dt == LLOID_F64 ? host_finite((const double *)data, n, s->sscale)
                                     : host_finite((const float *)data, n, s->sscale);
    if (!fin) return fail(LLOID_EDATA, "stride holds a non-finite sample; nothing was queued");
  }
  if (n > 0 && on_device) {
    HIP_TRY(launch_fill_u8(s->bad, sizeof(int), s->staging_stream));
    for (int64_t done = 0; done < n; done += s->push_max) {
      const int64_t m = std::min(n - done, s->push_max);
      HIP_TRY(launch_convert((const char *)data + done * esz, dt, m, s->check_buf, 0, m, s->sscale, s->bad,
                             s->staging_stream));
    }
    HIP_TRY(hipMemcpyAsync(s->hbad, s->bad, sizeof(int), hipMemcpyDeviceToHost, s->staging_stream));
    HIP_TRY(hipStreamSynchronize(s->staging_stream));
    if (*s->hbad) return fail(LLOID_EDATA, "stride holds a non-finite sample; nothing was queued");
  }
  // copy the stride into staging entries of at most push_max samples, each
  // queued for the library thread as soon as it is copied
  int64_t done = 0;
  while (done < n) {
    const int64_t m = std::min(n - done, s->push_max);
    lk.lock();
    s->cv_done.wait(lk, [&] { return !s->ring_free.empty() || s->error != LLOID_OK; });
    if (s->error != LLOID_OK) return stored_error(s);
    const int g = s->ring_free.back();
    s->ring_free.pop_back();
    lk.unlock();
    const char *src = (const char *)data + done * esz;
    if (on_device) {
      HIP_TRY(hipMemcpyAsync(s->ring[g].dev, src, (size_t)m * esz, hipMemcpyDeviceToDevice, s->staging_stream));
      HIP_TRY(hipStreamSynchronize(s->staging_stream));
    } else {
      std::memcpy(s->ring[g].host, src, (size_t)m * esz);
    }
    Item it;
    it.kind = Item::kStride;
    it.det = detector;
    it.t0 = t0 + done;
    it.n = m;
    it.dt = dt;
    it.ring = g;
    it.on_device = on_device;
    it.pushed_at = now;
    lk.lock();
    s->inbox.push_back(it);
    s->accepted[detector] = t0 + done + m;
    lk.unlock();
    s->cv_sub.notify_all();
    done += m;
  }
  return LLOID_OK;
  ABI_GUARD_END
}

extern "C" lloid_status lloid_stream_flush(lloid_stream *s) {
  ABI_GUARD_BEGIN
  if (!s) return fail(LLOID_EINVAL, "NULL stream");
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->flushed) {
    const int64_t end = s->accepted[0];
    for (int64_t a : s->accepted)
      if (a != end) return fail(LLOID_EORDER, "detectors hold different amounts of strain");
    Item it;
    it.kind = Item::kFlush;
    it.t0 = end;
    it.pushed_at = Clock::now();
    s->inbox.push_back(it);
    s->flushed = true;
    s->cv_sub.notify_all();
  }
  wait_submitted(s, lk);
  wait_completed(s, lk);
  return stored_error(s);
  ABI_GUARD_END
}

extern "C" lloid_status lloid_stream_poll(lloid_stream *s, lloid_trigger *out, int64_t cap, int64_t *n_out,
                                          int32_t wait_ms) {
  ABI_GUARD_BEGIN
  if (!s || !n_out || cap < 0 || (cap > 0 && !out)) return fail(LLOID_EINVAL, "bad argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (wait_ms != 0) {
    // every stride pushed before this call filtered, or the time is up
    auto idle = [&] {
      return s->error != LLOID_OK ||
             (s->inbox.empty() && !s->sub_busy && s->seq_completed >= s->seq_enqueued);
    };
    if (wait_ms < 0) s->cv_done.wait(lk, idle);
    else s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), idle);
  }
  const int64_t m = std::min<int64_t>(cap, (int64_t)s->out.size());
  std::copy(s->out.begin(), s->out.begin() + m, out);
  s->out.erase(s->out.begin(), s->out.begin() + m);
  *n_out = m;
  return stored_error(s);
  ABI_GUARD_END
}

extern "C" lloid_status lloid_stream_stats_get(const lloid_stream *s, lloid_stream_stats *out) {
  ABI_GUARD_BEGIN
  if (!s || !out) return fail(LLOID_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof *out);
  out->ticks = s->ticks_run;
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
  out->active_slots = s->adm.n_active();
  out->queued_banks = s->adm.n_queued();
  out->bytes_in_use = s->adm.used();
  out->graph_captures = s->graph_captures;
  out->graph_replays = s->graph_replays;
  out->queued_strides = (int64_t)s->inbox.size();
  out->ticks_in_flight = (int64_t)s->inflight.size();
  return LLOID_OK;
  ABI_GUARD_END
}

extern "C" lloid_status lloid_stream_stats_reset(lloid_stream *s) {
  if (!s) return fail(LLOID_EINVAL, "NULL stream");
  std::lock_guard<std::mutex> lk(s->mu);
  s->lat_ms.clear();
  s->ticks_run = 0;
  s->windows = 0;
  s->triggers = 0;
  s->graph_captures = 0;
  s->graph_replays = 0;
  return LLOID_OK;
}

extern "C" lloid_status lloid_stream_destroy(lloid_stream *s) {
  if (!s) return LLOID_OK;
  free_stream(s);
  return LLOID_OK;
}
