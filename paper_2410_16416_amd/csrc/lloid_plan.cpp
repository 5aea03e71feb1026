// Host-only planning logic (see lloid_plan.h).
#include "lloid_plan.h"

#include <algorithm>
#include <climits>
#include <cstring>

namespace lloid {

UpPlan up_plan(int64_t t0, int64_t t1, int level) {
  UpPlan p;
  // an odd level starts with one x2 hop at its own (lowest) rate, the rest are x4
  for (int lev = level; lev > 0;) {
    const int r = (lev % 2) ? 2 : 4;
    p.r.push_back(r);
    p.lev_in.push_back(lev);
    lev -= r == 4 ? 2 : 1;
    p.lev_out.push_back(lev);
  }
  const int H = (int)p.r.size();
  p.in.resize(H);
  p.out.resize(H);
  // top-down: a hop's outputs, in whole 32-sample tiles from a multiple of 32,
  // read the 64 source samples of each tile from n0 / R - (32 - 32 / R)
  // (n0 and the span are multiples of 32, so the divisions are exact)
  Range want{t0, t1};
  for (int h = H - 1; h >= 0; --h) {
    p.out[h] = want;
    const int64_t a = floor_div(want.lo, 32) * 32;
    const int64_t span = round_up(want.hi - a, kUpCols);
    const int R = p.r[h], c = 32 - 32 / R;
    p.in[h] = {a / R - c, (a + span - 32) / R - c + 64};
    want = p.in[h];
  }
  return p;
}

std::vector<int64_t> low_ld(int64_t t_len, int level) {
  const UpPlan p = up_plan(0, 1, level);   // hop rates only
  const int H = (int)p.r.size();
  std::vector<int64_t> ld(H);
  int64_t want = t_len;
  for (int h = H - 1; h >= 0; --h) {
    // worst case: the first output sits 31 samples past a tile start
    const int64_t span = round_up(want + 31, kUpCols);
    const int64_t in = (span - 32) / p.r[h] + 64;
    ld[h] = round_up(in, 64);
    want = in;
  }
  return ld;
}

int32_t Admission::add(int64_t bytes, bool *active) {
  if (budget_ > 0 && bytes > budget_) {
    *active = false;
    return -1;
  }
  S s;
  s.bytes = bytes;
  s.present = true;
  const int32_t id = (int32_t)slots_.size();
  slots_.push_back(s);
  queue_.push_back(id);
  admit_queued();
  *active = slots_[id].active;
  return id;
}

bool Admission::remove(int32_t slot) {
  if (!present(slot)) return false;
  S &s = slots_[slot];
  if (s.active) used_ -= s.bytes;
  else queue_.erase(std::remove(queue_.begin(), queue_.end(), slot), queue_.end());
  s.active = false;
  s.present = false;
  admit_queued();
  return true;
}

int32_t Admission::n_active() const {
  int32_t n = 0;
  for (const S &s : slots_) n += s.active;
  return n;
}

void Admission::admit_queued() {
  while (!queue_.empty()) {
    S &q = slots_[queue_.front()];
    if (budget_ > 0 && used_ + q.bytes > budget_) break;
    used_ += q.bytes;
    q.active = true;
    queue_.pop_front();
  }
}

int64_t ready_until(const ReadyState &st) {
  int64_t data_end = INT64_MAX;
  for (int64_t p : st.pushed) data_end = std::min(data_end, p);
  if (st.n_end >= 0) data_end = st.n_end;
  int64_t best = st.w_next;
  for (int64_t wb = st.w_next + 1; wb <= st.w_next + st.max_w; ++wb) {
    const int64_t t0 = st.win.start(st.w_next);
    int64_t t1 = st.win.start(wb);
    if (st.n_end >= 0) {
      if (t0 >= st.n_end) break;
      t1 = std::min(t1, st.n_end);
    } else if (t1 > data_end) {
      break;
    }
    bool ok = true;
    for (const ReadySlice &sl : st.slices) {
      // outputs [t0 - margin, t1 + margin): the peaks' sub-sample refinement
      // and signal-consistency lags read up to margin samples past t1
      const Range r = need_ranges(t0 - sl.margin, t1 + sl.margin, sl.level + 1)[sl.level];
      for (const auto &av : st.avail)
        if (r.hi - sl.shift > av[sl.level]) ok = false;
      if (!ok) break;
    }
    if (!ok) break;
    best = wb;
    if (st.n_end >= 0 && t1 >= st.n_end) break;
  }
  return best;
}

static uint16_t bf16_round(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest, ties to even (finite values)
  return (uint16_t)(u >> 16);
}

float bf16_value(uint16_t bits) {
  const uint32_t u = (uint32_t)bits << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

void bf16_split(float x, uint16_t *hi, uint16_t *lo) {
  *hi = bf16_round(x);
  *lo = bf16_round(x - bf16_value(*hi));   // exact in FP32: x and hi share the exponent range
}

}  // namespace lloid
