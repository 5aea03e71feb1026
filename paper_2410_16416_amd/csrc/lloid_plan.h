// Host-only planning logic of the filtering path: integer range arithmetic of
// the multi-rate resampling, the interpolation hops of a slice, trigger
// windows, the device-memory admission of serving banks and the window
// readiness of a stream.  No HIP types or calls: the runtime uses these, and
// a CPU test (built with address and undefined-behaviour sanitizers) checks
// them against brute force and their invariants.
#pragma once

#include <stdint.h>

#include <deque>
#include <vector>

namespace lloid {

// Half-band resampler: g[n], |n| <= kHalfQ, zero at even n != 0.
constexpr int kHalfQ = 32;
constexpr int kHalfTaps = 2 * kHalfQ + 1;
// Output samples of one interpolation task (32 channels x kUpCols samples).
constexpr int kUpCols = 128;
constexpr int kMaxLevel = 7;       // lowest slice rate f0 / 128
constexpr int kMaxAutocorrHalf = 512;
constexpr int kMaxHops = 4;        // interpolation hops of a level-7 slice: x2, x4, x4, x4

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
inline int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
inline int64_t ceil_div(int64_t a, int64_t b) { return -floor_div(-a, b); }

struct Range {
  int64_t lo = 0, hi = 0;  // absolute indices [lo, hi)
  int64_t size() const { return hi > lo ? hi - lo : 0; }
};

// interpolation reads w[j] with |n - 2j| <= Q and decimation reads u[2k - m]
// with |m| <= Q: the range a level needs from the one above it
inline Range halo_up(Range r) { return {ceil_div(r.lo - kHalfQ, 2), floor_div(r.hi - 1 + kHalfQ, 2) + 1}; }

inline std::vector<Range> need_ranges(int64_t t0, int64_t t1, int n_levels) {
  std::vector<Range> need(n_levels);
  need[0] = {t0, t1};
  for (int k = 1; k < n_levels; ++k) need[k] = halo_up(need[k - 1]);
  return need;
}

// Trigger windows: window w starts at floor(w p / q).
struct Windows {
  int64_t p = 1, q = 1;
  int64_t start(int64_t w) const { return (w * p) / q; }
  int64_t count(int64_t n) const { return ceil_div(n * q, p); }   // windows intersecting [0, n)
};

// Interpolation hops of a slice at `level` for full-rate outputs [t0, t1):
// hop h maps level lev_in[h] to lev_out[h] by r[h] on range out[h] (aligned
// tiles), reading in[h]; the FIR must produce in[0].
struct UpPlan {
  std::vector<int> r, lev_in, lev_out;
  std::vector<Range> in, out;
};
UpPlan up_plan(int64_t t0, int64_t t1, int level);
// Row pitch (elements) of each channel-major low-rate buffer of a slice for
// outputs spanning t_len samples, an upper bound over output positions:
// [0] the FIR output, [h] the output of hop h - 1.
std::vector<int64_t> low_ld(int64_t t_len, int level);

// Device-memory admission of serving banks: banks enter slots in arrival
// order while their bytes fit the budget (0: no limit); the others wait and
// are admitted, still in arrival order, as removals free budget.  A queued
// bank never lets a later one pass it.
class Admission {
 public:
  explicit Admission(int64_t budget = 0) : budget_(budget) {}
  // Add a bank needing `bytes`; returns its slot id and sets *active.  A bank
  // that alone exceeds a nonzero budget is refused: -1.
  int32_t add(int64_t bytes, bool *active);
  // Remove an active or queued slot; false if there is no such slot.
  bool remove(int32_t slot);
  bool active(int32_t slot) const { return slot >= 0 && slot < (int32_t)slots_.size() && slots_[slot].active; }
  bool present(int32_t slot) const { return slot >= 0 && slot < (int32_t)slots_.size() && slots_[slot].present; }
  int64_t used() const { return used_; }
  int64_t budget() const { return budget_; }
  int32_t n_slots() const { return (int32_t)slots_.size(); }
  int32_t n_active() const;
  int32_t n_queued() const { return (int32_t)queue_.size(); }

 private:
  struct S {
    int64_t bytes = 0;
    bool present = false, active = false;
  };
  void admit_queued();
  int64_t budget_ = 0, used_ = 0;
  std::vector<S> slots_;
  std::deque<int32_t> queue_;
};

// Window readiness of a stream: the largest window end wb in (w_next,
// w_next + max_w] such that every window below wb is computable now, or
// w_next when none is.  A window range [w_next, wb) needs full-rate outputs
// [t0, t1) = [start(w_next), min(start(wb), n_end)) plus `margin` samples on
// each side; a slice at `level` whose filter starts `shift` samples (at its
// rate) before the output reads its level up to the need range's end minus
// that shift, which every detector must have computed (avail[level]).
struct ReadySlice {
  int level = 0;
  int64_t shift = 0;   // start tap / decimation factor
  int64_t margin = 0;  // operand samples beyond each end of the outputs
};
struct ReadyState {
  Windows win;
  int64_t w_next = 0;
  int max_w = 1;
  int64_t n_end = -1;                        // data end once flushed (-1 while streaming)
  std::vector<int64_t> pushed;               // per detector: full-rate samples received
  std::vector<std::vector<int64_t>> avail;   // per detector, per level: computed frontier (exclusive)
  std::vector<ReadySlice> slices;            // every slice of every active bank
};
int64_t ready_until(const ReadyState &st);

// BF16 (8-bit significand) pair of a finite FP32 value, as bit patterns:
// hi = x rounded to nearest (ties to even), lo = (x - hi) rounded likewise,
// so that hi + lo carries 16 significant bits of x (the interpolation
// filters of the BF16 operand path are split this way).
void bf16_split(float x, uint16_t *hi, uint16_t *lo);
float bf16_value(uint16_t bits);

}  // namespace lloid
