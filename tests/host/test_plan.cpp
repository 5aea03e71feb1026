// CPU tests of the host-only planning logic (lloid_plan.h), built with the
// address and undefined-behaviour sanitizers by tests/test_host_plan.py.
// Each check compares the planner with a brute-force or model computation
// written independently here, or with an invariant the runtime relies on.
#include "lloid_plan.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

using namespace lloid;

static int g_fail = 0;
#define CHECK(cond, ...)                                            \
  do {                                                              \
    if (!(cond)) {                                                  \
      std::fprintf(stderr, "FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond); \
      std::fprintf(stderr, __VA_ARGS__);                            \
      std::fprintf(stderr, "\n");                                   \
      if (++g_fail > 20) std::exit(1);                              \
    }                                                               \
  } while (0)

// floor(a / b) and ceil(a / b) by stepping, for small values
static int64_t bf_floor(int64_t a, int64_t b) {
  int64_t q = 0;
  while (q * b > a) --q;
  while ((q + 1) * b <= a) ++q;
  return q;
}
static int64_t bf_ceil(int64_t a, int64_t b) { return -bf_floor(-a, b); }

// halo_up by brute force: the level-(k+1) samples j that the level-k range
// [lo, hi) reads, either way round: interpolation (|n - 2 j| <= Q) and
// decimation (level-k sample n is computed from j... the same set)
static Range bf_halo(Range r) {
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  for (int64_t n = r.lo; n < r.hi; ++n)
    for (int64_t j = bf_floor(n - kHalfQ, 2) - 2; j <= bf_ceil(n + kHalfQ, 2) + 2; ++j)
      if (std::llabs(n - 2 * j) <= kHalfQ) lo = std::min(lo, j), hi = std::max(hi, j + 1);
  return {lo, hi};
}

static void test_arith_and_halo() {
  for (int64_t a = -300; a <= 300; ++a)
    for (int64_t b : {1, 2, 3, 4, 32, 64, 128}) {
      CHECK(floor_div(a, b) == bf_floor(a, b), "floor_div(%lld, %lld)", (long long)a, (long long)b);
      CHECK(ceil_div(a, b) == bf_ceil(a, b), "ceil_div(%lld, %lld)", (long long)a, (long long)b);
    }
  for (int64_t lo = -80; lo <= 80; lo += 7)
    for (int64_t len = 1; len <= 70; len += 3) {
      const Range r{lo, lo + len}, h = halo_up(r), b = bf_halo(r);
      CHECK(h.lo == b.lo && h.hi == b.hi, "halo_up([%lld, %lld)) = [%lld, %lld), brute force [%lld, %lld)",
            (long long)r.lo, (long long)r.hi, (long long)h.lo, (long long)h.hi, (long long)b.lo, (long long)b.hi);
    }
}

static void test_windows() {
  for (int64_t p = 1; p <= 40; ++p)
    for (int64_t q = 1; q <= 7; ++q) {
      const Windows w{p, q};
      // windows tile the axis: consecutive starts, nonempty when p >= q
      if (p >= q)
        for (int64_t k = 0; k < 50; ++k) CHECK(w.start(k + 1) > w.start(k), "empty window %lld (p %lld q %lld)", (long long)k, (long long)p, (long long)q);
      for (int64_t n = 1; n <= 200; ++n) {
        int64_t cnt = 0;   // windows intersecting [0, n), by enumeration
        while (w.start(cnt) < n) ++cnt;
        CHECK(w.count(n) == cnt, "count(%lld) = %lld, enumeration %lld (p %lld q %lld)", (long long)n,
              (long long)w.count(n), (long long)cnt, (long long)p, (long long)q);
      }
    }
}

// the composite x R filter has support |t| <= 32 (R - 1): output n of a hop
// reads source u with |n - R u| <= 32 (R - 1)
static void test_up_plan() {
  std::mt19937_64 rng(7);
  for (int level = 1; level <= kMaxLevel; ++level) {
    for (int trial = 0; trial < 120; ++trial) {
      const int64_t t0 = (int64_t)(rng() % 20000) - 10000;
      const int64_t t1 = t0 + 1 + (int64_t)(rng() % 3000);
      const UpPlan p = up_plan(t0, t1, level);
      const int H = (int)p.r.size();
      CHECK(H >= 1 && H <= kMaxHops, "level %d: %d hops", level, H);
      // the hop chain goes from the slice's level down to level 0
      CHECK(p.lev_in[0] == level && p.lev_out[H - 1] == 0, "level %d chain", level);
      int drop = 0;
      for (int h = 0; h < H; ++h) {
        CHECK((p.r[h] == 2 && p.lev_in[h] - p.lev_out[h] == 1) || (p.r[h] == 4 && p.lev_in[h] - p.lev_out[h] == 2),
              "hop %d of level %d", h, level);
        CHECK(h == 0 || p.lev_in[h] == p.lev_out[h - 1], "hop %d of level %d does not chain", h, level);
        CHECK(h == 0 || p.r[h] == 4, "only the first hop may be x2 (level %d)", level);
        drop += p.lev_in[h] - p.lev_out[h];
      }
      CHECK(drop == level, "level %d: the hops drop %d levels", level, drop);
      CHECK(p.out[H - 1].lo == t0 && p.out[H - 1].hi == t1, "last hop's outputs");
      for (int h = 0; h < H; ++h) {
        const int R = p.r[h];
        const int64_t half = 32 * (R - 1);
        // every tile the hop computes: 32-sample tiles from a multiple of 32,
        // in runs of kUpCols; each reads 64 source samples from n0 / R - (32 - 32 / R)
        const int64_t a = bf_floor(p.out[h].lo, 32) * 32;
        for (int64_t n0 = a; n0 < p.out[h].hi; n0 += 32) {
          const int64_t s0 = n0 / R - (32 - 32 / R);
          CHECK(s0 >= p.in[h].lo && s0 + 64 <= p.in[h].hi, "level %d hop %d tile %lld reads outside in[h]", level, h,
                (long long)n0);
          // the 64-sample window covers the support of every output of the tile
          for (int64_t n = n0; n < n0 + 32; ++n) {
            const int64_t ulo = bf_ceil(n - half, R), uhi = bf_floor(n + half, R);
            CHECK(ulo >= s0 && uhi < s0 + 64, "level %d hop %d output %lld needs [%lld, %lld], window [%lld, %lld)",
                  level, h, (long long)n, (long long)ulo, (long long)uhi, (long long)s0, (long long)(s0 + 64));
          }
        }
        // the hop below produces exactly the range this hop reads
        if (h > 0) CHECK(p.out[h - 1].lo == p.in[h].lo && p.out[h - 1].hi == p.in[h].hi, "hop %d input", h);
      }
      // low_ld bounds every buffer's row for outputs of this length wherever they start
      const std::vector<int64_t> ld = low_ld(t1 - t0, level);
      CHECK((int)ld.size() == H, "low_ld size");
      for (int h = 0; h < H; ++h)
        CHECK(p.in[h].size() <= ld[h] && ld[h] % 64 == 0, "level %d t [%lld, %lld): in[%d] %lld > ld %lld", level,
              (long long)t0, (long long)t1, h, (long long)p.in[h].size(), (long long)ld[h]);
    }
  }
}

// Admission against a model: arrival-order queue, greedy admission from its
// head, budget never exceeded, refusals only for banks above the budget.
static void test_admission() {
  std::mt19937_64 rng(11);
  for (int trial = 0; trial < 400; ++trial) {
    const int64_t budget = trial % 5 == 0 ? 0 : 50 + (int64_t)(rng() % 200);
    Admission adm(budget);
    struct M {
      int64_t bytes;
      bool present, active;
    };
    std::vector<M> model;
    std::vector<int32_t> queue;   // model queue, arrival order
    int64_t used = 0;
    auto model_admit = [&]() {
      while (!queue.empty()) {
        M &m = model[queue.front()];
        if (budget > 0 && used + m.bytes > budget) break;
        used += m.bytes;
        m.active = true;
        queue.erase(queue.begin());
      }
    };
    for (int op = 0; op < 60; ++op) {
      if (rng() % 3 != 0 || model.empty()) {
        const int64_t bytes = 1 + (int64_t)(rng() % 120);
        bool active = false;
        const int32_t id = adm.add(bytes, &active);
        if (budget > 0 && bytes > budget) {
          CHECK(id == -1 && !active, "a bank above the budget must be refused");
          continue;
        }
        CHECK(id == (int32_t)model.size(), "slot ids are consecutive");
        model.push_back(M{bytes, true, false});
        queue.push_back(id);
        model_admit();
        CHECK(active == model[id].active, "add: active %d, model %d", (int)active, (int)model[id].active);
      } else {
        const int32_t id = (int32_t)(rng() % (model.size() + 1)) - 1;   // sometimes -1 or a removed slot
        const bool ok = adm.remove(id);
        const bool mok = id >= 0 && model[id].present;
        CHECK(ok == mok, "remove(%d): %d, model %d", id, (int)ok, (int)mok);
        if (mok) {
          if (model[id].active) used -= model[id].bytes;
          else queue.erase(std::find(queue.begin(), queue.end(), id));
          model[id].present = model[id].active = false;
          model_admit();
        }
      }
      CHECK(adm.used() == used, "used %lld, model %lld", (long long)adm.used(), (long long)used);
      CHECK(budget == 0 || adm.used() <= budget, "budget exceeded");
      CHECK(adm.n_queued() == (int32_t)queue.size(), "queue length");
      int32_t act = 0;
      for (size_t i = 0; i < model.size(); ++i) {
        CHECK(adm.active((int32_t)i) == model[i].active, "slot %zu activity", i);
        CHECK(adm.present((int32_t)i) == model[i].present, "slot %zu presence", i);
        act += model[i].active;
      }
      CHECK(adm.n_active() == act, "active count");
      // arrival order: the head of the queue does not fit (else it would be active)
      if (!queue.empty() && budget > 0) CHECK(used + model[queue.front()].bytes > budget, "queue head fits");
    }
  }
}

// ready_until against its definition, checked window by window with the
// level ranges from the brute-force halo
static bool computable(const ReadyState &st, int64_t wb) {
  const int64_t t0 = st.win.start(st.w_next);
  int64_t t1 = st.win.start(wb);
  if (st.n_end >= 0) {
    if (t0 >= st.n_end) return false;
    t1 = std::min(t1, st.n_end);
  } else {
    for (int64_t p : st.pushed)
      if (t1 > p) return false;
  }
  for (const ReadySlice &sl : st.slices) {
    Range r{t0 - sl.margin, t1 + sl.margin};
    for (int k = 0; k < sl.level; ++k) r = bf_halo(r);
    for (const auto &av : st.avail)
      if (r.hi - sl.shift > av[sl.level]) return false;
  }
  return true;
}

static void test_ready_until() {
  std::mt19937_64 rng(13);
  for (int trial = 0; trial < 1200; ++trial) {
    ReadyState st;
    st.win = Windows{64 + (int64_t)(rng() % 200), 1 + (int64_t)(rng() % 3)};
    st.w_next = (int64_t)(rng() % 20);
    st.max_w = 1 + (int)(rng() % 6);
    const int n_det = 1 + (int)(rng() % 3), n_lev = 1 + (int)(rng() % 4);
    const int64_t base = st.win.start(st.w_next);
    st.n_end = rng() % 4 == 0 ? base + (int64_t)(rng() % 600) - 50 : -1;
    for (int d = 0; d < n_det; ++d) {
      st.pushed.push_back(base + (int64_t)(rng() % 800));
      std::vector<int64_t> av;
      for (int k = 0; k < n_lev; ++k) av.push_back((base >> k) + (int64_t)(rng() % 500) - 50);
      st.avail.push_back(av);
    }
    const int n_sl = (int)(rng() % 4);
    for (int i = 0; i < n_sl; ++i)
      st.slices.push_back(ReadySlice{(int)(rng() % n_lev), (int64_t)(rng() % 300), (int64_t)(rng() % 40)});
    const int64_t wb = ready_until(st);
    CHECK(wb >= st.w_next && wb <= st.w_next + st.max_w, "ready_until out of range");
    // every window end up to wb is computable (each a prefix of the next)...
    for (int64_t x = st.w_next + 1; x <= wb; ++x) CHECK(computable(st, x), "trial %d: window end %lld not computable", trial, (long long)x);
    // ...and the next one is not, unless the cap or the flushed end stopped it
    if (wb < st.w_next + st.max_w) {
      const bool flushed_end = st.n_end >= 0 && wb > st.w_next && st.win.start(wb) >= st.n_end;
      if (!flushed_end) CHECK(!computable(st, wb + 1), "trial %d: window end %lld computable but not taken", trial, (long long)(wb + 1));
    }
  }
}

// bf16_split against rounding written out in double arithmetic: the two
// BF16 neighbours of x (8-bit significands) and the nearer one, ties to the
// even significand; then the error bound of the pair
static double bf_bf16_round(double x) {
  if (x == 0.0) return 0.0;
  const double ax = std::fabs(x);
  int e;
  std::frexp(ax, &e);                     // ax in [2^(e-1), 2^e)
  const double ulp = std::ldexp(1.0, e - 8);
  const double lo = std::floor(ax / ulp) * ulp, hi = lo + ulp;
  double r;
  if (ax - lo < hi - ax) r = lo;
  else if (ax - lo > hi - ax) r = hi;
  else r = (std::fmod(lo / ulp, 2.0) == 0.0) ? lo : hi;
  return x < 0 ? -r : r;
}

static void test_bf16_split() {
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> mant(1.0, 2.0);
  std::uniform_int_distribution<int> ex(-40, 40);
  std::vector<float> xs = {1.0f, 1.0f + 0x1p-8f, 1.0f + 3 * 0x1p-8f, -1.0f - 0x1p-8f, 0.0f, 0x1p-20f * 1.2345f,
                           0.63661977f, -0.21220659f};
  for (int i = 0; i < 20000; ++i) {
    const float x = (float)(std::ldexp(mant(rng), ex(rng)) * ((i & 1) ? -1.0 : 1.0));
    xs.push_back(x);
  }
  for (float x : xs) {
    uint16_t h, l;
    bf16_split(x, &h, &l);
    const double hv = bf16_value(h), lv = bf16_value(l);
    CHECK(hv == bf_bf16_round(x), "hi of %a is %a, want %a", (double)x, hv, bf_bf16_round(x));
    CHECK(lv == bf_bf16_round((double)x - hv), "lo of %a is %a, want %a", (double)x, lv, bf_bf16_round((double)x - hv));
    CHECK(std::fabs((double)x - hv - lv) <= std::ldexp(std::fabs((double)x), -16), "pair of %a misses by %a",
          (double)x, (double)x - hv - lv);
  }
  // ties go to the even significand
  uint16_t h, l;
  bf16_split(1.0f + 0x1p-8f, &h, &l);
  CHECK(bf16_value(h) == 1.0f && bf16_value(l) == 0x1p-8f, "tie below");
  bf16_split(1.0f + 3 * 0x1p-8f, &h, &l);
  CHECK(bf16_value(h) == 1.0f + 0x1p-6f && bf16_value(l) == -0x1p-8f, "tie above");
}

int main() {
  test_bf16_split();
  test_arith_and_halo();
  test_windows();
  test_up_plan();
  test_admission();
  test_ready_until();
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("host planning checks passed\n");
  return 0;
}
