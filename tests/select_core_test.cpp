// CPU test of the selection phase's threshold rule with batched passes
// (select_core.h): for synthetic cluster-count functions of the threshold
// (monotone, a jump across the window that makes the rule step back and
// forth, pseudo-random), the batched rule must end on the same threshold
// (bit for bit) and count as the rule run one threshold per pass, for every
// slot count, and never run more passes than it.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <random>

#include "../paper_2408_14070_amd/csrc/select_core.h"

using namespace rid::selcore;

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "CHECK failed line %d: %s\n", __LINE__, #c); \
      return 1;                                                         \
    }                                                                   \
  } while (0)

using CountFn = std::function<int(float)>;

struct Serial {
  float t;
  int count, passes;
  bool incomplete;
};

// the rule as stated: one clustering per threshold
static Serial serial_rule(const CountFn& f, float t0, int lower, int upper, bool adapt) {
  float t = t0;
  for (int it = 0;; ++it) {
    const int c = f(t);
    if (c < 0) return {t, c, it + 1, true};
    if (!adapt || (c >= lower && c <= upper) || it == 100) return {t, c, it + 1, false};
    t = c > upper ? t * 1.1f : t / 1.1f;
  }
}

static uint32_t bits(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  return u;
}

static int compare(const CountFn& f, float t0, int lower, int upper, bool adapt, int T,
                   int* passes_out) {
  const Serial ref = serial_rule(f, t0, lower, upper, adapt);
  float last[kMaxSlots];
  auto pass = [&](const float* ts, int n, int* counts) -> int {
    for (int j = 0; j < n; ++j) {
      last[j] = ts[j];
      counts[j] = f(ts[j]);
    }
    return 0;
  };
  Outcome o;
  const int r = adjust_threshold(t0, lower, upper, adapt, T, pass, o);
  if (ref.incomplete) {
    CHECK(r == kIncomplete);
    return 0;
  }
  CHECK(r == 0);
  CHECK(bits(o.t) == bits(ref.t));
  CHECK(o.count == ref.count);
  CHECK(o.slot >= 0 && o.slot < T && bits(last[o.slot]) == bits(o.t));
  CHECK(o.passes >= 1 && o.passes <= ref.passes);
  if (!adapt) CHECK(o.passes == 1);
  *passes_out = o.passes;
  return 0;
}

int main() {
  std::mt19937 rng(12345);
  std::uniform_real_distribution<float> U(0.f, 1.f);
  const int slots[] = {1, 2, 3, 16, 24, 32};
  int cases = 0;
  for (int trial = 0; trial < 600; ++trial) {
    const int kind = trial % 4;
    CountFn f;
    if (kind == 0) {          // count falls as the threshold grows
      const double a = 5.0 + 495.0 * U(rng), p = 0.5 + 2.5 * U(rng);
      f = [a, p](float t) { return (int)(a / std::pow((double)t, p)); };
    } else if (kind == 1) {   // every frame its own cluster below tc, one above
      const float tc = 0.5f + 4.5f * U(rng);
      f = [tc](float t) { return t < tc ? 100 : 3; };
    } else if (kind == 2) {   // no order at all
      const uint32_t h = rng();
      f = [h](float t) { return (int)(((bits(t) ^ h) * 2654435761u) >> 26); };
    } else {                  // monotone, but thresholds above tc leave a pass unfinished
      const double a = 200.0 * (0.5 + U(rng));
      const float tc = 1.f + 20.f * U(rng);
      f = [a, tc](float t) { return t > tc ? -1 : (int)(a / (double)t); };
    }
    const float scales[] = {0.01f, 0.1f, 1.f, 10.f, 100.f};
    const float t0 = scales[rng() % 5] * (0.5f + 1.5f * U(rng));
    const int lower = 1 + (int)(rng() % 40), upper = lower + (int)(rng() % 20);
    for (int T : slots)
      for (int adapt = 0; adapt < 2; ++adapt) {
        int passes = 0;
        if (compare(f, t0, lower, upper, adapt != 0, T, &passes)) {
          std::fprintf(stderr, "trial %d kind %d T %d adapt %d t0 %g window [%d, %d]\n", trial,
                       kind, T, adapt, t0, lower, upper);
          return 1;
        }
        ++cases;
      }
  }
  // 15 steps up from 2.6 (the count falls into [30, 45] at 9.87): one pass of
  // 24 slots holds them all; 16 slots need two
  const CountFn drop = [](float t) { return t < 9.8f ? 1000 : 35; };
  int p24 = 0, p16 = 0;
  CHECK(compare(drop, 2.6f, 30, 45, true, 24, &p24) == 0 && p24 == 1);
  CHECK(compare(drop, 2.6f, 30, 45, true, 16, &p16) == 0 && p16 == 2);
  // 4 steps down from 2.6 (the count rises into the window below 1.9): the
  // first pass's downward slots hold them
  const CountFn rise = [](float t) { return t > 1.9f ? 5 : 35; };
  int pd = 0;
  CHECK(compare(rise, 2.6f, 30, 45, true, 24, &pd) == 0 && pd == 1);
  // a pass's own error comes back unchanged
  Outcome o;
  auto failing = [](const float*, int, int*) -> int { return -3; };
  CHECK(adjust_threshold(1.f, 1, 2, true, 8, failing, o) == -3);
  std::printf("select core ok: %d cases\n", cases);
  return 0;
}
