// Host-side rule of the selection phase's threshold adjustment ("Selection";
// "SelectorConfig": cluster_threshold, numb_cluster_lower / _upper), with the
// clustering passes batched over several thresholds.  Pure C++ (no HIP): the
// library drives it with GPU passes, a CPU test with simulated cluster
// counts.
//
// The rule: cluster at t; while the count is above `upper` multiply t by 1.1,
// while below `lower` divide it by 1.1 (FP32), at most kMaxAdjust times.
// Every pass is a deterministic function of t, so a pass may cluster the
// thresholds the rule would reach next if the count stayed on its side of
// the window; the rule then takes its steps over those counts in its own
// order and asks for another pass only at a threshold the last pass does not
// hold.  The outcome is the one-threshold-per-pass outcome.
#pragma once

namespace rid {
namespace selcore {

constexpr int kMaxAdjust = 100;
constexpr float kFactor = 1.1f;
constexpr int kMaxSlots = 32;
constexpr int kIncomplete = 1;   // a pass left the slot the rule ended on unfinished

// The thresholds of a pass that starts at t: t, then (dir > 0) the upward
// chain t*1.1, (t*1.1)*1.1, ..., (dir < 0) the downward chain t/1.1, ...,
// or (dir == 0, the first pass) two thirds of the slots upward and the rest
// downward.  Each step is the rule's own FP32 operation on the previous one.
inline void slot_thresholds(float t, int dir, int T, float* ts) {
  const int up = dir > 0 ? T - 1 : dir < 0 ? 0 : (2 * (T - 1) + 2) / 3;
  ts[0] = t;
  for (int j = 1; j < T; ++j) {
    if (j <= up) ts[j] = ts[j - 1] * kFactor;
    else ts[j] = (j == up + 1 ? ts[0] : ts[j - 1]) / kFactor;
  }
}

struct Outcome {
  float t = 0.f;    // the threshold the rule ended on
  int slot = 0;     // its slot in the last pass
  int count = 0;    // its cluster count
  int passes = 0;   // passes run
};

// pass(ts, T, counts) clusters T thresholds and returns 0 with counts[k] the
// cluster count of ts[k] (negative: that slot did not finish), or a nonzero
// status, which is returned as is.  T in [1, kMaxSlots]; adapt == false runs
// one pass at t0.  Returns 0, the pass's status, or kIncomplete.
template <class PassFn>
int adjust_threshold(float t0, int lower, int upper, bool adapt, int T, PassFn&& pass,
                     Outcome& out) {
  float ts[kMaxSlots];
  int counts[kMaxSlots];
  int nt = 0, dir = 0;
  float t = t0;
  out = Outcome{};
  for (int it = 0;; ++it) {
    int k = 0;
    while (k < nt && !(ts[k] == t)) ++k;
    if (k == nt) {   // not among the last pass's thresholds
      nt = T;
      slot_thresholds(t, dir, T, ts);
      const int r = pass(ts, T, counts);
      if (r != 0) return r;
      ++out.passes;
      k = 0;
    }
    if (counts[k] < 0) return kIncomplete;
    out.t = t;
    out.slot = k;
    out.count = counts[k];
    if (!adapt || (counts[k] >= lower && counts[k] <= upper) || it == kMaxAdjust) return 0;
    dir = counts[k] > upper ? 1 : -1;
    t = dir > 0 ? t * kFactor : t / kFactor;
  }
}

}  // namespace selcore
}  // namespace rid
