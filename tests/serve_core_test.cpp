// CPU test of the serving core (arena allocator + batching policy) with a
// simulated executor: random requests of several models arrive over time,
// batches run for a time proportional to their walkers, memory is released
// on completion.  Checks the invariants the library's scheduler relies on.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "../paper_2408_14070_amd/csrc/serve_core.h"

using namespace rid::serve;

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "CHECK failed line %d: %s\n", __LINE__, #c); \
      return 1;                                                    \
    }                                                              \
  } while (0)

static int arena_test() {
  Arena a(1 << 20);
  size_t o1, o2, o3;
  CHECK(a.alloc(1000, &o1) && a.alloc(300000, &o2) && a.alloc(5000, &o3));
  CHECK(o1 % kAlign == 0 && o2 % kAlign == 0 && o3 % kAlign == 0);
  CHECK(a.release(o2));
  CHECK(!a.release(o2));                      // double free rejected
  size_t o4;
  CHECK(a.alloc(290000, &o4) && o4 == o2);    // first fit reuses the hole
  CHECK(a.release(o1) && a.release(o3) && a.release(o4));
  CHECK(a.in_use() == 0 && a.largest_free() == (size_t)(1 << 20));  // coalesced
  size_t big;
  CHECK(!a.alloc((1 << 20) + 1, &big));
  return 0;
}

struct Running {
  std::vector<int64_t> tickets;
  size_t off;
  double end;
  int model;
  int slot;
};

// fail_at > 0: the completion poll of the fail_at-th finishing batch reports
// a device error (a status other than success and not-ready), which must
// fail that batch's requests, every queued one, and refuse later arrivals.
constexpr int kSuccess = 0, kNotReady = 600, kDeviceError = 719;
constexpr int kOk = 0, kErr = -3;

static int sim(bool fifo, int slots, int max_batch, size_t budget, unsigned seed,
               int fail_at = 0) {
  std::mt19937 rng(seed);
  std::vector<ModelShape> models = {{22, 2, 4}, {200, 38, 4}, {1000, 120, 8}};
  Arena arena(budget);
  std::deque<Waiting> q;
  std::vector<Running> run;
  std::set<int64_t> done;
  std::vector<std::vector<int64_t>> order(models.size());   // submission order per model
  std::vector<int64_t> last_started(models.size(), 0);
  std::vector<bool> slot_busy(slots, false);
  std::map<int64_t, int> status;   // finished tickets -> status
  int fatal = kOk, finished_batches = 0;
  auto mark = [&](int64_t t, int st) {
    status[t] = st;
    done.insert(t);
  };
  const int n_req = 400;
  double t = 0.0, next_arrival = 0.0;
  int submitted = 0;
  int64_t ticket = 1;
  while ((int)done.size() < n_req) {
    // arrivals
    while (submitted < n_req && next_arrival <= t) {
      const int m = rng() % models.size();
      const int w = 1 + rng() % 256;
      if (models[m].batch_bytes(w) > budget || fatal != kOk) {   // refused at submission
        ++submitted;
        done.insert(-(int64_t)submitted);
        next_arrival += std::exponential_distribution<double>(1.0)(rng);
        continue;
      }
      q.push_back({ticket, m, w});
      order[m].push_back(ticket);
      ++ticket;
      ++submitted;
      next_arrival += std::exponential_distribution<double>(1.0)(rng);
    }
    if (fatal != kOk) {
      drain_waiting(q, fatal, mark);                 // nothing more is launched
    }
    // schedule while slots are free and memory admits
    while ((int)run.size() < slots && !q.empty()) {
      std::vector<size_t> pick = form_batch(q, max_batch, fifo);
      CHECK(!pick.empty() && pick[0] == 0);          // oldest request first
      int walkers = 0, model = q[pick[0]].model;
      for (size_t i : pick) {
        CHECK(q[i].model == model);                  // one model per batch
        walkers += q[i].walkers;
      }
      if (fifo) CHECK(pick.size() == 1);
      if (pick.size() > 1) CHECK(walkers <= max_batch);
      size_t off;
      if (!admit(q, pick, models[model], arena, &off, &walkers)) {
        CHECK(!run.empty());                         // something will free memory
        break;
      }
      CHECK(!pick.empty() && pick[0] == 0);          // shrinking keeps the oldest
      CHECK(arena.in_use() <= budget);
      int slot = 0;
      while (slot_busy[slot]) ++slot;
      CHECK(slot < slots);
      slot_busy[slot] = true;
      Running r{{}, off, t + 1e-3 * walkers, model, slot};
      for (size_t i : pick) {
        // FIFO within a model: tickets start in submission order
        CHECK(q[i].ticket > last_started[model]);
        last_started[model] = q[i].ticket;
        r.tickets.push_back(q[i].ticket);
      }
      for (auto it = pick.rbegin(); it != pick.rend(); ++it) q.erase(q.begin() + *it);
      run.push_back(r);
    }
    // advance to the next event
    double t_next = submitted < n_req ? next_arrival : 1e300;
    for (auto& r : run) t_next = r.end < t_next ? r.end : t_next;
    t = t_next;
    for (size_t i = 0; i < run.size();) {
      const int query = run[i].end <= t
                            ? (++finished_batches == fail_at ? kDeviceError : kSuccess)
                            : kNotReady;
      const Poll pr = poll_outcome(query, kSuccess, kNotReady);
      if (pr == Poll::pending) {
        ++i;
        continue;
      }
      for (int64_t tk : run[i].tickets) CHECK(!done.count(tk));   // completes exactly once
      const size_t before = arena.in_use();
      const int st = retire(pr, run[i].tickets, run[i].off, run[i].slot, arena, slot_busy, kOk,
                            kErr, &fatal, mark);
      CHECK(arena.in_use() < before);                 // its block went back
      CHECK(!slot_busy[run[i].slot]);
      CHECK(st == (pr == Poll::done ? kOk : kErr));
      for (int64_t tk : run[i].tickets) CHECK(status.at(tk) == st);
      run.erase(run.begin() + i);
    }
  }
  CHECK(arena.in_use() == 0);
  CHECK(q.empty());
  if (fail_at > 0) {
    CHECK(fatal == kErr);
    // every request that finished after the failure carries the error
    int n_err = 0;
    for (auto& kv : status) n_err += kv.second == kErr;
    CHECK(n_err >= 1);
  } else {
    CHECK(fatal == kOk);
    for (auto& kv : status) CHECK(kv.second == kOk);
  }
  return 0;
}

static int poll_test() {
  CHECK(poll_outcome(kNotReady, kSuccess, kNotReady) == Poll::pending);
  CHECK(poll_outcome(kSuccess, kSuccess, kNotReady) == Poll::done);
  // any other status (an asynchronous kernel or copy error) is final
  CHECK(poll_outcome(kDeviceError, kSuccess, kNotReady) == Poll::failed);
  CHECK(poll_outcome(1, kSuccess, kNotReady) == Poll::failed);
  return 0;
}

int main() {
  if (arena_test()) return 1;
  if (poll_test()) return 1;
  const size_t MB = 1 << 20;
  if (sim(false, 4, 4096, 512 * MB, 1)) return 1;      // roomy budget
  if (sim(false, 4, 512, 16 * MB, 2)) return 1;       // tight budget: admission waits
  if (sim(true, 1, 4096, 64 * MB, 3)) return 1;       // FIFO baseline
  if (sim(false, 8, 64, 8 * MB, 4)) return 1;         // small batches, many slots
  if (sim(false, 4, 4096, 512 * MB, 5, 7)) return 1;  // device error in the 7th batch
  if (sim(false, 4, 512, 16 * MB, 6, 30)) return 1;   // ... under admission pressure
  if (sim(true, 1, 4096, 64 * MB, 7, 1)) return 1;    // ... in the first FIFO batch
  std::printf("serve core ok\n");
  return 0;
}
