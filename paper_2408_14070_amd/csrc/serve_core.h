// Host-side core of the serving loop: the HBM arena allocator and the
// continuous-batching policy.  Pure C++ (no HIP): the library's executor
// drives it with real streams, and a CPU test drives it with a simulated
// executor.
//
// Policy.  Requests wait in arrival order.  When an execution slot is free
// the scheduler takes the OLDEST waiting request, then every later waiting
// request of the same model (system + ensemble), in arrival order, while the
// batch stays within max_batch_walkers; the batch is admitted only if its
// device memory fits the arena now.  A batch that does not fit waits for
// in-flight batches to finish and free memory (requests that arrive
// meanwhile join later batches).  A request whose memory can never fit the
// budget is rejected at submission.  FIFO mode (one request per batch, one
// slot) is the unbatched baseline.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace rid {
namespace serve {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, capacity) with coalescing of free ranges.
class Arena {
 public:
  explicit Arena(size_t capacity = 0) { reset(capacity); }
  void reset(size_t capacity) {
    cap_ = capacity;
    free_.clear();
    used_.clear();
    if (capacity) free_[0] = capacity;
    in_use_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_[*off] = bytes;
        in_use_ += bytes;
        return true;
      }
    }
    return false;
  }
  bool release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    size_t start = off, len = u->second;
    in_use_ -= len;
    used_.erase(u);
    auto nx = free_.lower_bound(start);
    if (nx != free_.end() && nx->first == start + len) {
      len += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == start) {
        start = pv->first;
        len += pv->second;
        free_.erase(pv);
      }
    }
    free_[start] = len;
    return true;
  }
  size_t capacity() const { return cap_; }
  size_t in_use() const { return in_use_; }
  size_t largest_free() const {
    size_t m = 0;
    for (auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }

 private:
  size_t cap_ = 0, in_use_ = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  std::map<size_t, size_t> used_;
};

struct Waiting {
  int64_t ticket;
  int model;
  int walkers;
};

// Device bytes a batch of `walkers` walkers of a model needs: inputs,
// outputs and the kernels' intermediates, each region 256-byte aligned.
struct ModelShape {
  int n_atoms = 0, n_cv = 0, K = 0;
  size_t batch_bytes(int walkers) const {
    const size_t w = (size_t)walkers;
    return align_up(w * n_atoms * 3 * 4)       // positions
           + align_up(w * (3 * n_atoms + 3) * 4)  // records: forces, energy, eps, sigma
           + align_up(w)                       // flags
           + align_up(w * K * 4)               // per-member A
           + align_up(w * K * n_cv * 4)        // per-member g
           + align_up(w * 2 * n_cv * 4);       // encoding (large systems)
  }
};

// Admission: allocate device memory for the longest prefix of `pick` (the
// batch in arrival order) that fits the arena now.  Shrinks `pick` to that
// prefix and returns true, or returns false (nothing fits; wait for memory).
inline bool admit(const std::deque<Waiting>& q, std::vector<size_t>& pick,
                  const ModelShape& shape, Arena& arena, size_t* off, int* walkers) {
  while (!pick.empty()) {
    int w = 0;
    for (size_t i : pick) w += q[i].walkers;
    if (arena.alloc(shape.batch_bytes(w), off)) {
      *walkers = w;
      return true;
    }
    pick.pop_back();
  }
  return false;
}

// Outcome of polling an in-flight batch's completion event.  Only the
// runtime's "not ready" status means the batch is still running; success
// means it finished; any other status is a device error (a failed kernel
// or copy), and the batch must not be polled again: its event may never
// signal.
enum class Poll { pending, done, failed };
inline Poll poll_outcome(int query_status, int success, int not_ready) {
  if (query_status == not_ready) return Poll::pending;
  return query_status == success ? Poll::done : Poll::failed;
}

// Retire an in-flight batch whose poll was not pending: each of its requests
// is finished with ok_status, or after a device error with err_status (and
// *fatal is set, so later submissions are refused and waiting requests are
// failed instead of launched); its arena block and stream slot are freed.
// mark(ticket, status) finishes one request.  Returns the status given.
template <class Mark>
inline int retire(Poll p, const std::vector<int64_t>& tickets, size_t dev_off, int slot,
                  Arena& dev, std::vector<bool>& slot_busy, int ok_status, int err_status,
                  int* fatal, Mark&& mark) {
  const int st = p == Poll::done ? ok_status : err_status;
  if (p == Poll::failed && *fatal == ok_status) *fatal = err_status;
  for (int64_t t : tickets) mark(t, st);
  dev.release(dev_off);
  slot_busy[slot] = false;
  return st;
}

// Finish every waiting request with `status` (server stopping, or fatal
// after a device error) and empty the queue.
template <class Mark>
inline void drain_waiting(std::deque<Waiting>& q, int status, Mark&& mark) {
  for (const Waiting& w : q) mark(w.ticket, status);
  q.clear();
}

// Choose the next batch from the waiting queue (indices into `q`).  Returns
// an empty vector if the queue is empty.
inline std::vector<size_t> form_batch(const std::deque<Waiting>& q, int max_batch_walkers,
                                      bool fifo) {
  std::vector<size_t> pick;
  if (q.empty()) return pick;
  const int model = q.front().model;
  int total = 0;
  for (size_t i = 0; i < q.size(); ++i) {
    if (q[i].model != model) continue;
    if (!pick.empty() && (fifo || total + q[i].walkers > max_batch_walkers)) break;
    pick.push_back(i);
    total += q[i].walkers;
    if (fifo) break;
  }
  return pick;
}

}  // namespace serve
}  // namespace rid
