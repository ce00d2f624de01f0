// Serving loop: continuous batching of bias-force requests from many
// walkers of different systems and ensembles on one GPU.
//
// A request is a block of walkers of one registered model (system +
// ensemble + trust levels).  Ensemble weights and system tables stay
// resident.  A host request's positions are staged in pinned host memory
// and its results copied back; a device request's positions are read from
// the caller's device buffer and its results written to the caller's device
// buffers (walker state resident in HBM: no PCIe traffic), by one gather and
// one scatter launch per batch over the batch's device requests.  A
// scheduler thread forms batches (serve_core.h policy), admits them against
// an HBM arena of fixed budget, and runs each batch on one of several
// streams: one host-to-device copy per member request, the MLP kernel fed
// from positions, the deviation/switch/chain-rule kernel writing one record
// per walker (forces, then energy, eps, sigma), and one device-to-host copy
// per request, then an event.  HIP calls and host copies run outside the
// server lock.  A completion thread
// polls the events, frees the batch's memory and wakes waiters and the
// scheduler, so requests that arrive while batches are on the GPU are
// admitted as slots and memory free up.  Results do not depend on the
// batch a request lands in: every kernel computes each walker's row
// independently, with a fixed reduction order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rid_internal.h"
#include "serve_core.h"

namespace rid {
namespace {

using clk = std::chrono::steady_clock;

struct ServeModel {
  rid_system_impl* sys;
  rid_ensemble_impl* ens;
  float eps0, eps1;
  serve::ModelShape shape;
};

// Device buffers of a device request (caller owned).
struct DevIo {
  const float* pos = nullptr;    // [w][N][3]
  float* force = nullptr;        // [w][N][3] or null
  float* energy = nullptr;       // [w] or null
  float* eps = nullptr;
  float* sigma = nullptr;
};

struct Req {
  int model = 0;
  int walkers = 0;
  size_t pin_off = 0;
  float* pin = nullptr;          // [w][N][3] positions, then [w] output records
  bool own_pin = false;          // pinned block outside the staging arena
  bool dev = false;              // device request: io instead of pin
  DevIo io;
  clk::time_point arrival, done_at;
  bool done = false;
  rid_status status = RID_OK;
};

struct Part {
  float* pin;                    // host request: its pinned block (else null)
  DevIo io;                      // device request: its buffers
  int walkers;
};

struct Batch {
  std::vector<int64_t> tickets;
  std::vector<Part> parts;       // the requests, in the batch's row order
  int model = 0, walkers = 0, slot = 0;
  size_t dev_off = 0;
};

// Device requests of one gather / scatter launch (kernel arguments).
constexpr int kMaxDevParts = 32;
struct DevParts {
  int n;                         // parts in this launch
  int row0[kMaxDevParts];        // first batch row of each part
  int walkers[kMaxDevParts];
  DevIo io[kMaxDevParts];
};

// positions of the device parts into the batch's rows: block row y = part
__global__ void serve_gather_kernel(DevParts p, float* pos, int n3) {
  const int q = blockIdx.y;
  const long long count = (long long)p.walkers[q] * n3;
  const float* src = p.io[q].pos;
  float* dst = pos + (long long)p.row0[q] * n3;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// the batch's walker records (3N forces, energy, eps, sigma) into the device
// parts' output buffers
__global__ void serve_scatter_kernel(DevParts p, const float* rec, int n3) {
  const int q = blockIdx.y;
  const int rf = n3 + 3;
  const long long count = (long long)p.walkers[q] * rf;
  const float* src = rec + (long long)p.row0[q] * rf;
  const DevIo& io = p.io[q];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    const long long w = i / rf;
    const int j = (int)(i - w * rf);
    const float v = src[i];
    if (j < n3) {
      if (io.force) io.force[w * n3 + j] = v;
    } else if (j == n3) {
      if (io.energy) io.energy[w] = v;
    } else if (j == n3 + 1) {
      if (io.eps) io.eps[w] = v;
    } else if (io.sigma) {
      io.sigma[w] = v;
    }
  }
}

// One walker's output record: 3N forces, energy, eps, sigma.
inline int rec_floats(int n_atoms) { return 3 * n_atoms + 3; }

// Pinned layout of one request: positions, then the output records.
inline size_t pin_pos_bytes(int w, int n_atoms) {
  return serve::align_up((size_t)w * n_atoms * 3 * 4);
}
inline size_t pin_bytes(int w, int n_atoms) {
  return pin_pos_bytes(w, n_atoms) + (size_t)w * rec_floats(n_atoms) * 4;
}

}  // namespace

struct Server {
  int device = 0;
  size_t budget = 0;
  int n_slots = 1, max_batch = 4096;
  bool fifo = false;
  void* dev_base = nullptr;
  void* pin_base = nullptr;
  serve::Arena dev, pin;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<bool> slot_busy;
  std::vector<ServeModel> models;

  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_poll;   // cv_poll: a batch went in flight
  std::deque<serve::Waiting> waiting;
  std::unordered_map<int64_t, Req> reqs;
  std::vector<Batch> inflight;
  int64_t next_ticket = 1;
  int launching = 0;               // batches being launched outside the lock
  int waiters = 0;                 // threads inside rid_server_wait
  bool stop = false;
  int fatal = RID_OK;              // first device error; then nothing more is launched
  std::thread sched, poller;

  // statistics
  std::vector<double> lat_us;
  int64_t walkers_done = 0, requests_done = 0, batches = 0, batch_walkers = 0;
  int64_t admission_waits = 0, max_inflight = 0;
  bool have_first = false;
  clk::time_point first_arrival, last_done;

  void run_scheduler();
  void run_poller();
  // queue a filled-in request (under the lock); returns its ticket
  int64_t enqueue(Req& r) {
    r.arrival = clk::now();
    if (!have_first) {
      first_arrival = r.arrival;
      have_first = true;
    }
    const int64_t t = next_ticket++;
    const int model = r.model, w = r.walkers;
    reqs.emplace(t, r);
    waiting.push_back({t, model, w});
    cv_sched.notify_all();
    return t;
  }
  // finish request t with status st (under the lock)
  void mark(int64_t t, int st) {
    Req& r = reqs[t];
    r.status = (rid_status)st;
    r.done = true;
    r.done_at = clk::now();
  }
  rid_status launch(const Batch& b, const ServeModel& m);
};

rid_status Server::launch(const Batch& b, const ServeModel& m) {
  const int W = b.walkers, N = m.sys->n_atoms, n = m.sys->n_cv, K = m.ens->K;
  const int RF = rec_floats(N);
  unsigned char* base = static_cast<unsigned char*>(dev_base) + b.dev_off;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base + off;
    off += serve::align_up(bytes);
    return p;
  };
  float* pos = reinterpret_cast<float*>(take((size_t)W * N * 3 * 4));
  float* rec = reinterpret_cast<float*>(take((size_t)W * RF * 4));
  uint8_t* flags = reinterpret_cast<uint8_t*>(take((size_t)W));
  float* A = reinterpret_cast<float*>(take((size_t)W * K * 4));
  float* g = reinterpret_cast<float*>(take((size_t)W * K * n * 4));
  float* x = reinterpret_cast<float*>(take((size_t)W * 2 * n * 4));
  hipStream_t st = streams[b.slot];
  // device parts in groups of kMaxDevParts (one gather and one scatter
  // launch per group), host parts one copy each way
  std::vector<DevParts> groups;
  int wo = 0;
  for (const auto& pr : b.parts) {
    if (pr.pin) {
      RID_HIP(hipMemcpyAsync(pos + (size_t)wo * N * 3, pr.pin, (size_t)pr.walkers * N * 3 * 4,
                             hipMemcpyHostToDevice, st));
    } else {
      if (groups.empty() || groups.back().n == kMaxDevParts) groups.push_back(DevParts{});
      DevParts& g = groups.back();
      g.row0[g.n] = wo;
      g.walkers[g.n] = pr.walkers;
      g.io[g.n] = pr.io;
      ++g.n;
    }
    wo += pr.walkers;
  }
  auto grid_for = [&](const DevParts& g, int per_walker) {
    int most = 0;
    for (int q = 0; q < g.n; ++q) most = std::max(most, g.walkers[q]);
    const long long count = (long long)most * per_walker;
    return dim3((unsigned)std::min<long long>((count + 255) / 256, 1024), (unsigned)g.n);
  };
  for (const DevParts& g : groups) {
    hipLaunchKernelGGL(serve_gather_kernel, grid_for(g, 3 * N), dim3(256), 0, st, g, pos, 3 * N);
    RID_HIP(hipGetLastError());
  }
  const TorsionInput tin{m.sys, pos};
  rid_status rs = launch_mlp_from_pos(*m.ens, tin, W, A, g, st);
  if (rs == RID_EUNSUPPORTED) {   // too many torsion atoms for the in-kernel gather
    rs = launch_cv_eval(*m.sys, pos, W, nullptr, x, st);
    if (rs == RID_OK) rs = launch_mlp(*m.ens, x, W, A, g, st);
  }
  if (rs != RID_OK) return rs;
  rs = launch_bias_scatter(*m.sys, K, pos, W, A, g, nullptr, m.eps0, m.eps1, rec, rec + 3 * N,
                           rec + 3 * N + 1, rec + 3 * N + 2, flags, st, RF);
  if (rs != RID_OK) return rs;
  for (const DevParts& g : groups) {
    hipLaunchKernelGGL(serve_scatter_kernel, grid_for(g, RF), dim3(256), 0, st, g, rec, 3 * N);
    RID_HIP(hipGetLastError());
  }
  wo = 0;
  for (const auto& pr : b.parts) {
    if (pr.pin) {
      unsigned char* out = reinterpret_cast<unsigned char*>(pr.pin) + pin_pos_bytes(pr.walkers, N);
      RID_HIP(hipMemcpyAsync(out, rec + (size_t)wo * RF, (size_t)pr.walkers * RF * 4,
                             hipMemcpyDeviceToHost, st));
    }
    wo += pr.walkers;
  }
  RID_HIP(hipEventRecord(events[b.slot], st));
  return RID_OK;
}

void Server::run_scheduler() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  while (!stop) {
    if (fatal != RID_OK && !waiting.empty()) {
      // a device error stopped the server: fail what is still queued
      serve::drain_waiting(waiting, fatal, [&](int64_t t, int st) { mark(t, st); });
      cv_done.notify_all();
      continue;
    }
    int slot = -1;
    for (int s = 0; s < n_slots; ++s)
      if (!slot_busy[s]) {
        slot = s;
        break;
      }
    if (waiting.empty() || slot < 0) {
      cv_sched.wait(lk);
      continue;
    }
    std::vector<size_t> pick = serve::form_batch(waiting, max_batch, fifo);
    Batch b;
    b.model = waiting[pick.front()].model;
    size_t off = 0;
    if (!serve::admit(waiting, pick, models[b.model].shape, dev, &off, &b.walkers)) {
      // admission: wait for an in-flight batch to finish and free memory
      ++admission_waits;
      if (inflight.empty()) {
        // the arena is empty and the oldest request still does not fit
        // (submission checks this, so only reachable on a logic error)
        Req& r = reqs[waiting.front().ticket];
        r.status = RID_ENOMEM;
        r.done = true;
        r.done_at = clk::now();
        waiting.pop_front();
        cv_done.notify_all();
        continue;
      }
      cv_sched.wait(lk);
      continue;
    }
    b.dev_off = off;
    b.slot = slot;
    for (size_t i : pick) {
      const int64_t t = waiting[i].ticket;
      b.tickets.push_back(t);
      const Req& r = reqs[t];
      b.parts.push_back(Part{r.dev ? nullptr : r.pin, r.io, r.walkers});
    }
    for (auto it = pick.rbegin(); it != pick.rend(); ++it) waiting.erase(waiting.begin() + *it);
    slot_busy[slot] = true;
    const ServeModel m = models[b.model];   // register() may grow the table meanwhile
    ++launching;
    lk.unlock();
    rid_status rs = launch(b, m);
    lk.lock();
    --launching;
    if (rs != RID_OK) {
      // the launch itself failed: this batch's requests carry its status
      serve::retire(serve::Poll::failed, b.tickets, off, slot, dev, slot_busy, RID_OK, rs,
                    &fatal, [&](int64_t t, int st) { mark(t, st); });
      cv_done.notify_all();
      continue;
    }
    ++batches;
    batch_walkers += b.walkers;
    inflight.push_back(std::move(b));
    max_inflight = std::max<int64_t>(max_inflight, (int64_t)inflight.size());
    cv_poll.notify_one();
  }
}

void Server::run_poller() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  while (!stop || !inflight.empty() || launching > 0) {
    bool any = false;
    for (size_t i = 0; i < inflight.size();) {
      Batch& b = inflight[i];
      const serve::Poll pr =
          serve::poll_outcome((int)hipEventQuery(events[b.slot]), (int)hipSuccess,
                              (int)hipErrorNotReady);
      if (pr == serve::Poll::pending) {
        ++i;
        continue;
      }
      // finished, or a device error (its event may never signal): either
      // way the batch leaves the in-flight list and its waiters wake
      if (pr == serve::Poll::failed) (void)hipGetLastError();
      serve::retire(pr, b.tickets, b.dev_off, b.slot, dev, slot_busy, RID_OK, RID_EDEVICE,
                    &fatal, [&](int64_t t, int st) { mark(t, st); });
      inflight.erase(inflight.begin() + i);
      any = true;
    }
    if (any) {
      cv_done.notify_all();
      cv_sched.notify_all();
    }
    if (inflight.empty()) {
      if (stop && launching == 0) break;
      cv_poll.wait_for(lk, std::chrono::milliseconds(2));
    } else if (!any) {
      // poll again in ~10 us (a sleep this short would overshoot by the
      // timer slack, tens of microseconds)
      lk.unlock();
      const auto until = clk::now() + std::chrono::microseconds(10);
      while (clk::now() < until) std::this_thread::yield();
      lk.lock();
    }
  }
}

}  // namespace rid

using namespace rid;

struct rid_server_s {
  Server s;
};

extern "C" {

rid_status rid_server_create(size_t hbm_budget_bytes, int n_streams,
                             int max_batch_walkers, int flags, rid_server* out) {
  if (!out) return fail(RID_EINVAL, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes < (1u << 20) || n_streams < 1 || n_streams > 16 || max_batch_walkers < 1)
    return fail(RID_EINVAL, "need budget >= 1 MiB, 1 <= n_streams <= 16, max_batch_walkers >= 1");
  rid_server_s* h = new (std::nothrow) rid_server_s();
  if (!h) return fail(RID_ENOMEM, "host allocation failed");
  Server& s = h->s;
  (void)hipGetDevice(&s.device);
  s.fifo = (flags & RID_SERVE_FIFO) != 0;
  s.n_slots = s.fifo ? 1 : n_streams;
  s.max_batch = max_batch_walkers;
  s.budget = hbm_budget_bytes;
  const size_t pin_cap = (size_t)1 << 30;     // pinned staging arena
  if (hipMalloc(&s.dev_base, hbm_budget_bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete h;
    return fail(RID_ENOMEM, "HBM budget allocation failed");
  }
  if (hipHostMalloc(&s.pin_base, pin_cap, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(s.dev_base);
    delete h;
    return fail(RID_ENOMEM, "pinned staging allocation failed");
  }
  s.dev.reset(hbm_budget_bytes);
  s.pin.reset(pin_cap);
  s.streams.resize(s.n_slots);
  s.events.resize(s.n_slots);
  s.slot_busy.assign(s.n_slots, false);
  for (int i = 0; i < s.n_slots; ++i) {
    if (hipStreamCreateWithFlags(&s.streams[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.events[i], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      for (int j = 0; j < i; ++j) {
        (void)hipStreamDestroy(s.streams[j]);
        (void)hipEventDestroy(s.events[j]);
      }
      (void)hipFree(s.dev_base);
      (void)hipHostFree(s.pin_base);
      delete h;
      return fail(RID_EDEVICE, "stream creation failed");
    }
  }
  s.sched = std::thread([&s] { s.run_scheduler(); });
  s.poller = std::thread([&s] { s.run_poller(); });
  *out = h;
  return RID_OK;
}

rid_status rid_server_register(rid_server srv, rid_system sys, rid_ensemble ens,
                               float eps0, float eps1, int* model_id) {
  if (!srv || !sys || !ens || !model_id) return fail(RID_EINVAL, "NULL argument");
  if (!(eps0 >= 0.f) || !(eps0 < eps1)) return fail(RID_EINVAL, "trust levels need 0 <= eps0 < eps1");
  if (sys->impl.n_cv != ens->impl.n_cv) return fail(RID_EINVAL, "system and ensemble disagree on n_cv");
  if (!cv_kinds_match(sys->impl, ens->impl))
    return fail(RID_EINVAL, "the ensemble's angular mask does not match the system's CV kinds");
  Server& s = srv->s;
  rid_ensemble_impl& e = ens->impl;
  if (e.frag_dirty) {
    rid_status rs = pack_ensemble_weights(e, nullptr);
    if (rs != RID_OK) return rs;
    RID_HIP(hipStreamSynchronize(nullptr));
    e.frag_dirty = false;
  }
  std::lock_guard<std::mutex> lk(s.mu);
  ServeModel m{&sys->impl, &e, eps0, eps1, {}};
  m.shape.n_atoms = sys->impl.n_atoms;
  m.shape.n_cv = sys->impl.n_cv;
  m.shape.K = e.K;
  s.models.push_back(m);
  *model_id = (int)s.models.size() - 1;
  return RID_OK;
}

rid_status rid_server_submit(rid_server srv, int model_id, const float* host_pos,
                             int n_walkers, int64_t* ticket) {
  if (!srv || !host_pos || !ticket) return fail(RID_EINVAL, "NULL argument");
  Server& s = srv->s;
  std::unique_lock<std::mutex> lk(s.mu);
  if (model_id < 0 || model_id >= (int)s.models.size()) return fail(RID_EINVAL, "unknown model id");
  if (n_walkers < 1) return fail(RID_EINVAL, "n_walkers must be >= 1");
  if (s.fatal != RID_OK) return fail((rid_status)s.fatal, "server stopped after a device error");
  if (s.stop) return fail(RID_EINVAL, "server is being destroyed");
  const ServeModel& m = s.models[model_id];
  if (m.shape.batch_bytes(n_walkers) > s.dev.capacity())
    return fail(RID_ENOMEM, "request larger than the HBM budget");
  const int N = m.shape.n_atoms;
  const size_t pb = pin_bytes(n_walkers, N);
  size_t poff = 0;
  Req r;
  r.model = model_id;
  r.walkers = n_walkers;
  if (s.pin.alloc(pb, &poff)) {
    r.pin_off = poff;
    r.pin = reinterpret_cast<float*>(static_cast<unsigned char*>(s.pin_base) + poff);
  } else {
    // staging arena full (many requests outstanding): a pinned block of its
    // own, so a client that submits many requests before waiting never
    // blocks here
    lk.unlock();
    void* p = nullptr;
    const bool ok = hipHostMalloc(&p, pb, hipHostMallocDefault) == hipSuccess;
    if (!ok) (void)hipGetLastError();
    lk.lock();
    if (!ok) return fail(RID_ENOMEM, "pinned staging allocation failed");
    r.pin = static_cast<float*>(p);
    r.own_pin = true;
  }
  // the block is ours until the request is enqueued: copy without the lock
  lk.unlock();
  std::memcpy(r.pin, host_pos, (size_t)n_walkers * N * 3 * 4);
  lk.lock();
  *ticket = s.enqueue(r);
  return RID_OK;
}

rid_status rid_server_submit_device(rid_server srv, int model_id, const float* d_pos,
                                    int n_walkers, float* d_force, float* d_energy,
                                    float* d_eps, float* d_sigma, int64_t* ticket) {
  if (!srv || !d_pos || !ticket) return fail(RID_EINVAL, "NULL argument");
  Server& s = srv->s;
  std::lock_guard<std::mutex> lk(s.mu);
  if (model_id < 0 || model_id >= (int)s.models.size()) return fail(RID_EINVAL, "unknown model id");
  if (n_walkers < 1) return fail(RID_EINVAL, "n_walkers must be >= 1");
  if (s.fatal != RID_OK) return fail((rid_status)s.fatal, "server stopped after a device error");
  if (s.stop) return fail(RID_EINVAL, "server is being destroyed");
  if (s.models[model_id].shape.batch_bytes(n_walkers) > s.dev.capacity())
    return fail(RID_ENOMEM, "request larger than the HBM budget");
  Req r;
  r.model = model_id;
  r.walkers = n_walkers;
  r.dev = true;
  r.io = DevIo{d_pos, d_force, d_energy, d_eps, d_sigma};
  *ticket = s.enqueue(r);
  return RID_OK;
}

rid_status rid_server_wait(rid_server srv, int64_t ticket, float* host_force,
                           float* host_energy, float* host_eps, float* host_sigma,
                           double* latency_us) {
  if (!srv) return fail(RID_EINVAL, "NULL argument");
  Server& s = srv->s;
  std::unique_lock<std::mutex> lk(s.mu);
  if (s.reqs.find(ticket) == s.reqs.end()) return fail(RID_EINVAL, "unknown ticket");
  // counted from here to the last touch of the server below: destroy waits
  // until no waiter is left before it frees anything
  ++s.waiters;
  // look the request up again after every wake-up: other threads' submits
  // may rehash the table (references stay valid, iterators do not)
  Req& r = s.reqs.find(ticket)->second;
  s.cv_done.wait(lk, [&] { return r.done; });
  const rid_status st = r.status;
  const Req done = r;   // this waiter owns the finished request from here on
  const int N = s.models[r.model].shape.n_atoms;
  lk.unlock();
  if (st == RID_OK && !done.dev) {
    const int w = done.walkers, RF = rec_floats(N);
    const float* rec = reinterpret_cast<const float*>(
        reinterpret_cast<const unsigned char*>(done.pin) + pin_pos_bytes(w, N));
    for (int i = 0; i < w; ++i) {
      const float* ri = rec + (size_t)i * RF;
      if (host_force) std::memcpy(host_force + (size_t)i * 3 * N, ri, (size_t)3 * N * 4);
      if (host_energy) host_energy[i] = ri[3 * N];
      if (host_eps) host_eps[i] = ri[3 * N + 1];
      if (host_sigma) host_sigma[i] = ri[3 * N + 2];
    }
  }
  if (done.own_pin) (void)hipHostFree(done.pin);
  lk.lock();
  if (st == RID_OK) {
    const double us = std::chrono::duration<double, std::micro>(done.done_at - done.arrival).count();
    if (latency_us) *latency_us = us;
    s.lat_us.push_back(us);
    s.walkers_done += done.walkers;
    s.requests_done += 1;
    if (done.done_at > s.last_done) s.last_done = done.done_at;
  }
  if (!done.dev && !done.own_pin) s.pin.release(done.pin_off);
  s.reqs.erase(ticket);
  --s.waiters;
  if (s.stop) s.cv_done.notify_all();   // wake destroy, which waits for the last waiter
  lk.unlock();
  if (st != RID_OK) return fail(st, "request failed (device error, or the server was destroyed)");
  return RID_OK;
}

rid_status rid_server_replay(rid_server srv, const rid_replay_request* reqs, int n,
                             double* latency_us, double* submit_lag_us, double* wall_s) {
  if (!srv || !reqs || n < 1) return fail(RID_EINVAL, "need a server and n >= 1 requests");
  for (int i = 0; i < n; ++i)
    if (!reqs[i].pos || reqs[i].n_walkers < 1 || !(reqs[i].arrival_s >= 0.0) ||
        (i > 0 && reqs[i].arrival_s < reqs[i - 1].arrival_s))
      return fail(RID_EINVAL, "requests need positions, walkers >= 1 and arrival times in order");
  std::vector<int64_t> tickets(n, 0);
  std::vector<rid_status> sub(n, RID_OK);
  std::mutex m;
  std::condition_variable cv;
  int submitted = 0;
  const clk::time_point t0 = clk::now();
  // the submitting thread releases each request at its arrival time: a
  // sleep until ~100 us before it, then a spin
  std::thread producer([&] {
    for (int i = 0; i < n; ++i) {
      const rid_replay_request& q = reqs[i];
      const clk::time_point due =
          t0 + std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(q.arrival_s));
      const clk::time_point wake = due - std::chrono::microseconds(100);
      if (clk::now() < wake) std::this_thread::sleep_until(wake);
      while (clk::now() < due) std::this_thread::yield();
      if (submit_lag_us)
        submit_lag_us[i] = std::chrono::duration<double, std::micro>(clk::now() - due).count();
      int64_t t = 0;
      const rid_status rs =
          q.device ? rid_server_submit_device(srv, q.model_id, q.pos, q.n_walkers, q.force,
                                              q.energy, q.eps, q.sigma, &t)
                   : rid_server_submit(srv, q.model_id, q.pos, q.n_walkers, &t);
      {
        std::lock_guard<std::mutex> lk(m);
        tickets[i] = t;
        sub[i] = rs;
        submitted = i + 1;
      }
      cv.notify_one();
    }
  });
  rid_status first_err = RID_OK;
  for (int i = 0; i < n; ++i) {
    {
      std::unique_lock<std::mutex> lk(m);
      cv.wait(lk, [&] { return submitted > i; });
    }
    double lat = 0.0;
    rid_status rs = sub[i];
    if (rs == RID_OK)
      rs = rid_server_wait(srv, tickets[i], reqs[i].device ? nullptr : reqs[i].force,
                           reqs[i].device ? nullptr : reqs[i].energy,
                           reqs[i].device ? nullptr : reqs[i].eps,
                           reqs[i].device ? nullptr : reqs[i].sigma, &lat);
    if (latency_us) latency_us[i] = rs == RID_OK ? lat : -1.0;
    if (rs != RID_OK && first_err == RID_OK) first_err = rs;
  }
  producer.join();
  if (wall_s) *wall_s = std::chrono::duration<double>(clk::now() - t0).count();
  if (first_err != RID_OK) return fail(first_err, "a replayed request failed");
  return RID_OK;
}

rid_status rid_server_stats(rid_server srv, rid_server_stats_t* out) {
  if (!srv || !out) return fail(RID_EINVAL, "NULL argument");
  Server& s = srv->s;
  std::lock_guard<std::mutex> lk(s.mu);
  std::memset(out, 0, sizeof(*out));
  out->requests_done = s.requests_done;
  out->walkers_done = s.walkers_done;
  out->batches = s.batches;
  out->admission_waits = s.admission_waits;
  out->max_inflight_batches = s.max_inflight;
  out->mean_batch_walkers = s.batches ? (double)s.batch_walkers / s.batches : 0.0;
  if (!s.lat_us.empty()) {
    std::vector<double> v = s.lat_us;
    std::sort(v.begin(), v.end());
    auto q = [&](double f) { return v[std::min(v.size() - 1, (size_t)(f * (v.size() - 1) + 0.5))]; };
    out->p50_us = q(0.50);
    out->p99_us = q(0.99);
    out->max_us = v.back();
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_us = sum / v.size();
    const double span = std::chrono::duration<double>(s.last_done - s.first_arrival).count();
    out->walker_steps_per_s = span > 0 ? s.walkers_done / span : 0.0;
  }
  return RID_OK;
}

void rid_server_reset_stats(rid_server srv) {
  if (!srv) return;
  Server& s = srv->s;
  std::lock_guard<std::mutex> lk(s.mu);
  s.lat_us.clear();
  s.walkers_done = s.requests_done = s.batches = s.batch_walkers = 0;
  s.admission_waits = s.max_inflight = 0;
  s.have_first = false;
}

void rid_server_destroy(rid_server srv) {
  if (!srv) return;
  Server& s = srv->s;
  {
    std::lock_guard<std::mutex> lk(s.mu);
    s.stop = true;
  }
  s.cv_sched.notify_all();
  s.cv_poll.notify_all();
  if (s.sched.joinable()) s.sched.join();
  if (s.poller.joinable()) s.poller.join();   // returns once nothing is in flight
  {
    // requests never launched are failed, and their waiters (if any) must
    // leave rid_server_wait before the server's memory goes away
    std::unique_lock<std::mutex> lk(s.mu);
    serve::drain_waiting(s.waiting, RID_EINVAL, [&](int64_t t, int st) { s.mark(t, st); });
    s.cv_done.notify_all();
    s.cv_done.wait(lk, [&] { return s.waiters == 0; });
  }
  for (auto st : s.streams) (void)hipStreamSynchronize(st);
  for (auto st : s.streams) (void)hipStreamDestroy(st);
  for (auto ev : s.events) (void)hipEventDestroy(ev);
  if (s.dev_base) (void)hipFree(s.dev_base);
  if (s.pin_base) (void)hipHostFree(s.pin_base);
  delete srv;
}

}  // extern "C"
