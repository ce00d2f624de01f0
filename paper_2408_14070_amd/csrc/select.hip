// Selection phase ("Selection"; "SelectorConfig": cluster_threshold,
// numb_cluster_lower / numb_cluster_upper, max_selection): the CV frames
// whose model deviation reaches the lower trust level are clustered with a
// distance threshold, the threshold is adapted until the cluster count lies
// in the window, and one representative per cluster is selected.
//
// Clustering (the paper names a threshold, not the algorithm): frames in
// order; a frame joins the first cluster, in founding order, whose leader is
// within the threshold, otherwise it founds a cluster and leads it.  The
// distance is periodic in every angular CV (differences wrapped to
// (-pi, pi]; raw CVs unwrapped), each square optionally weighted by the CV's
// clustering weight (the CV settings' "weights"), and the decision
// d^2 <= t^2 is taken in FP32 with the squares summed in CV order,
// contraction off, so the labels do not depend on the launch shape.
//
// GPU form of the sequential rule, exact: frames go in chunks.  A parallel
// kernel compares every frame of the chunk with all leaders founded before
// it (one wave per frame, lanes over leaders, first hit by ballot); a
// single workgroup then resolves the chunk's unmatched frames in order
// against the leaders founded inside the chunk (kept in LDS) and founds new
// ones.  A frame's
// first match among the earlier leaders is its first match overall, because
// later leaders only append.  Chunks grow from 64 frames, so the first
// leaders are found by the single wave over few frames and most frames are
// then resolved by the parallel kernel.  With threshold adjustment, one pass
// clusters up to kSlots thresholds side by side (blockIdx.y = slot, each with
// its own workspace); select_core.h takes the rule's steps over their counts.
#include "device_common.h"
#include "select_core.h"

namespace rid {
namespace {

using namespace dev;

constexpr int kPending = -3;       // unmatched after the parallel pass
constexpr int kFiltered = -2;      // eps below eps0
constexpr int kOverCap = -1;       // would found a cluster past the cap
constexpr int kMatchWaves = 4;
constexpr int kMaxSelCv = 256;
constexpr int kChunkMax = 8192;
constexpr int kLdsRows = 16384;    // floats for the new leaders, and again for a frame group
constexpr int kSlots = 24;         // thresholds clustered side by side in one pass
static_assert(kSlots <= selcore::kMaxSlots, "slot count");

struct ClusterArgs {
  const float* s;        // [B][n] frames
  const float* eps;      // [B] or null (no filter)
  float eps0, t2;
  int B, n, cap, chunk;
  float* LT;             // [n][cap] leaders' CVs, CV-major
  int* leader;           // [cap] frame index of each leader
  int* state;            // [0] leaders so far, [1] next frame, [2] over the cap
  int* labels;           // [B]
  unsigned long long* pend;   // [ceil(B/64)] bit f%64 of word f/64: frame f unmatched
  const uint8_t* raw;    // [n] or null: CVs with raw[i] = 1 are not periodic
  const float* w;        // [n] or null: per-CV weights of the squared differences
};

// Thresholds clustered in one pass: slot k (blockIdx.y) clusters at t2[k]
// into its own workspace, the pointers above advanced by k strides.
struct ClusterSlots {
  float t2[kSlots];
  long long sLT, sLabels;   // floats of LT, ints of labels per slot (labels: 0 with one slot)
  int sLeader, sPend;       // ints of leader, words of pend per slot
};
constexpr int kStateInts = 4;   // ints of state per slot

__device__ inline ClusterArgs slot_args(const ClusterArgs& a0, const ClusterSlots& sl) {
  const int k = blockIdx.y;
  ClusterArgs a = a0;
  a.t2 = sl.t2[k];
  a.LT += k * sl.sLT;
  a.labels += k * sl.sLabels;
  a.leader += k * sl.sLeader;
  a.pend += (size_t)k * sl.sPend;
  a.state += k * kStateInts;
  return a;
}

// Squared distance leader - frame with non-periodic CVs (raw non-null:
// raw[i] = 1 leaves the difference unwrapped) and/or per-CV weights (w
// non-null: each square is multiplied by w[i] before it is added);
// otherwise as leader_d2.
__device__ inline float leader_d2_general(const float* lead, long long ls, const float* x, int n,
                                          const uint8_t* raw, const float* w) {
#pragma clang fp contract(off)
  constexpr float kPi = 3.14159265358979f;
  constexpr float kTwoPi = 6.28318530717959f;
  float acc = 0.f;
  for (int i = 0; i < n; ++i) {
    float d = lead[i * ls] - x[i];
    if (!raw || !raw[i]) {
      if (d > kPi) d = d - kTwoPi;
      if (d <= -kPi) d = d + kTwoPi;
    }
    float sq = d * d;
    if (w) sq = sq * w[i];
    acc = acc + sq;
  }
  return acc;
}

// Squared periodic distance leader - frame, the leader's CV i at lead[i * ls],
// the frame's at x[i]; FP32, CV order, no fused multiply-add.
__device__ inline float leader_d2(const float* lead, long long ls, const float* x, int n,
                                  const uint8_t* raw, const float* w) {
#pragma clang fp contract(off)
  if (raw || w) return leader_d2_general(lead, ls, x, n, raw, w);
  constexpr float kPi = 3.14159265358979f;
  constexpr float kTwoPi = 6.28318530717959f;
  float acc = 0.f;
#pragma unroll 8
  for (int i = 0; i < n; ++i) {   // unrolled: loads issue ahead, sum order unchanged
    float d = lead[i * ls] - x[i];
    if (d > kPi) d = d - kTwoPi;
    if (d <= -kPi) d = d + kTwoPi;
    acc = acc + d * d;
  }
  return acc;
}

__global__ void sel_init_kernel(int* state, unsigned long long* pend, int words) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  state += blockIdx.y * kStateInts;
  pend += (size_t)blockIdx.y * words;
  if (t < 3) state[t] = 0;
  for (int w = t; w < words; w += gridDim.x * blockDim.x) pend[w] = 0ull;
}

// Frames [f_next, f_next + chunk): filtered, matched to the first earlier
// leader within the threshold, over the cap (no match and no room for a new
// cluster), or marked unmatched in the bit mask.
__global__ __launch_bounds__(kMatchWaves * kWave) void sel_match_kernel(ClusterArgs a0,
                                                                        ClusterSlots sl) {
  const ClusterArgs a = slot_args(a0, sl);
  __shared__ float xs[kMatchWaves][kMaxSelCv];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int f0 = a.state[1];
  const int f = f0 + blockIdx.x * kMatchWaves + wave;
  if (f >= min(a.B, f0 + a.chunk)) return;
  if (a.eps && !(a.eps[f] >= a.eps0)) {
    if (lane == 0) a.labels[f] = kFiltered;
    return;
  }
  const int n = a.n;
  for (int i = lane; i < n; i += kWave) xs[wave][i] = a.s[(size_t)f * n + i];
  __builtin_amdgcn_wave_barrier();
  const int nl = a.state[0];
  int lab = kPending;
  for (int j0 = 0; j0 < nl; j0 += kWave) {
    const int j = j0 + lane;
    const bool hit = j < nl && leader_d2(a.LT + j, a.cap, xs[wave], n, a.raw, a.w) <= a.t2;
    const unsigned long long m = __ballot(hit);
    if (m) {
      lab = j0 + __ffsll((long long)m) - 1;
      break;
    }
  }
  if (lane == 0) {
    if (lab == kPending && nl >= a.cap) {   // the cap is full: nothing left to found
      lab = kOverCap;
      a.state[2] = 1;
    }
    a.labels[f] = lab;
    if (lab == kPending) atomicOr(&a.pend[f >> 6], 1ull << (f & 63));
  }
}

// The chunk's unmatched frames, in order, against the leaders founded in
// this chunk (LDS, nlmax at most); new leaders are founded here.  The chunk's
// mask words come in one batch of loads, the unmatched frames' CVs in groups
// of up to gmax frames.  Per group, each thread first matches a frame
// against the chunk's leaders founded before the group (its first match
// overall if any, since later leaders only append); the walk then founds a
// leader at the first frame still unmatched, after which the rest of the
// group is matched in parallel against that leader before the walk
// resumes, so every frame meets the leaders founded before it in founding
// order.  If the cap is full or the LDS holds nlmax new leaders when
// another is due, the walk stops at that frame and the next chunk starts
// there.  The mask words read are cleared for the next round.
constexpr int kResolveWaves = 4;
constexpr int kXbBatch = 16;
__global__ __launch_bounds__(kResolveWaves * kWave) void sel_resolve_kernel(ClusterArgs a0,
                                                                            ClusterSlots sl,
                                                                            int nlmax, int gmax) {
  const ClusterArgs a = slot_args(a0, sl);
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int sh[6];   // new leaders so far, stop frame, over the cap, walk start,
                          // end of the matched run, the frame founding a leader
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int f0 = a.state[1];
  if (f0 >= a.B) return;
  const int n = a.n;
  const int f_end = min(a.B, f0 + a.chunk);
  const int n_start = a.state[0];
  const int w0 = f0 >> 6, w1 = (f_end - 1) >> 6;     // mask words of the chunk
  const int nw = w1 - w0 + 1;                         // <= kChunkMax / 64 + 1
  unsigned long long* pm = reinterpret_cast<unsigned long long*>(smem);   // [nw]
  int* grp = reinterpret_cast<int*>(pm + (kChunkMax / 64 + 2));          // [gmax]
  int* gm = grp + gmax;                                                  // [gmax]
  float* NL = reinterpret_cast<float*>(gm + gmax);                      // [nlmax][n]
  float* XB = NL + (size_t)nlmax * n;                                    // [gmax][n]
  for (int w = tid; w < nw; w += kResolveWaves * kWave) {
    unsigned long long m = a.pend[w0 + w];
    const int lo = (w0 + w) << 6;
    if (lo < f0) m &= ~0ull << (f0 - lo);                   // frames before the chunk
    if (lo + 64 > f_end) m &= (f_end - lo >= 64) ? ~0ull : ((1ull << (f_end - lo)) - 1ull);
    pm[w] = m;
    a.pend[w0 + w] = 0ull;
  }
  if (tid == 0) {
    sh[0] = 0;
    sh[1] = f_end;
    sh[2] = a.state[2];
  }
  __syncthreads();
  // every thread walks the mask words identically
  int wi = 0;
  unsigned long long cur = pm[0];
  for (;;) {
    const int n_new0 = sh[0];
    if (sh[1] != f_end) break;
    int g = 0;
    while (g < gmax) {
      while (cur == 0ull && wi + 1 < nw) cur = pm[++wi];
      if (cur == 0ull) break;
      const int b = __ffsll((long long)cur) - 1;
      cur &= cur - 1;
      if (tid == 0) grp[g] = ((w0 + wi) << 6) + b;
      ++g;
    }
    if (g == 0) break;
    __syncthreads();
    // the group's CVs into LDS, kXbBatch loads in flight per thread (element
    // e = q n + i stepped by the thread count without divisions; past the
    // end, q is clamped to the last frame and the value is not stored)
    {
      constexpr int kNT = kResolveWaves * kWave;
      const int tot = g * n, dq = kNT / n, di = kNT % n;
      for (int e0 = 0; e0 < tot; e0 += kXbBatch * kNT) {
        int q = (e0 + tid) / n, i = (e0 + tid) - q * n;
        float v[kXbBatch];
#pragma unroll
        for (int j = 0; j < kXbBatch; ++j) {
          v[j] = a.s[(size_t)grp[min(q, g - 1)] * n + i];
          q += dq;
          i += di;
          if (i >= n) {
            i -= n;
            ++q;
          }
        }
#pragma unroll
        for (int j = 0; j < kXbBatch; ++j) {
          const int e = e0 + tid + j * kNT;
          if (e < tot) XB[e] = v[j];
        }
      }
    }
    __syncthreads();
    // a thread per frame, the chunk's leaders in founding order up to the
    // first within the threshold (few leaders: lanes over them would idle)
    for (int q = tid; q < g; q += kResolveWaves * kWave) {
      int hitj = -1;
      for (int j = 0; j < n_new0; ++j)
        if (leader_d2(NL + (size_t)j * n, 1, XB + (size_t)q * n, n, a.raw, a.w) <= a.t2) {
          hitj = j;
          break;
        }
      gm[q] = hitj;
    }
    __syncthreads();
    // ordered walk: wave 0 finds the first frame at or after the walk's
    // start that no leader matches (a ballot per 64 frames); the frames
    // before it are labelled in parallel, and it founds a leader, after
    // which the rest of the group is matched in parallel against that
    // leader before the walk goes on.  With no room for another leader
    // (the cap is full, or this launch's LDS rows are) the walk stops at
    // that frame instead, and the next round starts there: its match kernel
    // then labels every remaining frame against all leaders, in parallel.
    int start = 0;
    for (;;) {
      if (wave == 0) {
        int first = g;
        for (int q0 = start; q0 < g; q0 += kWave) {
          const int q = q0 + lane;
          const unsigned long long m = __ballot(q < g && gm[q] < 0);
          if (m) {
            first = q0 + __ffsll((long long)m) - 1;
            break;
          }
        }
        if (lane == 0) {
          const int n_new = sh[0];
          int next = g, lead = -1;
          if (first < g) {
            if (n_start + n_new >= a.cap || n_new >= nlmax) {
              sh[1] = grp[first];
              next = first;
            } else {
              lead = first;
              next = first + 1;
              sh[0] = n_new + 1;
            }
          }
          sh[3] = next;
          sh[4] = first;
          sh[5] = lead;
        }
      }
      __syncthreads();
      const int mend = sh[4], lead = sh[5], jn = sh[0] - 1;
      for (int q = start + tid; q < mend; q += kResolveWaves * kWave)
        a.labels[grp[q]] = n_start + gm[q];
      if (lead >= 0) {
        const int out = n_start + jn;
        const float* xl = XB + (size_t)lead * n;
        for (int i = tid; i < n; i += kResolveWaves * kWave) {
          NL[(size_t)jn * n + i] = xl[i];
          a.LT[(size_t)i * a.cap + out] = xl[i];
        }
        if (tid == 0) {
          a.leader[out] = grp[lead];
          a.labels[grp[lead]] = out;
        }
      }
      start = sh[3];
      if (sh[1] != f_end || start >= g) break;
      // (the new leader's CVs are read from the group tile, where they are
      // already in place for every thread)
      const float* xl = XB + (size_t)lead * n;
      for (int q = start + tid; q < g; q += kResolveWaves * kWave)
        if (gm[q] < 0 && leader_d2(xl, 1, XB + (size_t)q * n, n, a.raw, a.w) <= a.t2) gm[q] = jn;
      __syncthreads();
    }
    __syncthreads();
  }
  if (tid == 0) {
    a.state[0] = n_start + sh[0];
    a.state[1] = sh[1];
    a.state[2] = sh[2];
  }
}

size_t resolve_lds(int n, int nlmax, int gmax) {
  return sizeof(unsigned long long) * (kChunkMax / 64 + 2) + 2 * sizeof(int) * (size_t)gmax +
         sizeof(float) * ((size_t)nlmax + gmax) * n;
}

// Device memory of one clustering call (one allocation): `slots` copies of
// the per-pass buffers (labels only with more than one slot; one slot
// writes the caller's).
struct ClusterWs {
  void* buf = nullptr;
  ~ClusterWs() {
    if (buf) (void)hipFree(buf);
  }
};

// One clustering pass at thresholds t[0..T) side by side (slot k at t[k]);
// synchronises the stream.  On return st_h[k * kStateInts + 0..2] = {leaders,
// next frame, over the cap} of slot k.
rid_status cluster_pass(ClusterArgs a, ClusterSlots sl, const float* t, int T, int nlmax,
                        int gmax, hipStream_t st, int* st_h) {
  for (int k = 0; k < T; ++k) sl.t2[k] = t[k] * t[k];
  const int words = (a.B + 63) / 64;
  hipLaunchKernelGGL(sel_init_kernel, dim3(std::min((words + 255) / 256 + 1, 1024), T), dim3(256),
                     0, st, a.state, a.pend, words);
  RID_HIP(hipGetLastError());
  const size_t lds = resolve_lds(a.n, nlmax, gmax);
  static size_t attr = 0;
  if (lds > 64 * 1024 && lds > attr) {
    RID_HIP(hipFuncSetAttribute((const void*)sel_resolve_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = lds;
  }
  // rounds: chunks growing from 64 frames until they cover B, then one full
  // chunk per possible stop: one per nlmax leaders founded (a launch's LDS
  // rows), one where the cap fills, and one more
  long long covered = 0;
  int c = 64;
  std::vector<int> chunks;
  while (covered < a.B) {
    chunks.push_back(c);
    covered += c;
    c = std::min(2 * c, kChunkMax);
  }
  const int stops = (a.cap + nlmax - 1) / nlmax;
  for (int i = 0; i <= stops + 1; ++i) chunks.push_back(kChunkMax);
  for (int ch : chunks) {
    a.chunk = ch;
    hipLaunchKernelGGL(sel_match_kernel, dim3((ch + kMatchWaves - 1) / kMatchWaves, T),
                       dim3(kMatchWaves * kWave), 0, st, a, sl);
    RID_HIP(hipGetLastError());
    hipLaunchKernelGGL(sel_resolve_kernel, dim3(1, T), dim3(kResolveWaves * kWave), (uint32_t)lds,
                       st, a, sl, nlmax, gmax);
    RID_HIP(hipGetLastError());
  }
  RID_HIP(hipMemcpyAsync(st_h, a.state, sizeof(int) * kStateInts * T, hipMemcpyDeviceToHost, st));
  RID_HIP(hipStreamSynchronize(st));
  return RID_OK;
}

}  // namespace

rid_status launch_cluster(const float* s, int B, int n, const uint8_t* raw, const float* w,
                          const float* eps,
                          float eps0, float threshold, int lower, int upper, int adapt, int cap,
                          int* labels, int* leaders, int leaders_out, int* n_leaders,
                          int* n_clusters, float* t_used, hipStream_t st) {
  const int words = (B + 63) / 64;
  // slots: one without adaptation; with it as many as fit in 256 MiB, at most kSlots
  const size_t per_slot = sizeof(float) * (size_t)n * cap + sizeof(int) * (size_t)cap +
                          sizeof(int) * (size_t)B + sizeof(unsigned long long) * words +
                          sizeof(int) * kStateInts;
  const int T = adapt ? (int)std::max<size_t>(1, std::min<size_t>(kSlots, (256u << 20) / per_slot))
                      : 1;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t b_lt = al(sizeof(float) * (size_t)n * cap * T), b_ld = al(sizeof(int) * (size_t)cap * T),
               b_st = al(sizeof(int) * kStateInts * T),
               b_pd = al(sizeof(unsigned long long) * (size_t)words * T),
               b_lb = T > 1 ? al(sizeof(int) * (size_t)B * T) : 0;
  ClusterWs ws;
  RID_HIP(hipMalloc(&ws.buf, b_lt + b_ld + b_st + b_pd + b_lb));
  unsigned char* wp = static_cast<unsigned char*>(ws.buf);
  float* ws_LT = reinterpret_cast<float*>(wp);
  int* ws_leader = reinterpret_cast<int*>(wp + b_lt);
  int* ws_state = reinterpret_cast<int*>(wp + b_lt + b_ld);
  unsigned long long* ws_pend = reinterpret_cast<unsigned long long*>(wp + b_lt + b_ld + b_st);
  int* ws_labels = T > 1 ? reinterpret_cast<int*>(wp + b_lt + b_ld + b_st + b_pd) : nullptr;
  ClusterArgs a{};
  a.s = s;
  a.raw = raw;
  a.w = w;
  a.eps = eps;
  a.eps0 = eps0;
  a.B = B;
  a.n = n;
  a.cap = cap;
  a.LT = ws_LT;
  a.leader = ws_leader;
  a.state = ws_state;
  a.labels = T > 1 ? ws_labels : labels;
  a.pend = ws_pend;
  ClusterSlots sl{};
  sl.sLT = (long long)n * cap;
  sl.sLabels = T > 1 ? B : 0;
  sl.sLeader = cap;
  sl.sPend = words;
  const int nlmax = kLdsRows / n;                       // >= 64 for n <= 256
  const int gmax = std::min(256, kLdsRows / n);
  // threshold adjustment (first iteration of the workflow), T thresholds
  // per pass (select_core.h)
  std::vector<int> st_h((size_t)kStateInts * T);
  auto pass = [&](const float* ts, int nts, int* counts) -> int {
    const rid_status r = cluster_pass(a, sl, ts, nts, nlmax, gmax, st, st_h.data());
    if (r != RID_OK) return r;
    for (int j = 0; j < nts; ++j) {
      const int* sj = st_h.data() + (size_t)j * kStateInts;
      counts[j] = sj[1] < B ? -1 : sj[0] + (sj[2] ? 1 : 0);
    }
    return 0;
  };
  selcore::Outcome res;
  const int rr = selcore::adjust_threshold(threshold, lower, upper, adapt != 0, T, pass, res);
  if (rr == selcore::kIncomplete)
    return fail(RID_EDEVICE, "clustering did not reach the last frame");
  if (rr != 0) return (rid_status)rr;
  const int k = res.slot, count = res.count;
  const float t = res.t;
  const int* sk = st_h.data() + (size_t)k * kStateInts;
  if (T > 1)
    RID_HIP(hipMemcpyAsync(labels, ws_labels + (size_t)k * B, sizeof(int) * (size_t)B,
                           hipMemcpyDeviceToDevice, st));
  const int nl = std::min(sk[0], leaders_out);
  if (leaders && nl > 0)
    RID_HIP(hipMemcpyAsync(leaders, ws_leader + (size_t)k * cap, sizeof(int) * (size_t)nl,
                           hipMemcpyDeviceToDevice, st));
  RID_HIP(hipStreamSynchronize(st));
  if (n_leaders) *n_leaders = nl;
  *n_clusters = count;
  if (t_used) *t_used = t;
  return RID_OK;
}

}  // namespace rid
