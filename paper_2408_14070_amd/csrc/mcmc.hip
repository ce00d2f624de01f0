// MCMC on the ensemble's learned free energy in CV space ("Dimension
// reduction phase": many walkers, a temperature, histograms of every CV and
// of a projected pair; the projected PMF is -kT ln p).
//
// Per step t and walker w: proposal s' = wrap(s + step (2u - 1)) on every
// CV, the ensemble-mean free energy at s' from the MLP kernel, acceptance
// when u_n < exp(-(Abar(s') - Abar(s))/kT) (decided in FP64), then the
// walker's current state is counted.  The uniforms come from Philox4x32-10
// (Salmon et al., SC 2011): counter (w, t mod 2^32, t div 2^32, block j),
// key = the seed's two 32-bit halves; word 4j+i of the walker's blocks is
// its i-th uniform of the step, u = (2 (x >> 9) + 1) 2^-24 (exact in FP32).
// Words 0..n-1 drive the proposal, word n the acceptance.  Histogram counts
// are integer atomics, so the result does not depend on their order.
//
// Raw CVs (angular mask 0: distances) walk in their box [lo_i, hi_i] (the
// dimension-reduction settings' lower and upper CV bounds): the proposal
// moves them by step (hi_i - lo_i) / 2pi (2u - 1) without wrapping, a move
// that takes any raw CV outside its box is rejected (flag computed with the
// proposal), they enter the network as (s, 0), and they are binned over
// their box.
//
// One wave per walker, lanes over CVs.  A step kernel issues every load it
// needs (member energies, the current state and the proposal, the walker's
// acceptance count) before it waits, keeps the updated state in registers
// for the counts and the next proposal, and counts acceptances per walker:
// one atomic per workgroup adds them to the caller's total at the end.  The
// per-CV counts go to one of several private copies of the histograms
// (walker w to copy w mod copies), so walkers in the same bin rarely hit the
// same counter; the copies are added to the caller's histograms at the end
// of the call.
#include "device_common.h"

namespace rid {
namespace {

using namespace dev;

constexpr float kPi = 3.14159265358979f;
constexpr float kTwoPi = 6.28318530717959f;
constexpr int kMcmcWaves = 4;

// Uniform number `word` of walker w at step t.
__device__ inline float mcmc_uniform(int w, long long t, int word, unsigned long long seed) {
  uint32_t c[4] = {(uint32_t)w, (uint32_t)((unsigned long long)t & 0xFFFFFFFFull),
                   (uint32_t)((unsigned long long)t >> 32), (uint32_t)(word >> 2)};
  philox4x32_10(c, (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32));
  const uint32_t x = c[word & 3];
  return philox_uniform(x);
}

__device__ inline float wrap_pi(float s) {
  if (s >= kPi) s -= kTwoPi;
  if (s < -kPi) s += kTwoPi;
  return s;
}

__device__ inline int cv_bin(float s, int nbins) {
  const int b = (int)floorf((s + kPi) * ((float)nbins / kTwoPi));
  return min(max(b, 0), nbins - 1);
}

struct McmcArgs {
  float* s;                 // [W][n] current state (in/out)
  float* sp;                // [W][n] proposal
  float* xp;                // [W][2n] its encoding, the MLP input
  double* acur;             // [W] Abar of the current state
  const float* A;           // [K][W] member free energies from the MLP
  int W, n, K;
  double kT;
  float step;
  unsigned long long seed;
  int proj0, proj1, nbins;
  unsigned* hist1;          // [copies][n][nbins] private copies of the counts
  int copies;
  unsigned* hist2;          // [nbins][nbins] or null
  unsigned long long* accepted;
  unsigned long long* acc_count;   // [W] acceptances of this call, per walker
  const uint8_t* raw;       // [n] 1 = raw CV (null: every CV angular)
  const float* lo;          // [n] box of the raw CVs
  const float* hi;          // [n]
  int* inbox;               // [W] the pending proposal keeps every raw CV in its box
};

// Bin of CV i's value v: the circle for angles, the box for raw CVs.
__device__ inline int bin_of(const McmcArgs& a, int i, float v) {
  if (a.raw && a.raw[i]) {
    const float l = a.lo[i], h = a.hi[i];
    const int b = (int)floorf((v - l) * ((float)a.nbins / (h - l)));
    return min(max(b, 0), a.nbins - 1);
  }
  return cv_bin(v, a.nbins);
}

// CV i moved from v by the uniform u: wrapped on the circle, or scaled to its
// box and unwrapped for a raw CV (in_box says whether it stays inside).
__device__ inline float step_cv(const McmcArgs& a, int i, float v, float u, bool& in_box) {
  if (a.raw && a.raw[i]) {
    const float l = a.lo[i], h = a.hi[i];
    const float vp = v + a.step * ((h - l) * (1.f / kTwoPi)) * (2.f * u - 1.f);
    in_box = vp >= l && vp <= h;
    return vp;
  }
  in_box = true;
  return wrap_pi(v + a.step * (2.f * u - 1.f));
}

// (x_i, x_{n+i}): (cos v, sin v), or (v, 0) for a raw CV
__device__ inline void encode_cv(const McmcArgs& a, int i, float v, float* x) {
  if (a.raw && a.raw[i]) {
    x[i] = v;
    x[a.n + i] = 0.f;
    return;
  }
  float sn, cs;
  sincosf(v, &sn, &cs);
  x[i] = cs;
  x[a.n + i] = sn;
}

// Abar of walker w: lane k holds member k (K <= 64); the sum is in FP64, so
// its order does not matter at FP32 inputs.  Every lane of the wave calls it.
__device__ inline double member_mean(const McmcArgs& a, int w, int lane) {
  const float ak = lane < a.K ? a.A[(size_t)lane * a.W + w] : 0.f;
  return wave_sum((double)ak) / a.K;
}

// Proposal of step t for walker w (one wave, lanes over CVs), its encoding
// and its box flag.
__device__ inline void propose(const McmcArgs& a, int w, long long t, int lane) {
  bool ok = true;
  for (int i = lane; i < a.n; i += kWave) {
    const float u = mcmc_uniform(w, t, i, a.seed);
    bool in_box;
    const float v = step_cv(a, i, a.s[(size_t)w * a.n + i], u, in_box);
    ok = ok && in_box;
    a.sp[(size_t)w * a.n + i] = v;
    encode_cv(a, i, v, a.xp + (size_t)w * 2 * a.n);
  }
  ok = __all(ok);
  if (lane == 0) a.inbox[w] = ok ? 1 : 0;
}

// Encoding of the (wrapped) current state, to evaluate its energy.
__global__ __launch_bounds__(kMcmcWaves * kWave) void mcmc_encode_kernel(McmcArgs a) {
  const int w = blockIdx.x * kMcmcWaves + threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (w >= a.W) return;
  if (lane == 0) a.acc_count[w] = 0ull;
  for (int i = lane; i < a.n; i += kWave) {
    const float s0 = a.s[(size_t)w * a.n + i];   // any real angle (raw CVs as given)
    const float v = (a.raw && a.raw[i]) ? s0
                                         : wrap_pi(s0 - kTwoPi * floorf((s0 + kPi) / kTwoPi));
    a.s[(size_t)w * a.n + i] = v;
    encode_cv(a, i, v, a.xp + (size_t)w * 2 * a.n);
  }
}

// Energy of the current state, then the first proposal (step t).
__global__ __launch_bounds__(kMcmcWaves * kWave) void mcmc_start_kernel(McmcArgs a,
                                                                        long long t) {
  const int w = blockIdx.x * kMcmcWaves + threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (w >= a.W) return;
  const double m = member_mean(a, w, lane);
  if (lane == 0) a.acur[w] = m;
  propose(a, w, t, lane);
}

// Metropolis decision of step t, the counts, and the proposal of step t+1.
__global__ __launch_bounds__(kMcmcWaves * kWave) void mcmc_step_kernel(McmcArgs a, long long t,
                                                                       int last) {
  const int w = blockIdx.x * kMcmcWaves + threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (w >= a.W) return;
  const int n = a.n;
  const size_t row = (size_t)w * n;
  unsigned* h1 = a.hist1 + (size_t)(w % a.copies) * n * a.nbins;
  // every load first: member energies (lane k), the walker's Abar and count,
  // the first chunk of the state and of the proposal
  const float ak = lane < a.K ? a.A[(size_t)lane * a.W + w] : 0.f;
  const double acur = a.acur[w];
  const unsigned long long cnt = a.acc_count[w];
  const bool inbox = a.raw ? a.inbox[w] != 0 : true;
  const int i0c = min(lane, n - 1);
  float sc = a.s[row + i0c], spc = a.sp[row + i0c];
  // the random numbers do not depend on the loads
  const float un = mcmc_uniform(w, t, n, a.seed);
  float unext = last ? 0.f : mcmc_uniform(w, t + 1, i0c, a.seed);
  const double ap = wave_sum((double)ak) / a.K;
  const bool acc = inbox && (double)un < exp(-(ap - acur) / a.kT);
  float p0 = 0.f, p1 = 0.f;
  bool ok = true;                       // the next proposal stays in the box
  for (int i0 = 0; i0 < n; i0 += kWave) {
    const int i = i0 + lane;
    if (i0 > 0) {
      const int ic = min(i, n - 1);
      sc = a.s[row + ic];
      spc = a.sp[row + ic];
      if (!last) unext = mcmc_uniform(w, t + 1, ic, a.seed);
    }
    const float v = acc ? spc : sc;
    if (a.hist2) {
      if (a.proj0 >= i0 && a.proj0 < i0 + kWave) p0 = __shfl(v, a.proj0 - i0);
      if (a.proj1 >= i0 && a.proj1 < i0 + kWave) p1 = __shfl(v, a.proj1 - i0);
    }
    if (i < n) {
      if (acc) a.s[row + i] = v;
      atomicAdd(&h1[(size_t)i * a.nbins + bin_of(a, i, v)], 1u);
      if (!last) {
        bool in_box;
        const float vp = step_cv(a, i, v, unext, in_box);
        ok = ok && in_box;
        a.sp[row + i] = vp;
        encode_cv(a, i, vp, a.xp + 2 * row);
      }
    }
  }
  if (a.raw && !last) ok = __all(ok);
  if (lane == 0) {
    if (acc) {
      a.acur[w] = ap;
      a.acc_count[w] = cnt + 1ull;
    }
    if (a.raw && !last) a.inbox[w] = ok ? 1 : 0;
    if (a.hist2)
      atomicAdd(&a.hist2[(size_t)bin_of(a, a.proj0, p0) * a.nbins + bin_of(a, a.proj1, p1)],
                1u);
  }
}

// Zeroes the private histogram copies (a kernel: the call may be captured in
// a graph).
__global__ void mcmc_hist_zero_kernel(unsigned* h, size_t count) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count;
       e += (size_t)gridDim.x * blockDim.x)
    h[e] = 0u;
}

// Adds the private copies to the caller's per-CV histograms.
__global__ void mcmc_hist_sum_kernel(const unsigned* h, int copies, size_t per_copy,
                                     unsigned* out) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < per_copy;
       e += (size_t)gridDim.x * blockDim.x) {
    unsigned v = 0u;
    for (int c = 0; c < copies; ++c) v += h[c * per_copy + e];
    out[e] += v;
  }
}

// Adds the call's per-walker acceptance counts to the caller's total.
__global__ __launch_bounds__(256) void mcmc_count_kernel(const unsigned long long* cnt, int W,
                                                         unsigned long long* total) {
  __shared__ unsigned long long part[256 / kWave];
  unsigned long long v = 0;
  for (int w = blockIdx.x * 256 + threadIdx.x; w < W; w += gridDim.x * 256) v += cnt[w];
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o);
  if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int q = 0; q < 256 / kWave; ++q) s += part[q];
    if (s) atomicAdd(total, s);
  }
}

}  // namespace

rid_status launch_mcmc(rid_ensemble_impl& e, float* s, int W, long long n_steps, long long t0,
                       double kT, float step, unsigned long long seed, int proj0, int proj1,
                       int nbins, unsigned* hist1, unsigned* hist2,
                       unsigned long long* accepted, hipStream_t st) {
  const int n = e.n_cv, K = e.K;
  rid_status r;
  const size_t wn = (size_t)W * n;
  // private histogram copies: up to 32, within 16 MiB
  const size_t per_copy = (size_t)n * nbins;
  const int copies = (int)std::max<size_t>(
      1, std::min<size_t>(32, ((size_t)16 << 20) / (sizeof(unsigned) * per_copy)));
  // workspace: Abar (FP64) [W], acceptance counts [W], proposal [W][n], its
  // encoding [W][2n], the proposals' box flags [W], the histogram copies
  const size_t off_h = (2 * sizeof(double) * (size_t)W + sizeof(float) * 3 * wn +
                        sizeof(int) * (size_t)W + 255) / 256 * 256;
  if ((r = e.ws_cons.ensure(off_h + sizeof(unsigned) * per_copy * copies + 256)) != RID_OK)
    return r;
  if ((r = e.ws_A.ensure(sizeof(float) * K * (size_t)W)) != RID_OK) return r;
  if (e.frag_dirty) {
    if ((r = pack_ensemble_weights(e, st)) != RID_OK) return r;
    e.frag_dirty = false;
  }
  unsigned char* base = e.ws_cons.as<unsigned char>();
  McmcArgs a{};
  a.s = s;
  a.acur = reinterpret_cast<double*>(base);
  a.acc_count = reinterpret_cast<unsigned long long*>(base + sizeof(double) * (size_t)W);
  a.sp = reinterpret_cast<float*>(base + 2 * sizeof(double) * (size_t)W);
  a.xp = a.sp + wn;
  a.inbox = reinterpret_cast<int*>(a.xp + 2 * wn);
  if (!e.raw.empty()) {
    a.raw = e.d_raw;
    a.lo = e.d_bounds;
    a.hi = e.d_bounds + n;
  }
  a.A = e.ws_A.as<float>();
  a.W = W;
  a.n = n;
  a.K = K;
  a.kT = kT;
  a.step = step;
  a.seed = seed;
  a.proj0 = proj0;
  a.proj1 = proj1;
  a.nbins = nbins;
  a.hist1 = reinterpret_cast<unsigned*>(base + off_h);
  a.copies = copies;
  a.hist2 = hist2;
  a.accepted = accepted;
  const dim3 grid((W + kMcmcWaves - 1) / kMcmcWaves), block(kMcmcWaves * kWave);
  hipLaunchKernelGGL(mcmc_encode_kernel, grid, block, 0, st, a);
  RID_HIP(hipGetLastError());
  if ((r = launch_mlp(e, a.xp, W, e.ws_A.as<float>(), nullptr, st)) != RID_OK) return r;
  if (n_steps == 0) return RID_OK;
  hipLaunchKernelGGL(mcmc_hist_zero_kernel,
                     dim3((unsigned)std::min<size_t>((per_copy * copies + 255) / 256, 1024)),
                     dim3(256), 0, st, a.hist1, per_copy * copies);
  RID_HIP(hipGetLastError());
  hipLaunchKernelGGL(mcmc_start_kernel, grid, block, 0, st, a, t0);
  RID_HIP(hipGetLastError());
  for (long long t = t0; t < t0 + n_steps; ++t) {
    if ((r = launch_mlp(e, a.xp, W, e.ws_A.as<float>(), nullptr, st)) != RID_OK) return r;
    hipLaunchKernelGGL(mcmc_step_kernel, grid, block, 0, st, a, t,
                       (int)(t + 1 == t0 + n_steps));
    RID_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(mcmc_hist_sum_kernel,
                     dim3((unsigned)std::min<size_t>((per_copy + 255) / 256, 1024)), dim3(256), 0,
                     st, a.hist1, copies, per_copy, hist1);
  RID_HIP(hipGetLastError());
  if (accepted) {
    hipLaunchKernelGGL(mcmc_count_kernel, dim3(std::min((W + 255) / 256, 1024)), dim3(256), 0,
                       st, a.acc_count, W, accepted);
    RID_HIP(hipGetLastError());
  }
  return RID_OK;
}

}  // namespace rid
