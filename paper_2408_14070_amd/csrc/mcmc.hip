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
#include "device_common.h"

namespace rid {
namespace {

using namespace dev;

constexpr float kPi = 3.14159265358979f;
constexpr float kTwoPi = 6.28318530717959f;
constexpr int kMcmcWaves = 4;

__device__ inline void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Uniform number `word` of walker w at step t.
__device__ inline float mcmc_uniform(int w, long long t, int word, unsigned long long seed) {
  uint32_t c[4] = {(uint32_t)w, (uint32_t)((unsigned long long)t & 0xFFFFFFFFull),
                   (uint32_t)((unsigned long long)t >> 32), (uint32_t)(word >> 2)};
  philox4x32_10(c, (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32));
  const uint32_t x = c[word & 3];
  return (float)(2u * (x >> 9) + 1u) * 5.9604644775390625e-8f;   // 2^-24
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
  unsigned* hist1;          // [n][nbins]
  unsigned* hist2;          // [nbins][nbins] or null
  unsigned long long* accepted;
};

__device__ inline double member_mean(const McmcArgs& a, int w) {
  double m = 0.0;
  for (int k = 0; k < a.K; ++k) m += (double)a.A[(size_t)k * a.W + w];
  return m / a.K;
}

// Proposal of step t for walker w (one wave, lanes over CVs) and its encoding.
__device__ inline void propose(const McmcArgs& a, int w, long long t, int lane) {
  for (int i = lane; i < a.n; i += kWave) {
    const float u = mcmc_uniform(w, t, i, a.seed);
    const float v = wrap_pi(a.s[(size_t)w * a.n + i] + a.step * (2.f * u - 1.f));
    a.sp[(size_t)w * a.n + i] = v;
    float sn, cs;
    sincosf(v, &sn, &cs);
    a.xp[(size_t)w * 2 * a.n + i] = cs;
    a.xp[(size_t)w * 2 * a.n + a.n + i] = sn;
  }
}

// Encoding of the (wrapped) current state, to evaluate its energy.
__global__ __launch_bounds__(kMcmcWaves * kWave) void mcmc_encode_kernel(McmcArgs a) {
  const int w = blockIdx.x * kMcmcWaves + threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (w >= a.W) return;
  for (int i = lane; i < a.n; i += kWave) {
    const float s0 = a.s[(size_t)w * a.n + i];   // any real angle
    const float v = wrap_pi(s0 - kTwoPi * floorf((s0 + kPi) / kTwoPi));
    a.s[(size_t)w * a.n + i] = v;
    float sn, cs;
    sincosf(v, &sn, &cs);
    a.xp[(size_t)w * 2 * a.n + i] = cs;
    a.xp[(size_t)w * 2 * a.n + a.n + i] = sn;
  }
}

// Energy of the current state, then the first proposal (step t).
__global__ __launch_bounds__(kMcmcWaves * kWave) void mcmc_start_kernel(McmcArgs a,
                                                                        long long t) {
  const int w = blockIdx.x * kMcmcWaves + threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (w >= a.W) return;
  if (lane == 0) a.acur[w] = member_mean(a, w);
  propose(a, w, t, lane);
}

// Metropolis decision of step t, the counts, and the proposal of step t+1.
__global__ __launch_bounds__(kMcmcWaves * kWave) void mcmc_step_kernel(McmcArgs a, long long t,
                                                                       int last) {
  const int w = blockIdx.x * kMcmcWaves + threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (w >= a.W) return;
  const double ap = member_mean(a, w);
  const float un = mcmc_uniform(w, t, a.n, a.seed);
  const bool acc = (double)un < exp(-(ap - a.acur[w]) / a.kT);
  if (acc) {
    for (int i = lane; i < a.n; i += kWave) a.s[(size_t)w * a.n + i] = a.sp[(size_t)w * a.n + i];
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (lane == 0) {
    if (acc) {
      a.acur[w] = ap;
      if (a.accepted) atomicAdd(a.accepted, 1ull);
    }
    if (a.hist2) {
      const int b0 = cv_bin(a.s[(size_t)w * a.n + a.proj0], a.nbins);
      const int b1 = cv_bin(a.s[(size_t)w * a.n + a.proj1], a.nbins);
      atomicAdd(&a.hist2[(size_t)b0 * a.nbins + b1], 1u);
    }
  }
  for (int i = lane; i < a.n; i += kWave)
    atomicAdd(&a.hist1[(size_t)i * a.nbins + cv_bin(a.s[(size_t)w * a.n + i], a.nbins)], 1u);
  if (!last) propose(a, w, t + 1, lane);
}

}  // namespace

rid_status launch_mcmc(rid_ensemble_impl& e, float* s, int W, long long n_steps, long long t0,
                       double kT, float step, unsigned long long seed, int proj0, int proj1,
                       int nbins, unsigned* hist1, unsigned* hist2,
                       unsigned long long* accepted, hipStream_t st) {
  const int n = e.n_cv, K = e.K;
  rid_status r;
  const size_t wn = (size_t)W * n;
  // workspace: proposal [W][n], its encoding [W][2n], Abar (FP64) [W]
  if ((r = e.ws_cons.ensure(sizeof(float) * 3 * wn + sizeof(double) * (size_t)W + 256)) !=
      RID_OK)
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
  a.sp = reinterpret_cast<float*>(base + sizeof(double) * (size_t)W);
  a.xp = a.sp + wn;
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
  a.hist1 = hist1;
  a.hist2 = hist2;
  a.accepted = accepted;
  const dim3 grid((W + kMcmcWaves - 1) / kMcmcWaves), block(kMcmcWaves * kWave);
  hipLaunchKernelGGL(mcmc_encode_kernel, grid, block, 0, st, a);
  RID_HIP(hipGetLastError());
  if ((r = launch_mlp(e, a.xp, W, e.ws_A.as<float>(), nullptr, st)) != RID_OK) return r;
  if (n_steps == 0) return RID_OK;
  hipLaunchKernelGGL(mcmc_start_kernel, grid, block, 0, st, a, t0);
  RID_HIP(hipGetLastError());
  for (long long t = t0; t < t0 + n_steps; ++t) {
    if ((r = launch_mlp(e, a.xp, W, e.ws_A.as<float>(), nullptr, st)) != RID_OK) return r;
    hipLaunchKernelGGL(mcmc_step_kernel, grid, block, 0, st, a, t,
                       (int)(t + 1 == t0 + n_steps));
    RID_HIP(hipGetLastError());
  }
  return RID_OK;
}

}  // namespace rid
