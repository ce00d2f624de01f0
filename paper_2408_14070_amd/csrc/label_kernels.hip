// Restrained-MD mean-force labels ("Labeling phase", restrained method).
//
// Under a stiff harmonic restraint kappa/2 (s - s0)^2 the mean force on a CV
// is the trajectory average of the spring force kappa * (s0 - s_t) (angle
// differences wrapped to (-pi, pi] for periodic CVs).  Labels whose block
// standard error exceeds std_threshold are dropped.
//
// One workgroup per configuration; thread p handles (CV i = p % n,
// block b = p / n), so consecutive lanes read consecutive CVs of one frame
// (coalesced rows of the [T][n] slab).  Every sum is FP64 in a fixed order:
// frames within a block, then blocks, then the tail frames.  HBM-bound: each
// trajectory value is read exactly once.
#include "rid_internal.h"

namespace rid {
namespace {

constexpr int kBlocks = 10;
constexpr int kThreads = 384;   // the 10 x 38 (block, CV) tasks of a 38-CV system in one pass

struct LabelArgs {
  const float* traj;   // [M][T][n]
  const float* s0;     // [M][n]
  int M, T, n;
  double thr;
  float kappa[256];
  uint32_t mask[8];    // bit i: CV i is periodic
  double* F;           // [M][n]
  double* se;          // [M][n] or null
  uint8_t* keep;       // [M] or null
};

__device__ inline double wrap(double d) {
  const double pi = 3.141592653589793;   // nearest double to pi
  if (d > pi) d -= 2.0 * pi;
  if (d <= -pi) d += 2.0 * pi;
  return d;
}

__global__ __launch_bounds__(kThreads) void label_kernel(LabelArgs a) {
  extern __shared__ double bs[];           // [kBlocks][n] block sums, then [n] tail
  __shared__ double red[kThreads / 64];
  const int m = blockIdx.x, n = a.n, T = a.T;
  const int bsz = T / kBlocks;
  const float* tr = a.traj + (size_t)m * T * n;
  for (int p = threadIdx.x; p < kBlocks * n; p += kThreads) {
    const int i = p % n, b = p / n;
    const double s0 = a.s0[(size_t)m * n + i];
    const double kap = a.kappa[i];
    const bool per = (a.mask[i >> 5] >> (i & 31)) & 1u;
    double acc = 0.0;
    const float* col = tr + (size_t)b * bsz * n + i;
#pragma unroll 8
    for (int t = 0; t < bsz; ++t) {
      double d = s0 - (double)col[(size_t)t * n];
      if (per) d = wrap(d);
      acc += kap * d;
    }
    bs[b * n + i] = acc;
  }
  // tail frames (T not a multiple of the block count) count in the mean only
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const double s0 = a.s0[(size_t)m * n + i];
    const double kap = a.kappa[i];
    const bool per = (a.mask[i >> 5] >> (i & 31)) & 1u;
    double acc = 0.0;
    for (int t = kBlocks * bsz; t < T; ++t) {
      double d = s0 - (double)tr[(size_t)t * n + i];
      if (per) d = wrap(d);
      acc += kap * d;
    }
    bs[kBlocks * n + i] = acc;
  }
  __syncthreads();
  double worst = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    double tot = 0.0, mbar = 0.0;
    for (int b = 0; b < kBlocks; ++b) {
      tot += bs[b * n + i];
      mbar += bs[b * n + i] / bsz;
    }
    tot += bs[kBlocks * n + i];
    mbar /= kBlocks;
    double var = 0.0;
    for (int b = 0; b < kBlocks; ++b) {
      const double dm = bs[b * n + i] / bsz - mbar;
      var += dm * dm;
    }
    var /= (kBlocks - 1);
    const double se = sqrt(var / kBlocks);
    a.F[(size_t)m * n + i] = tot / T;
    if (a.se) a.se[(size_t)m * n + i] = se;
    worst = se > worst ? se : worst;
  }
  // max over the workgroup: wave butterfly, then waves through LDS
  for (int off = 1; off < 64; off <<= 1) {
    const double o = __shfl_xor(worst, off);
    worst = o > worst ? o : worst;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = worst;
  __syncthreads();
  if (threadIdx.x == 0 && a.keep) {
    double w = red[0];
    for (int j = 1; j < kThreads / 64; ++j) w = red[j] > w ? red[j] : w;
    a.keep[m] = w <= a.thr ? 1 : 0;
  }
}

}  // namespace

rid_status launch_mf_label_impl(const float* traj, const float* s0,
                                const float* kappa, const uint8_t* mask, int M,
                                int T, int n, float thr, double* F, double* se,
                                uint8_t* keep, hipStream_t st) {
  LabelArgs a{};
  a.traj = traj;
  a.s0 = s0;
  a.M = M;
  a.T = T;
  a.n = n;
  a.thr = thr;
  for (int i = 0; i < n; ++i) {
    a.kappa[i] = kappa[i];
    if (!mask || mask[i]) a.mask[i >> 5] |= 1u << (i & 31);
  }
  a.F = F;
  a.se = se;
  a.keep = keep;
  const size_t lds = sizeof(double) * (kBlocks + 1) * (size_t)n;
  launch_timed(kProfLabel, label_kernel, dim3(M), dim3(kThreads), (uint32_t)lds, st, a);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

}  // namespace rid
