// Stand-alone kernels of the CV side of the path:
//
//  cv_eval_kernel       torsions of each walker ("CV selection": backbone
//                       phi/psi) and the periodic encoding [cos s | sin s]
//  embed_kernel         [cos s | sin s] from given CVs
//  reduce_kernel        ensemble mean force and model deviation (FP64)
//  scatter_kernel       F_a = sum_i f_i ds_i/dr_a for a given CV force, or the
//                       full deviation + switch + chain rule tail of the bias
//
// One 64-lane wave per walker.  The walker's torsion atoms are gathered once
// into LDS (a sorted unique-atom list makes the gather walk the coordinate
// array forward); the torsion Jacobian is recomputed rather than stored (48
// bytes per CV would exceed the positions themselves).  The atom forces are
// assembled through a fixed-order CSR inverse map (atom -> (cv, slot)), so
// there are no atomics and results are bitwise reproducible.  The fused bias
// kernel (mlp_kernels.hip) runs the same device code inside one launch.
#include "device_common.h"

namespace rid {
namespace {

using namespace dev;

__global__ void cv_eval_kernel(const float* pos, int n_atoms, const int* uniq,
                               int U, const int* lq, int n, float* s, float* x) {
  extern __shared__ float sp[];
  const int w = blockIdx.x;
  gather_atoms(sp, pos + (size_t)w * n_atoms * 3, uniq, U, threadIdx.x, blockDim.x);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const Torsion t = torsion(sp, lq + 4 * i);
    float cs, sn;
    torsion_cos_sin(t, cs, sn);
    const float sv = t.deg ? 0.f : atan2f(t.Y, t.X);
    if (s) s[(size_t)w * n + i] = sv;
    if (x) {
      x[(size_t)w * 2 * n + i] = cs;
      x[(size_t)w * 2 * n + n + i] = sn;
    }
  }
}

__global__ void embed_kernel(const float* s, int B, int n, float* x) {
  const size_t total = (size_t)B * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t w = e / n, i = e - w * n;
    float sn, cs;
    sincosf(s[e], &sn, &cs);
    x[w * 2 * n + i] = cs;
    x[w * 2 * n + n + i] = sn;
  }
}

__global__ void reduce_kernel(int K, int n, int B, const float* A,
                              const float* g, float* eps, float* gbar,
                              float* A_t, float* g_t) {
  extern __shared__ float gb[];
  const int w = blockIdx.x;
  const double e = ensemble_stats(g, K, B, n, w, gb, threadIdx.x);
  if (threadIdx.x == 0) eps[w] = (float)e;
  __syncthreads();
  if (gbar)
    for (int i = threadIdx.x; i < n; i += blockDim.x) gbar[(size_t)w * n + i] = gb[i];
  if (A_t)
    for (int k = threadIdx.x; k < K; k += blockDim.x)
      A_t[(size_t)w * K + k] = A[(size_t)k * B + w];
  if (g_t)
    for (int e2 = threadIdx.x; e2 < K * n; e2 += blockDim.x) {
      const int k = e2 / n, i = e2 - k * n;
      g_t[((size_t)w * K + k) * n + i] = g[((size_t)k * B + w) * n + i];
    }
}

struct ScatterArgs {
  SysView sv;
  const float* pos;
  int K, B;
  const float* A;
  const float* g;
  const float* fcv;
  double eps0, eps1;
  float* force;
  float* energy;
  float* eps;
  float* sigma;
  uint8_t* flags;
};

__global__ void scatter_kernel(ScatterArgs a) {
  extern __shared__ float sm[];
  scatter_walker(a.sv, a.pos, blockIdx.x, a.K, a.B, a.A, a.g, a.fcv, a.eps0, a.eps1,
                 a.force, a.energy, a.eps, a.sigma, a.flags, sm, threadIdx.x);
}

}  // namespace

rid_status launch_cv_eval(const rid_system_impl& s, const float* pos, int B,
                          float* d_s, float* d_x, hipStream_t st) {
  const size_t lds = sizeof(float) * 3 * s.n_uniq;
  launch_timed(kProfCv, cv_eval_kernel, dim3(B), dim3(kWave), (uint32_t)lds, st, pos,
               s.n_atoms, s.d_uniq, s.n_uniq, s.d_lquads, s.n_cv, d_s, d_x);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

rid_status launch_embed(const float* s, int B, int n, float* x, hipStream_t st) {
  const size_t total = (size_t)B * n;
  const int grid = (int)std::min<size_t>((total + 255) / 256, 8192);
  launch_timed(kProfEmbed, embed_kernel, dim3(grid), dim3(256), 0, st, s, B, n, x);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

rid_status launch_ensemble_reduce(int K, int n, int B, const float* A,
                                  const float* g, float* eps, float* gbar,
                                  float* A_t, float* g_t, hipStream_t st) {
  launch_timed(kProfReduce, reduce_kernel, dim3(B), dim3(kWave),
               (uint32_t)(sizeof(float) * n), st, K, n, B, A, g, eps, gbar, A_t, g_t);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

rid_status launch_bias_scatter(const rid_system_impl& s, int K, const float* pos,
                               int B, const float* A, const float* g,
                               const float* fcv, float eps0, float eps1,
                               float* force, float* energy, float* eps,
                               float* sigma, uint8_t* flags, hipStream_t st) {
  ScatterArgs a{};
  a.sv = SysView{s.n_atoms, s.n_uniq, s.n_cv, s.d_uniq, s.d_lquads, s.d_csr_ptr,
                 s.d_csr_ent, s.d_atom_local};
  a.pos = pos;
  a.K = K;
  a.B = B;
  a.A = A;
  a.g = g;
  a.fcv = fcv;
  a.eps0 = eps0;
  a.eps1 = eps1;
  a.force = force;
  a.energy = energy;
  a.eps = eps;
  a.sigma = sigma;
  a.flags = flags;
  const size_t lds = sizeof(float) * scatter_lds_floats(s.n_uniq, s.n_cv);
  launch_timed(kProfScatter, scatter_kernel, dim3(B), dim3(kWave), (uint32_t)lds, st, a);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

}  // namespace rid
