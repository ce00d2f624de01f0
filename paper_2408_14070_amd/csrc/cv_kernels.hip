// Stand-alone kernels of the CV side of the path:
//
//  cv_eval_kernel       torsions of each walker ("CV selection": backbone
//                       phi/psi) and the periodic encoding [cos s | sin s];
//                       distance rows (atom pairs) encoded raw as (s, 0)
//  embed_kernel         [cos s | sin s] from given CVs (raw ones as (s, 0))
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

// kCvWaves walkers per block (one wave each); the unique-atom list and the
// local quads are copied into LDS once per block.
constexpr int kCvWaves = 4;

__global__ __launch_bounds__(kCvWaves * kWave) void cv_eval_kernel(
    const float* pos, int n_atoms, const int* uniq, int U, const int* lq, int n, int B,
    float* s, float* x) {
  extern __shared__ float smc[];
  int* t_uniq = reinterpret_cast<int*>(smc);
  int* t_lq = t_uniq + U;
  // the system's tables are one array that starts uniq | lquads
  copy_ints(t_uniq, uniq, U + 4 * n, threadIdx.x, kCvWaves * kWave);
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int w = blockIdx.x * kCvWaves + wave;
  if (w >= B) return;
  float* sp = smc + U + 4 * n + wave * 3 * U;
  gather_atoms(sp, pos + (size_t)w * n_atoms * 3, t_uniq, U, lane, kWave);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (int i = lane; i < n; i += kWave) {
    float cs, sn, sv;
    if (t_lq[4 * i + 2] < 0) {
      // distance row: s = |r_b - r_a|, encoded raw as (s, 0)
      const Pair d = pair(sp, t_lq + 4 * i);
      sv = d.deg ? 0.f : d.r;
      cs = sv;
      sn = 0.f;
    } else {
      const Torsion t = torsion(sp, t_lq + 4 * i);
      torsion_cos_sin(t, cs, sn);
      sv = t.deg ? 0.f : atan2f(t.Y, t.X);
    }
    if (s) s[(size_t)w * n + i] = sv;
    if (x) {
      x[(size_t)w * 2 * n + i] = cs;
      x[(size_t)w * 2 * n + n + i] = sn;
    }
  }
}

__global__ void embed_kernel(const float* s, int B, int n, const uint8_t* raw, float* x) {
  const size_t total = (size_t)B * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t w = e / n, i = e - w * n;
    float sn, cs;
    if (raw && raw[i]) {
      cs = s[e];
      sn = 0.f;
    } else {
      sincosf(s[e], &sn, &cs);
    }
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
  size_t fstride, ostride;
};

// The system's small index tables (unique atoms, local quads, CSR inverse
// map and, when it fits, the atom -> local map) are copied into LDS once per
// block and shared by its kScatterWaves walkers (one wave each), so the
// per-walker chain has no dependent global index loads.  REG: each wave first
// issues the loads of its walker's member results (held in registers), the
// table copy runs while they are in flight, and the atom gather follows the
// barrier, so a walker waits on memory twice in all; otherwise the members'
// results are read inside the statistics (any K and n).
constexpr int kScatterWaves = 4;
constexpr int kLocalMapMaxAtoms = 4096;

__host__ __device__ inline int scatter_table_ints(int U, int n, int n_atoms) {
  return U + 4 * n + (U + 1) + 4 * n + (n_atoms <= kLocalMapMaxAtoms ? n_atoms : 0);
}

template <bool REG>
__global__ __launch_bounds__(kScatterWaves * kWave) void scatter_kernel(ScatterArgs a) {
  extern __shared__ float sm[];
  const SysView& g = a.sv;
  const int U = g.U, n = g.n;
  const bool loc_lds = g.n_atoms <= kLocalMapMaxAtoms;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int w = blockIdx.x * kScatterWaves + wave;
  const bool live = w < a.B;
  int* t = reinterpret_cast<int*>(sm);
  int* t_uniq = t;
  int* t_lq = t_uniq + U;
  int* t_ptr = t_lq + 4 * n;
  int* t_ent = t_ptr + U + 1;
  int* t_loc = t_ent + 4 * n;
  // the system's tables are one array in this order; the first
  // kGatherBatch entries per thread are loaded before the walker's own
  // loads and stored after them, so all of them are in flight together
  constexpr int nt = kScatterWaves * kWave;
  const int n_tab = scatter_table_ints(U, n, g.n_atoms);
  int ti[kGatherBatch], tv[kGatherBatch];
#pragma unroll
  for (int m = 0; m < kGatherBatch; ++m) {
    ti[m] = min((int)threadIdx.x + m * nt, n_tab - 1);
    tv[m] = g.uniq[ti[m]];
  }
  WalkerRegs r;
  if (REG && live) walker_prefetch(r, a.A, a.g, a.fcv, a.K, a.B, n, w, lane);
#pragma unroll
  for (int m = 0; m < kGatherBatch; ++m) t[ti[m]] = tv[m];
  if (n_tab > kGatherBatch * nt)
    copy_ints(t, g.uniq, n_tab, threadIdx.x + kGatherBatch * nt, nt);
  __syncthreads();
  const SysView lv{g.n_atoms, U, n, t_uniq, t_lq, t_ptr, t_ent,
                   loc_lds ? t_loc : g.atom_local};
  if (!live) return;
  float* ws = sm + scatter_table_ints(U, n, g.n_atoms) + wave * scatter_lds_floats(U, n);
  if (!REG) {
    scatter_walker(lv, a.pos, w, a.K, a.B, a.A, a.g, a.fcv, a.eps0, a.eps1, a.force,
                   a.energy, a.eps, a.sigma, a.flags, ws, lane, a.fstride, a.ostride);
    return;
  }
  float* sp = ws;                 // [U][3] positions
  float* fc = sp + 3 * U;         // [n] CV force
  float* ct = fc + n;             // [n][4][3] per-slot force contributions
  float* fl = ct + 12 * n;        // [U][3] assembled forces
  // the atom gather: when it is one batch (3U <= kGatherBatch * 64) its
  // loads stay in flight through the statistics below
  const float* pw = a.pos + (size_t)w * g.n_atoms * 3;
  const int n3 = 3 * U;
  const bool one = n3 <= kGatherBatch * kWave;
  int jc[kGatherBatch];
  float pv[kGatherBatch];
  if (one) {
#pragma unroll
    for (int m = 0; m < kGatherBatch; ++m) {
      jc[m] = min(lane + m * kWave, n3 - 1);
      const int u = jc[m] / 3;
      pv[m] = pw[3 * t_uniq[u] + (jc[m] - 3 * u)];
    }
  } else {
    gather_atoms(sp, pw, t_uniq, U, lane, kWave);
  }
  float sig = 1.f;
  if (a.g) {
    double abar;
    const double e = scatter_stats_reg(r, a.K, n, fc, abar, lane);
    sig = switch_outputs(e, abar, a.eps0, a.eps1, w, a.energy, a.eps, a.sigma, lane,
                         a.ostride);
  } else {
#pragma unroll
    for (int p = 0; p < kRegPasses; ++p)
      if (lane + p * kWave < n) fc[lane + p * kWave] = r.g[p][0];
  }
  if (one)
#pragma unroll
    for (int m = 0; m < kGatherBatch; ++m) sp[jc[m]] = pv[m];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  scatter_forces(lv, sp, fc, ct, fl, sig, w, a.force, a.flags, lane, a.fstride);
}

}  // namespace

rid_status launch_cv_eval(const rid_system_impl& s, const float* pos, int B,
                          float* d_s, float* d_x, hipStream_t st) {
  const size_t lds = sizeof(float) * (s.n_uniq + 4 * s.n_cv + kCvWaves * 3 * (size_t)s.n_uniq);
  if (lds > 64 * 1024) return fail(RID_EUNSUPPORTED, "too many torsion atoms for cv_eval");
  launch_timed(kProfCv, cv_eval_kernel, dim3((B + kCvWaves - 1) / kCvWaves),
               dim3(kCvWaves * kWave), (uint32_t)lds, st, pos, s.n_atoms, s.d_uniq, s.n_uniq,
               s.d_lquads, s.n_cv, B, d_s, d_x);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

rid_status launch_embed(const float* s, int B, int n, const uint8_t* raw, float* x,
                        hipStream_t st) {
  const size_t total = (size_t)B * n;
  const int grid = (int)std::min<size_t>((total + 255) / 256, 8192);
  launch_timed(kProfEmbed, embed_kernel, dim3(grid), dim3(256), 0, st, s, B, n, raw, x);
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
                               float* sigma, uint8_t* flags, hipStream_t st,
                               int rec_stride) {
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
  a.fstride = rec_stride > 0 ? (size_t)rec_stride : (size_t)s.n_atoms * 3;
  a.ostride = rec_stride > 0 ? (size_t)rec_stride : 1;
  const size_t lds =
      sizeof(float) * (scatter_table_ints(s.n_uniq, s.n_cv, s.n_atoms) +
                       (size_t)kScatterWaves * scatter_lds_floats(s.n_uniq, s.n_cv));
  if (lds > 160 * 1024) return fail(RID_EUNSUPPORTED, "too many torsion atoms for the scatter");
  static size_t attr[2] = {0, 0};
  // members' results in registers when they fit (K <= 8, n <= 128)
  const bool reg = (g == nullptr || K <= kRegMembers) && s.n_cv <= kRegPasses * kWave;
  auto kern = reg ? scatter_kernel<true> : scatter_kernel<false>;
  if (lds > 64 * 1024 && lds > attr[reg]) {
    RID_HIP(hipFuncSetAttribute((const void*)kern,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr[reg] = lds;
  }
  launch_timed(kProfScatter, kern, dim3((B + kScatterWaves - 1) / kScatterWaves),
               dim3(kScatterWaves * kWave), (uint32_t)lds, st, a);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

}  // namespace rid
