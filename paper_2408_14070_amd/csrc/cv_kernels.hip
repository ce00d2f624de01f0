// Torsion CVs, ensemble statistics, trust-level switch and the chain rule
// back to the atoms.
//
//  cv_eval_kernel       torsions of each walker ("CV selection": backbone
//                       phi/psi) and the periodic encoding [cos s | sin s]
//  embed_kernel         [cos s | sin s] from given CVs
//  reduce_kernel        ensemble mean force and model deviation (FP64)
//  bias_scatter_kernel  deviation + switch + bias energy, then
//                       F_a = sum_i f_i ds_i/dr_a written densely per walker
//
// One 64-lane wave per walker.  The walker's torsion atoms are gathered once
// into LDS (a sorted unique-atom list makes the gather walk the coordinate
// array forward); the torsion Jacobian is recomputed in the scatter rather
// than stored (48 bytes per CV would exceed the positions themselves).  The
// atom forces are assembled through a fixed-order CSR inverse map
// (atom -> (cv, slot)), so there are no atomics and results are bitwise
// reproducible.
#include "rid_internal.h"

namespace rid {
namespace {

constexpr float kDegTol = 1e-12f;  // |n1|^2, |n2|^2 threshold (nm^4)
constexpr int kWave = 64;

struct V3 {
  float x, y, z;
};
__device__ inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline V3 ld3(const float* p, int a) { return {p[3 * a], p[3 * a + 1], p[3 * a + 2]}; }

__device__ inline void gather_atoms(float* sp, const float* pw, const int* uniq,
                                    int U) {
  for (int j = threadIdx.x; j < 3 * U; j += blockDim.x) {
    const int u = j / 3;
    sp[j] = pw[3 * uniq[u] + (j - 3 * u)];
  }
}

struct Torsion {
  V3 b1, b2, b3, n1, n2;
  float nn1, nn2, X, Y, lb2;
  bool deg;
};

__device__ inline Torsion torsion(const float* sp, const int* q) {
  Torsion t;
  const V3 ra = ld3(sp, q[0]), rb = ld3(sp, q[1]), rc = ld3(sp, q[2]), rd = ld3(sp, q[3]);
  t.b1 = sub(rb, ra);
  t.b2 = sub(rc, rb);
  t.b3 = sub(rd, rc);
  t.n1 = cross(t.b1, t.b2);
  t.n2 = cross(t.b2, t.b3);
  t.nn1 = dot(t.n1, t.n1);
  t.nn2 = dot(t.n2, t.n2);
  t.lb2 = sqrtf(dot(t.b2, t.b2));
  t.X = dot(t.n1, t.n2);
  t.Y = t.lb2 * dot(t.b1, t.n2);
  t.deg = !(t.nn1 >= kDegTol && t.nn2 >= kDegTol);
  return t;
}

__global__ void cv_eval_kernel(const float* pos, int n_atoms, const int* uniq,
                               int U, const int* lq, int n, float* s, float* x) {
  extern __shared__ float sp[];
  const int w = blockIdx.x;
  gather_atoms(sp, pos + (size_t)w * n_atoms * 3, uniq, U);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const Torsion t = torsion(sp, lq + 4 * i);
    float sv = 0.f, cs = 1.f, sn = 0.f;
    if (!t.deg) {
      sv = atan2f(t.Y, t.X);
      const float r = sqrtf(t.X * t.X + t.Y * t.Y);
      cs = t.X / r;
      sn = t.Y / r;
    }
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

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m);
  return v;
}

// Ensemble statistics of one walker from g [K][B][n] (FP32) in FP64:
// gbar_i = (1/K) sum_k g_ki; with d_k = g_k - g_0 (exact in FP64),
// eps^2 = (1/K) sum_k sum_i (d_ki - dbar_i)^2.  Lane-strided over i.
// Writes gbar into out_gbar[i] (LDS or global) and returns eps (all lanes).
__device__ inline double ensemble_stats(const float* g, int K, int B, int n,
                                        int w, float* out_gbar) {
  double ss = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double g0 = g[(size_t)w * n + i];
    double dsum = 0.0, gsum = g0;
    for (int k = 1; k < K; ++k) {
      const double gk = g[((size_t)k * B + w) * n + i];
      dsum += gk - g0;
      gsum += gk;
    }
    const double dbar = dsum / K;
    double q = dbar * dbar;  // member 0: d_0 = 0
    for (int k = 1; k < K; ++k) {
      const double dk = (double)g[((size_t)k * B + w) * n + i] - g0 - dbar;
      q += dk * dk;
    }
    ss += q;
    out_gbar[i] = (float)(gsum / K);
  }
  ss = wave_sum(ss);
  return sqrt(ss / K);
}

__global__ void reduce_kernel(int K, int n, int B, const float* A,
                              const float* g, float* eps, float* gbar,
                              float* A_t, float* g_t) {
  extern __shared__ float gb[];
  const int w = blockIdx.x;
  const double e = ensemble_stats(g, K, B, n, w, gb);
  if (threadIdx.x == 0) eps[w] = (float)e;
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
  const float* pos;
  int n_atoms, U, n, K, B;
  const int* uniq;
  const int* lq;
  const int* csr_ptr;
  const int* csr_ent;
  const int* atom_local;
  const float* A;     // [K][B] or null
  const float* g;     // [K][B][n] or null (then fcv is the CV force)
  const float* fcv;   // [B][n]
  double eps0, eps1;
  float* force;
  float* energy;
  float* eps;
  float* sigma;
  uint8_t* flags;
};

__global__ void bias_scatter_kernel(ScatterArgs a) {
  extern __shared__ float sm[];
  const int U = a.U, n = a.n;
  float* sp = sm;                 // [U][3] positions
  float* fc = sp + 3 * U;         // [n] CV force
  float* ct = fc + n;             // [n][4][3] per-slot force contributions
  float* fl = ct + 12 * n;        // [U][3] assembled forces
  const int w = blockIdx.x;
  gather_atoms(sp, a.pos + (size_t)w * a.n_atoms * 3, a.uniq, U);

  float sig = 1.f;
  if (a.g) {
    const double e = ensemble_stats(a.g, a.K, a.B, n, w, fc);
    double abar = 0.0;
    for (int k = 0; k < a.K; ++k) abar += (double)a.A[(size_t)k * a.B + w];
    abar /= a.K;
    // trust-level switch: decision in FP64, value in FP32
    if (e < a.eps0) {
      sig = 1.f;
    } else if (e >= a.eps1) {
      sig = 0.f;
    } else {
      const float t = (float)((e - a.eps0) / (a.eps1 - a.eps0));
      sig = 0.5f * (1.f + cosf(3.14159265358979f * t));
    }
    if (threadIdx.x == 0) {
      if (a.energy) a.energy[w] = -sig * (float)abar;
      if (a.eps) a.eps[w] = (float)e;
      if (a.sigma) a.sigma[w] = sig;
    }
  } else {
    for (int i = threadIdx.x; i < n; i += blockDim.x) fc[i] = a.fcv[(size_t)w * n + i];
  }
  __syncthreads();

  bool deg_any = false;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const Torsion t = torsion(sp, a.lq + 4 * i);
    float* c = ct + 12 * i;
    if (t.deg) {
      deg_any = true;
      for (int j = 0; j < 12; ++j) c[j] = 0.f;
      continue;
    }
    const float f = sig * fc[i];
    const float i1 = 1.f / t.nn1, i2 = 1.f / t.nn2;
    const float p1 = dot(t.b1, t.b2) / t.lb2;
    const float p3 = dot(t.b3, t.b2) / t.lb2;
    const float ca = -t.lb2 * i1;              // slot a: ca n1
    const float cd = t.lb2 * i2;               // slot d: cd n2
    const float cb1 = (t.lb2 + p1) * i1, cb2 = p3 * i2;     // slot b
    const float cc2 = -(t.lb2 + p3) * i2, cc1 = -p1 * i1;   // slot c
    c[0] = f * ca * t.n1.x; c[1] = f * ca * t.n1.y; c[2] = f * ca * t.n1.z;
    c[3] = f * (cb1 * t.n1.x + cb2 * t.n2.x);
    c[4] = f * (cb1 * t.n1.y + cb2 * t.n2.y);
    c[5] = f * (cb1 * t.n1.z + cb2 * t.n2.z);
    c[6] = f * (cc2 * t.n2.x + cc1 * t.n1.x);
    c[7] = f * (cc2 * t.n2.y + cc1 * t.n1.y);
    c[8] = f * (cc2 * t.n2.z + cc1 * t.n1.z);
    c[9] = f * cd * t.n2.x; c[10] = f * cd * t.n2.y; c[11] = f * cd * t.n2.z;
  }
  const bool any = __any(deg_any);
  if (a.flags && threadIdx.x == 0) a.flags[w] = any ? 1 : 0;
  __syncthreads();
  for (int u = threadIdx.x; u < U; u += blockDim.x) {
    float fx = 0.f, fy = 0.f, fz = 0.f;
    for (int e = a.csr_ptr[u]; e < a.csr_ptr[u + 1]; ++e) {
      const float* c = ct + 3 * a.csr_ent[e];
      fx += c[0];
      fy += c[1];
      fz += c[2];
    }
    fl[3 * u] = fx;
    fl[3 * u + 1] = fy;
    fl[3 * u + 2] = fz;
  }
  __syncthreads();
  float* out = a.force + (size_t)w * a.n_atoms * 3;
  for (int e = threadIdx.x; e < 3 * a.n_atoms; e += blockDim.x) {
    const int atom = e / 3;
    const int loc = a.atom_local[atom];
    out[e] = loc >= 0 ? fl[3 * loc + (e - 3 * atom)] : 0.f;
  }
}

}  // namespace

rid_status launch_cv_eval(const rid_system_impl& s, const float* pos, int B,
                          float* d_s, float* d_x, hipStream_t st) {
  const size_t lds = sizeof(float) * 3 * s.n_uniq;
  ProfScope ps(kProfCv, st);
  hipLaunchKernelGGL(cv_eval_kernel, dim3(B), dim3(kWave), lds, st, pos,
                     s.n_atoms, s.d_uniq, s.n_uniq, s.d_lquads, s.n_cv, d_s, d_x);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

rid_status launch_embed(const float* s, int B, int n, float* x, hipStream_t st) {
  const size_t total = (size_t)B * n;
  const int grid = (int)std::min<size_t>((total + 255) / 256, 8192);
  ProfScope ps(kProfEmbed, st);
  hipLaunchKernelGGL(embed_kernel, dim3(grid), dim3(256), 0, st, s, B, n, x);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

rid_status launch_ensemble_reduce(int K, int n, int B, const float* A,
                                  const float* g, float* eps, float* gbar,
                                  float* A_t, float* g_t, hipStream_t st) {
  ProfScope ps(kProfReduce, st);
  hipLaunchKernelGGL(reduce_kernel, dim3(B), dim3(kWave), sizeof(float) * n, st,
                     K, n, B, A, g, eps, gbar, A_t, g_t);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

rid_status launch_bias_scatter(const rid_system_impl& s, int K, const float* pos,
                               int B, const float* A, const float* g,
                               const float* fcv, float eps0, float eps1,
                               float* force, float* energy, float* eps,
                               float* sigma, uint8_t* flags, hipStream_t st) {
  ScatterArgs a{};
  a.pos = pos;
  a.n_atoms = s.n_atoms;
  a.U = s.n_uniq;
  a.n = s.n_cv;
  a.K = K;
  a.B = B;
  a.uniq = s.d_uniq;
  a.lq = s.d_lquads;
  a.csr_ptr = s.d_csr_ptr;
  a.csr_ent = s.d_csr_ent;
  a.atom_local = s.d_atom_local;
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
  const size_t lds = sizeof(float) * (6 * (size_t)s.n_uniq + 13 * (size_t)s.n_cv);
  ProfScope ps(kProfScatter, st);
  hipLaunchKernelGGL(bias_scatter_kernel, dim3(B), dim3(kWave), lds, st, a);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

}  // namespace rid
