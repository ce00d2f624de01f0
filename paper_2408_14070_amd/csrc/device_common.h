// Device-side building blocks shared by the kernels of the bias path:
// torsion geometry and its gradient, ensemble statistics, the trust-level
// switch and the per-walker chain rule to atoms.
#pragma once

#include "rid_internal.h"

namespace rid {
namespace dev {

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

// Positions of the torsion atoms of one walker into sp[U][3]; threads
// [t0, t0 + nt) cooperate (a wave or a whole workgroup).
__device__ inline void gather_atoms(float* sp, const float* pw, const int* uniq,
                                    int U, int t0, int nt) {
  for (int j = t0; j < 3 * U; j += nt) {
    const int u = j / 3;
    sp[j] = pw[3 * uniq[u] + (j - 3 * u)];
  }
}

struct Torsion {
  V3 b1, b2, b3, n1, n2;
  float nn1, nn2, X, Y, lb2;
  bool deg;
};

// Torsion of quad q (local atom indices into sp):
// s = atan2(|b2| b1.n2, n1.n2), n1 = b1 x b2, n2 = b2 x b3.
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

// cos s, sin s straight from the geometry (degenerate: s = 0).
__device__ inline void torsion_cos_sin(const Torsion& t, float& cs, float& sn) {
  if (t.deg) {
    cs = 1.f;
    sn = 0.f;
    return;
  }
  const float r = sqrtf(t.X * t.X + t.Y * t.Y);
  cs = t.X / r;
  sn = t.Y / r;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m);
  return v;
}

// Ensemble statistics of walker w from g [K][B][n] (FP32) in FP64, one wave:
// gbar_i = (1/K) sum_k g_ki; with d_k = g_k - g_0 (exact in FP64),
// eps^2 = (1/K) sum_k sum_i (d_ki - dbar_i)^2.  Writes gbar into out_gbar[i];
// returns eps in every lane.
__device__ inline double ensemble_stats(const float* g, int K, int B, int n,
                                        int w, float* out_gbar, int lane) {
  double ss = 0.0;
  for (int i = lane; i < n; i += kWave) {
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

// Trust-level switch: decision in FP64 (eps against the thresholds), value in
// FP32: 1 below eps0, 0 at or above eps1, (1 + cos(pi t)) / 2 between.
__device__ inline float switch_sigma(double e, double eps0, double eps1) {
  if (e < eps0) return 1.f;
  if (e >= eps1) return 0.f;
  const float t = (float)((e - eps0) / (eps1 - eps0));
  return 0.5f * (1.f + cosf(3.14159265358979f * t));
}

struct SysView {
  int n_atoms, U, n;
  const int* uniq;
  const int* lq;
  const int* csr_ptr;
  const int* csr_ent;
  const int* atom_local;
};

// LDS floats one wave needs for scatter_walker.
__host__ __device__ inline int scatter_lds_floats(int U, int n) { return 6 * U + 13 * n; }

// Whole tail of the bias for walker w, executed by ONE wave (lane 0..63):
// deviation, switch, bias energy, torsion Jacobians and the fixed-order CSR
// assembly of atomic forces, written densely (zeros for atoms in no torsion).
// With g == nullptr the CV force is fcv[w] and sigma = 1 (no statistics).
// Outputs: forces at force + w * fstride, energy/eps/sigma at index w * ostride.
__device__ inline void scatter_walker(const SysView& sv, const float* pos, int w,
                                      int K, int B, const float* A, const float* g,
                                      const float* fcv, double eps0, double eps1,
                                      float* force, float* energy, float* eps_out,
                                      float* sigma_out, uint8_t* flags, float* sm,
                                      int lane, size_t fstride, size_t ostride) {
  const int U = sv.U, n = sv.n;
  float* sp = sm;                 // [U][3] positions
  float* fc = sp + 3 * U;         // [n] CV force
  float* ct = fc + n;             // [n][4][3] per-slot force contributions
  float* fl = ct + 12 * n;        // [U][3] assembled forces
  gather_atoms(sp, pos + (size_t)w * sv.n_atoms * 3, sv.uniq, U, lane, kWave);
  float sig = 1.f;
  if (g) {
    const double e = ensemble_stats(g, K, B, n, w, fc, lane);
    double abar = 0.0;
    for (int k = 0; k < K; ++k) abar += (double)A[(size_t)k * B + w];
    abar /= K;
    sig = switch_sigma(e, eps0, eps1);
    if (lane == 0) {
      if (energy) energy[w * ostride] = -sig * (float)abar;
      if (eps_out) eps_out[w * ostride] = (float)e;
      if (sigma_out) sigma_out[w * ostride] = sig;
    }
  } else {
    for (int i = lane; i < n; i += kWave) fc[i] = fcv[(size_t)w * n + i];
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  bool deg_any = false;
  for (int i = lane; i < n; i += kWave) {
    const Torsion t = torsion(sp, sv.lq + 4 * i);
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
    const float ca = -t.lb2 * i1;                           // slot a: ca n1
    const float cd = t.lb2 * i2;                            // slot d: cd n2
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
  if (flags && lane == 0) flags[w] = any ? 1 : 0;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (int u = lane; u < U; u += kWave) {
    float fx = 0.f, fy = 0.f, fz = 0.f;
    for (int e = sv.csr_ptr[u]; e < sv.csr_ptr[u + 1]; ++e) {
      const float* c = ct + 3 * sv.csr_ent[e];
      fx += c[0];
      fy += c[1];
      fz += c[2];
    }
    fl[3 * u] = fx;
    fl[3 * u + 1] = fy;
    fl[3 * u + 2] = fz;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  float* out = force + (size_t)w * fstride;
  for (int e = lane; e < 3 * sv.n_atoms; e += kWave) {
    const int atom = e / 3;
    const int loc = sv.atom_local[atom];
    out[e] = loc >= 0 ? fl[3 * loc + (e - 3 * atom)] : 0.f;
  }
}

}  // namespace dev
}  // namespace rid
