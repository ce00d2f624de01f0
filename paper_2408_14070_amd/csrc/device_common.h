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
// [t0, t0 + nt) cooperate (a wave or a whole workgroup).  Coordinates go in
// chunks of kGatherBatch per thread: a chunk's index loads are all issued
// before its coordinate loads, and those before the first store, so a chunk
// costs two memory round trips rather than two per coordinate.
constexpr int kGatherBatch = 4;
__device__ inline void gather_atoms(float* sp, const float* pw, const int* uniq,
                                    int U, int t0, int nt) {
  const int n3 = 3 * U;
  for (int j0 = t0; j0 < n3; j0 += kGatherBatch * nt) {
    // slots past the end are clamped to the last coordinate: they load and
    // store that coordinate's own value again, so nothing sits behind a
    // branch (the compiler would sink a guarded load next to its store)
    int jc[kGatherBatch], a[kGatherBatch];
#pragma unroll
    for (int m = 0; m < kGatherBatch; ++m) {
      jc[m] = min(j0 + m * nt, n3 - 1);
      const int u = jc[m] / 3;
      a[m] = 3 * uniq[u] + (jc[m] - 3 * u);
    }
    float v[kGatherBatch];
#pragma unroll
    for (int m = 0; m < kGatherBatch; ++m) v[m] = pw[a[m]];
#pragma unroll
    for (int m = 0; m < kGatherBatch; ++m) sp[jc[m]] = v[m];
  }
}

// count ints from global memory into LDS, threads [t0, t0 + nt), with
// kGatherBatch loads per thread in flight (slots past the end are clamped to
// the last element and write its own value again).
__device__ inline void copy_ints(int* dst, const int* src, int count, int t0, int nt) {
  for (int i0 = t0; i0 < count; i0 += kGatherBatch * nt) {
    int ic[kGatherBatch], v[kGatherBatch];
#pragma unroll
    for (int m = 0; m < kGatherBatch; ++m) {
      ic[m] = min(i0 + m * nt, count - 1);
      v[m] = src[ic[m]];
    }
#pragma unroll
    for (int m = 0; m < kGatherBatch; ++m) dst[ic[m]] = v[m];
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

// Distance CV of pair row q (q[0], q[1]; q[2] = q[3] = -1 mark the row):
// s = |r_b - r_a|; degenerate (direction undefined) below sqrt(kDegTol).
struct Pair {
  V3 d;        // r_a - r_b
  float r;
  bool deg;
};

__device__ inline Pair pair(const float* sp, const int* q) {
  Pair p;
  p.d = sub(ld3(sp, q[0]), ld3(sp, q[1]));
  const float r2 = dot(p.d, p.d);
  p.deg = !(r2 >= kDegTol);
  p.r = sqrtf(r2);
  return p;
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

// One DPP lane move of an FP64 value (both halves), all lanes active.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes (all active), returned in every lane: DPP moves
// within each row of 16 lanes (quad swaps, then the half-row and row
// mirrors pair the partial sums), then the four row sums in row order.
__device__ inline double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
  v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
  v += dpp_f64<0x141>(v);   // row_half_mirror: quad 0 <-> quad 1 of 8 lanes
  v += dpp_f64<0x140>(v);   // row_mirror: half 0 <-> half 1 of 16 lanes
  double r = readlane_f64(v, 0) + readlane_f64(v, 16);
  r += readlane_f64(v, 32);
  r += readlane_f64(v, 48);
  return r;
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

// Chain rule of walker w with its CV force fc[n] (in LDS) scaled by sig and
// its torsion atoms in sp[U][3]: torsion Jacobians, the fixed-order CSR
// assembly of atomic forces, written densely (zeros for atoms in no torsion)
// at force + w * fstride, and the walker's degenerate-torsion flag.  ct and
// fl are the wave's LDS scratch ([n][4][3] and [U][3]).  One wave.
__device__ inline void scatter_forces(const SysView& sv, const float* sp, const float* fc,
                                      float* ct, float* fl, float sig, int w,
                                      float* force, uint8_t* flags, int lane,
                                      size_t fstride) {
  const int U = sv.U, n = sv.n;
  bool deg_any = false;
  for (int i = lane; i < n; i += kWave) {
    float* c = ct + 12 * i;
    if (sv.lq[4 * i + 2] < 0) {
      // distance row: ds/dr_a = (r_a - r_b)/s, ds/dr_b the negative (its
      // CSR entries name slots 0 and 1 only)
      const Pair d = pair(sp, sv.lq + 4 * i);
      if (d.deg) {
        deg_any = true;
        for (int j = 0; j < 6; ++j) c[j] = 0.f;
        continue;
      }
      const float f = sig * fc[i] / d.r;
      c[0] = f * d.d.x; c[1] = f * d.d.y; c[2] = f * d.d.z;
      c[3] = -c[0]; c[4] = -c[1]; c[5] = -c[2];
      continue;
    }
    const Torsion t = torsion(sp, sv.lq + 4 * i);
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
  // every unique atom has at least one entry; the first kCsrBatch entries
  // of an atom are read in one batch (indices clamped to its last entry,
  // contributions past the end are zero), any further ones in order
  constexpr int kCsrBatch = 4;
  for (int u = lane; u < U; u += kWave) {
    const int e0 = sv.csr_ptr[u], e1 = sv.csr_ptr[u + 1];
    int ent[kCsrBatch];
#pragma unroll
    for (int j = 0; j < kCsrBatch; ++j) ent[j] = sv.csr_ent[min(e0 + j, e1 - 1)];
    float fx = 0.f, fy = 0.f, fz = 0.f;
#pragma unroll
    for (int j = 0; j < kCsrBatch; ++j) {
      const float* c = ct + 3 * ent[j];
      const bool on = e0 + j < e1;
      fx += on ? c[0] : 0.f;
      fy += on ? c[1] : 0.f;
      fz += on ? c[2] : 0.f;
    }
    for (int e = e0 + kCsrBatch; e < e1; ++e) {
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
  // a lane writes whole atoms, kGatherBatch of them per batch of LDS reads
  // (atoms past the end are clamped to the last one and write its values
  // again)
  float* out = force + (size_t)w * fstride;
  const int na = sv.n_atoms;
  for (int a0 = lane; a0 < na; a0 += kGatherBatch * kWave) {
    int ac[kGatherBatch], loc[kGatherBatch];
#pragma unroll
    for (int m = 0; m < kGatherBatch; ++m) {
      ac[m] = min(a0 + m * kWave, na - 1);
      loc[m] = sv.atom_local[ac[m]];
    }
#pragma unroll
    for (int m = 0; m < kGatherBatch; ++m) {
      const int l3 = 3 * max(loc[m], 0);
      const float x = fl[l3], y = fl[l3 + 1], z = fl[l3 + 2];
      const bool on = loc[m] >= 0;
      out[3 * ac[m]] = on ? x : 0.f;
      out[3 * ac[m] + 1] = on ? y : 0.f;
      out[3 * ac[m] + 2] = on ? z : 0.f;
    }
  }
}

// Writes the walker's energy, deviation and sigma (lane 0) and returns sigma.
__device__ inline float switch_outputs(double e, double abar, double eps0, double eps1,
                                       int w, float* energy, float* eps_out,
                                       float* sigma_out, int lane, size_t ostride) {
  const float sig = switch_sigma(e, eps0, eps1);
  if (lane == 0) {
    if (energy) energy[w * ostride] = -sig * (float)abar;
    if (eps_out) eps_out[w * ostride] = (float)e;
    if (sigma_out) sigma_out[w * ostride] = sig;
  }
  return sig;
}

// Whole tail of the bias for walker w, executed by ONE wave (lane 0..63):
// deviation, switch, bias energy and the chain rule to atoms.  With
// g == nullptr the CV force is fcv[w] and sigma = 1 (no statistics).
// Outputs: forces at force + w * fstride, energy/eps/sigma at index w * ostride.
// Reads the members' results with dependent loads; scatter kernels that can
// hold them in registers use scatter_stats_reg instead.
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
    sig = switch_outputs(e, abar, eps0, eps1, w, energy, eps_out, sigma_out, lane, ostride);
  } else {
    for (int i = lane; i < n; i += kWave) fc[i] = fcv[(size_t)w * n + i];
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  scatter_forces(sv, sp, fc, ct, fl, sig, w, force, flags, lane, fstride);
}

// Register-resident form of the per-walker statistics for K <= kRegMembers
// and n <= kRegPasses * 64: a lane loads its CVs' values of every member
// (g [K][B][n], or fcv when g is null) and the members' A into registers in
// one batch, before anything waits on memory.  Indices past K or n are
// clamped to valid ones (loaded, never used), so no load is guarded by a
// branch.  The arithmetic is ensemble_stats' in the same order.
constexpr int kRegMembers = 8;
constexpr int kRegPasses = 2;
struct WalkerRegs {
  float g[kRegPasses][kRegMembers];
  float a[kRegMembers];
};

__device__ inline void walker_prefetch(WalkerRegs& r, const float* A, const float* g,
                                       const float* fcv, int K, int B, int n, int w,
                                       int lane) {
  // one branch-free load pattern for both forms: the CV force fcv [B][n] is
  // g with one member; without g the A loads re-read that array (unused)
  const float* src = g ? g : fcv;
  const int Ke = g ? K : 1;
  const float* ab = g ? A : fcv;
#pragma unroll
  for (int p = 0; p < kRegPasses; ++p) {
    const int i = min(lane + p * kWave, n - 1);
#pragma unroll
    for (int k = 0; k < kRegMembers; ++k)
      r.g[p][k] = src[((size_t)min(k, Ke - 1) * B + w) * n + i];
  }
#pragma unroll
  for (int k = 0; k < kRegMembers; ++k) r.a[k] = ab[(size_t)min(k, Ke - 1) * B + w];
}

// Deviation, mean force into fc[n] and A-bar from the prefetched registers.
__device__ inline double scatter_stats_reg(const WalkerRegs& r, int K, int n, float* fc,
                                           double& abar, int lane) {
  double ss = 0.0;
#pragma unroll
  for (int p = 0; p < kRegPasses; ++p) {
    const int i = lane + p * kWave;
    if (i < n) {
      const double g0 = r.g[p][0];
      double dsum = 0.0, gsum = g0;
#pragma unroll
      for (int k = 1; k < kRegMembers; ++k)
        if (k < K) {
          const double gk = r.g[p][k];
          dsum += gk - g0;
          gsum += gk;
        }
      const double dbar = dsum / K;
      double q = dbar * dbar;
#pragma unroll
      for (int k = 1; k < kRegMembers; ++k)
        if (k < K) {
          const double dk = (double)r.g[p][k] - g0 - dbar;
          q += dk * dk;
        }
      ss += q;
      fc[i] = (float)(gsum / K);
    }
  }
  ss = wave_sum(ss);
  abar = 0.0;
#pragma unroll
  for (int k = 0; k < kRegMembers; ++k)
    if (k < K) abar += (double)r.a[k];
  abar /= K;
  return sqrt(ss / K);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of two
// 32x32 -> 64-bit multiplications, the key bumped by the Weyl constants
// between rounds; counter c in/out, key (k0, k1).
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

// A 32-bit word to a uniform in (0, 1): (2 (x >> 9) + 1) 2^-24, exact in FP32.
__device__ inline float philox_uniform(uint32_t x) {
  return (float)(2u * (x >> 9) + 1u) * 5.9604644775390625e-8f;
}

}  // namespace dev
}  // namespace rid
