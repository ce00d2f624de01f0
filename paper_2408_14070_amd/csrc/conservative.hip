// Conservative switching: the bias force as the exact negative gradient of
// E = -sigma(eps) Abar, including the switching band where sigma depends on
// the walker through the model deviation:
//   f = sigma gbar + Abar sigma'(eps) d eps/ds,
//   d eps/ds = sum_k H_k w_k,  w_k = (g_k - gbar) / (K eps),
// with H_k the Hessian of member k's free energy in s.  FP32 ensembles of
// padded width <= 256 get H_k w_k from one fused forward-over-reverse
// kernel (hvp_kernel: primal and tangent rows share every weight fragment).
// Other ensembles (wider, 16-bit, residual, raw CVs) use the mean-force
// sweeps of the training path in input mode: with rho_x = (dx/ds) w_k held
// fixed, the tangent and adjoint sweeps give d(rho_x . dA_k/dx)/dx; the
// angle chain adds (d rho_x/ds)^T dA_k/dx (zero for a raw CV).
// The frozen-switch path (rid_bias_force) is the same where sigma' = 0.
#include "device_common.h"

namespace rid {
namespace {

using namespace dev;

constexpr int kPrepWaves = 4;

// One wave per walker: deviation (FP64, as in the scatter), switch value and
// slope, energy / eps / sigma outputs, mean force, w_k into rho [B][K][n]
// (zero where the slope or eps is zero), and Abar * sigma'(eps).
__global__ __launch_bounds__(kPrepWaves * kWave) void cons_prep_kernel(
    const float* A, const float* g, int K, int B, int n, double eps0, double eps1,
    float* gbar, float* rho, float* coef, float* sig_w, float* energy, float* eps_out,
    float* sigma_out) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int w = blockIdx.x * kPrepWaves + wave;
  if (w >= B) return;
  // the members' results in registers, loaded in one batch, when they fit
  // (same arithmetic, same order as the load-as-you-go form)
  const bool reg = K <= kRegMembers && n <= kRegPasses * kWave;
  WalkerRegs r;
  double e, abar = 0.0;
  if (reg) {
    walker_prefetch(r, A, g, nullptr, K, B, n, w, lane);
    e = scatter_stats_reg(r, K, n, gbar + (size_t)w * n, abar, lane);
  } else {
    e = ensemble_stats(g, K, B, n, w, gbar + (size_t)w * n, lane);
    for (int k = 0; k < K; ++k) abar += (double)A[(size_t)k * B + w];
    abar /= K;
  }
  const float sig = switch_outputs(e, abar, eps0, eps1, w, energy, eps_out, sigma_out, lane, 1);
  double slope = 0.0;
  if (e >= eps0 && e < eps1) {
    const double t = (e - eps0) / (eps1 - eps0);
    slope = -0.5 * 3.14159265358979323846 / (eps1 - eps0) * sin(3.14159265358979323846 * t);
  }
  if (lane == 0) {
    coef[w] = (float)(abar * slope);
    sig_w[w] = sig;
  }
  const bool on = slope != 0.0 && e > 0.0;
  if (reg) {
#pragma unroll
    for (int p = 0; p < kRegPasses; ++p) {
      const int i = lane + p * kWave;
      if (i < n) {
        double gs = 0.0;
#pragma unroll
        for (int k = 0; k < kRegMembers; ++k)
          if (k < K) gs += (double)r.g[p][k];
        const double gb = gs / K;
#pragma unroll
        for (int k = 0; k < kRegMembers; ++k)
          if (k < K) {
            const double d = (double)r.g[p][k] - gb;
            rho[((size_t)w * K + k) * n + i] = on ? (float)(d / (K * e)) : 0.f;
          }
      }
    }
    return;
  }
  for (int i = lane; i < n; i += kWave) {
    double gs = 0.0;
    for (int k = 0; k < K; ++k) gs += (double)g[((size_t)k * B + w) * n + i];
    const double gb = gs / K;
    for (int k = 0; k < K; ++k) {
      const double d = (double)g[((size_t)k * B + w) * n + i] - gb;
      rho[((size_t)w * K + k) * n + i] = on ? (float)(d / (K * e)) : 0.f;
    }
  }
}

// CV force per (walker, CV): sigma gbar + Abar sigma' sum_k H_k w_k, where
// member k's term in s is  -sin s_i lx[i] + cos s_i lx[n+i]
//                          - w_ki (cos s_i u0[i] + sin s_i u0[n+i])
// (lx = d J_k/dx from the input-mode sweep, u0 = dA_k/dx); for a raw CV
// (encoded (s_i, 0): linear) it is lx[i].  Members summed in order.
__global__ void cons_combine_kernel(const float* s, const float* rho, const float* lam_x,
                                    long long slab_lam, const float* u0, const float* gbar,
                                    const float* coef, const float* sig_w, int K, int B,
                                    int n, const uint8_t* raw, float* fcv) {
  const long long total = (long long)B * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(e / n), i = (int)(e - (long long)b * n);
    float sn, cs;
    sincosf(s[e], &sn, &cs);
    const bool r = raw && raw[i];
    float de = 0.f;
    if (coef[b] != 0.f) {
      for (int k = 0; k < K; ++k) {
        const float* lx = lam_x + k * slab_lam + (long long)b * 2 * n;
        const float* u = u0 + ((long long)k * B + b) * 2 * n;
        const float wk = rho[((long long)b * K + k) * n + i];
        de += r ? lx[i] : -sn * lx[i] + cs * lx[n + i] - wk * (cs * u[i] + sn * u[n + i]);
      }
    }
    fcv[e] = sig_w[b] * gbar[e] + coef[b] * de;
  }
}

// The same with the fused kernel's per-member terms T [K][B][n] (read only
// where coef is nonzero: the kernel skips tiles outside the band).
__global__ void cons_combine_terms_kernel(const float* T, const float* gbar, const float* coef,
                                          const float* sig_w, int K, int B, int n,
                                          float* fcv) {
  const long long total = (long long)B * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(e / n);
    const float cb = coef[b];
    float de = 0.f;
    if (cb != 0.f) {
      if (K <= kRegMembers) {
        // every member's term in flight at once, added in member order
        float t[kRegMembers];
#pragma unroll
        for (int k = 0; k < kRegMembers; ++k) t[k] = T[min(k, K - 1) * total + e];
#pragma unroll
        for (int k = 0; k < kRegMembers; ++k)
          if (k < K) de += t[k];
      } else {
        for (int k = 0; k < K; ++k) de += T[k * total + e];
      }
    }
    fcv[e] = sig_w[b] * gbar[e] + cb * de;
  }
}

}  // namespace

rid_status launch_bias_conservative(const rid_system_impl& s, rid_ensemble_impl& e,
                                    const float* pos, int B, float eps0, float eps1,
                                    float* force, float* energy, float* eps, float* sigma,
                                    uint8_t* flags, hipStream_t st) {
  const int K = e.K, n = e.n_cv;
  rid_status r;
  // workspace: s [B][n], gbar [B][n], fcv [B][n], rho [B][K][n], coef [B],
  // sigma [B], and the fused kernel's terms [K][B][n]
  const size_t nb = (size_t)B * n;
  const bool fused = hvp_fused_supported(e);
  if ((r = e.ws_cons.ensure(sizeof(float) * (3 * nb + nb * K * (fused ? 2 : 1) +
                                             2 * (size_t)B))) != RID_OK)
    return r;
  float* d_s = e.ws_cons.as<float>();
  float* d_gbar = d_s + nb;
  float* d_fcv = d_gbar + nb;
  float* d_rho = d_fcv + nb;
  float* d_coef = d_rho + nb * K;
  float* d_sig = d_coef + B;
  if ((r = e.ws_A.ensure(sizeof(float) * K * (size_t)B)) != RID_OK) return r;
  if ((r = e.ws_g.ensure(sizeof(float) * K * nb)) != RID_OK) return r;
  if ((r = e.ws_x.ensure(sizeof(float) * 2 * nb)) != RID_OK) return r;
  if (e.frag_dirty) {
    if ((r = pack_ensemble_weights(e, st)) != RID_OK) return r;
    e.frag_dirty = false;
  }
  float* A = e.ws_A.as<float>();
  float* g = e.ws_g.as<float>();
  if ((r = launch_cv_eval(s, pos, B, d_s, e.ws_x.as<float>(), st)) != RID_OK) return r;
  if ((r = launch_mlp(e, e.ws_x.as<float>(), B, A, g, st)) != RID_OK) return r;
  hipLaunchKernelGGL(cons_prep_kernel, dim3((B + kPrepWaves - 1) / kPrepWaves),
                     dim3(kPrepWaves * kWave), 0, st, A, g, K, B, n, (double)eps0,
                     (double)eps1, d_gbar, d_rho, d_coef, d_sig, energy, eps, sigma);
  RID_HIP(hipGetLastError());
  const int grid = (int)std::min<size_t>((nb + 255) / 256, 4096);
  if (fused) {
    float* d_T = d_sig + B;
    if ((r = launch_hvp(e, e.ws_x.as<float>(), d_rho, d_coef, B, d_T, st)) != RID_OK) return r;
    hipLaunchKernelGGL(cons_combine_terms_kernel, dim3(grid), dim3(256), 0, st, d_T, d_gbar,
                       d_coef, d_sig, K, B, n, d_fcv);
    RID_HIP(hipGetLastError());
    return launch_bias_scatter(s, 0, pos, B, nullptr, nullptr, d_fcv, 0.0f, 1.0f, force,
                               nullptr, nullptr, nullptr, flags, st);
  }
  InputHvp hvp;
  if ((r = launch_mf_grad(e, d_s, nullptr, d_rho, B, nullptr, nullptr, nullptr, st, &hvp)) !=
      RID_OK)
    return r;
  hipLaunchKernelGGL(cons_combine_kernel, dim3(grid), dim3(256), 0, st, d_s, d_rho, hvp.lam_x,
                     hvp.slab_lam, hvp.u0, d_gbar, d_coef, d_sig, K, B, n,
                     e.raw.empty() ? nullptr : e.d_raw, d_fcv);
  RID_HIP(hipGetLastError());
  return launch_bias_scatter(s, 0, pos, B, nullptr, nullptr, d_fcv, 0.0f, 1.0f, force,
                             nullptr, nullptr, nullptr, flags, st);
}

}  // namespace rid
