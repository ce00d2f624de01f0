// Mean-force fitting step ("Training phase"): the models' CV gradients are
// fitted to mean-force labels, so the loss gradient in the weights needs the
// derivative of dA/ds -- a double backward.
//
// With rho_b = 2 (g_b - F_b) / B mapped to the input x (rho_x), the weight
// gradient of L = (1/B) sum_b |g_b - F_b|^2 equals the gradient of
// J = sum_b rho_x,b . dA/dx with rho_x held fixed:
//   primal   h_l = tanh(W_l h_{l-1} + b_l)                 (h_0 = x)
//   backward v_L = w_o (1-h_L^2), u_{l-1} = W_l^T v_l, v_l = u_l (1-h_l^2)
//   tangent  zd_l = W_l hd_{l-1}, hd_l = (1-h_l^2) zd_l     (hd_0 = rho_x)
//   adjoint  lam_hd_L = w_o, lam_h_L = 0; for l = L..1:
//            lam_zd = (1-h_l^2) lam_hd, lam_h -= 2 h_l zd_l lam_hd,
//            lam_z = (1-h_l^2) lam_h,
//            dW_l = lam_z^T h_{l-1} + lam_zd^T hd_{l-1}, db_l = sum lam_z,
//            [lam_h ; lam_hd]_{l-1} = [lam_z ; lam_zd] W_l
//   dw_o = sum hd_L, db_o = 0.
// Then one Adam step on the FP32 masters.
//
// General form (the sweeps as separate GEMMs: wide and 16-bit ensembles,
// residual networks, dropout on them, mixed angular masks).  With t_l =
// tanh(z_l), dropout factors S_l (1 without dropout) and d_l = S_l (1 - t_l^2):
//   primal   h_l = S_l t_l (+ h_{l-1} for a residual layer l >= 2)
//   backward u_L = w_o, v_l = u_l d_l, u_{l-1} = W_l^T v_l (+ u_l, residual)
//   tangent  hd_l = d_l zd_l (+ hd_{l-1}, residual)
//   adjoint  lam_zd = d_l lam_hd, lam_z = d_l (lam_h - 2 t_l zd_l lam_hd),
//            [lam_h ; lam_hd]_{l-1} = [lam_z ; lam_zd] W_l (+ [lam_h ; lam_hd]_l,
//            residual)
// Raw CVs (angular mask 0) enter as (s, 0): their mean force is dA/dx_i and
// rho reaches the input as (rho_i, 0).
//
// Layout: batched over the K members; "stacked" tensors hold the primal
// quantity in rows [0, B) and the tangent one in rows [B, 2B) of each
// member's slab, so one GEMM moves both halves, and the weight gradient is a
// single contraction over 2B rows.  All GEMMs are one hand-written FP32-MFMA
// kernel (64x64 tiles, LDS double buffering, arbitrary strides, fused
// epilogues); the weight-gradient GEMM is split along the batch with a
// fixed-order reduction, so the whole step is deterministic.
#include "device_common.h"

namespace rid {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, LDK = BK + 4;   // BM, BN: split-K sizing
constexpr int kThreads = 256;

enum Epi {
  EPI_STORE = 0,      // C = acc
  EPI_BIAS_TANH = 1,  // C = tanh(acc + bias[n])
  EPI_GEN = 2         // r = acc + add; C = r (if C); C2 = r * mul + add2 (if C2)
};

struct GemmArgs {
  const float* A;
  long long sAb, sAm, sAk;
  const float* Bm;
  long long sBb, sBk, sBn;
  float* C;
  long long sCb, sCm, sCn, sCs;   // sCs: split-K slab stride
  float* C2;                      // second output (EPI_GEN): C's row and
  long long sC2b;                 // column strides, own batch stride
  const float* bias;
  long long sBiasb;
  // EPI_GEN operands (each null or indexed like C, with its own batch stride)
  const float* add;
  long long sAddb;
  const float* mul;
  long long sMulb;
  const float* add2;
  long long sAdd2b;
  int M, N, Kc, batch, ksplit, kchunk, mode;
  int modeA, modeB;               // operand load modes (TileLoad), set by gemm()
};

// One operand tile of TR rows x BK contraction into LDS [row][k].  Element
// (r, k) of the operand is at X[r * sR + k * sK].  Modes: 0 scalar loads,
// k fastest; 1 scalar, rows fastest; 2 float4 along k (sK == 1); 3 float4
// along rows (sR == 1).  The float4 modes need 16-byte alignment and an
// extent along the vector that is a multiple of 4 (gemm() checks).
template <int TR, int BKT = BK>
struct TileLoad {
  static constexpr int NS = TR * BKT / kThreads;   // elements per thread
  float v[NS];
  // Branch-free loads (the mode is uniform; the two mappings are selected,
  // an element outside the operand reads its first one), so every load of a
  // tile is in flight before anything waits on one.  The outside elements
  // are zeroed when the tile is stored to LDS, after the block's MFMAs.
  // VEC: the float4 modes (chosen at compile time, so that no branch joins
  // the two load paths: a join makes the compiler wait on the loads there).
  unsigned long long in_mask;
  template <bool VEC>
  __device__ inline void load(const float* X, long long sR, long long sK, int mode, int r0,
                              int R, int kb, int k_end, int tid) {
    static_assert(NS <= 64, "one mask bit per element");
    in_mask = 0ull;
    if constexpr (VEC && NS >= 4) {
      const bool kv = mode == 2;
#pragma unroll
      for (int j = 0; j < NS / 4; ++j) {
        const int idx = tid + kThreads * j;
        const int r = kv ? idx / (BKT / 4) : (idx % (TR / 4)) * 4;
        const int k = kv ? (idx % (BKT / 4)) * 4 : idx / (TR / 4);
        const int gr = r0 + r, gk = kb + k;
        const bool in = gr < R && gk < k_end;
        in_mask |= (unsigned long long)in << j;
        const f4 x = *reinterpret_cast<const f4*>(X + (in ? gr * sR + gk * sK : 0));
        v[4 * j] = x[0];
        v[4 * j + 1] = x[1];
        v[4 * j + 2] = x[2];
        v[4 * j + 3] = x[3];
      }
    } else {
      const bool kf = (mode & 1) == 0;     // modes 0 and 2: k fastest
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const int idx = tid + kThreads * j;
        const int k = kf ? idx % BKT : idx / TR;
        const int r = kf ? idx / BKT : idx % TR;
        const int gr = r0 + r, gk = kb + k;
        const bool in = gr < R && gk < k_end;
        in_mask |= (unsigned long long)in << j;
        v[j] = X[in ? gr * sR + gk * sK : 0];
      }
    }
  }
  template <bool VEC>
  __device__ inline void store(float (*S)[BKT + 4], int mode, int tid) const {
    if constexpr (VEC && NS >= 4) {
#pragma unroll
      for (int j = 0; j < NS / 4; ++j) {
        const int idx = tid + kThreads * j;
        const bool in = (in_mask >> j) & 1ull;
        const f4 x = in ? f4{v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]}
                        : f4{0.f, 0.f, 0.f, 0.f};
        if (mode == 2) {
          const int r = idx / (BKT / 4), k = (idx % (BKT / 4)) * 4;
          *reinterpret_cast<f4*>(&S[r][k]) = x;
        } else {
          const int k = idx / (TR / 4), r = (idx % (TR / 4)) * 4;
#pragma unroll
          for (int e = 0; e < 4; ++e) S[r + e][k] = x[e];
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const int idx = tid + kThreads * j;
        int r, k;
        if ((mode & 1) == 0) { k = idx % BKT; r = idx / BKT; } else { r = idx % TR; k = idx / TR; }
        S[r][k] = ((in_mask >> j) & 1ull) ? v[j] : 0.f;
      }
    }
  }
};

__device__ inline float tanh_fast(float z) {
  const float e = __expf(2.f * z);
  return 1.f - 2.f * __builtin_amdgcn_rcpf(1.f + e);
}

// C[b] = A[b] (M x Kc) * B[b] (Kc x N) on FP32 MFMA, tiles of TM x TN with
// 4 waves of (TM/2) x (TN/2); operands staged through double-buffered LDS
// in contraction blocks of BKT.  128 x 128 tiles (16 accumulator tiles per
// wave) reuse each LDS operand fragment four times; 64 x 64 tiles serve
// narrow shapes.  Grids too small to fill the chip (small batches) take
// 64-deep blocks: each block costs about one memory latency, so a deeper
// block divides the latency-bound time of such a GEMM by four.
template <int TM, int TN, int BKT, bool VA, bool VB>
__global__ __launch_bounds__(kThreads) void gemm_f32_kernel(GemmArgs g) {
  constexpr int WM = TM / 2, WN = TN / 2;           // wave tile
  constexpr int TI = WM / 16, TJ = WN / 16;         // 16 x 16 MFMA tiles per wave
  static_assert(BKT % 16 == 0, "contraction blocks of whole 16-deep MFMA sets");
  __shared__ __attribute__((aligned(16))) float As[2][TM][BKT + 4];
  __shared__ __attribute__((aligned(16))) float Bs[2][TN][BKT + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b = blockIdx.z / g.ksplit, s = blockIdx.z % g.ksplit;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int k_begin = s * g.kchunk;
  const int k_end = min(g.Kc, k_begin + g.kchunk);
  const float* A = g.A + b * g.sAb;
  const float* Bp = g.Bm + b * g.sBb;
  TileLoad<TM, BKT> ta;
  TileLoad<TN, BKT> tb;
  auto load = [&](int kb) {
    ta.template load<VA>(A, g.sAm, g.sAk, g.modeA, m0, g.M, kb, k_end, tid);
    tb.template load<VB>(Bp, g.sBn, g.sBk, g.modeB, n0, g.N, kb, k_end, tid);
  };
  auto store = [&](int buf) {
    ta.template store<VA>(As[buf], g.modeA, tid);
    tb.template store<VB>(Bs[buf], g.modeB, tid);
  };

  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  const int r = lane & 15, gq = lane >> 4;
  f4 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  int buf = 0;
  load(k_begin);
  store(0);
  __syncthreads();
  for (int kb = k_begin; kb < k_end; kb += BKT) {
    const bool more = kb + BKT < k_end;
    if (more) load(kb + BKT);
#pragma unroll
    for (int sb = 0; sb < BKT / 16; ++sb) {
      f4 a[TI], bb[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i)
        a[i] = *reinterpret_cast<const f4*>(&As[buf][wm + i * 16 + r][16 * sb + 4 * gq]);
#pragma unroll
      for (int j = 0; j < TJ; ++j)
        bb[j] = *reinterpret_cast<const f4*>(&Bs[buf][wn + j * 16 + r][16 * sb + 4 * gq]);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j)
            acc[i][j] =
                __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][e], bb[j][e], acc[i][j], 0, 0, 0);
    }
    if (more) {
      store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  // Epilogue, one row of 16 x 16 tiles at a time: the operands it reads
  // (bias, add, mul, add2) are loaded for all of the row's elements before
  // any is used (an element outside C reads element 0 and is not stored),
  // so their loads are in flight together.
  float* C = g.C ? g.C + b * g.sCb + s * g.sCs : nullptr;
  constexpr int E = TJ * 4;
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    long long ci[E];
    bool in[E];
    float bi[TJ], ad[E], mu[E], a2[E];
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int n = n0 + wn + j * 16 + r;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + i * 16 + 4 * gq + q;
        in[4 * j + q] = n < g.N && m < g.M;
        ci[4 * j + q] = in[4 * j + q] ? m * g.sCm + n * g.sCn : 0;
      }
      bi[j] = 0.f;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) ad[e] = mu[e] = a2[e] = 0.f;
    if (g.mode == EPI_BIAS_TANH) {
#pragma unroll
      for (int j = 0; j < TJ; ++j) bi[j] = g.bias[b * g.sBiasb + min(n0 + wn + j * 16 + r, g.N - 1)];
    } else if (g.mode == EPI_GEN) {
      if (g.add)
#pragma unroll
        for (int e = 0; e < E; ++e) ad[e] = g.add[b * g.sAddb + ci[e]];
      if (g.C2) {
#pragma unroll
        for (int e = 0; e < E; ++e) mu[e] = g.mul[b * g.sMulb + ci[e]];
        if (g.add2)
#pragma unroll
          for (int e = 0; e < E; ++e) a2[e] = g.add2[b * g.sAdd2b + ci[e]];
      }
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = 4 * j + q;
        if (!in[e]) continue;
        const float v = acc[i][j][q];
        if (g.mode == EPI_STORE) {
          C[ci[e]] = v;
        } else if (g.mode == EPI_BIAS_TANH) {
          C[ci[e]] = tanh_fast(v + bi[j]);
        } else {
          const float rr = g.add ? v + ad[e] : v;
          if (C) C[ci[e]] = rr;
          if (g.C2) {
            float o = rr * mu[e];
            if (g.add2) o += a2[e];
            g.C2[b * g.sC2b + ci[e]] = o;
          }
        }
      }
  }
}

// x = [cos s | sin s] into the primal half of every member's stacked slab
// (raw CVs, raw[i] = 1: (s_i, 0))
__global__ void train_embed_kernel(const float* s, int B, int n, int K, const uint8_t* raw,
                                   float* HH0, long long slab) {
  const long long total = (long long)K * B * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / ((long long)B * n));
    const long long r = e - (long long)k * B * n;
    const int b = (int)(r / n), i = (int)(r - (long long)b * n);
    const float si = s[(long long)b * n + i];
    float sn, cs;
    sincosf(si, &sn, &cs);
    const bool is_raw = raw && raw[i];
    float* row = HH0 + k * slab + (long long)b * 2 * n;
    row[i] = is_raw ? si : cs;
    row[n + i] = is_raw ? 0.f : sn;
  }
}

// Activation stage of hidden layer l (1-based) from its tanh branch
// T = tanh(z_l) [K][B][w]: h_l = S t (+ h_{l-1} when residual) into the
// primal half of the stacked slab, and d_l = S (1 - t^2) into D.  S is the
// dropout factor: unit j of sample b of member k is kept when the uniform of
// word j mod 4 of the Philox4x32-10 block with counter (b, step, 16 k + l,
// j div 4) and key (seed) is >= p, scaled by 1/(1 - p); 1 without dropout.
// b is the sample's index in the whole batch: row r of a chunk is sample
// row_base + r.  A thread handles the 4 units of one block.
__global__ void act_kernel(const float* T, int l, int w, int B, int K, int row_base,
                           float drop_p, float drop_inv, unsigned long long seed,
                           uint32_t step, const float* Hprev, long long slab_prev, float* H,
                           long long slab, float* D) {
  const int nq = (w + 3) / 4;
  const long long total = (long long)K * B * nq;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / ((long long)B * nq));
    const long long rq = e - (long long)k * B * nq;
    const int b = (int)(rq / nq), q = (int)(rq - (long long)b * nq);
    // the four units' loads first (units past w re-read the last one, and a
    // missing Hprev re-reads T; neither is used), the mask bits meanwhile
    const long long ob = ((long long)k * B + b) * w;               // [K][B][w]
    const float* hsrc = Hprev ? Hprev + (long long)k * slab_prev + (long long)b * w : T + ob;
    float tv[4], hv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = min(4 * q + u, w - 1);
      tv[u] = T[ob + j];
      hv[u] = hsrc[j];
    }
    uint32_t c[4] = {(uint32_t)(row_base + b), step, (uint32_t)(16 * k + l), (uint32_t)q};
    if (drop_p > 0.f)
      dev::philox4x32_10(c, (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32));
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = 4 * q + u;
      if (j >= w) break;
      const float sc = drop_p > 0.f ? (dev::philox_uniform(c[u]) >= drop_p ? drop_inv : 0.f)
                                    : 1.f;
      const float t = tv[u];
      float h = sc * t;
      if (Hprev) h += hv[u];
      H[(long long)k * slab + (long long)b * w + j] = h;
      D[ob + j] = sc * (1.f - t * t);
    }
  }
}

// The layer weights of every member into the aligned copy: block row
// y = k L + l copies layer l's matrix (row-major [out][in], cnt floats) of
// member k from master + k*pm + src[l] to wpad + k*pmp + dst[l], its blocks
// striding over the matrix (contiguous, coalesced, no index arithmetic).
struct WpadCopy {
  long long src[kMaxHidden], dst[kMaxHidden], cnt[kMaxHidden];
  int L;
};
__global__ void wpad_copy_kernel(const float* master, long long pm, float* wpad, long long pmp,
                                 WpadCopy c) {
  const int k = blockIdx.y / c.L, l = blockIdx.y - k * c.L;
  const float* src = master + k * pm + c.src[l];
  float* dst = wpad + k * pmp + c.dst[l];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < c.cnt[l];
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

// out[k][b][j] = w_o[k][j] (the top of the reverse sweeps: u_L, lam_hd_L),
// into rows [r0, r0 + B) of a [K][rows][w] slab (the other rows, if any, 0)
__global__ void top_kernel(const float* master, long long per_model, int wo_off, int w, int B,
                           int K, int rows, int r0, float* out) {
  const long long total = (long long)K * rows * w;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / ((long long)rows * w));
    const long long r = e - (long long)k * rows * w;
    const int row = (int)(r / w), j = (int)(r - (long long)row * w);
    out[e] = (row >= r0 && row < r0 + B) ? master[k * per_model + wo_off + j] : 0.f;
  }
}

// v_L = w_o d_L
__global__ void vlast_kernel(const float* DL, const float* master, long long per_model,
                             int wo_off, int w, int B, int K, float* V) {
  const long long total = (long long)K * B * w;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / ((long long)B * w));
    const long long r = e - (long long)k * B * w;
    const int j = (int)(r % w);
    V[e] = master[k * per_model + wo_off + j] * DL[e];
  }
}

// g = chain(u0, s); residual; per-row squared residual; rho_x into the
// tangent half of the stacked input slab.  With an upstream gradient
// rho [B][K][n] given instead of labels, rho_x is built from it directly.
// One wave per (member, sample) row, lanes over the CVs; the row's squared
// residual is a fixed-order shuffle sum over the lanes.  B rows of a batch
// of B_norm samples (rho = 2 (g - F) / B_norm); row b of member k's squared
// residual goes to loss_rows[k * loss_ld + b].
constexpr int kResWaves = 4;
__global__ __launch_bounds__(kResWaves * 64) void residual_kernel(
    const float* s, const float* F, const float* rho_in, const float* U0, int B, int B_norm,
    int n, int K, const uint8_t* raw, float* HH0, long long slab, float* loss_rows,
    long long loss_ld) {
  const long long e = (long long)blockIdx.x * kResWaves + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (e >= (long long)K * B) return;
  const int k = (int)(e / B), b = (int)(e - (long long)k * B);
  const float* u = U0 + e * 2 * n;
  float* rx = HH0 + k * slab + ((long long)B + b) * 2 * n;
  float acc = 0.f;
  // (every load of a CV first, without branches: a null raw table reads the
  // CV bytes of s instead, unused; F or rho_in, whichever is given)
  const uint8_t* rawp = raw ? raw : reinterpret_cast<const uint8_t*>(s);
  for (int i = lane; i < n; i += 64) {
    const float sv = s[(long long)b * n + i];
    const uint8_t rv = rawp[i];
    const float ua = u[i], ub = u[n + i];
    const float fv = rho_in ? rho_in[((long long)b * K + k) * n + i] : F[(long long)b * n + i];
    float sn, cs;
    sincosf(sv, &sn, &cs);
    if (raw && rv) {                  // raw CV: x_i = s_i, dx/ds = (1, 0)
      sn = -1.f;
      cs = 0.f;
    }
    float rho;
    if (rho_in) {
      rho = fv;
    } else {
      const float gi = -sn * ua + cs * ub;
      const float ri = gi - fv;
      acc += ri * ri;
      rho = 2.f * ri / (float)B_norm;
    }
    rx[i] = -sn * rho;
    rx[n + i] = cs * rho;
  }
  if (loss_rows) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
    if (lane == 0) loss_rows[(long long)k * loss_ld + b] = acc;
  }
}

// Adjoint stage of layer l: given t_l, d_l, zd_l (each [K][B][w]) and the
// stacked (lam_h ; lam_hd) of layer l, produce the stacked (lam_z ; lam_zd).
__global__ void adjoint_kernel(const float* Tl, const float* Dl, const float* Zd,
                               const float* LAM, long long slab_lam, int w, int B, int K,
                               float* S, long long slab_s) {
  const long long total = (long long)K * B * w;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / ((long long)B * w));
    const long long r = e - (long long)k * B * w;   // row-major offset inside the primal half
    const float t = Tl[e], d = Dl[e], zd = Zd[e];
    const float lh = LAM[k * slab_lam + r];
    const float lhd = LAM[k * slab_lam + (long long)B * w + r];
    S[k * slab_s + r] = d * (lh - 2.f * t * zd * lhd);   // lam_z
    S[k * slab_s + (long long)B * w + r] = d * lhd;       // lam_zd
  }
}

// Column sums out[k][j] = sum_b X[k][b][j] in two fixed-order stages.
// Stage 1: block (column tile of 64, row chunk of kColRows, member); lanes
// are columns (coalesced rows), the 4 waves take interleaved rows and are
// combined in wave order -> part[chunk][k][j].
constexpr int kColRows = 64;     // 4 row chunks per 256 rows: enough workgroups in flight
__global__ __launch_bounds__(256) void colsum_partial_kernel(const float* X, long long slab,
                                                             int B, int w, float* part, int K) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  const int chunk = blockIdx.y, k = blockIdx.z;
  const int r0 = chunk * kColRows, r1 = min(B, r0 + kColRows);
  float acc = 0.f;
  if (j < w) {
    const float* p = X + k * slab + j;
#pragma unroll 4
    for (int b = r0 + wave; b < r1; b += 4) acc += p[(long long)b * w];
  }
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && j < w)
    part[((long long)chunk * K + k) * w + j] =
        ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Stage 2: out[k][j] = the chunk partials summed in chunk order, into the
// gradient buffer at grad + k*per_model + dst_off + j (added to what it
// holds when accumulate is set).  A block covers 64 outputs; each of its 4
// waves sums a quarter of the chunks (in order) and the quarters are
// combined in wave order.
__global__ __launch_bounds__(256) void colsum_final_kernel(const float* part, int chunks, int w,
                                                           int K, float* grad,
                                                           long long per_model, int dst_off,
                                                           int accumulate) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;     // output k*w + j
  const int cq = (chunks + 3) / 4;
  const int c0 = wave * cq, c1 = min(chunks, c0 + cq);
  float acc = 0.f;
  if (e < K * w) {
#pragma unroll 4
    for (int c = c0; c < c1; ++c) acc += part[(long long)c * K * w + e];
  }
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && e < K * w) {
    const int k = e / w, j = e - k * w;
    const float v = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    float* o = grad + k * per_model + dst_off + j;
    *o = accumulate ? *o + v : v;
  }
}

// dW[k] = sum over split-K slabs (fixed order) -> gradient buffer (added to
// what it holds when accumulate is set); with bpart, also db[k] = the
// slabs' bias partials bpart[s][k][out] summed in slab order, to b_off
__global__ void splitk_reduce_kernel(const float* part, long long slab_s, int ks,
                                     int out, int in, int K, float* grad,
                                     long long per_model, int w_off, int accumulate,
                                     const float* bpart, int b_off) {
  const long long total = (long long)K * out * in;
  const long long all = total + (bpart ? (long long)K * out : 0);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < all;
       e += (long long)gridDim.x * blockDim.x) {
    float* o;
    const float* src;
    long long stride;
    if (e < total) {
      src = part + e;
      stride = slab_s;
      const int k = (int)(e / ((long long)out * in));
      const long long r = e - (long long)k * out * in;
      o = grad + k * per_model + w_off + r;
    } else {
      const long long eb = e - total;                 // k * out + j
      src = bpart + eb;
      stride = (long long)K * out;
      const int k = (int)(eb / out);
      o = grad + k * per_model + b_off + (eb - (long long)k * out);
    }
    // slabs added in order, eight loads in flight
    float acc = 0.f;
    int s = 0;
    for (; s + 8 <= ks; s += 8) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = src[(s + j) * stride];
#pragma unroll
      for (int j = 0; j < 8; ++j) acc += v[j];
    }
    for (; s < ks; ++s) acc += src[s * stride];
    *o = accumulate ? *o + acc : acc;
  }
}

// The step's last launch, one block per member k: the loss, the mean of the
// member's per-row losses rows[k][0:B] (each thread adds its rows in row
// order, eight loads in flight, then a fixed pairwise tree), and the output
// bias's gradient set to zero (it never reaches grad_s A).
__global__ __launch_bounds__(256) void train_finish_kernel(const float* rows, int B, float* loss,
                                                           float* grad, long long per_model,
                                                           int zero_off) {
  __shared__ float red[256];
  const int k = blockIdx.x;
  if (threadIdx.x == 0 && grad) grad[k * per_model + zero_off] = 0.f;
  if (!rows || !loss) return;     // uniform over the block
  const float* r = rows + (long long)k * B;
  float acc = 0.f;
  int b = threadIdx.x;
  for (; b + 7 * 256 < B; b += 8 * 256) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = r[b + j * 256];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += v[j];
  }
  for (; b < B; b += 256) acc += r[b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[k] = red[0] / (float)B;
}

__global__ void adam_kernel(float* theta, float* m, float* v, const float* g,
                            long long n, float lr, float c1, float c2) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = 0.9f * m[e] + 0.1f * gi;
    const float vi = 0.999f * v[e] + 0.001f * gi * gi;
    m[e] = mi;
    v[e] = vi;
    theta[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  }
}

// Weight-gradient GEMM: C_s[b] = sum over the k-chunk s of A[b][k][m] B[b][k][n]
// (A: [Kc][M] rows, m contiguous; B: [Kc][N] rows, n contiguous -- the
// stacked lam and activation slabs, whose contraction index is the row).
// The 32x32x2 FP32 MFMA takes A as 32 m x 2 k with lane l holding
// (m = l % 32, k = l / 32), and B likewise, so each lane loads one float of
// each operand straight from the row-major slabs with coalesced 128-byte
// row segments: no LDS staging, no transposes, no barriers in the loop.
// A workgroup owns a 64 x 64 tile of one member and one k-chunk; its four
// waves take consecutive quarters of the chunk (two rows per k-step, 2 x 2
// MFMA tiles per wave, loads issued WG_PF k-steps ahead) and their partial
// tiles are added through LDS in a fixed order ((w0 + w2) + (w1 + w3)), so
// the result does not depend on timing.  With csum, the workgroups of the
// first column tile also sum A over the rows below csum_rows (the bias
// gradient: lam_z over the primal rows), per split slab.
struct WgradArgs {
  const float* A;
  long long sAb;
  int lda;
  const float* B;
  long long sBb;
  int ldb;
  float* C;           // tile of split s, member b: C + s*sCs + b*sCb, [M][N]
  long long sCs, sCb;
  float* csum;        // bias sums of split s, member b: csum + s*csum_ss + b*csum_sb, [M]
  long long csum_ss, csum_sb;
  int csum_rows;
  int M, N, Kc, batch, ksplit, kchunk;
};

typedef float f16v __attribute__((ext_vector_type(16)));
#ifndef RID_WG_PF
#define RID_WG_PF 6
#endif
constexpr int kWgPF = RID_WG_PF;   // k-steps of loads in flight per wave
constexpr int kWgLdsStride = 65;   // padded row of a partial tile in LDS

__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs g) {
  __shared__ float red[2][64][kWgLdsStride];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lo = lane & 31, hi = lane >> 5;
  const int b = blockIdx.z / g.ksplit, s = blockIdx.z % g.ksplit;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int c_begin = s * g.kchunk, c_end = min(g.Kc, c_begin + g.kchunk);
  // this wave's quarter of the chunk, in whole k-steps of two rows
  const int steps = (c_end - c_begin + 1) / 2;
  const int q = (steps + 3) / 4;
  const int k_begin = c_begin + 2 * min(steps, wave * q);
  const int k_end = min(c_end, c_begin + 2 * min(steps, (wave + 1) * q));
  const float* A = g.A + b * g.sAb;
  const float* Bp = g.B + b * g.sBb;
  // the lane's element of a k-step: row k + hi, its column clamped into the
  // operand.  A lane whose column lies outside only feeds accumulator rows
  // or columns that are never stored, so its value needs no masking.  Every
  // wave's range holds an even number of rows (chunks and quarters are
  // whole k-steps of an even Kc), so row k + hi is always inside it.
  // Offsets from the (uniform) row start are per-lane constants.
  // Buffer loads: the lane's byte offset in the vector offset, the row's in
  // the scalar offset, so the loop does no address arithmetic.
  const int ma = min(m0 + lo, g.M - 1), mb = min(m0 + 32 + lo, g.M - 1);
  const int na = min(n0 + lo, g.N - 1), nb = min(n0 + 32 + lo, g.N - 1);
  const int oa0 = 4 * (hi * g.lda + ma), oa1 = 4 * (hi * g.lda + mb);
  const int ob0 = 4 * (hi * g.ldb + na), ob1 = 4 * (hi * g.ldb + nb);
  const __amdgpu_buffer_rsrc_t ra =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(A), (short)0, 0x7FFFFFF0, 0x00020000);
  const __amdgpu_buffer_rsrc_t rb =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(Bp), (short)0, 0x7FFFFFF0, 0x00020000);
  const bool csum_wg = g.csum && blockIdx.x == 0;
  const int csum_end = min(k_end, g.csum_rows);

  f16v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f16v{};
  float cs0 = 0.f, cs1 = 0.f;
  // ring of loaded k-steps: [slot][a0, a1, b0, b1]
  float ring[kWgPF][4];
  auto issue = [&](int slot, int k) {
    const int sa = 4 * k * g.lda, sb = 4 * k * g.ldb;   // row byte offsets (uniform)
    ring[slot][0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ra, oa0, sa, 0));
    ring[slot][1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ra, oa1, sa, 0));
    ring[slot][2] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, ob0, sb, 0));
    ring[slot][3] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, ob1, sb, 0));
  };
  // k-steps of the wave; loads run kWgPF steps ahead through the ring.  The
  // main loop has no conditional code (a step past the last one re-reads
  // the last, and is never consumed), so the loads stay in flight.
  const int nst = (k_end - k_begin) / 2;
  auto step_row = [&](int t) { return k_begin + 2 * min(t, nst - 1); };
  auto consume = [&](int p, int t) {
    const float a0 = ring[p][0], a1 = ring[p][1], b0 = ring[p][2], b1 = ring[p][3];
    if (csum_wg) {
      const bool in = k_begin + 2 * t + hi < csum_end;
      cs0 += in ? a0 : 0.f;
      cs1 += in ? a1 : 0.f;
    }
    acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
  };
  if (nst > 0) {
#pragma unroll
    for (int p = 0; p < kWgPF; ++p) issue(p, step_row(p));
    const int nfull = nst / kWgPF;
    for (int blk = 0; blk < nfull; ++blk) {
#pragma unroll
      for (int p = 0; p < kWgPF; ++p) {
        const int t = blk * kWgPF + p;
        consume(p, t);
        issue(p, step_row(t + kWgPF));
      }
    }
    const int rem = nst - nfull * kWgPF;
#pragma unroll
    for (int p = 0; p < kWgPF; ++p)
      if (p < rem) consume(p, nfull * kWgPF + p);
  }
  // accumulator element v of a 32 x 32 tile: row 8 (v / 4) + 4 hi + v % 4,
  // column lo.  Waves 2, 3 park their tiles; waves 0, 1 add them; wave 1
  // parks the sum; wave 0 adds it and writes the slab.
  // (one accumulator tile at a time: the scheduling barriers keep the
  // compiler from reading all four tiles into registers at once)
  auto park = [&](int slot) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int v = 0; v < 16; ++v)
          red[slot][32 * i + 8 * (v / 4) + 4 * hi + (v % 4)][32 * j + lo] = acc[i][j][v];
        __builtin_amdgcn_sched_barrier(0);
      }
  };
  auto take = [&](int slot) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int v = 0; v < 16; ++v)
          acc[i][j][v] += red[slot][32 * i + 8 * (v / 4) + 4 * hi + (v % 4)][32 * j + lo];
        __builtin_amdgcn_sched_barrier(0);
      }
  };
  // the bias sums: combine the two row parities of a lane pair, then the
  // waves in the same fixed order through LDS (column 64 of the tile rows)
  __shared__ float cred[4][64];
  if (csum_wg) {
    cs0 += __shfl_xor(cs0, 32);
    cs1 += __shfl_xor(cs1, 32);
    if (hi == 0) {
      cred[wave][lo] = cs0;
      cred[wave][32 + lo] = cs1;
    }
  }
  if (wave >= 2) park(wave - 2);
  __syncthreads();
  if (wave < 2) take(wave);
  __syncthreads();
  if (wave == 1) park(0);
  __syncthreads();
  if (wave == 0) {
    take(0);
    park(1);
  }
  __syncthreads();
  // the summed tile, stored by all waves: a row per wave and store, one
  // column per lane (256-byte row segments)
  float* Ct = g.C + s * g.sCs + b * g.sCb + (long long)m0 * g.N + n0;
  for (int r = wave; r < 64 && m0 + r < g.M; r += 4)
    if (n0 + lane < g.N) Ct[(long long)r * g.N + lane] = red[1][r][lane];
  if (csum_wg && wave == 0) {
    const int m = m0 + lane;
    const float v = (cred[0][lane] + cred[2][lane]) + (cred[1][lane] + cred[3][lane]);
    if (m < g.M) g.csum[s * g.csum_ss + b * g.csum_sb + m] = v;
  }
}

inline int grid1d(long long total) {
  return (int)std::min<long long>((total + 255) / 256, 4096);
}

// Load mode of one operand (see TileLoad): float4 along the unit-stride
// dimension when alignment and extents allow, else scalar.
int load_mode(const float* X, long long sR, long long sK, long long sBatch, int R, int Kc) {
  const bool al = (reinterpret_cast<uintptr_t>(X) % 16 == 0) && sBatch % 4 == 0;
  if (sK == 1) return (al && sR % 4 == 0 && Kc % 4 == 0) ? 2 : 0;
  if (sR == 1) return (al && sK % 4 == 0 && R % 4 == 0) ? 3 : 1;
  return 0;
}

// One tile shape, with the float4 load modes of the two operands as
// compile-time choices.
template <int TM, int TN, int BKT>
void launch_gemm_tile(dim3 grid, const GemmArgs& g, hipStream_t st) {
  const bool va = g.modeA >= 2, vb = g.modeB >= 2;
  if (va && vb)
    hipLaunchKernelGGL((gemm_f32_kernel<TM, TN, BKT, true, true>), grid, dim3(kThreads), 0, st, g);
  else if (va)
    hipLaunchKernelGGL((gemm_f32_kernel<TM, TN, BKT, true, false>), grid, dim3(kThreads), 0, st, g);
  else if (vb)
    hipLaunchKernelGGL((gemm_f32_kernel<TM, TN, BKT, false, true>), grid, dim3(kThreads), 0, st, g);
  else
    hipLaunchKernelGGL((gemm_f32_kernel<TM, TN, BKT, false, false>), grid, dim3(kThreads), 0, st, g);
}

#ifndef RID_GEMM_DEEP_WGS
#define RID_GEMM_DEEP_WGS 256
#endif
rid_status gemm(const GemmArgs& g0, hipStream_t st) {
  GemmArgs g = g0;
  if (g.ksplit < 1) g.ksplit = 1;
  if (g.kchunk <= 0) g.kchunk = round_up(g.Kc, BK);
  g.modeA = load_mode(g.A, g.sAm, g.sAk, g.sAb, g.M, g.Kc);
  g.modeB = load_mode(g.Bm, g.sBn, g.sBk, g.sBb, g.N, g.Kc);
  // 128 x 128 tiles only when they still give every CU several workgroups
  // (one 4-wave workgroup per CU leaves one wave per SIMD to hide latency);
  // 32 x 64 tiles when 64 x 64 would leave CUs with fewer than two
  const long long tiles128 =
      (long long)((g.N + 127) / 128) * ((g.M + 127) / 128) * g.batch * g.ksplit;
  const long long tiles64 =
      (long long)((g.N + 63) / 64) * ((g.M + 63) / 64) * g.batch * g.ksplit;
  if (g.M >= 128 && g.N >= 128 && tiles128 >= 1024) {
    dim3 grid((g.N + 127) / 128, (g.M + 127) / 128, g.batch * g.ksplit);
    launch_gemm_tile<128, 128, BK>(grid, g, st);
  } else if (g.M > 32 && tiles64 < 512) {
    dim3 grid((g.N + 63) / 64, (g.M + 31) / 32, g.batch * g.ksplit);
    // fewer workgroups than CUs: latency-bound, 64-deep contraction blocks
    const long long wgs = (long long)grid.x * grid.y * grid.z;
    if (wgs < RID_GEMM_DEEP_WGS && g.kchunk >= 64)
      launch_gemm_tile<32, 64, 64>(grid, g, st);
    else
      launch_gemm_tile<32, 64, BK>(grid, g, st);
  } else {
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, g.batch * g.ksplit);
    launch_gemm_tile<64, 64, BK>(grid, g, st);
  }
  RID_HIP(hipGetLastError());
  return RID_OK;
}

rid_status wgrad(const WgradArgs& a, hipStream_t st) {
  // the kernel reads two rows per k-step inside each wave's range: chunks
  // and the contraction must hold whole k-steps
  if (a.kchunk % 2 != 0 || a.Kc % 2 != 0 || a.M < 1 || a.N < 1 || a.Kc < 1)
    return fail(RID_EINVAL, "weight-gradient GEMM: bad shape");
  // row byte offsets are 32-bit scalar offsets (passes are sized to fit)
  if ((long long)a.Kc * std::max(a.lda, a.ldb) * 4 > 0x7FFFFFFFLL)
    return fail(RID_EUNSUPPORTED, "weight-gradient GEMM: slab too large for 32-bit offsets");
  const dim3 grid((a.N + 63) / 64, (a.M + 63) / 64, a.batch * a.ksplit);
  hipLaunchKernelGGL(wgrad_kernel, grid, dim3(256), 0, st, a);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

// dW_l and db_l of one chunk of rows into the gradient (member k at
// G + k*pm, dW_l at w_off, db_l at b_off).  With one split and no earlier
// chunk to add to, the kernel writes the gradient itself; otherwise it
// writes one slab per split (part, bpart) and splitk_reduce_kernel adds them
// in split order, onto the gradient when accumulate is set.  The operands,
// shape and split of g are set by the caller.
rid_status wgrad_into_grad(WgradArgs g, float* part, float* bpart, float* G, long long pm,
                           long long w_off, long long b_off, bool accumulate, hipStream_t st) {
  rid_status rs;
  const long long mn = (long long)g.M * g.N;
  if (g.ksplit == 1 && !accumulate) {
    g.C = G + w_off; g.sCs = 0; g.sCb = pm;
    g.csum = G + b_off; g.csum_ss = 0; g.csum_sb = pm;
    return wgrad(g, st);
  }
  g.C = part; g.sCs = g.batch * mn; g.sCb = mn;
  g.csum = bpart; g.csum_ss = (long long)g.batch * g.M; g.csum_sb = g.M;
  if ((rs = wgrad(g, st)) != RID_OK) return rs;
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid1d(g.batch * (long long)g.M * (g.N + 1))),
                     dim3(256), 0, st, part, g.batch * mn, g.ksplit, g.M, g.N, g.batch, G, pm,
                     (int)w_off, accumulate ? 1 : 0, bpart, (int)b_off);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

// out[k][j] = sum_{b<B} X[k*slab + b*w + j] -> grad[k*per_model + dst_off + j]
// (+= when accumulate)
rid_status colsum(const float* X, long long slab, int B, int w, int K, float* part,
                  float* grad, long long per_model, int dst_off, bool accumulate,
                  hipStream_t st) {
  const int chunks = (B + kColRows - 1) / kColRows;
  hipLaunchKernelGGL(colsum_partial_kernel, dim3((w + 63) / 64, chunks, K), dim3(256), 0, st,
                     X, slab, B, w, part, K);
  RID_HIP(hipGetLastError());
  hipLaunchKernelGGL(colsum_final_kernel, dim3((K * w + 63) / 64), dim3(256), 0, st, part,
                     chunks, w, K, grad, per_model, dst_off, accumulate ? 1 : 0);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

// Rows per pass over the batch: all B when the pass's stored activations
// (floats_per_row floats a row) fit the budget, else equal chunks, each a
// multiple of 64 rows and at least 64, that do.  A pass also stays below
// the rows whose 2R-row slabs of width wmax the weight-gradient kernel can
// address with 32-bit byte offsets (about 500 k rows at width 512).
int chunk_rows(long long floats_per_row, int B, size_t budget, int wmax) {
  const long long cap = ((1LL << 31) - 1) / (8LL * std::max(wmax, 1));
  const long long fit =
      std::min(cap, (long long)(budget / (sizeof(float) * (size_t)floats_per_row)));
  if (fit >= B) return B;
  const long long step = std::max<long long>(64, fit / 64 * 64);
  const long long chunks = (B + step - 1) / step;
  return (int)std::min<long long>(step, (B + chunks - 1) / chunks + 63) / 64 * 64;
}

// Split of the 2R-row weight-gradient contraction of a pass of R rows:
// split-K slabs until the tiles times slabs reach RID_WG_TARGET workgroups
// (512: two per CU; more slabs cost more partial traffic than the extra
// workgroups gain -- measured 1024 +6 %, 256 +6 %, 128 +31 % per training
// step), each slab at least 256 rows.
#ifndef RID_WG_TARGET
#define RID_WG_TARGET 512
#endif
void wgrad_split(int K, int tiles_max, int R, int* ks, int* kchunk) {
  int s = 1;
  while (s < 64 && (long long)K * tiles_max * s < RID_WG_TARGET && 2LL * R / (s * 2) >= 256)
    s *= 2;
  *ks = s;
  *kchunk = round_up((2 * R + s - 1) / s, BK);
}

// The training step with the sweeps fused into one kernel (train_kernel):
// it writes [h ; hd] of every layer input and [lam_z ; lam_zd] of every
// layer, then the batch reductions run as before: dW_l = S_l^T [h ; hd]_{l-1}
// (split over the 2R rows), db_l = column sums of lam_z, dw_o = column sums
// of hd_L.  A batch larger than the training budget allows runs in chunks of
// Bc rows, in row order: each chunk's reductions are added to the gradient
// in chunk order, so the step stays deterministic, and only one chunk's
// activations are ever held.  Workspace regions are 256-byte aligned (the
// kernel stores float4).
rid_status mf_grad_fused(rid_ensemble_impl& e, const float* s, const float* F,
                         const float* rho, int B, float* loss, float* grad_out,
                         float** grad_used, hipStream_t st, const std::vector<int>& w,
                         const std::vector<long long>& w_off,
                         const std::vector<long long>& b_off, long long wo_off,
                         int tiles_max) {
  const int K = e.K, L = e.L, n = e.n_cv;
  int wmax = 0;
  for (int v : w) wmax = std::max(wmax, v);
  long long per_row = 0;
  for (int l = 0; l <= L; ++l) per_row += (long long)K * 2 * w[l] * (l > 0 ? 2 : 1);
  const int Bc = chunk_rows(per_row, B, e.train_budget, wmax);
  int ks_max, kc;
  wgrad_split(K, tiles_max, Bc, &ks_max, &kc);
  auto al = [](long long v) { return (v + 63) / 64 * 64; };
  std::vector<long long> hh(L + 1), sl(L);
  long long tot = 0;
  for (int l = 0; l <= L; ++l) {
    hh[l] = tot;
    tot = al(tot + (long long)K * 2 * Bc * w[l]);
  }
  for (int l = 1; l <= L; ++l) {
    sl[l - 1] = tot;
    tot = al(tot + (long long)K * 2 * Bc * w[l]);
  }
  long long part_slab = 0;
  for (int l = 0; l < L; ++l) part_slab = std::max(part_slab, (long long)K * w[l + 1] * w[l]);
  const long long part = tot; tot = al(tot + part_slab * ks_max);
  const long long grad = tot; tot = al(tot + (long long)e.n_params);
  const long long lrows = tot; tot = al(tot + (long long)K * B);
  const long long cpart = tot; tot = al(tot + (long long)((Bc + kColRows - 1) / kColRows) * K * wmax);
  const long long bpart = tot; tot = al(tot + (long long)ks_max * K * wmax);
  rid_status rs = e.ws_train.ensure(sizeof(float) * tot);
  if (rs != RID_OK) return rs;
  float* W = e.ws_train.as<float>();
  const long long pm = (long long)e.per_model;
  float* G = grad_out ? grad_out : W + grad;
  if (grad_used) *grad_used = G;
  ProfScope ps(kProfTrain, st);
  if (e.frag_dirty) {
    if ((rs = pack_ensemble_weights(e, st)) != RID_OK) return rs;
    e.frag_dirty = false;
  }
  TrainIo io{};
  io.loss_ld = B;
  io.B_norm = B;
  io.drop_p = e.drop_p;
  io.drop_seed = e.drop_seed;
  io.step = (uint32_t)((unsigned long long)e.step & 0xFFFFFFFFull);
  for (int l = 0; l <= L; ++l) io.hh[l] = W + hh[l];
  for (int l = 0; l < L; ++l) io.sl[l] = W + sl[l];
  for (int r0 = 0; r0 < B; r0 += Bc) {
    const int R = std::min(Bc, B - r0);
    const bool acc = r0 > 0;
    int ks, kchunk;
    wgrad_split(K, tiles_max, R, &ks, &kchunk);
    io.s = s + (size_t)r0 * n;
    io.F = rho ? nullptr : F + (size_t)r0 * n;
    io.rho = rho ? rho + (size_t)r0 * K * n : nullptr;
    io.loss_rows = rho ? nullptr : W + lrows + r0;
    io.row_base = r0;
    if ((rs = launch_train_sweeps(e, io, R, st)) != RID_OK) return rs;
    for (int l = L; l >= 1; --l) {
      // dW_l = S^T [h ; hd]_{l-1} (contraction over the 2R stacked rows);
      // db_l = sum over the primal rows of lam_z, in the same pass
      WgradArgs g{};
      g.A = W + sl[l - 1]; g.sAb = 2LL * R * w[l]; g.lda = w[l];
      g.B = W + hh[l - 1]; g.sBb = 2LL * R * w[l - 1]; g.ldb = w[l - 1];
      g.csum_rows = R;
      g.M = w[l]; g.N = w[l - 1]; g.Kc = 2 * R; g.batch = K; g.ksplit = ks; g.kchunk = kchunk;
      if ((rs = wgrad_into_grad(g, W + part, W + bpart, G, pm, w_off[l - 1], b_off[l - 1], acc,
                                st)) != RID_OK)
        return rs;
    }
    if ((rs = colsum(W + hh[L] + (long long)R * w[L], 2LL * R * w[L], R, w[L], K, W + cpart,
                     G, pm, (int)wo_off, acc, st)) != RID_OK)
      return rs;
  }
  hipLaunchKernelGGL(train_finish_kernel, dim3(K), dim3(256), 0, st,
                     rho ? nullptr : W + lrows, B, loss, G, pm, (int)(wo_off + w[L]));
  RID_HIP(hipGetLastError());
  return RID_OK;
}

}  // namespace

// Gradient in the packed parameter layout of
//   F given:   L = sum_k (1/B) sum_b |g_k(s_b) - F_b|^2      (loss[k] written)
//   rho given: J = sum_k sum_b rho[b][k] . g_k(s_b)
// into grad_out (or the workspace's gradient slot when grad_out is null).
// Returns the gradient pointer through *grad_used.  Both forms hold at most
// the ensemble's training budget of activations: a larger batch is taken in
// chunks of rows whose weight-gradient contributions are added in chunk order.
// The aligned weight copy of the general sweeps, allocated on first use and
// refreshed when the masters have changed since it was made.
rid_status ensure_wpad(rid_ensemble_impl& e, const std::vector<int>& w,
                       const std::vector<long long>& w_off, hipStream_t st) {
  const int L = e.L;
  e.wpad_off.assign(L, 0);
  long long off = 0;
  for (int l = 0; l < L; ++l) {
    e.wpad_off[l] = off;
    off += ((long long)w[l + 1] * w[l] + 3) / 4 * 4;
  }
  e.wpad_pm = off;
  const void* before = e.wpad.ptr;
  rid_status rs = e.wpad.ensure(sizeof(float) * (size_t)e.K * e.wpad_pm);
  if (rs != RID_OK) return rs;
  if (e.wpad.ptr != before) e.wpad_gen = 0;    // a new buffer holds nothing yet
  if (e.wpad_gen == e.master_gen) return RID_OK;
  WpadCopy c{};
  c.L = L;
  long long cmax = 1;
  for (int l = 0; l < L; ++l) {
    c.src[l] = w_off[l];
    c.dst[l] = e.wpad_off[l];
    c.cnt[l] = (long long)w[l + 1] * w[l];
    cmax = std::max(cmax, c.cnt[l]);
  }
  const unsigned bx = (unsigned)std::min<long long>((cmax + 255) / 256, 256);
  hipLaunchKernelGGL(wpad_copy_kernel, dim3(bx, e.K * L), dim3(256), 0, st, e.d_master,
                     (long long)e.per_model, e.wpad.as<float>(), e.wpad_pm, c);
  RID_HIP(hipGetLastError());
  e.wpad_gen = e.master_gen;
  return RID_OK;
}

rid_status launch_mf_grad(rid_ensemble_impl& e, const float* s, const float* F,
                          const float* rho, int B, float* loss, float* grad_out,
                          float** grad_used, hipStream_t st, InputHvp* hvp) {
  // input mode (hvp != null, rho given): the same primal, tangent and
  // adjoint sweeps, but the adjoint runs down to the input instead of
  // forming weight gradients
  const bool input_mode = hvp != nullptr;
  if (input_mode && !rho) return fail(RID_EINVAL, "input mode needs an upstream gradient");
  const int K = e.K, L = e.L, n = e.n_cv, X = 2 * n;
  std::vector<int> w(L + 1);
  w[0] = X;
  for (int l = 0; l < L; ++l) w[l + 1] = e.widths[l];
  int wmax = X;
  for (int v : w) wmax = std::max(wmax, v);
  // packed offsets inside one model's block
  std::vector<long long> w_off(L), b_off(L);
  long long off = 0;
  for (int l = 0; l < L; ++l) {
    w_off[l] = off;
    off += (long long)w[l + 1] * w[l];
    b_off[l] = off;
    off += w[l + 1];
  }
  const long long wo_off = off;
  const long long pm = (long long)e.per_model;
  int tiles_max = 0;
  for (int l = 0; l < L; ++l)
    tiles_max = std::max(tiles_max, ((w[l + 1] + BM - 1) / BM) * ((w[l] + BN - 1) / BN));

  if (!input_mode && train_fused_supported(e))
    return mf_grad_fused(e, s, F, rho, B, loss, grad_out, grad_used, st, w, w_off, b_off,
                         wo_off, tiles_max);

  // the general form: residual layers, dropout (training only), raw CVs
  const bool res = e.resnet;
  const float drop_p = input_mode ? 0.f : e.drop_p;
  const float drop_inv = drop_p > 0.f ? 1.f / (1.f - drop_p) : 1.f;
  const uint8_t* raw = e.raw.empty() ? nullptr : e.d_raw;
  auto skip = [&](int l) { return res && l >= 2; };   // layer l (1-based) adds its input

  // rows per pass (input mode hands per-row results back: one pass)
  long long per_row = (long long)K * (8 + (res ? 2 : 0)) * wmax;
  for (int l = 0; l <= L; ++l) per_row += (long long)K * w[l] * (l > 0 ? 5 : 2);
  const int Bc = input_mode ? B : chunk_rows(per_row, B, e.train_budget, wmax);
  int ks_max, kc;
  wgrad_split(K, tiles_max, Bc, &ks_max, &kc);

  // workspace (floats), sized for Bc rows; a pass of R <= Bc rows uses the
  // same regions with R-row strides
  std::vector<long long> hh(L + 1), zd(L + 1), tt(L + 1), dd(L + 1);
  long long tot = 0;
  for (int l = 0; l <= L; ++l) {
    hh[l] = tot;
    tot += (long long)K * 2 * Bc * w[l];
  }
  for (int l = 1; l <= L; ++l) {
    zd[l] = tot; tot += (long long)K * Bc * w[l];
    tt[l] = tot; tot += (long long)K * Bc * w[l];
    dd[l] = tot; tot += (long long)K * Bc * w[l];
  }
  const long long vA = tot; tot += (long long)K * Bc * wmax;
  const long long vB = tot; tot += (long long)K * Bc * wmax;
  const long long uA = tot; tot += res ? (long long)K * Bc * wmax : 0;
  const long long uB = tot; tot += res ? (long long)K * Bc * wmax : 0;
  const long long lamA = tot; tot += (long long)K * 2 * Bc * wmax;
  const long long lamB = tot; tot += (long long)K * 2 * Bc * wmax;
  const long long sbuf = tot; tot += (long long)K * 2 * Bc * wmax;
  long long part_slab = 0;
  for (int l = 0; l < L; ++l) part_slab = std::max(part_slab, (long long)K * w[l + 1] * w[l]);
  const long long part = tot; tot += part_slab * ks_max;
  const long long grad = tot; tot += (long long)e.n_params;
  const long long lrows = tot; tot += (long long)K * B;
  const long long cpart = tot; tot += (long long)((Bc + kColRows - 1) / kColRows) * K * wmax;
  const long long bpart = tot; tot += (long long)ks_max * K * wmax;
  rid_status rs = e.ws_train.ensure(sizeof(float) * tot);
  if (rs != RID_OK) return rs;
  float* W = e.ws_train.as<float>();
  float* P = e.d_master;
  float* G = grad_out ? grad_out : W + grad;
  if (grad_used) *grad_used = G;
  ProfScope ps(kProfTrain, st);
  const uint32_t step32 = (uint32_t)((unsigned long long)e.step & 0xFFFFFFFFull);
  // the weight operands come from the aligned copy (float4 loads)
  if ((rs = ensure_wpad(e, w, w_off, st)) != RID_OK) return rs;
  const float* WP = e.wpad.as<float>();
  const long long pmp = e.wpad_pm;
  const std::vector<long long>& wq = e.wpad_off;

  for (int r0 = 0; r0 < B; r0 += Bc) {
    const int R = std::min(Bc, B - r0);
    const bool acc = r0 > 0;
    int ks, kchunk;
    wgrad_split(K, tiles_max, R, &ks, &kchunk);
    const float* sR = s + (size_t)r0 * n;
    const float* FR = rho ? nullptr : F + (size_t)r0 * n;
    const float* rhoR = rho ? rho + (size_t)r0 * K * n : nullptr;
    auto slab = [&](int l) { return 2LL * R * w[l]; };
    // ---- primal forward: t_l = tanh(W_l h_{l-1} + b_l), then h_l and d_l ----
    hipLaunchKernelGGL(train_embed_kernel, dim3(grid1d((long long)K * R * n)), dim3(256), 0,
                       st, sR, R, n, K, raw, W + hh[0], slab(0));
    RID_HIP(hipGetLastError());
    for (int l = 1; l <= L; ++l) {
      GemmArgs g{};
      g.A = W + hh[l - 1]; g.sAb = slab(l - 1); g.sAm = w[l - 1]; g.sAk = 1;
      g.Bm = WP + wq[l - 1]; g.sBb = pmp; g.sBk = 1; g.sBn = w[l - 1];
      g.C = W + tt[l]; g.sCb = (long long)R * w[l]; g.sCm = w[l]; g.sCn = 1;
      g.bias = P + b_off[l - 1]; g.sBiasb = pm;
      g.M = R; g.N = w[l]; g.Kc = w[l - 1]; g.batch = K; g.mode = EPI_BIAS_TANH;
      if ((rs = gemm(g, st)) != RID_OK) return rs;
      hipLaunchKernelGGL(act_kernel, dim3(grid1d((long long)K * R * ((w[l] + 3) / 4))),
                         dim3(256), 0, st, W + tt[l], l, w[l], R, K, r0, drop_p, drop_inv,
                         e.drop_seed, step32, skip(l) ? W + hh[l - 1] : nullptr, slab(l - 1),
                         W + hh[l], slab(l), W + dd[l]);
      RID_HIP(hipGetLastError());
    }
    // ---- primal backward to u0: v_l = u_l d_l, u_{l-1} = W_l^T v_l (+ u_l) ----
    hipLaunchKernelGGL(vlast_kernel, dim3(grid1d((long long)K * R * w[L])), dim3(256), 0, st,
                       W + dd[L], P, pm, (int)wo_off, w[L], R, K, W + vA);
    RID_HIP(hipGetLastError());
    long long uin = uA, uout = uB;
    if (res) {   // u_L = w_o
      hipLaunchKernelGGL(top_kernel, dim3(grid1d((long long)K * R * w[L])), dim3(256), 0, st,
                         P, pm, (int)wo_off, w[L], R, K, R, 0, W + uin);
      RID_HIP(hipGetLastError());
    }
    long long vin = vA, vout = vB;
    for (int l = L; l >= 1; --l) {
      GemmArgs g{};
      g.A = W + vin; g.sAb = (long long)R * w[l]; g.sAm = w[l]; g.sAk = 1;
      g.Bm = WP + wq[l - 1]; g.sBb = pmp; g.sBk = w[l - 1]; g.sBn = 1;
      g.sCb = (long long)R * w[l - 1]; g.sCm = w[l - 1]; g.sCn = 1;
      g.M = R; g.N = w[l - 1]; g.Kc = w[l]; g.batch = K;
      if (l > 1) {
        // v_{l-1} = (W_l^T v_l (+ u_l)) d_{l-1}; with a skip u_{l-1} is kept
        g.mode = EPI_GEN;
        g.C = skip(l) ? W + uout : nullptr;
        g.add = skip(l) ? W + uin : nullptr; g.sAddb = (long long)R * w[l];
        g.C2 = W + vout; g.sC2b = (long long)R * w[l - 1];
        g.mul = W + dd[l - 1]; g.sMulb = (long long)R * w[l - 1];
      } else {
        g.mode = EPI_STORE;
        g.C = W + vout;
      }
      if ((rs = gemm(g, st)) != RID_OK) return rs;
      std::swap(vin, vout);
      if (skip(l)) std::swap(uin, uout);
    }
    // vin now holds u0 [K][R][2n]
    hipLaunchKernelGGL(residual_kernel,
                       dim3((unsigned)(((long long)K * R + kResWaves - 1) / kResWaves)),
                       dim3(kResWaves * 64), 0, st,
                       sR, FR, rhoR, W + vin, R, B, n, K, raw, W + hh[0], slab(0),
                       rho ? nullptr : W + lrows + r0, (long long)B);
    RID_HIP(hipGetLastError());
    // ---- tangent forward: zd_l = W_l hd_{l-1}, hd_l = d_l zd_l (+ hd_{l-1}) ----
    for (int l = 1; l <= L; ++l) {
      GemmArgs g{};
      g.A = W + hh[l - 1] + (long long)R * w[l - 1]; g.sAb = slab(l - 1); g.sAm = w[l - 1];
      g.sAk = 1;
      g.Bm = WP + wq[l - 1]; g.sBb = pmp; g.sBk = 1; g.sBn = w[l - 1];
      g.C = W + zd[l]; g.sCb = (long long)R * w[l]; g.sCm = w[l]; g.sCn = 1;
      g.C2 = W + hh[l] + (long long)R * w[l]; g.sC2b = slab(l);
      g.mul = W + dd[l]; g.sMulb = (long long)R * w[l];
      if (skip(l)) {
        g.add2 = W + hh[l - 1] + (long long)R * w[l - 1];
        g.sAdd2b = slab(l - 1);
      }
      g.M = R; g.N = w[l]; g.Kc = w[l - 1]; g.batch = K; g.mode = EPI_GEN;
      if ((rs = gemm(g, st)) != RID_OK) return rs;
    }
    // ---- adjoint sweep with weight gradients (or down to the input) ----
    long long lin = lamA, lout = lamB;
    // top: lam_h_L = 0, lam_hd_L = w_o (stacked rows [0, R) and [R, 2R))
    hipLaunchKernelGGL(top_kernel, dim3(grid1d((long long)K * 2 * R * w[L])), dim3(256), 0, st,
                       P, pm, (int)wo_off, w[L], R, K, 2 * R, R, W + lin);
    RID_HIP(hipGetLastError());
    for (int l = L; l >= 1; --l) {
      hipLaunchKernelGGL(adjoint_kernel, dim3(grid1d((long long)K * R * w[l])), dim3(256), 0,
                         st, W + tt[l], W + dd[l], W + zd[l], W + lin, 2LL * R * w[l], w[l], R,
                         K, W + sbuf, 2LL * R * w[l]);
      RID_HIP(hipGetLastError());
      // dW_l = S^T [h_{l-1}; hd_{l-1}]  (contraction over 2R rows, split)
      if (!input_mode) {
        WgradArgs g{};
        g.A = W + sbuf; g.sAb = 2LL * R * w[l]; g.lda = w[l];
        g.B = W + hh[l - 1]; g.sBb = slab(l - 1); g.ldb = w[l - 1];
        // db_l = sum over the primal rows of lam_z, in the same pass
        g.csum_rows = R;
        g.M = w[l]; g.N = w[l - 1]; g.Kc = 2 * R; g.batch = K; g.ksplit = ks;
        g.kchunk = kchunk;
        if ((rs = wgrad_into_grad(g, W + part, W + bpart, G, pm, w_off[l - 1], b_off[l - 1],
                                  acc, st)) != RID_OK)
          return rs;
      }
      if (l > 1 || input_mode) {
        // [lam_h ; lam_hd]_{l-1} = [lam_z ; lam_zd] W_l (+ [lam_h ; lam_hd]_l)
        GemmArgs g{};
        g.A = W + sbuf; g.sAb = 2LL * R * w[l]; g.sAm = w[l]; g.sAk = 1;
        g.Bm = WP + wq[l - 1]; g.sBb = pmp; g.sBk = w[l - 1]; g.sBn = 1;
        g.C = W + lout; g.sCb = 2LL * R * w[l - 1]; g.sCm = w[l - 1]; g.sCn = 1;
        g.M = 2 * R; g.N = w[l - 1]; g.Kc = w[l]; g.batch = K;
        if (skip(l)) {
          g.mode = EPI_GEN;
          g.add = W + lin; g.sAddb = 2LL * R * w[l];
        } else {
          g.mode = EPI_STORE;
        }
        if ((rs = gemm(g, st)) != RID_OK) return rs;
        std::swap(lin, lout);
      }
    }
    if (input_mode) {
      // lin: [lam_h0 ; lam_hd0] per member (rows [0, B): d J / dx); vin: u0
      hvp->lam_x = W + lin;
      hvp->u0 = W + vin;
      hvp->slab_lam = 2LL * B * X;
      return RID_OK;
    }
    // dw_o = sum_b hd_L
    if ((rs = colsum(W + hh[L] + (long long)R * w[L], slab(L), R, w[L], K, W + cpart, G, pm,
                     (int)wo_off, acc, st)) != RID_OK)
      return rs;
  }
  // the loss, and db_o = 0 (the output bias never reaches grad_s A)
  hipLaunchKernelGGL(train_finish_kernel, dim3(K), dim3(256), 0, st,
                     rho ? nullptr : W + lrows, B, loss, G, pm, (int)(wo_off + w[L]));
  RID_HIP(hipGetLastError());
  return RID_OK;
}

rid_status launch_train_step(rid_ensemble_impl& e, const float* s, const float* F,
                             int B, float lr, float* loss, hipStream_t st) {
  float* G = nullptr;
  rid_status rs = launch_mf_grad(e, s, F, nullptr, B, loss, nullptr, &G, st);
  if (rs != RID_OK) return rs;
  // ---- Adam ----
  const int t = (int)(e.step + 1);
  const float c1 = 1.f - std::pow(0.9f, (float)t);
  const float c2 = 1.f - std::pow(0.999f, (float)t);
  ProfScope ps(kProfTrain, st);
  hipLaunchKernelGGL(adam_kernel, dim3(grid1d((long long)e.n_params)), dim3(256), 0, st,
                     e.d_master, e.d_m, e.d_v, G, (long long)e.n_params, lr, c1, c2);
  RID_HIP(hipGetLastError());
  e.step += 1;
  e.frag_dirty = true;
  ++e.master_gen;
  return RID_OK;
}

}  // namespace rid
