// Ensemble MLP free-energy models: the fused forward + input-gradient kernel
// (fed straight from atom positions on the bias path) and the weight packer.
//
// Method ("Training phase"): each ensemble member is an MLP with tanh hidden
// layers and a scalar output A(x); the bias needs the mean force
// g = dA/ds (Box 2), obtained by one reverse sweep through the same layers.
// x = [cos s | sin s].
//
// Kernel design (gfx950):
//  * One workgroup owns R = 16*RT walkers of ONE member.  Its waves split the
//    hidden units; each wave streams its units' weight fragments straight
//    from L2 into VGPRs (no weight reuse inside a workgroup, so no LDS hop)
//    with buffer loads whose k-chunk offset sits in a scalar register.  The
//    loads run a few k-steps ahead of the MFMAs through a register ring that
//    scheduling barriers keep in order, and continue across layers (weights
//    do not depend on activations).  The weights are the MFMA A operand and
//    the activations the B operand, so each lane ends up holding 4
//    consecutive units of one walker: one packed LDS store per 4 outputs,
//    and the bias enters as the accumulator's initial value.
//  * The activation tile (shared by all waves) lives in LDS, ping-ponged
//    between two buffers so each layer needs one barrier; it holds x, then
//    h_1 .. h_L, then the reverse-sweep vectors v_l.
//  * tanh'(z_l) = 1 - h_l^2 is computed in FP32 and kept in VGPRs for the
//    reverse sweep (FP32 for the FP32 path; FP16 for the 16-bit plans except
//    the all-BF16 one, whose 64-walker tiles would not fit an FP32 copy):
//    nothing goes to HBM between layers.
//  * 16-bit arithmetic plans (Plan below) choose the operand format of the
//    first layer, of the hidden-layer forward GEMMs and of the reverse sweep
//    separately.  The precision form runs the hidden-layer forward GEMMs in
//    BF16 and the first layer and the reverse sweep in FP16 (same MFMA rate):
//    the mean force is linear in the reverse sweep's roundings but sees the
//    forward sweep's only through tanh', so the reverse sweep's operand
//    format sets most of the force error.  The reverse vectors carry a
//    per-member power-of-two scale (exact) that keeps them inside FP16's
//    range.
//  * Forward weights and biases are stored pre-multiplied by 2/ln 2, so the
//    epilogue evaluates tanh from exp2 of the GEMM output and one reciprocal.
//  * Blocks are mapped XCD-aware: when K divides 8, member k runs on XCDs
//    {k*8/K, ...}, so each XCD's L2 holds only its members' weights.
//  * On the bias path each workgroup can compute the torsions of its walkers
//    itself from the positions (small batches: the encoding never goes
//    through HBM; large batches encode once in a separate kernel).  The
//    FP64 deviation, switch and chain rule run in a second kernel: handing
//    the members' results to one workgroup inside this launch needs
//    device-scope fences, which on gfx950 write back and invalidate the
//    whole per-XCD L2 and so evict the weights the other workgroups stream.
#include <type_traits>

#include "device_common.h"

namespace rid {
namespace {

using namespace dev;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

struct F32 {
  using T = float;
  static constexpr int KF = 16;
  // a: 16 rows x 16 contraction, b: 16 contraction x 16 columns (4 steps)
  __device__ static inline void mma(const uint4& a, const uint4& b, f4& c) {
    f4 av = __builtin_bit_cast(f4, a);
    f4 bv = __builtin_bit_cast(f4, b);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0], bv[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1], bv[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2], bv[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(av[3], bv[3], c, 0, 0, 0);
  }
  __device__ static inline T from_float(float v) { return v; }
};

struct BF16 {
  using T = __bf16;
  static constexpr int KF = 32;
  __device__ static inline void mma(const uint4& a, const uint4& b, f4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                __builtin_bit_cast(bf8, b), c,
                                                0, 0, 0);
  }
  __device__ static inline T from_float(float v) { return (__bf16)v; }
};

struct F16 {
  using T = _Float16;
  static constexpr int KF = 32;
  __device__ static inline void mma(const uint4& a, const uint4& b, f4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a),
                                               __builtin_bit_cast(h8, b), c,
                                               0, 0, 0);
  }
  __device__ static inline T from_float(float v) { return (_Float16)v; }
};

// Arithmetic plan of the MLP kernel: MFMA operand format of the first layer
// (P1), of the hidden-layer forward GEMMs (PH) and of the reverse sweep (PB),
// and the storage type of tanh' between the sweeps (S).  The formats of one
// plan share an element size, so the activation tile's layout is the same
// for every layer.
template <class P1_, class PH_, class PB_, class S_>
struct Plan {
  using P1 = P1_;
  using PH = PH_;
  using PB = PB_;
  using S = S_;
};
using PlanF32 = Plan<F32, F32, F32, float>;
using PlanBF16 = Plan<F16, BF16, F16, _Float16>;      // the BF16 precision form
using PlanF16 = Plan<F16, F16, F16, _Float16>;
using PlanBF16All = Plan<BF16, BF16, BF16, __bf16>;   // every operand BF16

// Four consecutive elements of type T as one register group.
template <class T> struct Pack4;
template <> struct Pack4<float> {
  f4 v;
  __device__ inline void set(const f4& x) { v = x; }
  __device__ inline f4 get() const { return v; }
  __device__ inline void store(float* dst) const { *reinterpret_cast<f4*>(dst) = v; }
};
template <class H> struct Pack16 {
  typedef H h2 __attribute__((ext_vector_type(2)));
  typedef float fl2 __attribute__((ext_vector_type(2)));
  uint2 v;
  // two packed round-to-nearest-even conversions (v_cvt_pk_*_f32)
  __device__ inline void set(const f4& x) {
    v.x = __builtin_bit_cast(uint32_t, __builtin_convertvector((fl2{x[0], x[1]}), h2));
    v.y = __builtin_bit_cast(uint32_t, __builtin_convertvector((fl2{x[2], x[3]}), h2));
  }
  __device__ inline f4 get() const {
    f4 r;
    r[0] = (float)__builtin_bit_cast(H, (unsigned short)(v.x & 0xffffu));
    r[1] = (float)__builtin_bit_cast(H, (unsigned short)(v.x >> 16));
    r[2] = (float)__builtin_bit_cast(H, (unsigned short)(v.y & 0xffffu));
    r[3] = (float)__builtin_bit_cast(H, (unsigned short)(v.y >> 16));
    return r;
  }
  __device__ inline void store(H* dst) const { *reinterpret_cast<uint2*>(dst) = v; }
};
template <> struct Pack4<__bf16> : Pack16<__bf16> {};

// two consecutive elements of type T (one 4- or 8-byte LDS store)
template <class T> struct Pack2 {
  typedef T t2 __attribute__((ext_vector_type(2)));
  typedef float fl2 __attribute__((ext_vector_type(2)));
  __device__ static inline void store(T* dst, float a, float b) {
    *reinterpret_cast<t2*>(dst) = __builtin_convertvector((fl2{a, b}), t2);
  }
};
template <> struct Pack2<float> {
  __device__ static inline void store(float* dst, float a, float b) {
    *reinterpret_cast<float2*>(dst) = make_float2(a, b);
  }
};
template <> struct Pack4<_Float16> : Pack16<_Float16> {};

// Forward weights and biases are stored multiplied by 2/ln 2, so a forward
// GEMM yields y = 2 z / ln 2 and exp(2z) = 2^y takes no multiply.
constexpr float kTanhPrescale = 2.8853900817779268f;

// tanh and its derivative from one exponential and one reciprocal, given the
// pre-scaled pre-activation y: with r = 1 / (1 + 2^y):  tanh z = 1 - 2r,
// 1 - tanh^2 z = (1 - h)(1 + h).  Saturates cleanly (2^y -> inf gives r = 0;
// 2^y -> 0 gives r = 1).  Absolute error of a few 1e-7, below the FP32
// rounding of the GEMM that feeds it.
__device__ inline float tanh_and_grad(float y, float& d) {
  const float e = __builtin_amdgcn_exp2f(y);
  const float r = __builtin_amdgcn_rcpf(1.f + e);
  const float h = __builtin_fmaf(-2.f, r, 1.f);
  d = __builtin_fmaf(-h, h, 1.f);
  return h;
}

struct MlpArgs {
  const float* x;      // [B][2n] input encoding (plain kernel)
  int B, n, K, L, XP, n_tiles, xcd_grp;
  const unsigned char* frag;
  unsigned long long frag_model_bytes;
  unsigned fwd_off[kMaxHidden];
  unsigned bwd_off[kMaxHidden];
  const float* bias;   // [K][L][NP]
  const float* wo;     // [K][NP]
  const float* bo;     // [K]
  const float* vscale; // [K][2] power-of-two scale folded into wo and its inverse
  float* A_out;        // [K][B]
  float* g_out;        // [K][B][n]
  // LDS layout (byte offsets; activation buffer 0 starts at 0)
  unsigned off_u0, off_red, off_xs, off_ph0, off_wo;
  int u0p;             // parts of the input-gradient contraction (u0_split or 1)
  int rc;              // walkers per torsion-gather pass (bias path)
  // torsion input (bias path)
  SysView sv;
  const float* pos;    // [B][n_atoms][3]
  // encoding input: CVs with raw[i] = 1 are non-angular, encoded (s_i, 0),
  // so dA/ds_i = dA/dx_i (null: every CV angular)
  const uint8_t* raw;
};

__device__ inline void map_block(int b, int K, int grp, int& k, int& tile) {
  if (grp > 0) {
    int x = b & 7;
    k = x / grp;
    tile = (b >> 3) * grp + (x % grp);
  } else {
    k = b % K;
    tile = b / K;
  }
}

// acc[rt][c] += W(units of tile jt0 + c, 0:KL) * act(walkers of rt, 0:KL)^T
// (output tile: 16 units x 16 walkers; lane holds units 4(lane/16)+q of
// walker lane%16)
// Software pipeline: weight fragments (from L2/HBM) are loaded PD k-steps
// ahead through a ring of PD+1 register slots; activation fragments (LDS)
// either one k-step ahead through two slots (ADB) or next to their use.
// Scheduling barriers pin "issue next loads -> MFMAs of this step", so the
// compiler cannot sink a global load next to its first use and expose the
// memory latency; without ADB they let LDS reads and ALU work move freely.
#ifndef RID_PD_FP32
#define RID_PD_FP32 2
#endif
#ifndef RID_PD_16
#define RID_PD_16 1
#endif
#ifndef RID_ADB_FP32
#define RID_ADB_FP32 1
#endif
#ifndef RID_ADB_16
#define RID_ADB_16 1
#endif
#ifndef RID_SCHED
#define RID_SCHED 1
#endif
template <bool ALL>
__device__ inline void sched_fence() {
#if RID_SCHED
  // mask: instruction classes allowed to cross (ALU, VALU, SALU, MFMA, DS,
  // transcendental) -- everything except vector-memory loads and stores
  __builtin_amdgcn_sched_barrier(ALL ? 0 : 0x078F);
#endif
}

// Activation rows are padded by this many bytes (bank spread of the
// row-strided LDS accesses).
#ifndef RID_ACT_PAD_BYTES
#define RID_ACT_PAD_BYTES 16
#endif

// Hidden-layer GEMMs: passes over the contraction and weight pipeline depth
// (PD+1 must divide passes * k-steps: 1 or 3).
#ifndef RID_NPASS_FP32
#define RID_NPASS_FP32 1
#endif
#ifndef RID_NPASS_16
#define RID_NPASS_16 1
#endif
#ifndef RID_PDH_FP32
#define RID_PDH_FP32 3
#endif
#ifndef RID_PDH_16
#define RID_PDH_16 1
#endif

// Where a wave's weight fragments come from: a buffer resource over one
// member's fragments (range-checked by the hardware), the byte offset of
// k-chunk 0 of the wave's first unit tile, and the bytes per k-chunk.  A
// load is one buffer_load_dwordx4 with the lane's 16 bytes as the only
// vector offset; the k-chunk goes into the scalar offset and the tile into
// the instruction's immediate, so no vector registers hold addresses.
struct WSrc {
  __amdgpu_buffer_rsrc_t r;
  int soff, kstride;
  __device__ inline uint4 ld(int kk, int c, int lane) const {
    return __builtin_bit_cast(
        uint4, __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16 + c * kFragBytes,
                                                     soff + kk * kstride, 0));
  }
  __device__ inline WSrc tiles_from(int c) const {
    return WSrc{r, soff + c * kFragBytes, kstride};
  }
};

// Weight ring: slot kt % (PD+1) holds the fragments of k-step kt.
template <int PD, int CT>
struct WRing {
  uint4 w[PD + 1][CT];
};

// Issue the loads of k-steps 0..PD-1 of a layer into the ring.
template <int PD, int CT>
__device__ inline void ring_preload(WRing<PD, CT>& wr, const WSrc& src, int n_kt, int lane) {
#pragma unroll
  for (int s = 0; s < PD; ++s)
    if (s < n_kt)
#pragma unroll
      for (int c = 0; c < CT; ++c) wr.w[s][c] = src.ld(s, c, lane);
}

// The k-loop of a GEMM with a run-time contraction length (first layer,
// input-gradient GEMM).  On entry the ring holds the first PD k-steps; the
// following ones are issued PD steps ahead.
template <class P, int RT, int CT, int PD>
__device__ inline void gemm_run(f4 (&acc)[RT][CT], WRing<PD, CT>& wr,
                                const typename P::T* act, int as, const WSrc& src, int n_kt,
                                int lane) {
  constexpr int KF = P::KF;
  constexpr bool WIDE = sizeof(typename P::T) == 4;
  constexpr bool ADB = WIDE ? RID_ADB_FP32 : RID_ADB_16;
  constexpr int S = PD + 1;
  constexpr int U = (S % 2) ? 2 * S : S;      // unroll: static ring indices
  const int r = lane & 15, g = lane >> 4;
  const typename P::T* arow = act + r * as + g * (KF / 4);
  uint4 a[ADB ? 2 : 1][RT];
  if (ADB && n_kt > 0)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
      a[0][rt] = *reinterpret_cast<const uint4*>(arow + rt * 16 * as);
  for (int kb = 0; kb < n_kt; kb += U) {
#pragma unroll
    for (int i = 0; i < U; ++i) {
      const int kt = kb + i;
      if (kt < n_kt) {
        const int kp = kt + PD;
        if (kp < n_kt)
#pragma unroll
          for (int c = 0; c < CT; ++c)
            wr.w[(i + PD) % S][c] = src.ld(kp, c, lane);
        if (ADB && kt + 1 < n_kt)
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
            a[(i + 1) % 2][rt] =
                *reinterpret_cast<const uint4*>(arow + rt * 16 * as + (kt + 1) * KF);
        sched_fence<ADB>();
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          const uint4 av = ADB ? a[i % 2][rt]
                               : *reinterpret_cast<const uint4*>(arow + rt * 16 * as + kt * KF);
#pragma unroll
          for (int c = 0; c < CT; ++c) P::mma(wr.w[i % S][c], av, acc[rt][c]);
        }
        sched_fence<ADB>();
      }
    }
  }
}

template <class P, int RT, int CT, int PD>
__device__ inline void gemm_tiles(f4 (&acc)[RT][CT], const typename P::T* act, int as,
                                  const WSrc& src, int n_kt, int lane) {
  WRing<PD, CT> wr;
  ring_preload<PD, CT>(wr, src, n_kt, lane);
  gemm_run<P, RT, CT, PD>(acc, wr, act, as, src, n_kt, lane);
}

// Hidden-layer GEMM (contraction length NK k-steps, known at compile time),
// in NPASS passes over the contraction, each computing CT/NPASS of the
// wave's unit tiles (two passes halve the weight registers per k-step at
// the price of reading the activations from LDS once per pass).  The
// weight ring streams all passes as one sequence of NPASS*NK steps, and
// after the last MFMA it already issues the next layer's first PD steps
// (weights do not depend on activations), so a layer starts with its
// weights in flight through the previous epilogue and barrier.  Slot
// numbering stays step % S across layers because S divides NPASS*NK.
template <class P, int RT, int CT, int NPASS, int PD, int NK>
__device__ inline void gemm_hidden(f4 (&acc)[RT][CT], WRing<PD, CT / NPASS>& wr,
                                   const typename P::T* act, int as, const WSrc& src,
                                   bool has_next, const WSrc& next, int lane) {
  constexpr int KF = P::KF;
  constexpr int S = PD + 1;
  constexpr int CH = CT / NPASS;
  constexpr int NV = NPASS * NK;
  static_assert(CH * NPASS == CT && NV % S == 0, "ring slots must line up across layers");
  const int r = lane & 15, g = lane >> 4;
  const typename P::T* arow = act + r * as + g * (KF / 4);
  uint4 a[2][RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) a[0][rt] = *reinterpret_cast<const uint4*>(arow + rt * 16 * as);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int vp = v + PD;                     // weight step issued now
    if (vp < NV) {
#pragma unroll
      for (int c = 0; c < CH; ++c) wr.w[vp % S][c] = src.ld(vp % NK, (vp / NK) * CH + c, lane);
    } else if (has_next) {
#pragma unroll
      for (int c = 0; c < CH; ++c) wr.w[vp % S][c] = next.ld(vp - NV, c, lane);
    }
    if (v + 1 < NV) {
      const int kn = (v + 1) % NK;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        a[(v + 1) % 2][rt] = *reinterpret_cast<const uint4*>(arow + rt * 16 * as + kn * KF);
    }
    sched_fence<true>();
    const int cb = (v / NK) * CH;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int c = 0; c < CH; ++c) P::mma(wr.w[v % S][c], a[v % 2][rt], acc[rt][cb + c]);
    sched_fence<true>();
  }
}

// Parts the input-gradient GEMM's contraction is cut into: 4 for FP32 (it
// divides the NP/16 k-steps of every padded width); the 16-bit kernels keep
// one (their tiles are 4x wider, and the partials would cost registers).
template <class P, int NP>
__host__ __device__ constexpr int u0_split() {
  return sizeof(typename P::T) == 4 ? 4 : 1;
}

// GRAD = false: the free energies only (the forward sweep, no tanh' stash,
// no reverse sweep, no g output).
template <class PL, int NP, int RT, int NW, int LM, bool FROM_POS, bool GRAD, bool RES>
__global__ __launch_bounds__(NW * 64) void mlp_kernel(MlpArgs p) {
  using P = typename PL::PH;         // hidden-layer forward GEMMs
  using P1 = typename PL::P1;        // first layer
  using PB = typename PL::PB;        // reverse sweep
  using T = typename P::T;
  using T1 = typename P1::T;
  using TB = typename PB::T;
  static_assert(sizeof(T1) == sizeof(T) && sizeof(TB) == sizeof(T) && P1::KF == P::KF &&
                    PB::KF == P::KF, "one element size per plan");
  using SP = Pack4<T>;               // hidden activations
  using SB = Pack4<TB>;              // reverse vectors
  using SS = Pack4<typename PL::S>;  // tanh' between the sweeps
  static_assert(!RES || sizeof(T) == 4, "residual form: FP32 tiles");
  constexpr int KF = P::KF;
  constexpr int CT = NP / (16 * NW);
  constexpr int R = 16 * RT;
  constexpr int JT = NP / 16;
  static_assert(CT >= 1 && CT * 16 * NW == NP, "width/wave split");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int k, tile;
  map_block(blockIdx.x, p.K, p.xcd_grp, k, tile);
  if (tile >= p.n_tiles) return;
  const int row0 = tile * R;
  const int n = p.n, L = p.L, XP = p.XP, X2 = 2 * p.n;
  const int AW = NP > XP ? NP : XP;           // activation tile width
  const int AS = AW + RID_ACT_PAD_BYTES / (int)sizeof(T);    // row stride (+16 bytes)
  const int BUF = R * AS;                     // elements per ping-pong buffer
  T* act = reinterpret_cast<T*>(smem);
  T1* act1 = reinterpret_cast<T1*>(smem);      // the input tile (first layer's format)
  float* u0 = reinterpret_cast<float*>(smem + p.off_u0);
  const int US = XP + 4;
  float* red = reinterpret_cast<float*>(smem + p.off_red);   // [NW][R]
  float* xs = reinterpret_cast<float*>(smem + p.off_xs);     // [R][2n] FP32 cos|sin
  float* wos = reinterpret_cast<float*>(smem + p.off_wo);    // [NP] output weights

  const unsigned char* fbase = p.frag + (size_t)k * p.frag_model_bytes;
  const float* bias = p.bias + (size_t)k * L * NP;
  const float* wo = p.wo + (size_t)k * NP;

  // first forward layer's weights and biases go in flight before the input
  // tile is built
  constexpr int PD = sizeof(T) == 4 ? RID_PD_FP32 : RID_PD_16;
  constexpr bool WIDE = sizeof(T) == 4;
  constexpr int NPASS = WIDE ? RID_NPASS_FP32 : RID_NPASS_16;
  constexpr int CH = CT / NPASS;     // unit tiles per pass of a hidden-layer GEMM
  constexpr int NK = NP / KF;        // k-steps of a hidden-layer GEMM
  constexpr int U0_SPLIT = u0_split<P, NP>();
  constexpr int PDW = WIDE ? RID_PDH_FP32 : RID_PDH_16;
  constexpr int PDH = (NPASS * NK) % (PDW + 1) == 0 ? PDW : 1;   // its weight pipeline depth
  const int jt0 = wave * CT;
  const int uq = 4 * (lane >> 4);    // first of this lane's 4 units in a tile
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<unsigned char*>(fbase), (short)0, (int)p.frag_model_bytes, 0x00020000);
  // fragments of one layer (byte offset off) for this wave's unit tiles
  auto wsrc = [&](unsigned off) {
    return WSrc{rsrc, (int)off + jt0 * kFragBytes, JT * kFragBytes};
  };
  // plain input: the first column batch of the tile's encoding is loaded
  // before anything else, so its loads return ahead of the weight and bias
  // loads queued behind them (rows of the tile go to the waves in turn; a
  // wave's lanes cover a row in float2 columns)
  constexpr int RW = FROM_POS ? 1 : R / NW;   // rows per wave (R = 16 RT)
  static_assert(FROM_POS || RW * NW == R, "rows per wave");
  float2 xv[RW];
  auto load_x = [&](int cb) {
    const int col = cb + lane;                // float2 column
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      const int row = row0 + wave * RW + j;
      xv[j] = (col < p.n && row < p.B)
                  ? *reinterpret_cast<const float2*>(p.x + (size_t)row * X2 + 2 * col)
                  : make_float2(0.f, 0.f);
    }
  };
  if constexpr (!FROM_POS) load_x(0);
  WRing<PD, CT> wr;                  // first layer
  WRing<PDH, CH> wh;                 // hidden layers (passes of CH tiles)
  ring_preload<PD, CT>(wr, wsrc(p.fwd_off[0]), XP / KF, lane);
  f4 bnext[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c)
    bnext[c] = *reinterpret_cast<const f4*>(bias + (jt0 + c) * 16 + uq);

  for (int i = threadIdx.x; i < NP; i += NW * 64) wos[i] = wo[i];   // published below

  // ---------------- input tile: x = [cos s | sin s] -> buffer 0 ----------------
  if constexpr (FROM_POS) {
    // torsions of the tile's walkers, p.rc walkers per pass (the gather
    // scratch lives in buffer 1).  Gather: a lane owns coordinates
    // j = lane + 64m of the unique-atom list and copies them for the walkers
    // of its wave (walkers to the waves in turn); then a lane per torsion.
    // Coordinates go in chunks of kGatherBatch per lane: the chunk's index
    // loads, then its coordinate loads for all of the wave's walkers, then
    // the stores.  Slots past the end are clamped to the last coordinate or
    // walker of the pass (they store that slot's own value again), so no
    // load sits behind a branch; walkers past B get zeros.
    float* sp = reinterpret_cast<float*>(smem + p.off_ph0);   // [rc][U][3]
    const int U3 = 3 * p.sv.U;
    constexpr int WPW = (R + NW - 1) / NW;    // walkers per wave and pass, at most
    constexpr int QB = WPW < 4 ? WPW : 4;     // walkers per batch of loads
    static_assert(WPW % QB == 0, "walker batches");
    const size_t wstride = (size_t)p.sv.n_atoms * 3;
    for (int c0 = 0; c0 < R; c0 += p.rc) {
      const int rc = R - c0 < p.rc ? R - c0 : p.rc;
      for (int j0 = lane; j0 < U3; j0 += kGatherBatch * 64) {
        int jc[kGatherBatch], a[kGatherBatch];
#pragma unroll
        for (int m = 0; m < kGatherBatch; ++m) {
          jc[m] = min(j0 + m * 64, U3 - 1);
          const int u = jc[m] / 3;
          a[m] = 3 * p.sv.uniq[u] + (jc[m] - 3 * u);
        }
#pragma unroll 1
        for (int q0 = 0; q0 < WPW && wave + q0 * NW < rc; q0 += QB) {
          float v[QB][kGatherBatch];
#pragma unroll
          for (int q = 0; q < QB; ++q) {
            const int il = min(wave + (q0 + q) * NW, rc - 1);
            const int row = min(row0 + c0 + il, p.B - 1);
#pragma unroll
            for (int m = 0; m < kGatherBatch; ++m) v[q][m] = p.pos[row * wstride + a[m]];
          }
#pragma unroll
          for (int q = 0; q < QB; ++q) {
            const int il = min(wave + (q0 + q) * NW, rc - 1);
            const bool in_b = row0 + c0 + il < p.B;
#pragma unroll
            for (int m = 0; m < kGatherBatch; ++m)
              sp[il * U3 + jc[m]] = in_b ? v[q][m] : 0.f;
          }
        }
      }
      __syncthreads();
      for (int il = wave; il < rc; il += NW) {
        const int i = c0 + il;
        for (int c = lane; c < n; c += 64) {
          float cs = 0.f, sn = 0.f;
          if (row0 + i < p.B) {
            const Torsion t = torsion(sp + il * U3, p.sv.lq + 4 * c);
            torsion_cos_sin(t, cs, sn);
          }
          xs[i * X2 + c] = cs;
          xs[i * X2 + n + c] = sn;
          act1[i * AS + c] = P1::from_float(cs);
          act1[i * AS + n + c] = P1::from_float(sn);
        }
      }
      __syncthreads();
    }
    for (int i = wave; i < R; i += NW)
      for (int c = X2 + lane; c < XP; c += 64) act1[i * AS + c] = P1::from_float(0.f);
  } else {
    // the column batches of the tile (the first one is already in xv);
    // padding columns [X2, XP) get zeros (X2 is even)
    const int h2 = X2 / 2, hp = XP / 2;
    for (int cb = 0; cb < hp; cb += 64) {
      const int col = cb + lane;              // float2 column
      if (cb > 0) load_x(cb);
      if (col < hp) {
#pragma unroll
        for (int j = 0; j < RW; ++j) {
          const int i = wave * RW + j;
          Pack2<T1>::store(act1 + i * AS + 2 * col, xv[j].x, xv[j].y);
          if (col < h2) *reinterpret_cast<float2*>(xs + i * X2 + 2 * col) = xv[j];
        }
      }
    }
  }
  __syncthreads();

  const int wl = lane & 15;          // walker within a 16-walker tile
  SS st[LM - 1][RT][CT];             // tanh' of hidden layers 1..L-1
  // 16-bit plans: the packed w_o carries a per-member power-of-two scale
  // (exact), so the reverse vectors start scaled; the scale is undone where
  // A and g are written (uniform loads of its inverse there)
  constexpr bool SCALED = sizeof(T) == 2;
  auto a_total = [&](int i) {
    if constexpr (SCALED) {
      float a = 0.f;
      for (int w = 0; w < NW; ++w) a += red[w * R + i];
      return __builtin_fmaf(a, p.vscale[2 * k + 1], p.bo[k]);
    } else {
      float a = p.bo[k];
      for (int w = 0; w < NW; ++w) a += red[w * R + i];
      return a;
    }
  };
  int cur = 0;

  // ---------------- forward: h_l = tanh(W_l h_{l-1} + b_l) ----------------
  // tile epilogues: tanh and its derivative; a layer before the last stores
  // h_l into the other buffer and stashes tanh'; the last layer stores
  // v_L = w_o * tanh' and accumulates the lane's part of A = w_o . h_L.
  // Residual form (RES): hidden layers after the first add their input,
  // h_l = h_{l-1} + tanh(z_l), read from the layer's input buffer at the
  // lane's own four units (all hidden layers share the padded width).
  float apart[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) apart[rt] = 0.f;
  f4 ares[RT][CT];                   // RES: dA/dh of the layer being reversed
  auto skip_in = [&](const T* in, int rt, int c) {
    return *reinterpret_cast<const f4*>(in + (rt * 16 + wl) * AS + (jt0 + c) * 16 + uq);
  };
  auto mid_tile = [&](int l, int rt, int c, const f4& z, const T* in, T* out) {
    f4 h, d;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float dq;
      h[q] = tanh_and_grad(z[q], dq);
      d[q] = dq;
    }
    if constexpr (RES) {
      if (l >= 1) h += skip_in(in, rt, c);
    }
    SP o;
    o.set(h);
    o.store(out + (rt * 16 + wl) * AS + (jt0 + c) * 16 + uq);
    if constexpr (GRAD) st[l][rt][c].set(d);
  };
  auto last_tile = [&](int rt, int c, const f4& z, const T* in, bool skip, T* out) {
    const int u = (jt0 + c) * 16 + uq;
    const f4 w4 = *reinterpret_cast<const f4*>(wos + u);
    f4 h, d;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float dq;
      h[q] = tanh_and_grad(z[q], dq);
      d[q] = dq;
    }
    if constexpr (RES) {
      if (skip) h += skip_in(in, rt, c);
      ares[rt][c] = w4;              // dA/dh_L = w_o
    }
    apart[rt] += w4[0] * h[0] + w4[1] * h[1] + w4[2] * h[2] + w4[3] * h[3];
    if constexpr (GRAD) {
      SB o;
      o.set(w4 * d);
      o.store(reinterpret_cast<TB*>(out) + (rt * 16 + wl) * AS + u);
    }
  };
  // the GEMM after forward layer l: forward layer l+1, or the first backward
  auto next_after_fwd = [&](int l) {
    return wsrc(l + 1 < L ? p.fwd_off[l + 1] : p.bwd_off[L > 1 ? L - 1 : 0]);
  };
  auto load_bias = [&](int l) {
#pragma unroll
    for (int c = 0; c < CT; ++c)
      bnext[c] = *reinterpret_cast<const f4*>(bias + l * NP + (jt0 + c) * 16 + uq);
  };

  {  // layer 1 (input width XP): one pass over all CT tiles
    T* out = act + BUF;
    f4 acc[RT][CT];
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[rt][c] = bnext[c];
    gemm_run<P1, RT, CT, PD>(acc, wr, act1, AS, wsrc(p.fwd_off[0]), XP / KF, lane);
    if (L > 1) {
      ring_preload<PDH, CH>(wh, next_after_fwd(0), NK, lane);
      load_bias(1);
#pragma unroll
      for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) mid_tile(0, rt, c, acc[rt][c], act, out);
    } else {
#pragma unroll
      for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) last_tile(rt, c, acc[rt][c], act, false, out);
    }
    cur = 1;
    __syncthreads();
  }
  // hidden layers before the last
#pragma unroll
  for (int l = 1; l < LM - 1; ++l) {
    if (l < L - 1) {
      const T* in = act + cur * BUF;
      T* out = act + (cur ^ 1) * BUF;
      f4 acc[RT][CT];
#pragma unroll
      for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt][c] = bnext[c];
      gemm_hidden<P, RT, CT, NPASS, PDH, NK>(acc, wh, in, AS, wsrc(p.fwd_off[l]), true,
                                             next_after_fwd(l), lane);
      load_bias(l + 1);
#pragma unroll
      for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) mid_tile(l, rt, c, acc[rt][c], in, out);
      cur ^= 1;
      __syncthreads();
    }
  }
  if (L > 1) {  // the last hidden layer (index L-1)
    const T* in = act + cur * BUF;
    T* out = act + (cur ^ 1) * BUF;
    f4 acc[RT][CT];
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[rt][c] = bnext[c];
    gemm_hidden<P, RT, CT, NPASS, PDH, NK>(acc, wh, in, AS, wsrc(p.fwd_off[L - 1]), GRAD,
                                           wsrc(p.bwd_off[L - 1]), lane);
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) last_tile(rt, c, acc[rt][c], in, true, out);
    cur ^= 1;
    __syncthreads();
  }
  // A = w_o . h_L + b_o: the lanes' partials reduced over the 4 unit groups,
  // then (after the last barrier) over the waves
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    float v = apart[rt];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (lane < 16) red[wave * R + rt * 16 + wl] = v;
  }
  if constexpr (!GRAD) {
    __syncthreads();
    for (int i = threadIdx.x; i < R; i += NW * 64) {
      const float a = a_total(i);
      if (row0 + i < p.B) p.A_out[(size_t)k * p.B + row0 + i] = a;
    }
    return;
  }

  // ------------- reverse sweep: v_{l-1} = (W_l^T v_l) * tanh'_{l-1} -------------
  // Residual form: the skip of layer l carries dA/dh_l on, so
  // dA/dh_{l-1} = W_l^T v_l + dA/dh_l (kept per lane in ares) and
  // v_{l-1} = dA/dh_{l-1} * tanh'_{l-1}.
  auto bwd_tile = [&](int l, int rt, int c, const f4& y, T* out) {
    SB o;
    if constexpr (RES) {
      ares[rt][c] += y;
      o.set(ares[rt][c] * st[l - 1][rt][c].get());
    } else {
      o.set(y * st[l - 1][rt][c].get());
    }
    o.store(reinterpret_cast<TB*>(out) + (rt * 16 + wl) * AS + (jt0 + c) * 16 + uq);
  };
#pragma unroll
  for (int l = LM - 1; l >= 1; --l) {
    if (l < L) {
      const T* in = act + cur * BUF;
      T* out = act + (cur ^ 1) * BUF;
      f4 acc[RT][CT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[rt][c] = f4{0.f, 0.f, 0.f, 0.f};
      gemm_hidden<PB, RT, CT, NPASS, PDH, NK>(acc, wh, reinterpret_cast<const TB*>(in), AS,
                                              wsrc(p.bwd_off[l]), l >= 2,
                                              wsrc(p.bwd_off[l >= 2 ? l - 1 : l]), lane);
#pragma unroll
      for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) bwd_tile(l, rt, c, acc[rt][c], out);
      cur ^= 1;
      __syncthreads();
    }
  }
  // layer 1 backward: u0 = W_1^T v_1.  Its XP/16 column tiles are too few
  // to spread evenly over the waves, so each tile's contraction is cut into
  // p.u0p parts (U0_SPLIT, or 1 when that many partial tiles would not fit
  // the LDS); the parts' partial sums go to LDS (u0 part q at
  // u0 + q * R * US) and are added in part order when u0 is read.
  // v_1 sits in buffer 1 (2L-1 buffer flips), so u0 may alias buffer 0.
  if constexpr (U0_SPLIT == 1) {
    // one part (16-bit tiles): the plain form
    {
      const T* in = act + cur * BUF;
      const int JT0 = XP / 16;
      for (int t = wave; t < JT0; t += NW) {
        f4 a1[RT][1];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) a1[rt][0] = f4{0.f, 0.f, 0.f, 0.f};
        gemm_tiles<PB, RT, 1, 7>(
            a1, reinterpret_cast<const TB*>(in), AS,
            WSrc{rsrc, (int)p.bwd_off[0] + t * kFragBytes, JT0 * kFragBytes}, NK, lane);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          *reinterpret_cast<f4*>(u0 + (rt * 16 + wl) * US + t * 16 + uq) = a1[rt][0];
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < R; i += NW * 64) {
      const float a = a_total(i);
      if (row0 + i < p.B) p.A_out[(size_t)k * p.B + row0 + i] = a;
    }
    const float ivs = SCALED ? p.vscale[2 * k + 1] : 1.f;
    for (int e = threadIdx.x; e < R * n; e += NW * 64) {
      const int i = e / n, c = e - i * n;
      const int row = row0 + i;
      if (row < p.B) {
        const float cs = xs[i * X2 + c];
        const float sn = xs[i * X2 + n + c];
        float gv = -sn * u0[i * US + c] + cs * u0[i * US + n + c];
        if constexpr (!FROM_POS) {
          if (p.raw && p.raw[c]) gv = u0[i * US + c];
        }
        p.g_out[((size_t)k * p.B + row) * n + c] = SCALED ? gv * ivs : gv;
      }
    }
  } else {
    // PARTS is U0_SPLIT (the common case, compile-time loops) or 1
    auto u0_stage = [&](auto parts_c) {
      constexpr int PARTS = decltype(parts_c)::value;
      const T* in = act + cur * BUF;
      const int JT0 = XP / 16;
      constexpr int KQ = NK / PARTS;            // k-steps per part
      for (int it = wave; it < JT0 * PARTS; it += NW) {
        const int t = it / PARTS, q = it - t * PARTS;
        f4 a1[RT][1];
  #pragma unroll
        for (int rt = 0; rt < RT; ++rt) a1[rt][0] = f4{0.f, 0.f, 0.f, 0.f};
        gemm_tiles<PB, RT, 1, 7>(
            a1, reinterpret_cast<const TB*>(in) + q * KQ * KF, AS,
            WSrc{rsrc, (int)p.bwd_off[0] + t * kFragBytes + q * KQ * JT0 * kFragBytes,
                 JT0 * kFragBytes},
            KQ, lane);
        float* uq0 = u0 + q * R * US;
  #pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          *reinterpret_cast<f4*>(uq0 + (rt * 16 + wl) * US + t * 16 + uq) = a1[rt][0];
      }
    };
    const bool full = U0_SPLIT == 1 || p.u0p == U0_SPLIT;
    if (full)
      u0_stage(std::integral_constant<int, U0_SPLIT>{});
    else
      u0_stage(std::integral_constant<int, 1>{});
    __syncthreads();
    // A = sum of the waves' partial dot products + b_o
    for (int i = threadIdx.x; i < R; i += NW * 64) {
      const float a = a_total(i);
      if (row0 + i < p.B) p.A_out[(size_t)k * p.B + row0 + i] = a;
    }
    // chain to the angles: g_i = -sin s_i u0[i] + cos s_i u0[n+i]
    auto chain = [&](auto parts_c) {
      constexpr int PARTS = decltype(parts_c)::value;
      auto u0_at = [&](int i, int c) {
        float v = u0[i * US + c];
  #pragma unroll
        for (int q = 1; q < PARTS; ++q) v += u0[q * R * US + i * US + c];
        return v;
      };
      const float ivs = SCALED ? p.vscale[2 * k + 1] : 1.f;
      for (int e = threadIdx.x; e < R * n; e += NW * 64) {
        const int i = e / n, c = e - i * n;
        const int row = row0 + i;
        if (row < p.B) {
          const float cs = xs[i * X2 + c];
          const float sn = xs[i * X2 + n + c];
          float gv = -sn * u0_at(i, c) + cs * u0_at(i, n + c);
          if constexpr (!FROM_POS) {
            if (p.raw && p.raw[c]) gv = u0_at(i, c);
          }
          p.g_out[((size_t)k * p.B + row) * n + c] = SCALED ? gv * ivs : gv;
        }
      }
    };
    if (full)
      chain(std::integral_constant<int, U0_SPLIT>{});
    else
      chain(std::integral_constant<int, 1>{});
  }
}

// ---------------------------------------------------------------------------
// Hessian-vector products for conservative switching (FP32 ensembles).
// For walker w and member k, with rho_x = (dx/ds) w_k (w_k the walker's
// deviation direction, zero outside the switching band):
//   u0  = dA_k/dx                          (reverse sweep, as in mlp_kernel)
//   u0d = H_x rho_x = d/dt u0(x + t rho_x)  (forward-over-reverse)
// and the member's term of d eps/ds, chained to the angles:
//   T_k[i] = -sin s_i u0d[i] + cos s_i u0d[n+i] - w_ki (cos s_i u0[i] + sin s_i u0[n+i]).
// Tangent recurrences: zd_1 = W_1 rho_x, hd_l = tanh'_l zd_l,
// zd_{l+1} = W_{l+1} hd_l, dd_l = -2 h_l hd_l (tangent of tanh'),
// vd_L = w_o dd_L, vd_{l-1} = (W_l^T vd_l) tanh'_{l-1} + (W_l^T v_l) dd_{l-1},
// u0d = W_1^T vd_1.
// One workgroup owns 16 walkers of one member.  Rows 0-15 of its activation
// tile are the walkers' primal vectors and rows 16-31 their tangents, so
// every weight fragment streamed from L2 feeds both (the MFMA B operand
// spans two 16-row tiles), and tanh' and its tangent stay in registers
// between the sweeps.  One 16-unit tile per wave.
// ---------------------------------------------------------------------------
struct HvpArgs {
  const float* x;      // [B][2n] encoding cos s | sin s
  const float* rho;    // [B][K][n] w_k
  const float* coef;   // [B] Abar sigma'(eps): a tile whose walkers are all 0 is skipped
  float* T_out;        // [K][B][n]
  int B, n, K, L, XP, n_tiles, xcd_grp;
  const unsigned char* frag;
  unsigned long long frag_model_bytes;
  unsigned fwd_off[kMaxHidden];
  unsigned bwd_off[kMaxHidden];
  const float* bias;   // [K][L][NP], pre-scaled like the forward weights
  const float* wo;     // [K][NP]
  unsigned off_u0, off_xs, off_rs, off_wo;   // LDS byte offsets
};

// ln 2 / 2: undoes the forward pre-scale on the tangent rows (no bias there)
constexpr float kTanhUnscale = 0.34657359027997264f;

template <int NP, int NW, int LM>
__global__ __launch_bounds__(NW * 64) void hvp_kernel(HvpArgs p) {
  using P = F32;
  constexpr int KF = P::KF;
  constexpr int RT = 2;                       // primal rows, tangent rows
  constexpr int CT = NP / (16 * NW);
  static_assert(CT == 1 && 16 * NW == NP, "one unit tile per wave");
  constexpr int R = 16 * RT;
  constexpr int JT = NP / 16;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int k, tile;
  map_block(blockIdx.x, p.K, p.xcd_grp, k, tile);
  if (tile >= p.n_tiles) return;
  const int row0 = tile * 16;
  // every wave takes the same vote, so a skipped tile leaves as a whole
  if (!__any(p.coef[min(row0 + (lane & 15), p.B - 1)] != 0.f)) return;

  const int n = p.n, L = p.L, XP = p.XP, X2 = 2 * p.n;
  const int AW = NP > XP ? NP : XP;
  const int AS = AW + RID_ACT_PAD_BYTES / 4;
  const int BUF = R * AS;
  float* act = reinterpret_cast<float*>(smem);
  float* u0 = reinterpret_cast<float*>(smem + p.off_u0);
  const int US = XP + 4;
  float* xs = reinterpret_cast<float*>(smem + p.off_xs);    // [16][2n]
  float* rs = reinterpret_cast<float*>(smem + p.off_rs);    // [16][n] w_k
  float* wos = reinterpret_cast<float*>(smem + p.off_wo);   // [NP]

  const unsigned char* fbase = p.frag + (size_t)k * p.frag_model_bytes;
  const float* bias = p.bias + (size_t)k * L * NP;
  const float* wo = p.wo + (size_t)k * NP;
  constexpr int PD = RID_PD_FP32;
  constexpr int NK = NP / KF;
  constexpr int U0_SPLIT = u0_split<P, NP>();
  constexpr int PDH = NK % (RID_PDH_FP32 + 1) == 0 ? RID_PDH_FP32 : 1;
  const int jt0 = wave;
  const int wl = lane & 15;
  const int uq = 4 * (lane >> 4);
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<unsigned char*>(fbase), (short)0, (int)p.frag_model_bytes, 0x00020000);
  auto wsrc = [&](unsigned off) {
    return WSrc{rsrc, (int)off + jt0 * kFragBytes, JT * kFragBytes};
  };
  WRing<PD, 1> wr;
  WRing<PDH, 1> wh;
  ring_preload<PD, 1>(wr, wsrc(p.fwd_off[0]), XP / KF, lane);
  f4 bnext = *reinterpret_cast<const f4*>(bias + jt0 * 16 + uq);
  for (int i = threadIdx.x; i < NP; i += NW * 64) wos[i] = wo[i];

  // input tile: rows 0-15 x, rows 16-31 rho_x = [-sin s w | cos s w],
  // columns [2n, XP) zero; walkers past B are zero rows
  for (int e = threadIdx.x; e < 16 * XP; e += NW * 64) {
    const int i = e / XP, c = e - i * XP;
    const int row = row0 + i;
    float xv = 0.f, tv = 0.f;
    if (row < p.B && c < X2) {
      const int ci = c < n ? c : c - n;
      xv = p.x[(size_t)row * X2 + c];
      const float other = p.x[(size_t)row * X2 + (c < n ? c + n : c - n)];
      const float w = p.rho[((size_t)row * p.K + k) * n + ci];
      tv = c < n ? -other * w : other * w;
      xs[i * X2 + c] = xv;
      if (c < n) rs[i * n + c] = w;
    }
    act[i * AS + c] = xv;
    act[(16 + i) * AS + c] = tv;
  }
  __syncthreads();

  f4 sd[LM - 1], sdd[LM - 1];   // tanh' and its tangent, hidden layers 1..L-1
  int cur = 0;
  auto store_pair = [&](float* out, const f4& prim, const f4& tang) {
    *reinterpret_cast<f4*>(out + wl * AS + jt0 * 16 + uq) = prim;
    *reinterpret_cast<f4*>(out + (16 + wl) * AS + jt0 * 16 + uq) = tang;
  };
  // forward epilogue: y, yd are the pre-scaled GEMM outputs of the two rows
  auto fwd_core = [&](const f4& y, const f4& yd, f4& h, f4& d, f4& hd, f4& dd) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float dq;
      h[q] = tanh_and_grad(y[q], dq);
      d[q] = dq;
      hd[q] = dq * (yd[q] * kTanhUnscale);
      dd[q] = -2.f * h[q] * hd[q];
    }
  };
  auto mid_epi = [&](int l, const f4& y, const f4& yd, float* out) {
    f4 h, d, hd, dd;
    fwd_core(y, yd, h, d, hd, dd);
    store_pair(out, h, hd);
    sd[l] = d;
    sdd[l] = dd;
  };
  auto last_epi = [&](const f4& y, const f4& yd, float* out) {
    const f4 w4 = *reinterpret_cast<const f4*>(wos + jt0 * 16 + uq);
    f4 h, d, hd, dd;
    fwd_core(y, yd, h, d, hd, dd);
    store_pair(out, w4 * d, w4 * dd);    // v_L, vd_L
  };
  auto next_after_fwd = [&](int l) {
    return wsrc(l + 1 < L ? p.fwd_off[l + 1] : p.bwd_off[L > 1 ? L - 1 : 0]);
  };
  auto init_fwd = [&](f4 (&acc)[RT][1]) {
    acc[0][0] = bnext;
    acc[1][0] = f4{0.f, 0.f, 0.f, 0.f};
  };

  {  // layer 1
    float* out = act + BUF;
    f4 acc[RT][1];
    init_fwd(acc);
    gemm_run<P, RT, 1, PD>(acc, wr, act, AS, wsrc(p.fwd_off[0]), XP / KF, lane);
    if (L > 1) {
      ring_preload<PDH, 1>(wh, next_after_fwd(0), NK, lane);
      bnext = *reinterpret_cast<const f4*>(bias + NP + jt0 * 16 + uq);
      mid_epi(0, acc[0][0], acc[1][0], out);
    } else {
      last_epi(acc[0][0], acc[1][0], out);
    }
    cur = 1;
    __syncthreads();
  }
#pragma unroll
  for (int l = 1; l < LM - 1; ++l) {
    if (l < L - 1) {
      const float* in = act + cur * BUF;
      float* out = act + (cur ^ 1) * BUF;
      f4 acc[RT][1];
      init_fwd(acc);
      gemm_hidden<P, RT, 1, 1, PDH, NK>(acc, wh, in, AS, wsrc(p.fwd_off[l]), true,
                                        next_after_fwd(l), lane);
      bnext = *reinterpret_cast<const f4*>(bias + (l + 1) * NP + jt0 * 16 + uq);
      mid_epi(l, acc[0][0], acc[1][0], out);
      cur ^= 1;
      __syncthreads();
    }
  }
  if (L > 1) {
    const float* in = act + cur * BUF;
    float* out = act + (cur ^ 1) * BUF;
    f4 acc[RT][1];
    init_fwd(acc);
    gemm_hidden<P, RT, 1, 1, PDH, NK>(acc, wh, in, AS, wsrc(p.fwd_off[L - 1]), true,
                                      wsrc(p.bwd_off[L - 1]), lane);
    last_epi(acc[0][0], acc[1][0], out);
    cur ^= 1;
    __syncthreads();
  }
  // reverse: v_{l-1} = y tanh'_{l-1}, vd_{l-1} = yd tanh'_{l-1} + y dd_{l-1}
#pragma unroll
  for (int l = LM - 1; l >= 1; --l) {
    if (l < L) {
      const float* in = act + cur * BUF;
      float* out = act + (cur ^ 1) * BUF;
      f4 acc[RT][1];
      acc[0][0] = f4{0.f, 0.f, 0.f, 0.f};
      acc[1][0] = f4{0.f, 0.f, 0.f, 0.f};
      gemm_hidden<P, RT, 1, 1, PDH, NK>(acc, wh, in, AS, wsrc(p.bwd_off[l]), l >= 2,
                                        wsrc(p.bwd_off[l >= 2 ? l - 1 : l]), lane);
      const f4 y = acc[0][0], yd = acc[1][0];
      store_pair(out, y * sd[l - 1], yd * sd[l - 1] + y * sdd[l - 1]);
      cur ^= 1;
      __syncthreads();
    }
  }
  // u0 | u0d = W_1^T [v_1 | vd_1], contraction split as in mlp_kernel; the
  // vectors sit in buffer 1 (2L-1 flips), so u0 may alias buffer 0
  {
    const float* in = act + cur * BUF;
    const int JT0 = XP / 16;
    constexpr int KQ = NK / U0_SPLIT;
    for (int it = wave; it < JT0 * U0_SPLIT; it += NW) {
      const int t = it / U0_SPLIT, q = it - t * U0_SPLIT;
      f4 a1[RT][1];
      a1[0][0] = f4{0.f, 0.f, 0.f, 0.f};
      a1[1][0] = f4{0.f, 0.f, 0.f, 0.f};
      gemm_tiles<P, RT, 1, 7>(
          a1, in + q * KQ * KF, AS,
          WSrc{rsrc, (int)p.bwd_off[0] + t * kFragBytes + q * KQ * JT0 * kFragBytes,
               JT0 * kFragBytes},
          KQ, lane);
      float* uq0 = u0 + q * R * US;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        *reinterpret_cast<f4*>(uq0 + (rt * 16 + wl) * US + t * 16 + uq) = a1[rt][0];
    }
  }
  __syncthreads();
  auto u0_at = [&](int i, int c) {
    float v = u0[i * US + c];
#pragma unroll
    for (int q = 1; q < U0_SPLIT; ++q) v += u0[q * R * US + i * US + c];
    return v;
  };
  for (int e = threadIdx.x; e < 16 * n; e += NW * 64) {
    const int i = e / n, c = e - i * n;
    const int row = row0 + i;
    if (row < p.B) {
      const float cs = xs[i * X2 + c], sn = xs[i * X2 + n + c];
      const float hv = -sn * u0_at(16 + i, c) + cs * u0_at(16 + i, n + c);
      const float cu = cs * u0_at(i, c) + sn * u0_at(i, n + c);
      p.T_out[((size_t)k * p.B + row) * n + c] = hv - rs[i * n + c] * cu;
    }
  }
}

// ---------------------------------------------------------------------------
// Mean-force training sweeps (FP32 ensembles), one workgroup per 16 samples
// and member.  Loss L = (1/B) sum_b |g(s_b) - F_b|^2 with g = dA/ds.  Its
// parameter gradient is the gradient of J = sum_b rho_b . g(s_b), with
// rho = 2 (g - F) / B held fixed (or an upstream rho given by the caller),
// and J is the tangent of A along rho_x = (dx/ds) rho.  The kernel runs,
// from LDS and registers:
//   primal forward      h_l = tanh(W_l h_{l-1} + b_l)            rows 0-15
//   primal reverse      v_L = w_o tanh'_L, v_{l-1} = (W_l^T v_l) tanh'_{l-1},
//                       u0 = W_1^T v_1, g, residual, rho_x       rows 0-15
//   tangent forward     zd_l = W_l hd_{l-1}, hd_l = tanh'_l zd_l  rows 16-31
//   adjoint of J        lam_zd = tanh' lam_hd,
//                       lam_z = tanh' (lam_h - 2 h zd lam_hd),
//                       [lam_h ; lam_hd]_{l-1} = W_l^T [lam_z ; lam_zd]_l,
//                       top: lam_hd = w_o, lam_h = 0             rows 0-31
// and writes what the batch-reduced weight gradients need: [h ; hd] of
// every layer input (x ; rho_x first) and [lam_z ; lam_zd] of every layer,
// each as [K][2B][width], plus the samples' squared residuals.  h and zd
// of this lane's units stay in VGPRs between the sweeps.
// Dropout (training only): hidden unit j of layer l of sample b is kept with
// probability 1 - p and then scaled by 1/(1 - p): word j mod 4 of the
// Philox4x32-10 block with counter (b, step, 16 member + l, j div 4), kept
// when its uniform is >= p.  The scaled output S tanh(z) has derivative
// S (1 - tanh^2) in every sweep; the second-order term keeps the unscaled
// tanh.  Without dropout S = 1.
// ---------------------------------------------------------------------------
struct TrainArgs {
  const float* s;      // [B][n]
  const float* F;      // [B][n] labels (null when rho is given)
  const float* rho;    // [B][K][n] upstream gradient of g, or null
  float* hh[kMaxHidden + 1];   // [K][2B][wd[j]]
  float* sl[kMaxHidden];       // [K][2B][wd[j+1]]
  float* loss_rows;    // row b of member k at loss_rows[k * loss_ld + b], or null
  long long loss_ld;
  int row_base;        // batch index of row 0 (dropout counters)
  int B_norm;          // the whole batch's size (rho scale)
  int B, n, K, L, XP, n_tiles, xcd_grp;
  int wd[kMaxHidden + 1];      // 2n, then the hidden widths
  const unsigned char* frag;
  unsigned long long frag_model_bytes;
  unsigned fwd_off[kMaxHidden];
  unsigned bwd_off[kMaxHidden];
  const float* bias;   // [K][L][NP], pre-scaled
  const float* wo;     // [K][NP]
  unsigned off_u0, off_xs, off_wo;
  float drop_p, drop_inv;       // rate and 1/(1 - rate); 0 and 1 without dropout
  unsigned long long drop_seed;
  uint32_t step;
};

template <int NP, int NW, int LM>
__global__ __launch_bounds__(NW * 64) void train_kernel(TrainArgs p) {
  using P = F32;
  constexpr int KF = P::KF;
  static_assert(16 * NW == NP, "one unit tile per wave");
  constexpr int JT = NP / 16;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int k, tile;
  map_block(blockIdx.x, p.K, p.xcd_grp, k, tile);
  if (tile >= p.n_tiles) return;
  const int row0 = tile * 16;
  const int n = p.n, L = p.L, XP = p.XP, X2 = 2 * p.n, B = p.B;
  const int AW = NP > XP ? NP : XP;
  const int AS = AW + RID_ACT_PAD_BYTES / 4;
  const int BUF = 32 * AS;
  float* act = reinterpret_cast<float*>(smem);
  float* u0 = reinterpret_cast<float*>(smem + p.off_u0);
  const int US = XP + 4;
  float* xs = reinterpret_cast<float*>(smem + p.off_xs);    // [16][2n]
  float* wos = reinterpret_cast<float*>(smem + p.off_wo);   // [NP]

  const unsigned char* fbase = p.frag + (size_t)k * p.frag_model_bytes;
  const float* bias = p.bias + (size_t)k * L * NP;
  const float* wo = p.wo + (size_t)k * NP;
  constexpr int PD = RID_PD_FP32;
  constexpr int NK = NP / KF;
  constexpr int U0_SPLIT = u0_split<P, NP>();
  constexpr int PDH = NK % (RID_PDH_FP32 + 1) == 0 ? RID_PDH_FP32 : 1;
  const int jt0 = wave;
  const int wl = lane & 15;
  const int uq = 4 * (lane >> 4);
  const int u = jt0 * 16 + uq;       // this lane's first unit
  const int brow = row0 + wl;        // this lane's sample
  const bool in_b = brow < B;
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<unsigned char*>(fbase), (short)0, (int)p.frag_model_bytes, 0x00020000);
  auto wsrc = [&](unsigned off) {
    return WSrc{rsrc, (int)off + jt0 * kFragBytes, JT * kFragBytes};
  };
  WRing<PD, 1> wr;
  WRing<PDH, 1> wh;
  ring_preload<PD, 1>(wr, wsrc(p.fwd_off[0]), XP / KF, lane);
  f4 bnext = *reinterpret_cast<const f4*>(bias + u);
  for (int i = threadIdx.x; i < NP; i += NW * 64) wos[i] = wo[i];
  // dropout keep bits of this lane's 4 units, 4 bits per hidden layer
  unsigned mbits = 0xFFFFFFFFu;
  if (p.drop_p > 0.f) {
    mbits = 0u;
    for (int j = 0; j < L; ++j) {
      uint32_t c[4] = {(uint32_t)(p.row_base + brow), p.step, (uint32_t)(16 * k + j + 1),
                       (uint32_t)(u >> 2)};
      philox4x32_10(c, (uint32_t)(p.drop_seed & 0xFFFFFFFFull), (uint32_t)(p.drop_seed >> 32));
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (philox_uniform(c[q]) >= p.drop_p) mbits |= 1u << (4 * j + q);
    }
  }
  auto dsc = [&](int j) {       // the dropout factors of hidden layer j (0-based)
    f4 r;
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = ((mbits >> (4 * j + q)) & 1u) ? p.drop_inv : 0.f;
    return r;
  };

  // 4 units of row r (0 .. 2B-1) of a [K][2B][w] array; units past w are
  // padding and stay unwritten
  auto put4 = [&](float* base, int w, int r, const f4& v) {
    if (u >= w) return;
    float* dst = base + ((size_t)k * 2 * B + r) * w + u;
    if ((w & 3) == 0) {
      *reinterpret_cast<f4*>(dst) = v;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (u + q < w) dst[q] = v[q];
    }
  };
  auto lds4 = [&](float* buf, int r, const f4& v) {
    *reinterpret_cast<f4*>(buf + r * AS + u) = v;
  };

  // input tile: x = [cos s | sin s] in rows 0-15 (and to hh[0]), zeros past
  // 2n and past B
  for (int e = threadIdx.x; e < 16 * XP; e += NW * 64) {
    const int i = e / XP, c = e - i * XP;
    const int row = row0 + i;
    float v = 0.f;
    if (row < B && c < X2) {
      float sn, cs;
      sincosf(p.s[(size_t)row * n + (c < n ? c : c - n)], &sn, &cs);
      v = c < n ? cs : sn;
      xs[i * X2 + c] = v;
      p.hh[0][((size_t)k * 2 * B + row) * X2 + c] = v;
    }
    act[i * AS + c] = v;
  }
  __syncthreads();

  f4 hs[LM];        // h of layers 0..L-1
  f4 zs[LM - 1];    // zd of layers 0..L-2
  int cur = 0;
  auto next_after_fwd = [&](int j) {
    return wsrc(j + 1 < L ? p.fwd_off[j + 1] : p.bwd_off[L > 1 ? L - 1 : 0]);
  };
  // primal forward epilogue of layer j: h to the next buffer (and HBM), or
  // v_L = w_o tanh'_L at the top
  auto fwd_epi = [&](int j, f4& hj, const f4& y, float* out) {
    f4 h, d;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float dq;
      h[q] = tanh_and_grad(y[q], dq);
      d[q] = dq;
    }
    hj = h;
    const f4 sc = dsc(j);
    if (j < L - 1) {
      const f4 hsc = h * sc;
      lds4(out, wl, hsc);
      if (in_b) put4(p.hh[j + 1], p.wd[j + 1], brow, hsc);
    } else {
      lds4(out, wl, *reinterpret_cast<const f4*>(wos + u) * d * sc);
    }
  };

  // ---------------- primal forward ----------------
  {
    float* out = act + BUF;
    f4 acc[1][1];
    acc[0][0] = bnext;
    gemm_run<P, 1, 1, PD>(acc, wr, act, AS, wsrc(p.fwd_off[0]), XP / KF, lane);
    if (L > 1) {
      ring_preload<PDH, 1>(wh, next_after_fwd(0), NK, lane);
      bnext = *reinterpret_cast<const f4*>(bias + NP + u);
    }
    fwd_epi(0, hs[0], acc[0][0], out);
    cur = 1;
    __syncthreads();
  }
#pragma unroll
  for (int j = 1; j < LM; ++j) {
    if (j < L) {
      const float* in = act + cur * BUF;
      float* out = act + (cur ^ 1) * BUF;
      f4 acc[1][1];
      acc[0][0] = bnext;
      gemm_hidden<P, 1, 1, 1, PDH, NK>(acc, wh, in, AS, wsrc(p.fwd_off[j]), true,
                                       next_after_fwd(j), lane);
      if (j + 1 < L) bnext = *reinterpret_cast<const f4*>(bias + (j + 1) * NP + u);
      fwd_epi(j, hs[j], acc[0][0], out);
      cur ^= 1;
      __syncthreads();
    }
  }
  // ---------------- primal reverse to u0 ----------------
#pragma unroll
  for (int j = LM - 1; j >= 1; --j) {
    if (j < L) {
      const float* in = act + cur * BUF;
      float* out = act + (cur ^ 1) * BUF;
      f4 acc[1][1];
      acc[0][0] = f4{0.f, 0.f, 0.f, 0.f};
      gemm_hidden<P, 1, 1, 1, PDH, NK>(acc, wh, in, AS, wsrc(p.bwd_off[j]), j >= 2,
                                       wsrc(p.bwd_off[j >= 2 ? j - 1 : j]), lane);
      const f4 h = hs[j - 1];
      lds4(out, wl, acc[0][0] * ((1.f - h * h) * dsc(j - 1)));
      cur ^= 1;
      __syncthreads();
    }
  }
  // u0 = W_1^T v_1 (v_1 in buffer 1 after 2L-1 flips; the partials may
  // alias buffer 0)
  {
    const float* in = act + cur * BUF;
    const int JT0 = XP / 16;
    constexpr int KQ = NK / U0_SPLIT;
    for (int it = wave; it < JT0 * U0_SPLIT; it += NW) {
      const int t = it / U0_SPLIT, q = it - t * U0_SPLIT;
      f4 a1[1][1];
      a1[0][0] = f4{0.f, 0.f, 0.f, 0.f};
      gemm_tiles<P, 1, 1, 7>(
          a1, in + q * KQ * KF, AS,
          WSrc{rsrc, (int)p.bwd_off[0] + t * kFragBytes + q * KQ * JT0 * kFragBytes,
               JT0 * kFragBytes},
          KQ, lane);
      *reinterpret_cast<f4*>(u0 + q * 16 * US + wl * US + t * 16 + uq) = a1[0][0];
    }
  }
  ring_preload<PD, 1>(wr, wsrc(p.fwd_off[0]), XP / KF, lane);   // tangent layer 1
  __syncthreads();
  auto u0_at = [&](int i, int c) {
    float v = u0[i * US + c];
#pragma unroll
    for (int q = 1; q < U0_SPLIT; ++q) v += u0[q * 16 * US + i * US + c];
    return v;
  };
  // ---------------- residual and rho_x (a wave per sample) ----------------
  // rho_x goes to rows 16-31 of the buffer holding v_1 (its rows 0-15 are
  // dead after the u0 GEMM) and to the tangent half of hh[0]
  float* tin = act + cur * BUF + 16 * AS;
  for (int i = wave; i < 16; i += NW) {
    const int row = row0 + i;
    float acc = 0.f;
    for (int c = lane; c < n; c += 64) {
      float rx0 = 0.f, rx1 = 0.f;
      if (row < B) {
        const float cs = xs[i * X2 + c], sn = xs[i * X2 + n + c];
        float rho;
        if (p.rho) {
          rho = p.rho[((size_t)row * p.K + k) * n + c];
        } else {
          const float gi = -sn * u0_at(i, c) + cs * u0_at(i, n + c);
          const float ri = gi - p.F[(size_t)row * n + c];
          acc += ri * ri;
          rho = 2.f * ri / (float)p.B_norm;
        }
        rx0 = -sn * rho;
        rx1 = cs * rho;
        float* h0 = p.hh[0] + ((size_t)k * 2 * B + B + row) * X2;
        h0[c] = rx0;
        h0[n + c] = rx1;
      }
      tin[i * AS + c] = rx0;
      tin[i * AS + n + c] = rx1;
    }
    for (int c = X2 + lane; c < XP; c += 64) tin[i * AS + c] = 0.f;
    if (p.loss_rows && row < B) {
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
      if (lane == 0) p.loss_rows[(size_t)k * p.loss_ld + row] = acc;
    }
  }
  __syncthreads();

  // ---------------- tangent forward, then the adjoint's top ----------------
  // layer j epilogue: hd = tanh'_j zd; below the top hd goes on (rows 16-31)
  // and zd is kept; at the top the adjoint starts:
  // lam_zd = tanh'_L w_o, lam_z = tanh'_L (-2 h_L zd_L w_o)
  auto tan_epi = [&](int j, const f4& h, f4& zj, const f4& y, float* out) {
    const f4 zd = y * kTanhUnscale;
    const f4 d = (1.f - h * h) * dsc(j);
    const f4 hd = d * zd;
    if (in_b) put4(p.hh[j + 1], p.wd[j + 1], B + brow, hd);
    if (j < L - 1) {
      lds4(out, 16 + wl, hd);
      zj = zd;
    } else {
      const f4 w4 = *reinterpret_cast<const f4*>(wos + u);
      const f4 lzd = d * w4;
      const f4 lz = d * (-2.f * h * zd * w4);
      lds4(out, wl, lz);
      lds4(out, 16 + wl, lzd);
      if (in_b) {
        put4(p.sl[j], p.wd[j + 1], brow, lz);
        put4(p.sl[j], p.wd[j + 1], B + brow, lzd);
      }
    }
  };
  {
    const float* in = act + cur * BUF + 16 * AS;
    float* out = act + (cur ^ 1) * BUF;
    f4 acc[1][1];
    acc[0][0] = f4{0.f, 0.f, 0.f, 0.f};
    gemm_run<P, 1, 1, PD>(acc, wr, in, AS, wsrc(p.fwd_off[0]), XP / KF, lane);
    if (L > 1) ring_preload<PDH, 1>(wh, next_after_fwd(0), NK, lane);
    f4 dummy;
    tan_epi(0, hs[0], L > 1 ? zs[0] : dummy, acc[0][0], out);
    cur ^= 1;
    __syncthreads();
  }
#pragma unroll
  for (int j = 1; j < LM; ++j) {
    if (j < L) {
      const float* in = act + cur * BUF + 16 * AS;
      float* out = act + (cur ^ 1) * BUF;
      f4 acc[1][1];
      acc[0][0] = f4{0.f, 0.f, 0.f, 0.f};
      gemm_hidden<P, 1, 1, 1, PDH, NK>(acc, wh, in, AS, wsrc(p.fwd_off[j]), true,
                                       next_after_fwd(j), lane);
      f4 dummy;
      tan_epi(j, hs[j], j < LM - 1 ? zs[j < LM - 1 ? j : 0] : dummy, acc[0][0], out);
      cur ^= 1;
      __syncthreads();
    }
  }
  // ---------------- adjoint reverse (primal and tangent rows together) ----------------
#pragma unroll
  for (int j = LM - 1; j >= 1; --j) {
    if (j < L) {
      const float* in = act + cur * BUF;
      float* out = act + (cur ^ 1) * BUF;
      f4 acc[2][1];
      acc[0][0] = f4{0.f, 0.f, 0.f, 0.f};
      acc[1][0] = f4{0.f, 0.f, 0.f, 0.f};
      gemm_hidden<P, 2, 1, 1, PDH, NK>(acc, wh, in, AS, wsrc(p.bwd_off[j]), j >= 2,
                                       wsrc(p.bwd_off[j >= 2 ? j - 1 : j]), lane);
      const f4 h = hs[j - 1], zd = zs[j - 1];
      const f4 d = (1.f - h * h) * dsc(j - 1);
      const f4 lhd = acc[1][0];
      const f4 lzd = d * lhd;
      const f4 lz = d * (acc[0][0] - 2.f * h * zd * lhd);
      if (j >= 2) {
        lds4(out, wl, lz);
        lds4(out, 16 + wl, lzd);
      }
      if (in_b) {
        put4(p.sl[j - 1], p.wd[j], brow, lz);
        put4(p.sl[j - 1], p.wd[j], B + brow, lzd);
      }
      cur ^= 1;
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// weight packer: FP32 masters (packed layout) -> MFMA fragments, biases
// ---------------------------------------------------------------------------
struct PackLayer {
  unsigned w_off, b_off;  // float offsets inside one model's packed block
  int in, out;            // real widths
  int kin_pad;            // padded input width
  unsigned fwd_off, bwd_off;  // byte offsets inside one model's fragments
  int fmt_fwd, fmt_bwd;   // fragment formats (FragFmt)
};

// element format of a set of MFMA fragments
enum FragFmt { kFmtF32 = 0, kFmtBF16 = 1, kFmtF16 = 2 };

struct VecArgs {
  unsigned b_off[kMaxHidden];
  int out[kMaxHidden];
  unsigned wo_off;
  int last_w;
  int vscale_on;          // reverse vectors in a 16-bit format: scale them
};

struct PackAll {
  PackLayer layer[kMaxHidden];
  VecArgs va;
  int L, K, NP;
};

// One launch packs a whole ensemble: block row y < 2L packs layer y/2 in
// direction y%2 (0: forward fragments, contraction = the layer input,
// pre-scaled by 2/ln 2; 1: backward, contraction = the layer output), each
// in its plan's format; row 2L packs the biases (pre-scaled), w_o and b_o,
// zero-padded to NP.  When the reverse sweep runs in FP16, w_o is stored
// times a per-member power of two that puts max |w_o| in [128, 256), so
// v_L = w_o tanh'_L and the vectors after it stay far inside FP16's range
// (and clear of its subnormals) through the sweep; the kernel undoes the
// scale, exactly, in A and g.  vscale[k] = (scale, 1 / scale).
__global__ void pack_kernel(const float* master, size_t per_model, PackAll pa,
                            unsigned char* frag, size_t frag_model_bytes, float* bias,
                            float* wo, float* bo, float* vscale) {
  const int NP = pa.NP;
  if ((int)blockIdx.y == 2 * pa.L) {
    __shared__ float red[256];
    const VecArgs& va = pa.va;
    for (int k = blockIdx.x; k < pa.K; k += gridDim.x) {
      const float* m = master + (size_t)k * per_model;
      for (int l = 0; l < pa.L; ++l)
        for (int j = threadIdx.x; j < NP; j += blockDim.x)
          bias[((size_t)k * pa.L + l) * NP + j] =
              j < va.out[l] ? kTanhPrescale * m[va.b_off[l] + j] : 0.f;
      float mx = 0.f;
      for (int j = threadIdx.x; j < va.last_w; j += blockDim.x) mx = fmaxf(mx, fabsf(m[va.wo_off + j]));
      red[threadIdx.x] = mx;
      __syncthreads();
      for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
      }
      float sc = 1.f;
      if (va.vscale_on && red[0] > 0.f && red[0] < 3.0e38f) {
        int ex;
        (void)frexpf(red[0], &ex);            // red[0] = f 2^ex, f in [0.5, 1)
        sc = ldexpf(1.f, 8 - ex);             // red[0] sc in [128, 256)
      }
      for (int j = threadIdx.x; j < NP; j += blockDim.x)
        wo[(size_t)k * NP + j] = j < va.last_w ? m[va.wo_off + j] * sc : 0.f;
      if (threadIdx.x == 0) {
        bo[k] = m[va.wo_off + va.last_w];
        vscale[2 * k] = sc;
        vscale[2 * k + 1] = 1.f / sc;         // exact: sc is a power of two
      }
      __syncthreads();
    }
    return;
  }
  const PackLayer& pl = pa.layer[blockIdx.y >> 1];
  const int dir = blockIdx.y & 1;
  const int fmt = dir == 0 ? pl.fmt_fwd : pl.fmt_bwd;
  const int KF = fmt == kFmtF32 ? 16 : 32;
  const int E = fmt == kFmtF32 ? 4 : 8;       // elements per lane (16 bytes)
  const int kc = dir == 0 ? pl.kin_pad : NP;
  const int nc = dir == 0 ? NP : pl.kin_pad;
  const int JT = nc / 16, KT = kc / KF;
  const size_t total = (size_t)pa.K * KT * JT * 64;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
       t += (size_t)gridDim.x * blockDim.x) {
    const int lane = t % 64;
    size_t f = t / 64;
    const int jt = f % JT; f /= JT;
    const int kt = f % KT;
    const int k = (int)(f / KT);
    const float* W = master + (size_t)k * per_model + pl.w_off;
    const int col = jt * 16 + (lane & 15);
    float v[8];
    for (int e = 0; e < E; ++e) {
      const int kk = kt * KF + (KF / 4) * (lane >> 4) + e;
      // W is [out][in]; forward: (unit col = out, contraction kk = in);
      // backward: (unit col = in, contraction kk = out)
      const int o = dir == 0 ? col : kk;
      const int i = dir == 0 ? kk : col;
      v[e] = (o < pl.out && i < pl.in) ? W[(size_t)o * pl.in + i] : 0.f;
      if (dir == 0) v[e] *= kTanhPrescale;
    }
    uint4 out;
    if (fmt == kFmtF32) {
      out = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                       __float_as_uint(v[3]));
    } else {
      unsigned short hv[8];
      for (int e = 0; e < 8; ++e)
        hv[e] = fmt == kFmtBF16 ? __builtin_bit_cast(unsigned short, (__bf16)v[e])
                                : __builtin_bit_cast(unsigned short, (_Float16)v[e]);
      out = make_uint4(hv[0] | (unsigned)hv[1] << 16, hv[2] | (unsigned)hv[3] << 16,
                       hv[4] | (unsigned)hv[5] << 16, hv[6] | (unsigned)hv[7] << 16);
    }
    unsigned char* dst = frag + (size_t)k * frag_model_bytes +
                         (dir == 0 ? pl.fwd_off : pl.bwd_off) +
                         (((size_t)kt * JT + jt) * 64 + lane) * 16;
    *reinterpret_cast<uint4*>(dst) = out;
  }
}

inline unsigned align16(size_t v) { return (unsigned)((v + 15) / 16 * 16); }

// LDS layout of one instantiation; returns the total bytes.
size_t mlp_layout(int R, int NW, int AS, size_t tsize, int XP, int n, int U,
                  bool from_pos, int NPw, int u0_parts, MlpArgs& a) {
  const size_t buf = (size_t)R * AS * tsize;
  size_t off = 2 * buf;
  const size_t u0_bytes = (size_t)u0_parts * R * (XP + 4) * 4;
  if (u0_bytes <= buf) {
    a.off_u0 = 0;                       // buffer 0 is free in the last GEMM
  } else {
    a.off_u0 = align16(off);
    off = a.off_u0 + u0_bytes;
  }
  a.off_red = align16(off);
  off = a.off_red + (size_t)NW * R * 4;
  a.off_xs = align16(off);
  off = a.off_xs + (size_t)R * 2 * n * 4;
  a.off_wo = align16(off);              // output weights w_o [NP]
  off = a.off_wo + (size_t)NPw * 4;
  if (from_pos) {
    // gather scratch in buffer 1 (free before layer 1), in passes of rc
    // walkers; a shape with no room for one walker reports 0 passes
    a.off_ph0 = (unsigned)buf;
    const size_t per_walker = (size_t)3 * U * 4;
    a.rc = (int)std::min<size_t>((size_t)R, buf / per_walker);
  }
  return off;
}

template <class PL, int NP, int RT, int NW, int LM>
size_t lds_bytes(const rid_ensemble_impl& e, const TorsionInput* tin) {
  using P = typename PL::PH;
  using T = typename P::T;
  MlpArgs a{};
  const int AW = NP > e.XP ? NP : e.XP;
  const int AS = AW + RID_ACT_PAD_BYTES / (int)sizeof(T);
  return mlp_layout(16 * RT, NW, AS, sizeof(T), e.XP, e.n_cv,
                    tin ? tin->sys->n_uniq : 0, tin != nullptr, NP, u0_split<P, NP>(), a);
}

template <class PL, int NP, int RT, int NW, int LM, bool RES = false>
rid_status run_mlp(const rid_ensemble_impl& e, const float* x, int B,
                   float* A_out, float* g_out, const TorsionInput* tin,
                   hipStream_t st) {
  static size_t attr_bytes[3] = {0, 0, 0};   // dynamic-LDS limit set per kernel
  constexpr int R = 16 * RT;
  using P = typename PL::PH;
  using T = typename P::T;
  const bool from_pos = tin != nullptr;
  const int AW = NP > e.XP ? NP : e.XP;
  const int AS = AW + RID_ACT_PAD_BYTES / (int)sizeof(T);
  MlpArgs a{};
  a.u0p = u0_split<P, NP>();
  size_t lds = mlp_layout(R, NW, AS, sizeof(T), e.XP, e.n_cv,
                          from_pos ? tin->sys->n_uniq : 0, from_pos, NP, a.u0p, a);
  if (lds > 160 * 1024 && a.u0p > 1) {
    // wide inputs: one part, which fits the free activation buffer
    a = MlpArgs{};
    a.u0p = 1;
    lds = mlp_layout(R, NW, AS, sizeof(T), e.XP, e.n_cv,
                     from_pos ? tin->sys->n_uniq : 0, from_pos, NP, 1, a);
  }
  if (lds > 160 * 1024)
    return fail(RID_EUNSUPPORTED, "shape too large for the MLP kernel's LDS");
  if (from_pos && a.rc < 1)
    return fail(RID_EUNSUPPORTED, "too many torsion atoms to gather in-kernel");
  // without g_out only the free energies are computed (plain input only)
  const bool grad = g_out != nullptr;
  if (!grad && from_pos) return fail(RID_EUNSUPPORTED, "energy-only path takes the encoding");
  auto kern = !grad    ? mlp_kernel<PL, NP, RT, NW, LM, false, false, RES>
              : from_pos ? mlp_kernel<PL, NP, RT, NW, LM, true, true, RES>
                         : mlp_kernel<PL, NP, RT, NW, LM, false, true, RES>;
  const int ki = grad ? (from_pos ? 1 : 0) : 2;
  if (lds > 64 * 1024 && lds > attr_bytes[ki]) {
    RID_HIP(hipFuncSetAttribute((const void*)kern,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr_bytes[ki] = lds;
  }
  a.x = x; a.B = B; a.n = e.n_cv; a.K = e.K; a.L = e.L; a.XP = e.XP;
  a.n_tiles = (B + R - 1) / R;
  a.xcd_grp = (8 % e.K == 0) ? 8 / e.K : 0;
  a.frag = e.d_frag; a.frag_model_bytes = e.frag_bytes_per_model;
  for (int l = 0; l < e.L; ++l) {
    a.fwd_off[l] = (unsigned)e.layers[l].fwd_off;
    a.bwd_off[l] = (unsigned)e.layers[l].bwd_off;
  }
  a.bias = e.d_bias; a.wo = e.d_wo; a.bo = e.d_bo; a.vscale = e.d_vscale;
  a.A_out = A_out; a.g_out = g_out;
  a.raw = e.d_raw;
  if (from_pos) {
    const rid_system_impl& s = *tin->sys;
    a.sv = SysView{s.n_atoms, s.n_uniq, s.n_cv, s.d_uniq, s.d_lquads, s.d_csr_ptr,
                   s.d_csr_ent, s.d_atom_local};
    a.pos = tin->pos;
  }
  int grid;
  if (a.xcd_grp > 0)
    grid = 8 * ((a.n_tiles + a.xcd_grp - 1) / a.xcd_grp);
  else
    grid = a.n_tiles * e.K;
  launch_timed(kProfMlp, kern, dim3(grid), dim3(NW * 64), (uint32_t)lds, st, a);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

// 16-bit family: 64 walkers per workgroup when the tile fits LDS, else 32,
// else 16 (the widest inputs); deeper networks (5-6 hidden layers) take 32
// or 16.
template <class P, int NP, int NW>
rid_status run_16bit(const rid_ensemble_impl& e, const float* x, int B, float* A_out,
                     float* g_out, const TorsionInput* t, hipStream_t st) {
  // P: the arithmetic plan
  if (e.L <= 4) {
    if (lds_bytes<P, NP, 4, NW, 4>(e, t) <= 160 * 1024)
      return run_mlp<P, NP, 4, NW, 4>(e, x, B, A_out, g_out, t, st);
    if (lds_bytes<P, NP, 2, NW, 4>(e, t) <= 160 * 1024)
      return run_mlp<P, NP, 2, NW, 4>(e, x, B, A_out, g_out, t, st);
    return run_mlp<P, NP, 1, NW, 6>(e, x, B, A_out, g_out, t, st);
  }
  if (lds_bytes<P, NP, 2, NW, 6>(e, t) <= 160 * 1024)
    return run_mlp<P, NP, 2, NW, 6>(e, x, B, A_out, g_out, t, st);
  return run_mlp<P, NP, 1, NW, 6>(e, x, B, A_out, g_out, t, st);
}

#ifndef RID_16_NW512
#define RID_16_NW512 8
#endif

template <class P>
rid_status launch_16bit(const rid_ensemble_impl& e, const float* x, int B,
                        float* A_out, float* g_out, const TorsionInput* t, hipStream_t st) {
  switch (e.NP) {
    case 64:  return run_16bit<P, 64, 1>(e, x, B, A_out, g_out, t, st);
    case 128: return run_16bit<P, 128, 2>(e, x, B, A_out, g_out, t, st);
    case 256: return run_16bit<P, 256, 4>(e, x, B, A_out, g_out, t, st);
    case 512: return run_16bit<P, 512, RID_16_NW512>(e, x, B, A_out, g_out, t, st);
  }
  return fail(RID_EUNSUPPORTED, "no kernel for this padded width");
}

// FP32 at width 256: 16 waves of one unit tile each (4 per SIMD) hide the
// latencies of the short stages better than 8 waves of two tiles.
#ifndef RID_F32_NW256
#define RID_F32_NW256 16
#endif

rid_status dispatch(const rid_ensemble_impl& e, const float* x, int B, float* A_out,
                    float* g_out, const TorsionInput* t, hipStream_t st) {
  if (e.resnet) {
    // residual connections: FP32, 16-walker tiles
    if (e.prec != RID_FP32)
      return fail(RID_EUNSUPPORTED, "residual connections need an FP32 ensemble");
    switch (e.NP) {
      case 64:  return run_mlp<PlanF32, 64, 1, 1, 6, true>(e, x, B, A_out, g_out, t, st);
      case 128: return run_mlp<PlanF32, 128, 1, 2, 6, true>(e, x, B, A_out, g_out, t, st);
      case 256: return run_mlp<PlanF32, 256, 1, RID_F32_NW256, 6, true>(e, x, B, A_out, g_out, t, st);
      case 512: return run_mlp<PlanF32, 512, 1, 8, 6, true>(e, x, B, A_out, g_out, t, st);
    }
    return fail(RID_EUNSUPPORTED, "no kernel for this padded width");
  }
  if (e.prec == RID_FP32) {
    switch (e.NP) {
      case 64:  return run_mlp<PlanF32, 64, 1, 1, 6>(e, x, B, A_out, g_out, t, st);
      case 128: return run_mlp<PlanF32, 128, 1, 2, 6>(e, x, B, A_out, g_out, t, st);
      case 256:
        // free energies only (MCMC): 32-walker tiles feed two MFMA tiles from
        // each weight fragment, taken while they still keep 3/4 of the CUs busy
        if (!g_out && !t && (long long)((B + 31) / 32) * e.K >= 192)
          return run_mlp<PlanF32, 256, 2, RID_F32_NW256, 6>(e, x, B, A_out, g_out, t, st);
        return run_mlp<PlanF32, 256, 1, RID_F32_NW256, 6>(e, x, B, A_out, g_out, t, st);
      case 512: return run_mlp<PlanF32, 512, 1, 8, 6>(e, x, B, A_out, g_out, t, st);
    }
    return fail(RID_EUNSUPPORTED, "no kernel for this padded width");
  }
  switch (e.prec) {
    case RID_BF16:     return launch_16bit<PlanBF16>(e, x, B, A_out, g_out, t, st);
    case RID_FP16:     return launch_16bit<PlanF16>(e, x, B, A_out, g_out, t, st);
    case RID_BF16_ALL: return launch_16bit<PlanBF16All>(e, x, B, A_out, g_out, t, st);
    default: break;
  }
  return fail(RID_EUNSUPPORTED, "unknown precision");
}

size_t hvp_layout(int NP, int XP, int n, HvpArgs& a) {
  constexpr int R = 32;
  const int AS = (NP > XP ? NP : XP) + RID_ACT_PAD_BYTES / 4;
  const size_t buf = (size_t)R * AS * 4;
  size_t off = 2 * buf;
  // the u0 partials (u0_split gives 4 parts at every FP32 width)
  const size_t u0_bytes = (size_t)u0_split<F32, 64>() * R * (XP + 4) * 4;
  if (u0_bytes <= buf) {
    a.off_u0 = 0;                       // buffer 0 is free in the last GEMM
  } else {
    a.off_u0 = align16(off);
    off = a.off_u0 + u0_bytes;
  }
  a.off_xs = align16(off);
  off = a.off_xs + (size_t)16 * 2 * n * 4;
  a.off_rs = align16(off);
  off = a.off_rs + (size_t)16 * n * 4;
  a.off_wo = align16(off);
  return a.off_wo + (size_t)NP * 4;
}

template <int NP>
rid_status run_hvp(const rid_ensemble_impl& e, const float* x, const float* rho,
                   const float* coef, int B, float* T, hipStream_t st) {
  constexpr int NW = NP / 16;
  static size_t attr = 0;
  HvpArgs a{};
  const size_t lds = hvp_layout(NP, e.XP, e.n_cv, a);
  if (lds > 160 * 1024) return fail(RID_EUNSUPPORTED, "shape too large for the HVP kernel");
  auto kern = hvp_kernel<NP, NW, kMaxHidden>;
  if (lds > 64 * 1024 && lds > attr) {
    RID_HIP(hipFuncSetAttribute((const void*)kern,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = lds;
  }
  a.x = x; a.rho = rho; a.coef = coef; a.T_out = T;
  a.B = B; a.n = e.n_cv; a.K = e.K; a.L = e.L; a.XP = e.XP;
  a.n_tiles = (B + 15) / 16;
  a.xcd_grp = (8 % e.K == 0) ? 8 / e.K : 0;
  a.frag = e.d_frag; a.frag_model_bytes = e.frag_bytes_per_model;
  for (int l = 0; l < e.L; ++l) {
    a.fwd_off[l] = (unsigned)e.layers[l].fwd_off;
    a.bwd_off[l] = (unsigned)e.layers[l].bwd_off;
  }
  a.bias = e.d_bias; a.wo = e.d_wo;
  const int grid = a.xcd_grp > 0 ? 8 * ((a.n_tiles + a.xcd_grp - 1) / a.xcd_grp)
                                  : a.n_tiles * e.K;
  launch_timed(kProfHvp, kern, dim3(grid), dim3(NW * 64), (uint32_t)lds, st, a);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

size_t train_layout(int NP, int XP, int n, TrainArgs& a) {
  const int AS = (NP > XP ? NP : XP) + RID_ACT_PAD_BYTES / 4;
  const size_t buf = (size_t)32 * AS * 4;
  size_t off = 2 * buf;
  // the u0 partials of 16 rows (4 parts at every FP32 width)
  const size_t u0_bytes = (size_t)u0_split<F32, 64>() * 16 * (XP + 4) * 4;
  if (u0_bytes <= buf) {
    a.off_u0 = 0;                       // buffer 0 is free in the u0 GEMM
  } else {
    a.off_u0 = align16(off);
    off = a.off_u0 + u0_bytes;
  }
  a.off_xs = align16(off);
  off = a.off_xs + (size_t)16 * 2 * n * 4;
  a.off_wo = align16(off);
  return a.off_wo + (size_t)NP * 4;
}

template <int NP>
rid_status run_train(const rid_ensemble_impl& e, const TrainIo& io, int B, hipStream_t st) {
  constexpr int NW = NP / 16;
  static size_t attr = 0;
  TrainArgs a{};
  const size_t lds = train_layout(NP, e.XP, e.n_cv, a);
  if (lds > 160 * 1024) return fail(RID_EUNSUPPORTED, "shape too large for the training kernel");
  auto kern = train_kernel<NP, NW, kMaxHidden>;
  if (lds > 64 * 1024 && lds > attr) {
    RID_HIP(hipFuncSetAttribute((const void*)kern,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = lds;
  }
  a.s = io.s; a.F = io.F; a.rho = io.rho; a.loss_rows = io.loss_rows;
  a.loss_ld = io.loss_ld; a.row_base = io.row_base; a.B_norm = io.B_norm;
  for (int j = 0; j <= e.L; ++j) a.hh[j] = io.hh[j];
  for (int j = 0; j < e.L; ++j) a.sl[j] = io.sl[j];
  a.B = B; a.n = e.n_cv; a.K = e.K; a.L = e.L; a.XP = e.XP;
  a.n_tiles = (B + 15) / 16;
  a.xcd_grp = (8 % e.K == 0) ? 8 / e.K : 0;
  a.wd[0] = 2 * e.n_cv;
  for (int j = 0; j < e.L; ++j) a.wd[j + 1] = e.widths[j];
  a.frag = e.d_frag; a.frag_model_bytes = e.frag_bytes_per_model;
  for (int l = 0; l < e.L; ++l) {
    a.fwd_off[l] = (unsigned)e.layers[l].fwd_off;
    a.bwd_off[l] = (unsigned)e.layers[l].bwd_off;
  }
  a.bias = e.d_bias; a.wo = e.d_wo;
  a.drop_p = io.drop_p;
  a.drop_inv = io.drop_p > 0.f ? 1.f / (1.f - io.drop_p) : 1.f;
  a.drop_seed = io.drop_seed;
  a.step = io.step;
  const int grid = a.xcd_grp > 0 ? 8 * ((a.n_tiles + a.xcd_grp - 1) / a.xcd_grp)
                                  : a.n_tiles * e.K;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NW * 64), (uint32_t)lds, st, a);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

}  // namespace

// Kernel family: (precision, padded width, depth) -> instantiation.
// FP32: 16 walkers per workgroup, the units split over the waves (16 waves of
// one 16-unit tile at width 256).  16-bit: 64 walkers per workgroup (32 for
// deep networks or wide inputs) to cut the L2 weight stream per FLOP; 64
// units per wave.  g_out == nullptr: free energies only.
rid_status launch_mlp(const rid_ensemble_impl& e, const float* x, int B,
                      float* A_out, float* g_out, hipStream_t st) {
  return dispatch(e, x, B, A_out, g_out, nullptr, st);
}

bool hvp_fused_supported(const rid_ensemble_impl& e) {
  // plain MLPs on periodic inputs (residual and raw-CV ensembles take the
  // training sweeps in input mode)
  if (e.prec != RID_FP32 || e.NP > 256 || e.L > kMaxHidden || e.resnet || !e.raw.empty())
    return false;
  HvpArgs a{};
  return hvp_layout(e.NP, e.XP, e.n_cv, a) <= 160 * 1024;
}

rid_status launch_hvp(const rid_ensemble_impl& e, const float* x, const float* rho,
                      const float* coef, int B, float* T, hipStream_t st) {
  if (e.prec == RID_FP32) {
    switch (e.NP) {
      case 64:  return run_hvp<64>(e, x, rho, coef, B, T, st);
      case 128: return run_hvp<128>(e, x, rho, coef, B, T, st);
      case 256: return run_hvp<256>(e, x, rho, coef, B, T, st);
    }
  }
  return fail(RID_EUNSUPPORTED, "no fused HVP kernel for this ensemble");
}

bool train_fused_supported(const rid_ensemble_impl& e) {
  // plain MLPs on periodic inputs (residual and raw-CV ensembles take the
  // sweeps as separate GEMMs)
  if (e.prec != RID_FP32 || e.NP > 256 || e.L > kMaxHidden || e.resnet || !e.raw.empty())
    return false;
  TrainArgs a{};
  return train_layout(e.NP, e.XP, e.n_cv, a) <= 160 * 1024;
}

rid_status launch_train_sweeps(const rid_ensemble_impl& e, const TrainIo& io, int B,
                               hipStream_t st) {
  if (e.prec == RID_FP32) {
    switch (e.NP) {
      case 64:  return run_train<64>(e, io, B, st);
      case 128: return run_train<128>(e, io, B, st);
      case 256: return run_train<256>(e, io, B, st);
    }
  }
  return fail(RID_EUNSUPPORTED, "no fused training kernel for this ensemble");
}

rid_status launch_mlp_from_pos(const rid_ensemble_impl& e, const TorsionInput& tin,
                               int B, float* A_out, float* g_out, hipStream_t st) {
  // the in-kernel gather computes torsions only: systems with distance CVs
  // take the encoding from cv_eval_kernel
  if (tin.sys->has_dist) return RID_EUNSUPPORTED;
  return dispatch(e, nullptr, B, A_out, g_out, &tin, st);
}

rid_status pack_ensemble_weights(rid_ensemble_impl& e, hipStream_t st) {
  ++e.master_gen;     // the masters may have changed: copies made from them are stale
  const int L = e.L;
  PackAll pa{};
  pa.L = L;
  pa.K = e.K;
  pa.NP = e.NP;
  unsigned off = 0;
  int prev = 2 * e.n_cv;
  for (int l = 0; l < L; ++l) {
    PackLayer& pl = pa.layer[l];
    pl.w_off = off;
    pl.in = prev;
    pl.out = e.widths[l];
    off += (unsigned)(pl.out * pl.in);
    pl.b_off = off;
    pa.va.b_off[l] = off;
    pa.va.out[l] = pl.out;
    off += (unsigned)pl.out;
    pl.kin_pad = e.layers[l].kin_pad;
    pl.fwd_off = (unsigned)e.layers[l].fwd_off;
    pl.bwd_off = (unsigned)e.layers[l].bwd_off;
    // the plan's formats: first layer, hidden-layer forward, reverse sweep
    switch (e.prec) {
      case RID_BF16:
        pl.fmt_fwd = l == 0 ? kFmtF16 : kFmtBF16;
        pl.fmt_bwd = kFmtF16;
        break;
      case RID_FP16:
        pl.fmt_fwd = pl.fmt_bwd = kFmtF16;
        break;
      case RID_BF16_ALL:
        pl.fmt_fwd = pl.fmt_bwd = kFmtBF16;
        break;
      default:
        pl.fmt_fwd = pl.fmt_bwd = kFmtF32;
        break;
    }
    prev = pl.out;
  }
  pa.va.wo_off = off;
  pa.va.last_w = prev;
  pa.va.vscale_on = e.prec == RID_BF16 || e.prec == RID_FP16;
  const dim3 grid(256, 2 * L + 1), block(256);
  hipLaunchKernelGGL(pack_kernel, grid, block, 0, st, e.d_master, e.per_model, pa, e.d_frag,
                     e.frag_bytes_per_model, e.d_bias, e.d_wo, e.d_bo, e.d_vscale);
  RID_HIP(hipGetLastError());
  return RID_OK;
}

}  // namespace rid
