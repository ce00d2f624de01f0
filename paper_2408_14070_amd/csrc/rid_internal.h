// Internal declarations shared by the library's translation units.
// Not part of the public ABI (include/rid.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <hip/hip_bf16.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rid.h"

namespace rid {

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
rid_status fail(rid_status st, const std::string& msg);
inline rid_status hip_fail(hipError_t e, const char* what) {
  return fail(RID_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define RID_HIP(expr)                                        \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return ::rid::hip_fail(e_, #expr); \
  } while (0)

// Device buffer that grows on demand (never shrinks until destroyed).
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  rid_status ensure(size_t need);
  void release();
  template <class T> T* as() const { return static_cast<T*>(ptr); }
};

// ---------------------------------------------------------------------------
// optional kernel timing (rid_profile_enable): a pair of hipEvents around a
// launch on the launching stream; no synchronisation at record time.
// ---------------------------------------------------------------------------
enum ProfKind {
  kProfCv = 0, kProfMlp = 1, kProfScatter = 2, kProfReduce = 3, kProfEmbed = 4,
  kProfTrain = 5, kProfLabel = 6, kProfHvp = 7, kProfKinds = 8
};
bool prof_enabled();
hipEvent_t prof_event();                 // from the pool, not yet recorded
hipEvent_t prof_record(hipStream_t st);
void prof_push(int kind, hipEvent_t a, hipEvent_t b);

// Launch one kernel; when timing is on, its start and end timestamps are
// taken by the dispatch itself (hipExtLaunchKernelGGL events), so the
// measured time is the kernel's own and no marker packets sit between
// launches.
template <typename K, typename... Args>
inline void launch_timed(int kind, K kern, dim3 grid, dim3 block, uint32_t lds,
                         hipStream_t st, Args... args) {
  if (prof_enabled()) {
    hipEvent_t a = prof_event(), b = prof_event();
    if (a && b) {
      hipExtLaunchKernelGGL(kern, grid, block, lds, st, a, b, 0, args...);
      prof_push(kind, a, b);
      return;
    }
  }
  hipLaunchKernelGGL(kern, grid, block, lds, st, args...);
}
struct ProfScope {
  int kind;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(int k, hipStream_t s) : kind(k), st(s) {
    if (prof_enabled()) a = prof_record(st);
  }
  ~ProfScope() {
    if (a) prof_push(kind, a, prof_record(st));
  }
};

// ---------------------------------------------------------------------------
// MFMA fragment geometry shared by the weight packer and the kernels.
// A "fragment" covers 16 output columns x KF contraction indices and is
// stored as 64 lanes x 16 bytes: lane l holds column (l % 16) and the KF/4
// consecutive contraction indices starting at (KF/4) * (l / 16).
//   FP32 (v_mfma_f32_16x16x4_f32 issued four times): KF = 16, 4 floats/lane
//   BF16 / FP16 (v_mfma_f32_16x16x32_{bf16,f16}):    KF = 32, 8 values/lane
// ---------------------------------------------------------------------------
constexpr int kFragBytes = 1024;
inline int kf_of(rid_precision p) { return p == RID_FP32 ? 16 : 32; }
inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

constexpr int kMaxHidden = 6;
// default device budget of the training sweeps' stored activations (512 MiB)
constexpr size_t kTrainBudgetDefault = (size_t)512 << 20;
constexpr int kMaxWidth = 512;

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct LayerDev {
  // forward fragments: contraction = padded input width, columns = NP
  // backward fragments: contraction = NP, columns = padded input width
  size_t fwd_off = 0, bwd_off = 0;   // byte offsets inside frag buffer
  int kin_pad = 0;                   // padded input width of this layer
};

struct rid_system_impl {
  int n_atoms = 0, n_cv = 0;
  std::vector<int32_t> quads;        // host copy [n_cv][4]
  // unique atoms touched by torsions (sorted) and quads in local indices
  std::vector<int32_t> uniq;
  int n_uniq = 0;
  // The device tables below are consecutive pieces of ONE allocation, in
  // this order (uniq | lquads | csr_ptr | csr_ent | atom_local), so a kernel
  // can copy any prefix of them into LDS as one flat array.
  int32_t* d_tables = nullptr;
  int32_t* d_uniq = nullptr;         // [n_uniq]
  int32_t* d_lquads = nullptr;       // [n_cv][4] local indices into uniq
  // inverse map local atom -> (cv, slot) entries, CSR, fixed order
  int32_t* d_csr_ptr = nullptr;      // [n_uniq + 1]
  int32_t* d_csr_ent = nullptr;      // [4 n_cv] entry = cv * 4 + slot
  int32_t* d_atom_local = nullptr;   // [n_atoms] local index or -1
  int max_deg = 0;
  std::vector<uint8_t> mask;         // [n_cv] 1 = torsion (angular), 0 = distance pair
  bool has_dist = false;             // any distance row (lquads slots 2, 3 are -1)
};

struct rid_ensemble_impl {
  int n_cv = 0, K = 0, L = 0;
  std::vector<int> widths;
  rid_precision prec = RID_FP32;
  int NP = 0;        // padded hidden width (multiple of 64)
  int XP = 0;        // padded input width (multiple of KF)
  int KF = 16;
  size_t n_params = 0;          // packed count (all models)
  size_t per_model = 0;         // packed count of one model
  // FP32 masters in packed layout + Adam moments (device)
  float* d_master = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  int64_t step = 0;
  float drop_p = 0.f;                  // training-time dropout rate of the hidden activations
  unsigned long long drop_seed = 0;
  bool resnet = false;                 // residual connections between hidden layers 2..L
  // device bytes the training sweeps may hold for one pass over the batch:
  // larger batches are split into chunks of rows that fit it
  size_t train_budget = kTrainBudgetDefault;
  // angular mask of the inputs: CVs with raw[i] = 1 enter as (s_i, 0)
  std::vector<uint8_t> raw;            // [n_cv] (empty: every CV angular)
  uint8_t* d_raw = nullptr;            // device copy, or null when no CV is raw
  // per-CV clustering weights of the selection metric (empty: all 1)
  std::vector<float> cvw;              // [n_cv]
  float* d_cvw = nullptr;              // device copy, or null when every weight is 1
  // MCMC box of the raw CVs: lower [n], then upper [n] (null until set)
  std::vector<float> bounds;
  float* d_bounds = nullptr;
  // kernel-layout parameters
  std::vector<LayerDev> layers;
  size_t frag_bytes_per_model = 0;
  unsigned char* d_frag = nullptr;   // [K][frag_bytes_per_model]
  float* d_bias = nullptr;           // [K][L][NP] zero padded
  float* d_wo = nullptr;             // [K][NP]
  float* d_bo = nullptr;             // [K]
  float* d_vscale = nullptr;         // [K][2] reverse-vector scale (a power of two), inverse
  // the layer weights again, each member's block and each layer's matrix
  // starting on 16 bytes (the general training sweeps read their weight
  // operand from it with float4 loads); rebuilt when master_gen moves on
  DevBuf wpad;                       // [K][wpad_pm] floats
  long long wpad_pm = 0;
  std::vector<long long> wpad_off;   // [L] offset of W_l inside a member's block
  unsigned long long master_gen = 1, wpad_gen = 0;
  // scratch
  bool frag_dirty = false;           // masters changed since the last pack
  DevBuf ws_x, ws_A, ws_g, ws_train, ws_cons;
};

// ---------------------------------------------------------------------------
// kernel launchers (defined in the .hip files)
// ---------------------------------------------------------------------------
rid_status launch_cv_eval(const rid_system_impl& s, const float* pos, int B,
                          float* d_s, float* d_x, hipStream_t st);
// x = [cos s | sin s]; CVs with raw[i] = 1 (raw may be null) as (s_i, 0)
rid_status launch_embed(const float* s, int B, int n, const uint8_t* raw, float* x,
                        hipStream_t st);
// The system's CV kinds must match the ensemble's angular mask (distance rows
// raw, torsion rows angular).
inline bool cv_kinds_match(const rid_system_impl& s, const rid_ensemble_impl& e) {
  for (int i = 0; i < s.n_cv; ++i) {
    const bool dist = s.has_dist && s.mask[i] == 0;
    const bool raw = !e.raw.empty() && e.raw[i] != 0;
    if (dist != raw) return false;
  }
  return true;
}
// Ensemble MLP fed straight from atom positions (torsions computed in-kernel).
struct TorsionInput {
  const rid_system_impl* sys;
  const float* pos;
};
rid_status launch_mlp_from_pos(const rid_ensemble_impl& e, const TorsionInput& tin,
                               int B, float* A_out, float* g_out, hipStream_t st);
// g_out == nullptr: the free energies only (no reverse sweep).
rid_status launch_mlp(const rid_ensemble_impl& e, const float* x, int B,
                      float* A_out, float* g_out, hipStream_t st);
// Fused Hessian-vector products of conservative switching: per member k the
// term T [K][B][n] of d eps/ds, from the encoding x [B][2n], w_k in
// rho [B][K][n] and the walkers' Abar sigma' in coef [B] (tiles with no
// walker in the band are skipped and their T left unwritten).  FP32
// ensembles of padded width <= 256 only (hvp_fused_supported).
bool hvp_fused_supported(const rid_ensemble_impl& e);
rid_status launch_hvp(const rid_ensemble_impl& e, const float* x, const float* rho,
                      const float* coef, int B, float* T, hipStream_t st);
// Fused sweeps of one mean-force training step (FP32 ensembles of padded
// width <= 256, train_fused_supported): from the samples s [B][n] and labels
// F [B][n] (or an upstream gradient rho [B][K][n] of the g outputs), writes
// hh[j] = [h_j ; hd_j] (j = 0: [x ; rho_x]) and sl[j] = [lam_z ; lam_zd] of
// layer j, each [K][2B][width], and the squared residual per sample
// loss_rows [K][B] (labels only).  The fragments must be packed from the
// current masters.
struct TrainIo {
  const float* s;
  const float* F;
  const float* rho;
  float* hh[kMaxHidden + 1];
  float* sl[kMaxHidden];
  float* loss_rows;                 // row b of member k at loss_rows[k * loss_ld + b]
  long long loss_ld;
  int row_base;                     // batch index of row 0 (a chunk of a larger batch)
  int B_norm;                       // the whole batch's size: rho = 2 (g - F) / B_norm
  float drop_p;                     // dropout rate (0: none)
  unsigned long long drop_seed;
  uint32_t step;                    // training step (mask counter)
};
// Threshold clustering of CV frames (selection); synchronises the stream.
// Copies the first min(leaders, leaders_out) leaders' frame indices.
rid_status launch_cluster(const float* s, int B, int n, const uint8_t* raw,
                          const float* w, const float* eps,
                          float eps0, float threshold, int lower, int upper, int adapt, int cap,
                          int* labels, int* leaders, int leaders_out, int* n_leaders,
                          int* n_clusters, float* t_used, hipStream_t st);
bool train_fused_supported(const rid_ensemble_impl& e);
rid_status launch_train_sweeps(const rid_ensemble_impl& e, const TrainIo& io, int B,
                               hipStream_t st);
rid_status launch_ensemble_reduce(int K, int n, int B, const float* A,
                                  const float* g, float* eps, float* gbar,
                                  float* A_t, float* g_t, hipStream_t st);
rid_status launch_bias_scatter(const rid_system_impl& s, int K, const float* pos,
                               int B, const float* A, const float* g,
                               const float* fcv, float eps0, float eps1,
                               float* force, float* energy, float* eps,
                               float* sigma, uint8_t* flags, hipStream_t st,
                               int rec_stride = 0);
// rec_stride > 0: walker records -- walker w's forces start at
// force + w * rec_stride and energy/eps/sigma use the same stride.
rid_status pack_ensemble_weights(rid_ensemble_impl& e, hipStream_t st);
// Input mode of the mean-force sweeps: with an upstream gradient rho
// [B][K][n], J_k = sum_b rho_kb . g_k(s_b) differentiated in the network
// input x with rho_x held fixed.  Results point into the ensemble's training
// workspace: lam_x [K][2B][2n] (rows [0, B) of member k hold d J_k / dx,
// member stride slab_lam) and u0 [K][B][2n] (dA_k/dx).
struct InputHvp {
  const float* lam_x = nullptr;
  const float* u0 = nullptr;
  long long slab_lam = 0;
};
rid_status launch_mf_grad(rid_ensemble_impl& e, const float* s, const float* F,
                          const float* rho, int B, float* loss, float* grad_out,
                          float** grad_used, hipStream_t st, InputHvp* hvp = nullptr);
rid_status launch_mcmc(rid_ensemble_impl& e, float* s, int W, long long n_steps, long long t0,
                       double kT, float step, unsigned long long seed, int proj0, int proj1,
                       int nbins, unsigned* hist1, unsigned* hist2,
                       unsigned long long* accepted, hipStream_t st);
rid_status launch_bias_conservative(const rid_system_impl& s, rid_ensemble_impl& e,
                                    const float* pos, int B, float eps0, float eps1,
                                    float* force, float* energy, float* eps, float* sigma,
                                    uint8_t* flags, hipStream_t st);
rid_status launch_train_step(rid_ensemble_impl& e, const float* s,
                             const float* F, int B, float lr, float* loss,
                             hipStream_t st);
// The bias path (rid_bias_force) with its scratch given: A [K][B], g
// [K][B][n], and x [B][2n] for the encoding when it goes through memory
// (null: taken from the ensemble's workspace, grown on demand).
rid_status bias_force_core(rid_system_impl& s, rid_ensemble_impl& e, const float* d_pos,
                           int B, float eps0, float eps1, float* A, float* g, float* x,
                           float* d_force, float* d_energy, float* d_eps, float* d_sigma,
                           uint8_t* d_flags, hipStream_t st);
rid_status launch_mf_label_impl(const float* traj, const float* s0,
                                const float* kappa, const uint8_t* mask, int M,
                                int T, int n, float thr, double* F, double* se,
                                uint8_t* keep, hipStream_t st);

}  // namespace rid

// Public handle types (opaque in include/rid.h).
struct rid_system_s {
  rid::rid_system_impl impl;
};
struct rid_ensemble_s {
  rid::rid_ensemble_impl impl;
};

namespace rid {
// Argument checks of rid_bias_force (and its no-allocation variant).
rid_status bias_force_check(const rid_system_s* sys, const rid_ensemble_s* ens,
                            const float* d_pos, int B, float eps0, float eps1,
                            const float* d_force);
}  // namespace rid
