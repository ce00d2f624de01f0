// C ABI of the library (declarations and contracts: include/rid.h).
// Host-side validation, handle construction and kernel sequencing only; all
// arithmetic of the path runs in the kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "rid_internal.h"

namespace rid {

static thread_local std::string g_err;

rid_status fail(rid_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

rid_status DevBuf::ensure(size_t need) {
  if (need <= bytes && ptr) return RID_OK;
  release();
  if (need == 0) need = 256;
  if (hipMalloc(&ptr, need) != hipSuccess) {
    ptr = nullptr;
    bytes = 0;
    (void)hipGetLastError();
    return fail(RID_ENOMEM, "device allocation of scratch memory failed");
  }
  bytes = need;
  return RID_OK;
}

void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

// ---- kernel timing -------------------------------------------------------
static std::mutex g_prof_mu;
static bool g_prof_on = false;
struct ProfPair {
  int kind;
  hipEvent_t a, b;
};
static std::vector<ProfPair> g_prof;
static std::vector<hipEvent_t> g_pool;

bool prof_enabled() { return g_prof_on; }

hipEvent_t prof_event() {
  hipEvent_t e = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_pool.empty()) {
      e = g_pool.back();
      g_pool.pop_back();
    }
  }
  if (!e && hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

hipEvent_t prof_record(hipStream_t st) {
  hipEvent_t e = prof_event();
  if (!e || hipEventRecord(e, st) != hipSuccess) return nullptr;
  return e;
}

void prof_push(int kind, hipEvent_t a, hipEvent_t b) {
  if (!a || !b) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.push_back({kind, a, b});
}

static void prof_recycle_locked() {
  for (auto& p : g_prof) {
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_prof.clear();
}

template <class T>
static rid_status dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(RID_ENOMEM, "device allocation failed");
  }
  return RID_OK;
}

template <class T>
static void dev_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

static size_t per_model_count(int n_cv, int L, const int* widths) {
  size_t per = 0;
  int prev = 2 * n_cv;
  for (int l = 0; l < L; ++l) {
    per += (size_t)widths[l] * prev + widths[l];
    prev = widths[l];
  }
  return per + prev + 1;
}

static void free_system(rid_system_impl& s) {
  dev_free(s.d_tables);
  s.d_uniq = s.d_lquads = s.d_csr_ptr = s.d_csr_ent = s.d_atom_local = nullptr;
}

static void free_ensemble(rid_ensemble_impl& e) {
  dev_free(e.d_master);
  dev_free(e.d_m);
  dev_free(e.d_v);
  dev_free(e.d_frag);
  dev_free(e.d_bias);
  dev_free(e.d_wo);
  dev_free(e.d_bo);
  dev_free(e.d_vscale);
  dev_free(e.d_raw);
  dev_free(e.d_cvw);
  dev_free(e.d_bounds);
  e.ws_x.release();
  e.wpad.release();
  e.ws_A.release();
  e.ws_g.release();
  e.ws_train.release();
  e.ws_cons.release();
}

}  // namespace rid

using namespace rid;

// Batches up to this many walkers gather torsion atoms inside the MLP kernel
// (one launch less); larger ones encode the CVs once into HBM first, so the
// K members' workgroups read a compact [B][2n] encoding instead of each
// re-reading the positions.
#ifndef RID_FROM_POS_MAX_B
#define RID_FROM_POS_MAX_B 4096
#endif

namespace rid {

rid_status bias_force_check(const rid_system_s* sys, const rid_ensemble_s* ens,
                            const float* d_pos, int B, float eps0, float eps1,
                            const float* d_force) {
  if (!sys || !ens || !d_pos || !d_force) return fail(RID_EINVAL, "NULL argument");
  if (B < 1) return fail(RID_EINVAL, "B must be >= 1");
  if (!(eps0 >= 0.f) || !(eps0 < eps1))
    return fail(RID_EINVAL, "trust levels need 0 <= eps0 < eps1");
  if (sys->impl.n_cv != ens->impl.n_cv)
    return fail(RID_EINVAL, "system and ensemble disagree on n_cv");
  if (!cv_kinds_match(sys->impl, ens->impl))
    return fail(RID_EINVAL, "the ensemble's angular mask does not match the system's CV kinds");
  return RID_OK;
}

rid_status bias_force_core(rid_system_impl& s, rid_ensemble_impl& e, const float* d_pos,
                           int B, float eps0, float eps1, float* A, float* g, float* x,
                           float* d_force, float* d_energy, float* d_eps, float* d_sigma,
                           uint8_t* d_flags, hipStream_t st) {
  rid_status r;
  if (e.frag_dirty) {
    if ((r = pack_ensemble_weights(e, st)) != RID_OK) return r;
    e.frag_dirty = false;
  }
  const TorsionInput tin{&s, d_pos};
  r = B <= RID_FROM_POS_MAX_B ? launch_mlp_from_pos(e, tin, B, A, g, st) : RID_EUNSUPPORTED;
  if (r == RID_EUNSUPPORTED) {
    // large batch, or too many torsion atoms for the in-kernel gather:
    // encode in HBM first
    if (!x) {
      if ((r = e.ws_x.ensure(sizeof(float) * 2 * e.n_cv * (size_t)B)) != RID_OK) return r;
      x = e.ws_x.as<float>();
    }
    if ((r = launch_cv_eval(s, d_pos, B, nullptr, x, st)) != RID_OK) return r;
    r = launch_mlp(e, x, B, A, g, st);
  }
  if (r != RID_OK) return r;
  return launch_bias_scatter(s, e.K, d_pos, B, A, g, nullptr, eps0, eps1, d_force, d_energy,
                             d_eps, d_sigma, d_flags, st);
}

}  // namespace rid

extern "C" {

const char* rid_last_error(void) { return g_err.c_str(); }

const char* rid_version(void) { return "rid-mi355x 0.1 (gfx950)"; }

rid_status rid_system_create(int n_atoms, int n_cv, const int32_t* quads,
                             const uint8_t* angular_mask, rid_system* out) {
  if (!out) return fail(RID_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_atoms < 1 || n_cv < 1 || !quads)
    return fail(RID_EINVAL, "need n_atoms >= 1, n_cv >= 1 and a quad table");
  if (n_cv > 256) return fail(RID_EUNSUPPORTED, "at most 256 CVs");
  for (int i = 0; i < n_cv; ++i) {
    if (angular_mask && angular_mask[i] > 1)
      return fail(RID_EINVAL, "angular_mask entries must be 0 or 1");
    // a torsion row names 4 atoms; a distance row (mask 0) names 2, then -1, -1
    const int na = (angular_mask && angular_mask[i] == 0) ? 2 : 4;
    for (int j = 0; j < 4; ++j) {
      const int a = quads[4 * i + j];
      if (j >= na) {
        if (a != -1)
          return fail(RID_EINVAL, "distance row " + std::to_string(i) + " must end in -1, -1");
        continue;
      }
      if (a < 0 || a >= n_atoms)
        return fail(RID_EINVAL, "quad " + std::to_string(i) + " has an atom index out of range");
      for (int j2 = 0; j2 < j; ++j2)
        if (quads[4 * i + j2] == a)
          return fail(RID_EINVAL, "quad " + std::to_string(i) + " repeats an atom");
    }
  }
  rid_system_s* h = new (std::nothrow) rid_system_s();
  if (!h) return fail(RID_ENOMEM, "host allocation failed");
  rid_system_impl& s = h->impl;
  s.n_atoms = n_atoms;
  s.n_cv = n_cv;
  s.quads.assign(quads, quads + 4 * (size_t)n_cv);
  s.mask.assign(n_cv, 1);
  for (int i = 0; i < n_cv; ++i)
    if (angular_mask && angular_mask[i] == 0) {
      s.mask[i] = 0;
      s.has_dist = true;
    }
  s.uniq.clear();
  for (int32_t a : s.quads)
    if (a >= 0) s.uniq.push_back(a);
  std::sort(s.uniq.begin(), s.uniq.end());
  s.uniq.erase(std::unique(s.uniq.begin(), s.uniq.end()), s.uniq.end());
  s.n_uniq = (int)s.uniq.size();
  std::vector<int32_t> atom_local(n_atoms, -1);
  for (int u = 0; u < s.n_uniq; ++u) atom_local[s.uniq[u]] = u;
  // local indices; the -1 slots of distance rows stay -1 (the kernels'
  // marker of a distance CV)
  std::vector<int32_t> lq(4 * (size_t)n_cv);
  for (size_t e = 0; e < lq.size(); ++e) lq[e] = s.quads[e] >= 0 ? atom_local[s.quads[e]] : -1;
  // CSR inverse map in (cv, slot) order over the rows' atoms.  The entry
  // array keeps 4 n_cv slots whatever the rows (the kernels copy the tables
  // with that layout); a distance row leaves two of them unused at the end,
  // past csr_ptr[n_uniq].
  std::vector<int32_t> ptr(s.n_uniq + 1, 0), ent(4 * (size_t)n_cv, 0);
  for (size_t e = 0; e < lq.size(); ++e)
    if (lq[e] >= 0) ptr[lq[e] + 1]++;
  for (int u = 0; u < s.n_uniq; ++u) {
    s.max_deg = std::max(s.max_deg, ptr[u + 1]);
    ptr[u + 1] += ptr[u];
  }
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  for (size_t e = 0; e < lq.size(); ++e)
    if (lq[e] >= 0) ent[fill[lq[e]]++] = (int32_t)e;
  // one allocation: uniq | lquads | csr_ptr | csr_ent | atom_local
  std::vector<int32_t> tab;
  tab.reserve(s.uniq.size() + lq.size() + ptr.size() + ent.size() + atom_local.size());
  tab.insert(tab.end(), s.uniq.begin(), s.uniq.end());
  tab.insert(tab.end(), lq.begin(), lq.end());
  tab.insert(tab.end(), ptr.begin(), ptr.end());
  tab.insert(tab.end(), ent.begin(), ent.end());
  tab.insert(tab.end(), atom_local.begin(), atom_local.end());
  rid_status st = dev_alloc(&s.d_tables, tab.size());
  if (st != RID_OK) {
    delete h;
    return st;
  }
  s.d_uniq = s.d_tables;
  s.d_lquads = s.d_uniq + s.uniq.size();
  s.d_csr_ptr = s.d_lquads + lq.size();
  s.d_csr_ent = s.d_csr_ptr + ptr.size();
  s.d_atom_local = s.d_csr_ent + ent.size();
  const hipError_t e =
      hipMemcpy(s.d_tables, tab.data(), 4 * tab.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_system(s);
    delete h;
    return hip_fail(e, "rid_system_create upload");
  }
  *out = h;
  return RID_OK;
}

void rid_system_destroy(rid_system sys) {
  if (!sys) return;
  (void)hipDeviceSynchronize();
  free_system(sys->impl);
  delete sys;
}

size_t rid_packed_param_count(int n_cv, int n_models, int n_hidden,
                              const int* widths) {
  if (n_cv < 1 || n_models < 1 || n_hidden < 0 || (n_hidden > 0 && !widths)) return 0;
  return per_model_count(n_cv, n_hidden, widths) * (size_t)n_models;
}

rid_status rid_ensemble_create(int n_cv, int n_models, int n_hidden,
                               const int* widths, rid_precision prec,
                               const float* params, rid_ensemble* out) {
  if (!out) return fail(RID_EINVAL, "out is NULL");
  *out = nullptr;
  if (!params || !widths) return fail(RID_EINVAL, "params and widths are required");
  if (prec != RID_FP32 && prec != RID_BF16 && prec != RID_FP16 && prec != RID_BF16_ALL)
    return fail(RID_EINVAL, "unknown precision");
  if (n_cv < 1 || n_cv > 256) return fail(RID_EUNSUPPORTED, "n_cv must be in [1, 256]");
  if (n_models < 1 || n_models > 64) return fail(RID_EUNSUPPORTED, "n_models must be in [1, 64]");
  if (n_hidden < 1 || n_hidden > kMaxHidden)
    return fail(RID_EUNSUPPORTED, "n_hidden must be in [1, 6]");
  int wmax = 0;
  for (int l = 0; l < n_hidden; ++l) {
    if (widths[l] < 1 || widths[l] > kMaxWidth)
      return fail(RID_EUNSUPPORTED, "hidden widths must be in [1, 512]");
    wmax = std::max(wmax, widths[l]);
  }
  rid_ensemble_s* h = new (std::nothrow) rid_ensemble_s();
  if (!h) return fail(RID_ENOMEM, "host allocation failed");
  rid_ensemble_impl& e = h->impl;
  e.n_cv = n_cv;
  e.K = n_models;
  e.L = n_hidden;
  e.widths.assign(widths, widths + n_hidden);
  e.prec = prec;
  e.KF = kf_of(prec);
  // the MLP kernels exist for padded widths 64, 128, 256 and 512 (zero
  // units pad the rest: their weights, biases and outputs stay 0)
  e.NP = wmax <= 64 ? 64 : wmax <= 128 ? 128 : wmax <= 256 ? 256 : 512;
  e.XP = round_up(2 * n_cv, e.KF);
  e.per_model = per_model_count(n_cv, n_hidden, widths);
  e.n_params = e.per_model * n_models;
  e.layers.resize(n_hidden);
  size_t off = 0;
  for (int l = 0; l < n_hidden; ++l) {
    LayerDev& ld = e.layers[l];
    ld.kin_pad = l == 0 ? e.XP : e.NP;
    ld.fwd_off = off;
    off += (size_t)(ld.kin_pad / e.KF) * (e.NP / 16) * kFragBytes;
    ld.bwd_off = off;
    off += (size_t)(e.NP / e.KF) * (ld.kin_pad / 16) * kFragBytes;
  }
  e.frag_bytes_per_model = off;
  rid_status st = RID_OK;
  if ((st = dev_alloc(&e.d_master, e.n_params)) != RID_OK ||
      (st = dev_alloc(&e.d_m, e.n_params)) != RID_OK ||
      (st = dev_alloc(&e.d_v, e.n_params)) != RID_OK ||
      (st = dev_alloc(&e.d_frag, e.frag_bytes_per_model * n_models)) != RID_OK ||
      (st = dev_alloc(&e.d_bias, (size_t)n_models * n_hidden * e.NP)) != RID_OK ||
      (st = dev_alloc(&e.d_wo, (size_t)n_models * e.NP)) != RID_OK ||
      (st = dev_alloc(&e.d_bo, (size_t)n_models)) != RID_OK ||
      (st = dev_alloc(&e.d_vscale, (size_t)2 * n_models)) != RID_OK) {
    free_ensemble(e);
    delete h;
    return st;
  }
  hipError_t he = hipMemcpy(e.d_master, params, e.n_params * 4, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemset(e.d_m, 0, e.n_params * 4);
  if (he == hipSuccess) he = hipMemset(e.d_v, 0, e.n_params * 4);
  if (he != hipSuccess) {
    free_ensemble(e);
    delete h;
    return hip_fail(he, "rid_ensemble_create upload");
  }
  st = pack_ensemble_weights(e, nullptr);
  if (st == RID_OK) {
    he = hipStreamSynchronize(nullptr);
    if (he != hipSuccess) st = hip_fail(he, "rid_ensemble_create pack");
  }
  if (st != RID_OK) {
    free_ensemble(e);
    delete h;
    return st;
  }
  *out = h;
  return RID_OK;
}

rid_status rid_ensemble_get_params(rid_ensemble ens, float* host_params) {
  if (!ens || !host_params) return fail(RID_EINVAL, "NULL argument");
  RID_HIP(hipDeviceSynchronize());
  RID_HIP(hipMemcpy(host_params, ens->impl.d_master, ens->impl.n_params * 4,
                    hipMemcpyDeviceToHost));
  return RID_OK;
}

rid_status rid_ensemble_set_params(rid_ensemble ens, const float* host_params) {
  if (!ens || !host_params) return fail(RID_EINVAL, "NULL argument");
  rid_ensemble_impl& e = ens->impl;
  RID_HIP(hipDeviceSynchronize());
  RID_HIP(hipMemcpy(e.d_master, host_params, e.n_params * 4, hipMemcpyHostToDevice));
  RID_HIP(hipMemset(e.d_m, 0, e.n_params * 4));
  RID_HIP(hipMemset(e.d_v, 0, e.n_params * 4));
  e.step = 0;
  rid_status st = pack_ensemble_weights(e, nullptr);
  if (st != RID_OK) return st;
  RID_HIP(hipStreamSynchronize(nullptr));
  return RID_OK;
}

rid_status rid_ensemble_load_params(rid_ensemble ens, const float* d_params,
                                    rid_stream stream) {
  if (!ens || !d_params) return fail(RID_EINVAL, "NULL argument");
  rid_ensemble_impl& e = ens->impl;
  hipStream_t st = (hipStream_t)stream;
  if (d_params != e.d_master)
    RID_HIP(hipMemcpyAsync(e.d_master, d_params, e.n_params * 4, hipMemcpyDeviceToDevice, st));
  rid_status r = pack_ensemble_weights(e, st);
  if (r != RID_OK) return r;
  e.frag_dirty = false;
  return RID_OK;
}

int64_t rid_ensemble_step(rid_ensemble ens) { return ens ? ens->impl.step : -1; }

rid_status rid_ensemble_set_dropout(rid_ensemble ens, float rate, uint64_t seed) {
  if (!ens) return fail(RID_EINVAL, "NULL argument");
  if (!(rate >= 0.f && rate < 1.f)) return fail(RID_EINVAL, "dropout rate must be in [0, 1)");
  ens->impl.drop_p = rate;
  ens->impl.drop_seed = seed;
  return RID_OK;
}

rid_status rid_ensemble_set_train_budget(rid_ensemble ens, size_t bytes) {
  if (!ens) return fail(RID_EINVAL, "NULL argument");
  ens->impl.train_budget = bytes ? bytes : kTrainBudgetDefault;
  return RID_OK;
}

rid_status rid_ensemble_set_cv_bounds(rid_ensemble ens, const float* lower,
                                      const float* upper) {
  if (!ens) return fail(RID_EINVAL, "NULL argument");
  rid_ensemble_impl& e = ens->impl;
  if ((lower == nullptr) != (upper == nullptr))
    return fail(RID_EINVAL, "give both bounds or neither");
  std::vector<float> b;
  if (lower) {
    b.resize(2 * (size_t)e.n_cv);
    for (int i = 0; i < e.n_cv; ++i) {
      if (!std::isfinite(lower[i]) || !std::isfinite(upper[i]) || !(lower[i] < upper[i]))
        return fail(RID_EINVAL, "every CV needs finite bounds with lower < upper");
      b[i] = lower[i];
      b[e.n_cv + i] = upper[i];
    }
  }
  RID_HIP(hipDeviceSynchronize());   // calls in flight may still read the old bounds
  dev_free(e.d_bounds);
  e.bounds.clear();
  if (b.empty()) return RID_OK;
  rid_status st = dev_alloc(&e.d_bounds, b.size());
  if (st != RID_OK) return st;
  RID_HIP(hipMemcpy(e.d_bounds, b.data(), b.size() * sizeof(float), hipMemcpyHostToDevice));
  e.bounds = b;
  return RID_OK;
}

rid_status rid_ensemble_set_angular_mask(rid_ensemble ens, const uint8_t* angular_mask) {
  if (!ens) return fail(RID_EINVAL, "NULL argument");
  rid_ensemble_impl& e = ens->impl;
  std::vector<uint8_t> raw;
  bool any = false;
  if (angular_mask) {
    raw.resize(e.n_cv);
    for (int i = 0; i < e.n_cv; ++i) {
      if (angular_mask[i] > 1) return fail(RID_EINVAL, "angular_mask entries must be 0 or 1");
      raw[i] = angular_mask[i] == 0;
      any = any || raw[i];
    }
  }
  RID_HIP(hipDeviceSynchronize());   // calls in flight may still read the old mask
  dev_free(e.d_raw);
  e.raw.clear();
  if (!any) return RID_OK;
  rid_status st = dev_alloc(&e.d_raw, (size_t)e.n_cv);
  if (st != RID_OK) return st;
  RID_HIP(hipMemcpy(e.d_raw, raw.data(), (size_t)e.n_cv, hipMemcpyHostToDevice));
  e.raw = raw;
  return RID_OK;
}

rid_status rid_ensemble_set_cv_weights(rid_ensemble ens, const float* weights) {
  if (!ens) return fail(RID_EINVAL, "NULL argument");
  rid_ensemble_impl& e = ens->impl;
  std::vector<float> w;
  bool all_one = true;
  if (weights) {
    w.assign(weights, weights + e.n_cv);
    for (float v : w) {
      if (!std::isfinite(v) || v < 0.f)
        return fail(RID_EINVAL, "CV weights must be finite and non-negative");
      all_one = all_one && v == 1.f;
    }
  }
  RID_HIP(hipDeviceSynchronize());   // calls in flight may still read the old weights
  dev_free(e.d_cvw);
  e.cvw.clear();
  if (all_one) return RID_OK;         // every weight 1: the unweighted metric, bit for bit
  rid_status st = dev_alloc(&e.d_cvw, sizeof(float) * (size_t)e.n_cv);
  if (st != RID_OK) return st;
  RID_HIP(hipMemcpy(e.d_cvw, w.data(), sizeof(float) * (size_t)e.n_cv, hipMemcpyHostToDevice));
  e.cvw = w;
  return RID_OK;
}

rid_status rid_adjust_trust_levels(int n_clusters, int numb_cluster_threshold, float scale,
                                   float* trust_lvl_1, float* trust_lvl_2) {
  if (!trust_lvl_1 || !trust_lvl_2) return fail(RID_EINVAL, "NULL argument");
  if (!std::isfinite(scale) || !(scale > 1.f)) return fail(RID_EINVAL, "scale must be finite and > 1");
  const float l1 = *trust_lvl_1, l2 = *trust_lvl_2;
  if (!std::isfinite(l1) || !std::isfinite(l2) || !(l1 >= 0.f) || !(l1 < l2))
    return fail(RID_EINVAL, "trust levels must satisfy 0 <= lvl_1 < lvl_2");
  if (n_clusters < numb_cluster_threshold) {
    *trust_lvl_1 = l1 * scale;
    *trust_lvl_2 = l2 * scale;
  }
  return RID_OK;
}

rid_status rid_ensemble_set_resnet(rid_ensemble ens, int enable) {
  if (!ens) return fail(RID_EINVAL, "NULL argument");
  const rid_ensemble_impl& e = ens->impl;
  if (enable) {
    for (int w : e.widths)
      if (w != e.widths[0])
        return fail(RID_EINVAL, "residual connections need hidden layers of equal width");
    if (e.prec != RID_FP32)
      return fail(RID_EUNSUPPORTED, "residual connections need an FP32 ensemble");
  }
  ens->impl.resnet = enable != 0;
  return RID_OK;
}

void rid_ensemble_destroy(rid_ensemble ens) {
  if (!ens) return;
  (void)hipDeviceSynchronize();
  free_ensemble(ens->impl);
  delete ens;
}

rid_status rid_cv_eval(rid_system sys, const float* d_pos, int B, float* d_s,
                       float* d_x, rid_stream stream) {
  if (!sys || !d_pos || !d_s) return fail(RID_EINVAL, "NULL argument");
  if (B < 1) return fail(RID_EINVAL, "B must be >= 1");
  return launch_cv_eval(sys->impl, d_pos, B, d_s, d_x, (hipStream_t)stream);
}

rid_status rid_model_dev(rid_ensemble ens, const float* d_s, int B, float* d_eps,
                         float* d_gbar, float* d_A, float* d_g,
                         rid_stream stream) {
  if (!ens || !d_s || !d_eps) return fail(RID_EINVAL, "NULL argument");
  if (B < 1) return fail(RID_EINVAL, "B must be >= 1");
  rid_ensemble_impl& e = ens->impl;
  const hipStream_t st = (hipStream_t)stream;
  rid_status r;
  if ((r = e.ws_x.ensure(sizeof(float) * 2 * e.n_cv * (size_t)B)) != RID_OK) return r;
  if ((r = e.ws_A.ensure(sizeof(float) * e.K * (size_t)B)) != RID_OK) return r;
  if ((r = e.ws_g.ensure(sizeof(float) * e.K * (size_t)B * e.n_cv)) != RID_OK) return r;
  if ((r = launch_embed(d_s, B, e.n_cv, e.d_raw, e.ws_x.as<float>(), st)) != RID_OK) return r;
  if (e.frag_dirty) {
    if ((r = pack_ensemble_weights(e, st)) != RID_OK) return r;
    e.frag_dirty = false;
  }
  if ((r = launch_mlp(e, e.ws_x.as<float>(), B, e.ws_A.as<float>(), e.ws_g.as<float>(), st)) != RID_OK)
    return r;
  return launch_ensemble_reduce(e.K, e.n_cv, B, e.ws_A.as<float>(), e.ws_g.as<float>(),
                                d_eps, d_gbar, d_A, d_g, st);
}

rid_status rid_cluster_frames(const float* d_s, int B, int n_cv, const float* d_eps,
                              float eps0, float threshold, int adapt, int lower, int upper,
                              int max_clusters, int* d_labels, int* d_leaders,
                              int* n_clusters, float* threshold_used, rid_stream stream) {
  if (!d_s || !d_labels || !d_leaders || !n_clusters) return fail(RID_EINVAL, "NULL argument");
  if (B < 1) return fail(RID_EINVAL, "B must be >= 1");
  if (n_cv < 1 || n_cv > 256) return fail(RID_EINVAL, "n_cv must be in [1, 256]");
  if (!(threshold > 0.f) || !std::isfinite(threshold))
    return fail(RID_EINVAL, "threshold must be positive and finite");
  if (max_clusters < 1) return fail(RID_EINVAL, "max_clusters must be >= 1");
  if (adapt && (lower < 1 || upper < lower)) return fail(RID_EINVAL, "need 1 <= lower <= upper");
  return launch_cluster(d_s, B, n_cv, nullptr, nullptr, d_eps, eps0, threshold, lower, upper,
                        adapt, max_clusters, d_labels, d_leaders, max_clusters, nullptr,
                        n_clusters, threshold_used, (hipStream_t)stream);
}

rid_status rid_select(rid_ensemble ens, const float* d_s, int B, float eps0, float threshold,
                      int adapt, int lower, int upper, int max_selection, float* d_eps,
                      int* d_labels, int* d_selected, int* n_selected, int* n_clusters,
                      float* threshold_used, rid_stream stream) {
  if (!ens || !d_s || !d_eps || !d_labels || !d_selected || !n_selected || !n_clusters)
    return fail(RID_EINVAL, "NULL argument");
  if (B < 1) return fail(RID_EINVAL, "B must be >= 1");
  if (!(threshold > 0.f) || !std::isfinite(threshold))
    return fail(RID_EINVAL, "threshold must be positive and finite");
  if (lower < 1 || upper < lower) return fail(RID_EINVAL, "need 1 <= lower <= upper");
  if (max_selection < 1) return fail(RID_EINVAL, "max_selection must be >= 1");
  rid_status r = rid_model_dev(ens, d_s, B, d_eps, nullptr, nullptr, nullptr, stream);
  if (r != RID_OK) return r;
  const int cap = std::max(upper, max_selection) + 1;
  return launch_cluster(d_s, B, ens->impl.n_cv, ens->impl.d_raw, ens->impl.d_cvw, d_eps, eps0,
                        threshold, lower, upper, adapt, cap, d_labels, d_selected, max_selection,
                        n_selected, n_clusters, threshold_used, (hipStream_t)stream);
}



rid_status rid_bias_force(rid_system sys, rid_ensemble ens, const float* d_pos,
                          int B, float eps0, float eps1, float* d_force,
                          float* d_energy, float* d_eps, float* d_sigma,
                          uint8_t* d_flags, rid_stream stream) {
  rid_status r = bias_force_check(sys, ens, d_pos, B, eps0, eps1, d_force);
  if (r != RID_OK) return r;
  rid_ensemble_impl& e = ens->impl;
  if ((r = e.ws_A.ensure(sizeof(float) * e.K * (size_t)B)) != RID_OK) return r;
  if ((r = e.ws_g.ensure(sizeof(float) * e.K * (size_t)B * e.n_cv)) != RID_OK) return r;
  return bias_force_core(sys->impl, e, d_pos, B, eps0, eps1, e.ws_A.as<float>(),
                         e.ws_g.as<float>(), nullptr, d_force, d_energy, d_eps, d_sigma,
                         d_flags, (hipStream_t)stream);
}

rid_status rid_bias_force_conservative(rid_system sys, rid_ensemble ens,
                                       const float* d_pos, int B, float eps0,
                                       float eps1, float* d_force, float* d_energy,
                                       float* d_eps, float* d_sigma, uint8_t* d_flags,
                                       rid_stream stream) {
  if (!sys || !ens || !d_pos || !d_force) return fail(RID_EINVAL, "NULL argument");
  if (B < 1) return fail(RID_EINVAL, "B must be >= 1");
  if (!(eps0 >= 0.f) || !(eps0 < eps1))
    return fail(RID_EINVAL, "trust levels need 0 <= eps0 < eps1");
  if (sys->impl.n_cv != ens->impl.n_cv)
    return fail(RID_EINVAL, "system and ensemble disagree on n_cv");
  if (!cv_kinds_match(sys->impl, ens->impl))
    return fail(RID_EINVAL, "the ensemble's angular mask does not match the system's CV kinds");
  return launch_bias_conservative(sys->impl, ens->impl, d_pos, B, eps0, eps1, d_force,
                                  d_energy, d_eps, d_sigma, d_flags, (hipStream_t)stream);
}

rid_status rid_mcmc_run(rid_ensemble ens, float* d_s, int W, int64_t n_steps,
                        int64_t step0, double kT, float step_size, uint64_t seed,
                        int proj0, int proj1, int nbins, uint32_t* d_hist1,
                        uint32_t* d_hist2, uint64_t* d_accepted, rid_stream stream) {
  if (!ens || !d_s || !d_hist1) return fail(RID_EINVAL, "NULL argument");
  if (W < 1 || n_steps < 0 || step0 < 0) return fail(RID_EINVAL, "need W >= 1, steps >= 0");
  if (!(kT > 0.0)) return fail(RID_EINVAL, "kT must be > 0");
  if (!(step_size > 0.f) || step_size > 3.14159265358979f)
    return fail(RID_EINVAL, "step_size must be in (0, pi]");
  const int n = ens->impl.n_cv;
  if (!ens->impl.raw.empty() && ens->impl.bounds.empty())
    return fail(RID_EINVAL, "raw CVs need their sampling box (rid_ensemble_set_cv_bounds)");
  if (nbins < 1 || proj0 < 0 || proj0 >= n || proj1 < 0 || proj1 >= n)
    return fail(RID_EINVAL, "need nbins >= 1 and projected indices in [0, n_cv)");
  return launch_mcmc(ens->impl, d_s, W, n_steps, step0, kT, step_size, seed, proj0, proj1,
                     nbins, d_hist1, d_hist2, reinterpret_cast<unsigned long long*>(d_accepted),
                     (hipStream_t)stream);
}

rid_status rid_cv_apply_force(rid_system sys, const float* d_pos,
                              const float* d_fcv, int B, float* d_force,
                              rid_stream stream) {
  if (!sys || !d_pos || !d_fcv || !d_force) return fail(RID_EINVAL, "NULL argument");
  if (B < 1) return fail(RID_EINVAL, "B must be >= 1");
  return launch_bias_scatter(sys->impl, 0, d_pos, B, nullptr, nullptr, d_fcv, 0.0f,
                             1.0f, d_force, nullptr, nullptr, nullptr, nullptr,
                             (hipStream_t)stream);
}

rid_status rid_mf_train_step(rid_ensemble ens, const float* d_s, const float* d_F,
                             int B, float lr, float* d_loss, rid_stream stream) {
  if (!ens || !d_s || !d_F) return fail(RID_EINVAL, "NULL argument");
  if (B < 1) return fail(RID_EINVAL, "B must be >= 1");
  if (!(lr >= 0.f)) return fail(RID_EINVAL, "lr must be >= 0");
  return launch_train_step(ens->impl, d_s, d_F, B, lr, d_loss, (hipStream_t)stream);
}

void rid_profile_enable(int mode) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (mode == 1) prof_recycle_locked();
  g_prof_on = mode != 0;
}

rid_status rid_profile_read(int kind, double* total_ms, int64_t* count) {
  if (!total_ms || !count || kind < 0 || kind >= kProfKinds)
    return fail(RID_EINVAL, "bad profile query");
  RID_HIP(hipDeviceSynchronize());
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double tot = 0.0;
  int64_t n = 0;
  for (auto& p : g_prof) {
    if (p.kind != kind) continue;
    float ms = 0.f;
    RID_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *count = n;
  return RID_OK;
}

rid_status rid_mf_loss_grad(rid_ensemble ens, const float* d_s, const float* d_F,
                            int B, float* d_loss, float* d_grad, rid_stream stream) {
  if (!ens || !d_s || !d_F || !d_grad) return fail(RID_EINVAL, "NULL argument");
  if (B < 1) return fail(RID_EINVAL, "B must be >= 1");
  float* used = nullptr;
  return launch_mf_grad(ens->impl, d_s, d_F, nullptr, B, d_loss, d_grad, &used,
                        (hipStream_t)stream);
}

rid_status rid_mf_grad(rid_ensemble ens, const float* d_s, const float* d_rho,
                       int B, float* d_grad, rid_stream stream) {
  if (!ens || !d_s || !d_rho || !d_grad) return fail(RID_EINVAL, "NULL argument");
  if (B < 1) return fail(RID_EINVAL, "B must be >= 1");
  float* used = nullptr;
  return launch_mf_grad(ens->impl, d_s, nullptr, d_rho, B, nullptr, d_grad, &used,
                        (hipStream_t)stream);
}

double rid_lr_exponential(int64_t step, double init_lr, int decay_steps,
                          double decay_rate) {
  if (decay_steps <= 0) return init_lr;
  return init_lr * std::pow(decay_rate, (double)step / (double)decay_steps);
}

rid_status rid_mf_label(const float* d_traj, const float* d_s0, const float* kappa,
                        const uint8_t* angular_mask, int M, int T, int n,
                        float std_threshold, double* d_F, double* d_se,
                        uint8_t* d_keep, rid_stream stream) {
  if (!d_traj || !d_s0 || !kappa || !d_F) return fail(RID_EINVAL, "NULL argument");
  if (M < 1 || n < 1 || n > 256 || T < 10)
    return fail(RID_EINVAL, "need M >= 1, 1 <= n <= 256 and T >= 10");
  return launch_mf_label_impl(d_traj, d_s0, kappa, angular_mask, M, T, n,
                              std_threshold, d_F, d_se, d_keep, (hipStream_t)stream);
}

}  // extern "C"
