/*
 * rid.h - C ABI of the Reinforced-Dynamics neural-bias hot path on MI355X.
 *
 * Method: "RiD-kit: Software package designed to do enhanced sampling using
 * reinforced dynamics" (arXiv 2408.14070).  Sections are cited by name.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units        nm, rad, kJ/mol (GROMACS units, as in the paper's examples).
 * Pointers     d_* are DEVICE pointers (hipMalloc'd or torch CUDA tensors),
 *              owned by the caller; the library never frees or retains them
 *              beyond the call.  Host arrays are read during the call only.
 * Layouts      row-major, contiguous, FP32 unless stated.  B = walkers (or
 *              samples) in the call, n = number of CVs, K = ensemble size.
 * Streams      rid_stream is a hipStream_t (NULL = legacy default stream).
 *              Every call after *_create is asynchronous on that stream:
 *              it validates its arguments on the host, enqueues kernels and
 *              returns.  create/destroy/get/set synchronise.
 * Work memory  a handle owns scratch memory for intermediates (grown on
 *              demand, RID_ENOMEM on failure).  Calls that share a handle
 *              must be ordered on one stream by the caller.
 * Errors       no exception crosses the ABI.  A non-OK status leaves outputs
 *              untouched and sets a thread-local message (rid_last_error).
 *              Device-side conditions (degenerate dihedrals) are reported
 *              through per-walker flags, never through the status.
 * Precision    see rid_precision.  The ensemble-variance reduction and the
 *              mean-force label averaging always run in FP64 on the device.
 */
#ifndef RID_H
#define RID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RID_OK = 0,
  RID_EINVAL = -1,        /* bad argument: NULL, size, threshold order, index */
  RID_ENOMEM = -2,        /* device allocation failed                         */
  RID_EDEVICE = -3,       /* HIP runtime error (launch, copy, no device)      */
  RID_EDEGENERATE = -4,   /* reserved: degenerate geometry (flags are used)   */
  RID_EUNSUPPORTED = -5   /* shape outside the compiled kernel family         */
} rid_status;

typedef enum {
  RID_FP32 = 0,     /* every GEMM on FP32 MFMA, FP32 activations            */
  RID_BF16 = 1,     /* the precision form: the hidden-layer forward GEMMs on
                       BF16 MFMA with FP32 accumulation (BF16 weights and
                       activations); the first layer (CV encoding -> first
                       hidden layer) and the reverse sweep that gives the
                       mean force on FP16 MFMA (same rate) with FP32
                       accumulation; tanh derivatives computed in FP32 and
                       stored in FP16 between the sweeps; CV geometry and the
                       switch in FP32; ensemble variance in FP64.  The reverse
                       vectors carry a per-member power-of-two scale (exact)
                       that keeps them inside FP16's range.  Measured max
                       normwise force error vs the FP64 oracle ~3e-3        */
  RID_FP16 = 2,     /* every GEMM on FP16 MFMA with FP32 accumulation (same
                       rate, 3 more mantissa bits than BF16); needs
                       |weights|, |hidden activations| < 65504              */
  RID_BF16_ALL = 3  /* every GEMM operand BF16, tanh' stored in BF16: the
                       plain BF16 form, kept for comparison (max normwise
                       force error ~2e-2: each reverse-sweep rounding enters
                       the mean force linearly)                             */
} rid_precision;

typedef struct rid_system_s* rid_system;
typedef struct rid_ensemble_s* rid_ensemble;
typedef void* rid_stream;

/* Thread-local text of the last non-OK status of this thread. */
const char* rid_last_error(void);

/* Library version string. */
const char* rid_version(void);

/* ------------------------------------------------------------------------
 * Systems: atoms and CVs ("CV selection": backbone phi/psi torsions of the
 * selected residues, 2n-2 torsions for n residues, periodic over 2 pi; and
 * interatomic distances, the `distance` type, where angular_mask is 0).
 *
 * quads         host int32 [n_cv][4], 0-based atom indices (a, b, c, d) of
 *               each torsion; the torsion is
 *               s = atan2(|b2| b1.(b2 x b3), (b1 x b2).(b2 x b3)) with
 *               b1 = r_b - r_a, b2 = r_c - r_b, b3 = r_d - r_c, in (-pi, pi].
 * angular_mask  host uint8 [n_cv] or NULL (= all 1).  A row whose entry is
 *               0 is a distance CV (the `distance` type of "CV selection"):
 *               quads[i] = (a, b, -1, -1), s = |r_b - r_a| (nm), not
 *               periodic; a pair closer than 1e-6 nm is degenerate (s = 0,
 *               no force, the walker's flag set).
 * Errors        RID_EINVAL for n_atoms < 1, n_cv < 1, an index outside
 *               [0, n_atoms), a row that repeats an atom, a distance row
 *               not ending in -1, -1, or a mask entry other than 0 or 1.
 * ------------------------------------------------------------------------ */
rid_status rid_system_create(int n_atoms, int n_cv, const int32_t* quads,
                             const uint8_t* angular_mask, rid_system* out);
void rid_system_destroy(rid_system sys);

/* ------------------------------------------------------------------------
 * Ensembles of MLP free-energy models ("Training phase": numb_models MLPs
 * of `neurons` hidden widths, tanh; numb_models > 1 for a model deviation).
 * Input of every model is the periodic encoding x = [cos s | sin s]
 * (length 2 n_cv); output is the scalar free energy A.
 *
 * params  host FP32, packed: for each model k, for each hidden layer l,
 *         W_l row-major [width_l][width_{l-1}] then b_l [width_l]; then
 *         w_o [width_L] and b_o [1].  rid_packed_param_count gives the size.
 *         The library re-lays the weights out on the device (MFMA fragment
 *         order, zero-padded widths, BF16 copies) and keeps FP32 masters
 *         plus Adam moments for training.
 * Limits  1 <= n_hidden <= 6, 1 <= width <= 512, 1 <= n_models <= 64,
 *         1 <= n_cv <= 256 (RID_EUNSUPPORTED outside).
 * ------------------------------------------------------------------------ */
size_t rid_packed_param_count(int n_cv, int n_models, int n_hidden,
                              const int* widths);
rid_status rid_ensemble_create(int n_cv, int n_models, int n_hidden,
                               const int* widths, rid_precision prec,
                               const float* params, rid_ensemble* out);
/* Checkpoint: copy the FP32 master parameters out / in (packed layout).
 * set_params also resets the Adam moments and step counter. */
rid_status rid_ensemble_get_params(rid_ensemble ens, float* host_params);
rid_status rid_ensemble_set_params(rid_ensemble ens, const float* host_params);
/* Load the packed FP32 parameters from device memory (d_params, caller
 * owned, n_params floats in the packed layout) into the masters and rebuild
 * the MFMA fragments, ordered on `stream` with the calls around it (no host
 * synchronisation).  The Adam moments and step counter are kept.  Used by
 * the autograd binding, whose parameter tensor is the source of truth for
 * every forward evaluation.  Errors: RID_EINVAL for NULL arguments. */
rid_status rid_ensemble_load_params(rid_ensemble ens, const float* d_params,
                                    rid_stream stream);
/* Number of Adam updates taken so far. */
int64_t rid_ensemble_step(rid_ensemble ens);
/* Training-time dropout of the hidden activations ("Training phase" lists a
 * dropout rate among the training settings).  With rate p > 0 every training
 * call (rid_mf_train_step, rid_mf_loss_grad, rid_mf_grad) keeps hidden unit j
 * of layer l (1-based) of sample b of member k with probability 1 - p and
 * scales it by 1/(1 - p): the unit is kept when the uniform
 * (2 (x >> 9) + 1) 2^-24 of word j mod 4 of the Philox4x32-10 block with
 * counter (b, step mod 2^32, 16 k + l, j div 4) and key (seed mod 2^32,
 * seed div 2^32) is >= p (FP32), step being rid_ensemble_step at the call.
 * The bias path, MCMC and selection evaluate the full network.  With
 * residual connections the mask scales each layer's tanh branch, not the
 * skip.  Errors: RID_EINVAL (NULL, p outside [0, 1)). */
rid_status rid_ensemble_set_dropout(rid_ensemble ens, float rate, uint64_t seed);
/* Device bytes the training calls (rid_mf_train_step, rid_mf_loss_grad,
 * rid_mf_grad) may hold for stored activations; a larger batch runs in
 * chunks of rows (multiples of 64, at least 64 rows however small the
 * budget).  0 restores the default (512 MiB).  The workspace already
 * allocated is kept until the ensemble is destroyed.  Errors: RID_EINVAL
 * (NULL). */
rid_status rid_ensemble_set_train_budget(rid_ensemble ens, size_t bytes);
/* rid_ensemble_set_resnet - residual connections (the `resnet` training
 * setting, "Training phase": hidden layers of equal width joined by residual
 * connections).  With enable != 0 every hidden layer after the first adds
 * its input, h_l = h_{l-1} + tanh(W_l h_{l-1} + b_l) for l >= 2 (the first
 * layer maps the CV encoding and has no skip); enable = 0 restores the plain
 * MLP.  The packed parameters are the same in both forms.  Takes effect on
 * the next call: every evaluation (rid_bias_force, rid_model_dev,
 * rid_select, rid_mcmc_run, the server), conservative switching and the
 * training calls use the residual form (training and conservative
 * switching through the general sweeps: the tangent and both adjoints carry
 * the skip too).  Errors: RID_EINVAL (NULL, hidden widths not all equal),
 * RID_EUNSUPPORTED (16-bit ensemble: the 16-bit kernels have no skip). */
rid_status rid_ensemble_set_resnet(rid_ensemble ens, int enable);
/* rid_ensemble_set_angular_mask - which network inputs are periodic (the
 * `angular_mask` setting of "CV selection").  angular_mask: host uint8
 * [n_cv] or NULL (= all 1).  An angular CV enters as (cos s, sin s) in
 * input slots (i, n_cv + i); a CV whose entry is 0 enters raw, as (s, 0) in
 * the same two slots (input width and packed parameters unchanged), and its
 * mean force is dA/dx_i.  rid_model_dev encodes its CVs with the mask;
 * rid_bias_force and the server need the system's distance rows to be the
 * ensemble's raw CVs (RID_EINVAL otherwise); rid_select leaves raw CVs
 * unwrapped in its clustering distance; the training calls fit dA/dx_i to
 * a raw CV's label and rid_bias_force_conservative uses its linear chain;
 * rid_mcmc_run walks raw CVs in their box (rid_ensemble_set_cv_bounds,
 * RID_EINVAL until it is set).  Synchronizes the device.  Errors:
 * RID_EINVAL (NULL ensemble, an entry other than 0 or 1), RID_ENOMEM. */
rid_status rid_ensemble_set_angular_mask(rid_ensemble ens, const uint8_t* angular_mask);
/* rid_ensemble_set_cv_bounds - sampling box of the raw CVs for rid_mcmc_run
 * (the dimension-reduction settings' `cv_lower_bound` / `cv_upper_bound`,
 * which the paper introduces for distance CVs).  lower, upper: host float
 * [n_cv] (entries of angular CVs are checked but unused), or both NULL to
 * clear.  A raw CV then moves by step (upper - lower) / 2pi (2u - 1), is
 * not wrapped, a proposal that takes any raw CV outside [lower, upper] is
 * rejected, and its histogram bins cover [lower, upper).  Synchronizes the
 * device.  Errors: RID_EINVAL (NULL ensemble, one bound NULL, a non-finite
 * bound or lower >= upper), RID_ENOMEM. */
rid_status rid_ensemble_set_cv_bounds(rid_ensemble ens, const float* lower,
                                      const float* upper);
void rid_ensemble_destroy(rid_ensemble ens);

/* ------------------------------------------------------------------------
 * rid_cv_eval - CVs of B walkers ("CV selection"): torsions, and distances
 * for the system's distance rows (x = (s, 0) for those).
 *   d_pos  [B][n_atoms][3]   atom positions (whole molecules, no PBC)
 *   d_s    [B][n_cv]         torsions in (-pi, pi]; distances in nm
 *   d_x    [B][2 n_cv] or NULL: [cos s | sin s], computed from the geometry
 *          (cos s = X/sqrt(X^2+Y^2), sin s = Y/sqrt(X^2+Y^2)); a distance
 *          row's slots hold (s, 0).
 * A degenerate torsion (|b1 x b2|^2 or |b2 x b3|^2 < 1e-12 nm^4) gives
 * s = 0, x = (1, 0).
 * ------------------------------------------------------------------------ */
rid_status rid_cv_eval(rid_system sys, const float* d_pos, int B, float* d_s,
                       float* d_x, rid_stream stream);

/* ------------------------------------------------------------------------
 * rid_model_dev - ensemble mean forces and model deviation at given CVs.
 * Box 2 defines the mean force as F(s) = grad_s A(s); the uncertainty
 * indicator is the standard deviation of the ensemble's predictions
 * ("Development of the protocol", "Training phase"), taken here as
 *   eps = sqrt( (1/K) sum_k |g_k - gbar|^2 ),  g_k = grad_s A_k(s),
 * accumulated in FP64 (shifted by member 0, so identical members give 0).
 *   d_s     [B][n_cv]  CVs (any real values; periodic unless the ensemble's
 *                      angular mask marks them raw)
 *   d_eps   [B]        model deviation (required)
 *   d_gbar  [B][n_cv]  ensemble-mean mean force, or NULL
 *   d_A     [B][K]     per-model free energies, or NULL
 *   d_g     [B][K][n_cv] per-model mean forces, or NULL
 * ------------------------------------------------------------------------ */
rid_status rid_model_dev(rid_ensemble ens, const float* d_s, int B,
                         float* d_eps, float* d_gbar, float* d_A, float* d_g,
                         rid_stream stream);

/* ------------------------------------------------------------------------
 * Selection phase ("Selection"; "SelectorConfig": cluster_threshold,
 * numb_cluster_lower / numb_cluster_upper, max_selection).  The paper has
 * the exploration's CV frames clustered, the frames of high model deviation
 * kept by the trust level, the threshold adjusted in the first iteration
 * until the cluster count falls in [lower, upper], and at most max_selection
 * clusters sent on, one representative each.
 *
 * rid_cluster_frames - threshold clustering of CV frames.  Frames are taken
 * in order; a frame joins the first cluster (in founding order) whose
 * leader lies within `threshold`, otherwise it founds a cluster and is its
 * leader (the representative).  Distance: sqrt(sum_i wrap(a_i - b_i)^2),
 * differences wrapped to (-pi, pi], decided as d^2 <= threshold^2 in FP32
 * with the squares summed in CV order (no fused multiply-add), so the
 * labels are reproducible bit for bit.
 *   d_s        [B][n_cv] device  frames, angles in [-pi, pi]
 *   d_eps      [B] device or NULL  frames with eps < eps0 are left out
 *   adapt      nonzero: while the count is above `upper` the threshold is
 *              multiplied by 1.1, while below `lower` divided by 1.1 (FP32),
 *              at most 100 times; *threshold_used (nullable) gets the last
 *   max_clusters  cap: a frame that would found one more cluster gets label
 *              -1 and *n_clusters reports max_clusters + 1
 *   d_labels   [B] device  OUT: cluster index, -1 (over the cap), -2 (left out)
 *   d_leaders  [max_clusters] device  OUT: frame index of each leader
 *   n_clusters host  OUT: clusters founded (+1 when the cap was hit)
 * Synchronises the stream; allocates and frees its scratch per call (with
 * adapt: up to 24 thresholds' labels, leaders and leader CVs, at most
 * 256 MiB, clustered side by side; the result is the one-threshold-at-a-
 * time result).
 * Errors: RID_EINVAL (NULL pointer, B < 1, n_cv outside [1, 256], threshold
 * not positive and finite, max_clusters < 1, adapt with lower < 1 or
 * upper < lower).
 *
 * rid_select - the selection phase: eps of every frame (as rid_model_dev)
 * into d_eps [B]; the frames with eps >= eps0 clustered as above with the
 * cap max(upper, max_selection) + 1 and the threshold adapted when adapt is
 * nonzero (the workflow's first iteration); the leaders of the first
 * max_selection clusters in d_selected [max_selection] (frame indices,
 * *n_selected of them).  d_labels, n_clusters, threshold_used as above.
 * The distance uses the ensemble's angular mask (raw CVs unwrapped) and its
 * clustering weights (rid_ensemble_set_cv_weights): d^2 =
 * sum_i w_i wrap(a_i - b_i)^2, each FP32 square multiplied by w_i before it
 * is added (all weights 1: the metric above, bit for bit).
 * Synchronises the stream.  Errors: as above, and max_selection < 1.
 *
 * rid_ensemble_set_cv_weights - the per-CV clustering weights of the CV
 * settings ("CV selection": `weights` weigh each CV in the selection
 * phase's clustering).  weights: host float [n_cv], finite and >= 0, or
 * NULL (= all 1).  A weight of 0 removes the CV from the distance.  Used by
 * rid_select only.  Synchronizes the device.  Errors: RID_EINVAL (NULL
 * ensemble, a negative or non-finite weight), RID_ENOMEM.
 *
 * rid_adjust_trust_levels - the trust levels of the next iteration
 * ("Selection phase", numb_cluster_threshold): when the number of clusters
 * of the current iteration's exploration frames (n_clusters, as rid_select
 * reports it) is below numb_cluster_threshold, both levels are multiplied
 * by `scale`; otherwise they are left unchanged.  The paper gives the
 * condition and, in its troubleshooting table, the direction (higher trust
 * levels encourage exploration), but not the amount: `scale` (> 1) is the
 * caller's.  trust_lvl_1, trust_lvl_2: host, in/out (eps0 < eps1).  Pure
 * host arithmetic (FP32 products), no device work.  Errors: RID_EINVAL
 * (NULL pointer, scale not finite or <= 1, levels not 0 <= lvl_1 < lvl_2).
 * ------------------------------------------------------------------------ */
rid_status rid_cluster_frames(const float* d_s, int B, int n_cv, const float* d_eps,
                              float eps0, float threshold, int adapt, int lower, int upper,
                              int max_clusters, int* d_labels, int* d_leaders,
                              int* n_clusters, float* threshold_used, rid_stream stream);
rid_status rid_select(rid_ensemble ens, const float* d_s, int B, float eps0, float threshold,
                      int adapt, int lower, int upper, int max_selection, float* d_eps,
                      int* d_labels, int* d_selected, int* n_selected, int* n_clusters,
                      float* threshold_used, rid_stream stream);
rid_status rid_ensemble_set_cv_weights(rid_ensemble ens, const float* weights);
rid_status rid_adjust_trust_levels(int n_clusters, int numb_cluster_threshold, float scale,
                                   float* trust_lvl_1, float* trust_lvl_2);

/* ------------------------------------------------------------------------
 * rid_bias_force - the per-MD-step neural bias of B walkers.
 * The bias is the inverted predicted PMF, applied only where the ensemble
 * agrees ("Development of the protocol"); trust_lvl_1/trust_lvl_2 bound the
 * trust level ("Overall workflow setting").  With Abar, gbar the ensemble
 * means and eps the model deviation (as rid_model_dev):
 *   sigma = 1 (eps < eps0); 0 (eps >= eps1);
 *           (1 + cos(pi (eps - eps0)/(eps1 - eps0)))/2 in between
 *   E     = -sigma Abar                       (bias energy)
 *   F_a   = sum_i sigma gbar_i ds_i/dr_a      (force, sigma held fixed)
 *   d_pos    [B][n_atoms][3]  positions
 *   d_force  [B][n_atoms][3]  OVERWRITTEN; atoms in no torsion get 0
 *   d_energy [B] | NULL, d_eps [B] | NULL, d_sigma [B] | NULL
 *   d_flags  [B] | NULL: 1 if any torsion of the walker is degenerate
 *            (that torsion contributes no force), else 0.
 * Errors: RID_EINVAL for eps0 < 0 or eps0 >= eps1, B < 1, NULL pos/force,
 *         n_cv mismatch between system and ensemble.
 * ------------------------------------------------------------------------ */
rid_status rid_bias_force(rid_system sys, rid_ensemble ens, const float* d_pos,
                          int B, float eps0, float eps1, float* d_force,
                          float* d_energy, float* d_eps, float* d_sigma,
                          uint8_t* d_flags, rid_stream stream);

/* ------------------------------------------------------------------------
 * rid_bias_force_noalloc - rid_bias_force for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * rid_bias_force (bit for bit: the same kernels run), but the per-call
 * scratch (A [K][B], g [K][B][n_cv], the CV encoding [B][2 n_cv]) lives in a
 * fixed 32 MiB device array of the library that each GPU holds until the
 * process ends, so the call performs no device allocation.  Limit:
 * K*B + K*B*n_cv + 2*B*n_cv floats (each part rounded up to 64 floats) must
 * not exceed rid_noalloc_scratch_floats() = 8388608, else RID_EINVAL before
 * any device work (e.g. 8 members, 38 CVs: B <= 21845).  All calls on one
 * GPU share that array: calls that may overlap on one GPU (other streams,
 * other threads) race and must be ordered by the caller.  The ensemble's
 * weights must already be packed (they are after create, set/load_params
 * and every training call's next use) -- repacking after training runs
 * in place and allocates nothing either.
 * ------------------------------------------------------------------------ */
rid_status rid_bias_force_noalloc(rid_system sys, rid_ensemble ens, const float* d_pos,
                                  int B, float eps0, float eps1, float* d_force,
                                  float* d_energy, float* d_eps, float* d_sigma,
                                  uint8_t* d_flags, rid_stream stream);
size_t rid_noalloc_scratch_floats(void);

/* ------------------------------------------------------------------------
 * rid_bias_force_conservative - the same bias with the switch differentiated
 * too, so the force is exactly -grad E of E = -sigma(eps) Abar everywhere,
 * including the switching band ("Overall workflow setting": trust levels;
 * "Development of the protocol": bias only where the ensemble agrees):
 *   f_i = sigma gbar_i + Abar sigma'(eps) d eps/ds_i,
 *   d eps/ds = sum_k H_k (g_k - gbar) / (K eps)   (H_k: Hessian of A_k in s)
 *   F_a = sum_i f_i ds_i/dr_a.
 * Where sigma' = 0 (eps < eps0 or eps >= eps1) the force equals
 * rid_bias_force's up to rounding.  The Hessian-vector products come from
 * FP32 tangent and adjoint sweeps of the members' FP32 master weights (also
 * for 16-bit ensembles, whose A and g come from the 16-bit kernels); they
 * cost several forward passes, over every walker.
 * Arguments, outputs, errors and flags as rid_bias_force.  Uses the
 * ensemble's training workspace: not concurrent with training or gradient
 * calls on the same ensemble.
 * ------------------------------------------------------------------------ */
rid_status rid_bias_force_conservative(rid_system sys, rid_ensemble ens,
                                       const float* d_pos, int B, float eps0,
                                       float eps1, float* d_force,
                                       float* d_energy, float* d_eps,
                                       float* d_sigma, uint8_t* d_flags,
                                       rid_stream stream);

/* ------------------------------------------------------------------------
 * rid_mcmc_run - Metropolis MCMC in CV space on the ensemble's free energy
 * ("Dimension reduction phase": numb_walkers walkers, numb_steps steps, a
 * temperature, histograms of every CV and of the projected pair
 * proj_cv_index; the projected PMF is -kT ln p).
 * Per step t and walker w: s' = wrap(s + step_size (2u - 1)) on every CV,
 * accepted when u_n < exp(-(Abar(s') - Abar(s))/kT), Abar the ensemble
 * mean free energy (kJ/mol) from the ensemble's kernels at its precision,
 * the decision in FP64; then the current state is counted.  Uniforms:
 * Philox4x32-10, counter (w, t mod 2^32, t div 2^32, j), key (seed mod 2^32,
 * seed div 2^32), word 4j+i -> u = (2 (x >> 9) + 1) 2^-24; words 0..n-1 drive
 * the proposal, word n the acceptance.  Steps step0 .. step0+n_steps-1, so
 * consecutive calls with consecutive step0 continue one chain.  Raw CVs
 * (an ensemble angular mask with zeros: distances) walk in the box of
 * rid_ensemble_set_cv_bounds: s'_i = s_i + step_size (hi_i - lo_i)/2pi
 * (2u - 1), unwrapped; a proposal with any raw CV outside its box is
 * rejected; their bins cover [lo_i, hi_i).
 *   d_s        [W][n_cv] angles (wrapped to [-pi, pi) on entry) and raw
 *              CVs (as given), in/out
 *   kT         k_B T in kJ/mol (> 0); step_size in (0, pi]
 *   nbins      bins over [-pi, pi) per CV (>= 1)
 *   d_hist1    [n_cv][nbins] uint32 counts, ACCUMULATED (caller zeroes)
 *   d_hist2    [nbins][nbins] uint32 counts of (s[proj0], s[proj1]),
 *              accumulated, or NULL
 *   d_accepted [1] uint64 accepted-move count, accumulated, or NULL
 * Uses the ensemble's scratch: not concurrent with other calls on it.
 * Errors: RID_EINVAL for NULL ens/d_s/d_hist1, W < 1, n_steps < 0,
 *         step0 < 0, kT <= 0, step_size outside (0, pi], nbins < 1, proj
 *         index outside [0, n_cv), raw CVs without a box.
 * ------------------------------------------------------------------------ */
rid_status rid_mcmc_run(rid_ensemble ens, float* d_s, int W, int64_t n_steps,
                        int64_t step0, double kT, float step_size, uint64_t seed,
                        int proj0, int proj1, int nbins, uint32_t* d_hist1,
                        uint32_t* d_hist2, uint64_t* d_accepted, rid_stream stream);

/* ------------------------------------------------------------------------
 * rid_cv_apply_force - chain a CV-space force to the atoms alone:
 *   F_a = sum_i f_i ds_i/dr_a.
 *   d_fcv [B][n_cv]; d_force [B][n_atoms][3] OVERWRITTEN.
 * ------------------------------------------------------------------------ */
rid_status rid_cv_apply_force(rid_system sys, const float* d_pos,
                              const float* d_fcv, int B, float* d_force,
                              rid_stream stream);

/* ------------------------------------------------------------------------
 * rid_mf_train_step - one mean-force fitting step of every member
 * ("Training phase": the models are trained to predict mean forces; the
 * learning rate decays exponentially, see rid_lr_exponential).
 * Loss of member k on the minibatch:
 *   L_k = (1/B) sum_b |grad_s A_k(s_b) - F_b|^2,
 * differentiated in the weights by a double-backward (tangent + adjoint)
 * sweep in FP32, followed by one Adam update (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected) of the FP32 masters with step size lr.
 *   d_s, d_F  [B][n_cv]   CVs and mean-force labels
 *   d_loss    [K] | NULL  loss of each member BEFORE the update
 * The step always runs in FP32 on the FP32 masters; a BF16/FP16 ensemble
 * has its 16-bit copies refreshed before its next evaluation.
 * Memory: the sweeps keep the activations of every layer (primal, tangent
 * and adjoint) for the rows of one pass.  A batch whose activations exceed
 * the ensemble's training budget (rid_ensemble_set_train_budget, 512 MiB by
 * default) is taken in equal chunks of rows, in row order, and the chunks'
 * gradient contributions are added in that order: the result depends on
 * the budget only through that summation order, and is reproducible for a
 * given budget.  Dropout masks and the 1/B scale are those of the whole
 * batch.
 * ------------------------------------------------------------------------ */
rid_status rid_mf_train_step(rid_ensemble ens, const float* d_s,
                             const float* d_F, int B, float lr, float* d_loss,
                             rid_stream stream);

/* Gradient of the same loss, without updating anything:
 *   d_loss [K] | NULL   per-member loss
 *   d_grad [n_params]   dL/dtheta in the packed parameter layout (sum over
 *                       members of the per-member losses; each member's
 *                       block holds its own gradient; output bias entries 0)
 */
rid_status rid_mf_loss_grad(rid_ensemble ens, const float* d_s, const float* d_F,
                            int B, float* d_loss, float* d_grad,
                            rid_stream stream);

/* Vector-Jacobian product of the mean forces (the backward of
 * rid_model_dev's d_g output): for an upstream gradient
 * d_rho [B][K][n_cv], writes d_grad [n_params] =
 *   d/dtheta sum_b sum_k rho[b][k] . grad_s A_k(s_b)
 * in the packed parameter layout (double backward through the MLPs). */
rid_status rid_mf_grad(rid_ensemble ens, const float* d_s, const float* d_rho,
                       int B, float* d_grad, rid_stream stream);

/* Exponential decay of the paper's training schedule:
 * init_lr * decay_rate^(step / decay_steps) (continuous). */
double rid_lr_exponential(int64_t step, double init_lr, int decay_steps,
                          double decay_rate);

/* ------------------------------------------------------------------------
 * rid_mf_label - mean-force labels from restrained-MD CV trajectories
 * ("Labeling phase", restrained method: harmonic restraints of stiffness
 * kappas; the mean force is the average spring force; std_threshold drops
 * labels that have not converged).  In FP64 on the device:
 *   F_i  = kappa_i (1/T) sum_t wrap(s0_i - s_{t,i})  (wrap to (-pi, pi]
 *          where angular_mask_i = 1)
 *   SE_i = std over 10 blocks of floor(T/10) frames of the block-mean
 *          spring force (denominator 9) / sqrt(10)
 *   keep = max_i SE_i <= std_threshold
 *   d_traj [M][T][n] FP32, d_s0 [M][n] FP32, kappa host [n],
 *   angular_mask host [n] | NULL (= all 1),
 *   d_F [M][n] FP64, d_se [M][n] FP64 | NULL, d_keep [M] | NULL.
 * Errors: RID_EINVAL for T < 10, M < 1, n < 1 or n > 256.
 * ------------------------------------------------------------------------ */
rid_status rid_mf_label(const float* d_traj, const float* d_s0,
                        const float* kappa, const uint8_t* angular_mask,
                        int M, int T, int n, float std_threshold, double* d_F,
                        double* d_se, uint8_t* d_keep, rid_stream stream);

/* ------------------------------------------------------------------------
 * Serving loop: continuous batching of bias-force requests from many
 * walkers of different systems, ensembles and precisions on one GPU (the
 * exploration phase runs many walkers at once, "Overall workflow setting":
 * numb_walkers).  Ensemble weights and system tables stay resident on the
 * device, and so may the walkers' positions and forces (device requests).
 * A scheduler thread takes the oldest waiting request plus every later
 * waiting request of the same model (up to max_batch_walkers), admits
 * the batch only when its device memory fits the HBM budget, and runs it on
 * one of n_streams streams (copies in, bias kernels, copies out).  Requests
 * that arrive while others run are admitted as slots and memory free up.
 * A request's results do not depend on the batch it lands in (each walker
 * is computed independently with a fixed reduction order).
 *
 * rid_server_create    hbm_budget_bytes is allocated at once and is the
 *                      admission budget; flags: RID_SERVE_FIFO = serve one
 *                      request at a time on one stream (baseline).
 * rid_server_register  model = (system, ensemble, trust levels); the handles
 *                      must outlive the server and must not be trained while
 *                      registered.  Returns a model id.
 * rid_server_submit    copies host_pos [n_walkers][n_atoms][3] into pinned
 *                      staging and queues the request; never blocks on
 *                      memory: when the 1 GiB staging arena is full the
 *                      request gets a pinned block of its own (RID_ENOMEM if
 *                      that allocation fails).  RID_ENOMEM if the request can
 *                      never fit the HBM budget; RID_EDEVICE once a device
 *                      error has stopped the server; RID_EINVAL while it is
 *                      being destroyed.  Thread-safe.
 * rid_server_submit_device  the same with the walker state resident in
 *                      device memory: d_pos [n_walkers][n_atoms][3] is read
 *                      and d_force [n_walkers][n_atoms][3], d_energy /
 *                      d_eps / d_sigma [n_walkers] (any may be NULL) are
 *                      written by the request's batch on the device (no host
 *                      staging, no PCIe copies).  The buffers are the
 *                      caller's and must stay valid, and d_pos unchanged,
 *                      until the request has been waited.  Same errors.
 * rid_server_wait      blocks until the request is done and copies its
 *                      results to the host arrays (any may be NULL; ignored
 *                      for a device request, whose results are then in its
 *                      device buffers):
 *                      force [n_walkers][n_atoms][3], energy/eps/sigma
 *                      [n_walkers]; latency_us = arrival (submit) to results
 *                      visible in host memory.  Each ticket is waited once.
 *                      A request whose batch hit a device error (a kernel or
 *                      copy failing asynchronously) returns RID_EDEVICE, and
 *                      so does every request queued after it: the server
 *                      launches nothing more.  A request still queued when
 *                      the server is destroyed returns RID_EINVAL.
 * rid_server_stats     latency percentiles and throughput of the requests
 *                      waited since creation or the last reset.
 * rid_server_destroy   stops accepting requests, lets in-flight batches
 *                      finish, fails the queued ones (RID_EINVAL) and waits
 *                      until every thread blocked in rid_server_wait has
 *                      returned before it frees the server.  No call on the
 *                      handle may start once destroy has been called.
 * ------------------------------------------------------------------------ */
typedef struct rid_server_s* rid_server;
#define RID_SERVE_FIFO 1
typedef struct {
  int64_t requests_done, walkers_done, batches, admission_waits;
  int64_t max_inflight_batches;
  double mean_batch_walkers;
  double p50_us, p99_us, mean_us, max_us;
  double walker_steps_per_s;   /* walkers done / (last done - first arrival) */
} rid_server_stats_t;

rid_status rid_server_create(size_t hbm_budget_bytes, int n_streams,
                             int max_batch_walkers, int flags, rid_server* out);
rid_status rid_server_register(rid_server srv, rid_system sys, rid_ensemble ens,
                               float eps0, float eps1, int* model_id);
rid_status rid_server_submit(rid_server srv, int model_id, const float* host_pos,
                             int n_walkers, int64_t* ticket);
rid_status rid_server_submit_device(rid_server srv, int model_id, const float* d_pos,
                                    int n_walkers, float* d_force, float* d_energy,
                                    float* d_eps, float* d_sigma, int64_t* ticket);
rid_status rid_server_wait(rid_server srv, int64_t ticket, float* host_force,
                           float* host_energy, float* host_eps, float* host_sigma,
                           double* latency_us);

/* rid_server_replay - an open-loop request trace driven from native threads,
 * for measuring the server (capacity, latency under an offered load)
 * without a client in the way.  One thread submits request i at
 * arrival_s[i] seconds after the call starts (sleeping, then spinning to
 * the instant; arrival times must not decrease), the calling thread waits
 * on every ticket in order.  Per request: latency_us[i] (arrival at the
 * server to results visible, as rid_server_wait; -1 if it failed),
 * submit_lag_us[i] (how late the submission was against its arrival time);
 * *wall_s = first arrival to last wait.  Any output may be NULL.  The
 * requests enter the server's statistics like any others.  Errors:
 * RID_EINVAL (NULL server or requests, n < 1, a request without positions,
 * walkers < 1, arrival times out of order); otherwise the first failing
 * request's status after every request has been waited. */
typedef struct {
  int model_id;
  int n_walkers;
  double arrival_s;          /* offset from the start of the replay           */
  const float* pos;          /* [n_walkers][n_atoms][3], host or device memory */
  int device;                /* 1: pos and the outputs below are device memory */
  float* force;              /* outputs (any may be NULL): host arrays when    */
  float* energy;             /* device == 0 (copied at the wait), device       */
  float* eps;                /* buffers written on the device when device == 1 */
  float* sigma;
} rid_replay_request;
rid_status rid_server_replay(rid_server srv, const rid_replay_request* reqs, int n,
                             double* latency_us, double* submit_lag_us, double* wall_s);
rid_status rid_server_stats(rid_server srv, rid_server_stats_t* out);
void rid_server_reset_stats(rid_server srv);
void rid_server_destroy(rid_server srv);

/* ------------------------------------------------------------------------
 * Kernel timing for benchmarks.  While enabled, every kernel the library
 * launches carries two hipEvents that take its start and end timestamps
 * from the dispatch itself (no synchronisation at launch).  Modes of
 * rid_profile_enable: 1 clears the collected timings and starts, 2 resumes
 * without clearing (to sample some launches of a longer run), 0 pauses and
 * keeps what was collected.  rid_profile_read synchronises the device and
 * returns, for one kernel family, the summed event-measured duration (ms)
 * and the launch count since the last clear.  Families: 0 torsion CVs, 1 fused ensemble MLP,
 * 2 deviation/switch/atom-force scatter, 3 ensemble reduction,
 * 4 CV embedding, 5 training step kernels, 6 mean-force labels,
 * 7 Hessian-vector products of conservative switching.
 * ------------------------------------------------------------------------ */
void rid_profile_enable(int mode);
rid_status rid_profile_read(int kind, double* total_ms, int64_t* count);

#ifdef __cplusplus
}
#endif
#endif /* RID_H */
