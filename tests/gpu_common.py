"""Shared helpers of the GPU parity tests: seeded workloads and tolerances.

Errors are measured against the FP64 oracle on the same FP32-rounded inputs;
"max" is the max over walkers of the normwise per-walker relative error
(max |dF| / max |F| over the walker's atoms), "rms" is |dF|_2 / |F|_2 over
the batch.

FP32 path: max <= 1e-5.
16-bit forms (tolerances derived from the arithmetic).  Rounding a value to
a format with p significant bits perturbs it by a relative amount of rms
about 2^-p / sqrt(3) x 0.7 (over a binade): 1.6e-3 for BF16 (p = 8), 2e-4
for FP16 (p = 11).  A 4-layer network has 19 rounding sites: the encoding,
each layer's forward weights, the 3 stored hidden activations, the 3 stored
tanh', the 4 reverse vectors and the 4 layers' reverse weights.  Each
reverse-sweep site perturbs the mean force linearly by about that rms
relative amount; the forward sites enter only through tanh' and are damped
(their relative effect is about a third as large).  Summed in quadrature
over independent sites, and with the normwise per-walker maximum about 3x
the rms over a few hundred walkers:
  * all-BF16 form: 12 reverse sites x 1.6e-3 -> rms ~5.5e-3, max ~1.8e-2;
    bounds max 2.5e-2, rms 1e-2;
  * BF16 precision form (BF16 hidden-layer forward GEMMs, FP16 first layer
    and reverse sweep, FP16 tanh'): 6 damped BF16 forward sites -> rms
    ~1e-3, max ~3e-3; bounds max 1e-2 (the precision form's target), rms 3e-3;
  * FP16 form: rms ~7e-4, max ~2e-3; bounds max 1e-2, rms 2e-3.
A rounding-site emulation of these plans in numpy reproduces the GPU's
measured all-BF16 error (max 1.77e-2, rms 5.57e-3 at 300 walkers)."""
from __future__ import annotations

import numpy as np

import ridgen
from oracle import rid_oracle as O

FP32_TOL = 1e-5
HALF_TOL = {"bf16": (1e-2, 3e-3), "fp16": (1e-2, 2e-3), "bf16_all": (2.5e-2, 1e-2)}  # (max, rms)


def workload(kind: str, B: int, seed: int = 1, K=None, widths=None, bias_std=0.0,
             wseed=1000):
    """(system, pos f32 [B][N][3], params f32, widths, K) for a named shape."""
    if kind == "dipeptide":
        sys_ = ridgen.system_dipeptide()
        K = K or 4
        widths = widths or [100, 100, 100]
    elif kind == "peptide20":
        sys_ = ridgen.system_peptide20()
        K = K or 4
        widths = widths or [256] * 4
    elif kind == "peptide61":
        sys_ = ridgen.system_peptide61()
        K = K or 4
        widths = widths or [512] * 4
    else:
        raise ValueError(kind)
    pos = ridgen.f32(ridgen.chain_coords(sys_, B, seed))
    params = ridgen.xavier_ensemble(2 * sys_.n_cv, widths, K, wseed, bias_std)
    return sys_, pos, params, list(widths), K


def oracle_models(params, n_cv, widths, K):
    return ridgen.unpack_params(params, 2 * n_cv, widths, K)


def wrapped_diff(a, b):
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return (d + np.pi) % (2 * np.pi) - np.pi


def assert_forces(F_gpu, F_ref, tol, what="force"):
    """tol: max bound, or (max bound, rms bound)."""
    tmax, trms = (tol, None) if np.isscalar(tol) else tol
    err = O.max_rel_err(F_gpu, F_ref)
    rms = O.rms_rel_err(F_gpu, F_ref)
    print(f"{what}: max_rel={err:.3e} rms_rel={rms:.3e} (tol {tol})", flush=True)
    assert err <= tmax, f"{what} max rel err {err:.3e} > {tmax}"
    if trms is not None:
        assert rms <= trms, f"{what} rms rel err {rms:.3e} > {trms}"
    return err, rms


def basin_fitted_ensemble(n=38, K=8, widths=(512, 512, 512, 512), n_fit=300, n_eval=4096,
                          seed=31):
    """A trained-like ensemble with the deviation structure of a real RiD
    ensemble, built without the GPU path: each member keeps its own Xavier
    hidden layers and gets output weights fitted (ridge least squares, FP64)
    to mean-force labels drawn inside one basin (every CV within 1 rad of a
    seeded centre; labels = -grad of the analytic PMF + noise 0.5).  The mean
    force is linear in the output weights, so the fit is closed form: members
    agree inside the basin and extrapolate differently outside it.

    Returns (params f32 packed, evaluation CVs [n_eval][n] f32 at seeded
    distances 0.3..pi from the centre, oracle eps of those CVs)."""
    widths = list(widths)
    models = ridgen.unpack_params(ridgen.xavier_ensemble(2 * n, widths, K, 1000),
                                  2 * n, widths, K)
    pmf = ridgen.analytic_pmf(n, 3)
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-np.pi, np.pi, n)

    def wrap(a):
        return np.mod(a + np.pi, 2 * np.pi) - np.pi

    s = wrap(mu + rng.uniform(-1.0, 1.0, (n_fit, n)))
    F = -pmf.grad(s) + rng.normal(0.0, 0.5, s.shape)
    fitted = []
    idx = np.arange(n)
    for Ws, bs, _, _ in models:
        # d h_L / d s_i for every CV i (forward-mode through the layers)
        h = O.embed(s)
        hd = np.zeros((n_fit, n, 2 * n))
        hd[:, idx, idx] = -np.sin(s)
        hd[:, idx, n + idx] = np.cos(s)
        for W, b in zip(Ws, bs):
            h = np.tanh(h @ W.T + b)
            hd = (1.0 - h ** 2)[:, None, :] * (hd @ W.T)
        J = hd.reshape(n_fit * n, -1)
        wo = np.linalg.solve(J.T @ J + 1e-3 * np.eye(J.shape[1]), J.T @ F.reshape(-1))
        fitted.append((Ws, bs, wo, 0.0))
    params = ridgen.f32(ridgen.pack_params(fitted))
    r = rng.uniform(0.3, np.pi, (n_eval, 1))
    s_eval = ridgen.f32(wrap(mu + r * rng.uniform(-1.0, 1.0, (n_eval, n))))
    models32 = ridgen.unpack_params(params, 2 * n, widths, K)
    _, g = O.ensemble_mean_force(models32, s_eval.astype(np.float64))
    _, eps = O.model_deviation(g)
    return params, s_eval, eps
