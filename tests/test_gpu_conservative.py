"""GPU parity of the conservative switching path (rid_bias_force_conservative:
the bias force as the exact -grad of E = -sigma(eps) Abar, the switch
differentiated too) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import ridgen

from oracle import rid_oracle as O
from tests.gpu_common import FP32_TOL, HALF_TOL, assert_forces, oracle_models, workload

pytestmark = pytest.mark.gpu

# Inside the band the force carries Abar sigma'(eps) d eps/ds with
# sigma = (1 + cos(pi t))/2, sigma' = -pi/(2 D) sin(pi t), t = (eps-eps0)/D,
# D = eps1 - eps0.  An error d eps in the FP32 deviation therefore moves
# sigma' by the relative amount (pi/D)|cot(pi t)| |d eps| and sigma by
# (pi/D)|tan(pi t/2)| |d eps|, which grow without bound at the band edges
# (a walker at t = 0.9996 measured 8e-4 while walkers away from the edges
# agree to ~1e-6).  Each walker is held to the FP32 bound plus twice that
# conditioning times its measured |d eps|.
def walker_bounds(eps_gpu, eps_ref, e0, e1):
    D = e1 - e0
    t = np.clip((eps_ref - e0) / D, 1e-12, 1 - 1e-12)
    cond = (np.pi / D) * (np.abs(1 / np.tan(np.pi * t)) + np.abs(np.tan(np.pi * t / 2)))
    inside = (eps_ref >= e0) & (eps_ref < e1)
    return FP32_TOL + np.where(inside, 2.0 * cond * np.abs(eps_gpu - eps_ref), 0.0)


def assert_walkers(F_gpu, F_ref, bound, what):
    B = len(F_ref)
    d = np.abs(F_gpu - F_ref).reshape(B, -1).max(axis=1)
    scale = np.abs(F_ref).reshape(B, -1).max(axis=1)
    rel = d / np.maximum(scale, 1e-30)
    worst = int(np.argmax(rel / bound))
    print(f"{what}: max_rel={rel.max():.3e} median={np.median(rel):.3e} "
          f"worst/bound={rel[worst] / bound[worst]:.2f}", flush=True)
    zero = scale == 0
    # no force in the oracle (sigma = 0): only a rounding-level residue where
    # the FP32 deviation sits on the other side of eps1
    assert np.all(d[zero] <= FP32_TOL * scale.max()), what + ": force where the oracle has none"
    assert np.all(rel[~zero] <= bound[~zero]), f"{what}: walker {worst} rel {rel[worst]:.3e} > {bound[worst]:.3e}"


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def rid():
    import paper_2408_14070_amd as r
    r.lib()
    return r


def _run(torch, rid, sys_, pos, params, widths, K, e0, e1, conservative, prec=0):
    S = rid.System(sys_.n_atoms, sys_.quads)
    E = rid.Ensemble(sys_.n_cv, widths, K, params, prec)
    out = rid.bias_force(S, E, torch.from_numpy(pos).cuda(), float(e0), float(e1),
                         conservative=conservative)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


# FP32 ensembles of padded width <= 256 take the fused Hessian-vector kernel,
# wider ones (and 16-bit ensembles) the training sweeps in input mode.
@pytest.mark.parametrize("kind,widths,K", [("peptide20", [256] * 4, 4), ("dipeptide", [100] * 3, 4),
                                           ("peptide20", [64, 64], 3), ("peptide20", [512] * 2, 2)])
def test_conservative_force_parity_in_the_band(torch, rid, kind, widths, K):
    sys_, pos, params, widths, K = workload(kind, 48, seed=21, K=K, widths=widths, bias_std=0.1)
    models = oracle_models(params, sys_.n_cv, widths, K)
    ref1 = O.bias_force(pos.astype(np.float64), sys_.quads, models, 1e30, 2e30)
    e0, e1 = np.quantile(ref1["eps"], [0.02, 0.98])
    ref = O.bias_force_conservative(pos.astype(np.float64), sys_.quads, models, e0, e1)
    inside = (ref["eps"] >= e0) & (ref["eps"] < e1)
    assert inside.mean() > 0.9
    out = _run(torch, rid, sys_, pos, params, widths, K, e0, e1, True)
    bound = walker_bounds(out["eps"].astype(np.float64), ref["eps"], e0, e1)
    assert_walkers(out["F"], ref["F"], bound, f"{kind} conservative")
    assert np.max(np.abs(out["E"] - ref["E"])) <= 1e-5 * max(1.0, np.abs(ref["E"]).max())
    assert np.max(np.abs(out["eps"] - ref["eps"])) <= 1e-5 * np.abs(ref["eps"]).max()
    # the switch's own gradient is a visible part of the force here
    frozen = O.bias_force(pos.astype(np.float64), sys_.quads, models, e0, e1)["F"]
    assert O.max_rel_err(frozen, ref["F"]) > 1e-2


def test_conservative_full_size_bench_config(torch, rid):
    # the benchmarked configuration: 1024 walkers, headline ensemble, the band
    # placed over every walker's deviation
    sys_, pos, params, widths, K = workload("peptide20", 1024, seed=1)
    models = oracle_models(params, sys_.n_cv, widths, K)
    ref1 = O.bias_force(pos.astype(np.float64), sys_.quads, models, 1e30, 2e30)
    e0, e1 = 0.5 * ref1["eps"].min(), 2.0 * ref1["eps"].max()
    ref = O.bias_force_conservative(pos.astype(np.float64), sys_.quads, models, e0, e1)
    out = _run(torch, rid, sys_, pos, params, widths, K, e0, e1, True)
    bound = walker_bounds(out["eps"].astype(np.float64), ref["eps"], e0, e1)
    assert_walkers(out["F"], ref["F"], bound, "conservative, 1024 walkers")


def test_conservative_band_on_one_tile_ragged_batch(torch, rid):
    # walkers sorted by deviation, the band between the 16th and the 32nd:
    # the first 16 walkers sit below it (sigma = 1, no switch gradient), the
    # next 16 inside, the last 13 above it (sigma = 0), so the fused kernel
    # skips two of its three 16-walker tiles, and the last tile is ragged
    sys_, pos, params, widths, K = workload("peptide20", 45, seed=24, bias_std=0.1)
    models = oracle_models(params, sys_.n_cv, widths, K)
    ref1 = O.bias_force(pos.astype(np.float64), sys_.quads, models, 1e30, 2e30)
    order = np.argsort(ref1["eps"])
    pos = np.ascontiguousarray(pos[order])
    ev = ref1["eps"][order]
    e0, e1 = 0.5 * (ev[15] + ev[16]), 0.5 * (ev[31] + ev[32])
    ref = O.bias_force_conservative(pos.astype(np.float64), sys_.quads, models, e0, e1)
    assert np.all(ref["sigma"][:16] == 1.0) and np.all(ref["sigma"][32:] == 0.0)
    assert np.all((ref["sigma"][16:32] > 0) & (ref["sigma"][16:32] < 1))
    out = _run(torch, rid, sys_, pos, params, widths, K, e0, e1, True)
    bound = walker_bounds(out["eps"].astype(np.float64), ref["eps"], e0, e1)
    assert_walkers(out["F"], ref["F"], bound, "band on the middle tile")
    frozen = _run(torch, rid, sys_, pos, params, widths, K, e0, e1, False)
    assert_forces(out["F"][:16], frozen["F"][:16], FP32_TOL, "below the band = frozen")
    assert np.all(out["F"][32:] == 0.0)


def test_conservative_equals_frozen_outside_the_band(torch, rid):
    sys_, pos, params, widths, K = workload("peptide20", 40, seed=22, bias_std=0.1)
    a = _run(torch, rid, sys_, pos, params, widths, K, 2.0, 3.0, True)     # all sigma = 1
    b = _run(torch, rid, sys_, pos, params, widths, K, 2.0, 3.0, False)
    assert np.all(a["sigma"] == 1.0)
    assert_forces(a["F"], b["F"], FP32_TOL, "conservative vs frozen, sigma = 1")
    c = _run(torch, rid, sys_, pos, params, widths, K, 1e-3, 2e-3, True)    # all sigma = 0
    assert np.all(c["sigma"] == 0.0) and np.all(c["F"] == 0.0) and np.all(c["E"] == 0.0)


def test_conservative_16bit_ensemble(torch, rid):
    # A and g from the BF16 kernel, the switch-gradient term from FP32 sweeps
    # of the masters.  A wide band (t in about [0.25, 0.35]) keeps sigma and
    # sigma' well conditioned in the ~1e-2 relative error BF16 puts on eps,
    # so the force is held to the BF16 bound.
    sys_, pos, params, widths, K = workload("peptide20", 32, seed=23, K=4, widths=[512] * 2,
                                            bias_std=0.1)
    models = oracle_models(params, sys_.n_cv, widths, K)
    ref1 = O.bias_force(pos.astype(np.float64), sys_.quads, models, 1e30, 2e30)
    e0, e1 = 0.3 * ref1["eps"].min(), 2.5 * ref1["eps"].max()
    ref = O.bias_force_conservative(pos.astype(np.float64), sys_.quads, models, e0, e1)
    assert np.all((ref["sigma"] > 0) & (ref["sigma"] < 1))
    out = _run(torch, rid, sys_, pos, params, widths, K, e0, e1, True, prec=1)
    assert_forces(out["F"], ref["F"], HALF_TOL["bf16"], "bf16 conservative")
    frozen = O.bias_force(pos.astype(np.float64), sys_.quads, models, e0, e1)["F"]
    assert O.max_rel_err(frozen, ref["F"]) > 4 * HALF_TOL["bf16"][0]


def test_conservative_at_256_cvs(torch, rid):
    # the widest input: the fused Hessian-vector kernel's tile does not fit
    # the LDS, so the switch gradient comes from the input-mode sweeps
    sys_ = ridgen.chain_system(129, 5)
    widths, K = [64, 64], 4
    pos = ridgen.f32(ridgen.chain_coords(sys_, 5, 31))
    params = ridgen.xavier_ensemble(2 * sys_.n_cv, widths, K, 1000, 0.1)
    models = oracle_models(params, sys_.n_cv, widths, K)
    ref1 = O.bias_force(pos.astype(np.float64), sys_.quads, models, 1e30, 2e30)
    e0, e1 = 0.5 * ref1["eps"].min(), 2.0 * ref1["eps"].max()
    ref = O.bias_force_conservative(pos.astype(np.float64), sys_.quads, models, e0, e1)
    out = _run(torch, rid, sys_, pos, params, widths, K, e0, e1, True)
    bound = walker_bounds(out["eps"].astype(np.float64), ref["eps"], e0, e1)
    assert_walkers(out["F"], ref["F"], bound, "conservative, 256 CVs")


def test_conservative_residual_ensemble(torch, rid):
    # residual networks take the training sweeps in input mode
    sys_, pos, params, widths, K = workload("peptide20", 40, seed=25, K=3, widths=[128] * 3,
                                            bias_std=0.1)
    models = [tuple(m[:4]) + (True,) for m in oracle_models(params, sys_.n_cv, widths, K)]
    ref1 = O.bias_force(pos.astype(np.float64), sys_.quads, models, 1e30, 2e30)
    e0, e1 = 0.5 * ref1["eps"].min(), 2.0 * ref1["eps"].max()
    ref = O.bias_force_conservative(pos.astype(np.float64), sys_.quads, models, e0, e1)
    S = rid.System(sys_.n_atoms, sys_.quads)
    E = rid.Ensemble(sys_.n_cv, widths, K, params)
    E.set_resnet(True)
    out = rid.bias_force(S, E, torch.from_numpy(pos).cuda(), float(e0), float(e1),
                         conservative=True)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in out.items()}
    bound = walker_bounds(out["eps"].astype(np.float64), ref["eps"], e0, e1)
    assert_walkers(out["F"], ref["F"], bound, "conservative, residual")
    frozen = O.bias_force(pos.astype(np.float64), sys_.quads, models, e0, e1)["F"]
    assert O.max_rel_err(frozen, ref["F"]) > 1e-2


def test_conservative_mixed_cv_table(torch, rid):
    # 38 torsions and 6 distances: the raw CVs' chain is linear
    sys_ = ridgen.with_distances(ridgen.system_peptide20(), 6)
    widths, K = [64, 64], 4
    pos = ridgen.f32(ridgen.chain_coords(sys_, 40, 27))
    params = ridgen.xavier_ensemble(2 * sys_.n_cv, widths, K, 1000, 0.1)
    models = oracle_models(params, sys_.n_cv, widths, K)
    p64 = pos.astype(np.float64)
    ref1 = O.bias_force(p64, sys_.quads, models, 1e30, 2e30, mask=sys_.mask)
    e0, e1 = 0.5 * ref1["eps"].min(), 2.0 * ref1["eps"].max()
    ref = O.bias_force_conservative(p64, sys_.quads, models, e0, e1, mask=sys_.mask)
    S = rid.System(sys_.n_atoms, sys_.quads, sys_.mask)
    E = rid.Ensemble(sys_.n_cv, widths, K, params)
    E.set_angular_mask(sys_.mask)
    out = rid.bias_force(S, E, torch.from_numpy(pos).cuda(), float(e0), float(e1),
                         conservative=True)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in out.items()}
    bound = walker_bounds(out["eps"].astype(np.float64), ref["eps"], e0, e1)
    assert_walkers(out["F"], ref["F"], bound, "conservative, mixed table")
    frozen = O.bias_force(p64, sys_.quads, models, e0, e1, mask=sys_.mask)["F"]
    assert O.max_rel_err(frozen, ref["F"]) > 1e-2
