"""GPU parity of the MCMC on the ensemble free energy (rid_mcmc_run) against
the FP64 oracle, through the C ABI: the generator-driven random walk, the
Metropolis decisions step by step, the histograms, chain continuation."""
import math

import numpy as np
import pytest

import ridgen
from oracle import rid_oracle as O

pytestmark = pytest.mark.gpu

KT_300K = O.BOLTZMANN_KJ_MOL_K * 300.0


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


def _ensemble(rid, n=38, widths=(64, 64), K=4, prec=0, bias_std=0.1, seed=1000, resnet=False):
    widths = list(widths)
    params = ridgen.xavier_ensemble(2 * n, widths, K, seed, bias_std)
    E = rid.Ensemble(n, widths, K, params, prec)
    models = ridgen.unpack_params(params, 2 * n, widths, K)
    if resnet:
        E.set_resnet(True)
        models = [m + (True,) for m in models]
    return E, models


def _wrapped(a, b):
    return np.abs(np.mod(a - b + math.pi, 2 * math.pi) - math.pi)


def test_infinite_temperature_walk_matches_the_generator(torch, rid):
    E, models = _ensemble(rid)
    W, T, step, seed = 128, 15, 0.7, 0x1234_5678_9ABC
    s0 = ridgen.f32(ridgen.torus_samples(W, 38, 4))
    s = torch.from_numpy(s0.copy()).cuda()
    out = rid.mcmc_run(E, s, T, 1e30, step, seed, step0=3, proj=(0, 5), nbins=17)
    torch.cuda.synchronize()
    ref = O.mcmc_run(models, s0.astype(np.float64), T, 1e30, step, seed, t0=3, proj=(0, 5),
                     nbins=17)
    assert np.max(_wrapped(s.cpu().numpy(), ref["s"])) < 2e-5
    assert int(out["accepted"].item()) == W * T
    h1 = out["hist1"].cpu().numpy().astype(np.int64)
    h2 = out["hist2"].cpu().numpy().astype(np.int64)
    assert h1.sum() == W * T * 38 and h2.sum() == W * T
    assert np.abs(h1 - ref["hist1"]).sum() <= 4   # bin-boundary rounding only
    assert np.abs(h2 - ref["hist2"]).sum() <= 4


# 300 K (the paper's temperature) accepts nearly every move of a random-init
# ensemble; kT = 0.01 kJ/mol rejects about half of them
# The second case is the headline ensemble at 2048 walkers, where the free
# energies come from 32-walker tiles (the energy-only kernel's large-batch form).
# The last case runs the residual network form (energy-only residual kernel).
@pytest.mark.parametrize("kT,widths,W,T,resnet", [(KT_300K, (128, 128), 256, 25, False),
                                                  (0.01, (128, 128), 256, 25, False),
                                                  (0.01, (256, 256, 256, 256), 2048, 8, False),
                                                  (0.01, (128, 128, 128), 256, 25, True)])
def test_metropolis_decisions_step_by_step(torch, rid, kT, widths, W, T, resnet):
    # one call per step; a walker may only leave the oracle's chain at a step
    # whose acceptance margin |ln u_n + dAbar/kT| is at rounding level
    E, models = _ensemble(rid, widths=widths, K=4, resnet=resnet)
    step, seed, n = 0.35, 77, 38
    s0 = ridgen.f32(ridgen.torus_samples(W, n, 5))
    ref = O.mcmc_run(models, s0.astype(np.float64), T, kT, step, seed, nbins=31,
                     keep_path=True)
    s = torch.from_numpy(s0.copy()).cuda()
    h1 = torch.zeros((n, 31), dtype=torch.int32, device="cuda")
    h2 = torch.zeros((31, 31), dtype=torch.int32, device="cuda")
    acc = torch.zeros(1, dtype=torch.int64, device="cuda")
    alive = np.ones(W, bool)
    prev = s0.astype(np.float64)
    lost_steps = 0
    for t in range(T):
        rid.mcmc_run(E, s, 1, kT, step, seed, step0=t, nbins=31, hist1=h1, hist2=h2,
                     accepted=acc)
        torch.cuda.synchronize()
        cur = s.cpu().numpy().astype(np.float64)
        off = alive & (np.max(_wrapped(cur, ref["path"][t]), axis=1) > 1e-4)
        for w in np.nonzero(off)[0]:
            u = O.mcmc_uniforms([w], t, n + 1, seed)[0]
            sp = O.wrap_torus(prev[w] + step * (2 * u[:n] - 1))
            dA = O.ensemble_energy(models, sp[None])[0] - O.ensemble_energy(models, prev[w][None])[0]
            margin = abs(math.log(u[n]) + dA / kT)
            assert margin < 1e-3, f"walker {w} step {t}: decision differs with margin {margin:.2e}"
        lost_steps += int(np.sum(~alive)) + int(np.sum(off))
        alive &= ~off
        prev = ref["path"][t]
    print(f"walkers on the oracle's chain after {T} steps: {alive.sum()} of {W}", flush=True)
    assert alive.mean() >= 0.98
    h1 = h1.cpu().numpy().astype(np.int64)
    assert h1.sum() == W * T * n and h2.sum().item() == W * T
    assert np.abs(h1 - ref["hist1"]).sum() <= 2 * n * lost_steps + 8
    a = int(acc.item())
    print(f"kT {kT:.3g}: accepted {a / (W * T):.3f} of the moves", flush=True)
    if kT < 0.1:
        assert 0.3 * W * T < a < 0.8 * W * T
    assert abs(a - ref["accepted"]) <= lost_steps + 2


def test_chain_continues_across_calls(torch, rid):
    E, _ = _ensemble(rid, widths=(64,), K=3)
    s0 = ridgen.f32(ridgen.torus_samples(64, 38, 6))
    a = torch.from_numpy(s0.copy()).cuda()
    b = torch.from_numpy(s0.copy()).cuda()
    ra = rid.mcmc_run(E, a, 12, KT_300K, 0.5, 9)
    hb1 = torch.zeros((38, 101), dtype=torch.int32, device="cuda")
    for t in range(0, 12, 4):
        rid.mcmc_run(E, b, 4, KT_300K, 0.5, 9, step0=t, hist1=hb1)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(ra["hist1"], hb1)


def test_bf16_metropolis_decisions_step_by_step(torch, rid):
    """The BF16 precision form's free energies (the forward sweep: FP16 first
    layer, BF16 hidden layers) on the precision form's ensemble shape.  The
    margin rule of the FP32 test, with the tolerance set by the measured
    error of Abar: a walker may only leave the oracle's chain at a step whose
    acceptance margin |ln u + dAbar/kT| is below 3 max|dAbar_err| / kT."""
    n, widths, K, W, T = 38, (512, 512, 512, 512), 8, 256, 10
    E, models = _ensemble(rid, n=n, widths=widths, K=K, prec=rid.RID_BF16, bias_std=0.1)
    kT, step, seed = 0.05, 0.35, 91
    # measured error of Abar on torus samples
    probe = ridgen.f32(ridgen.torus_samples(1024, n, 17))
    A = rid.model_dev(E, torch.from_numpy(probe).cuda())[2]
    torch.cuda.synchronize()
    abar = A.cpu().numpy().astype(np.float64).mean(axis=1)
    e_A = float(np.max(np.abs(abar - O.ensemble_energy(models, probe.astype(np.float64)))))
    tol = 3.0 * e_A / kT
    print(f"bf16 Abar error {e_A:.2e} kJ/mol -> margin tolerance {tol:.3f}", flush=True)
    assert e_A < 1e-2
    s0 = ridgen.f32(ridgen.torus_samples(W, n, 19))
    ref = O.mcmc_run(models, s0.astype(np.float64), T, kT, step, seed, nbins=31, keep_path=True)
    s = torch.from_numpy(s0.copy()).cuda()
    h1 = torch.zeros((n, 31), dtype=torch.int32, device="cuda")
    acc = torch.zeros(1, dtype=torch.int64, device="cuda")
    alive = np.ones(W, bool)
    prev = s0.astype(np.float64)
    lost = 0
    for t in range(T):
        rid.mcmc_run(E, s, 1, kT, step, seed, step0=t, nbins=31, hist1=h1, accepted=acc)
        torch.cuda.synchronize()
        cur = s.cpu().numpy().astype(np.float64)
        off = alive & (np.max(_wrapped(cur, ref["path"][t]), axis=1) > 1e-4)
        for w in np.nonzero(off)[0]:
            u = O.mcmc_uniforms([w], t, n + 1, seed)[0]
            sp = O.wrap_torus(prev[w] + step * (2 * u[:n] - 1))
            dA = O.ensemble_energy(models, sp[None])[0] - O.ensemble_energy(models, prev[w][None])[0]
            margin = abs(math.log(u[n]) + dA / kT)
            assert margin < tol, f"walker {w} step {t}: decision differs with margin {margin:.2e}"
        lost += int(np.sum(~alive)) + int(np.sum(off))
        alive &= ~off
        prev = ref["path"][t]
    a = int(acc.item())
    print(f"bf16: walkers on the oracle's chain after {T} steps: {alive.sum()} of {W}; "
          f"accepted {a / (W * T):.3f} (oracle {ref['accepted'] / (W * T):.3f})", flush=True)
    assert alive.mean() >= 0.9
    assert abs(a - ref["accepted"]) <= lost + 2
    assert 0.2 * W * T < a < 0.98 * W * T


def test_mcmc_argument_errors(torch, rid):
    E, _ = _ensemble(rid, widths=(64, 64), K=2)
    s = torch.from_numpy(ridgen.f32(ridgen.torus_samples(20, 38, 7))).cuda()
    with pytest.raises(rid.RidError):
        rid.mcmc_run(E, s, 1, -1.0, 0.3, 3)
    with pytest.raises(rid.RidError):
        rid.mcmc_run(E, s, 1, KT_300K, 4.0, 3)
    with pytest.raises(rid.RidError):
        rid.mcmc_run(E, s, 1, KT_300K, 0.3, 3, proj=(0, 38))


def test_mcmc_at_256_cvs(torch, rid):
    # the widest input (the energy-only MLP then sums its input-gradient
    # region in one part): the infinite-temperature walk is the generator's
    W, T, step, seed, n = 40, 6, 0.5, 99, 256
    E, models = _ensemble(rid, n=n, widths=(64, 64), K=3)
    s0 = ridgen.f32(ridgen.torus_samples(W, n, 6))
    ref = O.mcmc_run(models, s0.astype(np.float64), T, 1e30, step, seed, nbins=17)
    s = torch.from_numpy(s0.copy()).cuda()
    out = rid.mcmc_run(E, s, T, 1e30, step, seed, nbins=17)
    torch.cuda.synchronize()
    assert int(out["accepted"].item()) == W * T
    assert np.max(_wrapped(s.cpu().numpy().astype(np.float64), ref["s"])) < 2e-5
    h1 = out["hist1"].cpu().numpy().astype(np.int64)
    assert h1.sum() == W * T * n
    assert np.abs(h1 - ref["hist1"]).sum() <= 4   # bin-boundary rounding only


def test_mixed_table_box_walk_step_by_step(torch, rid):
    """38 torsions and 6 distance CVs: the raw CVs walk in their box [0.2,
    1.2] (proposals that leave it are rejected), the angles on the circle.
    Step by step against the oracle: a walker may only leave the oracle's
    chain where the acceptance margin or a raw CV's distance to its box wall
    is at rounding level."""
    base = ridgen.with_distances(ridgen.system_peptide20(), 6)
    n, widths, K, W, T = base.n_cv, [64, 64], 4, 256, 20
    mask = base.mask
    raw = mask == 0
    lo = np.where(raw, 0.2, -math.pi).astype(np.float32)
    hi = np.where(raw, 1.2, math.pi).astype(np.float32)
    params = ridgen.xavier_ensemble(2 * n, widths, K, 1000, 0.1)
    models = ridgen.unpack_params(params, 2 * n, widths, K)
    E = rid.Ensemble(n, widths, K, params)
    E.set_angular_mask(mask)
    s_chk = torch.zeros((4, n), dtype=torch.float32, device="cuda")
    with pytest.raises(rid.RidError):       # no box yet
        rid.mcmc_run(E, s_chk, 1, 0.05, 0.3, 1)
    E.set_cv_bounds(lo, hi)
    rng = np.random.default_rng(8)
    s0 = ridgen.f32(np.where(raw, rng.uniform(0.2, 1.2, (W, n)), ridgen.torus_samples(W, n, 8)))
    kT, step, seed = 0.05, 0.5, 123
    ref = O.mcmc_run(models, s0.astype(np.float64), T, kT, step, seed, nbins=21, proj=(0, 4),
                     keep_path=True, mask=mask, lower=lo.astype(np.float64),
                     upper=hi.astype(np.float64))
    s = torch.from_numpy(s0.copy()).cuda()
    h1 = torch.zeros((n, 21), dtype=torch.int32, device="cuda")
    h2 = torch.zeros((21, 21), dtype=torch.int32, device="cuda")
    acc = torch.zeros(1, dtype=torch.int64, device="cuda")
    alive = np.ones(W, bool)
    prev = s0.astype(np.float64)
    lost = 0
    span = (hi - lo).astype(np.float64)

    def dist(a, b):
        d = np.abs(a - b)
        return np.where(raw, d, np.abs(np.mod(a - b + math.pi, 2 * math.pi) - math.pi))

    for t in range(T):
        rid.mcmc_run(E, s, 1, kT, step, seed, step0=t, nbins=21, proj=(0, 4), hist1=h1,
                     hist2=h2, accepted=acc)
        torch.cuda.synchronize()
        cur = s.cpu().numpy().astype(np.float64)
        assert np.all((cur[:, raw] >= 0.2 - 1e-6) & (cur[:, raw] <= 1.2 + 1e-6))
        off = alive & (np.max(dist(cur, ref["path"][t]), axis=1) > 1e-4)
        for w in np.nonzero(off)[0]:
            u = O.mcmc_uniforms([w], t, n + 1, seed)[0]
            prop = prev[w] + step * span / (2 * math.pi) * (2 * u[:n] - 1)
            sp = np.where(raw, prop, O.wrap_torus(prop))
            wall = np.min(np.minimum(np.abs(sp[raw] - 0.2), np.abs(sp[raw] - 1.2)))
            dA = (O.ensemble_energy(models, sp[None], mask)[0]
                  - O.ensemble_energy(models, prev[w][None], mask)[0])
            margin = abs(math.log(u[n]) + dA / kT)
            assert margin < 1e-3 or wall < 1e-5, \
                f"walker {w} step {t}: differs with margin {margin:.2e}, wall {wall:.2e}"
        lost += int(np.sum(~alive)) + int(np.sum(off))
        alive &= ~off
        prev = ref["path"][t]
    print(f"walkers on the oracle's chain after {T} steps: {alive.sum()} of {W}; "
          f"accepted {int(acc.item()) / (W * T):.3f}", flush=True)
    assert alive.mean() >= 0.97
    a = int(acc.item())
    assert abs(a - ref["accepted"]) <= lost + 2
    assert 0.05 * W * T < a < 0.95 * W * T
    h1 = h1.cpu().numpy().astype(np.int64)
    assert h1.sum() == W * T * n and int(h2.sum().item()) == W * T
    assert np.abs(h1 - ref["hist1"]).sum() <= 2 * n * lost + 8


@pytest.mark.parametrize("nbins,W", [(31, 2048), (4096, 300), (31, 1)])
def test_histograms_count_every_walker_once_per_step(torch, rid, nbins, W):
    """Every step counts each walker once per CV and once in the pair
    histogram, whatever the number of private histogram copies (32 for small
    tables, fewer when n x nbins is large), and the counts add onto what
    the caller passes in."""
    n = 38
    E, _ = _ensemble(rid, n=n, widths=(64,), K=2)
    s = torch.from_numpy(ridgen.f32(ridgen.torus_samples(W, n, 12))).cuda()
    steps = 5
    h1 = torch.full((n, nbins), 3, dtype=torch.int32, device="cuda")
    h2 = torch.zeros((nbins, nbins), dtype=torch.int32, device="cuda")
    out = rid.mcmc_run(E, s, steps, KT_300K, 0.4, 17, nbins=nbins, hist1=h1, hist2=h2)
    torch.cuda.synchronize()
    per_cv = out["hist1"].to(torch.int64).sum(dim=1).cpu().numpy()
    assert np.all(per_cv == steps * W + 3 * nbins)
    assert int(out["hist2"].to(torch.int64).sum().item()) == steps * W
