"""GPU parity of distance CVs and mixed CV tables (angular mask) against the
FP64 oracle, through the C ABI: CV values and encoding, the bias force on a
chain with torsion and distance CVs, the chain rule alone, the model
deviation of a masked ensemble, degenerate pairs, the server, and the calls
that refuse non-angular CVs."""
import numpy as np
import pytest

import ridgen
from oracle import rid_oracle as O
from tests.gpu_common import FP32_TOL, HALF_TOL, assert_forces

pytestmark = pytest.mark.gpu


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


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _mixed(n_dist=6, base=None):
    return ridgen.with_distances(base or ridgen.system_peptide20(), n_dist)


def _ens(rid, sys_, widths, K, seed, resnet=False):
    params = ridgen.xavier_ensemble(2 * sys_.n_cv, widths, K, seed, 0.1)
    E = rid.Ensemble(sys_.n_cv, widths, K, params)
    E.set_angular_mask(sys_.mask)
    models = ridgen.unpack_params(params, 2 * sys_.n_cv, widths, K)
    if resnet:
        E.set_resnet(True)
        models = [m + (True,) for m in models]
    return E, models


def test_mixed_cv_eval_parity(torch, rid):
    sys_ = _mixed()
    pos = ridgen.f32(ridgen.chain_coords(sys_, 130, seed=3))
    S = rid.System(sys_.n_atoms, sys_.quads, sys_.mask)
    s, x = rid.cv_eval(S, _dev(torch, pos))
    torch.cuda.synchronize()
    s_ref = O.cv_values(pos.astype(np.float64), sys_.quads, sys_.mask)
    x_ref = O.embed(s_ref, sys_.mask)
    m = sys_.mask.astype(bool)
    s = s.cpu().numpy()
    ds = np.abs(s - s_ref)
    ds[:, m] = np.abs((ds[:, m] + np.pi) % (2 * np.pi) - np.pi)
    assert ds.max() <= FP32_TOL
    assert np.max(np.abs(x.cpu().numpy() - x_ref)) <= FP32_TOL
    assert np.all(x.cpu().numpy()[:, sys_.n_cv:][:, ~m] == 0.0)


# B = 300 spans many 16-walker tiles with a ragged end; the resnet case runs
# the residual kernel on the encoding path
@pytest.mark.parametrize("widths,K,B,resnet", [([256] * 4, 4, 300, False),
                                               ([100, 100, 100], 3, 45, False),
                                               ([256] * 4, 4, 77, True)])
def test_mixed_bias_force_parity(torch, rid, widths, K, B, resnet):
    sys_ = _mixed()
    print(f"mixed bias force: {sys_.n_cv} CVs ({int((sys_.mask == 0).sum())} distances) "
          f"{widths} K={K} B={B} resnet={resnet}", flush=True)
    pos = ridgen.f32(ridgen.chain_coords(sys_, B, seed=5))
    S = rid.System(sys_.n_atoms, sys_.quads, sys_.mask)
    E, models = _ens(rid, sys_, widths, K, 1005, resnet)
    # trust levels that keep sigma = 1: the whole ensemble-mean force
    ref = O.bias_force(pos.astype(np.float64), sys_.quads, models, 1e9, 2e9, mask=sys_.mask)
    out = rid.bias_force(S, E, _dev(torch, pos), 1e9, 2e9)
    torch.cuda.synchronize()
    assert_forces(out["F"].cpu().numpy(), ref["F"], FP32_TOL, "mixed F")
    scale = np.abs(ref["g"]).reshape(B, -1).max(axis=1)
    assert np.max(np.abs(out["eps"].cpu().numpy() - ref["eps"]) / scale) <= FP32_TOL
    E_ref = ref["E"]
    assert np.max(np.abs(out["E"].cpu().numpy() - E_ref)) <= FP32_TOL * max(1.0, np.abs(E_ref).max())
    assert not out["flags"].cpu().numpy().any()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_mixed_bias_force_16bit(torch, rid, prec):
    # the 16-bit encoding instances share the raw-CV chain; tolerance of the
    # 16-bit forms (operand rounding in every GEMM stage)
    sys_ = _mixed()
    B, K, widths = 300, 4, [256] * 4
    pos = ridgen.f32(ridgen.chain_coords(sys_, B, seed=11))
    params = ridgen.xavier_ensemble(2 * sys_.n_cv, widths, K, 1011, 0.1)
    S = rid.System(sys_.n_atoms, sys_.quads, sys_.mask)
    E = rid.Ensemble(sys_.n_cv, widths, K, params, rid.RID_BF16 if prec == "bf16" else rid.RID_FP16)
    E.set_angular_mask(sys_.mask)
    models = ridgen.unpack_params(params, 2 * sys_.n_cv, widths, K)
    ref = O.bias_force(pos.astype(np.float64), sys_.quads, models, 1e9, 2e9, mask=sys_.mask)
    out = rid.bias_force(S, E, _dev(torch, pos), 1e9, 2e9)
    torch.cuda.synchronize()
    assert_forces(out["F"].cpu().numpy(), ref["F"], HALF_TOL[prec], f"mixed {prec} F")


def test_mixed_cv_apply_force_parity(torch, rid):
    sys_ = _mixed()
    pos = ridgen.f32(ridgen.chain_coords(sys_, 20, seed=6))
    fcv = ridgen.f32(np.random.default_rng(7).normal(size=(20, sys_.n_cv)))
    S = rid.System(sys_.n_atoms, sys_.quads, sys_.mask)
    F = rid.cv_apply_force(S, _dev(torch, pos), _dev(torch, fcv))
    torch.cuda.synchronize()
    ref = O.apply_cv_force(pos.astype(np.float64), sys_.quads, fcv.astype(np.float64),
                           mask=sys_.mask)
    assert_forces(F.cpu().numpy(), ref, FP32_TOL, "mixed apply_force")


def test_masked_model_dev_parity(torch, rid):
    n, widths, K, B = 40, [256] * 4, 4, 500
    mask = np.ones(n, np.uint8)
    mask[::5] = 0
    params = ridgen.xavier_ensemble(2 * n, widths, K, 1006, bias_std=0.1)
    E = rid.Ensemble(n, widths, K, params)
    E.set_angular_mask(mask)
    rng = np.random.default_rng(8)
    s = ridgen.f32(np.where(mask.astype(bool), rng.uniform(-np.pi, np.pi, (B, n)),
                            rng.uniform(0.3, 1.5, (B, n))))
    eps, gbar, A, g = rid.model_dev(E, _dev(torch, s))
    torch.cuda.synchronize()
    models = ridgen.unpack_params(params, 2 * n, widths, K)
    A_ref, g_ref = O.ensemble_mean_force(models, s.astype(np.float64), mask)
    _, eps_ref = O.model_deviation(g_ref)
    assert_forces(g.cpu().numpy(), g_ref, FP32_TOL, "masked g")
    assert_forces(A.cpu().numpy(), A_ref, FP32_TOL, "masked A")
    scale = np.abs(g_ref).reshape(B, -1).max(axis=1)
    assert np.max(np.abs(eps.cpu().numpy() - eps_ref) / scale) <= FP32_TOL
    # clearing the mask gives the plain periodic encoding again
    E.set_angular_mask(None)
    _, _, _, g2 = rid.model_dev(E, _dev(torch, s))
    torch.cuda.synchronize()
    _, g_plain = O.ensemble_mean_force(models, s.astype(np.float64))
    assert_forces(g2.cpu().numpy(), g_plain, FP32_TOL, "unmasked g")


def test_coincident_pair_is_flagged(torch, rid):
    sys_ = _mixed(2)
    pos = ridgen.f32(ridgen.chain_coords(sys_, 4, seed=9))
    drow = int(np.nonzero(sys_.mask == 0)[0][0])
    a, b = sys_.quads[drow, :2]
    pos[1, b] = pos[1, a]                      # walker 1: the pair coincides
    S = rid.System(sys_.n_atoms, sys_.quads, sys_.mask)
    E, models = _ens(rid, sys_, [64, 64], 2, 1007)
    out = rid.bias_force(S, E, _dev(torch, pos), 1e9, 2e9)
    s, _ = rid.cv_eval(S, _dev(torch, pos))
    torch.cuda.synchronize()
    flags = out["flags"].cpu().numpy()
    assert flags[1] == 1 and flags[[0, 2, 3]].sum() == 0
    assert s.cpu().numpy()[1, drow] == 0.0
    ref = O.bias_force(pos.astype(np.float64), sys_.quads, models, 1e9, 2e9, mask=sys_.mask)
    keep = [0, 2, 3]
    assert_forces(out["F"].cpu().numpy()[keep], ref["F"][keep], FP32_TOL, "other walkers")


def test_mixed_server_matches_direct_call(torch, rid):
    sys_ = _mixed()
    S = rid.System(sys_.n_atoms, sys_.quads, sys_.mask)
    E, _ = _ens(rid, sys_, [256] * 4, 4, 1008)
    srv = rid.Server(1 << 30, n_streams=2)
    mid = srv.register(S, E, 2.0, 3.0)
    pos = ridgen.f32(ridgen.chain_coords(sys_, 37, 3))
    got = srv.wait(srv.submit(mid, pos))
    ref = rid.bias_force(S, E, _dev(torch, pos), 2.0, 3.0)
    torch.cuda.synchronize()
    assert np.array_equal(got["F"], ref["F"].cpu().numpy())
    assert np.array_equal(got["eps"], ref["eps"].cpu().numpy())
    srv.close()


def test_masked_select_matches_oracle(torch, rid):
    # exploration frames with every fourth CV turned into a raw, distance-like
    # value (not periodic): the deviation uses the raw encoding and the
    # clustering distance leaves those CVs unwrapped
    n, widths, K = 38, [64, 64], 4
    mask = np.ones(n, np.uint8)
    mask[::4] = 0
    raw = ~mask.astype(bool)
    params = ridgen.xavier_ensemble(2 * n, widths, K, 22, bias_std=0.1)
    models = ridgen.unpack_params(params, 2 * n, widths, K)
    s = ridgen.exploration_frames(16, 125, n, 30, 0.3, seed=15)
    s[:, raw] = (1.0 + 1.5 * s[:, raw]).astype(np.float32)
    eps_ref = O.frame_deviation(models, s.astype(np.float64), mask)
    e = np.sort(eps_ref)
    mid = len(e) // 2
    k = mid - 200 + int(np.argmax(np.diff(e[mid - 200:mid + 200])))
    eps0 = 0.5 * (e[k] + e[k + 1])
    gap = e[k + 1] - e[k]
    assert gap > 1e-4 * e[k]
    ref = O.select_frames(models, s, eps0, 0.5, 30, 45, 50, adapt=True, mask=mask)
    E = rid.Ensemble(n, widths, K, params)
    E.set_angular_mask(mask)
    out = rid.select(E, torch.from_numpy(s).cuda(), eps0, 0.5, 30, 45, 50, adapt=True)
    torch.cuda.synchronize()
    eps = out["eps"].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(eps - eps_ref) / eps_ref) < 1e-4
    assert np.min(np.abs(eps - eps0)) > 0.25 * gap
    print(f"masked selection: {len(ref['selected'])} of {ref['n_clusters']} clusters, "
          f"threshold {ref['threshold']}", flush=True)
    assert np.float32(out["threshold"]) == ref["threshold"]
    assert out["n_clusters"] == ref["n_clusters"]
    assert out["selected"].cpu().numpy().tolist() == ref["selected"]
    assert np.array_equal(out["labels"].cpu().numpy().astype(np.int64), ref["labels"])
    # the periodic clustering of the same frames differs (the mask matters)
    plain = O.leader_cluster(s, ref["threshold"], ref["keep"], 51)
    assert not np.array_equal(plain[0], ref["labels"])


def test_mixed_refusals(torch, rid):
    sys_ = _mixed()
    S = rid.System(sys_.n_atoms, sys_.quads, sys_.mask)
    E, _ = _ens(rid, sys_, [64, 64], 2, 1009)
    pos = _dev(torch, ridgen.f32(ridgen.chain_coords(sys_, 8, 1)))
    s = _dev(torch, ridgen.f32(ridgen.torus_samples(8, sys_.n_cv, 2)))
    # (training and conservative switching take mixed tables: their parity
    # is in tests/test_gpu_train.py and tests/test_gpu_conservative.py)
    # MCMC on raw CVs needs their sampling box first
    with pytest.raises(rid.RidError, match="EINVAL"):
        rid.mcmc_run(E, s.clone(), 1, 1.0, 0.3, 1)
    # the ensemble's mask must match the system's CV kinds
    E2, _ = _ens(rid, sys_, [64, 64], 2, 1010)
    E2.set_angular_mask(None)
    with pytest.raises(rid.RidError, match="EINVAL"):
        rid.bias_force(S, E2, pos, 2.0, 3.0)
    with pytest.raises(rid.RidError, match="EINVAL"):
        rid.bias_force(S, E2, pos, 2.0, 3.0, conservative=True)
    # malformed tables
    bad = sys_.quads.copy()
    drow = int(np.nonzero(sys_.mask == 0)[0][0])
    bad[drow, 3] = 5
    with pytest.raises(rid.RidError, match="EINVAL"):
        rid.System(sys_.n_atoms, bad, sys_.mask)
    bad_mask = sys_.mask.copy()
    bad_mask[0] = 2
    with pytest.raises(rid.RidError, match="EINVAL"):
        rid.System(sys_.n_atoms, sys_.quads, bad_mask)
