"""GPU parity of the selection phase (rid_cluster_frames, rid_select)
against the oracle, through the C ABI.  Cluster labels, leaders, counts and
adapted thresholds are integer / FP32-decided results: both sides decide
d^2 <= t^2 in the same FP32 arithmetic, so they must agree exactly."""
import functools

import numpy as np
import pytest

import ridgen
from oracle import rid_oracle as O

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


def _gpu_cluster(torch, rid, s, t, **kw):
    eps = kw.pop("eps", None)
    out = rid.cluster_frames(torch.from_numpy(s).cuda(), t,
                             eps=None if eps is None else torch.from_numpy(eps).cuda(), **kw)
    torch.cuda.synchronize()
    return (out["labels"].cpu().numpy().astype(np.int64), out["leaders"].cpu().numpy().tolist(),
            out["n_clusters"], out["threshold"])


@pytest.mark.parametrize("t", [0.8, 1.5, 3.0])
def test_cluster_matches_oracle_exactly(torch, rid, t):
    # 3000 frames of 38 CVs from 20 walkers over 30 basins: spans the growing
    # chunks (64, 128, ... frames) and a ragged last chunk
    s = ridgen.exploration_frames(20, 150, 38, 30, 0.3, seed=11)
    labels, leaders, n = O.leader_cluster(s, t)
    gl, gld, gn, _ = _gpu_cluster(torch, rid, s, t)
    print(f"t={t}: {n} clusters", flush=True)
    assert gn == n and gld == leaders
    assert np.array_equal(gl, labels)


def test_cluster_filter_and_cap(torch, rid):
    s = ridgen.exploration_frames(8, 100, 38, 20, 0.3, seed=12)
    eps = np.random.default_rng(3).uniform(0.0, 1.0, size=len(s)).astype(np.float32)
    keep = eps >= np.float32(0.4)
    labels, leaders, n = O.leader_cluster(s, 1.0, keep)
    gl, gld, gn, _ = _gpu_cluster(torch, rid, s, 1.0, eps=eps, eps0=0.4)
    assert gn == n and gld == leaders and np.array_equal(gl, labels)
    assert np.all(gl[~keep] == -2)
    # cap: 10 clusters at most, the count says "more"
    labels, leaders, n = O.leader_cluster(s, 0.5, keep, max_clusters=10)
    gl, gld, gn, _ = _gpu_cluster(torch, rid, s, 0.5, eps=eps, eps0=0.4, max_clusters=10)
    assert n == 11 and gn == 11 and gld == leaders and np.array_equal(gl, labels)
    assert np.any(gl == -1)


def test_cluster_cap_filling_in_a_late_chunk(torch, rid):
    # 23 clusters at t = 3 with leaders spread over the 3000 frames: a cap of
    # 20 fills inside a 2048-frame chunk, the walk stops there, and the
    # following rounds label the remaining frames (joined or over the cap)
    s = ridgen.exploration_frames(20, 150, 38, 30, 0.3, seed=11)
    labels, leaders, n = O.leader_cluster(s, 3.0, max_clusters=20)
    assert n == 21 and leaders[-1] > 1984
    gl, gld, gn, _ = _gpu_cluster(torch, rid, s, 3.0, max_clusters=20)
    assert gn == n and gld == leaders and np.array_equal(gl, labels)
    assert np.any(gl == -1)


@pytest.mark.parametrize("B,n", [(1, 38), (2, 1), (65, 3)])
def test_cluster_tiny_inputs(torch, rid, B, n):
    # a single frame founds the only cluster; one CV; a ragged second chunk
    s = ridgen.f32(ridgen.torus_samples(B, n, 21))
    for t in (0.3, 10.0):
        labels, leaders, nc = O.leader_cluster(s, t)
        gl, gld, gn, _ = _gpu_cluster(torch, rid, s, t)
        assert gn == nc and gld == leaders and np.array_equal(gl, labels)


def test_cluster_every_frame_filtered(torch, rid):
    # no frame reaches the lower trust level: no cluster, every label -2
    s = ridgen.f32(ridgen.torus_samples(300, 38, 22))
    eps = np.full(300, 0.1, np.float32)
    gl, gld, gn, _ = _gpu_cluster(torch, rid, s, 1.0, eps=eps, eps0=0.5)
    assert gn == 0 and gld == [] and np.all(gl == -2)


def test_cluster_many_leaders_restarts_chunks(torch, rid):
    # 256 CVs leave room for 64 new leaders per chunk in LDS; uniform frames
    # at a small threshold found hundreds, so the walk stops and restarts
    s = ridgen.torus_samples(600, 256, 13).astype(np.float32)
    labels, leaders, n = O.leader_cluster(s, 20.0)
    assert n > 300
    gl, gld, gn, _ = _gpu_cluster(torch, rid, s, 20.0)
    assert gn == n and gld == leaders and np.array_equal(gl, labels)


@pytest.mark.parametrize("t0", [0.05, 40.0])
def test_threshold_adaptation_matches_oracle(torch, rid, t0):
    s = ridgen.exploration_frames(40, 30, 6, 40, 0.05, seed=7)
    t, (labels, leaders, n) = O.adapt_threshold(s, t0, 30, 45)
    gl, gld, gn, gt = _gpu_cluster(torch, rid, s, t0, adapt=True, lower=30, upper=45)
    assert np.float32(gt) == t and gn == n and gld == leaders and np.array_equal(gl, labels)
    assert 30 <= gn <= 45


@functools.lru_cache(maxsize=None)
def _adapted_3000():
    s = ridgen.exploration_frames(20, 150, 38, 30, 0.3, seed=11)
    return s, O.adapt_threshold(s, 1.5, 30, 45)   # five steps up: 1.5 -> 2.42


@pytest.mark.parametrize("max_clusters", [4096, 560_000, 2_000_000])
def test_threshold_adaptation_with_few_slots(torch, rid, max_clusters):
    # 38 CVs: a cap of 560k clusters leaves room for 3 thresholds per pass in
    # the 256 MiB scratch budget, 2M for one (labels then go straight to the
    # caller's buffer); 4096 takes the full 24.  The cap is never reached.
    s, (t, (labels, leaders, n)) = _adapted_3000()
    gl, gld, gn, gt = _gpu_cluster(torch, rid, s, 1.5, adapt=True, lower=30, upper=45,
                                   max_clusters=max_clusters)
    print(f"cap {max_clusters}: t={t} n={n}", flush=True)
    assert np.float32(gt) == t and gn == n and gld == leaders and np.array_equal(gl, labels)


def test_threshold_adaptation_that_never_settles(torch, rid):
    # 50 frames at equal mutual distance sqrt(2) (frame i has CV i = 1):
    # below sqrt(2) every frame founds a cluster, at or above it one frame
    # leads them all, so the count never enters [10, 20]; the threshold
    # steps back and forth until the 100th adjustment ends the rule
    s = np.eye(50, dtype=np.float32)
    for t0 in (1.3, 1.5):
        t, (labels, leaders, n) = O.adapt_threshold(s, t0, 10, 20)
        gl, gld, gn, gt = _gpu_cluster(torch, rid, s, t0, adapt=True, lower=10, upper=20)
        assert n in (1, 50)
        assert np.float32(gt) == t and gn == n and gld == leaders and np.array_equal(gl, labels)


def test_select_matches_oracle(torch, rid):
    n, widths, K = 38, [64, 64], 4
    params = ridgen.xavier_ensemble(2 * n, widths, K, 21, bias_std=0.1)
    models = ridgen.unpack_params(params, 2 * n, widths, K)
    s = ridgen.exploration_frames(16, 125, n, 30, 0.3, seed=14)
    eps_ref = O.frame_deviation(models, s.astype(np.float64))
    # eps0 in the widest gap of the deviations around the median, so the FP32
    # deviation cannot fall on the other side
    e = np.sort(eps_ref)
    mid = len(e) // 2
    lo, hi = mid - 200, mid + 200
    k = lo + int(np.argmax(np.diff(e[lo:hi])))
    eps0 = 0.5 * (e[k] + e[k + 1])
    gap = e[k + 1] - e[k]
    assert gap > 1e-4 * e[k]
    ref = O.select_frames(models, s, eps0, 0.5, 30, 45, 50, adapt=True)
    E = rid.Ensemble(n, widths, K, params)
    out = rid.select(E, torch.from_numpy(s).cuda(), eps0, 0.5, 30, 45, 50, adapt=True)
    torch.cuda.synchronize()
    eps = out["eps"].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(eps - eps_ref) / eps_ref) < 1e-4
    assert np.min(np.abs(eps - eps0)) > 0.25 * gap
    print(f"selected {len(ref['selected'])} of {ref['n_clusters']} clusters, "
          f"threshold {ref['threshold']}", flush=True)
    assert np.float32(out["threshold"]) == ref["threshold"]
    assert out["n_clusters"] == ref["n_clusters"]
    assert out["selected"].cpu().numpy().tolist() == ref["selected"]
    assert np.array_equal(out["labels"].cpu().numpy().astype(np.int64), ref["labels"])


def test_select_benchmarked_workload_matches_oracle(torch, rid):
    """The selection the benchmark times: 20 000 frames, threshold 2.6
    adapted into [30, 45] (15 adjustments, chunks up to 8192 frames and
    full rounds), max_selection 50.  The oracle's result is stored by
    tests/golden/make_selection_golden.py (about a minute of CPU)."""
    import hashlib
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "selection_20k.json")))
    n, widths, K = 38, g["ensemble"]["widths"], g["ensemble"]["K"]
    params = ridgen.xavier_ensemble(2 * n, widths, K, g["ensemble"]["seed"])
    s = ridgen.exploration_frames(*g["frames"])
    E = rid.Ensemble(n, widths, K, params)
    out = rid.select(E, torch.from_numpy(s).cuda(), g["eps0"], g["threshold0"], *g["window"],
                     g["max_selection"], adapt=True)
    torch.cuda.synchronize()
    eps = out["eps"].cpu().numpy().astype(np.float64)
    # the FP32 deviations stay on the oracle's side of eps0
    assert np.min(np.abs(eps - g["eps0"])) > 0.25 * g["eps_gap"]
    assert int(np.sum(eps >= g["eps0"])) == g["n_kept"]
    labels = out["labels"].cpu().numpy().astype("<i8")
    print(f"threshold {out['threshold']}, {out['n_clusters']} clusters", flush=True)
    assert np.float32(out["threshold"]) == np.float32(g["threshold"])
    assert out["n_clusters"] == g["n_clusters"]
    # 30 clusters, under max_selection: the selected frames are every leader
    assert g["selected"] == g["leaders"][:g["max_selection"]]
    assert out["selected"].cpu().numpy().tolist() == g["selected"]
    assert hashlib.sha256(np.ascontiguousarray(labels).tobytes()).hexdigest() == g["labels_sha256"]


@pytest.mark.parametrize("masked", [False, True])
def test_weighted_select_matches_oracle(torch, rid, masked):
    """Selection with per-CV clustering weights (CV settings "weights"),
    alone and with an angular mask: labels, leaders, count and adapted
    threshold equal to the oracle's; weights of 1 give the unweighted
    result bit for bit, and the weights change the clustering."""
    n, widths, K = 38, [64, 64], 4
    params = ridgen.xavier_ensemble(2 * n, widths, K, 23, bias_std=0.1)
    models = ridgen.unpack_params(params, 2 * n, widths, K)
    s = ridgen.exploration_frames(16, 125, n, 30, 0.3, seed=16)
    mask = None
    if masked:
        mask = np.ones(n, np.uint8)
        mask[1::5] = 0
        raw = ~mask.astype(bool)
        s[:, raw] = (1.0 + 1.5 * s[:, raw]).astype(np.float32)
    w = np.random.default_rng(17).uniform(0.25, 2.0, n).astype(np.float32)
    w[[3, 11]] = 0.0                          # two CVs left out of the metric
    eps_ref = O.frame_deviation(models, s.astype(np.float64), mask)
    e = np.sort(eps_ref)
    mid = len(e) // 2
    k = mid - 200 + int(np.argmax(np.diff(e[mid - 200:mid + 200])))
    eps0 = 0.5 * (e[k] + e[k + 1])
    gap = e[k + 1] - e[k]
    assert gap > 1e-4 * e[k]
    ref = O.select_frames(models, s, eps0, 0.5, 30, 45, 50, adapt=True, mask=mask, weights=w)
    E = rid.Ensemble(n, widths, K, params)
    if masked:
        E.set_angular_mask(mask)
    E.set_cv_weights(w)
    sd = torch.from_numpy(s).cuda()
    out = rid.select(E, sd, eps0, 0.5, 30, 45, 50, adapt=True)
    torch.cuda.synchronize()
    eps = out["eps"].cpu().numpy().astype(np.float64)
    assert np.min(np.abs(eps - eps0)) > 0.25 * gap
    print(f"weighted selection (mask {masked}): {len(ref['selected'])} of "
          f"{ref['n_clusters']} clusters, threshold {ref['threshold']}", flush=True)
    assert np.float32(out["threshold"]) == ref["threshold"]
    assert out["n_clusters"] == ref["n_clusters"]
    assert out["selected"].cpu().numpy().tolist() == ref["selected"]
    assert np.array_equal(out["labels"].cpu().numpy().astype(np.int64), ref["labels"])
    # the weights matter: the unweighted clustering at the same threshold differs
    plain = O.leader_cluster(s, ref["threshold"], ref["keep"], 51, mask)
    assert not np.array_equal(plain[0], ref["labels"])
    # weights of 1 are the unweighted metric, bit for bit
    E.set_cv_weights(np.ones(n, np.float32))
    ones = rid.select(E, sd, eps0, 0.5, 30, 45, 50, adapt=True)
    E.set_cv_weights(None)
    none = rid.select(E, sd, eps0, 0.5, 30, 45, 50, adapt=True)
    torch.cuda.synchronize()
    assert np.array_equal(ones["labels"].cpu().numpy(), none["labels"].cpu().numpy())
    assert ones["threshold"] == none["threshold"] and ones["n_clusters"] == none["n_clusters"]
    ref1 = O.select_frames(models, s, eps0, 0.5, 30, 45, 50, adapt=True, mask=mask)
    assert np.array_equal(none["labels"].cpu().numpy().astype(np.int64), ref1["labels"])
    with pytest.raises(rid.RidError):
        E.set_cv_weights(-w)
    with pytest.raises(ValueError):
        E.set_cv_weights(w[:5])


def test_cluster_rejects_bad_arguments(torch, rid):
    s = torch.zeros((10, 300), dtype=torch.float32, device="cuda")
    with pytest.raises(rid.RidError):
        rid.cluster_frames(s, 1.0)
    s = torch.zeros((10, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(rid.RidError):
        rid.cluster_frames(s, 0.0)
    with pytest.raises(rid.RidError):
        rid.cluster_frames(s, 1.0, adapt=True, lower=5, upper=4)
