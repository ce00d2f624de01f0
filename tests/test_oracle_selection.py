"""Pins of the oracle's selection phase (model-deviation filter and
threshold clustering of CV frames) against hand-worked cases, brute force
and the limits of the threshold."""
import math

import numpy as np

import ridgen
from oracle import rid_oracle as O


def test_hand_worked_periodic_example():
    # one CV; threshold 0.2: 0.1 and 0.05 join frame 0; 3.0 founds cluster 1;
    # -3.1 is 2pi - 6.1 = 0.183 from 3.0 across the periodic boundary and
    # joins it; 1.5 founds cluster 2
    s = np.array([[0.0], [0.1], [3.0], [0.05], [-3.1], [1.5]])
    labels, leaders, n = O.leader_cluster(s, 0.2)
    assert labels.tolist() == [0, 0, 1, 0, 1, 2]
    assert leaders == [0, 2, 5] and n == 3
    # the same with 0.18 leaves -3.1 on its own
    labels, leaders, n = O.leader_cluster(s, 0.18)
    assert labels.tolist() == [0, 0, 1, 0, 2, 3] and leaders == [0, 2, 4, 5]


def test_fp32_distance_matches_fp64_periodic_distance():
    rng = np.random.default_rng(1)
    a = rng.uniform(-math.pi, math.pi, size=(500, 38)).astype(np.float32)
    b = rng.uniform(-math.pi, math.pi, size=(500, 38)).astype(np.float32)
    d = a.astype(np.float64) - b.astype(np.float64)
    d = (d + math.pi) % (2 * math.pi) - math.pi
    ref = np.sum(d * d, axis=1)
    got = O.cv_distance_sq_f32(a, b).astype(np.float64)
    assert np.max(np.abs(got - ref) / ref) < 1e-5
    # symmetric bit for bit (the wrap negates exactly)
    assert np.array_equal(O.cv_distance_sq_f32(a, b), O.cv_distance_sq_f32(b, a))
    # near-opposite boundary points are close
    assert abs(float(O.cv_distance_sq_f32([math.pi - 0.01], [-math.pi + 0.01])) - 0.0004) < 1e-6


def _brute_force_checks(s, labels, leaders, t, keep=None):
    t2 = np.float32(np.float32(t) * np.float32(t))
    B = len(s)
    d2 = O.cv_distance_sq_f32(s[:, None, :], s[None, :, :])     # [B][B]
    for L, f in enumerate(leaders):
        assert labels[f] == L
        # a leader is farther than the threshold from every earlier leader
        assert np.all(d2[f, leaders[:L]] > t2)
    for f in range(B):
        if keep is not None and not keep[f]:
            assert labels[f] == -2
            continue
        L = labels[f]
        assert 0 <= L < len(leaders)
        assert leaders[L] <= f
        if leaders[L] != f:
            assert d2[f, leaders[L]] <= t2
            # no earlier cluster would have taken it (first match)
            assert np.all(d2[f, leaders[:L]] > t2)


def test_brute_force_first_match_and_leader_separation():
    s = ridgen.exploration_frames(6, 60, 5, 7, 0.3, seed=3)
    for t in (0.5, 1.0, 2.0):
        labels, leaders, n = O.leader_cluster(s, t)
        assert n == len(leaders)
        _brute_force_checks(s, labels, leaders, t)


def test_threshold_limits():
    s = ridgen.exploration_frames(3, 40, 4, 5, 0.3, seed=4)
    labels, leaders, n = O.leader_cluster(s, 100.0)          # everything within
    assert n == 1 and np.all(labels == 0)
    labels, leaders, n = O.leader_cluster(s, 0.0)            # distinct frames
    assert n == len(s) and labels.tolist() == list(range(len(s)))


def test_mask_equals_run_on_kept_subset():
    s = ridgen.exploration_frames(4, 50, 6, 5, 0.3, seed=5)
    keep = np.random.default_rng(2).uniform(size=len(s)) < 0.6
    labels, leaders, n = O.leader_cluster(s, 1.2, keep)
    sub_labels, sub_leaders, sub_n = O.leader_cluster(s[keep], 1.2)
    idx = np.nonzero(keep)[0]
    assert n == sub_n
    assert leaders == [int(idx[i]) for i in sub_leaders]
    assert np.array_equal(labels[keep], sub_labels) and np.all(labels[~keep] == -2)
    _brute_force_checks(s, labels, leaders, 1.2, keep)


def test_cap_reports_more_than_cap():
    s = ridgen.exploration_frames(2, 50, 4, 5, 0.3, seed=6)
    labels, leaders, n = O.leader_cluster(s, 0.0, max_clusters=7)
    assert len(leaders) == 7 and n == 8
    assert labels.tolist()[:7] == list(range(7)) and np.all(labels[7:] == -1)


def test_adaptation_reaches_the_window_on_separated_clusters():
    # 40 basins far apart, tight spread: the count can be brought into
    # [30, 45] from a threshold that is too small and from one too large
    s = ridgen.exploration_frames(40, 30, 6, 40, 0.05, seed=7)
    for t0 in (0.01, 20.0):
        t, (labels, leaders, n) = O.adapt_threshold(s, t0, 30, 45)
        assert 30 <= n <= 45, (t0, t, n)
    # already inside: unchanged
    t1, _ = O.adapt_threshold(s, t, 30, 45)
    assert t1 == t


def test_selection_filters_and_caps():
    sys_n, widths, K = 4, [16, 16], 3
    params = ridgen.xavier_ensemble(2 * sys_n, widths, K, 11, bias_std=0.1)
    models = ridgen.unpack_params(params, 2 * sys_n, widths, K)
    s = ridgen.exploration_frames(5, 40, sys_n, 6, 0.3, seed=8).astype(np.float64)
    eps = O.frame_deviation(models, s)
    eps0 = float(np.quantile(eps, 0.4))
    r = O.select_frames(models, s, eps0, 0.5, 3, 6, 4, adapt=True)
    assert np.array_equal(r["keep"], eps >= eps0)
    assert len(r["selected"]) <= 4
    assert all(r["keep"][f] for f in r["selected"])
    assert r["selected"] == r["leaders"][:4]
    # identical members: no deviation, nothing reaches a positive eps0
    same = [models[0]] * 3
    assert np.all(O.frame_deviation(same, s) == 0.0)
    assert O.select_frames(same, s, 1e-9, 0.5, 3, 6, 4)["selected"] == []


# --- per-CV clustering weights (CV settings "weights") ---------------------

def test_unit_weights_are_the_unweighted_metric_bit_for_bit():
    rng = np.random.default_rng(11)
    a = rng.uniform(-math.pi, math.pi, size=(300, 38)).astype(np.float32)
    b = rng.uniform(-math.pi, math.pi, size=(300, 38)).astype(np.float32)
    assert np.array_equal(O.cv_distance_sq_f32(a, b, weights=np.ones(38)),
                          O.cv_distance_sq_f32(a, b))


def test_zero_weight_removes_the_cv_from_the_metric():
    # a zero weight contributes an exact 0 to the FP32 sum, so the distance
    # equals the distance over the remaining CVs (in the same order)
    rng = np.random.default_rng(12)
    a = rng.uniform(-math.pi, math.pi, size=(200, 9)).astype(np.float32)
    b = rng.uniform(-math.pi, math.pi, size=(200, 9)).astype(np.float32)
    w = np.ones(9)
    w[[2, 7]] = 0.0
    keep = [i for i in range(9) if w[i] != 0]
    assert np.array_equal(O.cv_distance_sq_f32(a, b, weights=w),
                          O.cv_distance_sq_f32(a[:, keep], b[:, keep]))


def test_weight_four_on_a_raw_cv_is_the_cv_scaled_by_two():
    # raw (non-angular) CVs are not wrapped, and multiplying a difference by
    # 2 or its FP32 square by 4 are both exact: the weighted metric equals
    # the unweighted metric on the table with that column doubled
    rng = np.random.default_rng(13)
    a = rng.uniform(0.3, 1.5, size=(200, 5)).astype(np.float32)
    b = rng.uniform(0.3, 1.5, size=(200, 5)).astype(np.float32)
    mask = np.array([1, 0, 1, 0, 1], dtype=np.uint8)
    w = np.array([1, 4, 1, 1, 1], dtype=np.float32)
    a2, b2 = a.copy(), b.copy()
    a2[:, 1] *= 2
    b2[:, 1] *= 2
    assert np.array_equal(O.cv_distance_sq_f32(a, b, mask, w), O.cv_distance_sq_f32(a2, b2, mask))


def test_weighted_clustering_against_brute_force():
    # every label is the first leader within the threshold under the
    # weighted metric, every leader is farther than the threshold from all
    # earlier leaders, and a heavy weight on one CV splits clusters the
    # unweighted metric merges
    rng = np.random.default_rng(14)
    centers = rng.uniform(-math.pi, math.pi, size=(6, 4))
    s = (centers[rng.integers(0, 6, 400)] + 0.15 * rng.standard_normal((400, 4)))
    s = ((s + math.pi) % (2 * math.pi) - math.pi).astype(np.float32)
    w = np.array([1.0, 0.25, 9.0, 1.0], dtype=np.float32)
    t = np.float32(0.9)
    labels, leaders, n = O.leader_cluster(s, t, weights=w)
    t2 = np.float32(t * t)
    for f in range(len(s)):
        d2 = [float(O.cv_distance_sq_f32(s[l], s[f], weights=w)) for l in leaders]
        within = [j for j, v in enumerate(d2) if v <= t2]
        assert labels[f] == within[0]
    for j, l in enumerate(leaders):
        for l0 in leaders[:j]:
            assert O.cv_distance_sq_f32(s[l0], s[l], weights=w) > t2
    _, _, n_flat = O.leader_cluster(s, t)
    w_heavy = np.array([1, 1, 400, 1], dtype=np.float32)
    _, _, n_heavy = O.leader_cluster(s, t, weights=w_heavy)
    assert n_heavy > n_flat


# --- trust-level adjustment (numb_cluster_threshold) ----------------------

def test_trust_levels_raised_only_below_the_cluster_threshold():
    # the paper's example: numb_cluster_threshold 15, trust levels 2 and 3
    assert O.adjust_trust_levels(14, 15, 2.0, 3.0, 1.5) == (3.0, 4.5)
    assert O.adjust_trust_levels(0, 15, 2.0, 3.0, 1.5) == (3.0, 4.5)
    assert O.adjust_trust_levels(15, 15, 2.0, 3.0, 1.5) == (2.0, 3.0)
    assert O.adjust_trust_levels(45, 15, 2.0, 3.0, 1.5) == (2.0, 3.0)
    # repeated adjustment compounds and keeps the ratio of the levels
    l1, l2 = 2.0, 3.0
    for _ in range(3):
        l1, l2 = O.adjust_trust_levels(5, 15, l1, l2, 2.0)
    assert (l1, l2) == (16.0, 24.0)
    for bad in [(1.0,), (0.5,), (math.inf,), (math.nan,)]:
        try:
            O.adjust_trust_levels(5, 15, 2.0, 3.0, *bad)
            assert False, bad
        except ValueError:
            pass
    try:
        O.adjust_trust_levels(5, 15, 3.0, 2.0, 1.5)
        assert False
    except ValueError:
        pass
