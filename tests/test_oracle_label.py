"""Pins of the oracle's restrained-MD mean-force estimate."""
import json
import math
import os

import numpy as np

import ridgen
from oracle import rid_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_config.json")


def test_gaussian_frames_recover_true_force():
    kappa = json.load(open(GOLDEN))["kappa_dihedral"]["value"]
    M, T, n, sd = 40, 2000, 6, 0.25
    traj, s0, F_true = ridgen.restrained_traj(M, T, n, kappa, seed=1, frame_std=sd)
    F, SE, keep = O.mf_label(traj, s0, np.full(n, kappa), np.ones(n), 1e9)
    # frames are rounded to FP32; the rounding bias is far below 4 sigma
    bound = 4 * kappa * sd / math.sqrt(T)
    assert np.max(np.abs(F - F_true)) < bound
    # block SE estimates kappa * sd / sqrt(T) for iid frames
    ratio = SE / (kappa * sd / math.sqrt(T))
    assert 0.3 < np.median(ratio) < 1.7


def test_wrap_example():
    traj = np.full((1, 10, 1), -math.pi + 0.01)
    s0 = np.array([[math.pi - 0.01]])
    F, SE, keep = O.mf_label(traj, s0, np.array([500.0]), np.array([1]), 5.0)
    assert abs(F[0, 0] - 500.0 * -0.02) < 1e-9
    assert SE[0, 0] == 0.0 and keep[0] == 1


def test_non_periodic_cv_is_not_wrapped():
    traj = np.full((1, 10, 1), -3.0)
    s0 = np.array([[3.0]])
    F, _, _ = O.mf_label(traj, s0, np.array([2.0]), np.array([0]), 5.0)
    assert F[0, 0] == 12.0


def test_threshold_decides_keep():
    rng = np.random.default_rng(5)
    traj = rng.normal(0.0, 0.3, size=(2, 100, 3))
    traj[1] = 0.0
    F, SE, keep = O.mf_label(traj, np.zeros((2, 3)), np.full(3, 500.0), np.ones(3), 1.0)
    assert keep[0] == 0 and keep[1] == 1
    assert np.all(SE[1] == 0.0)


def test_compensated_sum_matches_exact_sum():
    rng = np.random.default_rng(6)
    x = rng.normal(size=(3, 5000)) * 10.0 ** rng.integers(-8, 8, size=(3, 5000))
    got = O._neumaier_sum(x, axis=1)
    exact = np.array([math.fsum(r) for r in x])
    assert np.all(np.abs(got - exact) <= 2 * np.spacing(np.abs(exact)))


def test_block_standard_error_closed_form():
    """Blocks whose frames all carry one spring force: block j of 10 frames
    at force j (j = 0..9), then 5 tail frames at force 100.  The block means
    are 0..9, so SE = sqrt(sum (j - 4.5)^2 / 9 / 10) = sqrt(82.5 / 90) (a
    denominator of 10 instead of 9 would give sqrt(82.5 / 100)); the tail
    frames enter the mean force but no block.  kappa = 100 keeps every frame
    inside (-pi, pi], so the periodic and the raw CV agree."""
    kappa = 100.0
    forces = np.concatenate([np.repeat(np.arange(10.0), 10), np.full(5, 100.0)])
    traj = (-forces / kappa).reshape(1, 105, 1)      # spring = kappa (0 - s) = force
    for mask in (1, 0):
        F, SE, keep = O.mf_label(traj, np.zeros((1, 1)), np.array([kappa]), np.array([mask]),
                                 0.96)
        assert abs(F[0, 0] - (10 * 45.0 + 500.0) / 105) < 1e-12
        assert abs(SE[0, 0] - math.sqrt(82.5 / 90)) < 1e-12
        assert abs(SE[0, 0] - math.sqrt(82.5 / 100)) > 0.04
        assert keep[0] == 1                            # 0.957 <= 0.96
    _, _, keep = O.mf_label(traj, np.zeros((1, 1)), np.array([kappa]), np.array([1]), 0.95)
    assert keep[0] == 0
