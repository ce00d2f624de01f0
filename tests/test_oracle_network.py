"""Pins of the oracle's ensemble network, model deviation, switch and the
whole bias path: closed forms, finite differences, invariants."""
import math

import numpy as np
import pytest

import ridgen
from oracle import rid_oracle as O


def _models(n_in, widths, K, seed, bias_std=0.1):
    p = ridgen.xavier_ensemble(n_in, widths, K, seed, bias_std)
    return ridgen.unpack_params(p, n_in, widths, K)


def test_mlp_zero_hidden_layers_closed_form():
    rng = np.random.default_rng(1)
    n = 3
    wo = rng.normal(size=2 * n); bo = 0.4
    model = ([], [], wo, bo)
    s = rng.uniform(-3, 3, size=(5, n))
    A, g = O.ensemble_mean_force([model], s)
    expect_A = np.cos(s) @ wo[:n] + np.sin(s) @ wo[n:] + bo
    expect_g = -np.sin(s) * wo[:n] + np.cos(s) * wo[n:]
    assert np.allclose(A[:, 0], expect_A, rtol=0, atol=1e-14)
    assert np.allclose(g[:, 0], expect_g, rtol=0, atol=1e-14)


def test_mlp_one_unit_closed_form():
    rng = np.random.default_rng(2)
    w = rng.normal(size=4); b = 0.3; wo = np.array([1.7]); bo = -0.2
    model = ([w[None, :]], [np.array([b])], wo, bo)
    x = rng.normal(size=(6, 4))
    A, u0 = O.mlp_value_and_grad(model, x)
    t = np.tanh(x @ w + b)
    assert np.allclose(A, 1.7 * t - 0.2, atol=1e-14)
    assert np.allclose(u0, (1.7 * (1 - t * t))[:, None] * w[None, :], atol=1e-14)


def test_mlp_two_layers_written_out_by_hand():
    # width-2 layers with non-symmetric weights, every unit written out as a
    # scalar expression (catches a transposed operand or a dropped bias).
    W1 = np.array([[0.3, -1.1, 0.5], [0.9, 0.2, -0.4]]); b1 = np.array([0.1, -0.2])
    W2 = np.array([[1.3, -0.7], [0.25, 0.8]]); b2 = np.array([0.05, 0.3])
    wo = np.array([0.6, -1.4]); bo = 0.25
    x = np.array([0.2, -0.5, 0.9])
    p = math.tanh(0.3 * 0.2 - 1.1 * -0.5 + 0.5 * 0.9 + 0.1)
    q = math.tanh(0.9 * 0.2 + 0.2 * -0.5 - 0.4 * 0.9 - 0.2)
    r = math.tanh(1.3 * p - 0.7 * q + 0.05)
    t = math.tanh(0.25 * p + 0.8 * q + 0.3)
    A_hand = 0.6 * r - 1.4 * t + 0.25
    A, u0 = O.mlp_value_and_grad(([W1, W2], [b1, b2], wo, bo), x[None])
    assert abs(A[0] - A_hand) < 1e-15
    # dA/dx written out by the chain rule unit by unit
    dr, dt = 0.6 * (1 - r * r), -1.4 * (1 - t * t)
    dp = dr * 1.3 + dt * 0.25
    dq = dr * -0.7 + dt * 0.8
    dp *= 1 - p * p
    dq *= 1 - q * q
    grad = [dp * 0.3 + dq * 0.9, dp * -1.1 + dq * 0.2, dp * 0.5 + dq * -0.4]
    assert np.allclose(u0[0], grad, atol=1e-15)


def test_input_gradient_finite_differences():
    models = _models(6, [7, 5, 4], 1, seed=3)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(3, 6))
    A, u0 = O.mlp_value_and_grad(models[0], x)
    h = 1e-6
    for j in range(6):
        e = np.zeros(6); e[j] = h
        fd = (O.mlp_value_and_grad(models[0], x + e)[0] - O.mlp_value_and_grad(models[0], x - e)[0]) / (2 * h)
        assert np.max(np.abs(fd - u0[:, j])) < 1e-8


def test_mean_force_finite_differences_in_s():
    n = 4
    models = _models(2 * n, [9, 9], 2, seed=5)
    s = np.random.default_rng(6).uniform(-3, 3, size=(3, n))
    A, g = O.ensemble_mean_force(models, s)
    h = 1e-6
    for i in range(n):
        e = np.zeros(n); e[i] = h
        fd = (O.ensemble_mean_force(models, s + e)[0] - O.ensemble_mean_force(models, s - e)[0]) / (2 * h)
        assert np.max(np.abs(fd - g[:, :, i])) < 1e-8


def test_periodicity():
    n = 5
    models = _models(2 * n, [8, 8, 8], 3, seed=7)
    s = np.random.default_rng(8).uniform(-math.pi, math.pi, size=(4, n))
    m = np.random.default_rng(9).integers(-10, 11, size=s.shape)
    A1, g1 = O.ensemble_mean_force(models, s)
    A2, g2 = O.ensemble_mean_force(models, s + 2 * math.pi * m)
    assert np.max(np.abs(A1 - A2)) < 1e-12
    assert np.max(np.abs(g1 - g2)) < 1e-12


def test_model_deviation_identical_members_is_exactly_zero():
    g1 = np.random.default_rng(1).normal(size=(7, 1, 5))
    g = np.repeat(g1, 4, axis=1)
    gbar, eps = O.model_deviation(g)
    assert np.all(eps == 0.0)


def test_model_deviation_two_members():
    g = np.random.default_rng(2).normal(size=(6, 2, 3))
    gbar, eps = O.model_deviation(g)
    assert np.allclose(eps, np.linalg.norm(g[:, 0] - g[:, 1], axis=-1) / 2, atol=1e-15)
    assert np.allclose(gbar, 0.5 * (g[:, 0] + g[:, 1]), atol=1e-15)


def test_model_deviation_matches_population_variance():
    g = np.random.default_rng(3).normal(size=(6, 5, 4))
    gbar, eps = O.model_deviation(g)
    assert np.allclose(eps ** 2, np.var(g, axis=1, ddof=0).sum(axis=-1), atol=1e-14)
    perm = g[:, [3, 1, 4, 0, 2]]
    assert np.allclose(O.model_deviation(perm)[1], eps, atol=1e-14)


def test_single_member_has_zero_deviation():
    g = np.random.default_rng(4).normal(size=(3, 1, 4))
    assert np.all(O.model_deviation(g)[1] == 0.0)


def test_switch_limits_and_shape():
    e0, e1 = 2.0, 3.0
    sig, reg = O.switch(np.array([e0 - 1e-9, e0, 2.5, e1 - 1e-12, e1, 10.0, 0.0]), e0, e1)
    assert sig[0] == 1.0 and reg[0] == 0
    assert sig[1] == 1.0 and reg[1] == 1
    assert abs(sig[2] - 0.5) < 1e-15 and reg[2] == 1
    assert sig[3] < 1e-20 and reg[3] == 1
    assert sig[4] == 0.0 and reg[4] == 2
    assert sig[5] == 0.0 and sig[6] == 1.0
    e = np.linspace(1.5, 3.5, 2001)
    s, _ = O.switch(e, e0, e1)
    assert np.all(np.diff(s) <= 0)
    assert np.max(np.abs(np.diff(s))) < 2e-3       # continuous


def _bias_setup(seed=10):
    sys_ = ridgen.system_dipeptide()
    pos = ridgen.chain_coords(sys_, 4, seed=seed)
    models = _models(2 * sys_.n_cv, [6, 5], 4, seed=20)
    return sys_, pos, models


@pytest.mark.parametrize("band", ["full", "switching", "none"])
def test_bias_force_is_minus_gradient_of_energy(band):
    sys_, pos, models = _bias_setup()
    out = O.bias_force(pos, sys_.quads, models, 1e9, 2e9)
    eps = out["eps"]
    if band == "full":
        e0, e1 = 10 * eps.max(), 20 * eps.max()
    elif band == "switching":
        e0, e1 = 0.5 * eps.min(), 2.0 * eps.max()
    else:
        e0, e1 = 0.1 * eps.min(), 0.2 * eps.min()
    out = O.bias_force(pos, sys_.quads, models, e0, e1)
    sigma = out["sigma"]
    if band == "switching":
        assert np.all((sigma > 0) & (sigma < 1))
    F = out["F"]
    h = 1e-6
    fd = np.zeros_like(F)
    for a in range(sys_.n_atoms):
        for k in range(3):
            p1 = pos.copy(); p1[:, a, k] += h
            p2 = pos.copy(); p2[:, a, k] -= h
            fd[:, a, k] = -(O.bias_energy_frozen(p1, sys_.quads, models, sigma)
                            - O.bias_energy_frozen(p2, sys_.quads, models, sigma)) / (2 * h)
    scale = max(np.max(np.abs(F)), 1e-30)
    assert np.max(np.abs(fd - F)) <= 1e-6 * scale + (1e-12 if band == "none" else 0)
    if band == "none":
        assert np.all(F == 0.0) and np.all(out["E"] == 0.0)


def test_total_force_and_torque_vanish():
    sys_ = ridgen.system_peptide20()
    pos = ridgen.chain_coords(sys_, 3, seed=12)
    models = _models(2 * sys_.n_cv, [16, 16], 3, seed=30)
    out = O.bias_force(pos, sys_.quads, models, 2.0, 3.0)
    F = out["F"]
    scale = np.max(np.linalg.norm(F, axis=-1))
    assert np.max(np.abs(F.sum(axis=1))) < 1e-10 * scale
    assert np.max(np.abs(np.cross(pos, F).sum(axis=1))) < 1e-10 * scale


def test_metrics():
    ref = np.array([[1.0, -2.0], [0.5, 0.25]])
    test = ref + np.array([[0.02, 0.0], [0.0, -0.005]])
    assert abs(O.max_rel_err(test, ref) - 0.01) < 1e-15
