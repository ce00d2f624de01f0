"""Pins of the oracle's conservative switching (the switch differentiated
too): the input Hessian-vector product, the gradient of the model deviation
and the bias force, each against central finite differences, plus the
regions where it must reduce to the frozen-switch force."""
import math

import numpy as np
import pytest

import ridgen
from oracle import rid_oracle as O


def _models(n_in, widths, K, seed, bias_std=0.2):
    p = ridgen.xavier_ensemble(n_in, widths, K, seed, bias_std)
    return ridgen.unpack_params(p, n_in, widths, K)


@pytest.mark.parametrize("widths", [[], [7], [5, 4], [6, 6, 3]])
def test_input_hvp_finite_differences(widths):
    rng = np.random.default_rng(3)
    D = 6
    (m,) = _models(D, widths, 1, seed=11)
    x = rng.normal(size=(5, D))
    rho = rng.normal(size=(5, D))
    hv = O.mlp_input_hvp(m, x, rho)
    h = 1e-5
    fd = (O.mlp_value_and_grad(m, x + h * rho)[1] - O.mlp_value_and_grad(m, x - h * rho)[1]) / (2 * h)
    if not widths:   # A is linear in x: the Hessian is exactly zero
        assert np.all(hv == 0.0)
    else:
        assert np.max(np.abs(hv - fd)) <= 1e-8 * np.max(np.abs(fd))


def test_input_hvp_is_symmetric():
    # rho2 . H rho1 == rho1 . H rho2 (H is a Hessian)
    rng = np.random.default_rng(4)
    (m,) = _models(6, [8, 5], 1, seed=12)
    x = rng.normal(size=(3, 6))
    r1, r2 = rng.normal(size=(3, 6)), rng.normal(size=(3, 6))
    a = np.sum(r2 * O.mlp_input_hvp(m, x, r1), axis=1)
    b = np.sum(r1 * O.mlp_input_hvp(m, x, r2), axis=1)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-14)


def test_switch_slope_finite_differences():
    e0, e1 = 1.0, 2.5
    eps = np.linspace(1.05, 2.45, 15)
    h = 1e-7
    fd = (O.switch(eps + h, e0, e1)[0] - O.switch(eps - h, e0, e1)[0]) / (2 * h)
    assert np.allclose(O.switch_slope(eps, e0, e1), fd, atol=1e-7)
    assert np.all(O.switch_slope(np.array([0.5, 0.99, 2.5, 3.0]), e0, e1) == 0.0)
    assert O.switch_slope(np.array([1.75]), e0, e1)[0] == pytest.approx(-math.pi / 3.0)


def test_deviation_gradient_finite_differences():
    rng = np.random.default_rng(5)
    n = 4
    models = _models(2 * n, [6, 5], 3, seed=13)
    s = rng.uniform(-3, 3, size=(5, n))
    eps, de = O.deviation_gradient(models, s)
    h = 1e-6
    fd = np.zeros_like(s)
    for i in range(n):
        e = np.zeros(n); e[i] = h
        ep = O.model_deviation(O.ensemble_mean_force(models, s + e)[1])[1]
        em = O.model_deviation(O.ensemble_mean_force(models, s - e)[1])[1]
        fd[:, i] = (ep - em) / (2 * h)
    assert np.max(np.abs(de - fd)) <= 1e-7 * np.max(np.abs(fd))


def test_deviation_gradient_zero_for_identical_members():
    (m,) = _models(6, [5], 1, seed=14)
    s = np.random.default_rng(6).uniform(-3, 3, size=(4, 3))
    eps, de = O.deviation_gradient([m, m, m], s)
    assert np.all(eps == 0.0) and np.all(de == 0.0)


def _setup(seed=10):
    sys_ = ridgen.system_dipeptide()
    pos = ridgen.chain_coords(sys_, 4, seed=seed)
    models = _models(2 * sys_.n_cv, [6, 5], 4, seed=20)
    return sys_, pos, models


def test_conservative_force_is_minus_gradient_of_energy_in_the_band():
    sys_, pos, models = _setup()
    eps = O.bias_force(pos, sys_.quads, models, 1e9, 2e9)["eps"]
    e0, e1 = 0.5 * eps.min(), 2.0 * eps.max()
    out = O.bias_force_conservative(pos, sys_.quads, models, e0, e1)
    assert np.all((out["sigma"] > 0) & (out["sigma"] < 1))
    F = out["F"]
    h = 1e-6
    fd = np.zeros_like(F)
    for a in range(sys_.n_atoms):
        for k in range(3):
            p1 = pos.copy(); p1[:, a, k] += h
            p2 = pos.copy(); p2[:, a, k] -= h
            fd[:, a, k] = -(O.bias_energy(p1, sys_.quads, models, e0, e1)
                            - O.bias_energy(p2, sys_.quads, models, e0, e1)) / (2 * h)
    scale = np.max(np.abs(F))
    assert np.max(np.abs(fd - F)) <= 1e-6 * scale
    # the frozen-switch force misses the switch's own gradient here
    frozen = O.bias_force(pos, sys_.quads, models, e0, e1)["F"]
    assert np.max(np.abs(frozen - F)) > 1e-3 * scale


@pytest.mark.parametrize("band", ["full", "none"])
def test_conservative_force_equals_frozen_outside_the_band(band):
    sys_, pos, models = _setup(seed=11)
    eps = O.bias_force(pos, sys_.quads, models, 1e9, 2e9)["eps"]
    e0, e1 = (10 * eps.max(), 20 * eps.max()) if band == "full" else (0.1 * eps.min(), 0.2 * eps.min())
    a = O.bias_force_conservative(pos, sys_.quads, models, e0, e1)
    b = O.bias_force(pos, sys_.quads, models, e0, e1)
    assert np.array_equal(a["F"], b["F"])


def test_resnet_conservative_force_is_minus_grad_energy_in_the_band():
    sys_ = ridgen.system_dipeptide()
    pos = ridgen.chain_coords(sys_, 3, seed=12)
    models = [tuple(m[:4]) + (True,) for m in _models(2 * sys_.n_cv, [6, 6, 6], 3, seed=21)]
    eps = O.bias_force(pos, sys_.quads, models, 1e9, 2e9)["eps"]
    e0, e1 = 0.5 * eps.min(), 2.0 * eps.max()
    out = O.bias_force_conservative(pos, sys_.quads, models, e0, e1)
    assert np.all((out["sigma"] > 0) & (out["sigma"] < 1))
    F = out["F"]
    h = 1e-6
    fd = np.zeros_like(F)
    for a in range(sys_.n_atoms):
        for k in range(3):
            p1 = pos.copy(); p1[:, a, k] += h
            p2 = pos.copy(); p2[:, a, k] -= h
            fd[:, a, k] = -(O.bias_energy(p1, sys_.quads, models, e0, e1)
                            - O.bias_energy(p2, sys_.quads, models, e0, e1)) / (2 * h)
    assert np.max(np.abs(fd - F)) <= 1e-6 * np.max(np.abs(F))
