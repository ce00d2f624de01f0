"""Pins of the oracle's mean-force fitting: finite differences of the loss in
every parameter, the exact optimum of the linear model, Adam's first step and
the paper's learning-rate schedule."""
import json
import math
import os

import numpy as np

import ridgen
from oracle import rid_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_config.json")


def _model(n_in, widths, seed):
    p = ridgen.xavier_ensemble(n_in, widths, 1, seed, bias_std=0.2)
    return ridgen.unpack_params(p, n_in, widths, 1)[0]


def test_training_gradient_finite_differences():
    n, widths = 3, [5, 4]
    model = _model(2 * n, widths, 7)
    rng = np.random.default_rng(8)
    s = rng.uniform(-3, 3, size=(4, n))
    F = rng.normal(size=(4, n))
    loss, grads = O.train_loss_grad(model, s, F)
    assert abs(loss - O.train_loss(model, s, F)) < 1e-13
    theta = O.flat_model(model)
    g = O.flat_grad(grads)
    h = 1e-6
    fd = np.zeros_like(theta)
    for j in range(theta.size):
        t1 = theta.copy(); t1[j] += h
        t2 = theta.copy(); t2[j] -= h
        fd[j] = (O.train_loss(O.unflat_model(t1, 2 * n, widths), s, F)
                 - O.train_loss(O.unflat_model(t2, 2 * n, widths), s, F)) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-6 * np.max(np.abs(g))
    assert g[-1] == 0.0  # output bias never reaches grad_s A


def test_mean_force_vjp_finite_differences():
    n, widths = 4, [6, 5, 3]
    model = _model(2 * n, widths, 9)
    rng = np.random.default_rng(10)
    s = rng.uniform(-3, 3, size=(5, n))
    rho = rng.normal(size=(5, n))
    g = O.flat_grad(O.mean_force_vjp(model, s, rho))
    theta = O.flat_model(model)

    def J(th):
        _, gg = O.ensemble_mean_force([O.unflat_model(th, 2 * n, widths)], s)
        return float(np.sum(rho * gg[:, 0, :]))

    h = 1e-6
    fd = np.array([(J(theta + h * e) - J(theta - h * e)) / (2 * h)
                   for e in np.eye(theta.size)])
    assert np.max(np.abs(fd - g)) < 1e-6 * np.max(np.abs(g))


def _linear_problem(n=4, m=64):
    rng = np.random.default_rng(3)
    a = rng.uniform(0.5, 5.0, size=n)
    b = rng.uniform(-math.pi, math.pi, size=n)
    s = rng.uniform(-math.pi, math.pi, size=(m, n))
    F = a * np.sin(s - b)        # minus the gradient of sum a cos(s - b)
    return a, b, s, F


def test_linear_model_optimum_has_zero_gradient():
    a, b, s, F = _linear_problem()
    n = a.size
    wo = np.concatenate([-a * np.cos(b), -a * np.sin(b)])
    loss, grads = O.train_loss_grad(([], [], wo, 0.0), s, F)
    assert loss < 1e-28
    assert np.max(np.abs(grads[2])) < 1e-14


def test_adam_converges_to_linear_optimum():
    a, b, s, F = _linear_problem()
    n = a.size
    model = ([], [], np.zeros(2 * n), 0.0)
    state = [(np.zeros(2 * n + 1), np.zeros(2 * n + 1), 0)]
    for step in range(3000):
        [model], state, _ = O.train_step([model], s, F, state, lr=0.05 * 0.999 ** step)
    wo = model[2]
    assert np.allclose(wo[:n], -a * np.cos(b), atol=1e-3)
    assert np.allclose(wo[n:], -a * np.sin(b), atol=1e-3)


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = O.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)


def test_learning_rate_schedule_from_paper():
    cfg = json.load(open(GOLDEN))
    lr0, T, gam = cfg["init_lr"]["value"], cfg["decay_steps"]["value"], cfg["decay_rate"]["value"]
    assert (O.INIT_LR, O.DECAY_STEPS, O.DECAY_RATE) == (lr0, T, gam)
    assert O.lr_at(0) == lr0
    assert abs(O.lr_at(T) - lr0 * gam) < 1e-18
    assert abs(O.lr_at(10 * T) - lr0 * gam ** 10) < 1e-18
    assert abs(O.lr_at(T // 2) - lr0 * math.sqrt(gam)) < 1e-18


def test_dropout_gradient_finite_differences():
    n, widths = 3, [6, 5]
    model = _model(2 * n, widths, 17)
    rng = np.random.default_rng(18)
    s = rng.uniform(-3, 3, size=(5, n))
    F = rng.normal(size=(5, n))
    sc = O.dropout_scales(5, widths, 0.3, seed=123, step=2, member=1)
    assert any(np.any(x == 0.0) for x in sc) and any(np.any(x > 1.0) for x in sc)
    loss, grads = O.train_loss_grad(model, s, F, sc)
    assert abs(loss - O.train_loss(model, s, F, sc)) < 1e-13
    assert abs(loss - O.train_loss(model, s, F)) > 1e-6      # the masks matter
    theta = O.flat_model(model)
    g = O.flat_grad(grads)
    h = 1e-6
    fd = np.zeros_like(theta)
    for j in range(theta.size):
        t1 = theta.copy(); t1[j] += h
        t2 = theta.copy(); t2[j] -= h
        fd[j] = (O.train_loss(O.unflat_model(t1, 2 * n, widths), s, F, sc)
                 - O.train_loss(O.unflat_model(t2, 2 * n, widths), s, F, sc)) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-6 * np.max(np.abs(g))


def test_dropout_rate_zero_is_the_plain_gradient():
    n, widths = 4, [8, 8]
    model = _model(2 * n, widths, 19)
    rng = np.random.default_rng(20)
    s = rng.uniform(-3, 3, size=(6, n))
    F = rng.normal(size=(6, n))
    sc = O.dropout_scales(6, widths, 0.0, seed=5, step=0, member=0)
    assert all(np.all(x == 1.0) for x in sc)
    l0, g0 = O.train_loss_grad(model, s, F)
    l1, g1 = O.train_loss_grad(model, s, F, sc)
    assert l0 == l1 and np.array_equal(O.flat_grad(g0), O.flat_grad(g1))


def test_dropout_masks_statistics():
    B, widths, p = 2000, [64, 64], 0.3
    sc = O.dropout_scales(B, widths, p, seed=77, step=4, member=2)
    keep = np.concatenate([(x > 0).ravel() for x in sc])
    N = keep.size
    assert abs(keep.mean() - (1 - p)) < 4 * math.sqrt(p * (1 - p) / N)
    assert set(np.unique(np.concatenate([x.ravel() for x in sc]))) == {0.0, float(np.float32(1) / np.float32(0.7))}
    other = O.dropout_scales(B, widths, p, seed=77, step=5, member=2)
    member = O.dropout_scales(B, widths, p, seed=77, step=4, member=3)
    assert not np.array_equal(sc[0], other[0]) and not np.array_equal(sc[0], member[0])
    assert not np.array_equal(sc[0], sc[1][:, :64])
