"""Pins of the oracle's residual MLP (the `resnet` training setting): the
small-weight linear limit, reduction to one layer, a unit-by-unit scalar
evaluation, finite differences, and what stays plain."""
import math

import numpy as np
import pytest

import ridgen
from oracle import rid_oracle as O


def _res(model):
    return tuple(model[:4]) + (True,)


def _models(n_in, widths, K, seed, bias_std=0.1):
    p = ridgen.xavier_ensemble(n_in, widths, K, seed, bias_std)
    return ridgen.unpack_params(p, n_in, widths, K)


def test_resnet_linear_limit():
    # weights and biases of size a: tanh(z) = z + O(a^3), so the network is
    # the affine map h_1 = W_1 x + b_1, h_l = (I + W_l) h_{l-1} + b_l, and
    # dA/dx = W_1^T (I + W_2)^T ... (I + W_L)^T wo.  A dropped skip (W_l in
    # place of I + W_l), forward or reverse, changes A or dA/dx at first
    # order in a, far above the O(a^3) remainder.
    rng = np.random.default_rng(3)
    a = 1e-4
    n_in, w, L = 6, 5, 4
    Ws = [a * rng.normal(size=(w, n_in))] + [a * rng.normal(size=(w, w)) for _ in range(L - 1)]
    bs = [a * rng.normal(size=w) for _ in range(L)]
    wo = rng.normal(size=w); bo = 0.3
    x = rng.normal(size=(7, n_in))
    A, u0 = O.mlp_value_and_grad((Ws, bs, wo, bo, True), x)
    h = x @ Ws[0].T + bs[0]
    M = Ws[0]
    for W, b in zip(Ws[1:], bs[1:]):
        h = h @ (np.eye(w) + W).T + b
        M = (np.eye(w) + W) @ M
    A_lin = h @ wo + bo
    g_lin = wo @ M
    # the cubic remainder is ~ (a |x| sqrt(n_in))^3 / 3, below 1e-10 here
    assert np.max(np.abs(A - A_lin)) < 1e-9
    assert np.max(np.abs(u0 - g_lin[None, :])) < 1e-9
    # and the plain network is far from it (the skip matters at this size)
    A_plain, _ = O.mlp_value_and_grad((Ws, bs, wo, bo), x)
    assert np.max(np.abs(A_plain - A_lin)) > 1e-5


def test_resnet_zero_later_layers_reduce_to_one_layer():
    # W_l = 0, b_l = 0 for l >= 2: tanh(0) = 0, so every later layer passes
    # h_1 through and A = wo . tanh(W_1 x + b_1) + bo (the plain network
    # would give A = bo).
    rng = np.random.default_rng(4)
    n_in, w = 4, 3
    W1 = rng.normal(size=(w, n_in)); b1 = rng.normal(size=w)
    Ws = [W1, np.zeros((w, w)), np.zeros((w, w))]
    bs = [b1, np.zeros(w), np.zeros(w)]
    wo = rng.normal(size=w); bo = -0.7
    x = rng.normal(size=(5, n_in))
    A, u0 = O.mlp_value_and_grad((Ws, bs, wo, bo, True), x)
    t = np.tanh(x @ W1.T + b1)
    assert np.allclose(A, t @ wo + bo, rtol=0, atol=1e-14)
    assert np.allclose(u0, ((1 - t * t) * wo) @ W1, rtol=0, atol=1e-14)
    A_plain, _ = O.mlp_value_and_grad((Ws, bs, wo, bo), x)
    assert np.allclose(A_plain, bo, rtol=0, atol=1e-15)


def test_resnet_two_layers_written_out_by_hand():
    # width-2 layers, every unit a scalar expression; the second layer adds
    # its input (p, q) to its tanh outputs.
    W1 = np.array([[0.3, -1.1, 0.5], [0.9, 0.2, -0.4]]); b1 = np.array([0.1, -0.2])
    W2 = np.array([[1.3, -0.7], [0.25, 0.8]]); b2 = np.array([0.05, 0.3])
    wo = np.array([0.6, -1.4]); bo = 0.25
    x = np.array([[0.2, -0.5, 0.9]])
    p = math.tanh(0.3 * 0.2 - 1.1 * -0.5 + 0.5 * 0.9 + 0.1)
    q = math.tanh(0.9 * 0.2 + 0.2 * -0.5 - 0.4 * 0.9 - 0.2)
    r = math.tanh(1.3 * p - 0.7 * q + 0.05) + p
    t = math.tanh(0.25 * p + 0.8 * q + 0.3) + q
    A, _ = O.mlp_value_and_grad(([W1, W2], [b1, b2], wo, bo, True), x)
    assert abs(A[0] - (0.6 * r - 1.4 * t + 0.25)) < 1e-15


@pytest.mark.parametrize("widths", [[8, 8, 8], [5, 5, 5, 5, 5]])
def test_resnet_gradient_finite_differences(widths):
    n = 3
    m = _res(_models(2 * n, widths, 1, seed=11)[0])
    rng = np.random.default_rng(12)
    x = rng.normal(size=(4, 2 * n))
    _, u0 = O.mlp_value_and_grad(m, x)
    h = 1e-6
    fd = np.zeros_like(x)
    for j in range(2 * n):
        e = np.zeros(2 * n); e[j] = h
        fd[:, j] = (O.mlp_value_and_grad(m, x + e)[0] - O.mlp_value_and_grad(m, x - e)[0]) / (2 * h)
    assert np.max(np.abs(fd - u0)) < 1e-8


def test_resnet_mean_force_finite_differences_in_s():
    n = 4
    models = [_res(m) for m in _models(2 * n, [16, 16, 16], 2, seed=13)]
    rng = np.random.default_rng(14)
    s = rng.uniform(-math.pi, math.pi, size=(3, n))
    A, g = O.ensemble_mean_force(models, s)
    h = 1e-6
    for i in range(n):
        e = np.zeros(n); e[i] = h
        fd = (O.ensemble_mean_force(models, s + e)[0] - O.ensemble_mean_force(models, s - e)[0]) / (2 * h)
        assert np.max(np.abs(fd - g[:, :, i])) < 1e-8


def test_resnet_one_layer_is_plain():
    # no skip on the first layer: with one hidden layer both forms agree
    m = _models(6, [7], 1, seed=15)[0]
    x = np.random.default_rng(16).normal(size=(5, 6))
    A0, u0 = O.mlp_value_and_grad(m, x)
    A1, u1 = O.mlp_value_and_grad(_res(m), x)
    assert np.array_equal(A0, A1) and np.array_equal(u0, u1)


def test_resnet_refuses_unequal_widths():
    s = np.zeros((2, 3))
    with pytest.raises(ValueError):
        O.mlp_value_and_grad(_res(_models(6, [7, 5], 1, seed=18)[0]), O.embed(s))


def _flat_fd(loss_of, theta, h=1e-6):
    fd = np.zeros_like(theta)
    for j in range(theta.size):
        t1 = theta.copy(); t1[j] += h
        t2 = theta.copy(); t2[j] -= h
        fd[j] = (loss_of(t1) - loss_of(t2)) / (2 * h)
    return fd


@pytest.mark.parametrize("dropout", [False, True])
def test_resnet_training_gradient_finite_differences(dropout):
    """Loss gradient of a residual network on every parameter (three hidden
    layers: two skips), with the dropout masks held fixed when on."""
    n, widths = 3, [5, 5, 5]
    m = _res(_models(2 * n, widths, 1, seed=21, bias_std=0.2)[0])
    rng = np.random.default_rng(22)
    s = rng.uniform(-3, 3, size=(4, n))
    F = rng.normal(size=(4, n))
    sc = O.dropout_scales(4, widths, 0.3, seed=9, step=1, member=0) if dropout else None
    if dropout:
        assert any(np.any(x == 0.0) for x in sc)
    loss, grads = O.train_loss_grad(m, s, F, sc)
    assert abs(loss - O.train_loss(m, s, F, sc)) < 1e-13
    g = O.flat_grad(grads)
    fd = _flat_fd(lambda th: O.train_loss(O.unflat_model(th, 2 * n, widths, True), s, F, sc),
                  O.flat_model(m))
    assert np.max(np.abs(fd - g)) < 1e-6 * np.max(np.abs(g))
    # the skips matter: the plain network's gradient differs
    _, gp = O.train_loss_grad(tuple(m[:4]), s, F, sc)
    assert np.max(np.abs(O.flat_grad(gp) - g)) > 1e-3 * np.max(np.abs(g))


def test_resnet_vjp_finite_differences():
    n, widths = 4, [6, 6]
    m = _res(_models(2 * n, widths, 1, seed=23, bias_std=0.2)[0])
    rng = np.random.default_rng(24)
    s = rng.uniform(-3, 3, size=(5, n))
    rho = rng.normal(size=(5, n))
    g = O.flat_grad(O.mean_force_vjp(m, s, rho))

    def J(th):
        _, gg = O.ensemble_mean_force([O.unflat_model(th, 2 * n, widths, True)], s)
        return float(np.sum(rho * gg[:, 0, :]))

    fd = _flat_fd(J, O.flat_model(m))
    assert np.max(np.abs(fd - g)) < 1e-6 * np.max(np.abs(g))


def test_resnet_training_reduces_to_one_layer():
    """Later layers with zero weights and biases pass h_1 through unchanged
    (tanh(0) = 0): the residual network is the one-layer network, and so is
    the gradient of its first layer and output weights."""
    n, w = 3, 6
    (m1,) = _models(2 * n, [w], 1, seed=25, bias_std=0.2)
    Ws, bs, wo, bo = m1
    z = np.zeros((w, w))
    mres = ([Ws[0], z, z], [bs[0], np.zeros(w), np.zeros(w)], wo, bo, True)
    rng = np.random.default_rng(26)
    s = rng.uniform(-3, 3, size=(6, n))
    F = rng.normal(size=(6, n))
    l1, g1 = O.train_loss_grad(m1, s, F)
    lr, gr = O.train_loss_grad(mres, s, F)
    assert abs(l1 - lr) < 1e-13
    assert np.allclose(gr[0][0], g1[0][0], rtol=0, atol=1e-13)
    assert np.allclose(gr[1][0], g1[1][0], rtol=0, atol=1e-13)
    assert np.allclose(gr[2], g1[2], rtol=0, atol=1e-13)


def test_resnet_input_hvp_finite_differences():
    rng = np.random.default_rng(27)
    m = _res(_models(6, [7, 7, 7], 1, seed=28, bias_std=0.2)[0])
    x = rng.normal(size=(4, 6))
    rho = rng.normal(size=(4, 6))
    hv = O.mlp_input_hvp(m, x, rho)
    h = 1e-5
    fd = (O.mlp_value_and_grad(m, x + h * rho)[1] - O.mlp_value_and_grad(m, x - h * rho)[1]) / (2 * h)
    assert np.max(np.abs(hv - fd)) <= 1e-8 * np.max(np.abs(fd))


def test_resnet_dropout_value_and_grad_finite_differences():
    rng = np.random.default_rng(29)
    widths = [6, 6, 6]
    m = _res(_models(5, widths, 1, seed=30, bias_std=0.2)[0])
    x = rng.normal(size=(3, 5))
    sc = O.dropout_scales(3, widths, 0.4, seed=3, step=0, member=0)
    A, u0 = O.mlp_value_and_grad(m, x, sc)
    h = 1e-6
    for j in range(5):
        e = np.zeros(5); e[j] = h
        fd = (O.mlp_value_and_grad(m, x + e, sc)[0] - O.mlp_value_and_grad(m, x - e, sc)[0]) / (2 * h)
        assert np.max(np.abs(fd - u0[:, j])) < 1e-8
