"""Pins of the oracle's distance CVs and mixed CV tables (angular mask):
closed-form geometry, the pair Jacobian by finite differences, zero net
force and torque, a linear-model closed form of the mixed encoding, and
the whole mixed bias path as -grad E."""
import math

import numpy as np

import ridgen
from oracle import rid_oracle as O


def _models(n_in, widths, K, seed, bias_std=0.1):
    p = ridgen.xavier_ensemble(n_in, widths, K, seed, bias_std)
    return ridgen.unpack_params(p, n_in, widths, K)


def test_distance_closed_form():
    pos = np.zeros((1, 3, 3))
    pos[0, 1] = [3.0, 4.0, 0.0]
    pos[0, 2] = [3.0, 4.0, 12.0]
    s = O.distance_cv(pos, [[0, 1], [0, 2], [2, 1]])
    assert np.allclose(s[0], [5.0, 13.0, 12.0], rtol=0, atol=1e-15)


def test_distance_jacobian_finite_differences():
    rng = np.random.default_rng(1)
    pos = rng.normal(size=(3, 6, 3))
    pairs = np.array([[0, 3], [5, 1], [2, 4]])
    J = O.distance_jacobian(pos, pairs)
    h = 1e-6
    for i, (a, b) in enumerate(pairs):
        for slot, atom in enumerate((a, b)):
            for d in range(3):
                e = np.zeros_like(pos); e[:, atom, d] = h
                fd = (O.distance_cv(pos + e, pairs) - O.distance_cv(pos - e, pairs))[:, i] / (2 * h)
                assert np.max(np.abs(fd - J[:, i, slot, d])) < 1e-8


def test_pair_force_has_zero_net_force_and_torque():
    rng = np.random.default_rng(2)
    sys_ = ridgen.with_distances(ridgen.system_peptide20(), 6)
    pos = ridgen.chain_coords(sys_, 4, seed=3)
    fcv = rng.normal(size=(4, sys_.n_cv))
    F = O.apply_cv_force(pos, sys_.quads, fcv, mask=sys_.mask)
    assert np.max(np.abs(F.sum(axis=1))) < 1e-10
    assert np.max(np.abs(np.cross(pos, F).sum(axis=1))) < 1e-9


def test_mixed_table_values_and_all_ones_mask():
    sys_ = ridgen.with_distances(ridgen.system_peptide20(), 6)
    assert sys_.n_cv == 44 and int(sys_.mask.sum()) == 38
    pos = ridgen.chain_coords(sys_, 3, seed=4)
    s = O.cv_values(pos, sys_.quads, sys_.mask)
    m = sys_.mask.astype(bool)
    assert np.array_equal(s[:, m], O.dihedral(pos, sys_.quads[m]))
    d = np.linalg.norm(pos[:, sys_.quads[~m, 1]] - pos[:, sys_.quads[~m, 0]], axis=-1)
    assert np.allclose(s[:, ~m], d, rtol=0, atol=1e-14)
    # CA_r - CA_{r+3} of a folded-ish chain: a few tenths of a nm
    assert np.all((d > 0.1) & (d < 2.0))
    # an all-ones mask is the torsion path exactly
    base = ridgen.system_peptide20()
    models = _models(2 * base.n_cv, [32, 32], 2, seed=5)
    p0 = ridgen.chain_coords(base, 3, seed=4)
    a = O.bias_force(p0, base.quads, models, 2.0, 3.0)
    b = O.bias_force(p0, base.quads, models, 2.0, 3.0, mask=np.ones(base.n_cv, np.uint8))
    assert np.array_equal(a["F"], b["F"]) and np.array_equal(a["eps"], b["eps"])


def test_mixed_encoding_linear_model_closed_form():
    # no hidden layer: A = wo . x + bo with x = [c | t]; an angular CV has
    # g = -sin s wo[i] + cos s wo[n+i], a raw one g = wo[i] (its second
    # slot holds 0, so wo[n+i] never matters)
    rng = np.random.default_rng(6)
    n = 5
    mask = np.array([1, 0, 1, 0, 0], np.uint8)
    wo = rng.normal(size=2 * n); bo = 0.2
    s = rng.uniform(-2, 2, size=(4, n))
    A, g = O.ensemble_mean_force([([], [], wo, bo)], s, mask)
    m = mask.astype(bool)
    c = np.where(m, np.cos(s), s)
    t = np.where(m, np.sin(s), 0.0)
    assert np.allclose(A[:, 0], c @ wo[:n] + t @ wo[n:] + bo, rtol=0, atol=1e-14)
    expect = np.where(m, -np.sin(s) * wo[:n] + np.cos(s) * wo[n:], wo[:n])
    assert np.allclose(g[:, 0], expect, rtol=0, atol=1e-14)


def test_mixed_mean_force_finite_differences_in_s():
    n = 6
    mask = np.array([0, 1, 1, 0, 1, 0], np.uint8)
    models = _models(2 * n, [16, 16], 2, seed=7)
    s = np.random.default_rng(8).uniform(-2, 2, size=(3, n))
    A, g = O.ensemble_mean_force(models, s, mask)
    h = 1e-6
    for i in range(n):
        e = np.zeros(n); e[i] = h
        fd = (O.ensemble_mean_force(models, s + e, mask)[0]
              - O.ensemble_mean_force(models, s - e, mask)[0]) / (2 * h)
        assert np.max(np.abs(fd - g[:, :, i])) < 1e-8


def test_mixed_bias_force_is_minus_grad_energy():
    sys_ = ridgen.with_distances(ridgen.chain_system(5, 6), 2, stride=2, every=3)
    models = _models(2 * sys_.n_cv, [24, 24], 3, seed=9)
    pos = ridgen.chain_coords(sys_, 2, seed=10)
    out = O.bias_force(pos, sys_.quads, models, 1e9, 2e9, mask=sys_.mask)
    h = 1e-6
    for b in range(2):
        for a in range(sys_.n_atoms):
            for d in range(3):
                e = np.zeros_like(pos); e[b, a, d] = h
                Ep = O.bias_energy_frozen(pos + e, sys_.quads, models, out["sigma"], sys_.mask)[b]
                Em = O.bias_energy_frozen(pos - e, sys_.quads, models, out["sigma"], sys_.mask)[b]
                assert abs(-(Ep - Em) / (2 * h) - out["F"][b, a, d]) < 1e-7


def test_coincident_pair_is_degenerate():
    pos = np.zeros((2, 4, 3))
    pos[0] = [[0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 1]]
    pos[1] = pos[0]
    pos[1, 3] = pos[1, 0]                    # atoms 0 and 3 coincide
    cvs = np.array([[0, 1, 2, 3], [0, 3, -1, -1]])
    mask = np.array([1, 0], np.uint8)
    deg = O.cv_degenerate(pos, cvs, mask)
    assert not deg[0].any() and deg[1, 1]
    J = O.distance_jacobian(pos, cvs[1:, :2])
    assert np.all(J[1] == 0.0)


def test_masked_clustering_does_not_wrap_raw_cvs():
    # 3.0 and -3.1 are 0.18 apart through the periodic wrap, 6.1 apart on the
    # line: at threshold 0.2 they share a cluster only as an angle
    s = np.array([[3.0], [-3.1]], np.float32)
    lab_a, _, n_a = O.leader_cluster(s, 0.2)
    lab_d, _, n_d = O.leader_cluster(s, 0.2, mask=np.array([0], np.uint8))
    assert n_a == 1 and list(lab_a) == [0, 0]
    assert n_d == 2 and list(lab_d) == [0, 1]


def test_masked_distance_against_fp64_and_labels_by_brute_force():
    rng = np.random.default_rng(12)
    n = 7
    mask = np.array([1, 0, 1, 1, 0, 1, 0], np.uint8)
    m = mask.astype(bool)
    s = np.where(m, rng.uniform(-np.pi, np.pi, (300, n)), rng.uniform(0.2, 1.6, (300, n)))
    s = s.astype(np.float32)
    a, b = s[:150].astype(np.float64), s[150:].astype(np.float64)
    d = a - b
    d = np.where(m, (d + np.pi) % (2 * np.pi) - np.pi, d)
    exact = np.sum(d * d, axis=-1)
    got = O.cv_distance_sq_f32(s[:150], s[150:], mask).astype(np.float64)
    assert np.max(np.abs(got - exact) / np.maximum(exact, 1e-6)) < 1e-5
    t = np.float32(1.4)
    labels, leaders, nc = O.leader_cluster(s, t, mask=mask)
    L = s[leaders]
    for f in range(len(s)):
        d2 = O.cv_distance_sq_f32(L, s[f][None, :], mask)
        first = int(np.nonzero(d2 <= t * t)[0][0])
        assert labels[f] == first


def test_masked_training_gradient_finite_differences():
    """Training on a mixed table: raw CVs enter as (s, 0), their mean force
    is dA/dx_i and the label residual reaches the input as (rho_i, 0)."""
    n, widths = 4, [6, 5]
    mask = np.array([1, 0, 1, 0], np.uint8)
    (m,) = _models(2 * n, widths, 1, seed=31, bias_std=0.2)
    rng = np.random.default_rng(32)
    s = np.where(mask.astype(bool), rng.uniform(-3, 3, size=(5, n)), rng.uniform(0.3, 1.5, size=(5, n)))
    F = rng.normal(size=(5, n))
    loss, grads = O.train_loss_grad(m, s, F, mask=mask)
    assert abs(loss - O.train_loss(m, s, F, mask=mask)) < 1e-13
    assert abs(loss - O.train_loss(m, s, F)) > 1e-6          # the mask matters
    g = O.flat_grad(grads)
    theta = O.flat_model(m)
    h = 1e-6
    fd = np.array([(O.train_loss(O.unflat_model(theta + h * e, 2 * n, widths), s, F, mask=mask)
                    - O.train_loss(O.unflat_model(theta - h * e, 2 * n, widths), s, F, mask=mask))
                   / (2 * h) for e in np.eye(theta.size)])
    assert np.max(np.abs(fd - g)) < 1e-6 * np.max(np.abs(g))


def test_masked_deviation_gradient_finite_differences():
    n = 4
    mask = np.array([0, 1, 1, 0], np.uint8)
    models = _models(2 * n, [6, 5], 3, seed=33, bias_std=0.2)
    rng = np.random.default_rng(34)
    s = np.where(mask.astype(bool), rng.uniform(-3, 3, size=(4, n)), rng.uniform(0.3, 1.5, size=(4, n)))
    eps, de = O.deviation_gradient(models, s, mask)
    h = 1e-6
    fd = np.zeros_like(s)
    for i in range(n):
        e = np.zeros(n); e[i] = h
        ep = O.model_deviation(O.ensemble_mean_force(models, s + e, mask)[1])[1]
        em = O.model_deviation(O.ensemble_mean_force(models, s - e, mask)[1])[1]
        fd[:, i] = (ep - em) / (2 * h)
    assert np.max(np.abs(de - fd)) <= 1e-7 * np.max(np.abs(fd))


def test_masked_conservative_force_is_minus_grad_energy_in_the_band():
    sys_ = ridgen.with_distances(ridgen.chain_system(4, 6), 2, stride=2, every=3)
    models = _models(2 * sys_.n_cv, [10, 10], 3, seed=35, bias_std=0.2)
    pos = ridgen.chain_coords(sys_, 2, seed=36)
    eps = O.bias_force(pos, sys_.quads, models, 1e9, 2e9, mask=sys_.mask)["eps"]
    e0, e1 = 0.5 * eps.min(), 2.0 * eps.max()
    out = O.bias_force_conservative(pos, sys_.quads, models, e0, e1, mask=sys_.mask)
    assert np.all((out["sigma"] > 0) & (out["sigma"] < 1))
    F = out["F"]
    h = 1e-6
    fd = np.zeros_like(F)
    for a in range(sys_.n_atoms):
        for k in range(3):
            p1 = pos.copy(); p1[:, a, k] += h
            p2 = pos.copy(); p2[:, a, k] -= h
            fd[:, a, k] = -(O.bias_energy(p1, sys_.quads, models, e0, e1, sys_.mask)
                            - O.bias_energy(p2, sys_.quads, models, e0, e1, sys_.mask)) / (2 * h)
    assert np.max(np.abs(fd - F)) <= 1e-6 * np.max(np.abs(F))
