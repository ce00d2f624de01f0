"""Pins of the oracle's MCMC on the learned free energy: the generator's
published known-answer vectors, the infinite-temperature random walk, and
sampling of exp(-A/kT) for a closed-form one-CV model."""
import math

import numpy as np
import pytest

import ridgen
from oracle import rid_oracle as O

# Philox4x32-10 known-answer vectors (counter, key) -> output, as published
# with the generator's reference implementation.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_philox_known_answers(ctr, key, expect):
    assert tuple(int(x) for x in O.philox4x32(ctr, key)) == expect


def test_uniforms_are_exact_fp32_in_open_interval():
    u = O.mcmc_uniforms(np.arange(64), 5, 39, seed=2024)
    assert u.shape == (64, 39)
    assert np.all((u > 0) & (u < 1))
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    big = O.mcmc_uniforms(np.arange(4000), 1, 40, seed=7)
    assert abs(big.mean() - 0.5) < 0.003 and abs(big.var() - 1 / 12) < 0.002


def _linear_model(a, b, n=1):
    # zero hidden layers: A(s) = wo . [cos s | sin s] = a cos(s - b) for n = 1
    wo = np.array([a * math.cos(b), a * math.sin(b)])
    return ([], [], wo, 0.3)


def test_infinite_temperature_is_the_generator_random_walk():
    rng = np.random.default_rng(3)
    W, n, T, step, seed = 16, 3, 12, 0.4, 99
    models = [([], [], rng.normal(size=2 * n), 0.0)]
    s0 = rng.uniform(-math.pi, math.pi, (W, n))
    out = O.mcmc_run(models, s0, T, 1e300, step, seed, t0=5, proj=(0, 2), nbins=11,
                     keep_path=True)
    s = s0.copy()
    for t in range(5, 5 + T):
        u = O.mcmc_uniforms(np.arange(W), t, n + 1, seed)
        s = s + step * (2 * u[:, :n] - 1)
        s = np.mod(s + math.pi, 2 * math.pi) - math.pi
    assert np.allclose(out["s"], s, atol=1e-12)
    assert out["accepted"] == W * T
    assert out["hist1"].sum() == W * T * n and out["hist2"].sum() == W * T


def test_samples_boltzmann_density_of_a_closed_form_model():
    # A(s) = a cos(s - b) with a = 2 kT: p(s) ~ exp(-(a/kT) cos(s - b)), the
    # density at the minimum of A is e^4 times the density at its maximum
    kT, a, b = 1.0, 2.0, 0.7
    models = [_linear_model(a, b)]
    W, nb = 3000, 24
    s0 = np.random.default_rng(5).uniform(-math.pi, math.pi, (W, 1))
    burn = O.mcmc_run(models, s0, 100, kT, 1.2, seed=11, nbins=nb, proj=(0, 0))
    out = O.mcmc_run(models, burn["s"], 300, kT, 1.2, seed=11, t0=100, nbins=nb, proj=(0, 0))
    h = out["hist1"][0].astype(np.float64)
    p = h / h.sum()
    edges = np.linspace(-math.pi, math.pi, nb + 1)
    fine = np.linspace(-math.pi, math.pi, 200 * nb + 1)
    dens = np.exp(-(a / kT) * np.cos(fine - b))
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(fine))])
    exact = np.diff(np.interp(edges, fine, cdf)) / cdf[-1]
    assert np.max(np.abs(p - exact)) < 0.1 * exact.max()
    # projected PMF recovers A up to a constant where the bins are populated
    f = O.pmf_from_histogram(h, kT)
    centres = 0.5 * (edges[1:] + edges[:-1])
    ref = a * np.cos(centres - b)
    ref -= ref.min()
    assert np.max(np.abs(f - ref)) < 0.3


def test_acceptance_follows_the_metropolis_rule():
    # one step: accepted exactly where u_n < exp(-(A(s') - A(s))/kT)
    kT, step, seed = 0.5, 1.0, 4
    models = [_linear_model(1.5, -0.4)]
    W = 500
    s0 = np.random.default_rng(8).uniform(-math.pi, math.pi, (W, 1))
    out = O.mcmc_run(models, s0, 1, kT, step, seed, t0=7, proj=(0, 0), nbins=5)
    u = O.mcmc_uniforms(np.arange(W), 7, 2, seed)
    sp = np.mod(s0 + step * (2 * u[:, :1] - 1) + math.pi, 2 * math.pi) - math.pi
    A = lambda s: 1.5 * np.cos(s[:, 0] + 0.4) + 0.3
    acc = u[:, 1] < np.exp(-(A(sp) - A(s0)) / kT)
    assert 0.2 < acc.mean() < 0.95
    assert np.allclose(out["s"], np.where(acc[:, None], sp, s0), atol=1e-12)
    assert out["accepted"] == int(acc.sum())


def _lin_raw_model(w):
    # no hidden layer: A = w . x with x = (s, 0) for the raw CV
    return ([], [], np.array([w, 0.0]), 0.0)


def test_all_angular_mask_is_the_torus_chain():
    models = [tuple(m) for m in ridgen.unpack_params(
        ridgen.xavier_ensemble(6, [8], 2, 5, 0.1), 6, [8], 2)]
    s0 = ridgen.torus_samples(16, 3, 3)
    a = O.mcmc_run(models, s0, 12, 0.05, 0.4, 11, proj=(0, 2), nbins=9)
    b = O.mcmc_run(models, s0, 12, 0.05, 0.4, 11, proj=(0, 2), nbins=9,
                   mask=np.ones(3, np.uint8), lower=np.zeros(3), upper=np.ones(3))
    assert np.array_equal(a["s"], b["s"]) and a["accepted"] == b["accepted"]
    assert np.array_equal(a["hist1"], b["hist1"]) and np.array_equal(a["hist2"], b["hist2"])


def test_raw_cv_infinite_temperature_is_uniform_on_its_box():
    # a symmetric proposal with rejection outside the box has the uniform
    # density on the box as its stationary distribution; walkers start inside
    lo, hi, nb = 0.4, 1.6, 6
    W, T = 400, 400
    s0 = np.random.default_rng(1).uniform(lo, hi, (W, 1))
    out = O.mcmc_run([_lin_raw_model(0.0)], s0, T, 1e30, 1.0, 3, proj=(0, 0), nbins=nb,
                     mask=np.array([0], np.uint8), lower=[lo], upper=[hi])
    assert np.all((out["s"] >= lo) & (out["s"] <= hi))
    h = out["hist1"][0]
    assert h.sum() == W * T
    # every state stays in the box; counts per bin within 5 % of flat
    # (W T / nb = 26 667 per bin; the chains are correlated over ~10 steps)
    assert np.max(np.abs(h / (W * T / nb) - 1.0)) < 0.05
    assert out["accepted"] < W * T                    # the walls reject


def test_raw_cv_samples_the_boltzmann_density_of_a_linear_free_energy():
    # A(s) = a s on [lo, hi]: density proportional to exp(-a s / kT)
    lo, hi, a, kT, nb = 0.5, 2.5, 3.0, 1.0, 8
    W, T = 500, 500
    s0 = np.random.default_rng(2).uniform(lo, hi, (W, 1))
    out = O.mcmc_run([_lin_raw_model(a)], s0, T, kT, 1.5, 5, t0=0, proj=(0, 0), nbins=nb,
                     mask=np.array([0], np.uint8), lower=[lo], upper=[hi])
    edges = np.linspace(lo, hi, nb + 1)
    mass = np.exp(-a * edges[:-1] / kT) - np.exp(-a * edges[1:] / kT)
    mass /= mass.sum()
    h = out["hist1"][0] / (W * T)
    # the first half of the bins (95 % of the mass) within 10 %
    assert np.max(np.abs(h[:4] / mass[:4] - 1.0)) < 0.1
    pmf = O.pmf_from_histogram(out["hist1"][0], kT)
    centres = 0.5 * (edges[:-1] + edges[1:])
    assert np.max(np.abs(pmf[:4] - a * (centres[:4] - centres[0]))) < 0.25
