"""The seeded inputs: reproducible, shaped like the paper's systems."""
import json
import os

import numpy as np

import ridgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_config.json")


def test_torsion_count_follows_paper_rule():
    cfg = json.load(open(GOLDEN))
    n_res = len(cfg["chignolin_selected_resid"]["value"])
    sys_ = ridgen.chain_system(n_res, 10)
    assert sys_.n_cv == cfg["chignolin_angular_mask_len"]["value"] == 2 * n_res - 2


def test_workload_shapes():
    assert (ridgen.system_dipeptide().n_atoms, ridgen.system_dipeptide().n_cv) == (22, 2)
    assert (ridgen.system_peptide20().n_atoms, ridgen.system_peptide20().n_cv) == (200, 38)
    assert (ridgen.system_peptide61().n_atoms, ridgen.system_peptide61().n_cv) == (1000, 120)


def test_chain_geometry():
    sys_ = ridgen.system_peptide20()
    pos = ridgen.chain_coords(sys_, 6, seed=1)
    bb = sys_.backbone()
    P = pos[:, bb]
    bonds = np.linalg.norm(np.diff(P, axis=1), axis=-1)
    assert np.allclose(bonds, ridgen.BOND_NM, atol=1e-12)
    u = P[:, :-2] - P[:, 1:-1]
    v = P[:, 2:] - P[:, 1:-1]
    ang = np.arccos(np.sum(u * v, -1) / np.linalg.norm(u, axis=-1) / np.linalg.norm(v, axis=-1))
    assert ang.min() >= ridgen.ANGLE_CLIP[0] - 1e-9 and ang.max() <= ridgen.ANGLE_CLIP[1] + 1e-9
    assert np.array_equal(pos, ridgen.chain_coords(sys_, 6, seed=1))


def test_analytic_pmf_gradient_finite_differences():
    pmf = ridgen.analytic_pmf(12, seed=3, density=0.3)
    s = ridgen.torus_samples(5, 12, seed=1)
    g = pmf.grad(s)
    h = 1e-6
    for i in range(12):
        e = np.zeros(12); e[i] = h
        fd = (pmf.value(s + e) - pmf.value(s - e)) / (2 * h)
        assert np.max(np.abs(fd - g[:, i])) < 1e-8


def test_packed_params_round_trip():
    p = ridgen.xavier_ensemble(76, [256] * 4, 4, seed=1000)
    assert p.dtype == np.float32 and p.size == ridgen.packed_size(76, [256] * 4, 4) == 4 * 217345
    models = ridgen.unpack_params(p, 76, [256] * 4, 4)
    assert np.array_equal(ridgen.pack_params(models).astype(np.float32), p)
