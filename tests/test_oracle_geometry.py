"""Pins of the oracle's torsion CVs and their Cartesian gradient.

Checks against closed-form geometry, an independent construction (NeRF),
rigid-motion invariance and finite differences; none re-types the oracle's
formulas."""
import math

import numpy as np
import pytest

import ridgen
from oracle import rid_oracle as O


def _closed_form_quad(tau):
    # a=(1,0,0), b=0, c=(0,0,1), d=(cos tau, sin tau, 1): torsion is tau.
    return np.array([[1.0, 0, 0], [0, 0, 0], [0, 0, 1.0],
                     [math.cos(tau), math.sin(tau), 1.0]])


@pytest.mark.parametrize("tau", [0.0, 0.5, math.pi / 2, math.pi, -2.0, -math.pi / 3, 3.0])
def test_dihedral_closed_form(tau):
    pos = _closed_form_quad(tau)[None]
    s = O.dihedral(pos, np.array([[0, 1, 2, 3]]))[0, 0]
    d = (s - tau + math.pi) % (2 * math.pi) - math.pi
    assert abs(d) < 1e-15


def test_dihedral_cis_trans():
    # cis (d eclipses a) is 0 and trans is pi: the textbook convention.
    cis = np.array([[1.0, 0, 0], [0, 0, 0], [0, 0, 1], [1.0, 0, 1]])
    trans = np.array([[1.0, 0, 0], [0, 0, 0], [0, 0, 1], [-1.0, 0, 1]])
    q = np.array([[0, 1, 2, 3]])
    assert O.dihedral(cis[None], q)[0, 0] == 0.0
    assert abs(abs(O.dihedral(trans[None], q)[0, 0]) - math.pi) < 1e-15


def test_nerf_round_trip():
    sys_ = ridgen.system_peptide20()
    nb = len(sys_.backbone())
    rng = np.random.default_rng(11)
    tor = rng.uniform(-math.pi, math.pi, size=(5, nb))
    pos = ridgen.chain_coords(sys_, 5, seed=2, torsions=tor)
    s = O.dihedral(pos, sys_.quads)
    # torsion j places backbone atom j; phi_r places C_r (3r+2), psi_r
    # places N_{r+1} (3r+3).  Table order: psi_1, phi_2, psi_2, ..., phi_n.
    expect = []
    for r in range(sys_.n_res):
        if r > 0:
            expect.append(tor[:, 3 * r + 2])
        if r < sys_.n_res - 1:
            expect.append(tor[:, 3 * r + 3])
    expect = np.stack(expect, axis=1)
    d = (s - expect + math.pi) % (2 * math.pi) - math.pi
    assert np.max(np.abs(d)) < 1e-12


def _rot(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_rigid_motion_invariance():
    sys_ = ridgen.system_dipeptide()
    pos = ridgen.chain_coords(sys_, 8, seed=3)
    rng = np.random.default_rng(0)
    R = _rot(rng)
    pos2 = pos @ R.T + rng.normal(size=3)
    assert np.max(np.abs(O.dihedral(pos, sys_.quads) - O.dihedral(pos2, sys_.quads))) < 1e-12


def _wrapped(a):
    return (a + math.pi) % (2 * math.pi) - math.pi


def test_jacobian_finite_differences():
    sys_ = ridgen.system_peptide20()
    pos = ridgen.chain_coords(sys_, 3, seed=4)
    J = O.dihedral_jacobian(pos, sys_.quads)
    h = 1e-6
    worst = 0.0
    for b in range(pos.shape[0]):
        for i in range(0, sys_.n_cv, 5):
            for slot in range(4):
                a = sys_.quads[i, slot]
                for c in range(3):
                    p1 = pos.copy(); p1[b, a, c] += h
                    p2 = pos.copy(); p2[b, a, c] -= h
                    fd = _wrapped(O.dihedral(p1[b:b + 1], sys_.quads[i:i + 1])
                                  - O.dihedral(p2[b:b + 1], sys_.quads[i:i + 1]))[0, 0] / (2 * h)
                    scale = np.max(np.abs(J[b, i]))
                    worst = max(worst, abs(fd - J[b, i, slot, c]) / scale)
    assert worst < 1e-7


def test_jacobian_zero_net_force_and_torque():
    sys_ = ridgen.system_peptide61()
    pos = ridgen.chain_coords(sys_, 4, seed=5)
    J = O.dihedral_jacobian(pos, sys_.quads)            # [B][n][4][3]
    r = pos[:, sys_.quads]                              # [B][n][4][3]
    net = np.sum(J, axis=2)
    torque = np.sum(np.cross(r, J), axis=2)
    scale = np.max(np.abs(J))
    assert np.max(np.abs(net)) < 1e-12 * scale * 10
    assert np.max(np.abs(torque)) < 1e-12 * scale * 10


def test_apply_cv_force_is_gradient_of_linear_cv_function():
    # f = dE/ds for E = sum_i c_i s_i, so F = grad_r E, checked by FD.
    sys_ = ridgen.system_dipeptide()
    pos = ridgen.chain_coords(sys_, 2, seed=6)
    c = np.array([0.7, -1.3])
    F = O.apply_cv_force(pos, sys_.quads, np.broadcast_to(c, (2, 2)))
    h = 1e-6
    for b in range(2):
        for a in range(sys_.n_atoms):
            for k in range(3):
                p1 = pos.copy(); p1[b, a, k] += h
                p2 = pos.copy(); p2[b, a, k] -= h
                ds = _wrapped(O.dihedral(p1[b:b + 1], sys_.quads) - O.dihedral(p2[b:b + 1], sys_.quads))
                fd = float(ds[0] @ c) / (2 * h)
                assert abs(fd - F[b, a, k]) < 1e-6 * max(1.0, np.max(np.abs(F)))


def test_degenerate_dihedral_flagged_and_zeroed():
    pos = np.array([[[0.0, 0, 0], [0.15, 0, 0], [0.30, 0, 0], [0.4, 0.1, 0.05]]])
    q = np.array([[0, 1, 2, 3]])
    assert O.degenerate(pos, q)[0, 0]
    assert np.all(O.dihedral_jacobian(pos, q) == 0.0)
