"""Seeded synthetic inputs shared by the oracle's tests, the GPU parity tests
and the benchmark.

This module produces *inputs only*: atom coordinates of peptide-shaped
chains, dihedral (phi/psi) tables, ensemble weights, labelled mean-force
training sets, synthetic restrained-MD trajectories and serving traces.  It
holds none of the method's arithmetic (no dihedral evaluation, no network,
no model deviation, no switching, no force), so either side of a parity
comparison can consume it without sharing computation with the other.

Recipes (all FP64, then rounded to FP32 where the GPU consumes the value, so
both sides evaluate at the same point):

* Chain: backbone N, CA, C per residue placed by the natural-extension
  reference-frame construction (NeRF) with bond length 0.15 nm, bond angle
  1.911 rad + N(0, 0.3^2) clipped to [1.2, 2.6] rad and torsions uniform on
  [-pi, pi).  Residue-blocked atom numbering (N at offset 0, CA at 2, C at
  apr-2 for apr atoms per residue); the remaining atoms of a residue sit at
  0.1 nm from a backbone atom of that residue in a random direction; extra
  terminal atoms are appended the same way.  The torsion CVs follow the
  paper's "CV selection" paragraph: psi of the first residue, phi and psi of
  the middle ones, phi of the last (2n-2 torsions for n residues).
* Weights: Xavier-normal N(0, 2/(fan_in+fan_out)), untruncated, model k from
  seed+k; biases zero (benchmarks) or N(0, bias_std^2) (tests).
* Training labels (mean-force fitting): s uniform on the torus; labels are
  minus the gradient of the analytic PMF
  A(s) = sum_i a_i cos(s_i-b_i) + sum_{i<j} c_ij cos s_i cos s_j
  with a_i ~ U(0.5, 5), b_i ~ U[-pi, pi), each pair present with probability
  0.05 and c_ij ~ N(0, 1), plus iid N(0, noise^2) per component.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BOND_NM = 0.15
SIDE_NM = 0.10
ANGLE_MEAN = 1.911
ANGLE_STD = 0.3
ANGLE_CLIP = (1.2, 2.6)


# --------------------------------------------------------------------------
# peptide-shaped chains
# --------------------------------------------------------------------------
@dataclasses.dataclass
class ChainSystem:
    """Topology of a synthetic peptide-like chain."""

    n_res: int
    apr: int            # atoms per residue
    n_extra: int        # terminal atoms appended after the residues
    quads: np.ndarray   # int32 [n_cv][4], 0-based atom indices
    mask: np.ndarray    # uint8 [n_cv], 1 = periodic angle

    @property
    def n_atoms(self) -> int:
        return self.n_res * self.apr + self.n_extra

    @property
    def n_cv(self) -> int:
        return int(self.quads.shape[0])

    def backbone(self) -> np.ndarray:
        """Atom indices of N, CA, C in chain order."""
        idx = []
        for r in range(self.n_res):
            base = r * self.apr
            idx += [base, base + 2, base + self.apr - 2]
        return np.asarray(idx, dtype=np.int64)


def chain_system(n_res: int, apr: int, n_extra: int = 0) -> ChainSystem:
    """Torsion table psi_1, (phi_2, psi_2), ..., phi_n for an n_res chain."""
    if n_res < 2 or apr < 5:   # N, CA = N + 2, C = N + apr - 2 must be distinct
        raise ValueError("need n_res >= 2 and apr >= 5")
    N = lambda r: r * apr
    CA = lambda r: r * apr + 2
    C = lambda r: r * apr + apr - 2
    quads = []
    for r in range(n_res):
        if r > 0:  # phi_r = (C_{r-1}, N_r, CA_r, C_r)
            quads.append((C(r - 1), N(r), CA(r), C(r)))
        if r < n_res - 1:  # psi_r = (N_r, CA_r, C_r, N_{r+1})
            quads.append((N(r), CA(r), C(r), N(r + 1)))
    q = np.asarray(quads, dtype=np.int32)
    return ChainSystem(n_res, apr, n_extra, q, np.ones(len(q), np.uint8))


def with_distances(sys_: ChainSystem, n_dist: int, stride: int = 3,
                   every: int = 4) -> ChainSystem:
    """The chain's torsion table with n_dist distance CVs CA_r - CA_{r+stride}
    (r = 0, 1, ...) interleaved: one distance row after every ``every``
    torsion rows, the rest at the end.  Distance rows are (a, b, -1, -1)
    with angular mask 0."""
    ca = [r * sys_.apr + 2 for r in range(sys_.n_res)]
    pairs = [(ca[r], ca[r + stride]) for r in range(sys_.n_res - stride)][:n_dist]
    if len(pairs) < n_dist:
        raise ValueError("chain too short for that many distances")
    rows, mask, d = [], [], 0
    for i, q in enumerate(sys_.quads):
        rows.append(tuple(int(v) for v in q)); mask.append(1)
        if (i + 1) % every == 0 and d < n_dist:
            rows.append((pairs[d][0], pairs[d][1], -1, -1)); mask.append(0); d += 1
    for a, b in pairs[d:]:
        rows.append((a, b, -1, -1)); mask.append(0)
    return ChainSystem(sys_.n_res, sys_.apr, sys_.n_extra, np.asarray(rows, np.int32),
                       np.asarray(mask, np.uint8))


# Shapes of the workloads (atoms per residue chosen so the totals match).
def system_dipeptide() -> ChainSystem:      # 2 torsions, 22 atoms
    return chain_system(2, 11)


def system_peptide20() -> ChainSystem:      # 38 torsions, 200 atoms
    return chain_system(20, 10)


def system_peptide61() -> ChainSystem:      # 120 torsions, 1000 atoms
    return chain_system(61, 16, 24)


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def nerf_place(a, b, c, bond, angle, torsion):
    """Place d so that |cd| = bond, angle(b, c, d) = angle and the dihedral
    (a, b, c, d) = torsion (vectorised over leading axes)."""
    bc = _unit(c - b)
    nrm = _unit(np.cross(b - a, bc))
    m = np.stack([bc, np.cross(nrm, bc), nrm], axis=-1)  # columns
    d2 = np.stack([
        -bond * np.cos(angle),
        bond * np.sin(angle) * np.cos(torsion),
        bond * np.sin(angle) * np.sin(torsion),
    ], axis=-1)
    return c + np.einsum("...ij,...j->...i", m, d2)


def chain_coords(sys_: ChainSystem, n_walkers: int, seed: int,
                 torsions: np.ndarray | None = None,
                 angles: np.ndarray | None = None) -> np.ndarray:
    """FP64 coordinates [n_walkers][n_atoms][3] (nm).

    ``torsions``/``angles`` (shape [n_walkers][n_backbone]) override the
    random draws; entry j is the torsion/angle that places backbone atom j
    (entries 0..2 / 0..1 are unused)."""
    rng = np.random.default_rng(seed)
    bb = sys_.backbone()
    nb = len(bb)
    W = n_walkers
    ang = rng.normal(ANGLE_MEAN, ANGLE_STD, size=(W, nb))
    ang = np.clip(ang, *ANGLE_CLIP)
    tor = rng.uniform(-math.pi, math.pi, size=(W, nb))
    if angles is not None:
        ang = np.asarray(angles, dtype=np.float64)
    if torsions is not None:
        tor = np.asarray(torsions, dtype=np.float64)
    P = np.zeros((W, nb, 3))
    P[:, 1] = [BOND_NM, 0.0, 0.0]
    a1 = ang[:, 2]
    P[:, 2, 0] = BOND_NM - BOND_NM * np.cos(a1)
    P[:, 2, 1] = BOND_NM * np.sin(a1)
    for j in range(3, nb):
        P[:, j] = nerf_place(P[:, j - 3], P[:, j - 2], P[:, j - 1],
                             BOND_NM, ang[:, j], tor[:, j])
    pos = np.zeros((W, sys_.n_atoms, 3))
    pos[:, bb] = P
    is_bb = np.zeros(sys_.n_atoms, bool)
    is_bb[bb] = True
    side = np.nonzero(~is_bb)[0]
    # parent: a backbone atom of the same residue (terminal extras: last C)
    parents = []
    for a in side:
        r = a // sys_.apr
        if r >= sys_.n_res:
            parents.append(bb[-1])
        else:
            parents.append(bb[3 * r + (a % 3)])
    dirs = _unit(rng.normal(size=(W, len(side), 3)))
    pos[:, side] = pos[:, np.asarray(parents)] + SIDE_NM * dirs
    # rigid random placement so coordinates are not axis-aligned
    off = rng.uniform(0.5, 3.0, size=(W, 1, 3))
    return pos + off


def f32(a: np.ndarray) -> np.ndarray:
    """Round to FP32 (the values both sides consume)."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


# --------------------------------------------------------------------------
# ensemble weights, packed layout
# --------------------------------------------------------------------------
def packed_size(n_in: int, widths, n_models: int) -> int:
    per = 0
    prev = n_in
    for w in widths:
        per += w * prev + w
        prev = w
    per += prev + 1
    return per * n_models


def xavier_ensemble(n_in: int, widths, n_models: int, seed: int,
                    bias_std: float = 0.0) -> np.ndarray:
    """Packed FP32 parameters: for each model k, for each hidden layer l,
    W_l row-major [out][in] then b_l [out]; then w_o [last] and b_o."""
    out = []
    for k in range(n_models):
        rng = np.random.default_rng(seed + k)
        prev = n_in
        for w in widths:
            W = rng.normal(0.0, math.sqrt(2.0 / (prev + w)), size=(w, prev))
            b = rng.normal(0.0, bias_std, size=w) if bias_std > 0 else np.zeros(w)
            out += [W.ravel(), b]
            prev = w
        wo = rng.normal(0.0, math.sqrt(2.0 / (prev + 1)), size=prev)
        bo = rng.normal(0.0, bias_std, size=1) if bias_std > 0 else np.zeros(1)
        out += [wo, bo]
    return f32(np.concatenate(out))


def unpack_params(params: np.ndarray, n_in: int, widths, n_models: int):
    """Inverse of the packed layout: list over models of (Ws, bs, wo, bo)
    as FP64 arrays (pure slicing, no arithmetic)."""
    p = np.asarray(params, dtype=np.float64)
    models = []
    off = 0
    for _ in range(n_models):
        Ws, bs = [], []
        prev = n_in
        for w in widths:
            Ws.append(p[off:off + w * prev].reshape(w, prev)); off += w * prev
            bs.append(p[off:off + w]); off += w
            prev = w
        wo = p[off:off + prev]; off += prev
        bo = float(p[off]); off += 1
        models.append((Ws, bs, wo, bo))
    if off != p.size:
        raise ValueError("packed parameter size mismatch")
    return models


def pack_params(models) -> np.ndarray:
    out = []
    for Ws, bs, wo, bo in models:
        for W, b in zip(Ws, bs):
            out += [np.ravel(W), np.ravel(b)]
        out += [np.ravel(wo), np.atleast_1d(bo)]
    return np.concatenate(out)


# --------------------------------------------------------------------------
# analytic PMF and mean-force training data
# --------------------------------------------------------------------------
@dataclasses.dataclass
class AnalyticPMF:
    a: np.ndarray   # [n]
    b: np.ndarray   # [n]
    c: np.ndarray   # [n][n] symmetric, zero diagonal

    def value(self, s):
        s = np.asarray(s, np.float64)
        cs = np.cos(s)
        pair = 0.5 * np.einsum("...i,ij,...j->...", cs, self.c, cs)
        return np.sum(self.a * np.cos(s - self.b), axis=-1) + pair

    def grad(self, s):
        s = np.asarray(s, np.float64)
        return -self.a * np.sin(s - self.b) - np.sin(s) * (np.cos(s) @ self.c)


def analytic_pmf(n: int, seed: int = 3, density: float = 0.05) -> AnalyticPMF:
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 5.0, size=n)
    b = rng.uniform(-math.pi, math.pi, size=n)
    c = np.zeros((n, n))
    iu = np.triu_indices(n, 1)
    keep = rng.uniform(size=len(iu[0])) < density
    vals = rng.normal(0.0, 1.0, size=len(iu[0])) * keep
    c[iu] = vals
    c = c + c.T
    return AnalyticPMF(a, b, c)


def torus_samples(m: int, n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-math.pi, math.pi, size=(m, n))


def mf_training_set(m: int, n: int, pmf_seed: int = 3, sample_seed: int = 6,
                    noise_seed: int = 4, noise: float = 0.5):
    """(s [m][n] f32, F [m][n] f32, pmf): labels are minus the analytic
    PMF gradient plus Gaussian noise."""
    pmf = analytic_pmf(n, pmf_seed)
    s = torus_samples(m, n, sample_seed)
    F = -pmf.grad(s)
    if noise > 0:
        F = F + np.random.default_rng(noise_seed).normal(0.0, noise, size=F.shape)
    return f32(s), f32(F), pmf


# --------------------------------------------------------------------------
# restrained-MD-like CV trajectories (labelling workload)
# --------------------------------------------------------------------------
def restrained_traj(m: int, t: int, n: int, kappa: float, seed: int,
                    frame_std: float = 0.25):
    """Frames s_t ~ N(s0 - F_true/kappa, frame_std^2), wrapped to [-pi, pi).

    Returns (traj [m][t][n] f32, s0 [m][n] f32, F_true [m][n] f64)."""
    rng = np.random.default_rng(seed)
    s0 = rng.uniform(-math.pi, math.pi, size=(m, n))
    F_true = rng.normal(0.0, 20.0, size=(m, n))
    centre = s0 - F_true / kappa
    fr = centre[:, None, :] + rng.normal(0.0, frame_std, size=(m, t, n))
    fr = np.mod(fr + math.pi, 2 * math.pi) - math.pi
    return f32(fr), f32(s0), F_true


# --------------------------------------------------------------------------
# serving trace
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Request:
    arrival_s: float
    model_class: int   # index into the registered (system, ensemble) list
    n_walkers: int


def poisson_trace(n_req: int, rate_hz: float, n_classes: int, seed: int = 5,
                  max_walkers: int = 256):
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_req)
    t = np.cumsum(gaps)
    cls = rng.integers(0, n_classes, size=n_req)
    w = np.floor(np.exp(rng.uniform(0.0, math.log(max_walkers + 1), size=n_req)))
    w = np.clip(w, 1, max_walkers).astype(int)
    return [Request(float(t[i]), int(cls[i]), int(w[i])) for i in range(n_req)]


def exploration_frames(walkers: int, frames: int, n: int, n_basins: int, spread: float,
                       seed: int) -> np.ndarray:
    """CV frames [walkers * frames][n] (float32, angles in [-pi, pi)) shaped
    like an exploration phase's output: each walker starts in a random basin
    (centre uniform on the torus) and records a random walk around it that
    hops to another basin with probability 0.01 per frame; frames are listed
    walker by walker, in time order."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-math.pi, math.pi, size=(n_basins, n))
    out = np.empty((walkers * frames, n))
    for w in range(walkers):
        c = rng.integers(n_basins)
        x = centres[c] + rng.normal(0.0, spread, size=n)
        for t in range(frames):
            if rng.uniform() < 0.01:
                c = rng.integers(n_basins)
                x = centres[c] + rng.normal(0.0, spread, size=n)
            x = 0.7 * x + 0.3 * centres[c] + rng.normal(0.0, 0.5 * spread, size=n)
            out[w * frames + t] = x
    out = out - 2.0 * math.pi * np.floor((out + math.pi) / (2.0 * math.pi))
    return out.astype(np.float32)
