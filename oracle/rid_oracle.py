"""FP64 CPU oracle of the Reinforced-Dynamics neural-bias hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import this module.  It is plain, slow
and written to be checked by eye against the paper: numpy in float64, the
batch axis vectorised, no blocking, fusion or reordering beyond what each
definition states.  It shares no code with the GPU library.

Paper: "RiD-kit: Software package designed to do enhanced sampling using
reinforced dynamics" (arXiv 2408.14070).  Sections cited by name.  Where the
paper does not print a formula the reading taken is stated in the function
and listed (Z-numbers) with the other readings in the design notes.

Functions and what pins them (tests/test_oracle_*.py):

  dihedral            torsion CVs ("CV selection", torsion mode)
                      pinned: closed-form geometry, NeRF round trip,
                      rigid-motion invariance
  dihedral_jacobian   ds/dr (chain rule the bias uses to reach atoms)
                      pinned: central finite differences, zero net force and
                      torque per dihedral
  embed               [cos s | sin s] periodic input encoding; with an
                      angular mask, non-angular CVs as (s, 0)
                      pinned: 2pi periodicity of every downstream output;
                      mixed: linear-model closed form, FD in s
  distance_cv, cv_values, distance_jacobian
                      distance CVs and mixed CV tables ("CV selection",
                      `distance` type, `angular_mask`)
                      pinned: closed-form geometry, FD of the Jacobian,
                      zero net force and torque of a pair force, FD of the
                      whole mixed bias path
  mlp_value_and_grad  free-energy MLP A(x) and dA/dx ("Training phase":
                      MLP of `neurons` widths, tanh; optional residual
                      connections, the `resnet` setting)
                      pinned: closed forms for zero and one hidden layer,
                      finite differences of A in x; residual form: the
                      small-weight linear limit wo . prod(I + W_l) W_1 x,
                      reduction to one layer when the later layers are
                      zero, finite differences, one layer equals the plain
                      MLP
  ensemble_mean_force per-model mean force dA_k/ds (Box 2: F = grad_s A)
                      pinned: closed form for a linear model, FD in s
  model_deviation     ensemble standard deviation of the mean forces
                      ("Development of the protocol"; "Training phase")
                      pinned: identical members give exactly 0, K=2 closed
                      form, permutation invariance
  switch              trust-level switch ("Overall workflow setting")
                      pinned: limits, midpoint, monotone, continuity
  bias_force          whole path, atoms -> forces
                      pinned: force = -grad E by FD (sigma frozen), zero
                      total force and torque per walker
  mlp_input_hvp       Hessian-vector product of a model in its input
                      (plain and residual)
                      pinned: central FD of dA/dx along the vector
  deviation_gradient  d eps / d s (conservative switching), also on mixed
                      tables
                      pinned: central FD of eps in s (plain and masked)
  bias_force_conservative
                      -grad of E = -sigma(eps) Abar with the switch
                      differentiated too
                      pinned: force = -grad E by FD inside the switching
                      band (plain, residual and mixed tables); equals
                      bias_force where sigma is 0 or 1
  train_loss_grad     gradient of the mean-force loss in the weights
  mean_force_vjp      (plain, residual with or without dropout, mixed tables)
                      pinned: central FD on every parameter in each form;
                      exact least-squares solution of the linear model has
                      zero gradient; a residual network whose later layers
                      are zero has the one-layer network's gradient
  dropout_scales      training-time dropout of the hidden activations
                      (counter-based masks); pinned: finite differences of
                      the loss with the masks fixed, rate 0 reproduces the
                      plain gradient bit for bit, kept fraction within a
                      binomial bound, masks distinct per step and member
  adam_step / lr_at   optimiser and exponential LR decay ("Training phase")
                      pinned: one-step closed form; convergence on the linear
                      model to the analytic optimum
  philox4x32          counter-based generator of the MCMC
                      pinned: the published known-answer vectors
  mcmc_run            MCMC on the ensemble free energy ("Dimension
                      reduction phase"), histograms, pmf_from_histogram
                      pinned: infinite temperature is the plain random walk
                      of the generator; a one-CV closed-form model samples
                      exp(-A/kT); the PMF of that histogram recovers A
  mf_label            restrained-MD mean-force estimate ("Labeling phase")
                      pinned: Gaussian-frame closed form within 4 sigma, the
                      periodic wrap example, block standard error of iid
                      blocks
  leader_cluster      threshold clustering of CV frames ("Selection" phase;
  adapt_threshold     cluster threshold, cluster-count window, max_selection)
  select_frames       pinned: a hand-worked periodic example, brute-force
                      first-match and leader-separation checks, the two
                      threshold limits, a masked run equal to the run on
                      the kept subset, the window reached on well-separated
                      synthetic clusters
"""
from __future__ import annotations

import math

import numpy as np

# Default trust levels and optimiser schedule printed in the paper's example
# configuration ("Overall workflow setting", "Training phase").
TRUST_LVL_1 = 2.0
TRUST_LVL_2 = 3.0
INIT_LR = 8e-4
DECAY_STEPS = 120
DECAY_RATE = 0.96
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8
# Tolerance below which |n1|^2 or |n2|^2 marks a dihedral as degenerate (nm^4).
DEGENERATE_TOL = 1e-12


# --------------------------------------------------------------------------
# a1: torsion collective variables
# --------------------------------------------------------------------------
def _gather(pos, quads):
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(quads, dtype=np.int64)
    return pos[:, q[:, 0]], pos[:, q[:, 1]], pos[:, q[:, 2]], pos[:, q[:, 3]]


def dihedral(pos, quads):
    """Torsion angle s in (-pi, pi] of each quad (a, b, c, d), per walker.

    The paper's torsion CVs are backbone phi/psi ("CV selection").  Convention
    (IUPAC, as the MD engines use): b1 = r_b - r_a, b2 = r_c - r_b,
    b3 = r_d - r_c, n1 = b1 x b2, n2 = b2 x b3,
    s = atan2(|b2| b1 . n2, n1 . n2).

    pos: [B][n_atoms][3]; quads: [n][4] 0-based.  Returns s [B][n].
    """
    ra, rb, rc, rd = _gather(pos, quads)
    b1, b2, b3 = rb - ra, rc - rb, rd - rc
    n1 = np.cross(b1, b2)
    n2 = np.cross(b2, b3)
    X = np.sum(n1 * n2, axis=-1)
    Y = np.linalg.norm(b2, axis=-1) * np.sum(b1 * n2, axis=-1)
    return np.arctan2(Y, X)


def distance_cv(pos, pairs):
    """Distance CV s = |r_b - r_a| of each atom pair (a, b), per walker (the
    `distance` CV type of "CV selection").  pairs: [n][2] -> s [B][n]."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(pairs, dtype=np.int64)
    return np.linalg.norm(pos[:, q[:, 1]] - pos[:, q[:, 0]], axis=-1)


def distance_jacobian(pos, pairs):
    """ds/dr of each distance CV: slot a gets (r_a - r_b)/s, slot b its
    negative; a pair closer than sqrt(DEGENERATE_TOL) gets zeros.
    Returns [B][n][2][3]."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(pairs, dtype=np.int64)
    d = pos[:, q[:, 0]] - pos[:, q[:, 1]]
    r2 = np.sum(d * d, axis=-1, keepdims=True)
    u = d / np.sqrt(np.where(r2 < DEGENERATE_TOL, 1.0, r2))
    u = np.where(r2 < DEGENERATE_TOL, 0.0, u)
    return np.stack([u, -u], axis=2)


def _split_cvs(cvs, mask):
    """Rows of a mixed CV table: torsion quads where mask is 1, atom pairs
    (a, b, -1, -1) where it is 0.  Returns (mask bool [n], quads of the
    angular rows, pairs of the others)."""
    q = np.asarray(cvs, dtype=np.int64)
    m = np.ones(q.shape[0], bool) if mask is None else np.asarray(mask).astype(bool)
    return m, q[m], q[~m][:, :2]


def cv_values(pos, cvs, mask=None):
    """CV values of a mixed table (torsions where mask is 1, distances where
    it is 0), in table order.  [B][n]."""
    m, quads, pairs = _split_cvs(cvs, mask)
    pos = np.asarray(pos, dtype=np.float64)
    s = np.zeros((pos.shape[0], m.size))
    if quads.size:
        s[:, m] = dihedral(pos, quads)
    if pairs.size:
        s[:, ~m] = distance_cv(pos, pairs)
    return s


def cv_degenerate(pos, cvs, mask=None):
    """[B][n] bool: torsions as ``degenerate``; pairs closer than
    sqrt(DEGENERATE_TOL)."""
    m, quads, pairs = _split_cvs(cvs, mask)
    pos = np.asarray(pos, dtype=np.float64)
    out = np.zeros((pos.shape[0], m.size), bool)
    if quads.size:
        out[:, m] = degenerate(pos, quads)
    if pairs.size:
        out[:, ~m] = distance_cv(pos, pairs) ** 2 < DEGENERATE_TOL
    return out


def degenerate(pos, quads, tol=DEGENERATE_TOL):
    """[B][n] bool: dihedral whose |n1|^2 or |n2|^2 is below ``tol``."""
    ra, rb, rc, rd = _gather(pos, quads)
    b1, b2, b3 = rb - ra, rc - rb, rd - rc
    n1 = np.cross(b1, b2)
    n2 = np.cross(b2, b3)
    return (np.sum(n1 * n1, -1) < tol) | (np.sum(n2 * n2, -1) < tol)


def dihedral_jacobian(pos, quads):
    """ds/dr for the four atoms of every dihedral: [B][n][4][3].

    Closed form of the torsion gradient (Blondel & Karplus 1996) written in
    the b1, b2, b3 notation of ``dihedral``:
      ds/dr_a = -|b2| n1 / |n1|^2
      ds/dr_d = +|b2| n2 / |n2|^2
      ds/dr_b = (|b2| + b1.b2/|b2|) n1/|n1|^2 + (b3.b2/|b2|) n2/|n2|^2
      ds/dr_c = -(|b2| + b3.b2/|b2|) n2/|n2|^2 - (b1.b2/|b2|) n1/|n1|^2
    Degenerate dihedrals (see ``degenerate``) get a zero Jacobian.
    """
    ra, rb, rc, rd = _gather(pos, quads)
    b1, b2, b3 = rb - ra, rc - rb, rd - rc
    n1 = np.cross(b1, b2)
    n2 = np.cross(b2, b3)
    nn1 = np.sum(n1 * n1, -1, keepdims=True)
    nn2 = np.sum(n2 * n2, -1, keepdims=True)
    bad = (nn1 < DEGENERATE_TOL) | (nn2 < DEGENERATE_TOL)
    nn1 = np.where(bad, 1.0, nn1)
    nn2 = np.where(bad, 1.0, nn2)
    lb2 = np.linalg.norm(b2, axis=-1, keepdims=True)
    p1 = np.sum(b1 * b2, -1, keepdims=True) / lb2
    p3 = np.sum(b3 * b2, -1, keepdims=True) / lb2
    ga = -lb2 * n1 / nn1
    gd = lb2 * n2 / nn2
    gb = (lb2 + p1) * n1 / nn1 + p3 * n2 / nn2
    gc = -(lb2 + p3) * n2 / nn2 - p1 * n1 / nn1
    J = np.stack([ga, gb, gc, gd], axis=2)
    return np.where(bad[..., None], 0.0, J)


def apply_cv_force(pos, quads, fcv, n_atoms=None, mask=None):
    """Atomic forces F_a = sum_i f_i ds_i/dr_a.  fcv: [B][n] -> [B][N][3].
    With a mask, rows where it is 0 are distance pairs (a, b, -1, -1)."""
    pos = np.asarray(pos, dtype=np.float64)
    B, N, _ = pos.shape
    m, quads_a, pairs = _split_cvs(quads, mask)
    Ja = dihedral_jacobian(pos, quads_a) if quads_a.size else None
    Jd = distance_jacobian(pos, pairs) if pairs.size else None
    ia = np.cumsum(m) - 1             # row -> index among torsions / pairs
    idd = np.cumsum(~m) - 1
    F = np.zeros((B, N if n_atoms is None else n_atoms, 3))
    q = np.asarray(quads, dtype=np.int64)
    f = np.asarray(fcv, dtype=np.float64)
    for i in range(q.shape[0]):          # plain accumulation, CV by CV
        if m[i]:
            for slot in range(4):
                F[:, q[i, slot]] += f[:, i, None] * Ja[:, ia[i], slot]
        else:
            for slot in range(2):
                F[:, q[i, slot]] += f[:, i, None] * Jd[:, idd[i], slot]
    return F


# --------------------------------------------------------------------------
# a2/a3: ensemble of MLP free-energy models
# --------------------------------------------------------------------------
def embed(s, mask=None):
    """Periodic input encoding x = [cos s_1..cos s_n | sin s_1..sin s_n].

    With an angular mask (the `angular_mask` setting of "CV selection"), a
    CV whose entry is 0 is not periodic and enters raw.  Reading: it fills
    its own two slots as (s_i, 0), so x = [c | t] with (c_i, t_i) =
    (cos s_i, sin s_i) for angular CVs and (s_i, 0) for the others."""
    s = np.asarray(s, dtype=np.float64)
    if mask is None:
        return np.concatenate([np.cos(s), np.sin(s)], axis=-1)
    m = np.asarray(mask).astype(bool)
    c = np.where(m, np.cos(s), s)
    t = np.where(m, np.sin(s), 0.0)
    return np.concatenate([c, t], axis=-1)


def is_resnet(model):
    """True for a model with residual connections: (Ws, bs, wo, bo, True)."""
    return len(model) > 4 and bool(model[4])


def _plain_model(model, what):
    """The four parameter lists of a model without residual connections;
    a residual model is refused (``what`` is not built for it)."""
    if is_resnet(model):
        raise ValueError(what + " is defined here for plain MLPs only")
    return model[:4]


def mlp_value_and_grad(model, x, scales=None):
    """One free-energy model: A(x) and dA/dx.

    model = (Ws, bs, wo, bo): h_0 = x, h_l = tanh(W_l h_{l-1} + b_l),
    A = wo . h_L + bo.  Reverse sweep: u_L = wo, v_l = u_l * (1 - h_l^2),
    u_{l-1} = W_l^T v_l; dA/dx = u_0.  x: [B][D] -> (A [B], u0 [B][D]).
    scales (training with dropout): per hidden layer [B][w_l] factors that
    multiply h_l = tanh(z_l), and so its derivative (see dropout_scales).

    model = (Ws, bs, wo, bo, True): the `resnet` option of the training
    settings ("Training phase": residual connections, hidden layers of
    equal width).  Reading: every hidden layer after the first adds its
    input, h_l = h_{l-1} + tanh(W_l h_{l-1} + b_l) for l >= 2 (the first
    layer maps the CV encoding, of another width); the reverse sweep then
    carries the skip, u_{l-1} = W_l^T v_l + u_l for l >= 2, with
    v_l = u_l * (1 - tanh^2).  With dropout in a residual network the mask
    scales the layer's tanh branch, not the skip:
    h_l = h_{l-1} + S_l tanh(z_l).
    """
    Ws, bs, wo, bo = model[:4]
    res = is_resnet(model)
    if res and any(np.shape(W)[0] != np.shape(Ws[0])[0] for W in Ws):
        raise ValueError("residual connections need hidden layers of equal width")
    hs = [np.asarray(x, dtype=np.float64)]
    ts = [None]
    for l, (W, b) in enumerate(zip(Ws, bs)):
        t = np.tanh(hs[-1] @ W.T + b)
        ts.append(t)
        h = t if scales is None else t * scales[l]
        hs.append(h + hs[-1] if (res and l >= 1) else h)
    A = hs[-1] @ wo + bo
    u = np.broadcast_to(wo, hs[-1].shape)
    for l in range(len(Ws), 0, -1):
        d = 1.0 - ts[l] ** 2
        if scales is not None:
            d = d * scales[l - 1]
        v = u * d
        u = v @ Ws[l - 1] + (u if (res and l >= 2) else 0.0)
    return A, u


def mean_force_from_input_grad(s, u0, mask=None):
    """Chain dA/dx to the angles: g_i = -sin s_i u0[i] + cos s_i u0[n+i];
    a non-angular CV (mask 0, encoded (s_i, 0)) gets g_i = u0[i]."""
    s = np.asarray(s, dtype=np.float64)
    n = s.shape[-1]
    g = -np.sin(s) * u0[..., :n] + np.cos(s) * u0[..., n:]
    if mask is None:
        return g
    return np.where(np.asarray(mask).astype(bool), g, u0[..., :n])


def ensemble_mean_force(models, s, mask=None):
    """Per-model free energy and mean force (Box 2: F(s) = grad_s A(s)).

    s: [B][n] -> (A [B][K], g [B][K][n]).  mask: angular mask (see embed)."""
    x = embed(s, mask)
    As, gs = [], []
    for m in models:
        A, u0 = mlp_value_and_grad(m, x)
        As.append(A)
        gs.append(mean_force_from_input_grad(s, u0, mask))
    return np.stack(As, axis=1), np.stack(gs, axis=1)


# --------------------------------------------------------------------------
# a4/a5: model deviation and trust-level switch
# --------------------------------------------------------------------------
def model_deviation(g):
    """Ensemble mean force and model deviation.

    The paper takes the standard deviation of the ensemble's predictions as
    the uncertainty indicator.  Reading: population standard deviation of
    the K mean-force vectors, i.e. eps = sqrt((1/K) sum_k |g_k - gbar|^2),
    evaluated with a shift by member 0 (d_k = g_k - g_0) so identical members
    give exactly zero.  g: [B][K][n] -> (gbar [B][n], eps [B])."""
    g = np.asarray(g, dtype=np.float64)
    gbar = np.mean(g, axis=1)
    d = g - g[:, :1, :]
    dbar = np.mean(d, axis=1, keepdims=True)
    eps = np.sqrt(np.mean(np.sum((d - dbar) ** 2, axis=-1), axis=1))
    return gbar, eps


def switch(eps, eps0, eps1):
    """Trust-level switch sigma(eps) and regime r.

    trust_lvl_1 (eps0) and trust_lvl_2 (eps1) bound the trust level; the bias
    acts only where the uncertainty is low.  Reading: sigma = 1 below eps0,
    0 at or above eps1, and 1/2 (1 + cos(pi (eps-eps0)/(eps1-eps0))) between.
    Regime 0 = full bias, 1 = switching band (eps0 <= eps < eps1),
    2 = unbiased."""
    eps = np.asarray(eps, dtype=np.float64)
    t = (eps - eps0) / (eps1 - eps0)
    mid = 0.5 * (1.0 + np.cos(math.pi * t))
    sigma = np.where(eps < eps0, 1.0, np.where(eps >= eps1, 0.0, mid))
    regime = np.where(eps < eps0, 0, np.where(eps >= eps1, 2, 1)).astype(np.int8)
    return sigma, regime


def bias_force(pos, quads, models, eps0, eps1, n_atoms=None, mask=None):
    """Whole bias path for a batch of walkers.

    Bias energy E = -sigma(eps) * Abar (the inverted predicted PMF, only where
    the ensemble agrees); CV force f = sigma * gbar (sigma held fixed in the
    step); atomic force F_a = sum_i f_i ds_i/dr_a.

    Returns dict(F [B][N][3], E [B], eps [B], sigma [B], regime [B], s [B][n],
    A [B][K], g [B][K][n], gbar [B][n], flags [B]).
    With a mask, rows of ``quads`` where it is 0 are distance CVs (atom
    pairs (a, b, -1, -1)) that enter the networks raw (see embed)."""
    s = cv_values(pos, quads, mask)
    A, g = ensemble_mean_force(models, s, mask)
    gbar, eps = model_deviation(g)
    sigma, regime = switch(eps, eps0, eps1)
    E = -sigma * np.mean(A, axis=1)
    fcv = sigma[:, None] * gbar
    F = apply_cv_force(pos, quads, fcv, n_atoms, mask)
    flags = np.any(cv_degenerate(pos, quads, mask), axis=1).astype(np.uint8)
    return dict(F=F, E=E, eps=eps, sigma=sigma, regime=regime, s=s, A=A, g=g,
                gbar=gbar, flags=flags)


def bias_energy_frozen(pos, quads, models, sigma, mask=None):
    """E(r) = -sigma Abar(s(r)) with sigma given (finite-difference target)."""
    s = cv_values(pos, quads, mask)
    A, _ = ensemble_mean_force(models, s, mask)
    return -np.asarray(sigma) * np.mean(A, axis=1)


# --------------------------------------------------------------------------
# conservative switching: the switch differentiated as well
# --------------------------------------------------------------------------
def switch_slope(eps, eps0, eps1):
    """d sigma / d eps of the cosine switch: -pi/(2 (eps1-eps0)) sin(pi t)
    inside the band (eps0 <= eps < eps1), 0 outside."""
    eps = np.asarray(eps, dtype=np.float64)
    t = (eps - eps0) / (eps1 - eps0)
    slope = -0.5 * math.pi / (eps1 - eps0) * np.sin(math.pi * t)
    return np.where((eps >= eps0) & (eps < eps1), slope, 0.0)


def mlp_input_hvp(model, x, rho):
    """Hessian-vector product of one model in its input: H(x) rho with
    H = d^2 A / dx^2, as the forward-mode derivative of the reverse sweep
    of ``mlp_value_and_grad`` along rho.  Forward: h_l and its tangent
    hd_l = (1 - h_l^2) W_l hd_{l-1} (hd_0 = rho).  Reverse: v_L = wo (1 -
    h_L^2), u_{l-1} = W_l^T v_l, v_l = u_l (1 - h_l^2); its tangent uses
    d(1 - h^2) = -2 h hd.  x, rho: [B][D] -> [B][D].
    Residual networks: the tanh branch t_l and its tangent td_l = (1 - t_l^2)
    W_l hd_{l-1} enter the reverse sweep's derivative; h_l = h_{l-1} + t_l
    and hd_l = hd_{l-1} + td_l for l >= 2, and both u and its tangent ud
    carry the skip, u_{l-1} = W_l^T v_l + u_l."""
    Ws, bs, wo, bo = model[:4]
    res = is_resnet(model)
    hs = [np.asarray(x, dtype=np.float64)]
    hds = [np.asarray(rho, dtype=np.float64)]
    ts, tds = [None], [None]
    for l, (W, b) in enumerate(zip(Ws, bs), start=1):
        t = np.tanh(hs[-1] @ W.T + b)
        td = (1.0 - t ** 2) * (hds[-1] @ W.T)
        ts.append(t)
        tds.append(td)
        skip = res and l >= 2
        hs.append(t + hs[-1] if skip else t)
        hds.append(td + hds[-1] if skip else td)
    u = np.broadcast_to(wo, hs[-1].shape)
    ud = np.zeros_like(hs[-1])
    for l in range(len(Ws), 0, -1):
        v = u * (1.0 - ts[l] ** 2)
        vd = ud * (1.0 - ts[l] ** 2) - 2.0 * u * ts[l] * tds[l]
        skip = res and l >= 2
        u, ud = (v @ Ws[l - 1] + (u if skip else 0.0),
                 vd @ Ws[l - 1] + (ud if skip else 0.0))
    return ud


def deviation_gradient(models, s, mask=None):
    """d eps / d s of the model deviation (the reading of model_deviation).

    With w_k = (g_k - gbar) / (K eps), d eps/ds = sum_k H_k w_k, where H_k is
    the Hessian of A_k in s.  In the input x = [cos s | sin s], with
    J = dx/ds and rho = J w: H_k w = J^T H_x rho + (d rho/ds)^T dA/dx, the
    second term being -cos s_i w_i u0[i] - sin s_i w_i u0[n+i].  A raw CV
    (angular mask 0, encoded (s_i, 0)) has a linear encoding: its J^T slot
    is the identity on x_i and its second term vanishes.  eps = 0 gives 0.
    s: [B][n] -> (eps [B], deps_ds [B][n])."""
    s = np.asarray(s, dtype=np.float64)
    n = s.shape[-1]
    x = embed(s, mask)
    _, g = ensemble_mean_force(models, s, mask)
    gbar, eps = model_deviation(g)
    K = len(models)
    ang = np.ones(n, bool) if mask is None else np.asarray(mask).astype(bool)
    out = np.zeros_like(s)
    safe = np.where(eps > 0, eps, 1.0)
    for k, m in enumerate(models):
        w = (g[:, k, :] - gbar) / (K * safe[:, None])
        rho = rho_to_input(s, w, mask)
        _, u0 = mlp_value_and_grad(m, x)
        hx = mlp_input_hvp(m, x, rho)
        curv = -w * (np.cos(s) * u0[:, :n] + np.sin(s) * u0[:, n:])
        out += mean_force_from_input_grad(s, hx, mask) + np.where(ang, curv, 0.0)
    out[eps == 0] = 0.0
    return eps, out


def bias_force_conservative(pos, quads, models, eps0, eps1, n_atoms=None, mask=None):
    """Bias force that is exactly -grad E with E = -sigma(eps) Abar,
    including the switching band: f = sigma gbar + Abar sigma'(eps) deps/ds.
    Outside the band it equals bias_force.  Same outputs as bias_force."""
    out = bias_force(pos, quads, models, eps0, eps1, n_atoms, mask)
    s = out["s"]
    _, deps = deviation_gradient(models, s, mask)
    Abar = np.mean(out["A"], axis=1)
    fcv = out["sigma"][:, None] * out["gbar"] + \
        (Abar * switch_slope(out["eps"], eps0, eps1))[:, None] * deps
    out["fcv"] = fcv
    out["F"] = apply_cv_force(pos, quads, fcv, n_atoms, mask)
    return out


def bias_energy(pos, quads, models, eps0, eps1, mask=None):
    """E(r) = -sigma(eps(s(r))) Abar(s(r)), the switch evaluated at r
    (finite-difference target of the conservative force)."""
    s = cv_values(pos, quads, mask)
    A, g = ensemble_mean_force(models, s, mask)
    _, eps = model_deviation(g)
    sigma, _ = switch(eps, eps0, eps1)
    return -sigma * np.mean(A, axis=1)


# --------------------------------------------------------------------------
# a7: mean-force fitting, double backward, Adam
# --------------------------------------------------------------------------
def train_loss_grad(model, s, F, scales=None, mask=None):
    """Loss L = (1/B) sum_b |g(s_b) - F_b|^2 of one model and its gradient.

    The models are trained to predict mean forces ("Training phase"), i.e.
    the network's CV-gradient is fitted to the labels.  Since
    dL = sum_b rho_b . dg_b with rho_b = 2 (g_b - F_b)/B, the parameter
    gradient is that of the directional derivative J = sum_b rho_x,b . dA/dx
    (rho_x = rho mapped to x: [-sin s rho | cos s rho]) with rho_x held fixed:
      tangent:  hd_0 = rho_x, zd_l = W_l hd_{l-1}, hd_l = (1-h_l^2) zd_l,
                J = wo . hd_L
      adjoint:  lam_hd_L = wo, lam_h_L = 0; for l = L..1:
                lam_zd = (1-h_l^2) lam_hd;  lam_h += -2 h_l zd_l lam_hd
                lam_z  = (1-h_l^2) lam_h
                dW_l = lam_z h_{l-1}^T + lam_zd hd_{l-1}^T;  db_l = lam_z
                lam_hd_{l-1} = W_l^T lam_zd;  lam_h_{l-1} = W_l^T lam_z
      dwo = hd_L;  dbo = 0 (the constant never reaches grad_s A).
    Residual networks, dropout and angular masks as in mean_force_vjp.
    Returns (loss, (dWs, dbs, dwo, dbo)), all summed over the batch.
    """
    s = np.asarray(s, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    B, n = s.shape
    A, u0 = mlp_value_and_grad(model, embed(s, mask), scales)
    g = mean_force_from_input_grad(s, u0, mask)
    r = g - F
    loss = float(np.sum(r * r) / B)
    return loss, mean_force_vjp(model, s, 2.0 * r / B, scales, mask)


def rho_to_input(s, rho, mask=None):
    """A CV-space vector mapped to the network input by the encoding's
    Jacobian dx/ds: (rho_x[i], rho_x[n+i]) = (-sin s_i, cos s_i) rho_i for
    an angular CV, (rho_i, 0) for a raw one (encoded (s_i, 0))."""
    s = np.asarray(s, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    a = np.concatenate([-np.sin(s) * rho, np.cos(s) * rho], axis=-1)
    if mask is None:
        return a
    m = np.asarray(mask).astype(bool)
    return np.concatenate([np.where(m, a[..., :s.shape[-1]], rho),
                           np.where(m, a[..., s.shape[-1]:], 0.0)], axis=-1)


def mean_force_vjp(model, s, rho, scales=None, mask=None):
    """Gradient in the parameters of J = sum_b rho_b . g(s_b) for a given
    rho [B][n] (the tangent + adjoint sweep described in train_loss_grad).
    With dropout scales S_l the hidden output is S_l tanh(z_l): its
    derivative d_l = S_l (1 - t_l^2) (t_l = tanh(z_l)) replaces
    (1 - h_l^2) throughout, and the second-order term -2 t_l zd_l keeps the
    unscaled tanh.  Residual networks (h_l = h_{l-1} + S_l t_l for l >= 2):
    the tangent carries the skip too, hd_l = hd_{l-1} + d_l zd_l, and in the
    adjoint both lam_h_l and lam_hd_l flow unchanged into layer l-1 beside
    W_l^T [lam_z ; lam_zd]; everything else is the plain recipe.  With an
    angular mask, rho reaches the input through rho_to_input.
    Returns (dWs, dbs, dwo, dbo)."""
    Ws, bs, wo, bo = model[:4]
    res = is_resnet(model)
    s = np.asarray(s, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    x = embed(s, mask)
    rho_x = rho_to_input(s, rho, mask)
    # primal activations (ts: tanh before the dropout scale)
    hs = [x]
    ts = [None]
    for l, (W, b) in enumerate(zip(Ws, bs)):
        t = np.tanh(hs[-1] @ W.T + b)
        ts.append(t)
        h = t if scales is None else t * scales[l]
        hs.append(h + hs[-1] if (res and l >= 1) else h)
    ds = [None] + [(1.0 - ts[l] ** 2) * (1.0 if scales is None else scales[l - 1])
                   for l in range(1, len(Ws) + 1)]
    # tangent forward
    hds = [rho_x]
    zds = [None]
    for l, W in enumerate(Ws, start=1):
        zd = hds[-1] @ W.T
        zds.append(zd)
        hd = ds[l] * zd
        hds.append(hd + hds[-1] if (res and l >= 2) else hd)
    L = len(Ws)
    dWs = [None] * L
    dbs = [None] * L
    dwo = np.sum(hds[L], axis=0)
    lam_hd = np.broadcast_to(wo, hds[L].shape)
    lam_h = np.zeros_like(hs[L])
    for l in range(L, 0, -1):
        dl = ds[l]
        lam_zd = dl * lam_hd
        lam_z = dl * (lam_h - 2.0 * ts[l] * zds[l] * lam_hd)
        dWs[l - 1] = lam_z.T @ hs[l - 1] + lam_zd.T @ hds[l - 1]
        dbs[l - 1] = np.sum(lam_z, axis=0)
        skip = res and l >= 2
        lam_hd, lam_h = (lam_zd @ Ws[l - 1] + (lam_hd if skip else 0.0),
                         lam_z @ Ws[l - 1] + (lam_h if skip else 0.0))
    return (dWs, dbs, dwo, 0.0)


def train_loss(model, s, F, scales=None, mask=None):
    """Loss only (finite-difference target)."""
    s = np.asarray(s, dtype=np.float64)
    _, u0 = mlp_value_and_grad(model, embed(s, mask), scales)
    r = mean_force_from_input_grad(s, u0, mask) - np.asarray(F, dtype=np.float64)
    return float(np.sum(r * r) / r.shape[0])


def lr_at(step, init_lr=INIT_LR, decay_steps=DECAY_STEPS, decay_rate=DECAY_RATE):
    """Exponential learning-rate decay, continuous form:
    lr = init_lr * decay_rate ** (step / decay_steps); step counts updates
    already taken (0 for the first)."""
    return init_lr * decay_rate ** (step / decay_steps)


def adam_step(theta, grad, m, v, t, lr, b1=ADAM_B1, b2=ADAM_B2, eps=ADAM_EPS):
    """One Adam update (bias-corrected); t is the 1-based update count.
    Returns (theta', m', v')."""
    theta = np.asarray(theta, dtype=np.float64)
    grad = np.asarray(grad, dtype=np.float64)
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def flat_grad(grads):
    """Flatten a (dWs, dbs, dwo, dbo) tuple in the packed parameter order."""
    dWs, dbs, dwo, dbo = grads
    parts = []
    for dW, db in zip(dWs, dbs):
        parts += [np.ravel(dW), np.ravel(db)]
    parts += [np.ravel(dwo), np.atleast_1d(float(dbo))]
    return np.concatenate(parts)


def flat_model(model):
    Ws, bs, wo, bo = model[:4]
    parts = []
    for W, b in zip(Ws, bs):
        parts += [np.ravel(W), np.ravel(b)]
    parts += [np.ravel(wo), np.atleast_1d(float(bo))]
    return np.concatenate(parts).astype(np.float64)


def unflat_model(flat, n_in, widths, resnet=False):
    p = np.asarray(flat, dtype=np.float64)
    Ws, bs = [], []
    off, prev = 0, n_in
    for w in widths:
        Ws.append(p[off:off + w * prev].reshape(w, prev)); off += w * prev
        bs.append(p[off:off + w]); off += w
        prev = w
    wo = p[off:off + prev]; off += prev
    bo = float(p[off])
    return (Ws, bs, wo, bo, True) if resnet else (Ws, bs, wo, bo)


def train_step(models, s, F, states, lr, dropout=None, mask=None):
    """One mean-force fitting step for every member (same minibatch, models
    independent).  states: list of (m, v, t) per model (t = updates done).
    dropout: (rate, seed) or None; member k's masks are those of step t
    (dropout_scales).  mask: angular mask of the CVs.
    Returns (new_models, new_states, losses [K])."""
    new_models, new_states, losses = [], [], []
    widths = [W.shape[0] for W in models[0][0]]
    n_in = models[0][0][0].shape[1] if models[0][0] else models[0][2].size
    for k, (model, (m, v, t)) in enumerate(zip(models, states)):
        sc = None
        if dropout is not None and dropout[0] > 0.0:
            sc = dropout_scales(len(s), widths, dropout[0], dropout[1], t, k)
        loss, grads = train_loss_grad(model, s, F, sc, mask)
        theta, m2, v2 = adam_step(flat_model(model), flat_grad(grads), m, v,
                                  t + 1, lr)
        new_models.append(unflat_model(theta, n_in, widths, is_resnet(model)))
        new_states.append((m2, v2, t + 1))
        losses.append(loss)
    return new_models, new_states, np.asarray(losses)


# --------------------------------------------------------------------------
# MCMC on the learned free energy ("Dimension reduction phase")
# --------------------------------------------------------------------------
BOLTZMANN_KJ_MOL_K = 0.0083144626   # k_B in kJ/mol/K (GROMACS units)

PHILOX_M = (0xD2511F53, 0xCD9E8D57)
PHILOX_W = (0x9E3779B9, 0xBB67AE85)


def philox4x32(ctr, key):
    """Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers:
    as easy as 1, 2, 3", SC 2011), a counter-based generator: ten rounds of
    two 32x32->64 multiplications; the key is bumped by the Weyl constants
    between rounds.  ctr: [..., 4] integers < 2^32; key: (k0, k1).
    Returns [..., 4] uint32."""
    c = np.asarray(ctr, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    c0, c1, c2, c3 = (c[..., i].copy() for i in range(4))
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    mask = np.uint64(0xFFFFFFFF)
    for _ in range(10):
        p0 = np.uint64(PHILOX_M[0]) * c0
        p1 = np.uint64(PHILOX_M[1]) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0)), lo1, (hi0 ^ c3 ^ np.uint64(k1)), lo0
        k0 = (k0 + PHILOX_W[0]) & 0xFFFFFFFF
        k1 = (k1 + PHILOX_W[1]) & 0xFFFFFFFF
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def mcmc_uniforms(walkers, t, count, seed):
    """The uniforms of MCMC step t for the given walkers: word 4j+i of the
    Philox block with counter (walker, t mod 2^32, t div 2^32, j) and key
    (seed mod 2^32, seed div 2^32); a 32-bit word x gives
    u = (2 (x >> 9) + 1) 2^-24, exactly representable in FP32, in (0, 1).
    Returns [len(walkers)][count] float64."""
    w = np.asarray(walkers, dtype=np.uint64)
    nblk = (count + 3) // 4
    t = int(t)
    ctr = np.zeros((len(w), nblk, 4), dtype=np.uint64)
    ctr[:, :, 0] = w[:, None]
    ctr[:, :, 1] = t & 0xFFFFFFFF
    ctr[:, :, 2] = t >> 32
    ctr[:, :, 3] = np.arange(nblk, dtype=np.uint64)[None, :]
    x = philox4x32(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    x = x.reshape(len(w), nblk * 4)[:, :count].astype(np.float64)
    return (2.0 * np.floor(x / 512.0) + 1.0) * 2.0 ** -24


def dropout_scales(B, widths, rate, seed, step, member):
    """Inverted-dropout factors of one model for one training step (the
    paper names a dropout rate among the training settings; reading: every
    hidden activation tanh(z_l) of a sample is kept with probability
    1 - rate and scaled by 1/(1 - rate), dropped otherwise).  Unit j of
    hidden layer l (1-based) of sample b takes word j mod 4 of the
    Philox4x32-10 block with counter (b, step mod 2^32, 16 member + l,
    j div 4) and key (seed mod 2^32, seed div 2^32); the word x gives
    u = (2 (x >> 9) + 1) 2^-24 and the unit is kept when u >= rate, compared
    in FP32.  Returns [len(widths)] arrays [B][w_l] of 0 or 1/(1 - rate)."""
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    p32 = np.float32(rate)
    inv = float(np.float32(1.0) / (np.float32(1.0) - p32))
    out = []
    for l, w in enumerate(widths, start=1):
        nblk = (w + 3) // 4
        ctr = np.zeros((B, nblk, 4), dtype=np.uint64)
        ctr[:, :, 0] = np.arange(B, dtype=np.uint64)[:, None]
        ctr[:, :, 1] = int(step) & 0xFFFFFFFF
        ctr[:, :, 2] = 16 * int(member) + l
        ctr[:, :, 3] = np.arange(nblk, dtype=np.uint64)[None, :]
        x = philox4x32(ctr, key).reshape(B, nblk * 4)[:, :w].astype(np.float64)
        u = ((2.0 * np.floor(x / 512.0) + 1.0) * 2.0 ** -24).astype(np.float32)
        out.append(np.where(u >= p32, inv, 0.0))
    return out


def wrap_torus(s):
    """Map angles to [-pi, pi)."""
    s = np.asarray(s, dtype=np.float64)
    return s - 2.0 * math.pi * np.floor((s + math.pi) / (2.0 * math.pi))


def cv_bins(s, nbins):
    """Histogram bin of angles in [-pi, pi): floor((s + pi) nbins / 2pi),
    clamped to [0, nbins - 1]."""
    b = np.floor((np.asarray(s, np.float64) + math.pi) * (nbins / (2.0 * math.pi)))
    return np.clip(b, 0, nbins - 1).astype(np.int64)


def ensemble_energy(models, s, mask=None):
    """Abar(s): the ensemble mean of the members' free energies."""
    A, _ = ensemble_mean_force(models, s, mask)
    return np.mean(A, axis=1)


def box_bins(s, lo, hi, nbins):
    """Histogram bin of a raw CV in its box [lo, hi):
    floor((s - lo) nbins / (hi - lo)), clamped to [0, nbins - 1]."""
    b = np.floor((np.asarray(s, np.float64) - lo) * (nbins / (hi - lo)))
    return np.clip(b, 0, nbins - 1).astype(np.int64)


def mcmc_run(models, s0, n_steps, kT, step, seed, t0=0, proj=(0, 1), nbins=101,
             keep_path=False, mask=None, lower=None, upper=None):
    """Metropolis MCMC in CV space on the ensemble's free energy, the
    dimension-reduction phase: many walkers, a temperature, histograms of
    every CV and of one projected pair, PMF = -kT ln p.  Readings (the paper
    names walkers, steps, temperature, bins and projected indices only):
    target density exp(-Abar(s)/kT) with Abar the ensemble mean; proposal
    s' = wrap(s + step (2u - 1)) on every CV at once (u from mcmc_uniforms,
    words 0..n-1); accept when u_n < exp(-(Abar(s') - Abar(s))/kT) (word n);
    after each step the walker's current state is counted in the 1D
    histograms of every CV and the 2D histogram of the pair ``proj``.

    Raw CVs (angular mask 0, distances: the paper's `cv_type` "dis") walk in
    the box [lower_i, upper_i] of the dimension-reduction settings
    (`cv_lower_bound`, `cv_upper_bound`, which the paper introduces to bound
    distance CVs).  Reading: the proposal moves a raw CV by
    step (upper_i - lower_i) / 2pi (2u - 1) -- the same fraction of its
    range as the angles' step of the circle -- without wrapping; a proposal
    with a raw CV outside its box has zero target density and is rejected;
    raw CVs are binned over their box (box_bins).  A walker may start outside
    its box: it can then only move into it.

    s0: [W][n].  Returns dict(s, A, hist1 [n][nbins], hist2 [nbins][nbins],
    accepted, path [n_steps][W][n] when keep_path)."""
    s0 = np.asarray(s0, dtype=np.float64)
    W, n = s0.shape
    ang = np.ones(n, bool) if mask is None else np.asarray(mask).astype(bool)
    if not np.all(ang):
        lo = np.asarray(lower, dtype=np.float64)
        hi = np.asarray(upper, dtype=np.float64)
        if not np.all(hi[~ang] > lo[~ang]):
            raise ValueError("raw CVs need lower < upper")
        span = np.where(ang, 2.0 * math.pi, hi - lo)
    s = np.where(ang, wrap_torus(s0), s0)
    A = ensemble_energy(models, s, mask)
    hist1 = np.zeros((n, nbins), dtype=np.int64)
    hist2 = np.zeros((nbins, nbins), dtype=np.int64)
    accepted = 0
    path = []
    walkers = np.arange(W)

    def bins(v):
        b = cv_bins(v, nbins)
        if np.all(ang):
            return b
        return np.where(ang, b, box_bins(v, lo, hi, nbins))

    for t in range(t0, t0 + n_steps):
        u = mcmc_uniforms(walkers, t, n + 1, seed)
        if np.all(ang):
            sp = wrap_torus(s + step * (2.0 * u[:, :n] - 1.0))
            inbox = np.ones(W, bool)
        else:
            prop = s + step * span / (2.0 * math.pi) * (2.0 * u[:, :n] - 1.0)
            sp = np.where(ang, wrap_torus(prop), prop)
            inbox = np.all(ang | ((sp >= lo) & (sp <= hi)), axis=1)
        Ap = ensemble_energy(models, sp, mask)
        acc = inbox & (u[:, n] < np.exp(-(Ap - A) / kT))
        s = np.where(acc[:, None], sp, s)
        A = np.where(acc, Ap, A)
        accepted += int(np.sum(acc))
        b = bins(s)
        for i in range(n):
            hist1[i] += np.bincount(b[:, i], minlength=nbins)
        np.add.at(hist2, (b[:, proj[0]], b[:, proj[1]]), 1)
        if keep_path:
            path.append(s.copy())
    out = dict(s=s, A=A, hist1=hist1, hist2=hist2, accepted=accepted)
    if keep_path:
        out["path"] = np.stack(path)
    return out


def pmf_from_histogram(hist, kT):
    """Projected PMF -kT ln p of a histogram, shifted to a minimum of 0;
    empty bins give +inf."""
    h = np.asarray(hist, dtype=np.float64)
    with np.errstate(divide="ignore"):
        f = -kT * np.log(h / h.sum())
    return f - np.min(f[np.isfinite(f)])


# --------------------------------------------------------------------------
# a8: restrained-MD mean-force labels
# --------------------------------------------------------------------------
def wrap_angle(d):
    """Map a difference of two angles in (-2pi, 2pi) to (-pi, pi]."""
    d = np.asarray(d, dtype=np.float64)
    d = np.where(d > math.pi, d - 2.0 * math.pi, d)
    return np.where(d <= -math.pi, d + 2.0 * math.pi, d)


def _neumaier_sum(terms, axis):
    """Compensated (Neumaier) summation along ``axis``, term by term."""
    terms = np.moveaxis(np.asarray(terms, dtype=np.float64), axis, 0)
    s = np.zeros(terms.shape[1:])
    c = np.zeros(terms.shape[1:])
    for t in terms:
        tot = s + t
        c += np.where(np.abs(s) >= np.abs(t), (s - tot) + t, (t - tot) + s)
        s = tot
    return s + c


def mf_label(traj, s0, kappa, mask, std_threshold, n_blocks=10):
    """Mean force from a restrained trajectory ("Labeling phase").

    Under a stiff harmonic restraint kappa/2 (s - s0)^2 the mean force is the
    average spring force: F_i = kappa_i * mean_t wrap(s0_i - s_{t,i}) (wrap to
    (-pi, pi] for periodic CVs, mask 1).  Convergence: the frames are split
    into n_blocks equal blocks of floor(T/n_blocks) frames (the tail frames
    are left out of the blocks only); SE_i = std of the block means
    (n_blocks - 1 in the denominator) / sqrt(n_blocks).  A configuration is
    kept when max_i SE_i <= std_threshold.

    traj [M][T][n], s0 [M][n], kappa [n], mask [n] ->
    (F [M][n], SE [M][n], keep [M] uint8)."""
    traj = np.asarray(traj, dtype=np.float64)
    s0 = np.asarray(s0, dtype=np.float64)
    kappa = np.asarray(kappa, dtype=np.float64)
    mask = np.asarray(mask).astype(bool)
    M, T, n = traj.shape
    diff = s0[:, None, :] - traj
    diff = np.where(mask, wrap_angle(diff), diff)
    spring = kappa * diff
    F = _neumaier_sum(spring, axis=1) / T
    bsz = T // n_blocks
    blocks = spring[:, :bsz * n_blocks].reshape(M, n_blocks, bsz, n)
    bmean = _neumaier_sum(blocks, axis=2) / bsz
    bbar = np.mean(bmean, axis=1, keepdims=True)
    var = np.sum((bmean - bbar) ** 2, axis=1) / (n_blocks - 1)
    SE = np.sqrt(var / n_blocks)
    keep = (np.max(SE, axis=1) <= std_threshold).astype(np.uint8)
    return F, SE, keep


# --------------------------------------------------------------------------
# comparison metrics
# --------------------------------------------------------------------------
def max_rel_err(test, ref):
    """max over walkers of max|test - ref| / max|ref| (normwise per walker)."""
    test = np.asarray(test, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    B = ref.shape[0]
    d = np.abs(test - ref).reshape(B, -1).max(axis=1)
    r = np.abs(ref).reshape(B, -1).max(axis=1)
    return float(np.max(d / np.where(r > 0, r, 1.0)))


def rms_rel_err(test, ref):
    test = np.asarray(test, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(test - ref) / max(np.linalg.norm(ref), 1e-300))


# --------------------------------------------------------------------------
# next-3: selection ("Selection" phase; "SelectorConfig": cluster_threshold,
# numb_cluster_lower/upper, max_selection)
# --------------------------------------------------------------------------
def frame_deviation(models, s, mask=None):
    """Model deviation eps of CV frames s [B][n] (the uncertainty the
    selection filters on): model_deviation of the ensemble's mean forces."""
    _, g = ensemble_mean_force(models, s, mask)
    return model_deviation(g)[1]


def cv_distance_sq_f32(a, b, mask=None, weights=None):
    """Squared periodic distance between CV vectors a, b [..., n] (angles in
    [-pi, pi]) in the FP32 arithmetic the clustering decides in: per CV the
    FP32 difference wrapped to (-pi, pi] with FP32 constants, then the
    squares summed in CV order, every product and sum rounded to FP32 (no
    fused multiply-add).  CVs whose angular-mask entry is 0 (distances) are
    not periodic: their difference is not wrapped.
    weights: the per-CV clustering weights of the CV settings ("weights";
    reading: a weighted Euclidean metric, d^2 = sum_i w_i wrap(a_i - b_i)^2,
    each square multiplied by its weight in FP32 before it is added); None
    means every weight is 1."""
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    pi = np.float32(math.pi)
    two_pi = np.float32(2.0 * math.pi)
    w = None if weights is None else np.asarray(weights, dtype=np.float32)
    acc = np.zeros(np.broadcast(a[..., 0], b[..., 0]).shape, dtype=np.float32)
    for i in range(a.shape[-1]):
        d = (a[..., i] - b[..., i]).astype(np.float32)
        if mask is None or mask[i]:
            d = np.where(d > pi, (d - two_pi).astype(np.float32), d)
            d = np.where(d <= -pi, (d + two_pi).astype(np.float32), d)
        sq = (d * d).astype(np.float32)
        if w is not None:
            sq = (sq * w[i]).astype(np.float32)
        acc = (acc + sq).astype(np.float32)
    return acc


def leader_cluster(s, threshold, keep=None, max_clusters=None, mask=None, weights=None):
    """Threshold clustering of CV frames.  Reading (the paper names a cluster
    threshold and a window for the cluster count, not the algorithm): frames
    are taken in order; a kept frame joins the first cluster, in founding
    order, whose leader lies within the threshold (squared FP32 periodic
    distance <= threshold^2 in FP32), otherwise it founds a cluster and is
    its leader (the cluster's representative).  Frames not kept get label
    -2.  With max_clusters, a frame that would found cluster number
    max_clusters gets label -1 and the count is reported as
    max_clusters + 1 ("more than the cap").
    Returns (labels [B] int64, leaders [frame indices], n_clusters)."""
    s = np.asarray(s, dtype=np.float32)
    B = s.shape[0]
    t = np.float32(threshold)
    t2 = np.float32(t * t)
    labels = np.full(B, -2, dtype=np.int64)
    leaders = []
    over = False
    for f in range(B):
        if keep is not None and not keep[f]:
            continue
        if leaders:
            hit = np.nonzero(cv_distance_sq_f32(s[leaders], s[f][None, :], mask, weights) <= t2)[0]
            if hit.size:
                labels[f] = hit[0]
                continue
        if max_clusters is not None and len(leaders) >= max_clusters:
            labels[f] = -1
            over = True
            continue
        labels[f] = len(leaders)
        leaders.append(f)
    return labels, leaders, len(leaders) + (1 if over else 0)


THRESHOLD_FACTOR = np.float32(1.1)


def adapt_threshold(s, threshold, lower, upper, keep=None, max_clusters=None, max_iter=100,
                    mask=None, weights=None):
    """Reading of the threshold adjustment (first iteration only; the rule is
    not printed): while the cluster count is above `upper` the threshold is
    multiplied by 1.1, while below `lower` divided by 1.1 (FP32), at most
    max_iter adjustments.  Returns (threshold, leader_cluster result)."""
    t = np.float32(threshold)
    for it in range(max_iter + 1):
        res = leader_cluster(s, t, keep, max_clusters, mask, weights)
        n = res[2]
        if lower <= n <= upper or it == max_iter:
            return t, res
        t = np.float32(t * THRESHOLD_FACTOR) if n > upper else np.float32(t / THRESHOLD_FACTOR)
    return t, res


def select_frames(models, s, eps0, threshold, lower, upper, max_selection, adapt=True,
                  max_iter=100, mask=None, weights=None):
    """Selection: the frames whose model deviation reaches the lower trust
    level (eps >= eps0, reading: "high model deviation" relative to the
    trust level) are clustered, the threshold adapted into [lower, upper]
    when `adapt`, and the leaders of the first max_selection clusters are
    the selected frames.  Returns dict(eps, keep, threshold, labels,
    leaders, n_clusters, selected)."""
    eps = frame_deviation(models, s, mask)
    keep = eps >= eps0
    cap = max(upper, max_selection) + 1
    if adapt:
        t, (labels, leaders, n) = adapt_threshold(s, threshold, lower, upper, keep, cap, max_iter,
                                                  mask, weights)
    else:
        t = np.float32(threshold)
        labels, leaders, n = leader_cluster(s, t, keep, cap, mask, weights)
    return dict(eps=eps, keep=keep, threshold=t, labels=labels, leaders=leaders,
                n_clusters=n, selected=list(leaders[:max_selection]))


def adjust_trust_levels(n_clusters, numb_cluster_threshold, trust_lvl_1, trust_lvl_2, scale):
    """Trust levels for the next iteration ("Selection phase",
    numb_cluster_threshold).  The paper states only that the trust levels
    are adjusted when the number of clusters found in the current
    iteration's exploration frames is below numb_cluster_threshold, and
    (troubleshooting table) that raising them encourages exploration; the
    rule itself is in a cited paper.  Reading: below the threshold both
    levels are multiplied by `scale` (> 1, the caller's choice), keeping
    their ratio; otherwise they are returned unchanged.  FP32 products, as
    the library computes them."""
    if scale <= 1.0 or not math.isfinite(scale):
        raise ValueError("scale must be finite and above 1")
    if not (0.0 <= trust_lvl_1 < trust_lvl_2):
        raise ValueError("trust levels must satisfy 0 <= lvl_1 < lvl_2")
    if n_clusters < numb_cluster_threshold:
        return (float(np.float32(trust_lvl_1) * np.float32(scale)),
                float(np.float32(trust_lvl_2) * np.float32(scale)))
    return float(np.float32(trust_lvl_1)), float(np.float32(trust_lvl_2))
