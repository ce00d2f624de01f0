"""Why the BF16 precision form runs its reverse sweep in FP16: a rounding-site
emulation of the 16-bit MLP kernel's arithmetic plans, in numpy on the CPU,
measured against the FP64 oracle on the precision form's shape (38 torsion
CVs, 8 x [512 x 4], 120 walkers).

The emulation rounds, at each of the kernel's rounding sites, the FP32 value
to the plan's format (BF16 round-to-nearest-even, or FP16); products
accumulate in FP64 (the kernel accumulates in FP32, whose error is far
below any 16-bit rounding).  Sites: the CV encoding, each layer's forward
weights (pre-scaled by 2/ln 2 as the kernel stores them), the stored hidden
activations, the stored tanh', the reverse vectors and each layer's reverse
weights.  It reproduces the GPU's measured all-BF16 error (max 1.8e-2 on 300
walkers) and predicts the precision form's (measured 3e-3).  No part of the
GPU path is used."""
import numpy as np
import pytest

import ridgen
from oracle import rid_oracle as O

C = np.float32(2.8853900817779268)      # the kernel's forward pre-scale 2/ln 2
L = 4


def bf16(a):
    b = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def f16(a):
    return np.asarray(a, np.float32).astype(np.float16).astype(np.float32)


def exact(a):
    return np.asarray(a, np.float32)


def member_g(model, s, plan):
    """g = dA/ds of one member with the plan's roundings; plan maps a site
    name to its rounding (default exact)."""
    Ws, bs, wo, _ = model
    r = lambda name, v: plan.get(name, exact)(v)
    h = r("x", O.embed(s).astype(np.float32))
    ds = []
    for l in range(L):
        Wf = r(f"Wf{l + 1}", (C * Ws[l]).astype(np.float32)).astype(np.float64) / C
        z = (h.astype(np.float64) @ Wf.T + bs[l]).astype(np.float32)
        t = np.tanh(z.astype(np.float64)).astype(np.float32)
        ds.append((1.0 - t.astype(np.float64) ** 2).astype(np.float32))
        h = r(f"h{l + 1}", t) if l < L - 1 else t
    v = r(f"v{L}", (wo * ds[L - 1]).astype(np.float32))
    for l in range(L, 0, -1):
        y = v.astype(np.float64) @ r(f"Wb{l}", Ws[l - 1].astype(np.float32)).astype(np.float64)
        if l > 1:
            v = r(f"v{l - 1}", (y * r(f"d{l - 1}", ds[l - 2])).astype(np.float32))
    n = s.shape[1]
    return -np.sin(s) * y[:, :n] + np.cos(s) * y[:, n:]


FWD = ["x"] + [f"Wf{i}" for i in range(1, L + 1)] + [f"h{i}" for i in range(1, L)]
REV = [f"d{i}" for i in range(1, L)] + [f"v{i}" for i in range(1, L + 1)] + \
      [f"Wb{i}" for i in range(1, L + 1)]
PLANS = {
    # every operand BF16, tanh' stored BF16 (RID_BF16_ALL)
    "bf16_all": {k: bf16 for k in FWD + REV},
    # RID_BF16: BF16 hidden-layer forward GEMMs; first layer, tanh' storage
    # and the reverse sweep in FP16
    "bf16": {**{k: f16 for k in REV + ["x", "Wf1"]},
             **{k: bf16 for k in ["Wf2", "Wf3", "Wf4", "h1", "h2", "h3"]}},
    "fp16": {k: f16 for k in FWD + REV},                # RID_FP16
    "bf16_fwd_only": {k: bf16 for k in FWD},            # forward sites alone
    "bf16_rev_only": {k: bf16 for k in REV},            # reverse sites alone
}


@pytest.fixture(scope="module")
def setup():
    sys_ = ridgen.system_peptide20()
    pos = ridgen.f32(ridgen.chain_coords(sys_, 120, 1)).astype(np.float64)
    params = ridgen.xavier_ensemble(2 * sys_.n_cv, [512] * L, 8, 1000, 0.0)
    models = ridgen.unpack_params(params, 2 * sys_.n_cv, [512] * L, 8)
    ref = O.bias_force(pos, sys_.quads, models, 2.0, 3.0)
    return sys_, pos, models, ref


def force_error(setup, plan):
    sys_, pos, models, ref = setup
    g = np.stack([member_g(m, ref["s"], plan) for m in models], axis=1)
    gbar, eps = O.model_deviation(g)
    sig, _ = O.switch(eps, 2.0, 3.0)
    F = O.apply_cv_force(pos, sys_.quads, sig[:, None] * gbar)
    return O.max_rel_err(F, ref["F"]), O.rms_rel_err(F, ref["F"])


def test_exact_plan_reproduces_the_oracle(setup):
    mx, _ = force_error(setup, {})
    assert mx < 1e-6


def test_precision_plans(setup):
    err = {k: force_error(setup, p) for k, p in PLANS.items()}
    for k, (mx, rms) in err.items():
        print(f"{k:14s} max {mx:.2e} rms {rms:.2e}")
    # the all-BF16 arithmetic misses the precision form's 1e-2 target ...
    assert err["bf16_all"][0] > 1e-2
    # ... because of its reverse sweep: alone it carries most of the error
    # variance, the forward sites alone give a few times less
    assert err["bf16_rev_only"][1] ** 2 > 0.8 * err["bf16_all"][1] ** 2
    assert err["bf16_fwd_only"][1] < 0.35 * err["bf16_all"][1]
    # the precision form's plan keeps BF16 only where it is damped
    assert err["bf16"][0] < 5e-3 and err["bf16"][1] < 2e-3
    assert err["fp16"][0] < 3e-3
