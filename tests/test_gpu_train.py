"""GPU parity of the mean-force fitting step (double backward + Adam) and of
the autograd wrapper, against the FP64 oracle.

Gradient tolerance: the weight gradient is a sum over 2B rows of products of
FP32 activations that each carry ~1e-6 relative error after the forward,
primal-backward, tangent and adjoint sweeps; 1e-4 normwise per member (max
abs error over the member's gradient / its max magnitude) leaves a factor
~10 over the error measured at the full batch."""
import numpy as np
import pytest

import ridgen
from oracle import rid_oracle as O

pytestmark = pytest.mark.gpu
GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def rid():
    import paper_2408_14070_amd as r
    r.lib()
    return r


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _grad_ref(params, n, widths, K, s, F):
    models = ridgen.unpack_params(params, 2 * n, widths, K)
    losses, grads = [], []
    for m in models:
        loss, g = O.train_loss_grad(m, s.astype(np.float64), F.astype(np.float64))
        losses.append(loss)
        grads.append(O.flat_grad(g))
    return np.array(losses), np.stack(grads)


def _per_member_err(grad_gpu, grad_ref):
    K = grad_ref.shape[0]
    g = grad_gpu.reshape(K, -1).astype(np.float64)
    return max(np.max(np.abs(g[k] - grad_ref[k])) / np.max(np.abs(grad_ref[k])) for k in range(K))


# FP32 ensembles of padded width <= 256 take the fused sweep kernel (six
# hidden layers fill every register stash slot); the width-300 case and the
# 256-CV case (its input tile does not fit the fused kernel's LDS) take the
# sweeps as separate GEMMs.
@pytest.mark.parametrize("n,widths,K,B", [(3, [5, 4], 2, 4), (38, [256] * 4, 4, 4096),
                                          (7, [100, 33, 70], 3, 257), (2, [100] * 3, 4, 1000),
                                          (4, [32] * 6, 2, 50), (5, [300, 40], 2, 100),
                                          (256, [64, 64], 2, 20)])
def test_loss_grad_parity(torch, rid, n, widths, K, B):
    params = ridgen.xavier_ensemble(2 * n, widths, K, 1000, bias_std=0.1)
    s, F, _ = ridgen.mf_training_set(B, n)
    E = rid.Ensemble(n, widths, K, params)
    loss, grad = rid.mf_loss_grad(E, _dev(torch, s), _dev(torch, F))
    torch.cuda.synchronize()
    loss_ref, grad_ref = _grad_ref(params, n, widths, K, s, F)
    lerr = np.max(np.abs(loss.cpu().numpy() - loss_ref) / loss_ref)
    gerr = _per_member_err(grad.cpu().numpy(), grad_ref)
    print(f"n={n} widths={widths} K={K} B={B}: loss rel err {lerr:.2e}, grad err {gerr:.2e}")
    assert lerr <= 1e-5
    assert gerr <= GRAD_TOL
    # output-bias entries are exactly zero
    per = grad_ref.shape[1]
    assert np.all(grad.cpu().numpy().reshape(K, per)[:, -1] == 0.0)


def test_vjp_parity_and_autograd(torch, rid):
    n, widths, K, B = 6, [64, 48], 3, 77
    params = ridgen.xavier_ensemble(2 * n, widths, K, 7, bias_std=0.1)
    s = ridgen.f32(ridgen.torus_samples(B, n, 4))
    rho = ridgen.f32(np.random.default_rng(5).normal(size=(B, K, n)))
    E = rid.Ensemble(n, widths, K, params)
    grad = rid.mf_grad(E, _dev(torch, s), _dev(torch, rho))
    models = ridgen.unpack_params(params, 2 * n, widths, K)
    ref = np.stack([O.flat_grad(O.mean_force_vjp(m, s.astype(np.float64), rho[:, k, :]))
                    for k, m in enumerate(models)])
    assert _per_member_err(grad.cpu().numpy(), ref) <= GRAD_TOL
    # autograd wrapper: loss = sum(rho * g) -> params.grad equals the VJP
    P = _dev(torch, params).requires_grad_(True)
    g = rid.mean_force(_dev(torch, s), P, E)
    (g * _dev(torch, rho)).sum().backward()
    torch.cuda.synchronize()
    assert torch.equal(P.grad, grad)
    _, g_ref = O.ensemble_mean_force(models, s.astype(np.float64))
    assert O.max_rel_err(g.detach().cpu().numpy(), g_ref) <= 1e-5


def test_autograd_follows_params_tensor(torch, rid):
    """The autograd form evaluates the network its params tensor describes
    (the ensemble was created with other weights and never told), its
    gradient is the oracle's VJP there and agrees with a directional finite
    difference of the loss; an ensemble with a dropout rate is refused."""
    n, widths, K, B = 6, [64, 48], 3, 77
    p1 = ridgen.xavier_ensemble(2 * n, widths, K, 7, bias_std=0.1)
    p2 = ridgen.xavier_ensemble(2 * n, widths, K, 8, bias_std=0.1)
    s = ridgen.f32(ridgen.torus_samples(B, n, 4))
    rho = ridgen.f32(np.random.default_rng(5).normal(size=(B, K, n)))
    E = rid.Ensemble(n, widths, K, p1)
    sd, rd = _dev(torch, s), _dev(torch, rho)
    P = _dev(torch, p2).requires_grad_(True)
    g = rid.mean_force(sd, P, E)
    (g * rd).sum().backward()
    torch.cuda.synchronize()
    models2 = ridgen.unpack_params(p2, 2 * n, widths, K)
    ref = np.stack([O.flat_grad(O.mean_force_vjp(m, s.astype(np.float64), rho[:, k, :]))
                    for k, m in enumerate(models2)])
    _, g_ref = O.ensemble_mean_force(models2, s.astype(np.float64))
    assert O.max_rel_err(g.detach().cpu().numpy(), g_ref) <= 1e-5
    assert _per_member_err(P.grad.cpu().numpy(), ref) <= GRAD_TOL
    # central difference of L(P) = sum rho . g(P) along the unit gradient
    d = P.grad / P.grad.norm()
    h = 1e-2
    with torch.no_grad():
        lp = (rid.mean_force(sd, P + h * d, E) * rd).sum().item()
        lm = (rid.mean_force(sd, P - h * d, E) * rd).sum().item()
    fd, exact = (lp - lm) / (2 * h), (P.grad * d).sum().item()
    print(f"directional derivative: FD {fd:.6e} autograd {exact:.6e}")
    assert abs(fd - exact) <= 1e-3 * abs(exact)
    E.set_dropout(0.1, 1)
    with pytest.raises(ValueError):
        rid.mean_force(sd, P, E)


def test_train_steps_follow_oracle(torch, rid):
    n, widths, K, B = 38, [256] * 4, 4, 4096
    params = ridgen.xavier_ensemble(2 * n, widths, K, 1000)
    s_all, F_all, _ = ridgen.mf_training_set(3 * B, n)
    E = rid.Ensemble(n, widths, K, params)
    models = ridgen.unpack_params(params, 2 * n, widths, K)
    states = [(np.zeros(O.flat_model(m).size), np.zeros(O.flat_model(m).size), 0) for m in models]
    for step in range(3):
        sl = slice(step * B, (step + 1) * B)
        lr = O.lr_at(step)
        loss = rid.mf_train_step(E, _dev(torch, s_all[sl]), _dev(torch, F_all[sl]), lr)
        models, states, loss_ref = O.train_step(models, s_all[sl], F_all[sl], states, lr)
        torch.cuda.synchronize()
        lerr = np.max(np.abs(loss.cpu().numpy() - loss_ref) / loss_ref)
        print(f"step {step}: loss {loss.cpu().numpy()} rel err {lerr:.2e}")
        assert lerr <= 1e-4
    assert E.step == 3
    got = E.get_params().astype(np.float64).reshape(K, -1)
    ref = np.stack([O.flat_model(m) for m in models])
    # Adam moves every weight by about lr per step; entries whose gradient is
    # near zero may take the other sign, so compare against the step size.
    step_scale = 3 * O.INIT_LR
    d = np.abs(got - ref)
    assert np.quantile(d, 0.99) <= 0.05 * step_scale
    assert d.max() <= 2.5 * step_scale


def test_trained_ensemble_is_used_by_the_bias_path(torch, rid):
    sys_ = ridgen.system_dipeptide()
    n, widths, K = sys_.n_cv, [32, 32], 2
    params = ridgen.xavier_ensemble(2 * n, widths, K, 3, bias_std=0.1)
    E = rid.Ensemble(n, widths, K, params)
    S = rid.System(sys_.n_atoms, sys_.quads)
    s, F, _ = ridgen.mf_training_set(256, n)
    for step in range(5):
        rid.mf_train_step(E, _dev(torch, s), _dev(torch, F), 1e-2)
    new = E.get_params()
    assert not np.array_equal(new, params)
    pos = ridgen.f32(ridgen.chain_coords(sys_, 16, 2))
    out = rid.bias_force(S, E, _dev(torch, pos), 2.0, 3.0)
    torch.cuda.synchronize()
    ref = O.bias_force(pos.astype(np.float64), sys_.quads,
                       ridgen.unpack_params(new, 2 * n, widths, K), 2.0, 3.0)
    assert O.max_rel_err(out["F"].cpu().numpy(), ref["F"]) <= 1e-5


def test_training_is_deterministic(torch, rid):
    n, widths, K, B = 38, [256] * 4, 4, 2048
    params = ridgen.xavier_ensemble(2 * n, widths, K, 11)
    s, F, _ = ridgen.mf_training_set(B, n)
    S_, F_ = _dev(torch, s), _dev(torch, F)
    out = []
    for _ in range(2):
        E = rid.Ensemble(n, widths, K, params)
        for step in range(2):
            rid.mf_train_step(E, S_, F_, 1e-3)
        out.append(E.get_params())
    assert np.array_equal(out[0], out[1])


DROP_SEED = 0xABCDEF0123


def _grad_ref_dropout(params, n, widths, K, s, F, rate, step):
    models = ridgen.unpack_params(params, 2 * n, widths, K)
    losses, grads = [], []
    for k, m in enumerate(models):
        sc = O.dropout_scales(len(s), widths, rate, DROP_SEED, step, k)
        loss, g = O.train_loss_grad(m, s.astype(np.float64), F.astype(np.float64), sc)
        losses.append(loss)
        grads.append(O.flat_grad(g))
    return np.array(losses), np.stack(grads)


@pytest.mark.parametrize("n,widths,K,B", [(38, [256] * 4, 4, 4096), (7, [100, 33, 70], 3, 257)])
def test_loss_grad_parity_with_dropout(torch, rid, n, widths, K, B):
    params = ridgen.xavier_ensemble(2 * n, widths, K, 1000, bias_std=0.1)
    s, F, _ = ridgen.mf_training_set(B, n)
    E = rid.Ensemble(n, widths, K, params)
    E.set_dropout(0.2, DROP_SEED)
    loss, grad = rid.mf_loss_grad(E, _dev(torch, s), _dev(torch, F))
    torch.cuda.synchronize()
    loss_ref, grad_ref = _grad_ref_dropout(params, n, widths, K, s, F, 0.2, 0)
    lerr = np.max(np.abs(loss.cpu().numpy() - loss_ref) / loss_ref)
    gerr = _per_member_err(grad.cpu().numpy(), grad_ref)
    print(f"dropout 0.2 n={n} widths={widths}: loss rel err {lerr:.2e}, grad err {gerr:.2e}")
    assert lerr <= 1e-5 and gerr <= GRAD_TOL
    # the masks matter: the plain gradient is far outside the tolerance
    _, plain = _grad_ref(params, n, widths, K, s, F)
    assert _per_member_err(plain, grad_ref) > 100 * GRAD_TOL


def test_dropout_masks_follow_the_step_counter(torch, rid):
    n, widths, K, B = 6, [64, 48], 3, 300
    params = ridgen.xavier_ensemble(2 * n, widths, K, 31, bias_std=0.1)
    s, F, _ = ridgen.mf_training_set(B, n)
    E = rid.Ensemble(n, widths, K, params)
    E.set_dropout(0.3, DROP_SEED)
    rid.mf_train_step(E, _dev(torch, s), _dev(torch, F), 1e-3)
    torch.cuda.synchronize()
    assert E.step == 1
    p1 = E.get_params()
    loss, grad = rid.mf_loss_grad(E, _dev(torch, s), _dev(torch, F))
    torch.cuda.synchronize()
    loss_ref, grad_ref = _grad_ref_dropout(p1, n, widths, K, s, F, 0.3, 1)
    assert np.max(np.abs(loss.cpu().numpy() - loss_ref) / loss_ref) <= 1e-5
    assert _per_member_err(grad.cpu().numpy(), grad_ref) <= GRAD_TOL


def _grad_ref_general(params, n, widths, K, s, F, rate=0.0, step=0, resnet=False, mask=None):
    """Oracle loss and gradient per member, with the training-time dropout
    masks of `step` (rate > 0), residual connections and an angular mask."""
    models = ridgen.unpack_params(params, 2 * n, widths, K)
    losses, grads = [], []
    for k, m in enumerate(models):
        if resnet:
            m = tuple(m[:4]) + (True,)
        sc = O.dropout_scales(len(s), widths, rate, DROP_SEED, step, k) if rate > 0 else None
        loss, g = O.train_loss_grad(m, s.astype(np.float64), F.astype(np.float64), sc, mask)
        losses.append(loss)
        grads.append(O.flat_grad(g))
    return np.array(losses), np.stack(grads)


# The general sweeps (separate GEMMs): width 300 pads to 512, beyond the fused
# kernel; residual ensembles of any width; dropout on both.
@pytest.mark.parametrize("n,widths,K,B,rate,resnet", [(5, [300, 40], 2, 100, 0.1, False),
                                                      (6, [256] * 3, 2, 200, 0.0, True),
                                                      (4, [96] * 4, 3, 77, 0.25, True)])
def test_general_sweeps_dropout_and_residual(torch, rid, n, widths, K, B, rate, resnet):
    params = ridgen.xavier_ensemble(2 * n, widths, K, 33, bias_std=0.1)
    s, F, _ = ridgen.mf_training_set(B, n)
    E = rid.Ensemble(n, widths, K, params)
    if resnet:
        E.set_resnet(True)
    E.set_dropout(rate, DROP_SEED)
    loss, grad = rid.mf_loss_grad(E, _dev(torch, s), _dev(torch, F))
    torch.cuda.synchronize()
    loss_ref, grad_ref = _grad_ref_general(params, n, widths, K, s, F, rate, 0, resnet)
    lerr = np.max(np.abs(loss.cpu().numpy() - loss_ref) / loss_ref)
    gerr = _per_member_err(grad.cpu().numpy(), grad_ref)
    print(f"rate {rate} resnet {resnet} widths={widths}: loss rel err {lerr:.2e}, "
          f"grad err {gerr:.2e}", flush=True)
    assert lerr <= 1e-5 and gerr <= GRAD_TOL
    # the masks and the skips matter: the plain gradient is far off
    _, plain = _grad_ref(params, n, widths, K, s, F)
    assert _per_member_err(plain, grad_ref) > 100 * GRAD_TOL
    with pytest.raises(rid.RidError):
        E.set_dropout(1.0, 1)


def test_paper_training_config(torch, rid):
    """The paper's Train example for chignolin: 4 members of 4 hidden layers
    of 300 units (padded to 512), residual connections, dropout 0.1, batch
    128, init_lr / decay as printed, on the example's 18 torsion CVs: the
    gradient against the oracle, then three Adam steps (each with its own
    dropout masks) against the oracle's."""
    import json
    import os
    cfg = {k: v["value"] for k, v in json.load(open(os.path.join(
        os.path.dirname(__file__), "golden", "paper_config.json"))).items() if k != "_about"}
    n, widths, K = cfg["chignolin_angular_mask_len"], cfg["neurons"], cfg["numb_models"]
    B, rate = cfg["batch_size"], cfg["drop_out_rate"]
    assert cfg["resnet"] is True and (n, widths, K, B, rate) == (18, [300] * 4, 4, 128, 0.1)
    params = ridgen.xavier_ensemble(2 * n, widths, K, 1000, bias_std=0.1)
    s_all, F_all, _ = ridgen.mf_training_set(3 * B, n)
    E = rid.Ensemble(n, widths, K, params)
    E.set_resnet(True)
    E.set_dropout(rate, DROP_SEED)
    loss, grad = rid.mf_loss_grad(E, _dev(torch, s_all[:B]), _dev(torch, F_all[:B]))
    torch.cuda.synchronize()
    loss_ref, grad_ref = _grad_ref_general(params, n, widths, K, s_all[:B], F_all[:B], rate, 0,
                                           True)
    gerr = _per_member_err(grad.cpu().numpy(), grad_ref)
    print(f"paper config: loss {loss.cpu().numpy()}, grad err {gerr:.2e}", flush=True)
    assert np.max(np.abs(loss.cpu().numpy() - loss_ref) / loss_ref) <= 1e-5
    assert gerr <= GRAD_TOL
    models = [tuple(m[:4]) + (True,) for m in ridgen.unpack_params(params, 2 * n, widths, K)]
    states = [(np.zeros(O.flat_model(m).size), np.zeros(O.flat_model(m).size), 0) for m in models]
    for step in range(3):
        sl = slice(step * B, (step + 1) * B)
        lr = O.lr_at(step, cfg["init_lr"], cfg["decay_steps"], cfg["decay_rate"])
        loss = rid.mf_train_step(E, _dev(torch, s_all[sl]), _dev(torch, F_all[sl]), lr)
        models, states, loss_ref = O.train_step(models, s_all[sl], F_all[sl], states, lr,
                                                dropout=(rate, DROP_SEED))
        torch.cuda.synchronize()
        lerr = np.max(np.abs(loss.cpu().numpy() - loss_ref) / loss_ref)
        print(f"step {step}: loss rel err {lerr:.2e}", flush=True)
        assert lerr <= 1e-4
    assert E.step == 3
    got = E.get_params().astype(np.float64).reshape(K, -1)
    ref = np.stack([O.flat_model(m) for m in models])
    step_scale = 3 * O.INIT_LR
    d = np.abs(got - ref)
    assert np.quantile(d, 0.99) <= 0.05 * step_scale
    assert d.max() <= 2.5 * step_scale


@pytest.mark.parametrize("n,widths,K", [(38, [256] * 4, 4), (5, [300, 40], 2)])
def test_loss_grad_single_sample(torch, rid, n, widths, K):
    """A batch of one sample (two stacked rows in every weight-gradient
    contraction) on the fused and on the general sweeps."""
    params = ridgen.xavier_ensemble(2 * n, widths, K, 81, bias_std=0.1)
    s, F, _ = ridgen.mf_training_set(1, n)
    E = rid.Ensemble(n, widths, K, params)
    loss, grad = rid.mf_loss_grad(E, _dev(torch, s), _dev(torch, F))
    torch.cuda.synchronize()
    loss_ref, grad_ref = _grad_ref_general(params, n, widths, K, s, F)
    assert np.max(np.abs(loss.cpu().numpy() - loss_ref) / loss_ref) <= 1e-5
    assert _per_member_err(grad.cpu().numpy(), grad_ref) <= GRAD_TOL


def test_general_sweeps_follow_new_parameters(torch, rid):
    """The general sweeps (here: a layer wider than 256) read the layer
    weights from an aligned copy of the masters (the 70 x 33 matrix is not a
    whole number of 16-byte rows): after set_params, and after a training
    step, the gradient is the oracle's for the parameters the ensemble now
    holds."""
    n, widths, K, B = 5, [300, 33, 70], 2, 64
    pa = ridgen.xavier_ensemble(2 * n, widths, K, 71, bias_std=0.1)
    pb = ridgen.xavier_ensemble(2 * n, widths, K, 72, bias_std=0.1)
    s, F, _ = ridgen.mf_training_set(B, n)
    E = rid.Ensemble(n, widths, K, pa)
    for params in (pa, pb):
        E.set_params(params)
        loss, grad = rid.mf_loss_grad(E, _dev(torch, s), _dev(torch, F))
        torch.cuda.synchronize()
        loss_ref, grad_ref = _grad_ref_general(params, n, widths, K, s, F)
        assert np.max(np.abs(loss.cpu().numpy() - loss_ref) / loss_ref) <= 1e-5
        assert _per_member_err(grad.cpu().numpy(), grad_ref) <= GRAD_TOL
    rid.mf_train_step(E, _dev(torch, s), _dev(torch, F), 1e-3)
    pc = E.get_params()
    loss, grad = rid.mf_loss_grad(E, _dev(torch, s), _dev(torch, F))
    torch.cuda.synchronize()
    loss_ref, grad_ref = _grad_ref_general(pc, n, widths, K, s, F)
    assert np.max(np.abs(loss.cpu().numpy() - loss_ref) / loss_ref) <= 1e-5
    assert _per_member_err(grad.cpu().numpy(), grad_ref) <= GRAD_TOL


def test_masked_training_parity(torch, rid):
    """Training on the mixed table (38 torsions, 6 distances): raw CVs enter
    as (s, 0) and their mean force is dA/dx_i; residual and plain."""
    base = ridgen.with_distances(ridgen.system_peptide20(), 6)
    n, widths, K, B = base.n_cv, [64, 64], 3, 300
    m = base.mask.astype(bool)
    rng = np.random.default_rng(41)
    s = ridgen.f32(np.where(m, rng.uniform(-np.pi, np.pi, (B, n)), rng.uniform(0.3, 1.5, (B, n))))
    F = ridgen.f32(rng.normal(0.0, 2.0, (B, n)))
    params = ridgen.xavier_ensemble(2 * n, widths, K, 43, bias_std=0.1)
    for resnet in (False, True):
        E = rid.Ensemble(n, widths, K, params)
        E.set_angular_mask(base.mask)
        if resnet:
            E.set_resnet(True)
        loss, grad = rid.mf_loss_grad(E, _dev(torch, s), _dev(torch, F))
        torch.cuda.synchronize()
        loss_ref, grad_ref = _grad_ref_general(params, n, widths, K, s, F, resnet=resnet,
                                               mask=base.mask)
        gerr = _per_member_err(grad.cpu().numpy(), grad_ref)
        print(f"masked resnet={resnet}: grad err {gerr:.2e}", flush=True)
        assert np.max(np.abs(loss.cpu().numpy() - loss_ref) / loss_ref) <= 1e-5
        assert gerr <= GRAD_TOL
    _, unmasked = _grad_ref_general(params, n, widths, K, s, F)
    assert _per_member_err(unmasked, grad_ref) > 100 * GRAD_TOL


def test_large_batch_runs_in_chunks_under_the_budget(torch, rid):
    """Batch 16384 on the training shape (38 CVs, 4 x [256 x 4]): one pass
    over the whole batch would hold ~1.1 GB of activations, above the
    default 512 MiB budget, so the step runs in three chunks of rows.  Loss
    and gradient match the oracle over the whole batch, the device memory
    the call takes stays under the budget, and a second call is bitwise
    equal to the first."""
    n, widths, K, B = 38, [256] * 4, 4, 16384
    params = ridgen.xavier_ensemble(2 * n, widths, K, 1000, bias_std=0.1)
    s, F, _ = ridgen.mf_training_set(B, n)
    E = rid.Ensemble(n, widths, K, params)
    S_, F_ = _dev(torch, s), _dev(torch, F)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    loss, grad = rid.mf_loss_grad(E, S_, F_)
    torch.cuda.synchronize()
    # the training workspace, plus torch's block for the two outputs
    taken = free0 - torch.cuda.mem_get_info()[0]
    print(f"B={B}: device memory taken by the call {taken / 2**20:.0f} MiB", flush=True)
    assert taken <= (512 << 20)
    l1, g1 = loss.cpu().numpy(), grad.cpu().numpy()
    loss_ref, grad_ref = _grad_ref(params, n, widths, K, s, F)
    lerr = np.max(np.abs(l1 - loss_ref) / loss_ref)
    gerr = _per_member_err(g1, grad_ref)
    print(f"B={B} chunked: loss rel err {lerr:.2e}, grad err {gerr:.2e}", flush=True)
    assert lerr <= 1e-5 and gerr <= GRAD_TOL
    l2, g2 = rid.mf_loss_grad(E, S_, F_)
    torch.cuda.synchronize()
    assert np.array_equal(l2.cpu().numpy(), l1) and np.array_equal(g2.cpu().numpy(), g1)


# (n, widths, K, B, dropout rate, resnet): the fused sweeps, and the general
# sweeps with residual layers and dropout, on a ragged batch
CHUNK_CASES = [(38, [256] * 4, 4, 1000, 0.0, False), (38, [256] * 4, 4, 1000, 0.2, False),
               (5, [300, 40], 2, 333, 0.1, False), (6, [96] * 3, 3, 500, 0.25, True)]


@pytest.mark.parametrize("n,widths,K,B,rate,resnet", CHUNK_CASES)
def test_chunked_passes_equal_one_pass(torch, rid, n, widths, K, B, rate, resnet):
    """A budget too small for any pass forces 64-row chunks (the last one
    ragged): the loss equals the one-pass loss, the gradient differs from it
    only by the order of the chunk sums, the dropout masks stay those of the
    whole batch (the oracle's), and so does the upstream-gradient form."""
    params = ridgen.xavier_ensemble(2 * n, widths, K, 51, bias_std=0.1)
    s, F, _ = ridgen.mf_training_set(B, n)
    rho = ridgen.f32(np.random.default_rng(52).normal(size=(B, K, n)))
    S_, F_, R_ = _dev(torch, s), _dev(torch, F), _dev(torch, rho)
    out = []
    for budget in (0, 1):
        E = rid.Ensemble(n, widths, K, params)
        if resnet:
            E.set_resnet(True)
        E.set_dropout(rate, DROP_SEED)
        E.set_train_budget(budget)
        loss, grad = rid.mf_loss_grad(E, S_, F_)
        vjp = rid.mf_grad(E, S_, R_)
        torch.cuda.synchronize()
        out.append((loss.cpu().numpy(), grad.cpu().numpy(), vjp.cpu().numpy()))
    (l1, g1, v1), (lc, gc, vc) = out
    assert np.max(np.abs(lc - l1) / l1) <= 1e-6
    assert _per_member_err(gc, g1.astype(np.float64).reshape(K, -1)) <= 1e-5
    assert _per_member_err(vc, v1.astype(np.float64).reshape(K, -1)) <= 1e-5
    loss_ref, grad_ref = _grad_ref_general(params, n, widths, K, s, F, rate, 0, resnet)
    gerr = _per_member_err(gc, grad_ref)
    print(f"chunked {widths} rate {rate} resnet {resnet}: loss rel err "
          f"{np.max(np.abs(lc - loss_ref) / loss_ref):.2e}, grad err {gerr:.2e}", flush=True)
    assert np.max(np.abs(lc - loss_ref) / loss_ref) <= 1e-5 and gerr <= GRAD_TOL
