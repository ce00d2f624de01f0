"""GPU parity of the residual MLP form (the `resnet` training setting) against
the FP64 oracle, through the C ABI: bias force, model deviation, the
paper's own network shape, the switch back to the plain form, and the calls
that refuse residual ensembles."""
import numpy as np
import pytest

import ridgen
from oracle import rid_oracle as O
from tests.gpu_common import FP32_TOL, assert_forces, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def rid():
    import paper_2408_14070_amd as r
    r.lib()
    return r


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _res_models(params, n_cv, widths, K):
    return [m + (True,) for m in ridgen.unpack_params(params, 2 * n_cv, widths, K)]


def _bias_ref(sys_, pos, models, e0, e1):
    return O.bias_force(pos.astype(np.float64), sys_.quads, models, e0, e1)


# padded widths 64, 128, 256 (16 waves, the headline kernel's shape) and 512;
# 300 x 4 with K = 4 is the chignolin example's network (pads to 512);
# B = 1000 spans many 16-walker tiles and ends in a ragged one
@pytest.mark.parametrize("kind,widths,K,B", [("peptide20", [256] * 4, 4, 1000),
                                             ("peptide20", [300] * 4, 4, 203),
                                             ("dipeptide", [64] * 6, 5, 77),
                                             ("dipeptide", [100] * 2, 3, 40),
                                             ("peptide61", [512] * 3, 2, 33)])
def test_resnet_bias_force_parity(torch, rid, kind, widths, K, B):
    sys_, pos, params, widths, K = workload(kind, B, seed=21, K=K, widths=widths,
                                            bias_std=0.1)
    print(f"resnet bias force: {kind} {widths} K={K} B={B}", flush=True)
    S = rid.System(sys_.n_atoms, sys_.quads)
    E = rid.Ensemble(sys_.n_cv, widths, K, params)
    E.set_resnet(True)
    # the switch does not depend on the network form (its parity is covered
    # with the plain form): the trust levels here keep sigma = 1, so the
    # force is the whole ensemble-mean force
    ref = _bias_ref(sys_, pos, _res_models(params, sys_.n_cv, widths, K), 1e9, 2e9)
    out = rid.bias_force(S, E, _dev(torch, pos), 1e9, 2e9)
    torch.cuda.synchronize()
    eps = out["eps"].cpu().numpy()
    scale = np.abs(ref["g"]).reshape(B, -1).max(axis=1)
    assert np.max(np.abs(eps - ref["eps"]) / scale) <= FP32_TOL
    assert np.all(out["sigma"].cpu().numpy() == 1.0)
    assert_forces(out["F"].cpu().numpy(), ref["F"], FP32_TOL, f"resnet {widths}x{K} F")
    E_ref = ref["E"]
    assert np.max(np.abs(out["E"].cpu().numpy() - E_ref)) <= FP32_TOL * max(1.0, np.abs(E_ref).max())


def test_resnet_changes_the_result(torch, rid):
    # the residual form is a different function: the same parameters give
    # other forces with the skip on, and the plain ones again once it is off
    sys_, pos, params, widths, K = workload("peptide20", 64, seed=22, bias_std=0.1)
    S = rid.System(sys_.n_atoms, sys_.quads)
    E = rid.Ensemble(sys_.n_cv, widths, K, params)
    plain = rid.bias_force(S, E, _dev(torch, pos), 1e9, 2e9)["F"].cpu().numpy()
    E.set_resnet(True)
    res = rid.bias_force(S, E, _dev(torch, pos), 1e9, 2e9)["F"].cpu().numpy()
    E.set_resnet(False)
    again = rid.bias_force(S, E, _dev(torch, pos), 1e9, 2e9)["F"].cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(plain, again)
    assert O.max_rel_err(res, plain) > 1e-2


def test_resnet_model_dev_parity(torch, rid):
    n, widths, K, B = 38, [256] * 4, 4, 1024
    params = ridgen.xavier_ensemble(2 * n, widths, K, 1003, bias_std=0.1)
    s = ridgen.f32(ridgen.torus_samples(B, n, seed=8))
    E = rid.Ensemble(n, widths, K, params)
    E.set_resnet(True)
    eps, gbar, A, g = rid.model_dev(E, _dev(torch, s))
    torch.cuda.synchronize()
    A_ref, g_ref = O.ensemble_mean_force(_res_models(params, n, widths, K), s.astype(np.float64))
    gbar_ref, eps_ref = O.model_deviation(g_ref)
    assert_forces(g.cpu().numpy(), g_ref, FP32_TOL, "resnet g")
    assert_forces(A.cpu().numpy(), A_ref, FP32_TOL, "resnet A")
    scale = np.abs(g_ref).reshape(B, -1).max(axis=1)
    assert np.max(np.abs(eps.cpu().numpy() - eps_ref) / scale) <= FP32_TOL


def test_plain_width_300_network(torch, rid):
    # a width that is not a multiple of 128 pads to the next kernel width
    sys_, pos, params, widths, K = workload("peptide20", 50, seed=23, K=4, widths=[300] * 4,
                                            bias_std=0.1)
    S = rid.System(sys_.n_atoms, sys_.quads)
    E = rid.Ensemble(sys_.n_cv, widths, K, params)
    models = ridgen.unpack_params(params, 2 * sys_.n_cv, widths, K)
    ref = _bias_ref(sys_, pos, models, 1e9, 2e9)
    out = rid.bias_force(S, E, _dev(torch, pos), 1e9, 2e9)
    torch.cuda.synchronize()
    assert_forces(out["F"].cpu().numpy(), ref["F"], FP32_TOL, "plain 300x4 F")


def test_resnet_refusals(torch, rid):
    sys_, pos, params, widths, K = workload("dipeptide", 16, seed=24, K=2, widths=[64, 64])
    S = rid.System(sys_.n_atoms, sys_.quads)
    E = rid.Ensemble(sys_.n_cv, widths, K, params)
    E.set_resnet(True)
    # (training and conservative switching take residual ensembles: their
    # parity is in tests/test_gpu_train.py and tests/test_gpu_conservative.py)
    # unequal hidden widths, and 16-bit ensembles, are refused
    p2 = ridgen.xavier_ensemble(2 * sys_.n_cv, [64, 32], 2, 5, 0.0)
    E2 = rid.Ensemble(sys_.n_cv, [64, 32], 2, p2)
    with pytest.raises(rid.RidError, match="EINVAL"):
        E2.set_resnet(True)
    E3 = rid.Ensemble(sys_.n_cv, widths, K, params, rid.RID_BF16)
    with pytest.raises(rid.RidError, match="EUNSUPPORTED"):
        E3.set_resnet(True)


def test_resnet_server_matches_direct_call(torch, rid):
    sys_, pos, params, widths, K = workload("peptide20", 37, seed=25, bias_std=0.1)
    S = rid.System(sys_.n_atoms, sys_.quads)
    E = rid.Ensemble(sys_.n_cv, widths, K, params)
    E.set_resnet(True)
    srv = rid.Server(1 << 30, n_streams=2)
    mid = srv.register(S, E, 2.0, 3.0)
    got = srv.wait(srv.submit(mid, pos))
    ref = rid.bias_force(S, E, _dev(torch, pos), 2.0, 3.0)
    torch.cuda.synchronize()
    assert np.array_equal(got["F"], ref["F"].cpu().numpy())
    assert np.array_equal(got["eps"], ref["eps"].cpu().numpy())
    srv.close()
