"""GPU parity of the restrained-MD mean-force labels (FP64 on the device)
against the oracle's compensated-sum FP64 estimate."""
import math

import numpy as np
import pytest

import ridgen
from oracle import rid_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def rid():
    import paper_2408_14070_amd as r
    r.lib()
    return r


# (1024, 500, 38) is the benchmarked size, compared in full
@pytest.mark.parametrize("M,T,n", [(64, 500, 38), (7, 123, 5), (3, 10, 1), (16, 2000, 120),
                                   (1024, 500, 38)])
def test_label_parity(torch, rid, M, T, n):
    traj, s0, _ = ridgen.restrained_traj(M, T, n, 500.0, seed=M + T)
    mask = np.ones(n, np.uint8)
    if n > 2:
        mask[1] = 0
    kappa = np.full(n, 500.0, np.float32)
    F, se, keep = rid.mf_label(torch.from_numpy(traj).cuda(), torch.from_numpy(s0).cuda(),
                               kappa, mask, std_threshold=1.5)
    torch.cuda.synchronize()
    Fr, SEr, keepr = O.mf_label(traj, s0, kappa, mask, 1.5)
    F, se = F.cpu().numpy(), se.cpu().numpy()
    assert np.max(np.abs(F - Fr) / np.maximum(np.abs(Fr), 1.0)) <= 1e-12
    assert np.max(np.abs(se - SEr) / np.maximum(np.abs(SEr), 1e-3)) <= 1e-9
    assert np.array_equal(keep.cpu().numpy(), keepr)


def test_label_wrap_edge(torch, rid):
    traj = np.full((1, 10, 1), np.float32(-math.pi + 0.01), np.float32)
    s0 = np.full((1, 1), np.float32(math.pi - 0.01), np.float32)
    F, se, keep = rid.mf_label(torch.from_numpy(traj).cuda(), torch.from_numpy(s0).cuda(),
                               [500.0], None, 5.0)
    torch.cuda.synchronize()
    Fr, _, _ = O.mf_label(traj, s0, np.array([500.0]), np.array([1]), 5.0)
    assert abs(F.item() - Fr[0, 0]) <= 1e-12 * abs(Fr[0, 0])
    assert keep.item() == 1


@pytest.mark.parametrize("M,T,n", [(5, 500, 38), (3, 257, 3)])
def test_label_unaligned_slab(torch, rid, M, T, n):
    """A trajectory that does not start on 16 bytes gives the same bits as
    an aligned copy of it."""
    traj, s0, _ = ridgen.restrained_traj(M, T, n, 500.0, seed=7 * T + n)
    kappa = np.full(n, 500.0, np.float32)
    t = torch.from_numpy(traj).cuda()
    buf = torch.zeros(M * T * n + 1, dtype=torch.float32, device="cuda")
    buf[1:] = t.reshape(-1)
    tu = buf[1:].view(M, T, n)
    assert tu.data_ptr() % 16 != 0
    s0d = torch.from_numpy(s0).cuda()
    Fa, sea, ka = rid.mf_label(t, s0d, kappa, None, 1.5)
    Fu, seu, ku = rid.mf_label(tu, s0d, kappa, None, 1.5)
    torch.cuda.synchronize()
    assert torch.equal(Fa, Fu) and torch.equal(sea, seu) and torch.equal(ka, ku)
    Fr, _, _ = O.mf_label(traj, s0, kappa, np.ones(n, np.uint8), 1.5)
    assert np.max(np.abs(Fu.cpu().numpy() - Fr) / np.maximum(np.abs(Fr), 1.0)) <= 1e-12
