"""GPU tests of the serving form: continuous batching of requests from three
system classes and two precisions.  Each request's result must be the same
alone (a direct rid_bias_force call on just its walkers) and in the mix,
bitwise; FP32 requests also match the FP64 oracle."""
import threading

import numpy as np
import pytest

import ridgen
from oracle import rid_oracle as O
from tests.gpu_common import FP32_TOL, assert_forces

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


CLASSES = [
    ("dipeptide", ridgen.system_dipeptide, [100, 100, 100]),
    ("peptide20", ridgen.system_peptide20, [256] * 4),
    ("peptide61", ridgen.system_peptide61, [512] * 4),
]


def _models(rid):
    out = []
    for ci, (name, mk, widths) in enumerate(CLASSES):
        sys_ = mk()
        S = rid.System(sys_.n_atoms, sys_.quads)
        for prec in (rid.RID_FP32, rid.RID_BF16):
            K = 8 if (widths[0] == 512 and prec == rid.RID_BF16) else 4
            params = ridgen.xavier_ensemble(2 * sys_.n_cv, widths, K, 1000 + 10 * ci, 0.05)
            E = rid.Ensemble(sys_.n_cv, widths, K, params, prec)
            out.append(dict(sys=sys_, S=S, E=E, params=params, widths=widths, K=K, prec=prec,
                            name=f"{name}-{'fp32' if prec == 0 else 'bf16'}"))
    return out


def _direct(torch, rid, m, pos, e0, e1):
    o = rid.bias_force(m["S"], m["E"], torch.from_numpy(pos).cuda(), e0, e1)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def test_single_request_matches_direct_call(torch, rid):
    ms = _models(rid)
    srv = rid.Server(1 << 30, n_streams=2)
    m = ms[2]
    mid = srv.register(m["S"], m["E"], 2.0, 3.0)
    pos = ridgen.f32(ridgen.chain_coords(m["sys"], 37, 3))
    t = srv.submit(mid, pos)
    got = srv.wait(t)
    ref = _direct(torch, rid, m, pos, 2.0, 3.0)
    assert np.array_equal(got["F"], ref["F"])
    assert np.array_equal(got["eps"], ref["eps"])
    assert np.array_equal(got["E"], ref["E"])
    assert got["latency_us"] > 0
    srv.close()


def test_mixed_stream_is_batch_invariant(torch, rid):
    ms = _models(rid)
    srv = rid.Server(2 << 30, n_streams=4, max_batch_walkers=2048)
    ids = [srv.register(m["S"], m["E"], 2.0, 3.0) for m in ms]
    rng = np.random.default_rng(7)
    reqs = []
    for r in range(90):
        mi = int(rng.integers(0, len(ms)))
        w = int(np.clip(np.floor(np.exp(rng.uniform(0, np.log(257)))), 1, 256))
        pos = ridgen.f32(ridgen.chain_coords(ms[mi]["sys"], w, 100 + r))
        reqs.append((mi, pos))
    results = [None] * len(reqs)

    def client(part):
        # submit everything first so requests of several clients overlap on
        # the device and share batches, then collect
        tickets = [(i, srv.submit(ids[reqs[i][0]], reqs[i][1])) for i in part]
        for i, t in tickets:
            results[i] = srv.wait(t)

    threads = [threading.Thread(target=client, args=(range(k, len(reqs), 4),)) for k in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    st = srv.stats()
    print("serve stats:", st)
    assert st["requests_done"] == len(reqs)
    assert st["batches"] <= len(reqs)
    for i, (mi, pos) in enumerate(reqs):
        ref = _direct(torch, rid, ms[mi], pos, 2.0, 3.0)
        assert np.array_equal(results[i]["F"], ref["F"]), (i, ms[mi]["name"])
        assert np.array_equal(results[i]["sigma"], ref["sigma"])
    # FP32 requests against the oracle (a few)
    checked = 0
    for i, (mi, pos) in enumerate(reqs):
        m = ms[mi]
        if m["prec"] != rid.RID_FP32 or checked >= 4:
            continue
        models = ridgen.unpack_params(m["params"], 2 * m["sys"].n_cv, m["widths"], m["K"])
        ref = O.bias_force(pos.astype(np.float64), m["sys"].quads, models, 2.0, 3.0)
        assert_forces(results[i]["F"], ref["F"], FP32_TOL, f"served {m['name']}")
        checked += 1
    assert checked > 0
    srv.close()


def test_tight_budget_admits_as_memory_frees(torch, rid):
    ms = _models(rid)
    m = ms[4]                       # 1000-atom class, FP32
    srv = rid.Server(8 << 20, n_streams=4, max_batch_walkers=4096)
    mid = srv.register(m["S"], m["E"], 2.0, 3.0)
    poss = [ridgen.f32(ridgen.chain_coords(m["sys"], 200, 40 + i)) for i in range(12)]
    tickets = [srv.submit(mid, p) for p in poss]
    outs = [srv.wait(t) for t in tickets]
    st = srv.stats()
    print("tight budget stats:", st)
    assert st["requests_done"] == 12
    for p, o in zip(poss, outs):
        assert np.array_equal(o["F"], _direct(torch, rid, m, p, 2.0, 3.0)["F"])
    srv.close()


def test_request_larger_than_budget_is_rejected(torch, rid):
    ms = _models(rid)
    m = ms[4]
    srv = rid.Server(2 << 20, n_streams=1)
    mid = srv.register(m["S"], m["E"], 2.0, 3.0)
    with pytest.raises(rid.RidError) as ei:
        srv.submit(mid, ridgen.f32(ridgen.chain_coords(m["sys"], 256, 1)))
    assert ei.value.status == rid.RID_ENOMEM
    srv.close()


def test_fifo_baseline_mode(torch, rid):
    ms = _models(rid)
    srv = rid.Server(1 << 30, fifo=True)
    ids = [srv.register(m["S"], m["E"], 2.0, 3.0) for m in ms[:2]]
    poss = [ridgen.f32(ridgen.chain_coords(ms[i % 2]["sys"], 5 + i, i)) for i in range(6)]
    ts = [srv.submit(ids[i % 2], p) for i, p in enumerate(poss)]
    outs = [srv.wait(t) for t in ts]
    st = srv.stats()
    assert st["batches"] == 6 and st["mean_batch_walkers"] == np.mean([p.shape[0] for p in poss])
    for i, o in enumerate(outs):
        assert np.array_equal(o["F"], _direct(torch, rid, ms[i % 2], poss[i], 2.0, 3.0)["F"])
    srv.close()


def test_completion_is_signalled_without_a_poll_timeout(torch, rid):
    # The completion thread must wake when a batch is launched, not on its
    # idle timeout (2 ms): a 4-walker request's round trip is tens of
    # microseconds of kernels and copies.  The bound leaves a wide margin for
    # a loaded host while staying below the timeout.
    import time
    sys_ = ridgen.system_dipeptide()
    S = rid.System(sys_.n_atoms, sys_.quads)
    E = rid.Ensemble(sys_.n_cv, [100] * 3, 4, ridgen.xavier_ensemble(2 * sys_.n_cv, [100] * 3, 4, 5))
    srv = rid.Server(1 << 30, n_streams=2)
    mid = srv.register(S, E, 2.0, 3.0)
    pos = ridgen.f32(ridgen.chain_coords(sys_, 4, 1))
    srv.wait(srv.submit(mid, pos))
    rt = []
    for _ in range(50):
        t0 = time.perf_counter()
        srv.wait(srv.submit(mid, pos))
        rt.append(time.perf_counter() - t0)
    srv.close()
    med = float(np.median(rt))
    print(f"round trip median {1e6 * med:.0f} us", flush=True)
    assert med < 1e-3


def test_device_requests_in_the_mix_are_batch_invariant(torch, rid):
    """Walker state resident in device memory: every other request is a
    device request (positions read from and forces written to the caller's
    device tensors), mixed with host requests in the same batches; each
    result equals the direct call bit for bit."""
    ms = _models(rid)
    srv = rid.Server(2 << 30, n_streams=4, max_batch_walkers=2048)
    ids = [srv.register(m["S"], m["E"], 2.0, 3.0) for m in ms]
    rng = np.random.default_rng(9)
    reqs = []
    for r in range(80):
        mi = int(rng.integers(0, len(ms)))
        w = int(np.clip(np.floor(np.exp(rng.uniform(0, np.log(257)))), 1, 256))
        reqs.append((mi, ridgen.f32(ridgen.chain_coords(ms[mi]["sys"], w, 300 + r)), r % 2 == 0))
    outs = []
    f = dict(dtype=torch.float32, device="cuda")
    for i, (mi, pos, dev) in enumerate(reqs):
        if dev:
            N, w = ms[mi]["sys"].n_atoms, pos.shape[0]
            o = dict(F=torch.full((w, N, 3), float("nan"), **f), E=torch.empty(w, **f),
                     eps=torch.empty(w, **f), sigma=torch.empty(w, **f))
            outs.append((torch.from_numpy(pos).cuda(), o))
        else:
            outs.append(None)
    torch.cuda.synchronize()                  # inputs in place before the server reads them
    # submitted in one burst, so requests share batches
    tickets = [srv.submit_device(ids[mi], outs[i][0], outs[i][1]) if dev
               else srv.submit(ids[mi], pos) for i, (mi, pos, dev) in enumerate(reqs)]
    results = [srv.wait(t) for t in tickets]
    st = srv.stats()
    assert st["requests_done"] == len(reqs) and st["batches"] < len(reqs)
    for i, (mi, pos, dev) in enumerate(reqs):
        ref = _direct(torch, rid, ms[mi], pos, 2.0, 3.0)
        if dev:
            o = outs[i][1]
            got = {k: o[k].cpu().numpy() for k in ("F", "E", "eps", "sigma")}
        else:
            got = results[i]
        for k in ("F", "E", "eps", "sigma"):
            assert np.array_equal(got[k], ref[k]), (i, ms[mi]["name"], dev, k)
    srv.close()


def test_native_replay_of_an_open_loop_trace(torch, rid):
    """rid_server_replay: a Poisson trace submitted and waited from native
    threads, device requests; every result equals the direct call."""
    ms = _models(rid)[:4]
    srv = rid.Server(2 << 30, n_streams=4, max_batch_walkers=4096)
    ids = [srv.register(m["S"], m["E"], 2.0, 3.0) for m in ms]
    rng = np.random.default_rng(11)
    t, reqs, keep = 0.0, [], []
    f = dict(dtype=torch.float32, device="cuda")
    for r in range(120):
        t += float(rng.exponential(2e-4))
        mi = int(rng.integers(0, len(ms)))
        w = int(np.clip(np.floor(np.exp(rng.uniform(0, np.log(129)))), 1, 128))
        pos = ridgen.f32(ridgen.chain_coords(ms[mi]["sys"], w, 500 + r))
        p = torch.from_numpy(pos).cuda()
        out = dict(F=torch.empty((w, ms[mi]["sys"].n_atoms, 3), **f), eps=torch.empty(w, **f))
        keep.append((mi, pos, out))
        reqs.append(dict(model=ids[mi], arrival_s=t, pos=p, out=out))
    torch.cuda.synchronize()
    lat, lag, wall = srv.replay(reqs)
    print(f"replay: {len(reqs)} requests in {wall * 1e3:.1f} ms, p50 latency "
          f"{np.median(lat):.0f} us, max submit lag {lag.max():.0f} us", flush=True)
    assert np.all(lat > 0) and wall > 0
    for mi, pos, out in keep:
        ref = _direct(torch, rid, ms[mi], pos, 2.0, 3.0)
        assert np.array_equal(out["F"].cpu().numpy(), ref["F"])
        assert np.array_equal(out["eps"].cpu().numpy(), ref["eps"])
    srv.close()
