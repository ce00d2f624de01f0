#!/usr/bin/env python3
"""Benchmark of the RiD neural-bias hot path on one MI355X.

Workload (the metric's configuration): a 20-residue peptide-shaped chain
(200 atoms, 38 backbone torsion CVs), an ensemble of 4 tanh MLPs
76 -> [256 x 4] -> 1 in FP32, 1024 walkers, trust levels 2 / 3.  One step is
one rid_bias_force call: torsion CVs, ensemble forward + input gradient,
model deviation, switch, chain rule to atomic forces.  Inputs are resident
in HBM before the timed region; synthetic seeded data.

The JSON line also carries the precision form (BF16, 8 x [512 x 4],
16384 walkers) and the other rows of the path as extra fields.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import ridgen  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0


def mlp_flops_per_walker(n_cv, widths, K):
    """Algorithmic FLOPs of the ensemble forward + input-gradient sweep:
    2*in*out per layer forward and the same backward, plus the output dot."""
    f = 0
    prev = 2 * n_cv
    for w in widths:
        f += 2 * prev * w
        prev = w
    f += 2 * prev                 # output layer A = wo . h_L
    bwd = 0
    prev = 2 * n_cv
    for w in widths:
        bwd += 2 * prev * w
        prev = w
    return K * (f + bwd)


def build_case(rid, torch, sys_, B, K, widths, prec, seed=1):
    pos = ridgen.f32(ridgen.chain_coords(sys_, B, seed))
    params = ridgen.xavier_ensemble(2 * sys_.n_cv, widths, K, 1000)
    S = rid.System(sys_.n_atoms, sys_.quads)
    E = rid.Ensemble(sys_.n_cv, widths, K, params, prec)
    P = torch.from_numpy(pos).cuda()
    out = dict(
        F=torch.empty((B, sys_.n_atoms, 3), dtype=torch.float32, device="cuda"),
        E=torch.empty(B, dtype=torch.float32, device="cuda"),
        eps=torch.empty(B, dtype=torch.float32, device="cuda"),
        sigma=torch.empty(B, dtype=torch.float32, device="cuda"),
        flags=torch.empty(B, dtype=torch.uint8, device="cuda"),
    )
    return dict(S=S, E=E, P=P, out=out, pos=pos, params=params, sys=sys_, B=B, K=K,
                widths=widths)


def time_bias(rid, torch, case, steps, warmup, eps0=2.0, eps1=3.0):
    S, E, P, out = case["S"], case["E"], case["P"], case["out"]
    for _ in range(warmup):
        rid.bias_force(S, E, P, eps0, eps1, out=out)
    torch.cuda.synchronize()
    rid.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        rid.bias_force(S, E, P, eps0, eps1, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = {}
    for name, kind in (("cv_eval", rid.PROF_CV), ("mlp", rid.PROF_MLP),
                       ("scatter", rid.PROF_SCATTER)):
        tot, cnt = rid.profile_read(kind)
        if cnt:
            kern[name] = tot / cnt
    rid.profile_enable(False)
    return (t1 - t0), kern


def kernel_source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2408_14070_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.startswith("mlp_kernels"):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel_key):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
        rec = t.get(kernel_key)
        if rec and rec.get("source_hash") == kernel_source_hash():
            return rec.get("bytes_per_launch")
    except Exception:
        return None
    return None


def cpu_baseline(case, budget_s=12.0):
    """The FP64 oracle on the same batch, repeated for about budget_s."""
    from oracle import rid_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    sys_ = case["sys"]
    models = ridgen.unpack_params(case["params"], 2 * sys_.n_cv, case["widths"], case["K"])
    pos = case["pos"].astype(np.float64)
    sub = pos[:256]
    reps, walkers = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        O.bias_force(sub, sys_.quads, models, 2.0, 3.0)
        reps += 1
        walkers += len(sub)
    dt = time.perf_counter() - t0
    return {"value": walkers / dt, "unit": "walker-steps/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"{reps} x 256 walkers of the same workload (FP64 numpy oracle, "
                      f"{dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(walkers shard with no exchange; see the design notes). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2408_14070_amd as rid
    rid.lib()
    assert torch.cuda.is_available(), "needs an MI355X"

    sys20 = ridgen.system_peptide20()
    B, K, widths = 1024, 4, [256] * 4
    case = build_case(rid, torch, sys20, B, K, widths, rid.RID_FP32)
    elapsed, kern = time_bias(rid, torch, case, args.steps, args.warmup)
    ms_step = 1e3 * elapsed / args.steps
    value = B * args.steps / elapsed
    flop_launch = mlp_flops_per_walker(sys20.n_cv, widths, K) * B
    mlp_s = kern["mlp"] * 1e-3
    achieved = flop_launch / mlp_s / 1e12
    roof = {"bound": "mfma", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": traffic_for("mlp_fp32_c2"),
            "kernel": "mlp_kernel<F32,256,fused bias> (whole bias path in one launch)",
            "avg_launch_us": kern["mlp"] * 1e3,
            "flop_per_launch": flop_launch}
    rec = {
        "metric": "bias-force walker-steps/s",
        "value": value,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded peptide-shaped chains, Xavier-normal weights)",
        "config": {"workload": "peptide chain 20 residues / 200 atoms / 38 torsion CVs; "
                               "ensemble 4 x [256 x 4] tanh MLP, FP32; 1024 walkers; "
                               "trust levels 2/3",
                   "walkers": B, "n_cv": sys20.n_cv, "n_atoms": sys20.n_atoms,
                   "ensemble": K, "widths": widths, "precision": "fp32"},
        "roofline": roof,
        "kernels_us": {k: v * 1e3 for k, v in kern.items()},
        "latency_us_per_call": ms_step * 1e3,
    }
    if not args.no_extra:
        # precision form: BF16 MFMA, 8 x [512 x 4], 16384 walkers
        Bb, Kb, wb = 16384, 8, [512] * 4
        cb = build_case(rid, torch, sys20, Bb, Kb, wb, rid.RID_BF16)
        steps_b = max(10, args.steps // 10)
        el_b, kern_b = time_bias(rid, torch, cb, steps_b, max(3, args.warmup // 4))
        fl_b = mlp_flops_per_walker(sys20.n_cv, wb, Kb) * Bb
        ach_b = fl_b / (kern_b["mlp"] * 1e-3) / 1e12
        rec["precision_form"] = {
            "workload": "same chain; ensemble 8 x [512 x 4], BF16 MFMA / FP32 accumulate / "
                        "FP64 variance; 16384 walkers",
            "value": Bb * steps_b / el_b, "unit": "walker-steps/s",
            "ms_per_step": 1e3 * el_b / steps_b,
            "roofline": {"bound": "mfma", "achieved": ach_b, "peak": BF16_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": ach_b / BF16_PEAK_TFLOPS,
                         "traffic": traffic_for("mlp_bf16_c3"),
                         "avg_launch_us": kern_b["mlp"] * 1e3, "flop_per_launch": fl_b},
            "kernels_us": {k: v * 1e3 for k, v in kern_b.items()},
        }
        del cb
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
