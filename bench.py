#!/usr/bin/env python3
"""Benchmark of the RiD neural-bias hot path on one MI355X.

Headline (the metric's configuration): a 20-residue peptide-shaped chain
(200 atoms, 38 backbone torsion CVs), an ensemble of 4 tanh MLPs
76 -> [256 x 4] -> 1 in FP32, 1024 walkers, trust levels 2 / 3.  One step is
one rid_bias_force call: torsion CVs, ensemble forward + input gradient,
model deviation, switch, chain rule to atomic forces.  Inputs are resident
in HBM before the timed region; synthetic seeded data.

The same JSON line carries the other rows of the path as extra fields:
the 16-bit precision forms (8 x [512 x 4], 16384 walkers, BF16 and FP16),
the mean-force training step (4 x [256 x 4], batch 4096), the
restrained-trajectory label reduction, and the serving form (p50/p99
latency and throughput of a Poisson request stream against the one-at-a-
time FP32 baseline).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import ridgen  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0     # dense; FP16 has the same dense peak


def log(msg):
    """Progress on stderr; stdout carries only the JSON line."""
    print(f"# {msg}", file=sys.stderr, flush=True)


def layer_flops(n_cv, widths):
    """2 * in * out summed over the hidden layers."""
    f, prev = 0, 2 * n_cv
    for w in widths:
        f += 2 * prev * w
        prev = w
    return f


def mlp_flops_per_walker(n_cv, widths, K):
    """Algorithmic FLOPs of the ensemble forward + input-gradient sweep:
    2*in*out per layer forward and the same backward, plus the output dot."""
    return K * (2 * layer_flops(n_cv, widths) + 2 * widths[-1])


def conservative_flops_per_walker(n_cv, widths, K):
    """Algorithmic minimum of conservative switching: the frozen-switch path
    (forward + input-gradient sweep) plus, per member, the tangent of the
    forward sweep and the tangent of the reverse sweep (one layer product
    set each)."""
    return mlp_flops_per_walker(n_cv, widths, K) + K * 2 * layer_flops(n_cv, widths)


def hvp_kernel_flops_per_walker(n_cv, widths, K):
    """What the fused Hessian-vector kernel executes: it recomputes the
    primal forward and reverse sweeps from the encoding next to their
    tangents (4 layer product sets per member)."""
    return K * 4 * layer_flops(n_cv, widths)


def train_flops_per_sample(n_cv, widths, K):
    """Forward, primal backward, tangent forward (3 sweeps), adjoint
    propagation through layers 2..L (2 products each) and the two weight-
    gradient products of every layer."""
    F = layer_flops(n_cv, widths)
    F1 = 2 * (2 * n_cv) * widths[0]
    return K * (3 * F + 2 * (F - F1) + 2 * F + 2 * widths[-1])


def build_case(rid, torch, sys_, B, K, widths, prec, seed=1):
    pos = ridgen.f32(ridgen.chain_coords(sys_, B, seed))
    params = ridgen.xavier_ensemble(2 * sys_.n_cv, widths, K, 1000)
    S = rid.System(sys_.n_atoms, sys_.quads, sys_.mask)
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


def read_kernels(rid, kinds):
    kern = {}
    for name, kind in kinds:
        tot, cnt = rid.profile_read(kind)
        if cnt:
            kern[name] = tot / cnt     # ms per launch
    return kern


EVENT_EVERY = 8      # one bias-force call in this many carries kernel events


def time_bias(rid, torch, case, steps, warmup, eps0=2.0, eps1=3.0):
    """Timed region: `steps` bias-force calls bracketed by device
    synchronisation.  Every EVENT_EVERY-th call runs with the library's
    kernel timing on: each of its kernels carries HIP events that take the
    start and end timestamps from the dispatch, on the launching stream.
    Sampling keeps the events' own launch cost (a few microseconds per call)
    out of the step throughput while still timing launches spread over the
    whole region."""
    S, E, P, out = case["S"], case["E"], case["P"], case["out"]
    for _ in range(warmup):
        rid.bias_force(S, E, P, eps0, eps1, out=out)
    torch.cuda.synchronize()
    rid.profile_enable(True)
    rid.profile_enable(False)
    t0 = time.perf_counter()
    for i in range(steps):
        sample = i % EVENT_EVERY == 0
        if sample:
            rid.profile_enable(True, keep=True)
        rid.bias_force(S, E, P, eps0, eps1, out=out)
        if sample:
            rid.profile_enable(False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = read_kernels(rid, (("cv_eval", rid.PROF_CV), ("mlp", rid.PROF_MLP),
                              ("scatter", rid.PROF_SCATTER)))
    return (t1 - t0), kern


def call_percentiles(rid, torch, case, n=400, eps0=2.0, eps1=3.0):
    """Per-call GPU time of the bias force: n calls, each bracketed by events
    on the stream it runs on (torch's current stream), after the throughput
    region; p10 / p50 / p90 in microseconds."""
    S, E, P, out = case["S"], case["E"], case["P"], case["out"]
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n)]
    for a, b in ev:
        a.record()
        rid.bias_force(S, E, P, eps0, eps1, out=out)
        b.record()
    torch.cuda.synchronize()
    t = np.sort(np.array([a.elapsed_time(b) * 1e3 for a, b in ev]))
    return {"p10": float(np.percentile(t, 10)), "p50": float(np.percentile(t, 50)),
            "p90": float(np.percentile(t, 90)), "calls": n}


def kernel_source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2408_14070_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.startswith("mlp_kernels") or f == "device_common.h":
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def train_source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2408_14070_amd", "csrc")
    for f in ("train_kernels.hip", "mlp_kernels.hip", "device_common.h"):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


# training kernels the counter passes summarize: key, name test
TRAIN_PMC_KEYS = (("train_kernel_4x256_b4096", lambda n: "train_kernel<" in n),
                  ("wgrad_kernel_4x256_b4096", lambda n: "wgrad_kernel" in n))


def pmc_for(kernel_key):
    """Counter figures of one kernel family from the committed rocprofv3
    summary (profiles/pmc.json), if they were taken on the current kernel
    source (else None)."""
    path = os.path.join(ROOT, "profiles", "pmc.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel_key)
        want = (train_source_hash() if kernel_key in dict(TRAIN_PMC_KEYS)
                else kernel_source_hash())
        if rec and rec.get("source_hash") == want:
            return rec
    except Exception:
        return None
    return None


def traffic_for(kernel_key):
    rec = pmc_for(kernel_key)
    return rec.get("bytes_per_launch") if rec else None


def mfma_busy_for(kernel_key):
    rec = pmc_for(kernel_key)
    return rec.get("mfma_busy") if rec else None


PMC_COPY_BYTES = 256 << 20      # bytes read (and written) by the calibration copy
PMC_CASES = (("mlp_fp32_4x256_b1024", "FP32", 1024, 4, [256] * 4),
             ("mlp_bf16_8x512_b16384", "BF16", 16384, 8, [512] * 4),
             ("mlp_fp16_8x512_b16384", "FP16", 16384, 8, [512] * 4),
             ("mlp_bf16_all_8x512_b16384", "BF16_ALL", 16384, 8, [512] * 4),
             ("mlp_fp32_8x512_b16384", "FP32", 16384, 8, [512] * 4))


def pmc_workload(rid, torch, reps=3):
    """A short program for the rocprofv3 counter passes: a plain elementwise
    copy of known size (y = x * 1, reads and writes PMC_COPY_BYTES), then the
    bias path on the 200-atom chain for each PMC_CASES entry (the headline
    FP32 ensemble at 1024 walkers; the precision form's shape at 16384
    walkers in each arithmetic), `reps` launches each; then training steps
    of the differentiation form (4 x [256 x 4], batch 4096) after as many
    untimed ones."""
    x = torch.ones(PMC_COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    del x, y
    sys20 = ridgen.system_peptide20()
    for _, prec, B, K, widths in PMC_CASES:
        c = build_case(rid, torch, sys20, B, K, widths, getattr(rid, "RID_" + prec))
        for _ in range(reps):
            rid.bias_force(c["S"], c["E"], c["P"], 2.0, 3.0, out=c["out"])
        torch.cuda.synchronize()
        del c
    n, widths, K, Bt = 38, [256] * 4, 4, 4096
    s_all, F_all, _ = ridgen.mf_training_set(4 * Bt * reps, n)
    S = torch.from_numpy(s_all).cuda()
    F = torch.from_numpy(F_all).cuda()
    E = rid.Ensemble(n, widths, K, ridgen.xavier_ensemble(2 * n, widths, K, 1000))
    for i in range(2 * reps):
        rid.mf_train_step(E, S[i * Bt:(i + 1) * Bt], F[i * Bt:(i + 1) * Bt],
                          rid.lr_exponential(E.step))
    torch.cuda.synchronize()
    print("pmc workload done", flush=True)


def _demangle(names):
    """Demangled kernel names (c++filt), the others unchanged."""
    import subprocess
    mangled = sorted({n for n in names if n.startswith("_Z")})
    if not mangled:
        return {}
    try:
        r = subprocess.run(["c++filt"], input="\n".join(mangled), capture_output=True, text=True,
                           check=True)
        return dict(zip(mangled, r.stdout.splitlines()))
    except (OSError, subprocess.CalledProcessError):
        return {}


def _read_counters(d):
    """{(kernel name, counter): [value per dispatch]} from one rocprofv3
    --pmc pass: the CSV output, or the counters_collection view of its
    rocpd database."""
    import csv
    import glob
    import sqlite3
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        rows += [(r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"]))
                 for r in csv.DictReader(open(f))]
    for f in glob.glob(os.path.join(d, "**", "*.db"), recursive=True):
        con = sqlite3.connect(f)
        rows += [(k, c, float(v)) for k, c, v in
                 con.execute("select kernel_name, counter_name, value from counters_collection")]
        # each dispatch's duration once, as the pseudo-counter _duration_ns
        rows += [(k, "_duration_ns", float(v)) for k, v in
                 con.execute("select kernel_name, max(duration) from counters_collection "
                             "group by dispatch_id, kernel_name")]
        con.close()
    if not rows:
        raise SystemExit(f"no counter output under {d}")
    dm = _demangle([k for k, _, _ in rows])
    out = {}
    for k, c, v in rows:
        out.setdefault((dm.get(k, k), c), []).append(v)
    return out


def _mlp_signature(name):
    """(formats, (NP, RT, NW, LM), (FROM_POS, GRAD, RES)) of an mlp_kernel
    instance from its demangled or mangled name, or None.  Mangled names
    (the host demangler may not know _Float16): the Plan's first three
    template arguments are rid::(anonymous)::<format> names, written out
    (NS0_<n><name>E) or as substitutions S<k>_; the names met in the argument
    list enter the substitution table after rid, the anonymous namespace,
    mlp_kernel and Plan (indices 0-3), so S<k>_ is the (k - 3)-th of them."""
    import re
    m = re.search(r"mlp_kernel<[^<>]*Plan<([^<>]*)>\s*,\s*(\d+)\s*,\s*(\d+)\s*,\s*(\d+)\s*,"
                  r"\s*(\d+)\s*,\s*(true|false)\s*,\s*(true|false)\s*,\s*(true|false)", name)
    if m:
        fmts = [re.sub(r".*::", "", f.strip()) for f in m.group(1).split(",")][:3]
        ints = tuple(int(m.group(k)) for k in range(2, 6))
        flags = tuple(m.group(k) == "true" for k in range(6, 9))
        return fmts, ints, flags
    tag = "mlp_kernelINS0_4PlanI"
    i = name.find(tag)
    if i < 0:
        return None
    pos, seen, fmts = i + len(tag), [], []
    while len(fmts) < 3:
        m = re.match(r"NS0_(\d+)", name[pos:])
        if m:
            n = int(m.group(1))
            start = pos + m.end()
            fmt = name[start:start + n]
            pos = start + n + 1                  # past the closing E
            seen.append(fmt)
            fmts.append(fmt)
            continue
        m = re.match(r"S(\d*)_", name[pos:])
        if not m:
            return None
        k = int(m.group(1)) + 1 if m.group(1) else 0
        if not 4 <= k < 4 + len(seen):
            return None
        fmts.append(seen[k - 4])
        pos += m.end()
    m = re.search(r"ELi(\d+)ELi(\d+)ELi(\d+)ELi(\d+)ELb([01])ELb([01])ELb([01])E", name[pos:])
    if not m:
        return None
    return (fmts, tuple(int(m.group(k)) for k in range(1, 5)),
            tuple(m.group(k) == "1" for k in range(5, 8)))


def mlp_display(name):
    """A short readable name of an mlp_kernel instance (else None)."""
    sig = _mlp_signature(name)
    if sig is None:
        return None
    fmts, ints, flags = sig
    return ("mlp_kernel<Plan<" + ", ".join(fmts) + ">, " + ", ".join(map(str, ints)) + ", "
            + ", ".join("true" if f else "false" for f in flags) + ">")


def pmc_kernel_key(name):
    """The PMC_CASES key of an mlp_kernel launch from its name: the
    arithmetic plan's three MFMA formats, the padded width and the instance
    the benchmark's bias calls use (1024 walkers: torsions gathered in-kernel;
    16384 walkers: the encoding from memory), with the input gradient and no
    residual connections."""
    sig = _mlp_signature(name)
    if sig is None:
        return None
    fmts, (width, _, _, _), (from_pos, grad, res) = sig
    if not grad or res:
        return None
    plan = {("F32", "F32", "F32"): "fp32", ("F16", "BF16", "F16"): "bf16",
            ("F16", "F16", "F16"): "fp16", ("BF16", "BF16", "BF16"): "bf16_all"}.get(tuple(fmts))
    key = {("fp32", 256, True): "mlp_fp32_4x256_b1024",
           ("bf16", 512, False): "mlp_bf16_8x512_b16384",
           ("fp16", 512, False): "mlp_fp16_8x512_b16384",
           ("bf16_all", 512, False): "mlp_bf16_all_8x512_b16384",
           ("fp32", 512, False): "mlp_fp32_8x512_b16384"}
    return key.get((plan, width, from_pos))


N_CU, N_SIMD, N_XCD = 256, 4, 8


def pmc_summary(out_path, *dirs):
    """Summarize rocprofv3 --pmc passes over --pmc-workload (each pass in
    its own directory) into per-kernel figures:
      bytes_per_launch  FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each
                        scaled by what the counter reads for the calibration
                        copy of known size;
      mfma_busy         SQ_VALU_MFMA_BUSY_CYCLES / (4 SQ_BUSY_CU_CYCLES): the
                        fraction of SIMD cycles, on CUs busy with the kernel,
                        in which the matrix unit worked (the busy-cycle counter
                        sums over all SIMDs: an FP32 16x16x4 MFMA of 2048 FLOP
                        counts 32 cycles; SQ_BUSY_CU_CYCLES sums busy cycles
                        over the 256 CUs);
      mfma_busy_gpu     the same over every SIMD of the chip for the kernel's
                        whole GPU-active time: SQ_VALU_MFMA_BUSY_CYCLES /
                        (GRBM_GUI_ACTIVE / 8 XCDs x 1024 SIMDs) (the GRBM
                        counter sums the 8 XCDs' active cycles);
      mfma_flop         SQ_INSTS_VALU_MFMA_MOPS_* x 512 (the MOPS counters
                        count math operations in units of 512);
      l2_hit            TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum)."""
    table = {}
    for d in dirs:
        table.update(_read_counters(d))

    def mean(name_pred, counter):
        vals = [v for (k, c), vs in table.items() if c == counter and name_pred(k) for v in vs]
        return sum(vals) / len(vals) if vals else None

    def is_copy(name):
        return "MulFunctor" in name or "mul_kernel" in name

    res = {"_source": "rocprofv3 --pmc passes over bench.py --pmc-workload: " + ", ".join(dirs),
           "_formulas": pmc_summary.__doc__}
    cf, cw = mean(is_copy, "FETCH_SIZE"), mean(is_copy, "WRITE_SIZE")
    if cf and cw:
        res["_calibration"] = {"copy_bytes": PMC_COPY_BYTES, "fetch_kib": cf, "write_kib": cw,
                               "fetch_scale": PMC_COPY_BYTES / (cf * 1024.0),
                               "write_scale": PMC_COPY_BYTES / (cw * 1024.0)}
    for key, *_ in PMC_CASES:
        pick = (lambda n, key=key: pmc_kernel_key(n) == key)
        rec = {"source_hash": kernel_source_hash()}
        counters = sorted({c for (k, c) in table if pmc_kernel_key(k) == key})
        if not counters:
            continue
        for c in counters:
            rec[c] = mean(pick, c)
        if "_calibration" in res and "FETCH_SIZE" in rec and "WRITE_SIZE" in rec:
            cal = res["_calibration"]
            rec["fetch_bytes"] = rec["FETCH_SIZE"] * 1024.0 * cal["fetch_scale"]
            rec["write_bytes"] = rec["WRITE_SIZE"] * 1024.0 * cal["write_scale"]
            rec["bytes_per_launch"] = rec["fetch_bytes"] + rec["write_bytes"]
        busy = rec.get("SQ_VALU_MFMA_BUSY_CYCLES")
        if busy is not None and rec.get("SQ_BUSY_CU_CYCLES"):
            rec["mfma_busy"] = busy / (N_SIMD * rec["SQ_BUSY_CU_CYCLES"])
        if busy is not None and rec.get("GRBM_GUI_ACTIVE"):
            rec["mfma_busy_gpu"] = busy / (rec["GRBM_GUI_ACTIVE"] / N_XCD * N_CU * N_SIMD)
        mops = [rec.get(c) for c in ("SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F16",
                                     "SQ_INSTS_VALU_MFMA_MOPS_F32")]
        if any(v is not None for v in mops):
            rec["mfma_flop"] = 512.0 * sum(v or 0.0 for v in mops)
        if rec.get("TCC_HIT_sum") is not None and rec.get("TCC_MISS_sum") is not None:
            tot = rec["TCC_HIT_sum"] + rec["TCC_MISS_sum"]
            rec["l2_hit"] = rec["TCC_HIT_sum"] / tot if tot else None
        res[key] = rec
    # the training step's kernels (bench.py --pmc-workload runs a few steps):
    # MFMA busy as above and the effective clock = busy CU cycles per CU /
    # the dispatch's duration
    for key, pick in TRAIN_PMC_KEYS:
        counters = sorted({c for (k, c) in table if pick(k)})
        if "SQ_VALU_MFMA_BUSY_CYCLES" not in counters:
            continue
        rec = {"source_hash": train_source_hash()}
        for c in counters:
            rec[c] = mean(pick, c)
        if rec.get("SQ_BUSY_CU_CYCLES"):
            rec["mfma_busy"] = rec["SQ_VALU_MFMA_BUSY_CYCLES"] / (N_SIMD * rec["SQ_BUSY_CU_CYCLES"])
            if rec.get("_duration_ns"):
                rec["clock_ghz"] = rec["SQ_BUSY_CU_CYCLES"] / N_CU / rec["_duration_ns"]
        if rec.get("SQ_INSTS_VALU_MFMA_MOPS_F32") is not None:
            rec["mfma_flop"] = 512.0 * rec["SQ_INSTS_VALU_MFMA_MOPS_F32"]
        res[key] = rec
    with open(out_path, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))


def sample_outputs(case, n_sample, seed=0):
    """Host copies of the last bias-force call's outputs for a seeded sample
    of walkers (for the accuracy check of the CPU-baseline leg)."""
    B = case["B"]
    rows = np.sort(np.random.default_rng(seed).choice(B, min(n_sample, B), replace=False))
    o = case["out"]
    return {"rows": rows, "pos": case["pos"][rows], "sys": case["sys"],
            "params": case["params"], "widths": case["widths"], "K": case["K"],
            "F": o["F"].cpu().numpy()[rows], "eps": o["eps"].cpu().numpy()[rows],
            "sigma": o["sigma"].cpu().numpy()[rows]}


def _cpu_info():
    info = {"nproc": os.cpu_count()}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return info


def _time_oracle(O, sys_, models, sub, budget_s):
    reps, walkers = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        O.bias_force(sub, sys_.quads, models, 2.0, 3.0)
        reps += 1
        walkers += len(sub)
    return walkers / (time.perf_counter() - t0), reps


def cpu_baseline(case, samples, budget_s=10.0):
    """CPU-baseline leg: the FP64 oracle timed on the host on a bounded
    sample of the headline workload, with numpy's BLAS threads (the matrix
    products) and with one thread; then, on seeded samples of walkers of
    each benchmarked bias line, the oracle's forces beside the GPU's (max
    normwise per-walker and rms relative force error, eps error).  The
    oracle is test infrastructure: this leg is the only part of the
    benchmark that runs it."""
    from oracle import rid_oracle as O
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threadpool_limits, blas = None, 1
    sys_ = case["sys"]
    models = ridgen.unpack_params(case["params"], 2 * sys_.n_cv, case["widths"], case["K"])
    sub = case["pos"][:256].astype(np.float64)
    v_all, reps = _time_oracle(O, sys_, models, sub, budget_s)
    single = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            v1, reps1 = _time_oracle(O, sys_, models, sub, budget_s / 2)
        single = {"value": v1, "unit": "walker-steps/s", "threads": 1,
                  "sample": f"{reps1} x 256 walkers"}
    acc = {}
    tr = samples.get("training")
    if tr is not None:
        # the training step's loss and weight gradient (double backward) on
        # its benchmarked batch against the oracle's, per member: max
        # |dg| / max |g| over the packed parameters
        mods = ridgen.unpack_params(tr["params"], 2 * tr["n"], tr["widths"], tr["K"])
        g = tr["grad"].reshape(tr["K"], -1).astype(np.float64)
        gerr, lerr = 0.0, 0.0
        for k, m in enumerate(mods):
            lo, go = O.train_loss_grad(m, tr["s"].astype(np.float64), tr["F"].astype(np.float64))
            go = O.flat_grad(go)
            gerr = max(gerr, float(np.max(np.abs(g[k] - go)) / np.max(np.abs(go))))
            lerr = max(lerr, abs(float(tr["loss"][k]) - lo) / lo)
        acc["training_b4096"] = {"samples": int(tr["s"].shape[0]),
                                 "max_rel_grad_err": gerr, "max_rel_loss_err": lerr}
    for name, smp in samples.items():
        if name == "training":
            continue
        sm = smp["sys"]
        mods = ridgen.unpack_params(smp["params"], 2 * sm.n_cv, smp["widths"], smp["K"])
        ref = O.bias_force(smp["pos"].astype(np.float64), sm.quads, mods, 2.0, 3.0)
        acc[name] = {"walkers_sampled": int(len(smp["rows"])),
                     "max_rel_force_err": O.max_rel_err(smp["F"], ref["F"]),
                     "rms_rel_force_err": O.rms_rel_err(smp["F"], ref["F"]),
                     "max_rel_eps_err": float(np.max(np.abs(smp["eps"] - ref["eps"]) / ref["eps"])),
                     "regime_agreement_at_2_3": float(np.mean(
                         O.switch(smp["eps"].astype(np.float64), 2.0, 3.0)[1] == ref["regime"]))}
    return {"value": v_all, "unit": "walker-steps/s", "cores": int(blas),
            "kind": "oracle",
            "sample": f"{reps} x 256 walkers of the headline workload (FP64 numpy oracle; "
                      f"its matrix products use {blas} BLAS threads, the per-CV loops one)",
            "single_thread": single, "host": _cpu_info(),
            "accuracy_vs_oracle": acc}


PRECISION_ARITH = {
    "BF16": "hidden-layer forward GEMMs on BF16 MFMA, first layer and reverse sweep on "
            "FP16 MFMA, FP32 accumulate, FP32 tanh' arithmetic (stored FP16), FP32 switch, "
            "FP64 variance",
    "FP16": "every GEMM on FP16 MFMA, FP32 accumulate, FP32 tanh' arithmetic (stored FP16), "
            "FP32 switch, FP64 variance",
    "BF16_ALL": "every GEMM operand BF16 (the plain BF16 form, for comparison), FP32 "
                "accumulate, tanh' stored BF16, FP32 switch, FP64 variance",
    "FP32": "every GEMM on FP32 MFMA (the FP32 path at the precision form's shape)",
}


def bench_precision(rid, torch, sys20, prec, name, steps, warmup, samples):
    """The precision form's shape (8 x [512 x 4], 16384 walkers) in one
    arithmetic; its sampled outputs go to the CPU-baseline leg's accuracy
    check."""
    Bb, Kb, wb = 16384, 8, [512] * 4
    cb = build_case(rid, torch, sys20, Bb, Kb, wb, prec)
    el, kern = time_bias(rid, torch, cb, steps, warmup)
    call_pct = call_percentiles(rid, torch, cb, n=100)
    samples[name.lower()] = sample_outputs(cb, 128)
    fl = mlp_flops_per_walker(sys20.n_cv, wb, Kb) * Bb
    ach = fl / (kern["mlp"] * 1e-3) / 1e12
    peak = FP32_PEAK_TFLOPS if name == "FP32" else BF16_PEAK_TFLOPS
    return {
        "workload": f"same chain; ensemble 8 x [512 x 4], {PRECISION_ARITH[name]}; 16384 "
                    "walkers (CVs encoded once by cv_eval, then mlp_kernel)",
        "value": Bb * steps / el, "unit": "walker-steps/s", "ms_per_step": 1e3 * el / steps,
        "call_us_percentiles": call_pct,
        "roofline": {"bound": "mfma", "achieved": ach, "peak": peak,
                     "unit": "TFLOP/s", "frac": ach / peak,
                     "traffic": traffic_for(f"mlp_{name.lower()}_8x512_b16384"),
                     "mfma_busy": mfma_busy_for(f"mlp_{name.lower()}_8x512_b16384"),
                     "avg_launch_us": kern["mlp"] * 1e3, "flop_per_launch": fl},
        "kernels_us": {k: v * 1e3 for k, v in kern.items()},
    }


def bench_variants(rid, torch, sys20, steps, warmup):
    """The network and CV variants on the headline shape (1024 walkers,
    4 x [256 x 4] FP32): residual connections, and a mixed table with 6
    distance CVs beside the 38 torsions (encoded once by cv_eval)."""
    B, K, widths = 1024, 4, [256] * 4
    res = {}
    c = build_case(rid, torch, sys20, B, K, widths, rid.RID_FP32)
    c["E"].set_resnet(True)
    el, kern = time_bias(rid, torch, c, steps, warmup)
    fl = mlp_flops_per_walker(sys20.n_cv, widths, K) * B
    ach = fl / (kern["mlp"] * 1e-3) / 1e12
    res["resnet"] = {
        "workload": "headline chain and ensemble with residual connections between the "
                    "hidden layers (h_l = h_{l-1} + tanh(W_l h_{l-1} + b_l), l >= 2)",
        "value": B * steps / el, "unit": "walker-steps/s", "ms_per_step": 1e3 * el / steps,
        "roofline": {"bound": "mfma", "achieved": ach, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": ach / FP32_PEAK_TFLOPS,
                     "avg_launch_us": kern["mlp"] * 1e3, "flop_per_launch": fl},
        "kernels_us": {k: v * 1e3 for k, v in kern.items()},
    }
    mixed = ridgen.with_distances(sys20, 6)
    c = build_case(rid, torch, mixed, B, K, widths, rid.RID_FP32)
    c["E"].set_angular_mask(mixed.mask)
    el, kern = time_bias(rid, torch, c, steps, warmup)
    fl = mlp_flops_per_walker(mixed.n_cv, widths, K) * B
    ach = fl / (kern["mlp"] * 1e-3) / 1e12
    res["distance_cvs"] = {
        "workload": "headline chain with 6 CA-CA distance CVs among its 38 torsions (44 CVs, "
                    "angular mask 0 for the distances), headline ensemble shape",
        "value": B * steps / el, "unit": "walker-steps/s", "ms_per_step": 1e3 * el / steps,
        "roofline": {"bound": "mfma", "achieved": ach, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": ach / FP32_PEAK_TFLOPS,
                     "avg_launch_us": kern["mlp"] * 1e3, "flop_per_launch": fl},
        "kernels_us": {k: v * 1e3 for k, v in kern.items()},
    }
    return res


def bench_training(rid, torch, steps=20, warmup=3, samples=None):
    n, widths, K, B = 38, [256] * 4, 4, 4096
    s_all, F_all, _ = ridgen.mf_training_set(200_000, n)
    S = torch.from_numpy(s_all).cuda()
    F = torch.from_numpy(F_all).cuda()
    E = rid.Ensemble(n, widths, K, ridgen.xavier_ensemble(2 * n, widths, K, 1000))
    perm = torch.from_numpy(np.random.default_rng(6).permutation(200_000)).cuda()
    batches = [(S[perm[i * B:(i + 1) * B]].contiguous(), F[perm[i * B:(i + 1) * B]].contiguous())
               for i in range(steps + warmup)]
    for i in range(warmup):
        rid.mf_train_step(E, *batches[i], rid.lr_exponential(E.step))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    for i in range(steps):
        losses.append(rid.mf_train_step(E, *batches[warmup + i], rid.lr_exponential(E.step)))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if samples is not None:
        # the step's loss and gradient on its last batch at the ensemble's
        # current weights, for the CPU-baseline leg's oracle comparison
        sb, Fb = batches[warmup + steps - 1]
        lg, gg = rid.mf_loss_grad(E, sb, Fb)
        torch.cuda.synchronize()
        samples["training"] = dict(params=E.get_params(), n=n, widths=widths, K=K,
                                   s=sb.cpu().numpy(), F=Fb.cpu().numpy(),
                                   loss=lg.cpu().numpy(), grad=gg.cpu().numpy())
    fl = train_flops_per_sample(n, widths, K) * B
    step_s = (t1 - t0) / steps
    # the same step at 4x the batch: its activations exceed the training
    # budget, so each step runs in chunks of rows
    BL, big_steps = 16384, 4
    big = [(S[perm[i * BL:(i + 1) * BL]].contiguous(), F[perm[i * BL:(i + 1) * BL]].contiguous())
           for i in range(big_steps + 1)]
    rid.mf_train_step(E, *big[0], rid.lr_exponential(E.step))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for i in range(big_steps):
        rid.mf_train_step(E, *big[1 + i], rid.lr_exponential(E.step))
    torch.cuda.synchronize()
    big_s = (time.perf_counter() - t2) / big_steps
    # the paper's own Train example (chignolin: 18 torsion CVs, 4 x [300 x 4],
    # residual connections, dropout 0.1, batch 128): the general sweeps
    pn, pw, pK, pB = 18, [300] * 4, 4, 128
    ps_all, pF_all, _ = ridgen.mf_training_set(pB * 64, pn)
    PS = torch.from_numpy(ps_all).cuda()
    PF = torch.from_numpy(pF_all).cuda()
    PE = rid.Ensemble(pn, pw, pK, ridgen.xavier_ensemble(2 * pn, pw, pK, 1000))
    PE.set_resnet(True)
    PE.set_dropout(0.1, seed=7)
    pb = [(PS[i * pB:(i + 1) * pB], PF[i * pB:(i + 1) * pB]) for i in range(64)]
    for i in range(8):
        rid.mf_train_step(PE, *pb[i], rid.lr_exponential(PE.step))
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for i in range(8, 64):
        rid.mf_train_step(PE, *pb[i], rid.lr_exponential(PE.step))
    torch.cuda.synchronize()
    paper_s = (time.perf_counter() - t3) / 56
    return {
        "workload": "mean-force fitting, 38 CVs, ensemble 4 x [256 x 4], batch 4096 from "
                    "200k resident samples, double backward + Adam, FP32",
        "value": B / step_s, "unit": "samples/s", "ms_per_step": 1e3 * step_s,
        "flop_per_step": fl,
        "achieved_tflops": fl / step_s / 1e12, "frac_fp32_peak": fl / step_s / 1e12 / FP32_PEAK_TFLOPS,
        "loss_first_last": [float(losses[0].mean()), float(losses[-1].mean())],
        # MFMA busy and effective clock of the step's two MFMA kernels, from
        # the committed counter passes when they match the current sources
        "counters": {k: {"mfma_busy": r.get("mfma_busy"), "clock_ghz": r.get("clock_ghz")}
                     for k, r in ((k, pmc_for(k)) for k, _ in TRAIN_PMC_KEYS) if r} or None,
        "large_batch": {"batch": BL, "value": BL / big_s, "unit": "samples/s",
                        "ms_per_step": 1e3 * big_s,
                        "note": "activations of one pass over the batch (~1.1 GB) exceed "
                                "the 512 MiB training budget: the step runs in row chunks"},
        "paper_train_example": {"workload": "18 torsion CVs, 4 x [300 x 4], residual, "
                                            "dropout 0.1, batch 128 (separate GEMM sweeps)",
                                "value": pB / paper_s, "unit": "samples/s",
                                "ms_per_step": 1e3 * paper_s},
    }


def bench_conservative(rid, torch, case, steps=40, warmup=5):
    """Conservative switching on the headline workload, with the band placed
    over the ensemble's deviations so every walker takes the switch's own
    gradient; the frozen-switch path at the same thresholds for comparison."""
    S, E, P, out, B = case["S"], case["E"], case["P"], case["out"], case["B"]
    rid.bias_force(S, E, P, 1e29, 2e29, out=out)
    torch.cuda.synchronize()
    eps = out["eps"].cpu().numpy()
    e0, e1 = 0.5 * float(eps.min()), 2.0 * float(eps.max())
    res = {}
    for name, cons in (("frozen", False), ("conservative", True)):
        for _ in range(warmup):
            rid.bias_force(S, E, P, e0, e1, out=out, conservative=cons)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rid.bias_force(S, E, P, e0, e1, out=out, conservative=cons)
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / steps
    # kernel timing (dispatch events) on separate calls
    rid.profile_enable(True)
    for _ in range(steps):
        rid.bias_force(S, E, P, e0, e1, out=out, conservative=True)
    kern = read_kernels(rid, [("mlp", rid.PROF_MLP), ("hvp", rid.PROF_HVP)])
    rid.profile_enable(False)
    sys_ = case["sys"]
    fl = conservative_flops_per_walker(sys_.n_cv, case["widths"], case["K"]) * B
    st = res["conservative"]
    r = {"workload": "conservative switching (force = -grad E inside the band: "
                     "Abar sigma'(eps) d eps/ds added through per-member Hessian-vector "
                     "products), same chain / ensemble / 1024 walkers, band over all "
                     "walkers, FP32",
         "value": B / st, "unit": "walker-steps/s", "ms_per_step": 1e3 * st,
         "frozen_ms_per_step": 1e3 * res["frozen"],
         "flop_per_step": fl, "achieved_tflops": fl / st / 1e12,
         "frac_fp32_peak": fl / st / 1e12 / FP32_PEAK_TFLOPS,
         "kernels_us": {k: 1e3 * v for k, v in kern.items()}}
    if "hvp" in kern:
        kf = hvp_kernel_flops_per_walker(sys_.n_cv, case["widths"], case["K"]) * B
        r["hvp_kernel"] = {"flop_per_launch": kf, "avg_launch_us": 1e3 * kern["hvp"],
                           "achieved_tflops": kf / (kern["hvp"] * 1e-3) / 1e12,
                           "frac_fp32_peak": kf / (kern["hvp"] * 1e-3) / 1e12 / FP32_PEAK_TFLOPS}
    return r


def bench_mcmc(rid, torch, steps=400, warmup=20):
    """MCMC on the ensemble free energy with the dimension-reduction phase's
    walker count, temperature and binning (2000 walkers, 300 K, 101 bins,
    pair (0, 1)) on the headline chain's 38 CVs and ensemble."""
    n, widths, K, W = 38, [256] * 4, 4, 2000
    E = rid.Ensemble(n, widths, K, ridgen.xavier_ensemble(2 * n, widths, K, 1000))
    s = torch.from_numpy(ridgen.f32(ridgen.torus_samples(W, n, 8))).cuda()
    kT = 0.0083144626 * 300.0
    out = rid.mcmc_run(E, s, warmup, kT, 0.3, 2024)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = rid.mcmc_run(E, s, steps, kT, 0.3, 2024, step0=warmup, hist1=out["hist1"],
                       hist2=out["hist2"], accepted=out["accepted"])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"workload": "MCMC in CV space on the ensemble free energy: 2000 walkers, 38 torsion "
                        "CVs, ensemble 4 x [256 x 4] FP32, 300 K, step 0.3 rad, 1D histograms "
                        "of every CV + 2D of CVs (0, 1), 101 bins",
            "value": W / dt, "unit": "walker-steps/s", "us_per_step": 1e6 * dt,
            "acceptance": int(out["accepted"].item()) / (W * (steps + warmup)),
            "seconds_for_1e6_steps": 1e6 * dt}


def bench_selection(rid, torch):
    """Selection phase with the paper's SelectorConfig (cluster_threshold 2.6,
    window [30, 45], max_selection 50) on 20 walkers x 1000 exploration frames
    of the headline chain's 38 CVs, eps from the headline ensemble; eps0 at
    the median deviation (the random-initialised ensemble has no trained
    scale for the trust level)."""
    n, widths, K = 38, [256] * 4, 4
    E = rid.Ensemble(n, widths, K, ridgen.xavier_ensemble(2 * n, widths, K, 1000))
    s = torch.from_numpy(ridgen.exploration_frames(20, 1000, n, 60, 0.3, seed=15)).cuda()
    B = s.shape[0]
    eps, _, _, _ = rid.model_dev(E, s, want_g=False)
    eps0 = float(torch.quantile(eps, 0.5))
    rid.select(E, s, eps0, 2.6, 30, 45, 50)
    torch.cuda.synchronize()
    reps_sel = 5
    t0 = time.perf_counter()
    for _ in range(reps_sel):
        out = rid.select(E, s, eps0, 2.6, 30, 45, 50)
    t_sel = (time.perf_counter() - t0) / reps_sel
    # one clustering pass at the adapted threshold, and the deviation alone
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        c = rid.cluster_frames(s, out["threshold"], eps=eps, eps0=eps0, max_clusters=51)
    t_clu = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        rid.model_dev(E, s, want_g=False)
    torch.cuda.synchronize()
    t_dev = (time.perf_counter() - t0) / reps
    return {"workload": "selection: 20 walkers x 1000 exploration frames of 38 torsion CVs, "
                        "eps from the ensemble 4 x [256 x 4] FP32, eps0 at the median, "
                        "threshold 2.6 adapted into [30, 45], max_selection 50",
            "value": B / t_sel, "unit": "frames/s", "ms_per_call": 1e3 * t_sel,
            "threshold_used": out["threshold"], "clusters": out["n_clusters"],
            "selected": int(out["selected"].numel()),
            "ms_per_clustering_pass": 1e3 * t_clu, "ms_model_dev": 1e3 * t_dev,
            "clusters_at_that_threshold": c["n_clusters"]}


def bench_labels(rid, torch, reps=20):
    M, T, n = 1024, 500, 38
    traj, s0, _ = ridgen.restrained_traj(M, T, n, 500.0, seed=9)
    tr = torch.from_numpy(traj).cuda()
    s0d = torch.from_numpy(s0).cuda()
    kappa = np.full(n, 500.0, np.float32)
    for _ in range(3):
        rid.mf_label(tr, s0d, kappa, None, 5.0)
    torch.cuda.synchronize()
    rid.profile_enable(True)
    for _ in range(reps):
        rid.mf_label(tr, s0d, kappa, None, 5.0)
    torch.cuda.synchronize()
    tot, cnt = rid.profile_read(rid.PROF_LABEL)
    rid.profile_enable(False)
    us = 1e3 * tot / cnt
    byts = M * T * n * 4 + M * n * 4 + 2 * M * n * 8 + M
    return {"workload": "restrained-MD mean-force labels, 1024 configs x 500 frames x 38 CVs, "
                        "FP64 accumulation",
            "avg_launch_us": us, "bytes_per_launch": byts,
            "roofline": {"bound": "hbm", "achieved": byts / (us * 1e-6) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": byts / (us * 1e-6) / 1e9 / HBM_PEAK_GBS}}


SERVE_SYSTEMS = (("dipeptide", ridgen.system_dipeptide),     # 2 CVs, 22 atoms
                 ("peptide20", ridgen.system_peptide20),     # 38 CVs, 200 atoms
                 ("peptide61", ridgen.system_peptide61))     # 120 CVs, 1000 atoms
SERVE_WIDTHS = {100: [100] * 3, 256: [256] * 4, 512: [512] * 4}
SERVE_POOL = 256          # walkers of seeded positions per system class


def _serve_models(rid, torch, fp32_only):
    """One registered model per (system class, width, precision): widths
    100 / 256 / 512 ([100 x 3], [256 x 4], [512 x 4]), FP32 and BF16 (K = 8
    for 512-BF16, else 4), so a uniform model draw gives the classes, widths
    and precisions uniformly.  Each class also gets a device pool of
    SERVE_POOL walkers' seeded positions that its requests take slices of."""
    models, pools = [], []
    for ci, (name, mk) in enumerate(SERVE_SYSTEMS):
        sys_ = mk()
        S = rid.System(sys_.n_atoms, sys_.quads)
        pos = ridgen.f32(ridgen.chain_coords(sys_, SERVE_POOL, 7 + ci))
        pools.append(dict(sys=sys_, host=pos, dev=torch.from_numpy(pos).cuda()))
        for width, widths in SERVE_WIDTHS.items():
            for prec in ([rid.RID_FP32] if fp32_only else [rid.RID_FP32, rid.RID_BF16]):
                K = 8 if (width == 512 and prec == rid.RID_BF16) else 4
                E = rid.Ensemble(sys_.n_cv, widths, K,
                                 ridgen.xavier_ensemble(2 * sys_.n_cv, widths, K, 1000 + ci),
                                 prec)
                models.append(dict(cls=ci, S=S, E=E))
    return models, pools


def _serve_requests(torch, models, pools, n, seed, device):
    """n requests: model uniform, walkers log-uniform in [1, 256], a slice of
    the class's position pool; device requests get their own output slices
    (forces, eps) of per-class device buffers.  Returns (requests without
    arrival times, walkers [n], unit-rate Poisson gaps [n])."""
    rng = np.random.default_rng(seed)
    mi = rng.integers(0, len(models), size=n)
    w = np.clip(np.floor(np.exp(rng.uniform(0.0, math.log(257), size=n))), 1, 256).astype(int)
    off = [int(rng.integers(0, SERVE_POOL - int(w[i]) + 1)) for i in range(n)]
    gaps = rng.exponential(1.0, size=n)
    outs = {}
    if device:
        for c, pl in enumerate(pools):
            tot = int(sum(w[i] for i in range(n) if models[mi[i]]["cls"] == c))
            outs[c] = (torch.empty((max(tot, 1), pl["sys"].n_atoms, 3), dtype=torch.float32,
                                   device="cuda"),
                       torch.empty(max(tot, 1), dtype=torch.float32, device="cuda"), [0])
    reqs = []
    for i in range(n):
        m = models[mi[i]]
        pl = pools[m["cls"]]
        if device:
            F, eps, cur = outs[m["cls"]]
            o = dict(F=F[cur[0]:cur[0] + w[i]], eps=eps[cur[0]:cur[0] + w[i]])
            cur[0] += int(w[i])
            reqs.append(dict(model=int(mi[i]), pos=pl["dev"][off[i]:off[i] + w[i]], out=o))
        else:
            reqs.append(dict(model=int(mi[i]), pos=pl["host"][off[i]:off[i] + w[i]]))
    return reqs, w, gaps


def _serve_run(rid, torch, models, pools, fifo, device, n_warm=1000, n_meas=20000,
               loads=(0.25, 0.5, 0.75, 0.9), seed=5):
    """The serving protocol on one server: n_warm requests to warm up, then
    n_meas requests closed-loop (all offered at once: the capacity), then
    the same n_meas requests as a Poisson stream at each fraction of that
    capacity.  Latency = arrival at the server to results visible (device
    buffers for device requests)."""
    srv = rid.Server((8 << 30) if fifo else (64 << 30), n_streams=4, max_batch_walkers=8192,
                     fifo=fifo)
    ids = [srv.register(m["S"], m["E"], 2.0, 3.0) for m in models]
    assert ids == list(range(len(models)))
    warm, _, _ = _serve_requests(torch, models, pools, n_warm, seed + 100, device)
    reqs, w, gaps = _serve_requests(torch, models, pools, n_meas, seed, device)
    torch.cuda.synchronize()
    for q in warm:
        q["arrival_s"] = 0.0
    srv.replay(warm)

    def run(arrivals):
        for q, a in zip(reqs, arrivals):
            q["arrival_s"] = float(a)
        srv.reset_stats()
        lat, lag, wall = srv.replay(reqs)
        st = srv.stats()
        return {"requests": n_meas, "p50_us": float(np.percentile(lat, 50)),
                "p99_us": float(np.percentile(lat, 99)), "mean_us": float(lat.mean()),
                "walker_steps_per_s": float(w.sum()) / wall, "wall_s": wall,
                "batches": st["batches"], "mean_batch_walkers": st["mean_batch_walkers"],
                "max_inflight_batches": st["max_inflight_batches"],
                "max_submit_lag_us": float(lag.max()), "p99_submit_lag_us": float(np.percentile(lag, 99))}

    cap = run(np.zeros(n_meas))
    cap_req_s = n_meas / cap["wall_s"]
    out = {"capacity": cap, "capacity_req_per_s": cap_req_s, "loads": []}
    for f in loads:
        r = run(np.cumsum(gaps) / (f * cap_req_s))
        r.update({"load": f, "offered_req_per_s": f * cap_req_s,
                  "offered_walker_steps_per_s": f * cap["walker_steps_per_s"]})
        out["loads"].append(r)
    srv.close()
    return out


def bench_serving(rid, torch):
    """Serving form: requests over 3 system classes x widths 100/256/512 x
    FP32/BF16 (the model drawn uniformly), 1-256 walkers log-uniform, walker
    state device-resident (positions read from and forces written to device
    buffers), HBM budget 64 GiB; 1000 warm-up requests, 20 000 measured ones
    closed-loop for the capacity, then at offered loads 0.25 / 0.5 / 0.75 /
    0.9 x capacity (Poisson).  Baseline: the same trace over FP32 models
    served FIFO, one request at a time, at the same fractions of its own
    capacity.  The trace is replayed by the library's native driver."""
    mixed, pools = _serve_models(rid, torch, fp32_only=False)
    log("serving: batched, device-resident")
    batched = _serve_run(rid, torch, mixed, pools, fifo=False, device=True)
    log("serving: batched, host-staged capacity")
    host = _serve_run(rid, torch, mixed, pools, fifo=False, device=False, loads=())
    fp32, pools32 = _serve_models(rid, torch, fp32_only=True)
    log("serving: FIFO FP32 baseline")
    fifo = _serve_run(rid, torch, fp32, pools32, fifo=True, device=True)
    half = [r for r in batched["loads"] if r["load"] == 0.5][0]
    return {
        "workload": "Poisson requests over 3 system classes (2 CVs/22 atoms, 38/200, 120/1000) x "
                    "widths 100/256/512 x FP32/BF16 (K=8 for 512-BF16), 1-256 walkers "
                    "log-uniform, weights and walker state resident in HBM, HBM budget 64 GiB; "
                    "1000 warm-up + 20000 measured requests; loads 0.25/0.5/0.75/0.9 x capacity",
        "batched": batched, "batched_host_staged": {"capacity": host["capacity"]},
        "fifo_fp32": fifo,
        "p50_us": half["p50_us"], "p99_us": half["p99_us"],
        "walker_steps_per_s": batched["capacity"]["walker_steps_per_s"],
        "capacity_vs_fifo_fp32": batched["capacity"]["walker_steps_per_s"]
                                 / fifo["capacity"]["walker_steps_per_s"],
    }


def trace_summary(db, out_path, command):
    """Kernel statistics (calls, total, average, share of GPU time) of a
    rocprofv3 --kernel-trace --stats run, from its rocpd database, as text;
    the mlp_kernel families are named by their PMC_CASES key."""
    import sqlite3
    con = sqlite3.connect(db)
    rows = list(con.execute("select name, total_calls, total_duration, average, percentage "
                            "from top_kernels order by total_duration desc"))
    con.close()
    dm = _demangle([r[0] for r in rows])
    lines = [f"rocprofv3 kernel statistics (durations in microseconds)", f"command: {command}", "",
             f"{'calls':>7} {'total_us':>12} {'avg_us':>10} {'pct':>6}  kernel"]
    for name, calls, tot, avg, pct in rows:
        nm = mlp_display(name) or dm.get(name, name)
        key = pmc_kernel_key(name)
        short = nm.replace("rid::(anonymous namespace)::", "")
        if len(short) > 150:
            short = short[:150] + "..."
        lines.append(f"{calls:>7} {tot:>12.1f} {avg:>10.3f} {pct:>6.2f}  {short}"
                     + (f"   [{key}]" if key else ""))
    txt = "\n".join(lines) + "\n"
    with open(out_path, "w") as fh:
        fh.write(txt)
    print(txt)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # The GPU reaches its sustained clock only after ~20 ms of load (the first
    # few hundred headline steps run ~8 % slower): the default warmup covers
    # that, so the timed region measures the steady state of a long MD run.
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--trace-summary", nargs=3, metavar=("DB", "OUT", "COMMAND"),
                    help="render a rocprofv3 --kernel-trace --stats database as text")
    ap.add_argument("--pmc-workload", action="store_true",
                    help="run the short program the counter passes profile")
    ap.add_argument("--pmc-summary", nargs="+", metavar="OUT DIR",
                    help="summarize rocprofv3 --pmc passes (one directory each) into "
                         "per-kernel counter figures, written to OUT")
    args = ap.parse_args()
    if args.trace_summary:
        trace_summary(*args.trace_summary)
        return
    if args.pmc_summary:
        if len(args.pmc_summary) < 2:
            ap.error("--pmc-summary OUT DIR [DIR ...]")
        pmc_summary(*args.pmc_summary)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (walkers "
              "would shard across GPUs with no exchange between them). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2408_14070_amd as rid
    rid.lib()
    assert torch.cuda.is_available(), "needs an MI355X"
    log("library loaded")
    if args.pmc_workload:
        pmc_workload(rid, torch)
        return

    sys20 = ridgen.system_peptide20()
    B, K, widths = 1024, 4, [256] * 4
    case = build_case(rid, torch, sys20, B, K, widths, rid.RID_FP32)
    elapsed, kern = time_bias(rid, torch, case, args.steps, args.warmup)
    ms_step = 1e3 * elapsed / args.steps
    log(f"headline: {ms_step * 1e3:.1f} us per step")
    call_pct = call_percentiles(rid, torch, case)
    value = B * args.steps / elapsed
    flop_launch = mlp_flops_per_walker(sys20.n_cv, widths, K) * B
    achieved = flop_launch / (kern["mlp"] * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": traffic_for("mlp_fp32_4x256_b1024"),
            "mfma_busy": mfma_busy_for("mlp_fp32_4x256_b1024"),
            "kernel": "mlp_kernel<F32,256> (torsions gathered in-kernel + ensemble "
                      "forward + input-gradient sweep)",
            "avg_launch_us": kern["mlp"] * 1e3, "flop_per_launch": flop_launch}
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
        "kernel_events": f"1 call in {EVENT_EVERY} of the timed region",
        "latency_us_per_call": ms_step * 1e3,
        "call_us_percentiles": call_pct,
    }
    samples = {"fp32_headline": sample_outputs(case, 128)}
    if not args.no_extra:
        steps_b = max(10, args.steps // 10)
        wb = max(3, args.warmup // 4)
        log("precision forms")
        rec["precision_form"] = bench_precision(rid, torch, sys20, rid.RID_BF16, "BF16",
                                                steps_b, wb, samples)
        rec["precision_form_fp16"] = bench_precision(rid, torch, sys20, rid.RID_FP16, "FP16",
                                                     steps_b, wb, samples)
        rec["precision_form_bf16_all"] = bench_precision(rid, torch, sys20, rid.RID_BF16_ALL,
                                                         "BF16_ALL", steps_b, wb, samples)
        rec["precision_form_fp32"] = bench_precision(rid, torch, sys20, rid.RID_FP32, "FP32",
                                                     max(4, steps_b // 8), max(2, wb // 8),
                                                     samples)
        rec["precision_form"]["speedup_vs_fp32_same_shape"] = (
            rec["precision_form"]["value"] / rec["precision_form_fp32"]["value"])
        log("network and CV variants")
        rec["variants"] = bench_variants(rid, torch, sys20, steps_b, wb)
        log("conservative switching")
        rec["conservative"] = bench_conservative(rid, torch, case)
        log("mcmc")
        rec["mcmc"] = bench_mcmc(rid, torch)
        log("training")
        rec["training"] = bench_training(rid, torch, samples=samples)
        log("labels")
        rec["labels"] = bench_labels(rid, torch)
        log("selection")
        rec["selection"] = bench_selection(rid, torch)
        if not args.no_serve:
            log("serving")
            rec["serving"] = bench_serving(rid, torch)
    if not args.no_cpu_baseline:
        log("cpu baseline and sampled accuracy")
        rec["cpu_baseline"] = cpu_baseline(case, samples)
        # each line's force error against the FP64 oracle, from that leg
        acc = rec["cpu_baseline"]["accuracy_vs_oracle"]
        rec["accuracy"] = acc.get("fp32_headline")
        for key, name in (("precision_form", "bf16"), ("precision_form_fp16", "fp16"),
                          ("precision_form_bf16_all", "bf16_all"),
                          ("precision_form_fp32", "fp32")):
            if key in rec and name in acc:
                rec[key]["accuracy"] = acc[name]
        if "training" in rec and "training_b4096" in acc:
            rec["training"]["accuracy"] = acc["training_b4096"]
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
