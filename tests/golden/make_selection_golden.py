"""Write selection_20k.json: the oracle's selection of the benchmarked
selection workload (20 walkers x 1000 exploration frames of 38 torsion CVs,
deviation from the 4 x [256 x 4] ensemble of seed 1000, cluster threshold 2.6
adapted into [30, 45], max_selection 50).  Calls only the seeded generators
and the oracle.  eps0 is the midpoint of the widest gap between the oracle's
deviations within 200 ranks of the median, so a deviation evaluated in FP32
cannot fall on the other side of it (the GPU test checks the margin).

Usage: python tests/golden/make_selection_golden.py   (about a minute)."""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import ridgen  # noqa: E402
from oracle import rid_oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selection_20k.json")


def labels_digest(labels):
    return hashlib.sha256(np.ascontiguousarray(labels, dtype="<i8").tobytes()).hexdigest()


def main():
    n, widths, K = 38, [256] * 4, 4
    params = ridgen.xavier_ensemble(2 * n, widths, K, 1000)
    models = ridgen.unpack_params(params, 2 * n, widths, K)
    s = ridgen.exploration_frames(20, 1000, n, 60, 0.3, seed=15)
    eps = O.frame_deviation(models, s.astype(np.float64))
    e = np.sort(eps)
    mid = len(e) // 2
    lo, hi = mid - 200, mid + 200
    k = lo + int(np.argmax(np.diff(e[lo:hi])))
    eps0 = float(0.5 * (e[k] + e[k + 1]))
    gap = float(e[k + 1] - e[k])
    ref = O.select_frames(models, s, eps0, 2.6, 30, 45, 50, adapt=True)
    out = {
        "what": "oracle selection of the benchmarked selection workload",
        "frames": [20, 1000, n, 60, 0.3, 15],
        "ensemble": {"widths": widths, "K": K, "seed": 1000},
        "eps0": eps0, "eps_gap": gap, "threshold0": 2.6, "window": [30, 45],
        "max_selection": 50,
        "threshold": float(ref["threshold"]), "n_clusters": int(ref["n_clusters"]),
        "leaders": [int(v) for v in ref["leaders"]],
        "selected": [int(v) for v in ref["selected"]],
        "n_kept": int(np.sum(ref["keep"])),
        "labels_sha256": labels_digest(ref["labels"]),
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"wrote {OUT}: threshold {out['threshold']}, {out['n_clusters']} clusters")


if __name__ == "__main__":
    main()
