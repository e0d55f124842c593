"""Writes explore_d6_n10000.json: the oracle's exhaustive search (Algorithm 2,
rays by definition) of the d=6, N=10 000 uniform workload (uniform_cloud seed
0, the Descent draws of workloads.descent_draws(6)), summarised by its counts
and the SHA-256 of its sorted vertex keys and of its sorted unbounded edges
(key, omitted generator), int32 little-endian rows.  Calls only oracle/ (about
an hour on one core)."""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def rows_digest(a):
    rows = np.ascontiguousarray(oracle.sorted_rows(np.asarray(a, dtype=np.int32)), dtype="<i4")
    return hashlib.sha256(rows.tobytes()).hexdigest()


def main():
    d, n = 6, 10_000
    X = W.uniform_cloud(n, d, seed=0)
    t0 = time.time()
    m = oracle.explore(X, W.descent_draws(d))
    out = {
        "source": "oracle.explore (Algorithm 2, RayCast by definition in FP64) on "
                  "uniform_cloud(10000, 6, seed=0) with descent_draws(6)",
        "vertices": int(m["sigma"].shape[0]),
        "unbounded_edges": int(m["b_sigma"].shape[0]),
        "raycasts": int(m["raycasts"]),
        "sigma_sha256": rows_digest(m["sigma"]),
        "unbounded_sha256": rows_digest(np.column_stack([m["b_sigma"], m["b_omit"]])),
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "explore_d6_n10000.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
