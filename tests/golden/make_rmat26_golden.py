#!/usr/bin/env python3
"""Write the oracle's expected results for the R-MAT scale-26 workload.

The graph (R-MAT scale 26, edge factor 16: 2^26 ids, 2^30 records) is too large to replay
inside a GPU test, so this script runs the CPU oracle on it once and stores what a GPU solve
must reproduce bit for bit: the round count, every round's statistics, a SHA-256 of every
round's parents (int32 per name, -1 for names that are not nodes of the round), a SHA-256 of
the raw labels (uint32 per vertex) and of the canonical labels (smallest id of each
component, from the oracle's union-find).

It calls only the seeded input generator and the oracle.  It needs about 30 GB of host
memory and takes tens of minutes on one core:

    python tests/golden/make_rmat26_golden.py [--seed S] [--out FILE]
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

BENCH_SEED = graphgen.CONFIG_SEED_BASE + 1


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=lambda s: int(s, 0), default=BENCH_SEED)
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    out = args.out or os.path.join(HERE, "rmat%d_seed_%x.json" % (args.scale, args.seed))

    t0 = time.perf_counter()
    g = graphgen.workload_rmat(scale=args.scale)
    t_gen = time.perf_counter() - t0
    print("generated n=%d m=%d in %.1f s" % (g.n, g.m, t_gen), flush=True)

    t0 = time.perf_counter()
    res = oracle.run(g.n, g.src, g.dst, seed=args.seed, record_parents=True, parents_cap=16)
    t_run = time.perf_counter() - t0
    print("oracle: %d rounds in %.1f s" % (res.rounds, t_run), flush=True)
    for s in res.stats:
        print("  round %d: n_active=%d m_in=%d survive=%d m_out=%d finalised=%d" % s, flush=True)

    parents = [sha(res.parents[r].view(np.int32)) for r in range(res.parents.shape[0])]
    labels_sha = sha(res.labels.astype(np.uint32))
    del res.parents

    t0 = time.perf_counter()
    canon = oracle.components_min_id(g.n, g.src, g.dst)
    t_uf = time.perf_counter() - t0
    doc = {
        "workload": "R-MAT scale %d, edge factor 16, quadrants (0.57, 0.19, 0.19, 0.05) +-10%% per level, "
                    "permuted ids, graph seed 0x%x" % (args.scale, graphgen.CONFIG_SEED_BASE + 2),
        "n_vertices": g.n,
        "n_records": g.m,
        "seed": args.seed,
        "rounds": res.rounds,
        "stats": [list(s) for s in res.stats],
        "parents_sha256": parents,
        "labels_sha256": labels_sha,
        "canonical_labels_sha256": sha(canon.astype(np.uint32)),
        "components": int(np.unique(canon).size),
        "made_by": "tests/golden/make_rmat26_golden.py (graphgen + oracle only)",
        "oracle_seconds": round(t_run, 1),
        "union_find_seconds": round(t_uf, 1),
        "host": "%s, 1 thread" % cpu_model(),
    }
    with open(out + ".tmp", "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    os.replace(out + ".tmp", out)
    print("wrote %s" % out, flush=True)


if __name__ == "__main__":
    main()
