"""Writes tests/golden/paper_scale_replica.json: the oracle's merge of a
replica of the 100,000,000-vector uint8 workload at 1/100 scale.

The replica: 1,000,000 vectors from the workload's distribution
(inputs.paper_scale_u8: dim 96, 4,096 components, centres uniform on
[40, 215], sigma 30, uint8), cut into 50 sub-indexes of 2,000 +
Dirichlet(1, ..., 1) shares of the rest (largest-remainder rounding), in
order; each sub-index the exact 64-NN graph pruned to R = 32 (alpha 1.2)
with reverse edges (alpha 1.2) and the reachability repair; merged with
R = 32, L = 64, alpha = 1.2, MOS degree bound 8, unit costs.

Only oracle/ and the seeded input generators run here. The file holds
SHA-256 digests of the inputs (the uint8 rows, every sub-index graph) and
of the merged graph (offsets int64, neighbours int32, distances float64,
little-endian), the merged entry and sizes, and a sample of merged rows for
diagnostics. Run: python tests/golden/make_paper_scale_replica.py
(minutes on a few cores).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2602_17099_amd import inputs  # noqa: E402

SCALE = 0.01
M = 50
R, L, ALPHA, K, MOS = 32, 64, 1.2, 64, 8
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_scale_replica.json")


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def replica():
    total = int(round(100_000_000 * SCALE))
    sizes = inputs.dirichlet_sizes(M, total, int(round(200_000 * SCALE)), seed=inputs.SEED_BASE + 5)
    U = inputs.paper_scale_u8(total)
    return U, sizes


def main():
    O.lib()
    O.set_threads(os.cpu_count() or 1)
    t0 = time.perf_counter()
    U, sizes = replica()
    X = U.astype(np.float32)
    subs, b = [], 0
    for n in sizes:
        subs.append(O.build_graph(X[b:b + n], K, R, alpha=ALPHA, reverse=True, alpha_rev=ALPHA,
                                  repair=True))
        b += n
    t1 = time.perf_counter()
    ref = O.merge(subs, X, R=R, L=L, alpha=ALPHA, mos_degree=MOS)
    t2 = time.perf_counter()
    off, nb, ds = ref["offsets"], ref["nbrs"].astype(np.int32), ref["dists"].astype(np.float64)
    g = np.random.default_rng(7)
    sample = sorted(int(v) for v in g.choice(len(off) - 1, size=64, replace=False))
    doc = {
        "about": __doc__.strip().splitlines()[0],
        "scale": SCALE, "sizes": sizes, "R": R, "L": L, "alpha": ALPHA, "K": K,
        "mos_degree": MOS,
        "inputs_sha256": sha(U),
        "subindex_sha256": [sha(o.astype(np.int64), nbx.astype(np.int32), np.array([e], np.int32))
                            for o, nbx, e in subs],
        "merged_sha256": sha(off.astype(np.int64), nb, ds),
        "entry": int(ref["entry"]), "n_edges": int(off[-1]), "n_ops": len(ref["ops"]),
        "sample_rows": {str(v): nb[off[v]:off[v + 1]].tolist() for v in sample},
        "oracle_seconds": {"build": round(t1 - t0, 1), "merge": round(t2 - t1, 1),
                           "threads": O.get_threads()},
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {OUT}: {doc['n_ops']} operations, {doc['n_edges']} edges, "
          f"build {t1 - t0:.0f} s, merge {t2 - t1:.0f} s")


if __name__ == "__main__":
    main()
