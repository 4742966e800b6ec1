"""Benchmark: merged vertices/s of the RNSM merge on one MI355X.

Workload (default): two sub-indexes of 500,000 vectors each, dim 128,
integers 0..255 from a 64-component Gaussian mixture (sigma 30) stored as
float32, squared L2; each sub-index has out-degree <= 32; merge with R=32,
L=64, alpha=1.2; 10,000 held-out queries for recall@10. A step is one whole
merge (expansion, inversion, pivots, naive and sliding searches, prunes,
reverse edges, compaction) with every input already in HBM.

Prints one JSON line. Options: --steps K, --warmup W, --gpus N (only 1),
--workload {fp32-2x500k,tiny}, --no-cpu-baseline, --calib-copy (adds a plain
1 GiB device copy for counter calibration).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

# HBM traffic of the k_beam_search launches of one merge, from two rocprofv3
# --pmc passes (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) over
# `bench.py --one-stream --steps 1 --warmup 0 --no-cpu-baseline --no-recall`
# with --no-bf16 (float32 rows) or --bf16-only (bfloat16 copy), each counter
# scaled by what it reads for a plain 1 GiB device copy (FETCH_SIZE reads
# 0.5 GiB: factor 2.0; WRITE_SIZE 1 GiB: factor 1.0). The figures hold for the
# sources they were taken on only (sha256 of the files below); otherwise the
# line's traffic is null and its roofline falls back to algorithmic bytes.
COUNTER_SOURCES = ("paper_2602_17099_amd/csrc/rnsm_kernels.hip",
                   "paper_2602_17099_amd/csrc/rnsm_api.cpp")
SEARCH_COUNTERS = {
    "fp32": {
        "sources_sha256": "ebc676544128a85c4cacf5c8e908c9205a352fd442f3a7c8578972837dd48749",
        "kernel": "k_beam_search<0, 1, 4, false, 3>",
        "fetch_kib": [
            28591989.625,
            30219.625,
            2466223.5,
            107478.062,
            5587405.625,
            532523.188,
            14828072.562,
            1995516.625,
            19674610.438,
            18806222.812,
            18494874.688,
            11644181.688
        ],
        "write_kib": [
            174074.156,
            48.125,
            19571.875,
            193.125,
            38870.0,
            970.625,
            77168.125,
            3530.625,
            74595.625,
            32081.875,
            46043.125,
            19426.875
        ]
    },
    "bf16": {
        "sources_sha256": "ebc676544128a85c4cacf5c8e908c9205a352fd442f3a7c8578972837dd48749",
        "kernel": "k_beam_search<1, 1, 4, false, 2>",
        "fetch_kib": [
            10822339.812,
            3457.062,
            189460.0,
            8418.188,
            357927.562,
            20570.375,
            907637.875,
            62804.812,
            1749403.125,
            107732.25,
            2915054.812,
            188262.625,
            3539175.188,
            369166.438,
            4386432.875,
            830340.375,
            5137545.5,
            2632710.75,
            5386122.188,
            9264504.0,
            977815.562,
            1240407.125
        ],
        "write_kib": [
            159620.0,
            8.125,
            4910.625,
            25.0,
            9851.875,
            72.5,
            19501.875,
            247.5,
            38840.0,
            435.0,
            38661.25,
            775.625,
            38301.25,
            1491.25,
            37578.75,
            3314.375,
            35752.5,
            10318.125,
            28744.375,
            34956.25,
            4106.25,
            4607.5
        ]
    }
}
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in COUNTER_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def search_traffic(form="fp32"):
    """Measured HBM bytes per k_beam_search launch of the form (fp32, bf16),
    or None when the counters were taken on other sources."""
    c = SEARCH_COUNTERS.get(form)
    if not c or c["sources_sha256"] != sources_sha256():
        return None
    tot = sum(c["fetch_kib"]) * FETCH_FACTOR + sum(c["write_kib"]) * WRITE_FACTOR
    return tot * 1024.0 / len(c["fetch_kib"])


def roofline_line(alg_bytes_per_launch, ms_per_launch, launches_per_step, ms_per_step,
                  traffic_per_launch, peak=None):
    """The line's roofline of the search kernel. Time base: the exclusive
    launch time (each launch alone on the stream, HIP events on that stream).
    achieved / frac: measured HBM bytes (counters) per launch over that time
    when the counters match the sources, else the algorithmic bytes (basis
    says which). The algorithmic rate is reported beside it; it counts the
    re-reads that L2 and the Infinity Cache serve, so where it passes the HBM
    peak (per launch, or as algorithmic bytes per step over the whole step
    time) the line says cache_served."""
    peak = PEAK_HBM_GBS if peak is None else peak
    alg_gbs = alg_bytes_per_launch / (ms_per_launch * 1e6)
    step_gbs = alg_bytes_per_launch * launches_per_step / (ms_per_step * 1e6)
    if traffic_per_launch is not None:
        achieved, basis = traffic_per_launch / (ms_per_launch * 1e6), "hbm_counters"
    else:
        achieved, basis = alg_gbs, "algorithmic"
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": peak, "unit": "GB/s",
            "frac": round(achieved / peak, 4),
            "traffic": round(traffic_per_launch) if traffic_per_launch is not None else None,
            "basis": basis,
            "algorithmic_gbs": round(alg_gbs, 1), "algorithmic_frac": round(alg_gbs / peak, 4),
            "algorithmic_step_gbs": round(step_gbs, 1),
            "cache_served": bool(alg_gbs > peak or step_gbs > peak or
                                 (traffic_per_launch is not None and
                                  traffic_per_launch < alg_bytes_per_launch)),
            "bytes_per_launch": alg_bytes_per_launch, "ms_per_launch": ms_per_launch,
            "launches_per_step": launches_per_step,
            "time_base": "exclusive launch time: every search launch alone on one stream "
                         "(RNSM_ONE_STREAM=1 pass), HIP events on that stream"}

WORKLOADS = {
    "fp32-2x500k": dict(n=500_000, dim=128, R=32, L=64, alpha=1.2, K=64, nq=10_000,
                        gen="mixture_u8", build_alpha=1.2, reverse=True),
    "tiny": dict(n=5_000, dim=32, R=16, L=32, alpha=1.2, K=32, nq=500, gen="tiny_int",
                 build_alpha=1.0, reverse=False),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs(wl, seed_off=0):
    from paper_2602_17099_amd import inputs
    n2 = 2 * wl["n"]
    if wl["gen"] == "mixture_u8":
        X = inputs.mixture_u8(n2, wl["dim"], seed=inputs.SEED_BASE + 2)
        Q = inputs.mixture_u8(wl["nq"], wl["dim"], seed=inputs.SEED_BASE + 2, stream=1)
    else:
        allx = inputs.tiny_int(n2 + wl["nq"], wl["dim"], seed=inputs.SEED_BASE + 1)
        X, Q = allx[:n2], allx[n2:]
    return np.ascontiguousarray(X), np.ascontiguousarray(Q)


def build_graph_checked(pkg, Xi, knn, wl, info=None):
    """The builder with the reachability repair; with `info`, also the
    vertices reachable from the entry before the repair and the links it
    added."""
    kw = dict(alpha=wl["build_alpha"], reverse=wl["reverse"], alpha_rev=1.2)
    if info is not None:
        o0, b0, e0 = pkg.build_graph(Xi, knn, wl["R"], **kw)
        info.setdefault("reachable_before_repair", []).append(pkg.reachable(o0, b0, e0) / Xi.shape[0])
        del o0, b0
    off, nb, entry, links = pkg.build_graph(Xi, knn, wl["R"], repair=True, return_links=True, **kw)
    if info is not None:
        info.setdefault("repair_links", []).append(links)
        info.setdefault("reachable_after_repair", []).append(pkg.reachable(off, nb, entry) /
                                                              Xi.shape[0])
    return off, nb, entry


def build_subs(pkg, Xd, wl, parts=2, info=None):
    from paper_2602_17099_amd.prepare import knn_l2_exact
    subs = []
    n = Xd.shape[0] // parts
    for i in range(parts):
        Xi = Xd[i * n:(i + 1) * n]
        knn = knn_l2_exact(Xi, None, wl["K"], exclude_self=True)
        subs.append(build_graph_checked(pkg, Xi, knn, wl, info))
        del knn
    return subs


RECALL_EFS = (10, 16, 32, 64, 128)


def recall_sweep(pkg, off, nb, entry, Xd, Qd, gt):
    """recall@10 (Section 2.1) of searches from the entry at each beam."""
    return {str(ef): recall_at_10(pkg, off, nb, entry, Xd, Qd, gt, ef=ef) for ef in RECALL_EFS}


def slide_tradeoff(pkg, subs, Xd, Qd, gt, wl, steps=2):
    """The local-sliding trade-off (Section 4.2: sliding saves about
    (1 - |P|/|V|)(1 - ef_L/ef_N) of the naive search cost): RNSM with the
    naive beam at L and sliding beams ef_L <= L, against the cross-query
    merge (every source vertex a naive search) at beams up to L; each point
    is whole-merge time and recall@10 (query beam 64). `equal_recall` names
    the fastest RNSM point whose recall is within 0.002 of the cross-query
    merge at L."""
    import torch
    L = wl["L"]
    pts = []

    def run(flags, ef_naive, ef_slide):
        kw = dict(R=wl["R"], L=L, alpha=wl["alpha"], ef_naive=ef_naive, ef_slide=ef_slide,
                  flags=flags, dists=False)
        pkg.merge(subs, Xd, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            res = pkg.merge(subs, Xd, **kw)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        st = pkg.stats()
        rec = recall_at_10(pkg, res[0], res[1], res[3], Xd, Qd, gt)
        return {"ef_naive": ef_naive, "ef_slide": ef_slide, "ms_per_merge": 1000.0 * dt,
                "recall_at_10": rec, "ndc": sum(st["ndc"]), "pivots": st["n_pivots"]}

    for efs in sorted({16, 24, 32, 48, L}):
        if efs <= L:
            p = run(0, L, efs)
            p["form"] = "rnsm"
            pts.append(p)
    for efn in sorted({32, 48, L}):
        if efn <= L:
            p = run(pkg.FLAG_ALL_PIVOTS, efn, efn)
            p["form"] = "cross_query"
            pts.append(p)
    cm = [p for p in pts if p["form"] == "cross_query" and p["ef_naive"] == L][0]
    ok = [p for p in pts if p["form"] == "rnsm" and p["recall_at_10"] >= cm["recall_at_10"] - 0.002]
    best = min(ok, key=lambda p: p["ms_per_merge"]) if ok else None
    return {"points": pts, "equal_recall": None if best is None else
            {"rnsm": best, "cross_query": cm, "speedup": cm["ms_per_merge"] / best["ms_per_merge"]}}


def prune_rules(pkg, subs, Xd, Qd, gt, wl, steps=2):
    """The merge under each proximity-graph family's prune rule (Section 6's
    applicability experiment): alpha (the headline rule), alpha = 1 (NSG's
    MRNG), the SSG angle rule at 60 degrees and tau-MNG at tau = 5 (the angle
    and tau rules on the float32 walk); whole-merge time and recall@10."""
    import torch
    out = {}
    for name, kw in [("alpha_%g" % wl["alpha"], dict(alpha=wl["alpha"])),
                     ("mrng_alpha_1", dict(alpha=1.0)),
                     ("ssg_angle_60", dict(alpha=wl["alpha"], prune_rule=pkg.PRUNE_ANGLE,
                                           prune_param=60.0)),
                     ("tau_mng_5", dict(alpha=wl["alpha"], prune_rule=pkg.PRUNE_TAU,
                                        prune_param=5.0))]:
        args = dict(R=wl["R"], L=wl["L"], dists=False, **kw)
        pkg.merge(subs, Xd, **args)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            res = pkg.merge(subs, Xd, **args)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        st = pkg.stats()
        out[name] = {"ms_per_merge": 1000.0 * dt, "prune_ms": st["ms_prune"],
                     "prune_path": st["prune_path"],
                     "recall_at_10": recall_at_10(pkg, res[0], res[1], res[3], Xd, Qd, gt),
                     "mean_degree": float(res[0][-1].item()) / Xd.shape[0]}
    return out


def rebuild_baseline(pkg, Xd, Qd, gt, wl):
    """The rebuild the merge replaces: the same builder (exact k-NN, prune,
    reverse edges, repair) on the union of the sub-indexes' vectors."""
    import torch
    from paper_2602_17099_amd.prepare import knn_l2_exact
    torch.cuda.synchronize()
    t = time.perf_counter()
    knn = knn_l2_exact(Xd, None, wl["K"], exclude_self=True)
    info = {}
    off, nb, entry = build_graph_checked(pkg, Xd, knn, wl, info)
    del knn
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    return {"build_s": dt, "reachable_frac": info["reachable_after_repair"][0],
            "reachable_before_repair": info["reachable_before_repair"][0],
            "repair_links": info["repair_links"][0],
            "recall_at_10_by_ef": recall_sweep(pkg, off, nb, entry, Xd, Qd, gt)}


def incremental(pkg, Xd, Qd, gt, wl, parts=4):
    """The incremental scenario: the same vectors split into `parts` equal
    sub-indexes, merged one at a time into the growing index (a pairwise
    merge per step, the new sub-index as source). Sub-index builds are
    input preparation, outside the timed steps."""
    import torch
    subs = build_subs(pkg, Xd, wl, parts)
    n = Xd.shape[0] // parts
    torch.cuda.synchronize()
    acc = subs[0]
    steps = []
    t_all = 0.0
    for i in range(1, parts):
        Xi = Xd[:(i + 1) * n]
        t = time.perf_counter()
        off, nb, _, entry = pkg.merge([acc, subs[i]], Xi, R=wl["R"], L=wl["L"],
                                      alpha=wl["alpha"], dists=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        t_all += dt
        st = pkg.stats()
        steps.append({"index_size": int(i * n), "added": int(n), "ms": 1000.0 * dt,
                      "source_vertices": st["n_source_vertices"]})
        acc = (off, nb, entry)
    rec = recall_at_10(pkg, acc[0], acc[1], acc[2], Xd[:parts * n], Qd, gt) if gt is not None else None
    return {"parts": parts, "sub_index_size": int(n), "steps": steps, "ms_total": 1000.0 * t_all,
            "merged_vertices_per_s": (parts - 1) * n / t_all, "recall_at_10": rec}


def recall_at_10(pkg, off, nb, entry, Xd, Qd, gt, ef=64):
    import torch
    ids, _ = pkg.search(off, nb, entry, Xd, Qd, ef, 10)
    ids = ids.to(torch.int64)
    hit = (ids[:, :, None] == gt[:, None, :].to(torch.int64)).any(2).sum().item()
    return hit / (10 * Qd.shape[0])


PHASES = ("expansion", "naive", "sliding")


def time_merges(pkg, subs, Xd, wl, steps, warmup, search=None, flags=0, shape=None):
    """Time `steps` whole merges after `warmup`; per-phase event times and
    counts are summed over the timed steps."""
    import torch
    N = Xd.shape[0]
    R = wl["R"]
    out = (torch.empty(N + 1, dtype=torch.int64, device=Xd.device),
           torch.empty(N * R, dtype=torch.int32, device=Xd.device),
           torch.empty(N * R, dtype=torch.float32, device=Xd.device))
    kw = dict(R=R, L=wl["L"], alpha=wl["alpha"], search=search, out=out, flags=flags,
              search_shape=shape)
    for _ in range(warmup):
        pkg.merge(subs, Xd, **kw)
    torch.cuda.synchronize()
    agg = {"ms": [0.0] * 3, "bytes": [0.0] * 3, "ndc": [0] * 3, "launches": [0] * 3,
           "span_ms": 0.0}
    st = None
    t0 = time.perf_counter()
    for _ in range(steps):
        res = pkg.merge(subs, Xd, **kw)
        st = pkg.stats()
        agg["span_ms"] += st["ms_search_span"]
        for ph in range(3):
            agg["ms"][ph] += st["ms_search"][ph]
            agg["bytes"][ph] += st["bytes"][ph]
            agg["ndc"][ph] += st["ndc"][ph]
            agg["launches"][ph] += st["launches"][ph]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, agg, st, res


def autotune(pkg, subs, Xd, wl, args, ms_default, off, nb, bf16):
    """Search-shape autotuner on the target sub-index (its own rows as
    queries, beam L), then whole merges under the shape it picks, against the
    default shape's merges; the graph must not change."""
    import torch
    n0 = subs[0][0].shape[0] - 1
    o, b, e = subs[1]
    out = {}
    forms = [("fp32", None, ms_default)]
    if bf16 is not None:
        forms.append(("bf16", bf16[0], bf16[1]))
    for name, search, ms_def in forms:
        t = pkg.tune_search(o, b, e, Xd[n0:], wl["L"], n_sample=65536,
                            base_search=None if search is None else search[n0:])
        dt, _, _, res = time_merges(pkg, subs, Xd, wl, args.steps, args.warmup, search=search,
                                    shape=t["shape"])
        out[name] = {"shape": list(t["shape"]), "default_shape": list(t["default_shape"]),
                     "sample_ms": t["ms"], "default_sample_ms": t["default_ms"],
                     "sample_queries": t["n_queries"], "shapes_tried": t["n_tried"],
                     "ms_per_step": 1000.0 * dt / args.steps, "default_ms_per_step": ms_def,
                     "same_graph": bool(torch.equal(res[0], off) and torch.equal(res[1], nb))}
    return out


def multiway(pkg, scale, steps, warmup):
    """The many-sub-index inner-product workload at `scale` of its 10,000,000
    vectors: ten log-uniform sizes on [50,000, 2,000,000] x scale summing to
    10,000,000 x scale, an L2-normalised 256-component mixture in dim 96 cut
    into slabs along a seeded direction, sub-indexes from exact 64-NN pruned
    to R = 32, then MOS-ordered pairwise merges (degree bound 4, centroid
    costs) with R = 32, L = 64, alpha = 1.2. Reports merged vertices/s (source
    vertices over all operations per second), recall@10 of the merged graph,
    its invariants, and the search-shape autotuner against the default."""
    import torch
    from paper_2602_17099_amd import inputs
    from paper_2602_17099_amd.prepare import knn_float_exact
    IP = 1
    total = int(round(10_000_000 * scale))
    sizes = inputs.uneven_sizes(10, int(50_000 * scale), int(2_000_000 * scale), total,
                                seed=inputs.SEED_BASE + 3)
    t = time.perf_counter()
    X = inputs.mixture_unit(total, 96, comps=256, seed=inputs.SEED_BASE + 3)
    X = np.ascontiguousarray(X[inputs.slab_order(X, inputs.SEED_BASE + 33)])
    Q = inputs.mixture_unit(10_000, 96, comps=256, seed=inputs.SEED_BASE + 3, stream=1)
    log(f"multiway inputs {X.shape} sizes {sizes} in {time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    del X
    t = time.perf_counter()
    subs, b = [], 0
    for n in sizes:
        Xi = Xd[b:b + n]
        knn = knn_float_exact(Xi, None, 64, metric=IP, exclude_self=True)
        subs.append(pkg.build_graph(Xi, knn, 32, alpha=1.2, reverse=True, alpha_rev=1.2,
                                    metric=IP, repair=True))
        del knn
        b += n
        torch.cuda.synchronize()
        log(f"multiway sub-index of {n:,} built at {time.perf_counter() - t:.1f}s")
    torch.cuda.synchronize()
    log(f"multiway sub-indexes built in {time.perf_counter() - t:.1f}s")
    N = Xd.shape[0]
    kw = dict(R=32, L=64, alpha=1.2, metric=IP, mos_degree=4, flags=pkg.FLAG_CENTROID_COSTS,
              out=(torch.empty(N + 1, dtype=torch.int64, device=dev),
                   torch.empty(N * 32, dtype=torch.int32, device=dev),
                   torch.empty(N * 32, dtype=torch.float32, device=dev)))

    def run(shape=None, extra_flags=0):
        kw2 = dict(kw, flags=kw["flags"] | extra_flags)
        for _ in range(warmup):
            pkg.merge(subs, Xd, search_shape=shape, **kw2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = pkg.merge(subs, Xd, search_shape=shape, **kw2)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, pkg.stats(), res

    dt, st, (off, nb, ds, entry) = run()
    off_c, nb_c = off.clone(), nb.clone()
    # invariants: degree <= R, no self-loops, no repeated neighbour
    deg = off[1:] - off[:-1]
    row = torch.repeat_interleave(torch.arange(N, device=dev), deg)
    keys = row * N + nb.to(torch.int64)
    inv = {"max_degree": int(deg.max()), "self_loops": int((nb.to(torch.int64) == row).sum()),
           "repeated": int(keys.numel() - torch.unique(keys).numel())}
    del row, keys
    gt = knn_float_exact(Xd, Qd, 10, metric=IP, block=1024)
    ids, _ = pkg.search(off, nb, entry, Xd, Qd, 64, 10, metric=IP)
    rec = (ids.to(torch.int64)[:, :, None] == gt.to(torch.int64)[:, None, :]).any(2).sum().item()
    rec /= 10 * Qd.shape[0]
    big = max(range(len(sizes)), key=lambda i: sizes[i])
    b0 = sum(sizes[:big])
    o, g, e = subs[big]
    tune = pkg.tune_search(o, g, e, Xd[b0:b0 + sizes[big]], 64, n_sample=65536, metric=IP)
    dtt, _, rt = run(tuple(tune["shape"]))
    same = bool(torch.equal(rt[0], off_c) and torch.equal(rt[1], nb_c))
    # the batched form: operations sharing no sub-index in one round
    dtq, stq, rq = run(extra_flags=pkg.FLAG_BATCHED)
    batched = {"ms_per_merge": 1000.0 * dtq, "value": stq["n_source_vertices"] / dtq,
               "speedup_vs_plain": dt / dtq, "rounds": stq["n_rounds"],
               "same_graph": bool(torch.equal(rq[0], off_c) and torch.equal(rq[1], nb_c)),
               "phase_ms": {"expansion_search": stq["ms_search"][0], "order": stq["ms_order"],
                            "select": stq["ms_select"], "groups": stq["ms_groups"],
                            "group_search": stq["ms_search"][1],
                            "overflow_search": stq["ms_search"][2],
                            "prune_and_reverse": stq["ms_prune"], "total": stq["ms_total"]}}
    return {"workload": f"{len(sizes)} uneven slab sub-indexes, {N:,} L2-normalised vectors, "
                        f"dim 96, inner product, R=32, L=64, alpha=1.2, MOS degree 4",
            "scale_of_10M": scale, "sizes": sizes, "operations": st["n_ops"],
            "source_vertices": st["n_source_vertices"], "ms_per_merge": 1000.0 * dt,
            "value": st["n_source_vertices"] / dt, "unit": "merged vertices/s",
            "steps": steps, "warmup": warmup, "recall_at_10": rec, "invariants": inv,
            "phase_ms": {"expansion_search": st["ms_search"][0], "invert": st["ms_invert"],
                         "host_plan": st["ms_plan"], "naive_search": st["ms_search"][1],
                         "sliding_search": st["ms_search"][2], "prune_and_reverse": st["ms_prune"],
                         "compact": st["ms_compact"], "total": st["ms_total"]},
            "autotune": {"shape": list(tune["shape"]), "default_shape": list(tune["default_shape"]),
                         "sample_ms": tune["ms"], "default_sample_ms": tune["default_ms"],
                         "ms_per_merge": 1000.0 * dtt, "same_graph": same},
            "batched_form": batched}


def precision768(pkg, scale, steps, warmup):
    """The precision workload at `scale` of its 4,000,000 vectors: dim 768,
    per-dimension scale 1/sqrt(i), 1,024 components, L2-normalised, cosine;
    a random split into four equal sub-indexes (exact 96-NN pruned to
    R = 48); merged with R = 48, L = 96, alpha = 1.2 (MOS degree 2) from the
    float32 rows and from their bfloat16 copy (inexact here), each timed and
    scored by recall@10 against exact cosine neighbours."""
    import torch
    from paper_2602_17099_amd import inputs
    from paper_2602_17099_amd.prepare import knn_float_exact
    COS = 2
    n = int(round(1_000_000 * scale))
    t = time.perf_counter()
    X = inputs.mixture_unit(4 * n, 768, comps=1024, decay=True, seed=inputs.SEED_BASE + 4)
    X = X[inputs.rng(inputs.SEED_BASE + 44).permutation(len(X))]
    Q = inputs.mixture_unit(10_000, 768, comps=1024, decay=True, seed=inputs.SEED_BASE + 4,
                            stream=1)
    log(f"precision inputs {X.shape} in {time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    del X
    t = time.perf_counter()
    subs = []
    for i in range(4):
        Xi = Xd[i * n:(i + 1) * n]
        # unit rows: the inner-product order is the cosine order
        knn = knn_float_exact(Xi, None, 96, metric=1, exclude_self=True)
        subs.append(pkg.build_graph(Xi, knn, 48, alpha=1.2, reverse=True, alpha_rev=1.2,
                                    metric=COS, repair=True))
        del knn
        torch.cuda.synchronize()
        log(f"precision sub-index {i} built at {time.perf_counter() - t:.1f}s")
    N = Xd.shape[0]
    gt = knn_float_exact(Xd, Qd, 10, metric=1, block=1024)
    out = {"workload": f"4 random-split sub-indexes, {N:,} L2-normalised vectors, dim 768 "
                       f"(scale 1/sqrt(i)), cosine, R=48, L=96, alpha=1.2, MOS degree 2",
           "scale_of_4M": scale, "steps": steps, "warmup": warmup}
    bufs = (torch.empty(N + 1, dtype=torch.int64, device=dev),
            torch.empty(N * 48, dtype=torch.int32, device=dev),
            torch.empty(N * 48, dtype=torch.float32, device=dev))

    def timed(search, L, reps):
        kw = dict(R=48, L=L, alpha=1.2, metric=COS, mos_degree=2, search=search, out=bufs)
        for _ in range(warmup):
            pkg.merge(subs, Xd, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            off, nb, _, entry = pkg.merge(subs, Xd, **kw)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        st = pkg.stats()
        ids, _ = pkg.search(off, nb, entry, Xd, Qd, 96, 10, metric=COS)
        rec = (ids.to(torch.int64)[:, :, None] == gt.to(torch.int64)[:, None, :]).any(2)
        return dt, st, rec.sum().item() / (10 * Qd.shape[0])

    Xb = pkg.convert(Xd, torch.bfloat16)
    for name, search in [("fp32", None), ("bf16", Xb)]:
        dt, st, rec = timed(search, 96, steps)
        out[name] = {"ms_per_merge": 1000.0 * dt, "value": st["n_source_vertices"] / dt,
                     "unit": "merged vertices/s", "operations": st["n_ops"],
                     "source_vertices": st["n_source_vertices"],
                     "recall_at_10": rec,
                     "prune_path": st["prune_path"],
                     "phase_ms": {"expansion_search": st["ms_search"][0],
                                  "naive_search": st["ms_search"][1],
                                  "sliding_search": st["ms_search"][2],
                                  "prune_and_reverse": st["ms_prune"], "total": st["ms_total"]}}
        log(f"precision {name}: {out[name]}")
    out["bf16_speedup"] = out["bf16"]["value"] / out["fp32"]["value"]
    # equal recall: the bfloat16 form's beam L swept around the float32
    # form's 96; the smallest L whose recall is within 0.002 of float32's
    target = out["fp32"]["recall_at_10"] - 0.002
    sweep = {}
    for L in (80, 88, 96, 104, 112, 128):
        if L == 96:
            sweep[L] = (out["bf16"]["ms_per_merge"], out["bf16"]["recall_at_10"])
            continue
        dt, _, rec = timed(Xb, L, max(1, steps - 1))
        sweep[L] = (1000.0 * dt, rec)
    ok = [L for L in sorted(sweep) if sweep[L][1] >= target]
    Lq = ok[0] if ok else None
    out["bf16_equal_recall"] = {
        "sweep": {str(L): {"ms_per_merge": v[0], "recall_at_10": v[1]} for L, v in sweep.items()},
        "L": Lq,
        "speedup_vs_fp32": None if Lq is None else out["fp32"]["ms_per_merge"] / sweep[Lq][0]}
    log(f"precision bf16 equal recall: {out['bf16_equal_recall']}")
    return out


def exact_ndc(pkg, subs, Xd, wl, search=None):
    """Distance counts of one merge with the probing visited table, which
    evaluates every visited vertex exactly once (the method's own count)."""
    os.environ["RNSM_EXACT_VISITED"] = "1"
    try:
        pkg.merge(subs, Xd, R=wl["R"], L=wl["L"], alpha=wl["alpha"], search=search)
        st = pkg.stats()
    finally:
        del os.environ["RNSM_EXACT_VISITED"]
    assert st["exact_visited"] == 1
    return st["ndc"]


def search_roofline(agg, st, ndc_exact, steps, ms_per_step, form="fp32"):
    """Roofline of the k_beam_search launches (expansion, naive, sliding) of
    merges timed with every launch alone on one stream (agg from an
    RNSM_ONE_STREAM=1 pass): algorithmic bytes (re-evaluations caused by the
    forgetful visited table not counted) and, when the counters match the
    sources, measured HBM bytes, over the exclusive launch time."""
    rb = st["row_bytes"]
    tot_b = tot_ms = 0.0
    per = {}
    for ph in range(3):
        extra = agg["ndc"][ph] - steps * ndc_exact[ph]
        b = agg["bytes"][ph] - extra * rb
        per[PHASES[ph]] = {"algorithmic_gbs": b / (agg["ms"][ph] * 1e6) if agg["ms"][ph] else None,
                           "ms_per_launch": agg["ms"][ph] / max(1, agg["launches"][ph]),
                           "launches_per_step": agg["launches"][ph] / steps,
                           "ndc_inflation": agg["ndc"][ph] / max(1, steps * ndc_exact[ph])}
        tot_b += b
        tot_ms += agg["ms"][ph]
    launches = sum(agg["launches"])
    r = roofline_line(tot_b / launches, tot_ms / launches, launches / steps, ms_per_step,
                      search_traffic(form))
    r["kernel"] = "k_beam_search (expansion, naive and sliding launches)"
    r["per_phase"] = per
    return r


def host_cores():
    """Threads the oracle may use: OMP_NUM_THREADS where set (the CPU share of
    the machine), else the CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl):
    """The oracle's full merge on a replica of the workload with 1/8 of the
    vectors per sub-index (same distribution, dim and parameters; sub-indexes
    built by the oracle), timed on one thread and on all the host cores it may
    use (its searches and prunes of independent vertices spread over them)."""
    from oracle import oracle as O
    from paper_2602_17099_amd import inputs
    n = max(1000, wl["n"] // 8)
    if wl["gen"] == "mixture_u8":
        X = inputs.mixture_u8(2 * n, wl["dim"], seed=inputs.SEED_BASE + 2)
    else:
        X = inputs.tiny_int(2 * n, wl["dim"], seed=inputs.SEED_BASE + 1)
    subs = [O.build_graph(X[i * n:(i + 1) * n], wl["K"], wl["R"], alpha=wl["build_alpha"],
                          reverse=wl["reverse"], alpha_rev=1.2, repair=True) for i in range(2)]
    cores = host_cores()
    times = {}
    prev = O.get_threads()
    try:
        for t in (1, cores):
            O.set_threads(t)
            t0 = time.perf_counter()
            O.merge(subs, X, R=wl["R"], L=wl["L"], alpha=wl["alpha"])
            times[t] = time.perf_counter() - t0
    finally:
        O.set_threads(prev)
    return {"value": n / times[cores], "unit": "merged vertices/s", "cores": cores,
            "kind": "oracle", "value_1_core": n / times[1], "cpu_model": cpu_model(),
            "nproc": os.cpu_count(),
            "sample": f"full oracle merge of a 2 x {n} replica (same distribution, dim "
                      f"{wl['dim']}, R={wl['R']}, L={wl['L']}, alpha={wl['alpha']}): "
                      f"{times[cores]:.1f} s on {cores} threads, {times[1]:.1f} s on 1"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fp32-2x500k", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--calib-copy", action="store_true")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--cm", action="store_true",
                    help="also time the cross-query merge (every vertex a pivot) for comparison")
    ap.add_argument("--incremental", action="store_true",
                    help="also time the incremental scenario: 4 sub-indexes merged one at a time")
    ap.add_argument("--autotune", action="store_true",
                    help="also tune the search shape on the target sub-index and time merges "
                         "under the shape it picks (float32 and bfloat16 copies)")
    ap.add_argument("--multiway", type=float, default=0.0, metavar="SCALE",
                    help="only run the ten-sub-index inner-product workload at SCALE of its "
                         "10,000,000 vectors and print its JSON line")
    ap.add_argument("--precision768", type=float, default=0.0, metavar="SCALE",
                    help="only run the 768-d cosine precision workload at SCALE of its "
                         "4,000,000 vectors (float32 and bfloat16 search copies)")
    ap.add_argument("--calib-only", action="store_true",
                    help="only copy 1 GiB device to device (counter calibration) and exit")
    ap.add_argument("--one-stream", action="store_true",
                    help="every search launch alone on one stream for the whole run (for "
                         "profiles and counters: kernel times are then exclusive)")
    ap.add_argument("--no-rules", action="store_true",
                    help="skip the merges under the other proximity-graph prune rules")
    ap.add_argument("--no-slide-sweep", action="store_true",
                    help="skip the sliding-beam sweep against the cross-query merge")
    ap.add_argument("--no-rebuild", action="store_true",
                    help="skip the rebuild baseline (the builder on the union) and its recall")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched form (operations in rounds, device pivot selection, "
                         "one persistent pivot-group search per round)")
    ap.add_argument("--bf16-only", action="store_true",
                    help="only the bfloat16 form's merges (profiles and counters of its kernels)")
    args = ap.parse_args()
    if args.one_stream:
        os.environ["RNSM_ONE_STREAM"] = "1"
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if args.calib_only:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": a.numel() * 4}))
        return
    import paper_2602_17099_amd as pkg
    pkg.lib()
    if args.precision768 > 0:
        pr = precision768(pkg, args.precision768, max(1, min(args.steps, 3)), args.warmup)
        print(json.dumps({"precision768": pr}), flush=True)
        return
    if args.multiway > 0:
        mw = multiway(pkg, args.multiway, max(1, min(args.steps, 3)), args.warmup)
        print(json.dumps({"multiway": mw}), flush=True)
        return
    wl = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")

    t = time.perf_counter()
    X, Q = make_inputs(wl)
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    log(f"inputs {X.shape} in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    sub_info = {}
    subs = build_subs(pkg, Xd, wl, info=sub_info)
    torch.cuda.synchronize()
    log(f"sub-indexes built in {time.perf_counter() - t:.1f}s "
        f"(edges {[int(s[0][-1]) for s in subs]}, entries {[s[2] for s in subs]})")
    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read, 1 GiB written")

    def exclusive(search, dt_main, agg_main, st_main, steps_main):
        """Merges with every search launch alone on one stream, for the
        roofline's exclusive launch times (the run's own merges when it is
        one-stream already)."""
        if args.one_stream:
            return agg_main, st_main, steps_main
        ex_steps = max(1, min(args.steps, 3))
        os.environ["RNSM_ONE_STREAM"] = "1"
        try:
            _, agg_x, st_x, _ = time_merges(pkg, subs, Xd, wl, ex_steps, 1, search=search)
        finally:
            del os.environ["RNSM_ONE_STREAM"]
        return agg_x, st_x, ex_steps

    gt = None
    if wl["nq"] and not args.no_recall:
        from paper_2602_17099_amd.prepare import knn_l2_exact
        gt = knn_l2_exact(Xd, Qd, 10)

    if args.bf16_only:
        Xb = pkg.convert(Xd, torch.bfloat16)
        ndc_b = exact_ndc(pkg, subs, Xd, wl, search=Xb)
        dtb, aggb, stb, _ = time_merges(pkg, subs, Xd, wl, args.steps, args.warmup, search=Xb)
        ms_b = 1000.0 * dtb / args.steps
        aggx, stx, sx = exclusive(Xb, dtb, aggb, stb, args.steps)
        print(json.dumps({"bf16_form": {"value": args.steps * stb["n_source_vertices"] / dtb,
                                        "ms_per_step": ms_b,
                                        "roofline": search_roofline(aggx, stx, ndc_b, sx, ms_b,
                                                                    "bf16")}}), flush=True)
        return

    ndc_x = exact_ndc(pkg, subs, Xd, wl)
    dt, agg, st, res = time_merges(pkg, subs, Xd, wl, args.steps, args.warmup)
    n_src = st["n_source_vertices"]
    value = args.steps * n_src / dt
    ms_step = 1000.0 * dt / args.steps
    log(f"fp32: {ms_step:.2f} ms/step, {value / 1e6:.3f} M merged vertices/s; stats {st}")
    aggx, stx, sx = exclusive(None, dt, agg, st, args.steps)
    roof = search_roofline(aggx, stx, ndc_x, sx, ms_step, "fp32")
    log(f"fp32 search roofline {roof}")
    off, nb, ds, entry = res
    rec32 = None
    if gt is not None:
        rec32 = recall_at_10(pkg, off, nb, entry, Xd, Qd, gt)
        log(f"fp32 recall@10 (query ef 64) {rec32:.4f}")
    graphs = {"sub_indexes": sub_info, "merged_reachable_frac": pkg.reachable(off, nb, entry) / Xd.shape[0]}
    if gt is not None:
        graphs["merged_recall_at_10_by_ef"] = recall_sweep(pkg, off, nb, entry, Xd, Qd, gt)
        if not args.no_rebuild:
            graphs["rebuild"] = rebuild_baseline(pkg, Xd, Qd, gt, wl)
        if not args.no_slide_sweep:
            graphs["slide_tradeoff"] = slide_tradeoff(pkg, subs, Xd, Qd, gt, wl)
        if not args.no_rules:
            graphs["prune_rules"] = prune_rules(pkg, subs, Xd, Qd, gt, wl)
    log(f"graphs: {graphs}")

    bf16 = None
    if not args.no_bf16:
        Xb = pkg.convert(Xd, torch.bfloat16)  # library staging conversion (RNE)
        ndc_b = exact_ndc(pkg, subs, Xd, wl, search=Xb)
        dtb, aggb, stb, resb = time_merges(pkg, subs, Xd, wl, args.steps, args.warmup, search=Xb)
        vb = args.steps * stb["n_source_vertices"] / dtb
        ms_b = 1000.0 * dtb / args.steps
        recb = recall_at_10(pkg, resb[0], resb[1], resb[3], Xd, Qd, gt) if gt is not None else None
        same = bool(torch.equal(resb[0], off) and torch.equal(resb[1], nb))
        aggbx, stbx, sbx = exclusive(Xb, dtb, aggb, stb, args.steps)
        rb = search_roofline(aggbx, stbx, ndc_b, sbx, ms_b, "bf16")
        bf16 = {"value": vb, "ms_per_step": ms_b, "recall_at_10": recb,
                "phase_ms": {"expansion_search": stb["ms_search"][0],
                             "search_span": stb["ms_search_span"],
                             "prune_and_reverse": stb["ms_prune"], "compact": stb["ms_compact"],
                             "total": stb["ms_total"]},
                "speedup_vs_fp32": vb / value, "same_graph_as_fp32": same,
                "roofline": rb}
        log(f"bf16 search copy: {bf16}")

    # the batched form on the same inputs: same graph, its own time
    batched = None
    if not args.no_batched:
        batched = {}
        forms = [("fp32", None, value)]
        if bf16 is not None:
            forms.append(("bf16", Xb, bf16["value"]))
        for name, search, v_plain in forms:
            dtq, _, stq, resq = time_merges(pkg, subs, Xd, wl, args.steps, args.warmup,
                                            search=search, flags=pkg.FLAG_BATCHED)
            vq = args.steps * stq["n_source_vertices"] / dtq
            batched[name] = {"value": vq, "ms_per_step": 1000.0 * dtq / args.steps,
                             "speedup_vs_plain": vq / v_plain,
                             # against the line's plain float32 form (the same
                             # graph, so at equal recall@10)
                             "speedup_vs_plain_fp32": vq / value,
                             "same_graph": bool(torch.equal(resq[0], off) and
                                                torch.equal(resq[1], nb)),
                             "rounds": stq["n_rounds"],
                             "group_blocks": stq["group_blocks"],
                             "overflow_followers": stq["group_overflow"],
                             "select_rounds": stq["select_rounds"],
                             "phase_ms": {"expansion_search": stq["ms_search"][0],
                                          "order": stq["ms_order"], "select": stq["ms_select"],
                                          "groups": stq["ms_groups"],
                                          "group_search": stq["ms_search"][1],
                                          "overflow_search": stq["ms_search"][2],
                                          "prune_and_reverse": stq["ms_prune"],
                                          "total": stq["ms_total"]}}
        log(f"batched form: {batched}")

    # cross-query merge (every source vertex a pivot: naive searches only, no
    # expansion, greedy or sliding), the comparison the paper makes for RNSM;
    # fewer steps, since each merge runs ~5x the naive searches
    cm = None
    if args.cm:
        cm_steps = max(1, min(args.steps, 2))
        dtc, aggc, stc, resc = time_merges(pkg, subs, Xd, wl, cm_steps, 1,
                                           flags=pkg.FLAG_ALL_PIVOTS)
        vc = cm_steps * stc["n_source_vertices"] / dtc
        recc = recall_at_10(pkg, resc[0], resc[1], resc[3], Xd, Qd, gt) if gt is not None else None
        cm = {"value": vc, "ms_per_step": 1000.0 * dtc / cm_steps, "steps": cm_steps,
              "recall_at_10": recc, "rnsm_speedup": value / vc,
              "naive_searches": stc["queries"][1], "ndc": stc["ndc"][1]}
        log(f"cross-query merge: {cm}")

    tuned = None
    if args.autotune:
        tuned = autotune(pkg, subs, Xd, wl, args, ms_step, off, nb,
                         None if args.no_bf16 else (Xb, bf16["ms_per_step"]))
        log(f"autotuned search shape: {tuned}")

    inc = None
    if args.incremental:
        inc = incremental(pkg, Xd, Qd, gt, wl)
        log(f"incremental merge: {inc}")

    cpu = None
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        cpu = cpu_baseline(wl)
        log(f"cpu baseline in {time.perf_counter() - t:.1f}s: {cpu}")

    line = {
        "metric": "merged vertices/s at equal recall@10 (BF16 vs FP32); search-kernel HBM GB/s vs peak",
        "value": value, "unit": "merged vertices/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload if args.workload != "fp32-2x500k" else
                   "plain FP32: 2 x 500,000 vectors, dim 128, u8-valued mixture, L2SQ, "
                   "R=32, L=64, alpha=1.2",
                   "sub_index_size": wl["n"], "dim": wl["dim"], "R": wl["R"], "L": wl["L"],
                   "alpha": wl["alpha"], "parallelism": "single GPU"},
        "recall_at_10": rec32,
        "roofline": roof,
        "cpu_baseline": cpu,
        "bf16_form": bf16,
        "graphs": graphs,
        "batched_form": batched,
        "cross_query_merge": cm,
        "incremental": inc,
        "autotune": tuned,
        "phase_ms": {"expansion_search": st["ms_search"][0], "invert": st["ms_invert"],
                     "host_plan": st["ms_plan"], "naive_search": st["ms_search"][1],
                     "sliding_search": st["ms_search"][2], "prune_and_reverse": st["ms_prune"],
                     "compact": st["ms_compact"], "total": st["ms_total"]},
        "counts": {"pivots": st["n_pivots"], "followers": st["n_followers"],
                   "expansions": st["expansions"], "queries": st["queries"],
                   "reverse_edges": st["n_reverse_edges"], "ndc_exact": ndc_x,
                   "ndc_timed": st["ndc"], "visited_table_evictions": st["hash_evictions"]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
