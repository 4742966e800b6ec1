"""ctypes binding of the CPU reference (``rnsm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU baseline leg of the benchmark. The product package never imports it.

``build()`` compiles the C source with gcc into ``liboracle.so`` next to it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rnsm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# a test may point this at a deliberately broken copy of the oracle
_LIB_OVERRIDE = os.environ.get("RNSM_ORACLE_LIB")

L2SQ, IP, COSINE = 0, 1, 2
METRICS = {"l2sq": L2SQ, "ip": IP, "cosine": COSINE}

_lib = None


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall",
           "-Wno-unused-function", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            _lib = C.CDLL(_LIB_OVERRIDE)
            _setup(_lib)
            return _lib
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB)
        _setup(_lib)
    return _lib


class Params(C.Structure):
    _fields_ = [("R", C.c_int), ("ef_naive", C.c_int), ("ef_slide", C.c_int),
                ("alpha", C.c_float), ("metric", C.c_int), ("k", C.c_int), ("kplus", C.c_int),
                ("mos_degree", C.c_int), ("mos_diameter", C.c_int),
                ("use_centroids", C.c_int), ("all_pivots", C.c_int),
                ("prune_rule", C.c_int), ("prune_param", C.c_float)]


class Trace(C.Structure):
    _fields_ = [("nk", C.c_void_p), ("pivot_of", C.c_void_p), ("res_ids", C.c_void_p),
                ("res_d", C.c_void_p), ("ndc_expand", C.c_int64), ("ndc_naive", C.c_int64),
                ("ndc_slide", C.c_int64), ("n_pivots", C.c_int64)]


def _setup(L):
    P = C.c_void_p
    L.orc_set_threads.restype = None
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_get_threads.restype = C.c_int
    L.orc_get_threads.argtypes = []
    L.orc_dist_vec.restype = C.c_double
    L.orc_dist_vec.argtypes = [P, P, C.c_int, C.c_int, C.c_double, C.c_double]
    L.orc_beam_search.restype = C.c_int
    L.orc_beam_search.argtypes = [C.c_int64, P, P, C.c_int64, P, C.c_int, C.c_int, P, P, P,
                                  C.c_int, C.c_int, P, P, P]
    L.orc_prune.restype = C.c_int
    L.orc_prune.argtypes = [C.c_int64, P, C.c_int, P, C.c_int, C.c_int, P, C.c_float, C.c_int,
                            P, P]
    L.orc_expand_range.restype = C.c_int
    L.orc_expand_range.argtypes = [C.c_int64, P, P, C.c_int64, P, C.c_int, C.c_int, P, C.c_int,
                                   C.c_int, C.c_int64, C.c_int64, P]
    L.orc_expand.restype = C.c_int
    L.orc_expand.argtypes = [C.c_int64, P, P, C.c_int64, P, C.c_int, C.c_int, P, C.c_int,
                             C.c_int, P]
    L.orc_invert.restype = C.c_int
    L.orc_invert.argtypes = [C.c_int64, P, C.c_int, P, P]
    L.orc_pivots.restype = C.c_int
    L.orc_pivots.argtypes = [C.c_int64, P, P, P, P, P]
    L.orc_mos_cost.restype = None
    L.orc_mos_cost.argtypes = [C.c_int, P, C.c_int, P]
    L.orc_mos.restype = C.c_int
    L.orc_mos.argtypes = [C.c_int, P, C.c_int, C.c_int, P, C.c_int, P, P]
    L.orc_plan.restype = C.c_int
    L.orc_plan.argtypes = [C.c_int, P, P, C.c_int, C.c_int, C.c_int, P, C.c_int, P, P]
    L.orc_plan_cost.restype = C.c_int
    L.orc_plan_cost.argtypes = [C.c_int, P, P, C.c_int, C.c_int, P, C.c_int, P, P]
    L.orc_merge.restype = C.c_int
    L.orc_merge.argtypes = [C.c_int, P, P, P, P, P, C.c_int, P, P, P, P, P, P, P, P]
    L.orc_prune_rule.restype = C.c_int
    L.orc_prune_rule.argtypes = [C.c_int64, P, C.c_int, P, C.c_int, C.c_int, P, C.c_int, C.c_float,
                                 C.c_float, C.c_int, P, P]
    L.orc_knn.restype = C.c_int
    L.orc_knn.argtypes = [C.c_int64, P, C.c_int, C.c_int, C.c_int, P]
    L.orc_knn_queries.restype = C.c_int
    L.orc_knn_queries.argtypes = [C.c_int64, P, C.c_int64, P, C.c_int, C.c_int, C.c_int, P, P]
    L.orc_build.restype = C.c_int
    L.orc_build.argtypes = [C.c_int64, P, C.c_int, C.c_int, P, C.c_int, C.c_int, C.c_float,
                            C.c_int, C.c_float, P, P, P]
    L.orc_norms.restype = None
    L.orc_norms.argtypes = [P, C.c_int64, C.c_int, P]
    L.orc_reachable.restype = C.c_int64
    L.orc_reachable.argtypes = [C.c_int64, P, P, C.c_int32]
    L.orc_repair.restype = C.c_int64
    L.orc_repair.argtypes = [C.c_int64, P, C.c_int, C.c_int, C.c_int, P, P, C.c_int32]


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


def _i32(x):
    return np.ascontiguousarray(x, dtype=np.int32)


def _i64(x):
    return np.ascontiguousarray(x, dtype=np.int64)


def set_threads(n: int) -> None:
    """Threads of the loops over independent vertices (searches, prunes,
    k-NN rows); results do not depend on it."""
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def norms(X: np.ndarray) -> np.ndarray:
    X = _f32(X)
    out = np.empty(X.shape[0], dtype=np.float64)
    lib().orc_norms(_p(X), X.shape[0], X.shape[1], _p(out))
    return out


def dist(a, b, metric: int = L2SQ) -> float:
    a = _f32(a)
    b = _f32(b)
    na = float(np.sqrt((a.astype(np.float64) ** 2).sum()))
    nb = float(np.sqrt((b.astype(np.float64) ** 2).sum()))
    return lib().orc_dist_vec(_p(a), _p(b), a.shape[0], metric, na, nb)


def beam_search(offsets, nbrs, X, q, seeds, ef, metric=L2SQ, base=0, n=None):
    """Algorithm 1 on the graph (offsets, nbrs) whose vertex v is row base+v of X."""
    offsets, nbrs, X, q, seeds = _i64(offsets), _i32(nbrs), _f32(X), _f32(q), _i32(seeds)
    n = len(offsets) - 1 if n is None else n
    nrm = norms(X) if metric == COSINE else None
    ids = np.empty(max(ef, len(seeds)), dtype=np.int32)
    ds = np.empty(max(ef, len(seeds)), dtype=np.float64)
    ndc = np.zeros(1, dtype=np.int64)
    c = lib().orc_beam_search(n, _p(offsets), _p(nbrs), base, _p(X), X.shape[1], metric, _p(nrm),
                              _p(q), _p(seeds), len(seeds), ef, _p(ids), _p(ds), _p(ndc))
    return ids[:c].copy(), ds[:c].copy(), int(ndc[0])


def prune(p, W, X, alpha, R, metric=L2SQ):
    W, X = _i32(W), _f32(X)
    nrm = norms(X) if metric == COSINE else None
    ids = np.empty(max(1, len(W)), dtype=np.int32)
    ds = np.empty(max(1, len(W)), dtype=np.float64)
    c = lib().orc_prune(p, _p(W), len(W), _p(X), X.shape[1], metric, _p(nrm), float(alpha), R,
                        _p(ids), _p(ds))
    return ids[:c].copy(), ds[:c].copy()


def prune_rule(p, W, X, rule, R, alpha=1.0, param=0.0, metric=L2SQ):
    """Prune(p, W) under a proximity-graph rule: PRUNE_ALPHA (alpha), PRUNE_ANGLE
    (SSG, param = theta in degrees), PRUNE_TAU (tau-MNG, param = tau)."""
    W, X = _i32(W), _f32(X)
    nrm = norms(X) if metric == COSINE else None
    ids = np.empty(max(1, len(W)), dtype=np.int32)
    ds = np.empty(max(1, len(W)), dtype=np.float64)
    c = lib().orc_prune_rule(p, _p(W), len(W), _p(X), X.shape[1], metric, _p(nrm), int(rule),
                             float(alpha), float(param), R, _p(ids), _p(ds))
    return ids[:c].copy(), ds[:c].copy()


def expand(offsets, nbrs, X, k, kplus, metric=L2SQ, base=0, threads=1):
    """N_k of every vertex ([n x k], -1 padded), its independent searches
    spread over `threads` threads."""
    offsets, nbrs, X = _i64(offsets), _i32(nbrs), _f32(X)
    n = len(offsets) - 1
    nrm = norms(X) if metric == COSINE else None
    out = np.empty((n, k), dtype=np.int32)
    prev = get_threads()
    set_threads(max(1, threads))
    try:
        rc = lib().orc_expand(n, _p(offsets), _p(nbrs), base, _p(X), X.shape[1], metric, _p(nrm),
                              k, kplus, _p(out))
    finally:
        set_threads(prev)
    if rc != 0:
        raise RuntimeError("orc_expand failed")
    return out


def invert(nk):
    nk = _i32(nk)
    n, k = nk.shape
    off = np.empty(n + 1, dtype=np.int64)
    ids = np.empty(max(1, n * k), dtype=np.int32)
    lib().orc_invert(n, _p(nk), k, _p(off), _p(ids))
    return off, ids[: off[-1]].copy()


def pivots(rk_off, rk_ids):
    rk_off, rk_ids = _i64(rk_off), _i32(rk_ids)
    n = len(rk_off) - 1
    piv = np.empty(n, dtype=np.int32)
    order = np.empty(max(1, n), dtype=np.int32)
    npiv = np.zeros(1, dtype=np.int64)
    lib().orc_pivots(n, _p(rk_off), _p(rk_ids), _p(piv), _p(order), _p(npiv))
    return piv, order[: npiv[0]].copy()


def mos_cost(m, centroids=None):
    C_ = np.empty((m, m), dtype=np.float64)
    cen = None if centroids is None else np.ascontiguousarray(centroids, dtype=np.float64)
    lib().orc_mos_cost(m, _p(cen), 0 if cen is None else cen.shape[1], _p(C_))
    return C_


def mos(cost, R, delta=2):
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    m = cost.shape[0]
    cap = m * m
    edges = np.empty((cap, 2), dtype=np.int32)
    ne = np.zeros(1, dtype=np.int32)
    nf = np.zeros(1, dtype=np.int32)
    rc = lib().orc_mos(m, _p(cost), R, delta, _p(edges), cap, _p(ne), _p(nf))
    if rc != 0:
        raise ValueError(f"orc_mos failed: {rc}")
    return [tuple(int(v) for v in e) for e in edges[: ne[0]]], int(nf[0])


def plan(sizes, R, delta=2, centroids=None):
    """Operations (source, target) in execution order and the fallback count."""
    sizes = _i64(sizes)
    m = len(sizes)
    cen = None if centroids is None else np.ascontiguousarray(centroids, dtype=np.float64)
    ops = np.zeros((max(1, m * m), 2), dtype=np.int32)
    n = np.zeros(1, dtype=np.int32)
    nf = np.zeros(1, dtype=np.int32)
    rc = lib().orc_plan(m, _p(sizes), _p(cen), 0 if cen is None else cen.shape[1], R, delta,
                        _p(ops), m * m, _p(n), _p(nf))
    if rc != 0:
        raise ValueError(f"orc_plan failed: {rc}")
    return [tuple(int(v) for v in o) for o in ops[: n[0]]], int(nf[0])


def plan_cost(sizes, cost, R, delta=2):
    """Operations (source, target) in execution order from a cost matrix."""
    sizes = _i64(sizes)
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    m = len(sizes)
    ops = np.zeros((max(1, m * m), 2), dtype=np.int32)
    n = np.zeros(1, dtype=np.int32)
    nf = np.zeros(1, dtype=np.int32)
    rc = lib().orc_plan_cost(m, _p(sizes), _p(cost), R, delta, _p(ops), m * m, _p(n), _p(nf))
    if rc != 0:
        raise ValueError(f"orc_plan_cost failed: {rc}")
    return [tuple(int(v) for v in o) for o in ops[: n[0]]], int(nf[0])


PRUNE_ALPHA, PRUNE_ANGLE, PRUNE_TAU = 0, 1, 2


def merge(subs, X, R, L, alpha, metric=L2SQ, k=5, kplus=16, ef_slide=None, mos_degree=0,
          mos_diameter=2, use_centroids=False, all_pivots=False, trace=False,
          prune_rule=PRUNE_ALPHA, prune_param=0.0):
    """Whole merge. subs: list of (offsets, nbrs, entry) with local ids, in
    global-id order over the rows of X. Returns a dict with the merged CSR
    (global ids), FP64 edge distances, merged entry, operations and trace."""
    X = _f32(X)
    m = len(subs)
    sizes = _i64([len(s[0]) - 1 for s in subs])
    assert sizes.sum() == X.shape[0]
    offs = _i64(np.concatenate([_i64(s[0]) for s in subs]))
    nbrs = _i32(np.concatenate([_i32(s[1]) for s in subs])) if sum(len(s[1]) for s in subs) else np.zeros(1, np.int32)
    entries = _i32([s[2] for s in subs])
    P = Params(R=R, ef_naive=L, ef_slide=L if ef_slide is None else ef_slide, alpha=float(alpha),
               metric=metric, k=k, kplus=kplus, mos_degree=mos_degree, mos_diameter=mos_diameter,
               use_centroids=int(use_centroids), all_pivots=int(all_pivots),
               prune_rule=int(prune_rule), prune_param=float(prune_param))
    N = X.shape[0]
    rows = np.full((N, R), -1, dtype=np.int32)
    dists = np.full((N, R), np.inf, dtype=np.float64)
    deg = np.zeros(N, dtype=np.int32)
    entry = np.zeros(1, dtype=np.int32)
    ops = np.zeros((max(1, m * m), 2), dtype=np.int32)
    nops = np.zeros(1, dtype=np.int32)
    tr = Trace()
    keep = []
    if trace and m >= 2:
        # the first operation's source is only known after planning; size
        # the trace buffers for the largest sub-index
        nmax = int(sizes.max())
        res_w = max(L, P.ef_slide)
        t_nk = np.full((nmax, k), -1, dtype=np.int32)
        t_piv = np.full(nmax, -2, dtype=np.int32)
        t_ri = np.full((nmax, res_w), -1, dtype=np.int32)
        t_rd = np.full((nmax, res_w), np.inf, dtype=np.float64)
        keep = [t_nk, t_piv, t_ri, t_rd]
        tr.nk, tr.pivot_of, tr.res_ids, tr.res_d = (a.ctypes.data for a in keep)
    rc = lib().orc_merge(m, _p(sizes), _p(offs), _p(nbrs), _p(entries), _p(X), X.shape[1],
                         C.byref(P), _p(rows), _p(dists), _p(deg), _p(entry), _p(ops), _p(nops),
                         C.byref(tr) if trace else None)
    if rc != 0:
        raise ValueError(f"orc_merge failed: {rc}")
    offsets = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(deg, out=offsets[1:])
    mask = np.arange(R)[None, :] < deg[:, None]
    out = {
        "offsets": offsets,
        "nbrs": rows[mask].astype(np.int32),
        "dists": dists[mask],
        "entry": int(entry[0]),
        "ops": [tuple(int(v) for v in o) for o in ops[: nops[0]]],
        "rows": rows, "deg": deg,
    }
    if trace and m >= 2:
        s0 = out["ops"][0][0]
        ns = int(sizes[s0])
        out["trace"] = {"nk": t_nk[:ns], "pivot_of": t_piv[:ns], "res_ids": t_ri[:ns],
                        "res_d": t_rd[:ns], "ndc_expand": tr.ndc_expand,
                        "ndc_naive": tr.ndc_naive, "ndc_slide": tr.ndc_slide,
                        "n_pivots": tr.n_pivots, "source": s0}
    return out


def knn(X, K, metric=L2SQ):
    """Exact K-NN of every row (excluding itself) by (d, id), brute force in C."""
    X = _f32(X)
    n = X.shape[0]
    out = np.empty((n, K), dtype=np.int32)
    lib().orc_knn(n, _p(X), X.shape[1], metric, K, _p(out))
    return out


def knn_fast(X, K, metric=L2SQ, block=2048):
    """Same result as ``knn`` for larger n: candidate distances from a float64
    matrix product (exact when every value is an integer), then for float data
    the 2K best candidates are re-ranked by the direct double-precision
    distance. Rows are ordered by (d, id)."""
    X = _f32(X)
    n = X.shape[0]
    X64 = X.astype(np.float64)
    integral = bool(np.all(X64 == np.rint(X64))) and metric == L2SQ
    sq = (X64 * X64).sum(1)
    nrm = np.sqrt(sq)
    out = np.empty((n, K), dtype=np.int32)
    ids_all = np.arange(n, dtype=np.int64)
    for s in range(0, n, block):
        e = min(n, s + block)
        G = X64[s:e] @ X64.T
        if metric == L2SQ:
            D = sq[s:e, None] + sq[None, :] - 2.0 * G
        elif metric == IP:
            D = 1.0 - G
        else:
            D = 1.0 - G / (nrm[s:e, None] * nrm[None, :])
        if integral:
            D[np.arange(e - s), np.arange(s, e)] = 0.0
            key = np.rint(D).astype(np.int64)
            key[np.arange(e - s), np.arange(s, e)] = np.iinfo(np.int64).max // (n + 1)
            key = key * n + ids_all[None, :]
            part = np.argpartition(key, K - 1, axis=1)[:, :K]
            kk = np.take_along_axis(key, part, 1)
            o = np.argsort(kk, axis=1)
            out[s:e] = np.take_along_axis(part, o, 1)
        else:
            D[np.arange(e - s), np.arange(s, e)] = np.inf
            M = min(n - 1, 2 * K + 8)
            part = np.argpartition(D, M - 1, axis=1)[:, :M]
            for r in range(e - s):
                v = s + r
                cand = part[r]
                cand = cand[cand != v]
                dd = np.array([dist(X[v], X[c], metric) for c in cand])
                o = np.lexsort((cand, dd))
                out[v] = cand[o][:K]
    return out


def knn_queries(X, Q, K, metric=L2SQ):
    X, Q = _f32(X), _f32(Q)
    ids = np.empty((Q.shape[0], K), dtype=np.int32)
    ds = np.empty((Q.shape[0], K), dtype=np.float64)
    lib().orc_knn_queries(X.shape[0], _p(X), Q.shape[0], _p(Q), X.shape[1], metric, K, _p(ids),
                          _p(ds))
    return ids, ds


def build_graph(X, K, R, alpha=1.0, reverse=False, alpha_rev=1.2, metric=L2SQ, knn_ids=None,
                repair=False, return_links=False):
    """Sub-index builder: exact K-NN -> prune(alpha) to R [-> reverse edges
    and prune(alpha_rev)] -> entry closest to the centroid [-> reachability
    repair: every vertex the entry cannot reach is linked in from its
    nearest reached vertex].
    Returns (offsets int64, nbrs int32 local, entry) [, links added]."""
    X = _f32(X)
    n = X.shape[0]
    if knn_ids is None:
        knn_ids = knn(X, K, metric) if n <= 1500 else knn_fast(X, K, metric)
    knn_ids = _i32(knn_ids)
    offs = np.empty(n + 1, dtype=np.int64)
    nb = np.empty(max(1, n * R), dtype=np.int32)
    entry = np.zeros(1, dtype=np.int32)
    links = lib().orc_build(n, _p(X), X.shape[1], metric, _p(knn_ids), knn_ids.shape[1], R,
                            float(alpha), (1 if reverse else 0) | (2 if repair else 0),
                            float(alpha_rev), _p(offs), _p(nb), _p(entry))
    out = (offs, nb[: offs[-1]].copy(), int(entry[0]))
    return out + (int(links),) if return_links else out


def repair(X, rows, R, entry, metric=L2SQ):
    """The builder's reachability repair applied to `rows` (lists of ids, at
    most R each); returns (new rows, links added)."""
    X = _f32(X)
    n = X.shape[0]
    pad = np.full((n, R), -1, dtype=np.int32)
    deg = np.zeros(n, dtype=np.int32)
    for v, r in enumerate(rows):
        pad[v, :len(r)] = r
        deg[v] = len(r)
    links = lib().orc_repair(n, _p(X), X.shape[1], metric, R, _p(pad), _p(deg), int(entry))
    return [pad[v, :deg[v]].tolist() for v in range(n)], int(links)


def reachable(offsets, nbrs, entry):
    """Vertices reachable from the entry along the graph's edges (entry included)."""
    offsets, nbrs = _i64(offsets), _i32(nbrs)
    n = len(offsets) - 1
    return int(lib().orc_reachable(n, _p(offsets), _p(nbrs if len(nbrs) else np.zeros(1, np.int32)),
                                   int(entry)))


def search_graph(offsets, nbrs, X, Q, entry, ef, topk=10, metric=L2SQ):
    """Evaluator: beam search of every query from the entry, top-k ids."""
    offsets, nbrs, X, Q = _i64(offsets), _i32(nbrs), _f32(X), _f32(Q)
    out = np.full((Q.shape[0], topk), -1, dtype=np.int32)
    for i in range(Q.shape[0]):
        ids, _, _ = beam_search(offsets, nbrs, X, Q[i], [entry], max(ef, topk), metric)
        out[i, : min(topk, len(ids))] = ids[:topk]
    return out


def recall_at_k(found, truth, k=10):
    """Recall@K = |AKNN(q) & KNN(q)| / k averaged over queries (eq. recall_at_k)."""
    tot = 0
    for f, t in zip(found, truth):
        tot += len(set(int(v) for v in f[:k] if v >= 0) & set(int(v) for v in t[:k]))
    return tot / (k * len(found))


def to_bf16_bits(x):
    """float32 -> bfloat16 bit patterns (uint16) by the definition of round to
    nearest, ties to even: of the two bfloat16 values that bracket |x| (x
    with its low 16 bits cleared, and that value plus one bfloat16 ulp, the
    ulp taken past the largest finite value too), take the nearer in exact
    float64 arithmetic, on a tie the one whose last bit is 0. A value nearer
    2^128 than the largest finite bfloat16 becomes infinity; NaN gives a NaN
    pattern (0x7fc0 with the sign)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    sign = (u >> 31) & 1
    lo_mag = (u & 0x7FFFFFFF) & 0x7FFF0000
    lo_val = lo_mag.astype(np.uint32).view(np.float32).astype(np.float64)
    e = (lo_mag >> 23) & 0xFF
    ulp = np.where(e == 0, 2.0 ** -133, np.exp2(e.astype(np.float64) - 134.0))
    with np.errstate(invalid="ignore"):
        xv = np.abs(x.astype(np.float64))
        d_lo = xv - lo_val
        d_hi = (lo_val + ulp) - xv
        lo16 = lo_mag >> 16
        up = (d_hi < d_lo) | ((d_hi == d_lo) & ((lo16 & 1) == 1))
    r = (lo16 + up.astype(np.uint64)) | (sign << 15)
    r = np.where(np.isnan(x), 0x7FC0 | (sign << 15), r)
    return r.astype(np.uint16)


def bf16_bits_to_f32(b):
    """bfloat16 bit patterns -> float32 values (exact)."""
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32)
