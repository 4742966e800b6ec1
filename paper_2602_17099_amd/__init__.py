"""Python binding of librnsm (include/rnsm.h): argument marshalling only.

Every step of the merge runs in the HIP library; PyTorch only provides device
memory (tensors) and streams. If the library has not been built the calls
raise: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librnsm.so")

L2SQ, IP, COSINE = 0, 1, 2
F32, BF16, F16 = 0, 1, 2
FLAG_ALL_PIVOTS = 1
FLAG_CENTROID_COSTS = 2
FLAG_AUTOTUNE = 4
FLAG_HOST_OUT = 8
FLAG_NO_STATS = 16
FLAG_BATCHED = 32
PRUNE_ALPHA, PRUNE_ANGLE, PRUNE_TAU = 0, 1, 2
DEVICE, HOST = 0, 1

SYMBOLS = ["rnsm_merge", "rnsm_merge_simple", "mos_plan", "rnsm_select_pivots", "rnsm_search",
           "rnsm_search_noalloc", "rnsm_tune_search", "rnsm_build_graph", "rnsm_convert",
           "rnsm_get_stats", "rnsm_last_error", "rnsm_csr_free", "rnsm_select_pivots_device",
           "rnsm_reachable"]

_lib = None


class RnsmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"librnsm status {status}: {msg}")
        self.status = status


class Graph(C.Structure):
    _fields_ = [("n", C.c_int64), ("offsets", C.c_void_p), ("nbrs", C.c_void_p),
                ("entry", C.c_int32), ("mem", C.c_int)]


class Vectors(C.Structure):
    _fields_ = [("n", C.c_int64), ("dim", C.c_int32), ("f32", C.c_void_p),
                ("search_dtype", C.c_int), ("search", C.c_void_p), ("row_stride", C.c_int64),
                ("mem", C.c_int)]


class Params(C.Structure):
    _fields_ = [("R", C.c_int32), ("L", C.c_int32), ("alpha", C.c_float), ("metric", C.c_int),
                ("k_reverse", C.c_int32), ("k_expand", C.c_int32), ("ef_naive", C.c_int32),
                ("ef_slide", C.c_int32), ("mos_degree", C.c_int32), ("mos_diameter", C.c_int32),
                ("flags", C.c_uint32), ("stream", C.c_void_p),
                ("search_hash_bits", C.c_int32), ("search_waves_per_block", C.c_int32),
                ("max_device_bytes", C.c_int64), ("prune_rule", C.c_int32),
                ("prune_param", C.c_float)]


class SearchTuning(C.Structure):
    _fields_ = [("hash_bits", C.c_int32), ("waves_per_block", C.c_int32), ("ms", C.c_float),
                ("default_hash_bits", C.c_int32), ("default_waves_per_block", C.c_int32),
                ("default_ms", C.c_float), ("n_queries", C.c_int64), ("n_tried", C.c_int32)]


class Csr(C.Structure):
    _fields_ = [("offsets", C.c_void_p), ("nbrs", C.c_void_p), ("dists", C.c_void_p),
                ("entry", C.c_int32), ("n_edges", C.c_int64), ("mem", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("ms_total", C.c_double), ("ms_search", C.c_double * 3), ("ms_invert", C.c_double),
                ("ms_plan", C.c_double), ("ms_prune", C.c_double), ("ms_compact", C.c_double),
                ("n_ops", C.c_int64), ("n_source_vertices", C.c_int64), ("n_pivots", C.c_int64),
                ("n_followers", C.c_int64), ("n_reverse_edges", C.c_int64),
                ("queries", C.c_int64 * 3), ("ndc", C.c_int64 * 3), ("expansions", C.c_int64 * 3),
                ("adjacency", C.c_int64 * 3), ("launches", C.c_int64 * 3), ("bytes", C.c_double * 3),
                ("hash_evictions", C.c_int64), ("row_bytes", C.c_int32),
                ("exact_visited", C.c_int32), ("prune_path", C.c_int32),
                ("ms_search_span", C.c_double), ("search_hash_bits", C.c_int32),
                ("search_waves_per_block", C.c_int32), ("prune_rechecks", C.c_int64),
                ("n_rounds", C.c_int64), ("group_blocks", C.c_int64),
                ("group_overflow", C.c_int64), ("ms_order", C.c_double),
                ("ms_select", C.c_double), ("select_rounds", C.c_int64),
                ("ms_groups", C.c_double)]


def lib():
    """Load librnsm.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2602_17099_amd/build.py "
                               "(or __graft_entry__.build()) first")
        # torch first: its bundled HIP runtime carries the soname the library
        # links against, so the library binds to that one copy; loaded the
        # other way round, the process would hold two HIP runtimes and the
        # second would find no device
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.rnsm_merge.restype = C.c_int
        L.rnsm_merge.argtypes = [C.c_int32, P, P, P, P]
        L.rnsm_merge_simple.restype = C.c_int
        L.rnsm_merge_simple.argtypes = [C.c_int32, P, P, C.c_int32, C.c_int32, C.c_float, P]
        L.mos_plan.restype = C.c_int
        L.mos_plan.argtypes = [C.c_int32, P, P, C.c_int32, C.c_int32, C.c_int32, P, C.c_int32, P, P]
        L.rnsm_select_pivots.restype = C.c_int
        L.rnsm_select_pivots.argtypes = [C.c_int64, P, P, P, P, P, P, P]
        L.rnsm_tune_search.restype = C.c_int
        L.rnsm_tune_search.argtypes = [P, P, C.c_int32, C.c_int, C.c_int64, P, P]
        L.rnsm_search.restype = C.c_int
        L.rnsm_search.argtypes = [P, P, P, C.c_int64, P, C.c_int32, C.c_int32, C.c_int32, C.c_int,
                                  P, P, P]
        L.rnsm_search_noalloc.restype = C.c_int
        L.rnsm_search_noalloc.argtypes = L.rnsm_search.argtypes
        L.rnsm_build_graph.restype = C.c_int
        L.rnsm_build_graph.argtypes = [C.c_int64, P, C.c_int32, C.c_int, P, C.c_int32, C.c_int32,
                                       C.c_float, C.c_int32, C.c_float, P, P, P, P, P]
        L.rnsm_reachable.restype = C.c_int
        L.rnsm_reachable.argtypes = [C.c_int64, P, P, C.c_int32, P, P]
        L.rnsm_convert.restype = C.c_int
        L.rnsm_convert.argtypes = [P, C.c_int, P, C.c_int, C.c_int64, P]
        L.rnsm_get_stats.restype = C.c_int
        L.rnsm_get_stats.argtypes = [P]
        L.rnsm_last_error.restype = C.c_char_p
        L.rnsm_last_error.argtypes = []
        L.rnsm_select_pivots_device.restype = C.c_int
        L.rnsm_select_pivots_device.argtypes = [C.c_int64, P, P, P, P, P]
        L.rnsm_csr_free.restype = None
        L.rnsm_csr_free.argtypes = [P]
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        raise RnsmError(st, lib().rnsm_last_error().decode())


def last_error() -> str:
    return lib().rnsm_last_error().decode()


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _vectors(X, search=None):
    """Device rows: contiguous, or rows with unit column stride and a row
    stride (e.g. a column slice of a wider matrix), passed as row_stride."""
    import torch
    assert X.is_cuda and X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1
    v = Vectors(n=X.shape[0], dim=X.shape[1], f32=X.data_ptr(), search_dtype=F32, search=None,
                row_stride=X.stride(0) if X.shape[0] > 1 else 0, mem=DEVICE)
    if search is not None:
        assert search.is_cuda and search.shape == X.shape and search.stride() == X.stride()
        v.search_dtype = BF16 if search.dtype == torch.bfloat16 else F16
        assert search.dtype in (torch.bfloat16, torch.float16)
        v.search = search.data_ptr()
    return v


def merge(subs, X, R, L, alpha, metric=L2SQ, search=None, k=0, kplus=0, ef_naive=0,
          ef_slide=0, mos_degree=0, mos_diameter=0, flags=0, dists=True, stream=None,
          out=None, search_shape=None, max_device_bytes=0, prune_rule=0, prune_param=0.0):
    """Merge sub-indexes. subs: list of (offsets int64, nbrs int32, entry) device
    tensors with local ids, in global-id order over the rows of X (float32
    device [N, dim]). search: optional bf16/f16 copy of X that the searches
    read. search_shape: optional (hash_bits, waves_per_block) of the beam
    searches, e.g. from tune_search. Returns (offsets, nbrs, dists, entry)
    device tensors (global ids)."""
    import torch
    m = len(subs)
    gs = (Graph * m)()
    for i, (o, nb, e) in enumerate(subs):
        assert o.dtype == torch.int64 and nb.dtype == torch.int32 and o.is_cuda and nb.is_cuda
        gs[i] = Graph(n=o.shape[0] - 1, offsets=o.data_ptr(), nbrs=nb.data_ptr(), entry=int(e))
    v = _vectors(X, search)
    N = X.shape[0]
    dev = X.device
    if out is None:
        out = (torch.empty(N + 1, dtype=torch.int64, device=dev),
               torch.empty(N * R, dtype=torch.int32, device=dev),
               torch.empty(N * R, dtype=torch.float32, device=dev) if dists else None)
    o_off, o_nb, o_d = out
    csr = Csr(offsets=o_off.data_ptr(), nbrs=o_nb.data_ptr(),
              dists=None if o_d is None else o_d.data_ptr())
    p = Params(R=R, L=L, alpha=float(alpha), metric=metric, k_reverse=k, k_expand=kplus,
               ef_naive=ef_naive, ef_slide=ef_slide, mos_degree=mos_degree,
               mos_diameter=mos_diameter, flags=flags, stream=_stream(stream),
               max_device_bytes=int(max_device_bytes), prune_rule=int(prune_rule),
               prune_param=float(prune_param))
    if search_shape is not None:
        p.search_hash_bits, p.search_waves_per_block = (int(x) for x in search_shape)
    _check(lib().rnsm_merge(m, gs, C.byref(v), C.byref(p), C.byref(csr)))
    ne = int(csr.n_edges)
    return o_off, o_nb[:ne], (None if o_d is None else o_d[:ne]), int(csr.entry)


def merge_host(subs, X, R, L, alpha, metric=L2SQ, search=None, flags=0, **kw):
    """Merge from host (numpy) inputs into library-allocated host output:
    graphs and rows with mem = RNSM_HOST, RNSM_FLAG_HOST_OUT, the arrays
    copied out and released with rnsm_csr_free. subs: list of (offsets int64,
    nbrs int32, entry) numpy arrays; X: float32 [N, dim] (any row stride);
    search: optional numpy bfloat16-bits (uint16) / float16 copy of X.
    Returns (offsets, nbrs, dists, entry) numpy arrays (global ids)."""
    import numpy as np
    m = len(subs)
    keep = []
    gs = (Graph * m)()
    for i, (o, nb, e) in enumerate(subs):
        o = np.ascontiguousarray(o, dtype=np.int64)
        nb = np.ascontiguousarray(nb, dtype=np.int32)
        keep += [o, nb]
        gs[i] = Graph(n=o.shape[0] - 1, offsets=o.ctypes.data, nbrs=nb.ctypes.data if nb.size else None,
                      entry=int(e), mem=HOST)
    assert X.dtype == np.float32 and X.ndim == 2 and X.strides[1] == 4
    v = Vectors(n=X.shape[0], dim=X.shape[1], f32=X.ctypes.data, search_dtype=F32, search=None,
                row_stride=X.strides[0] // 4, mem=HOST)
    if search is not None:
        assert search.shape == X.shape and search.strides[1] == 2
        assert search.strides[0] // 2 == X.strides[0] // 4
        v.search_dtype = F16 if search.dtype == np.float16 else BF16
        v.search = search.ctypes.data
    p = Params(R=R, L=L, alpha=float(alpha), metric=metric, flags=flags | FLAG_HOST_OUT,
               stream=_stream(kw.pop("stream", None)), **kw)
    csr = Csr()
    _check(lib().rnsm_merge(m, gs, C.byref(v), C.byref(p), C.byref(csr)))
    try:
        assert csr.mem == HOST
        N = X.shape[0]
        ne = int(csr.n_edges)
        off = np.ctypeslib.as_array((C.c_int64 * (N + 1)).from_address(csr.offsets)).copy()
        nb = np.ctypeslib.as_array((C.c_int32 * max(ne, 1)).from_address(csr.nbrs))[:ne].copy()
        ds = np.ctypeslib.as_array((C.c_float * max(ne, 1)).from_address(csr.dists))[:ne].copy()
        return off, nb, ds, int(csr.entry)
    finally:
        lib().rnsm_csr_free(C.byref(csr))


def merge_simple(subs, X, R, L, alpha, stream=None):
    import torch
    m = len(subs)
    gs = (Graph * m)()
    for i, (o, nb, e) in enumerate(subs):
        gs[i] = Graph(n=o.shape[0] - 1, offsets=o.data_ptr(), nbrs=nb.data_ptr(), entry=int(e))
    v = _vectors(X)
    N = X.shape[0]
    o_off = torch.empty(N + 1, dtype=torch.int64, device=X.device)
    o_nb = torch.empty(N * R, dtype=torch.int32, device=X.device)
    csr = Csr(offsets=o_off.data_ptr(), nbrs=o_nb.data_ptr(), dists=None)
    _check(lib().rnsm_merge_simple(m, gs, C.byref(v), R, L, float(alpha), C.byref(csr)))
    return o_off, o_nb[: int(csr.n_edges)], int(csr.entry)


def stats() -> dict:
    """Counters of the last merge on this thread; per-phase arrays are
    [expansion, naive search, local sliding]."""
    s = Stats()
    _check(lib().rnsm_get_stats(C.byref(s)))
    out = {}
    for name, _ in Stats._fields_:
        v = getattr(s, name)
        out[name] = list(v) if hasattr(v, "__len__") else v
    return out


def mos_plan(sizes, degree_bound, diameter=2, centroids=None):
    """Host-only planner: (source, target) operations in execution order, and
    the number of fallback edges."""
    import numpy as np
    m = len(sizes)
    sz = np.ascontiguousarray(sizes, dtype=np.int64)
    cen = None if centroids is None else np.ascontiguousarray(centroids, dtype=np.float64)
    cap = m * m
    ops = np.zeros((cap, 2), dtype=np.int32)
    cnt = C.c_int32(0)
    fb = C.c_int32(0)
    _check(lib().mos_plan(m, sz.ctypes.data_as(C.c_void_p),
                          None if cen is None else cen.ctypes.data_as(C.c_void_p),
                          0 if cen is None else cen.shape[1], degree_bound, diameter,
                          ops.ctypes.data_as(C.c_void_p), cap, C.byref(cnt), C.byref(fb)))
    return [tuple(int(x) for x in o) for o in ops[: cnt.value]], fb.value


def select_pivots(rk_offsets, rk_ids):
    """Host-only lazy greedy over reverse k-NN lists (CSR, numpy): pivots in
    selection order, followers grouped by pivot, and each follower's pivot."""
    import numpy as np
    off = np.ascontiguousarray(rk_offsets, dtype=np.int64)
    ids = np.ascontiguousarray(rk_ids, dtype=np.int32)
    n = off.shape[0] - 1
    piv = np.empty(max(n, 1), dtype=np.int32)
    fol = np.empty(max(n, 1), dtype=np.int32)
    fp = np.empty(max(n, 1), dtype=np.int32)
    npv, nfl = C.c_int64(0), C.c_int64(0)
    _check(lib().rnsm_select_pivots(n, off.ctypes.data_as(C.c_void_p),
                                    ids.ctypes.data_as(C.c_void_p) if ids.size else None,
                                    piv.ctypes.data_as(C.c_void_p), C.byref(npv),
                                    fol.ctypes.data_as(C.c_void_p),
                                    fp.ctypes.data_as(C.c_void_p), C.byref(nfl)))
    return piv[: npv.value].copy(), fol[: nfl.value].copy(), fp[: nfl.value].copy()


def select_pivots_device(rk_offsets, rk_ids, stream=None):
    """Device pivot selection over reverse lists (device int64 offsets, int32
    ids): pivot_of device tensor (-1 pivots, else the pivot) and the count."""
    import torch
    n = rk_offsets.shape[0] - 1
    piv = torch.empty(max(n, 1), dtype=torch.int32, device=rk_offsets.device)
    npv = C.c_int64(0)
    _check(lib().rnsm_select_pivots_device(n, _ptr(rk_offsets), _ptr(rk_ids), _ptr(piv),
                                           C.byref(npv), _stream(stream)))
    return piv[:n], npv.value


def search(offsets, nbrs, entry, base, queries, ef, k, seeds=None, metric=L2SQ,
           base_search=None, stream=None, noalloc=False, out=None):
    """Beam search of every query row in one graph (local ids). noalloc: call
    rnsm_search_noalloc (the library's static scratch, no device allocation).
    out: optional (ids int32 [nq, k], dists float32 [nq, k]) device tensors."""
    import torch
    g = Graph(n=offsets.shape[0] - 1, offsets=offsets.data_ptr(), nbrs=nbrs.data_ptr(),
              entry=int(entry))
    v = _vectors(base, base_search)
    nq = queries.shape[0]
    if out is None:
        ids = torch.empty((nq, k), dtype=torch.int32, device=base.device)
        ds = torch.empty((nq, k), dtype=torch.float32, device=base.device)
    else:
        ids, ds = out
        assert ids.shape == (nq, k) and ds.shape == (nq, k)
    ns = 0
    if seeds is not None:
        assert seeds.dtype == torch.int32 and seeds.is_contiguous()
        ns = seeds.shape[1]
    fn = lib().rnsm_search_noalloc if noalloc else lib().rnsm_search
    _check(fn(C.byref(g), C.byref(v), C.c_void_p(queries.data_ptr()), nq,
                             _ptr(seeds), ns, ef, k, metric, C.c_void_p(ids.data_ptr()),
                             C.c_void_p(ds.data_ptr()), _stream(stream)))
    return ids, ds


def tune_search(offsets, nbrs, entry, base, ef, n_sample=65536, metric=L2SQ, base_search=None,
                stream=None):
    """Autotuner of the beam-search shape on one graph (its own rows as
    queries): a dict with the fastest (hash_bits, waves_per_block), the
    default's, and their times in ms."""
    g = Graph(n=offsets.shape[0] - 1, offsets=offsets.data_ptr(), nbrs=nbrs.data_ptr(),
              entry=int(entry))
    v = _vectors(base, base_search)
    t = SearchTuning()
    _check(lib().rnsm_tune_search(C.byref(g), C.byref(v), ef, metric, int(n_sample), C.byref(t),
                                  _stream(stream)))
    return {"shape": (t.hash_bits, t.waves_per_block), "ms": t.ms,
            "default_shape": (t.default_hash_bits, t.default_waves_per_block),
            "default_ms": t.default_ms, "n_queries": t.n_queries, "n_tried": t.n_tried}


def build_graph(X, knn, R, alpha=1.0, reverse=False, alpha_rev=1.2, metric=L2SQ, stream=None,
                repair=False, return_links=False):
    """Sub-index builder from exact k-NN lists (device int32 [n, K]);
    repair=True links in every vertex the entry cannot reach.
    Returns (offsets, nbrs, entry) [, repair links added]."""
    import torch
    n, dim = X.shape
    K = knn.shape[1]
    off = torch.empty(n + 1, dtype=torch.int64, device=X.device)
    nb = torch.empty(n * R, dtype=torch.int32, device=X.device)
    entry = C.c_int32(0)
    links = C.c_int64(0)
    opts = (1 if reverse else 0) | (2 if repair else 0)
    _check(lib().rnsm_build_graph(n, C.c_void_p(X.data_ptr()), dim, metric,
                                  C.c_void_p(knn.data_ptr()), K, R, float(alpha), opts,
                                  float(alpha_rev), C.c_void_p(off.data_ptr()),
                                  C.c_void_p(nb.data_ptr()), C.byref(entry), C.byref(links),
                                  _stream(stream)))
    ne = int(off[-1].item())
    out = (off, nb[:ne].clone(), entry.value)
    return out + (links.value,) if return_links else out


def reachable(off, nb, entry, stream=None):
    """Vertices reachable from the entry of a device CSR graph (rnsm_reachable)."""
    cnt = C.c_int64(0)
    n = off.shape[0] - 1
    _check(lib().rnsm_reachable(n, C.c_void_p(off.data_ptr()), C.c_void_p(nb.data_ptr()),
                                int(entry), C.byref(cnt), _stream(stream)))
    return cnt.value


_DT = {"float32": 0, "bfloat16": 1, "float16": 2, "uint8": 3}


def convert(src, dtype, stream=None):
    """Device conversion (rnsm_convert) of a contiguous float32 or uint8
    tensor to `dtype` (torch.bfloat16, torch.float16 or torch.float32);
    returns a new tensor of the same shape."""
    import torch
    assert src.is_cuda and src.is_contiguous()
    out = torch.empty(src.shape, dtype=dtype, device=src.device)
    st = _DT[str(src.dtype).replace("torch.", "")]
    dt = _DT[str(dtype).replace("torch.", "")]
    _check(lib().rnsm_convert(C.c_void_p(src.data_ptr()), st, C.c_void_p(out.data_ptr()), dt,
                              src.numel(), _stream(stream)))
    return out
