"""Host-side checks of the C ABI: the library loads, exports every entry
point the header declares, rejects bad arguments before any device work, and
its host-only planner matches the oracle's. No GPU needed."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pkg():
    import paper_2602_17099_amd as p
    if not os.path.exists(p.LIB_PATH):
        from paper_2602_17099_amd import build
        build.build()
    return p


def test_exports_every_declared_symbol(pkg):
    hdr = open(os.path.join(ROOT, "include", "rnsm.h")).read()
    names = set(re.findall(r"^\s*(?:rnsm_status|const char\*|void)\s+(\w+)\s*\(", hdr, re.M))
    assert names == set(pkg.SYMBOLS)
    L = C.CDLL(pkg.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_merge_rejects_bad_arguments_on_host(pkg):
    L = pkg.lib()
    g = (pkg.Graph * 2)()
    v = pkg.Vectors(n=10, dim=32, f32=None)
    p = pkg.Params(R=16, L=32, alpha=1.2)
    out = pkg.Csr()
    assert L.rnsm_merge(1, g, C.byref(v), C.byref(p), C.byref(out)) == 1
    assert "m = 1" in pkg.last_error()
    assert L.rnsm_merge(2, None, C.byref(v), C.byref(p), C.byref(out)) == 1
    out = pkg.Csr(offsets=8, nbrs=8)
    for field, val, msg in [("R", 0, "R = 0"), ("R", 65, "R = 65"), ("L", 0, "L = 0"),
                            ("L", 129, "L = 129"), ("alpha", 0.9, "alpha"),
                            ("k_reverse", 20, "k_reverse"), ("mos_diameter", 1, "mos_diameter")]:
        q = pkg.Params(R=16, L=32, alpha=1.2)
        setattr(q, field, val)
        assert L.rnsm_merge(2, g, C.byref(v), C.byref(q), C.byref(out)) == 1, field
        assert msg in pkg.last_error()
    for field, val in [("search_hash_bits", 7), ("search_hash_bits", 13),
                       ("search_waves_per_block", 5), ("search_waves_per_block", -1)]:
        q = pkg.Params(R=16, L=32, alpha=1.2)
        setattr(q, field, val)
        assert L.rnsm_merge(2, g, C.byref(v), C.byref(q), C.byref(out)) == 1, field
        assert field in pkg.last_error()
    q = pkg.Params(R=16, L=32, alpha=1.2, max_device_bytes=-1)
    assert L.rnsm_merge(2, g, C.byref(v), C.byref(q), C.byref(out)) == 1
    assert "max_device_bytes" in pkg.last_error()
    # host output needs no output buffers; the other checks still run
    q = pkg.Params(R=16, L=32, alpha=1.2, flags=pkg.FLAG_HOST_OUT)
    assert L.rnsm_merge(2, g, C.byref(v), C.byref(q), C.byref(pkg.Csr())) == 1
    assert "f32 is NULL" in pkg.last_error()
    # vectors
    assert L.rnsm_merge(2, g, C.byref(v), C.byref(p), C.byref(out)) == 1
    assert "f32 is NULL" in pkg.last_error()
    v2 = pkg.Vectors(n=10, dim=30, f32=8)
    assert L.rnsm_merge(2, g, C.byref(v2), C.byref(p), C.byref(out)) == 4  # unsupported dim
    v3 = pkg.Vectors(n=10, dim=32, f32=8)
    g[0] = pkg.Graph(n=5, offsets=8, nbrs=8, entry=7)
    g[1] = pkg.Graph(n=5, offsets=8, nbrs=8, entry=0)
    assert L.rnsm_merge(2, g, C.byref(v3), C.byref(p), C.byref(out)) == 1
    assert "entry 7" in pkg.last_error()
    g[0] = pkg.Graph(n=6, offsets=8, nbrs=8, entry=0)
    assert L.rnsm_merge(2, g, C.byref(v3), C.byref(p), C.byref(out)) == 1
    assert "vectors hold 10 rows" in pkg.last_error()


@pytest.mark.parametrize("m,R,cent,seed", [(2, 2, False, 0), (4, 2, False, 1), (4, 2, True, 2),
                                           (10, 4, True, 3), (10, 4, False, 4), (17, 5, True, 5),
                                           (50, 8, True, 6), (50, 8, False, 7), (30, 3, True, 8)])
def test_mos_plan_matches_oracle(pkg, orc, m, R, cent, seed):
    g = np.random.default_rng(seed)
    sizes = g.integers(1000, 5000, size=m)
    sizes[g.integers(0, m)] = sizes[0]  # a size tie
    cen = g.standard_normal((m, 7)) if cent else None
    ops, fb = pkg.mos_plan(sizes, R, 2, cen)
    ref, rfb = orc.plan(sizes, R, 2, cen)
    assert ops == ref and fb == rfb


def test_mos_plan_rejects(pkg):
    with pytest.raises(pkg.RnsmError):
        pkg.mos_plan([10, 20], 2, 1)
    with pytest.raises(pkg.RnsmError):
        pkg.mos_plan([10, 0], 2, 2)


def test_convert_rejects_on_host(pkg):
    # argument errors come back before any device work
    L = pkg.lib()
    buf = C.create_string_buffer(64)
    p = C.cast(buf, C.c_void_p)
    assert L.rnsm_convert(p, 1, p, 0, 4, None) == 1          # bf16 -> f32: unsupported
    assert L.rnsm_convert(p, 3, p, 3, 4, None) == 1          # u8 -> u8
    assert L.rnsm_convert(None, 0, p, 1, 4, None) == 1       # NULL source
    assert L.rnsm_convert(p, 0, p, 1, -1, None) == 1         # negative count
    assert "unsupported" in pkg.last_error() or "count" in pkg.last_error()
    assert L.rnsm_convert(None, 0, None, 1, 0, None) == 0    # nothing to do


# ------------------------------------------------- lazy greedy on the host

def _expected_groups(rk_off, rk_ids, pivot_of, order):
    """Followers grouped by pivot (selection order), each group in its
    pivot's list order, from the oracle's pivot assignment."""
    fol, fp = [], []
    for p in order.tolist():
        for y in rk_ids[rk_off[p]:rk_off[p + 1]].tolist():
            if pivot_of[y] == p:
                fol.append(y)
                fp.append(p)
    return fol, fp


def _skewed_knn(g, n, k, skew):
    """N_k lists drawn with popularity ~ rank^-skew, so a few reverse lists
    are long (well past 32, the greedy's bitmap levels) and many are empty."""
    w = 1.0 / np.arange(1, n + 1) ** skew
    perm = g.permutation(n)
    p = np.empty(n)
    p[perm] = w / w.sum()
    nk = np.empty((n, k), np.int32)
    for v in range(n):
        q = p.copy()
        q[v] = 0.0
        nk[v] = g.choice(n, k, replace=False, p=q / q.sum())
    return nk


@pytest.mark.parametrize("n,k,skew,seed", [(1, 0, 0.0, 0), (2, 1, 0.0, 1), (64, 3, 0.0, 2),
                                           (65, 3, 0.5, 3), (700, 5, 0.0, 4), (3000, 5, 0.8, 5),
                                           (3000, 7, 1.1, 6), (5000, 3, 0.3, 7)])
def test_select_pivots_matches_oracle(pkg, orc, n, k, skew, seed):
    # the merge's own host greedy (Algorithm 2, phase 2) against the oracle's
    # heap-based lazy greedy, itself pinned to an eager greedy
    g = np.random.default_rng(seed)
    if k == 0:
        off, ids = np.zeros(n + 1, np.int64), np.zeros(0, np.int32)
    else:
        off, ids = orc.invert(_skewed_knn(g, n, k, skew))
    piv, fol, fp = pkg.select_pivots(off, ids)
    pivot_of, order = orc.pivots(off, ids)
    assert piv.tolist() == order.tolist()
    efol, efp = _expected_groups(off, ids, pivot_of, order)
    assert fol.tolist() == efol and fp.tolist() == efp
    assert len(piv) + len(fol) == n
    assert sorted(piv.tolist() + fol.tolist()) == list(range(n))
    if skew >= 0.8:
        assert (np.diff(off) >= 32).any()  # the heap path ran


def test_select_pivots_long_random_lists(pkg, orc):
    # many bitmap words and every gain level, uniform random N_k
    g = np.random.default_rng(11)
    n, k = 100_000, 5
    # v + 1 + (0..n-2) mod n never names v; rows with a repeated id are redrawn
    nk = ((np.arange(n)[:, None] + 1 + g.integers(0, n - 1, size=(n, k))) % n).astype(np.int32)
    s = np.sort(nk, axis=1)
    for v in np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]:
        nk[v] = (v + 1 + g.choice(n - 1, k, replace=False)) % n
    off, ids = orc.invert(nk)
    piv, fol, fp = pkg.select_pivots(off, ids)
    pivot_of, order = orc.pivots(off, ids)
    assert np.array_equal(piv, order)
    efol, efp = _expected_groups(off, ids, pivot_of, order)
    assert fol.tolist() == efol and fp.tolist() == efp


def test_select_pivots_special_cases(pkg):
    # no vertices; lists all empty (every vertex its own pivot, in id order);
    # a star: the hub's list holds everyone else
    piv, fol, fp = pkg.select_pivots(np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert len(piv) == len(fol) == len(fp) == 0
    piv, fol, _ = pkg.select_pivots(np.zeros(6, np.int64), np.zeros(0, np.int32))
    assert piv.tolist() == [0, 1, 2, 3, 4] and len(fol) == 0
    n = 40
    off = np.array([0] * 8 + [n - 1] * (n - 7), np.int64)
    ids = np.array([y for y in range(n) if y != 7], np.int32)
    piv, fol, fp = pkg.select_pivots(off, ids)
    assert piv.tolist() == [7] and fol.tolist() == ids.tolist() and set(fp.tolist()) == {7}


def test_select_pivots_rejects(pkg):
    L = pkg.lib()
    for off, ids, msg in [([0, 1, 1], [0], "itself"), ([0, 2, 2], [1, 1], "repeated"),
                          ([0, 1, 1], [5], "out of range"), ([0, 2, 1], [1, 0], "decrease"),
                          ([1, 1, 1], [0], "rk_offsets[0]")]:
        with pytest.raises(pkg.RnsmError, match=msg.replace("[", r"\[").replace("]", r"\]")):
            pkg.select_pivots(np.array(off, np.int64), np.array(ids, np.int32))
    assert L.rnsm_select_pivots(-1, None, None, None, None, None, None, None) == 1
    z = np.zeros(3, np.int64)
    assert L.rnsm_select_pivots(2, z.ctypes.data_as(C.c_void_p), None, None, None, None, None,
                                None) == 1
    assert "NULL" in pkg.last_error()


def test_tune_search_rejects_on_host(pkg):
    # argument errors come back before any device work
    L = pkg.lib()
    t = pkg.SearchTuning()
    g = pkg.Graph(n=10, offsets=8, nbrs=8, entry=0)
    v = pkg.Vectors(n=10, dim=32, f32=8)
    ok = (C.byref(g), C.byref(v), 32, 0, 100, C.byref(t), None)
    for i, bad, msg in [(0, None, "NULL"), (2, 0, "ef"), (2, 129, "ef"), (3, 5, "metric"),
                        (4, 0, "n_sample"), (5, None, "NULL")]:
        args = list(ok)
        args[i] = bad
        assert L.rnsm_tune_search(*args) == 1, (i, bad)
        assert msg in pkg.last_error()
    g2 = pkg.Graph(n=11, offsets=8, nbrs=8, entry=0)
    assert L.rnsm_tune_search(C.byref(g2), *ok[1:]) == 1
    assert "mismatch" in pkg.last_error()
    g3 = pkg.Graph(n=10, offsets=8, nbrs=8, entry=10)
    assert L.rnsm_tune_search(C.byref(g3), *ok[1:]) == 1
    assert "entry" in pkg.last_error()


def test_search_rejects_on_host(pkg):
    # argument errors of the beam search come back before any device work
    L = pkg.lib()
    g = pkg.Graph(n=10, offsets=8, nbrs=8, entry=0)
    v = pkg.Vectors(n=10, dim=32, f32=8)
    ok = [C.byref(g), C.byref(v), C.c_void_p(8), 4, None, 0, 16, 10, 0, C.c_void_p(8), None, None]
    for i, bad, msg in [(0, None, "NULL"), (1, None, "NULL"), (2, None, "NULL"), (3, -1, "nq"),
                        (6, 0, "ef"), (6, 129, "ef"), (7, 0, "k"), (7, 17, "k"),
                        (8, 7, "metric"), (9, None, "NULL")]:
        args = list(ok)
        args[i] = bad
        assert L.rnsm_search(*args) == 1, (i, bad)
        assert msg in pkg.last_error()
    args = list(ok)
    args[4], args[5] = C.c_void_p(8), 0
    assert L.rnsm_search(*args) == 1 and "n_seeds" in pkg.last_error()
    g2 = pkg.Graph(n=11, offsets=8, nbrs=8, entry=0)
    assert L.rnsm_search(C.byref(g2), *ok[1:]) == 1 and "mismatch" in pkg.last_error()


def test_header_is_plain_c(tmp_path):
    # a C99 caller can include the header and name every entry point
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text('#include "rnsm.h"\n'
                   "int main(void) {\n"
                   "    rnsm_params p = {0};\n"
                   "    rnsm_search_tuning t;\n"
                   "    rnsm_stats s;\n"
                   "    typedef void (*fn)(void);\n"
                   "    fn f[] = {(fn)rnsm_merge, (fn)rnsm_merge_simple, (fn)mos_plan,\n"
                   "              (fn)rnsm_select_pivots, (fn)rnsm_search, (fn)rnsm_tune_search,\n"
                   "              (fn)rnsm_build_graph, (fn)rnsm_convert, (fn)rnsm_get_stats,\n"
                   "              (fn)rnsm_last_error, (fn)rnsm_reachable};\n"
                   "    (void)p; (void)t; (void)s; (void)f;\n"
                   "    return RNSM_FLAG_AUTOTUNE == 4u ? 0 : 1;\n"
                   "}\n")
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                        "-fsyntax-only", "-I", os.path.join(ROOT, "include"), str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_search_noalloc_rejects_on_host(pkg):
    # argument errors, and cosine norms beyond the static scratch, come back
    # before any device work
    L = pkg.lib()
    g = pkg.Graph(n=10, offsets=8, nbrs=8, entry=0)
    v = pkg.Vectors(n=10, dim=32, f32=8)
    ok = [C.byref(g), C.byref(v), C.c_void_p(8), 4, None, 0, 16, 10, 0, C.c_void_p(8), None, None]
    for i, bad, msg in [(0, None, "NULL"), (3, -1, "nq"), (6, 0, "ef"), (7, 17, "k")]:
        args = list(ok)
        args[i] = bad
        assert L.rnsm_search_noalloc(*args) == 1, (i, bad)
        assert msg in pkg.last_error()
    big = pkg.Graph(n=4_000_000, offsets=8, nbrs=8, entry=0)
    vb = pkg.Vectors(n=4_000_000, dim=32, f32=8)
    args = [C.byref(big), C.byref(vb), C.c_void_p(8), 500_000, None, 0, 16, 10, 2,
            C.c_void_p(8), None, None]
    assert L.rnsm_search_noalloc(*args) == 1
    assert "scratch" in pkg.last_error()


def test_csr_free_only_releases_library_arrays(pkg):
    # NULL and caller-owned device buffers are left alone
    L = pkg.lib()
    L.rnsm_csr_free(None)
    dev = pkg.Csr(offsets=8, nbrs=16, dists=24, entry=3, n_edges=5, mem=pkg.DEVICE)
    L.rnsm_csr_free(C.byref(dev))
    assert (dev.offsets, dev.nbrs, dev.dists, dev.entry, dev.n_edges) == (8, 16, 24, 3, 5)
    empty = pkg.Csr(mem=pkg.HOST)  # host arrays, all NULL: free(NULL) is a no-op
    L.rnsm_csr_free(C.byref(empty))
    assert empty.mem == pkg.DEVICE and not empty.offsets


def test_select_pivots_device_rejects_on_host(pkg):
    L = pkg.lib()
    n = C.c_int64(0)
    assert L.rnsm_select_pivots_device(-1, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8),
                                       C.byref(n), None) == 1
    assert L.rnsm_select_pivots_device(4, None, C.c_void_p(8), C.c_void_p(8), C.byref(n),
                                       None) == 1
    assert "NULL" in pkg.last_error()
    assert L.rnsm_select_pivots_device(0, None, None, None, C.byref(n), None) == 0

