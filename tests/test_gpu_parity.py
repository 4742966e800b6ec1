"""Parity of the HIP path with the CPU oracle, through the C ABI.

Integer-valued inputs make every float32 distance exact, so results must be
bit-identical to the oracle's (float64) results. Float inputs are compared
with the tolerances of the precision contract: edge overlap >= 99.5 %,
recall@10 within 0.002, stored distances within 1e-5 relative of float64.
"""
import numpy as np
import pytest

from paper_2602_17099_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def pkg():
    import paper_2602_17099_amd as p
    p.lib()
    return p


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _dsubs(subs, dev):
    return [(_t(o, dev), _t(nb, dev), e) for o, nb, e in subs]


def _rows(off, nb):
    return [nb[off[v]:off[v + 1]].tolist() for v in range(len(off) - 1)]


def _assert_same_merge(got, ref):
    off, nb, ds, entry = got
    off = off.cpu().numpy()
    nb = nb.cpu().numpy()
    assert entry == ref["entry"]
    if not np.array_equal(off, ref["offsets"]) or not np.array_equal(nb, ref["nbrs"]):
        a, b = _rows(off, nb), _rows(ref["offsets"], ref["nbrs"])
        bad = [v for v in range(len(b)) if a[v] != b[v]]
        raise AssertionError(f"{len(bad)} rows differ, first {bad[:5]}: "
                             f"gpu {a[bad[0]]} oracle {b[bad[0]]}")
    if ds is not None:
        assert np.array_equal(ds.cpu().numpy().astype(np.float64), ref["dists"])


# ------------------------------------------------------------- the search

@pytest.fixture(scope="module")
def search_case(orc):
    X = inputs.tiny_int(3000, 32, seed=101)
    Q = inputs.tiny_int(300, 32, seed=102)
    off, nb, entry = orc.build_graph(X, 24, 12, alpha=1.2, reverse=True)
    return X, Q, off, nb, entry


@pytest.mark.parametrize("ef", [1, 2, 16, 33, 64, 65, 100, 128])
def test_search_entry_bit_exact(dev, orc, pkg, search_case, ef):
    X, Q, off, nb, entry = search_case
    ids, ds = pkg.search(_t(off, dev), _t(nb, dev), entry, _t(X, dev), _t(Q, dev), ef, ef)
    ids, ds = ids.cpu().numpy(), ds.cpu().numpy()
    for i in range(0, len(Q), 7):
        rid, rd, _ = orc.beam_search(off, nb, X, Q[i], [entry], ef)
        n = len(rid)
        assert ids[i, :n].tolist() == rid.tolist(), i
        assert ds[i, :n].astype(np.float64).tolist() == rd.tolist(), i
        assert (ids[i, n:] == -1).all()


@pytest.mark.parametrize("ef,ns", [(8, 3), (32, 40), (64, 64), (96, 130)])
def test_search_seeds_bit_exact(dev, orc, pkg, search_case, ef, ns):
    X, Q, off, nb, entry = search_case
    g = np.random.default_rng(ef)
    seeds = g.integers(-1, len(X), size=(len(Q), ns)).astype(np.int32)
    seeds[:, 1] = seeds[:, 0]  # a duplicate seed
    ids, ds = pkg.search(_t(off, dev), _t(nb, dev), entry, _t(X, dev), _t(Q, dev), ef, ef,
                         seeds=_t(seeds, dev))
    ids, ds = ids.cpu().numpy(), ds.cpu().numpy()
    for i in range(0, len(Q), 11):
        rid, rd, _ = orc.beam_search(off, nb, X, Q[i], seeds[i], ef)
        assert ids[i, :len(rid)].tolist() == rid.tolist(), i
        assert ds[i, :len(rid)].astype(np.float64).tolist() == rd.tolist(), i


def test_search_out_of_range_seeds_ignored(dev, orc, pkg, search_case):
    # seed ids outside the graph are skipped like -1
    X, Q, off, nb, entry = search_case
    g = np.random.default_rng(5)
    seeds = g.integers(0, len(X), size=(len(Q), 20)).astype(np.int32)
    seeds[:, ::3] = len(X) + 7
    ids, _ = pkg.search(_t(off, dev), _t(nb, dev), entry, _t(X, dev), _t(Q, dev), 24, 24,
                        seeds=_t(seeds, dev))
    ids = ids.cpu().numpy()
    for i in range(0, len(Q), 10):
        s = np.where(seeds[i] >= len(X), -1, seeds[i])
        rid, _, _ = orc.beam_search(off, nb, X, Q[i], s, 24)
        assert ids[i, :len(rid)].tolist() == rid.tolist(), i


@pytest.mark.parametrize("dtype", ["bfloat16", "float16"])
def test_search_16bit_copy_on_integers(dev, orc, pkg, search_case, dtype):
    import torch
    X, Q, off, nb, entry = search_case
    dt = getattr(torch, dtype)
    Xd = _t(X, dev)
    ids, ds = pkg.search(_t(off, dev), _t(nb, dev), entry, Xd, _t(Q, dev).to(dt), 48, 48,
                         base_search=Xd.to(dt))
    ids = ids.cpu().numpy()
    for i in range(0, len(Q), 13):
        rid, _, _ = orc.beam_search(off, nb, X, Q[i], [entry], 48)
        assert ids[i, :len(rid)].tolist() == rid.tolist(), i


@pytest.mark.parametrize("dtype", ["bfloat16", "float16"])
def test_search_cosine_16bit_copy(dev, orc, pkg, search_case, dtype):
    # cosine on a 16-bit copy of integer rows: the copy holds the values
    # exactly and every dot2 sum is exact, so ids and distance bits equal the
    # float32 search's; those match the oracle's float64 cosine search
    import torch
    X, Q, off, nb, entry = search_case
    dt = getattr(torch, dtype)
    Xd, Qd = _t(X, dev), _t(Q, dev)
    i32, d32 = pkg.search(_t(off, dev), _t(nb, dev), entry, Xd, Qd, 40, 20, metric=2)
    i16, d16 = pkg.search(_t(off, dev), _t(nb, dev), entry, Xd, Qd.to(dt), 40, 20, metric=2,
                          base_search=Xd.to(dt))
    assert torch.equal(i32, i16)
    assert torch.equal(d32, d16)
    i32 = i32.cpu().numpy()
    same = tot = 0
    for i in range(0, len(Q), 7):
        rid, _, _ = orc.beam_search(off, nb, X, Q[i], [entry], 40, metric=2)
        same += len(set(rid[:20].tolist()) & set(i32[i].tolist()))
        tot += min(20, len(rid))
    assert same >= 0.99 * tot


def test_search_tiny_visited_table(dev, orc, pkg, search_case, monkeypatch):
    # a 64-slot visited table overflows: the beam must still be exact
    X, Q, off, nb, entry = search_case
    monkeypatch.setenv("RNSM_HASH_BITS", "6")
    ids, _ = pkg.search(_t(off, dev), _t(nb, dev), entry, _t(X, dev), _t(Q, dev), 64, 64)
    ids = ids.cpu().numpy()
    for i in range(0, len(Q), 17):
        rid, _, _ = orc.beam_search(off, nb, X, Q[i], [entry], 64)
        assert ids[i].tolist() == rid.tolist(), i


def test_search_duplicate_seeds_full_table(dev, orc, pkg, search_case, monkeypatch):
    # with an overflowing visited table both copies of a duplicated seed are
    # evaluated in the same batch; the beam must hold the vertex once
    X, Q, off, nb, entry = search_case
    monkeypatch.setenv("RNSM_HASH_BITS", "6")
    g = np.random.default_rng(7)
    seeds = g.integers(0, len(X), size=(len(Q), 120)).astype(np.int32)
    seeds[:, 60:] = seeds[:, :60]
    ids, ds = pkg.search(_t(off, dev), _t(nb, dev), entry, _t(X, dev), _t(Q, dev), 100, 100,
                         seeds=_t(seeds, dev))
    ids = ids.cpu().numpy()
    for i in range(0, len(Q), 9):
        rid, _, _ = orc.beam_search(off, nb, X, Q[i], seeds[i], 100)
        assert ids[i, :len(rid)].tolist() == rid.tolist(), i


# -------------------------------------------------------------- the merge

@pytest.fixture(scope="module")
def tiny(orc):
    # 2 sub-indexes x 5,000 vectors, dim 32, integers in [-8, 8]; each the
    # exact 32-NN graph pruned with alpha = 1 to R <= 16
    X = inputs.tiny_int(10000, 32, seed=inputs.SEED_BASE + 1)
    subs = [orc.build_graph(X[:5000], 32, 16, alpha=1.0), orc.build_graph(X[5000:], 32, 16, alpha=1.0)]
    return X, subs


def test_merge_tiny_bit_exact(dev, orc, pkg, tiny):
    X, subs = tiny
    ref = orc.merge(subs, X, R=16, L=32, alpha=1.2)
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=16, L=32, alpha=1.2)
    _assert_same_merge(got, ref)
    st = pkg.stats()
    assert st["n_source_vertices"] == 5000 and st["n_ops"] == 1
    assert st["n_pivots"] + st["n_followers"] == 5000


@pytest.mark.parametrize("chunk", ["1", "700"])
def test_merge_tiny_pivot_chunks_bit_exact(dev, orc, pkg, tiny, monkeypatch, chunk):
    # the searches start on pivot groups while the greedy still runs; many
    # small chunks must give the same graph and counts as one
    X, subs = tiny
    ref = orc.merge(subs, X, R=16, L=32, alpha=1.2, trace=True)
    monkeypatch.setenv("RNSM_PIVOT_CHUNK", chunk)
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=16, L=32, alpha=1.2)
    _assert_same_merge(got, ref)
    st = pkg.stats()
    assert st["n_pivots"] == ref["trace"]["n_pivots"]
    assert st["launches"][1] >= 3 and st["queries"][1] + st["queries"][2] == 5000


def test_merge_simple_entry_point(dev, orc, pkg, tiny):
    X, subs = tiny
    ref = orc.merge(subs, X, R=16, L=32, alpha=1.2)
    off, nb, entry = pkg.merge_simple(_dsubs(subs, dev), _t(X, dev), 16, 32, 1.2)
    assert np.array_equal(off.cpu().numpy(), ref["offsets"])
    assert np.array_equal(nb.cpu().numpy(), ref["nbrs"])


def test_merge_tiny_trace_steps(dev, orc, pkg, tiny):
    # pivots and the naive / sliding split must agree with the oracle's
    X, subs = tiny
    ref = orc.merge(subs, X, R=16, L=32, alpha=1.2, trace=True)
    pkg.merge(_dsubs(subs, dev), _t(X, dev), R=16, L=32, alpha=1.2)
    st = pkg.stats()
    tr = ref["trace"]
    assert st["n_pivots"] == tr["n_pivots"]
    # a forgetful visited table only adds re-evaluations
    ref_ndc = [tr["ndc_expand"], tr["ndc_naive"], tr["ndc_slide"]]
    assert all(g >= r for g, r in zip(st["ndc"], ref_ndc))


def test_merge_tiny_exact_visited_counts(dev, orc, pkg, tiny, monkeypatch):
    # with the probing visited table every vertex is evaluated once: the
    # distance counts of all three search phases equal the oracle's
    X, subs = tiny
    ref = orc.merge(subs, X, R=16, L=32, alpha=1.2, trace=True)
    monkeypatch.setenv("RNSM_EXACT_VISITED", "1")
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=16, L=32, alpha=1.2)
    _assert_same_merge(got, ref)
    st = pkg.stats()
    tr = ref["trace"]
    assert st["exact_visited"] == 1 and st["hash_evictions"] == 0
    assert st["ndc"] == [tr["ndc_expand"], tr["ndc_naive"], tr["ndc_slide"]]


@pytest.mark.parametrize("flags", [0, 1])
def test_merge_ragged_multi_op_bit_exact(dev, orc, pkg, flags):
    # five uneven sub-indexes: MOS plan with unit costs, several operations
    # per sub-index; flags=1 makes every source vertex a pivot
    sizes = [813, 2417, 1290, 3001, 655]
    X = inputs.tiny_int(sum(sizes), 32, seed=201)
    subs, b = [], 0
    for i, n in enumerate(sizes):
        subs.append(orc.build_graph(X[b:b + n], 24, 12, alpha=1.0))
        b += n
    ref = orc.merge(subs, X, R=12, L=24, alpha=1.2, all_pivots=bool(flags))
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=12, L=24, alpha=1.2, flags=flags)
    assert pkg.stats()["n_ops"] == len(ref["ops"])
    _assert_same_merge(got, ref)


def test_merge_hub_source_bit_exact(dev, orc, pkg):
    # a source sub-index whose every vertex has the origin as its nearest
    # neighbour (sign vectors scaled by 2: |x|^2 = 128 < |x - y|^2 ~ 256),
    # so the origin's reverse k-NN list is far longer than the greedy's
    # bitmap levels (its high-gain heap path)
    g = inputs.rng(1401)
    S = (2 * (2 * g.integers(0, 2, (700, 32)) - 1)).astype(np.float32)
    S[0] = 0.0
    T = inputs.tiny_int(900, 32, seed=1402)
    X = np.ascontiguousarray(np.concatenate([S, T]))
    subs = [orc.build_graph(X[:700], 24, 12, alpha=1.0), orc.build_graph(X[700:], 24, 12, alpha=1.0)]
    ref = orc.merge(subs, X, R=12, L=24, alpha=1.2, trace=True)
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=12, L=24, alpha=1.2)
    _assert_same_merge(got, ref)
    st = pkg.stats()
    assert st["n_pivots"] == ref["trace"]["n_pivots"]
    nk = orc.expand(*subs[0][:2], X[:700], 5, 16)
    assert (nk == 0).any(axis=1).sum() > 256  # the hub is in more than 256 N_k lists


def test_merge_many_long_lists_bit_exact(dev, orc, pkg, monkeypatch):
    # k = 40 of k+ = 48: several hundred source vertices have reverse k-NN
    # lists of 32 or more (the greedy's heap, not its bitmap levels); with a
    # prefix of 8 such lists copied ahead, the rest is fetched when the
    # greedy starts
    X = inputs.mixture_u8(2600, 16, comps=4, seed=1411)
    subs = [orc.build_graph(X[:1200], 48, 24, alpha=1.2, reverse=True),
            orc.build_graph(X[1200:], 48, 24, alpha=1.2, reverse=True)]
    nk = orc.expand(*subs[0][:2], X[:1200], 40, 48)
    rk_len = np.bincount(nk[nk >= 0].ravel(), minlength=1200)
    assert (rk_len >= 32).sum() > 64
    ref = orc.merge(subs, X, R=24, L=48, alpha=1.2, k=40, kplus=48, trace=True)
    monkeypatch.setenv("RNSM_GAIN_PREFIX", "8")
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=24, L=48, alpha=1.2, k=40, kplus=48)
    _assert_same_merge(got, ref)
    assert pkg.stats()["n_pivots"] == ref["trace"]["n_pivots"]


def test_incremental_merges_bit_exact(dev, orc, pkg):
    # the incremental scenario: sub-indexes merged one at a time into the
    # growing index, each step's merged graph (rows in prune order, degree up
    # to R) the next step's first input
    parts, n = 3, 1100
    X = inputs.mixture_u8(parts * n, 24, comps=6, seed=1421)
    subs = [orc.build_graph(X[i * n:(i + 1) * n], 24, 12, alpha=1.2, reverse=True)
            for i in range(parts)]
    acc_ref = subs[0]
    acc_got = _dsubs([subs[0]], dev)[0]
    for i in range(1, parts):
        Xi = np.ascontiguousarray(X[:(i + 1) * n])
        ref = orc.merge([acc_ref, subs[i]], Xi, R=12, L=24, alpha=1.2)
        got = pkg.merge([acc_got, _dsubs([subs[i]], dev)[0]], _t(Xi, dev), R=12, L=24,
                        alpha=1.2)
        _assert_same_merge(got, ref)
        acc_ref = (ref["offsets"], ref["nbrs"].astype(np.int32), ref["entry"])
        acc_got = (got[0], got[1], got[3])


def _drop_rows(g, every, at):
    off, nb, e = g
    n = len(off) - 1
    rows = [np.zeros(0, np.int32) if v % every == at else nb[off[v]:off[v + 1]]
            for v in range(n)]
    off2 = np.zeros(n + 1, np.int64)
    off2[1:] = np.cumsum([len(r) for r in rows])
    return off2, np.concatenate(rows).astype(np.int32), e


@pytest.mark.parametrize("case", ["one_vertex_source", "isolated_vertices"])
def test_merge_degenerate_bit_exact(dev, orc, pkg, case):
    # degenerate inputs the method allows (one sub-index alone is rejected:
    # m >= 2): a one-vertex source with no edges, vertices without edges in
    # both sub-indexes (their expansion and reverse lists are empty; the
    # source's entry is one of them, so its breadth-first order is one vertex
    # plus the unreached rest)
    X = inputs.tiny_int(701, 32, seed=1431)
    s0 = orc.build_graph(X[:400], 24, 12, alpha=1.0)
    if case == "one_vertex_source":
        subs = [(np.array([0, 0], np.int64), np.zeros(0, np.int32), 0), s0]
        Xm = np.concatenate([X[400:401], X[:400]])
    else:
        s1 = orc.build_graph(X[401:701], 24, 12, alpha=1.0)
        subs = [_drop_rows(s0, 7, 3), _drop_rows(s1, 5, 1)]
        Xm = np.concatenate([X[:400], X[401:701]])
    Xm = np.ascontiguousarray(Xm)
    ref = orc.merge(subs, Xm, R=12, L=24, alpha=1.2)
    got = pkg.merge(_dsubs(subs, dev), _t(Xm, dev), R=12, L=24, alpha=1.2)
    _assert_same_merge(got, ref)
    assert pkg.stats()["n_ops"] == len(ref["ops"])


def test_merge_centroid_costs_bit_exact(dev, orc, pkg):
    sizes = [700, 1500, 900, 1100, 600, 1300]
    # slab partition along a random direction: centroids differ
    X = inputs.mixture_u8(sum(sizes), 16, comps=8, seed=301)
    order = np.argsort(X @ inputs.rng(302).standard_normal(16), kind="stable")
    X = np.ascontiguousarray(X[order])
    subs, b = [], 0
    for n in sizes:
        subs.append(orc.build_graph(X[b:b + n], 16, 8, alpha=1.2, reverse=True))
        b += n
    ref = orc.merge(subs, X, R=8, L=16, alpha=1.2, use_centroids=True, mos_degree=3)
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=8, L=16, alpha=1.2, mos_degree=3, flags=2)
    _assert_same_merge(got, ref)


@pytest.fixture(scope="module")
def medium(orc):
    # the plain FP32 workload's shape at 1/25 scale: 0..255 integers from a
    # 64-component mixture, dim 128, R=32 sub-indexes; uneven split
    X = inputs.mixture_u8(40000, 128, seed=inputs.SEED_BASE + 2)
    n0 = 17011
    subs = [orc.build_graph(X[:n0], 64, 32, alpha=1.2, reverse=True),
            orc.build_graph(X[n0:], 64, 32, alpha=1.2, reverse=True)]
    return X, subs


@pytest.fixture(scope="module")
def medium_ref(orc, medium):
    X, subs = medium
    return orc.merge(subs, X, R=32, L=64, alpha=1.2)


# prune arithmetic: default (bfloat16 MFMA Gram, exact products on these
# integers), forced float32 walk, forced hi/lo split MFMA
PRUNE_PATHS = [(None, 1), ("walk", 0), ("split", 3)]


@pytest.mark.parametrize("mode,path", PRUNE_PATHS)
def test_merge_medium_bit_exact(dev, orc, pkg, medium, medium_ref, monkeypatch, mode, path):
    X, subs = medium
    if mode:
        monkeypatch.setenv("RNSM_PRUNE", mode)
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=32, L=64, alpha=1.2)
    assert pkg.stats()["prune_path"] == path
    _assert_same_merge(got, medium_ref)


@pytest.mark.parametrize("mode,path", PRUNE_PATHS)
@pytest.mark.parametrize("dim,R,L", [(96, 24, 48), (128, 64, 32), (64, 12, 24)])
def test_merge_prune_shapes_bit_exact(dev, orc, pkg, monkeypatch, dim, R, L, mode, path):
    # every MFMA fragment count (dim 64, 96, 128), R not a multiple of 16,
    # and R = 64 (one wavefront per block for the split form's LDS)
    X = inputs.mixture_u8(3000, dim, comps=16, seed=700 + dim)
    subs = [orc.build_graph(X[:1300], 2 * R, R, alpha=1.2, reverse=True),
            orc.build_graph(X[1300:], 2 * R, R, alpha=1.2, reverse=True)]
    ref = orc.merge(subs, X, R=R, L=L, alpha=1.2)
    if mode:
        monkeypatch.setenv("RNSM_PRUNE", mode)
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=R, L=L, alpha=1.2)
    assert pkg.stats()["prune_path"] == path
    _assert_same_merge(got, ref)


def test_tune_search_then_tuned_merge_bit_exact(dev, orc, pkg, medium, medium_ref):
    # the autotuner times every visited-table size and block shape on the
    # target graph; a merge under the shape it picks, or under the smallest
    # and largest tables, reaches the oracle's graph all the same
    X, subs = medium
    Xd = _t(X, dev)
    o, nb, e = _dsubs(subs, dev)[1]
    n0 = subs[0][0].shape[0] - 1
    t = pkg.tune_search(o, nb, e, Xd[n0:], 64, n_sample=8000)
    hb, w = t["shape"]
    assert 8 <= hb <= 12 and w in (1, 2, 4)
    assert t["ms"] > 0 and t["default_ms"] > 0 and t["ms"] <= t["default_ms"]
    assert t["n_queries"] == 8000 and 2 <= t["n_tried"] <= 16
    assert t["default_shape"] == (11, 1)  # float32 rows, L = 64, R = 32
    for shape in [t["shape"], (8, 4), (12, 1), (12, 2)]:
        got = pkg.merge(_dsubs(subs, dev), Xd, R=32, L=64, alpha=1.2, search_shape=shape)
        _assert_same_merge(got, medium_ref)
    # a 16-bit search copy: its own default (a 4 KB table), same graph
    t16 = pkg.tune_search(o, nb, e, Xd[n0:], 64, n_sample=3000, base_search=Xd[n0:].bfloat16())
    assert t16["default_shape"] == (10, 1) and t16["n_queries"] == 3000
    got = pkg.merge(_dsubs(subs, dev), Xd, R=32, L=64, alpha=1.2, search=Xd.bfloat16(),
                    search_shape=t16["shape"])
    _assert_same_merge(got, medium_ref)


def test_merge_autotune_flag_bit_exact(dev, orc, pkg, medium, medium_ref):
    # the merge tunes its own search shape (on the larger sub-index) and keeps
    # it for later merges of the same kind; the graph is the oracle's
    X, subs = medium
    Xd = _t(X, dev)
    shapes = set()
    for _ in range(2):
        got = pkg.merge(_dsubs(subs, dev), Xd, R=32, L=64, alpha=1.2, flags=pkg.FLAG_AUTOTUNE)
        _assert_same_merge(got, medium_ref)
        st = pkg.stats()
        shapes.add((st["search_hash_bits"], st["search_waves_per_block"]))
    assert len(shapes) == 1
    hb, w = shapes.pop()
    assert 8 <= hb <= 12 and w in (1, 2, 4)
    # a shape fixed by the caller wins over the flag
    got = pkg.merge(_dsubs(subs, dev), Xd, R=32, L=64, alpha=1.2, flags=pkg.FLAG_AUTOTUNE,
                    search_shape=(8, 2))
    _assert_same_merge(got, medium_ref)
    st = pkg.stats()
    assert (st["search_hash_bits"], st["search_waves_per_block"]) == (8, 2)
    # without either, the default shape (float32 rows, L = 64, R = 32)
    pkg.merge(_dsubs(subs, dev), Xd, R=32, L=64, alpha=1.2)
    st = pkg.stats()
    assert (st["search_hash_bits"], st["search_waves_per_block"]) == (11, 1)


@pytest.mark.parametrize("dtype", ["bfloat16", "float16"])
def test_merge_medium_16bit_search_bit_exact(dev, orc, pkg, medium, medium_ref, dtype):
    # 0..255 integers are exact in bfloat16 and float16: the reduced-precision
    # search reads different bytes but must reach the same graph (its
    # distances are exact, so the prune reuses them)
    import torch
    X, subs = medium
    ref = medium_ref
    Xd = _t(X, dev)
    got = pkg.merge(_dsubs(subs, dev), Xd, R=32, L=64, alpha=1.2,
                    search=Xd.to(getattr(torch, dtype)))
    _assert_same_merge(got, ref)


@pytest.mark.parametrize("mode,path", [(None, 3), ("walk", 0)])
@pytest.mark.parametrize("metric", [0, 1, 2])
def test_merge_float_data_tolerances(dev, orc, pkg, monkeypatch, metric, mode, path):
    # L2-normalised float vectors: float32 (walk) or hi/lo bfloat16 Gram
    # (MFMA) on the GPU against float64 in the oracle
    if mode:
        monkeypatch.setenv("RNSM_PRUNE", mode)
    X = inputs.mixture_unit(6000, 32, comps=32, seed=401 + metric)
    Q = inputs.mixture_unit(200, 32, comps=32, seed=401 + metric, stream=1)
    subs = [orc.build_graph(X[:2500], 32, 16, alpha=1.2, metric=metric, reverse=True),
            orc.build_graph(X[2500:], 32, 16, alpha=1.2, metric=metric, reverse=True)]
    ref = orc.merge(subs, X, R=16, L=32, alpha=1.2, metric=metric)
    off, nb, ds, entry = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=16, L=32, alpha=1.2,
                                   metric=metric)
    assert pkg.stats()["prune_path"] == path
    off, nb, ds = off.cpu().numpy(), nb.cpu().numpy(), ds.cpu().numpy()
    assert entry == ref["entry"]
    E_gpu = {(v, int(u)) for v in range(len(X)) for u in nb[off[v]:off[v + 1]]}
    E_ref = {(v, int(u)) for v in range(len(X)) for u in ref["nbrs"][ref["offsets"][v]:ref["offsets"][v + 1]]}
    assert len(E_gpu & E_ref) / len(E_ref) >= 0.995
    # stored float32 distances against a float64 recompute
    for v in range(0, len(X), 37):
        for j in range(off[v], off[v + 1]):
            d64 = orc.dist(X[v], X[nb[j]], metric)
            assert abs(ds[j] - d64) <= 1e-5 * max(abs(d64), 1e-3)
    gt, _ = orc.knn_queries(X, Q, 10, metric)
    r_gpu = orc.recall_at_k(orc.search_graph(off, nb, X, Q, entry, 32, metric=metric), gt)
    r_ref = orc.recall_at_k(orc.search_graph(ref["offsets"], ref["nbrs"], X, Q, ref["entry"], 32,
                                             metric=metric), gt)
    assert abs(r_gpu - r_ref) <= 0.002


# --------------------------------------------------------------- builder

@pytest.mark.parametrize("mode", [None, "walk", "split"])
@pytest.mark.parametrize("reverse", [False, True])
def test_build_graph_bit_exact(dev, orc, pkg, monkeypatch, reverse, mode):
    if mode:
        monkeypatch.setenv("RNSM_PRUNE", mode)
    X = inputs.mixture_u8(4000, 64, seed=501)
    knn = orc.knn_fast(X, 40)
    ref = orc.build_graph(X, 40, 20, alpha=1.2, reverse=reverse, alpha_rev=1.2, knn_ids=knn)
    off, nb, entry = pkg.build_graph(_t(X, dev), _t(knn, dev), 20, alpha=1.2, reverse=reverse,
                                     alpha_rev=1.2)
    assert entry == ref[2]
    assert np.array_equal(off.cpu().numpy(), ref[0])
    assert np.array_equal(nb.cpu().numpy(), ref[1])


@pytest.mark.parametrize("case", ["two_clusters", "many_pieces", "reverse_connected"])
def test_build_graph_repair_bit_exact(dev, orc, pkg, case):
    # the builder's reachability repair: the same links as the oracle's
    # (integer rows, so float32 distances are exact), every vertex reached
    g = inputs.rng(1611)
    if case == "two_clusters":
        X = np.concatenate([g.integers(-3, 4, (700, 16)),
                            g.integers(-3, 4, (500, 16)) + 40]).astype(np.float32)
        K, R, a, rev = 10, 6, 1.0, False
    elif case == "many_pieces":
        # 40 tight clusters, few neighbours each: many unreached pieces
        c = g.integers(0, 200, (40, 16))
        X = (c[g.integers(0, 40, 3000)] + g.integers(-2, 3, (3000, 16))).astype(np.float32)
        K, R, a, rev = 6, 4, 1.0, False
    else:
        X = inputs.mixture_u8(3000, 32, comps=12, seed=1612)
        K, R, a, rev = 24, 12, 1.2, True
    X = np.ascontiguousarray(X)
    knn = orc.knn_fast(X, K)
    base = orc.build_graph(X, K, R, alpha=a, reverse=rev, knn_ids=knn)
    *ref, links = orc.build_graph(X, K, R, alpha=a, reverse=rev, knn_ids=knn, repair=True,
                                  return_links=True)
    off, nb, entry, glinks = pkg.build_graph(_t(X, dev), _t(knn, dev), R, alpha=a, reverse=rev,
                                             repair=True, return_links=True)
    assert entry == ref[2] and glinks == links
    assert np.array_equal(off.cpu().numpy(), ref[0])
    assert np.array_equal(nb.cpu().numpy(), ref[1])
    n = X.shape[0]
    assert pkg.reachable(off, nb, entry) == orc.reachable(*ref) == n
    # the count before the repair, on the device and in the oracle
    b_off, b_nb = _t(base[0], dev), _t(base[1] if len(base[1]) else np.zeros(1, np.int32), dev)
    assert pkg.reachable(b_off, b_nb, base[2]) == orc.reachable(*base)
    if case != "reverse_connected":
        assert links >= 1 and orc.reachable(*base) < n


def test_reachable_on_merged_graph(dev, orc, pkg, tiny):
    X, subs = tiny
    off, nb, _, entry = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=16, L=32, alpha=1.2)
    ref = orc.merge(subs, X, R=16, L=32, alpha=1.2)
    assert pkg.reachable(off, nb, entry) == orc.reachable(ref["offsets"], ref["nbrs"], ref["entry"])
    for e in (0, 4999, 5000, 9999):
        assert pkg.reachable(off, nb, e) == orc.reachable(ref["offsets"], ref["nbrs"], e)


def test_reachable_rejects_bad_input(dev, pkg):
    off = _t(np.array([0, 2, 1], np.int64), dev)  # decreasing offsets
    nb = _t(np.array([1, 0], np.int32), dev)
    with pytest.raises(pkg.RnsmError):
        pkg.reachable(off, nb, 0)
    ok = _t(np.array([0, 1, 2], np.int64), dev)
    with pytest.raises(pkg.RnsmError):
        pkg.reachable(ok, nb, 5)


# ------------------------------------------------------------ bad inputs

def _bad(orc, kind):
    X = inputs.tiny_int(400, 32, seed=601)
    a = orc.build_graph(X[:200], 16, 8, alpha=1.0)
    b = orc.build_graph(X[200:], 16, 8, alpha=1.0)
    off, nb, e = (x.copy() if hasattr(x, "copy") else x for x in b)
    if kind == "self":
        nb[off[3]] = 3
    elif kind == "dup":
        nb[off[5] + 1] = nb[off[5]]
    elif kind == "range":
        nb[off[7]] = 200
    elif kind == "degree":
        return X, [a, b], 4
    elif kind == "offsets":
        off[10] = off[12] + 1
    return X, [a, (off, nb, e)], 8


@pytest.mark.parametrize("kind,msg", [("self", "self-loop"), ("dup", "duplicate"),
                                      ("range", "out of range"), ("degree", "degree above"),
                                      ("offsets", "non-decreasing")])
def test_merge_rejects_malformed_graphs(dev, orc, pkg, kind, msg):
    X, subs, R = _bad(orc, kind)
    with pytest.raises(pkg.RnsmError) as ei:
        pkg.merge(_dsubs(subs, dev), _t(X, dev), R=R, L=16, alpha=1.2)
    assert ei.value.status == 1 and msg in str(ei.value)


# ------------------------------------------------------ staging conversion

def test_convert_float32_to_16bit(dev, orc, pkg):
    # bfloat16 against the oracle's round-to-nearest-even definition, float16
    # against numpy's IEEE conversion; exact ties, subnormals, overflow,
    # infinities, NaN and a ragged count (not a multiple of 4)
    import torch
    g = inputs.rng(901)
    x = (g.standard_normal(100003) * np.exp2(g.integers(-150, 130, 100003))).astype(np.float32)
    ties = (g.integers(0, 1 << 16, 4000).astype(np.uint32) << 16 | 0x8000).view(np.float32)
    special = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 3.4028235e38, 65504.0, 65520.0,
                        6e-8, 1e-45, -1e-40, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8], dtype=np.float32)
    x = np.concatenate([x, ties, special])
    xd = _t(x, dev)
    b = pkg.convert(xd, torch.bfloat16).view(torch.int16).cpu().numpy().view(np.uint16)
    want = orc.to_bf16_bits(x)
    nan = np.isnan(x)
    assert np.array_equal(b[~nan], want[~nan])
    assert np.all(np.isnan(orc.bf16_bits_to_f32(b[nan])))
    h = pkg.convert(xd, torch.float16).view(torch.int16).cpu().numpy().view(np.uint16)
    with np.errstate(over="ignore"):
        hw = x.astype(np.float16).view(np.uint16)
    assert np.array_equal(h[~nan], hw[~nan])
    assert np.all(np.isnan(h[nan].view(np.float16)))


@pytest.mark.parametrize("dtype", ["float16", "bfloat16", "float32"])
def test_convert_uint8_exact(dev, pkg, dtype):
    import torch
    u = inputs.rng(902).integers(0, 256, 77777).astype(np.uint8)
    got = pkg.convert(_t(u, dev), getattr(torch, dtype)).float().cpu().numpy()
    assert np.array_equal(got, u.astype(np.float32))


@pytest.mark.parametrize("rule,param", [(1, 60.0), (1, 45.0), (2, 0.0), (2, 0.5), (2, 2.0)])
def test_merge_prune_rules_bit_exact(dev, orc, pkg, rule, param):
    # the SSG angle rule and the tau-MNG rule in the merge's source and
    # target prunes (the float32 walk), against the oracle: integer rows,
    # so every distance is exact and the decisions in double agree
    sizes = [1300, 2100, 900]
    X = inputs.tiny_int(sum(sizes), 32, seed=1661)
    subs, b = [], 0
    for n in sizes:
        subs.append(orc.build_graph(X[b:b + n], 24, 12, alpha=1.0))
        b += n
    ref = orc.merge(subs, X, R=12, L=24, alpha=1.2, prune_rule=rule, prune_param=param)
    for flags in (0, pkg.FLAG_BATCHED):
        got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=12, L=24, alpha=1.2, prune_rule=rule,
                        prune_param=param, flags=flags)
        assert pkg.stats()["prune_path"] == 0
        _assert_same_merge(got, ref)


def test_merge_prune_rules_rejected(dev, orc, pkg):
    X = inputs.tiny_int(600, 32, seed=1662)
    subs = _dsubs([orc.build_graph(X[:300], 16, 8, alpha=1.0),
                   orc.build_graph(X[300:], 16, 8, alpha=1.0)], dev)
    Xd = _t(X, dev)
    for kw in (dict(prune_rule=3), dict(prune_rule=1, prune_param=0.0),
               dict(prune_rule=1, prune_param=95.0), dict(prune_rule=2, prune_param=-1.0),
               dict(prune_rule=1, prune_param=60.0, metric=1)):
        with pytest.raises(pkg.RnsmError) as ei:
            pkg.merge(subs, Xd, R=8, L=16, alpha=1.2, **kw)
        assert ei.value.status == 1
