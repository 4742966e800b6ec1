"""The batched form's device pieces against the oracle, through the C ABI:
pivot selection on the device (the lazy greedy of Algorithm 2, phase 2, in
parallel rounds) and the batched merge (persistent pivot-group search over
the operations of each round of the plan, graph-captured rounds)."""
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


def _random_lists(orc, n, k, skew, seed):
    g = np.random.default_rng(seed)
    if skew > 0:  # a few vertices in many lists (long lists, many ties)
        p = 1.0 / np.arange(1, n + 1) ** skew
        p /= p.sum()
        nk = np.empty((n, k), np.int32)
        for v in range(n):
            c = g.choice(n, size=3 * k, replace=False, p=p)
            c = c[c != v][:k]
            nk[v] = c
    else:
        nk = np.argsort(g.random((n, n)), axis=1)[:, :k + 1]
        nk = np.array([[u for u in row if u != v][:k] for v, row in enumerate(nk)], np.int32)
    return orc.invert(nk)


@pytest.mark.parametrize("n,k,skew,seed", [(1, 0, 0.0, 0), (50, 3, 0.0, 1), (700, 5, 0.0, 2),
                                           (900, 5, 1.1, 3), (1500, 8, 1.6, 4)])
def test_device_pivot_selection_equals_greedy(dev, orc, pkg, n, k, skew, seed):
    if k == 0:
        off, ids = np.zeros(n + 1, np.int64), np.zeros(0, np.int32)
    else:
        off, ids = _random_lists(orc, n, k, skew, seed)
    ref, order = orc.pivots(off, ids)
    ids_d = _t(ids if len(ids) else np.zeros(1, np.int32), dev)
    got, npv = pkg.select_pivots_device(_t(off, dev), ids_d)
    assert npv == len(order)
    assert np.array_equal(got.cpu().numpy(), ref)


@pytest.mark.parametrize("batch,tail", [(1, 0), (1, 1 << 30), (3, 8192), (16, 0)])
def test_device_pivot_selection_rounds_and_tail(dev, orc, pkg, monkeypatch, batch, tail):
    # many rounds (a skewed list-length mix): rounds checked after every
    # `batch`, the last ones in one workgroup once at most `tail` vertices
    # are uncovered (0: never; 1 << 30: from the first check on)
    monkeypatch.setenv("RNSM_SELECT_BATCH", str(batch))
    monkeypatch.setenv("RNSM_SELECT_TAIL", str(tail))
    n, k = 20000, 5
    g = np.random.default_rng(7)
    p = 1.0 / np.arange(1, n + 1) ** 1.1
    cand = g.choice(n, size=(n, 4 * k), p=p / p.sum())
    nk = np.full((n, k), -1, np.int32)
    for v in range(n):
        row = [int(u) for u in dict.fromkeys(cand[v].tolist()) if u != v][:k]
        nk[v, :len(row)] = row
    off, ids = orc.invert(nk)
    ref, order = orc.pivots(off, ids)
    got, npv = pkg.select_pivots_device(_t(off, dev), _t(ids, dev))
    assert npv == len(order)
    assert np.array_equal(got.cpu().numpy(), ref)


def test_device_pivot_selection_on_expansion_lists(dev, orc, pkg):
    # the reverse lists of a real neighbour expansion (Algorithm 2, phase 1)
    X = inputs.mixture_u8(6000, 32, comps=16, seed=1701)
    off, nb, _ = orc.build_graph(X, 32, 16, alpha=1.2, reverse=True)
    nk = orc.expand(off, nb, X, 5, 16, threads=8)
    rk_off, rk_ids = orc.invert(nk)
    ref, order = orc.pivots(rk_off, rk_ids)
    got, npv = pkg.select_pivots_device(_t(rk_off, dev), _t(rk_ids, dev))
    assert npv == len(order) and np.array_equal(got.cpu().numpy(), ref)


def test_device_pivot_selection_rejects_bad_lists(dev, pkg):
    off = np.array([0, 1, 2], np.int64)
    for ids in ([1, 1], [0, 0], [5, 0]):  # a list naming its owner, an id out of range
        with pytest.raises(pkg.RnsmError) as ei:
            pkg.select_pivots_device(_t(off, dev), _t(np.array(ids, np.int32), dev))
        assert ei.value.status == 1


# ------------------------------------------------- the batched merge form

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


@pytest.fixture(scope="module")
def tiny(orc):
    X = inputs.tiny_int(10000, 32, seed=inputs.SEED_BASE + 1)
    subs = [orc.build_graph(X[:5000], 32, 16, alpha=1.0), orc.build_graph(X[5000:], 32, 16, alpha=1.0)]
    return X, subs


def test_batched_merge_tiny_bit_exact(dev, orc, pkg, tiny):
    X, subs = tiny
    ref = orc.merge(subs, X, R=16, L=32, alpha=1.2, trace=True)
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=16, L=32, alpha=1.2, flags=pkg.FLAG_BATCHED)
    _assert_same_merge(got, ref)
    st = pkg.stats()
    assert st["n_pivots"] == ref["trace"]["n_pivots"]
    assert st["n_source_vertices"] == 5000 and st["n_rounds"] == 1
    # one persistent launch searches every pivot group
    assert st["launches"][1] == 1 and st["queries"][1] + st["queries"][2] == 5000


def test_batched_merge_exact_visited_counts(dev, orc, pkg, tiny, monkeypatch):
    # probing visited table: every vertex evaluated once, so the naive and
    # sliding distance counts of the group search equal the oracle's
    X, subs = tiny
    ref = orc.merge(subs, X, R=16, L=32, alpha=1.2, trace=True)
    monkeypatch.setenv("RNSM_EXACT_VISITED", "1")
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=16, L=32, alpha=1.2, flags=pkg.FLAG_BATCHED)
    _assert_same_merge(got, ref)
    st = pkg.stats()
    tr = ref["trace"]
    assert st["exact_visited"] == 1 and st["hash_evictions"] == 0
    assert st["ndc"] == [tr["ndc_expand"], tr["ndc_naive"], tr["ndc_slide"]]


@pytest.mark.parametrize("all_pivots", [False, True])
@pytest.mark.parametrize("sizes", [[813, 2417, 1290, 3001, 655],
                                   [500, 700, 300, 900, 650, 820, 410, 1000]])
def test_batched_merge_ragged_rounds_bit_exact(dev, orc, pkg, sizes, all_pivots):
    # uneven sub-indexes, MOS plan with unit costs: operations that share no
    # sub-index run in one round (one group search for all of them)
    X = inputs.tiny_int(sum(sizes), 32, seed=201 + len(sizes))
    subs, b = [], 0
    for n in sizes:
        subs.append(orc.build_graph(X[b:b + n], 24, 12, alpha=1.0))
        b += n
    ref = orc.merge(subs, X, R=12, L=24, alpha=1.2, all_pivots=all_pivots)
    flags = pkg.FLAG_BATCHED | (1 if all_pivots else 0)
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=12, L=24, alpha=1.2, flags=flags)
    st = pkg.stats()
    assert st["n_ops"] == len(ref["ops"])
    if len(sizes) == 8:
        assert st["n_rounds"] < st["n_ops"]
    _assert_same_merge(got, ref)


def test_batched_merge_degenerate_bit_exact(dev, orc, pkg):
    # a one-vertex source with no edges
    X = inputs.tiny_int(401, 32, seed=1431)
    s0 = orc.build_graph(X[:400], 24, 12, alpha=1.0)
    subs = [(np.array([0, 0], np.int64), np.zeros(0, np.int32), 0), s0]
    Xm = np.ascontiguousarray(np.concatenate([X[400:401], X[:400]]))
    ref = orc.merge(subs, Xm, R=12, L=24, alpha=1.2)
    got = pkg.merge(_dsubs(subs, dev), _t(Xm, dev), R=12, L=24, alpha=1.2, flags=pkg.FLAG_BATCHED)
    _assert_same_merge(got, ref)


def test_batched_merge_long_lists_bit_exact(dev, orc, pkg):
    # hundreds of reverse k-NN lists of 32 or more (k = 40 of k+ = 48)
    X = inputs.mixture_u8(2600, 16, comps=4, seed=1411)
    subs = [orc.build_graph(X[:1200], 48, 24, alpha=1.2, reverse=True),
            orc.build_graph(X[1200:], 48, 24, alpha=1.2, reverse=True)]
    ref = orc.merge(subs, X, R=24, L=48, alpha=1.2, k=40, kplus=48, trace=True)
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=24, L=48, alpha=1.2, k=40, kplus=48,
                    flags=pkg.FLAG_BATCHED)
    _assert_same_merge(got, ref)
    assert pkg.stats()["n_pivots"] == ref["trace"]["n_pivots"]


@pytest.fixture(scope="module")
def medium(orc):
    X = inputs.mixture_u8(40000, 128, seed=inputs.SEED_BASE + 2)
    n0 = 17011
    subs = [orc.build_graph(X[:n0], 64, 32, alpha=1.2, reverse=True),
            orc.build_graph(X[n0:], 64, 32, alpha=1.2, reverse=True)]
    return X, subs, orc.merge(subs, X, R=32, L=64, alpha=1.2)


@pytest.mark.parametrize("dtype", [None, "bfloat16"])
def test_batched_merge_medium_bit_exact(dev, orc, pkg, medium, dtype):
    # the plain FP32 workload's shape at 1/25 scale; with a bfloat16 search
    # copy (0..255 integers are exact in it) the same graph
    import torch
    X, subs, ref = medium
    Xd = _t(X, dev)
    kw = {} if dtype is None else {"search": Xd.to(getattr(torch, dtype))}
    got = pkg.merge(_dsubs(subs, dev), Xd, R=32, L=64, alpha=1.2, flags=pkg.FLAG_BATCHED, **kw)
    _assert_same_merge(got, ref)
    # the plain form on the same inputs, for the same counts
    st_b = pkg.stats()
    pkg.merge(_dsubs(subs, dev), Xd, R=32, L=64, alpha=1.2, **kw)
    st_p = pkg.stats()
    assert st_b["n_pivots"] == st_p["n_pivots"]
    assert st_b["queries"] == st_p["queries"]


def test_batched_merge_repeated_calls(dev, orc, pkg, tiny, medium):
    # per-source buffers of one call are sized for that call: a smaller
    # merge after a larger one, then the larger again, all bit-exact
    X, subs = tiny
    Xm, subsm, refm = medium
    ref = orc.merge(subs, X, R=16, L=32, alpha=1.2)
    for case in ("m", "t", "m"):
        if case == "m":
            got = pkg.merge(_dsubs(subsm, dev), _t(Xm, dev), R=32, L=64, alpha=1.2,
                            flags=pkg.FLAG_BATCHED)
            _assert_same_merge(got, refm)
        else:
            got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=16, L=32, alpha=1.2,
                            flags=pkg.FLAG_BATCHED)
            _assert_same_merge(got, ref)
