"""The MFMA Gram prune against the float32 walk and the oracle, through the C
ABI (the edge-selection rule of Section 2.2 inside UpdateGraph, Section 4.2).

- Exact rows (small integers, every Gram and norm sum below 2^24): the
  bfloat16 MFMA Gram decides every pair exactly, so merges are bit-exact
  against the oracle, also above dim 128 (the K-sliced kernel).
- Float rows: the hi/lo split Gram decides pairs far from the alpha boundary
  and re-decides the others with the walk's own float32 arithmetic, so the
  merged graph equals the float32 walk's bit for bit (dims 64 to 768, squared
  L2, inner product, cosine), with the default band and with a wide one.
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


@pytest.mark.parametrize("dim", [256, 512, 768])
def test_ksliced_exact_rows_bit_exact(dev, orc, pkg, dim):
    X = inputs.tiny_int(2 * 700, dim, seed=1400 + dim, lo=-8, hi=8)
    subs = [orc.build_graph(X[:700], 32, 24, alpha=1.2, reverse=True),
            orc.build_graph(X[700:], 32, 24, alpha=1.2, reverse=True)]
    ref = orc.merge(subs, X, R=24, L=32, alpha=1.2)
    off, nb, ds, entry = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=24, L=32, alpha=1.2)
    assert pkg.stats()["prune_path"] == 1
    assert entry == ref["entry"]
    assert np.array_equal(off.cpu().numpy(), ref["offsets"])
    assert np.array_equal(nb.cpu().numpy(), ref["nbrs"])
    assert np.array_equal(ds.cpu().numpy().astype(np.float64), ref["dists"])


def _float_case(dim, metric, n, seed):
    if metric == 0:
        g = np.random.default_rng(seed)
        C = g.standard_normal((16, dim)) * 3.0
        X = (C[g.integers(0, 16, 2 * n)] + g.standard_normal((2 * n, dim))).astype(np.float32)
    else:
        X = inputs.mixture_unit(2 * n, dim, comps=16, decay=dim > 128, seed=seed)
        if metric == 2:  # cosine on rows that are not normalised
            X = (X * np.random.default_rng(seed + 1).uniform(0.5, 3.0, (2 * n, 1))).astype(np.float32)
    return np.ascontiguousarray(X)


@pytest.mark.parametrize("dim,metric", [(64, 0), (96, 1), (128, 2), (256, 0), (384, 1),
                                        (768, 2), (768, 0)])
def test_split_gram_equals_float32_walk(dev, orc, pkg, monkeypatch, dim, metric):
    n = 600
    X = _float_case(dim, metric, n, 1500 + dim + metric)
    subs = [orc.build_graph(X[:n], 32, 24, alpha=1.2, metric=metric, reverse=True),
            orc.build_graph(X[n:], 32, 24, alpha=1.2, metric=metric, reverse=True)]
    dsubs, Xd = _dsubs(subs, dev), _t(X, dev)
    run = lambda: [a.cpu() if hasattr(a, "cpu") else a
                   for a in pkg.merge(dsubs, Xd, R=24, L=32, alpha=1.2, metric=metric)]
    monkeypatch.setenv("RNSM_PRUNE", "walk")
    walk = run()
    assert pkg.stats()["prune_path"] == 0
    monkeypatch.delenv("RNSM_PRUNE")
    got = run()
    st = pkg.stats()
    assert st["prune_path"] == 3
    for a, b in zip(got, walk):
        assert (a == b) if isinstance(a, int) else bool((a == b).all())
    monkeypatch.setenv("RNSM_PRUNE_BAND", "-3")  # a wide band: many pairs re-decided
    wide = run()
    st_w = pkg.stats()
    assert st_w["prune_rechecks"] > st["prune_rechecks"] and st_w["prune_rechecks"] > 0
    for a, b in zip(wide, walk):
        assert (a == b) if isinstance(a, int) else bool((a == b).all())
    print(f"[split dim {dim} metric {metric}] rechecked pairs: default band "
          f"{st['prune_rechecks']}, band 2^-3 {st_w['prune_rechecks']}")


def test_split_gram_without_band_stays_within_tolerance(dev, orc, pkg, monkeypatch):
    # the estimate alone (no re-decision): still the float contract's overlap
    n, dim = 600, 768
    X = _float_case(dim, 2, n, 1600)
    subs = [orc.build_graph(X[:n], 32, 24, alpha=1.2, metric=2, reverse=True),
            orc.build_graph(X[n:], 32, 24, alpha=1.2, metric=2, reverse=True)]
    ref = orc.merge(subs, X, R=24, L=32, alpha=1.2, metric=2)
    monkeypatch.setenv("RNSM_PRUNE_BAND", "off")
    off, nb, _, _ = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=24, L=32, alpha=1.2, metric=2)
    st = pkg.stats()
    assert st["prune_path"] == 3 and st["prune_rechecks"] == 0
    off, nb = off.cpu().numpy(), nb.cpu().numpy()
    e = lambda o, b: {(v, int(u)) for v in range(len(o) - 1) for u in b[o[v]:o[v + 1]]}
    eg, er = e(off, nb), e(ref["offsets"], ref["nbrs"])
    assert len(eg & er) / len(er) >= 0.995


def _hub_case(scale=1.0, ns=2600, nt=3000, dim=32, seed=7):
    # sources near the origin, targets far from it except one hub at the
    # origin that every target row links to: almost every source keeps the
    # hub, which then gets some 2,500 reverse edges (candidate lists past
    # 1,024 go to the float32 walk, 16 at a time in key order)
    g = np.random.default_rng(seed)
    S = g.integers(-3, 4, (ns, dim)).astype(np.float32)
    T = (g.integers(4, 9, (nt, dim)) * g.choice([-1, 1], (nt, dim))).astype(np.float32)
    T[0] = 0
    X = np.ascontiguousarray(np.concatenate([S, T]) * np.float32(scale))
    s_off, s_nb = inputs.random_graph(ns, 8, seed=seed + 1)
    r = np.random.default_rng(seed + 2)
    adj = [[int(x) for x in r.choice(np.arange(1, nt), 12, replace=False)]]
    for v in range(1, nt):
        others = [int(x) for x in r.choice(np.arange(1, nt), 6, replace=False) if x != v]
        adj.append([0] + others[:5])
    t_off = np.zeros(nt + 1, np.int64)
    t_off[1:] = np.cumsum([len(a) for a in adj])
    t_nb = np.array([x for a in adj for x in a], np.int32)
    return X, [(s_off, s_nb, 0), (t_off, t_nb, 5)]


def test_long_reverse_list_bit_exact(dev, orc, pkg):
    X, subs = _hub_case()
    ref = orc.merge(subs, X, R=16, L=32, alpha=1.2)
    off, nb, ds, entry = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=16, L=32, alpha=1.2)
    st = pkg.stats()
    assert st["prune_path"] == 1 and st["n_reverse_edges"] > 2000
    nbh = nb.cpu().numpy()
    offh = off.cpu().numpy()
    assert sum(2600 in nbh[offh[v]:offh[v + 1]] for v in range(2600)) > 1024
    assert entry == ref["entry"]
    assert np.array_equal(offh, ref["offsets"]) and np.array_equal(nbh, ref["nbrs"])
    assert np.array_equal(ds.cpu().numpy().astype(np.float64), ref["dists"])


def test_long_reverse_list_float_equals_walk(dev, orc, pkg, monkeypatch):
    X, subs = _hub_case(scale=0.37)
    dsubs, Xd = _dsubs(subs, dev), _t(X, dev)
    got = pkg.merge(dsubs, Xd, R=16, L=32, alpha=1.2)
    assert pkg.stats()["prune_path"] == 3
    monkeypatch.setenv("RNSM_PRUNE", "walk")
    walk = pkg.merge(dsubs, Xd, R=16, L=32, alpha=1.2)
    for a, b in zip(got[:3], walk[:3]):
        assert bool((a == b).all())
    assert got[3] == walk[3]
