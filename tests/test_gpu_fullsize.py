"""Parity at the full size of the plain FP32 workload, in the launch
configuration the benchmark times: two sub-indexes of 500,000 vectors, dim
128, integers 0..255 from the 64-component mixture, R=32, L=64, alpha=1.2,
default expansion (k=5, k+=16).

The sub-index graphs come from the seeded projection-graph generator (a
proximity graph built on the CPU would take hours at this size, and graphs
built by the GPU builder may not feed the oracle); they are less navigable
than proximity graphs, which changes how far the searches go but not what
must match. Checks:
  - the oracle's expansion, reverse k-NN inversion and lazy greedy over all
    500,000 source vertices give exactly the GPU's pivot and follower counts;
  - sampled pivots and followers: the oracle's naive search (pivots), local
    sliding from the pivot's beam (followers) and prune reproduce the GPU's
    final row and distances bit for bit (integer data: exact distances);
  - sampled target vertices: the final row is the oracle's prune of the input
    row and the reverse edges present in the output (a property of the
    output; rows with no reverse edge are unchanged);
  - every row: degree <= R, ids in range, no self-loop, no duplicate; sampled
    stored distances equal a float64 recompute;
  - the bfloat16 search copy (exact on these integers) gives the same graph.
"""
import os

import numpy as np
import pytest

from paper_2602_17099_amd import inputs

pytestmark = pytest.mark.gpu

N_SUB, DIM, R, L, ALPHA = 500_000, 128, 32, 64, 1.2


@pytest.fixture(scope="module")
def case(orc):
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    import paper_2602_17099_amd as pkg
    pkg.lib()
    dev = torch.device("cuda:0")
    print(f"\n[fullsize] inputs 2 x {N_SUB} dim {DIM}", flush=True)
    X = inputs.mixture_u8(2 * N_SUB, DIM, seed=inputs.SEED_BASE + 2)
    subs = []
    for i in range(2):
        off, nb = inputs.projection_graph(X[i * N_SUB:(i + 1) * N_SUB], R,
                                          seed=inputs.SEED_BASE + 60 + i)
        subs.append((off, nb, 0))
    Xd = torch.from_numpy(X).to(dev)
    dsubs = [(torch.from_numpy(o).to(dev), torch.from_numpy(nb).to(dev), e) for o, nb, e in subs]
    print("[fullsize] merge (float32 search)", flush=True)
    off, nb, ds, entry = pkg.merge(dsubs, Xd, R=R, L=L, alpha=ALPHA)
    st = pkg.stats()
    print("[fullsize] merge (bfloat16 search)", flush=True)
    b_off, b_nb, _, b_entry = pkg.merge(dsubs, Xd, R=R, L=L, alpha=ALPHA,
                                        search=Xd.to(torch.bfloat16))
    same_bf16 = (b_entry == entry and torch.equal(b_off, off) and torch.equal(b_nb, nb))
    got = dict(off=off.cpu().numpy(), nb=nb.cpu().numpy(), ds=ds.cpu().numpy(), entry=entry,
               stats=st, same_bf16=bool(same_bf16))
    del Xd, dsubs
    torch.cuda.empty_cache()
    return X, subs, got


@pytest.fixture(scope="module")
def plan(orc, case):
    X, subs, _ = case
    return oracle_pivots(orc, X, subs)


def oracle_pivots(orc, X, subs):
    # operation and the oracle's pivots over the whole source sub-index
    ops, _ = orc.plan([N_SUB, N_SUB], 2)
    assert ops == [(0, 1)]
    s_off, s_nb, _ = subs[0]
    threads = max(1, min(16, os.cpu_count() or 1))
    print(f"[fullsize] oracle expansion on {threads} threads", flush=True)
    nk = orc.expand(s_off, s_nb, X[:N_SUB], 5, 16, threads=threads)
    rk_off, rk_ids = orc.invert(nk)
    pivot_of, order = orc.pivots(rk_off, rk_ids)
    assert pivot_of.min() >= -1  # every vertex a pivot (-1) or a follower
    return pivot_of, order


def test_fullsize_pivot_counts(case, plan):
    _, _, got = case
    pivot_of, order = plan
    st = got["stats"]
    assert st["n_ops"] == 1 and st["n_source_vertices"] == N_SUB
    assert st["n_pivots"] == len(order)
    assert st["n_followers"] == N_SUB - len(order)
    assert st["prune_path"] == 1  # exact bfloat16 Gram products on these integers


def _row(got, v):
    a, b = got["off"][v], got["off"][v + 1]
    return got["nb"][a:b], got["ds"][a:b]


def test_fullsize_sampled_source_rows(orc, case, plan):
    X, subs, got = case
    pivot_of, order = plan
    t_off, t_nb, t_entry = subs[1]
    s_off, s_nb, _ = subs[0]
    g = inputs.rng(811)
    piv = g.choice(order, 48, replace=False)
    fol = g.choice(np.flatnonzero(pivot_of >= 0), 48, replace=False)
    for u in list(piv) + list(fol):
        u = int(u)
        p = u if pivot_of[u] < 0 else int(pivot_of[u])
        res, _, _ = orc.beam_search(t_off, t_nb, X, X[p], [t_entry], L, base=N_SUB, n=N_SUB)
        if p != u:
            res, _, _ = orc.beam_search(t_off, t_nb, X, X[u], res, L, base=N_SUB, n=N_SUB)
        W = np.concatenate([s_nb[s_off[u]:s_off[u + 1]], res + N_SUB]).astype(np.int32)
        kept, d = orc.prune(u, W, X, ALPHA, R)
        row, dist = _row(got, u)
        assert np.array_equal(row, kept), f"source vertex {u} (pivot {p})"
        assert np.array_equal(dist.astype(np.float64), d), f"source vertex {u} distances"


def test_fullsize_sampled_target_rows(orc, case):
    X, subs, got = case
    t_off, t_nb, _ = subs[1]
    off, nb = got["off"], got["nb"]
    src_nb = nb[:off[N_SUB]]
    src_of = np.repeat(np.arange(N_SUB, dtype=np.int64), np.diff(off[:N_SUB + 1]))
    g = inputs.rng(812)
    indeg = np.bincount(src_nb[src_nb >= N_SUB] - N_SUB, minlength=N_SUB)
    a, b = np.flatnonzero(indeg > 0), np.flatnonzero(indeg == 0)
    # the most offered targets too: candidate lists of several hundred keys
    # (ordered in global scratch, not LDS)
    heavy = np.argsort(indeg, kind="stable")[-4:]
    with_rev = np.concatenate([g.choice(a, min(48, len(a)), replace=False), heavy]) + N_SUB
    without = g.choice(b, min(16, len(b)), replace=False) + N_SUB
    for v in list(with_rev) + list(without):
        v = int(v)
        vl = v - N_SUB
        row_in = (t_nb[t_off[vl]:t_off[vl + 1]] + N_SUB).astype(np.int32)
        rev = src_of[src_nb == v].astype(np.int32)
        row, dist = _row(got, v)
        if len(rev) == 0:
            assert np.array_equal(row, row_in), f"untouched target {v}"
            d64 = np.array([orc.dist(X[v], X[w]) for w in row])
            assert np.array_equal(dist.astype(np.float64), d64)
            continue
        kept, d = orc.prune(v, np.concatenate([row_in, rev]), X, ALPHA, R)
        assert np.array_equal(row, kept), f"target vertex {v}"
        assert np.array_equal(dist.astype(np.float64), d), f"target vertex {v} distances"


def test_fullsize_invariants(case):
    X, _, got = case
    off, nb, ds = got["off"], got["nb"], got["ds"]
    n = 2 * N_SUB
    assert got["entry"] == 0  # entry of the first of the two equal-size sub-indexes
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == len(nb)
    deg = np.diff(off)
    assert deg.max() <= R and deg.min() >= 1
    assert nb.min() >= 0 and nb.max() < n
    owner = np.repeat(np.arange(n, dtype=np.int64), deg)
    assert not np.any(nb == owner)
    keys = owner * n + nb
    assert len(np.unique(keys)) == len(keys)
    g = inputs.rng(813)
    pick = g.choice(len(nb), 4000, replace=False)
    a = X[owner[pick]].astype(np.float64)
    b = X[nb[pick]].astype(np.float64)
    assert np.array_equal(ds[pick].astype(np.float64), ((a - b) ** 2).sum(1))


def test_fullsize_bf16_search_same_graph(case):
    assert case[2]["same_bf16"]
