"""Parity on small inputs shaped like the other workload configurations
(many uneven sub-indexes with inner product; 768-d cosine with a bfloat16
search copy; uint8 data converted to float16 on the device with many
sub-indexes), through the C ABI, against the float64 oracle."""
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


def _build(orc, X, sizes, K, R, metric):
    subs, b = [], 0
    for n in sizes:
        subs.append(orc.build_graph(X[b:b + n], K, R, alpha=1.2, metric=metric, reverse=True))
        b += n
    return subs


def _edges(off, nb):
    return {(v, int(u)) for v in range(len(off) - 1) for u in nb[off[v]:off[v + 1]]}


def _float_checks(orc, got, ref, X, Q, metric, ef, overlap=0.995):
    # precision contract on float data: edge overlap, recall@10 within 0.002
    # of the oracle's graph, stored distances within 1e-5 of float64
    off, nb, ds, entry = got
    off, nb, ds = off.cpu().numpy(), nb.cpu().numpy(), ds.cpu().numpy()
    assert entry == ref["entry"]
    e_gpu, e_ref = _edges(off, nb), _edges(ref["offsets"], ref["nbrs"])
    frac = len(e_gpu & e_ref) / len(e_ref)
    if overlap is not None:
        assert frac >= overlap, f"edge overlap {frac:.4f}"
    for v in range(0, len(X), max(1, len(X) // 300)):
        for j in range(off[v], off[v + 1]):
            d64 = orc.dist(X[v], X[nb[j]], metric)
            assert abs(ds[j] - d64) <= 1e-5 * max(abs(d64), 1e-3)
    gt, _ = orc.knn_queries(X, Q, 10, metric)
    r_gpu = orc.recall_at_k(orc.search_graph(off, nb, X, Q, entry, ef, metric=metric), gt)
    r_ref = orc.recall_at_k(orc.search_graph(ref["offsets"], ref["nbrs"], X, Q, ref["entry"], ef,
                                             metric=metric), gt)
    assert abs(r_gpu - r_ref) <= 0.002, f"recall {r_gpu:.4f} vs oracle {r_ref:.4f}"
    return frac, r_gpu, r_ref


def test_many_uneven_subindexes_inner_product(dev, orc, pkg):
    # ten uneven sub-indexes (log-uniform sizes), L2-normalised 96-d mixture,
    # inner product, slab partition so that centroid costs differ, MOS order
    sizes = inputs.uneven_sizes(10, 300, 2400, 9000, seed=1101)
    X = inputs.mixture_unit(sum(sizes), 96, comps=64, seed=1102)
    X = np.ascontiguousarray(X[inputs.slab_order(X, 1103)])
    Q = inputs.mixture_unit(500, 96, comps=64, seed=1102, stream=1)
    subs = _build(orc, X, sizes, 32, 16, 1)
    ref = orc.merge(subs, X, R=16, L=32, alpha=1.2, metric=1, use_centroids=True)
    got = pkg.merge(_dsubs(subs, dev), _t(X, dev), R=16, L=32, alpha=1.2, metric=1, flags=2)
    st = pkg.stats()
    assert st["n_ops"] == len(ref["ops"]) and st["prune_path"] == 3
    _float_checks(orc, got, ref, X, Q, 1, 32)


@pytest.mark.parametrize("form", ["float32", "bfloat16"])
def test_768d_cosine(dev, orc, pkg, form):
    # 768-d, per-dimension scale 1/sqrt(i), L2-normalised, cosine; four
    # sub-indexes; R=48, L=96; the bfloat16 copy made by the library
    import torch
    X = inputs.mixture_unit(4 * 450, 768, comps=32, decay=True, seed=1201)
    Q = inputs.mixture_unit(1000, 768, comps=32, decay=True, seed=1201, stream=1)
    subs = _build(orc, X, [450] * 4, 96, 48, 2)
    ref = orc.merge(subs, X, R=48, L=96, alpha=1.2, metric=2)
    Xd = _t(X, dev)
    search = pkg.convert(Xd, torch.bfloat16) if form == "bfloat16" else None
    got = pkg.merge(_dsubs(subs, dev), Xd, R=48, L=96, alpha=1.2, metric=2, search=search)
    st = pkg.stats()
    assert st["prune_path"] == 3  # dim 768: K-sliced MFMA Gram, split rows
    frac, r_gpu, r_ref = _float_checks(orc, got, ref, X, Q, 2, 96, overlap=0.995)
    print(f"[768d {form}] edge overlap {frac:.5f}, recall {r_gpu:.4f} vs {r_ref:.4f}, "
          f"rechecked pairs {st['prune_rechecks']}")


def test_uint8_many_subindexes_float16_search(dev, orc, pkg):
    # uint8 data converted on the device (to float32 rows and a float16
    # search copy), twelve Dirichlet-sized sub-indexes, MOS degree bound 8:
    # integers exact in float16, so the merge is bit-exact
    import torch
    sizes = inputs.dirichlet_sizes(12, 7200, 200, seed=1301)
    U = inputs.mixture_u8(sum(sizes), 96, comps=64, seed=1302).astype(np.uint8)
    X = U.astype(np.float32)
    subs = _build(orc, X, sizes, 48, 32, 0)
    ref = orc.merge(subs, X, R=32, L=64, alpha=1.2, mos_degree=8)
    Ud = _t(U, dev)
    Xd = pkg.convert(Ud, torch.float32)
    H = pkg.convert(Ud, torch.float16)
    off, nb, ds, entry = pkg.merge(_dsubs(subs, dev), Xd, R=32, L=64, alpha=1.2, mos_degree=8,
                                   search=H)
    st = pkg.stats()
    assert st["n_ops"] == len(ref["ops"]) and st["prune_path"] == 1
    assert entry == ref["entry"]
    assert np.array_equal(off.cpu().numpy(), ref["offsets"])
    assert np.array_equal(nb.cpu().numpy(), ref["nbrs"])
    assert np.array_equal(ds.cpu().numpy().astype(np.float64), ref["dists"])


def test_inner_product_ten_subindexes_100k(dev, orc, pkg):
    # the ten-sub-index inner-product workload's shape at 1/100 of its
    # 10,000,000 vectors: log-uniform sizes summing to 100,000, 256-component
    # L2-normalised 96-d mixture in slabs along a seeded direction, exact
    # 64-NN sub-indexes pruned to R = 32 with reverse edges and the
    # reachability repair, MOS degree 4 on centroid costs, R=32, L=64: the
    # float precision contract against the oracle, and the batched form
    # equal to the plain one
    sizes = inputs.uneven_sizes(10, 1000, 40000, 100_000, seed=1501)
    X = inputs.mixture_unit(100_000, 96, comps=256, seed=1502)
    X = np.ascontiguousarray(X[inputs.slab_order(X, 1503)])
    Q = inputs.mixture_unit(1000, 96, comps=256, seed=1502, stream=1)
    subs, b = [], 0
    for n in sizes:
        subs.append(orc.build_graph(X[b:b + n], 64, 32, alpha=1.2, metric=1, reverse=True,
                                    repair=True))
        b += n
    ref = orc.merge(subs, X, R=32, L=64, alpha=1.2, metric=1, mos_degree=4, use_centroids=True)
    Xd = _t(X, dev)
    got = pkg.merge(_dsubs(subs, dev), Xd, R=32, L=64, alpha=1.2, metric=1, mos_degree=4, flags=2)
    st = pkg.stats()
    assert st["n_ops"] == len(ref["ops"])
    frac, r_gpu, r_ref = _float_checks(orc, got, ref, X, Q, 1, 64)
    print(f"[ip 100k] ops {st['n_ops']}, edge overlap {frac:.5f}, recall {r_gpu:.4f} vs "
          f"{r_ref:.4f}")
    bat = pkg.merge(_dsubs(subs, dev), Xd, R=32, L=64, alpha=1.2, metric=1, mos_degree=4,
                    flags=2 | pkg.FLAG_BATCHED)
    assert pkg.stats()["n_rounds"] < st["n_ops"]
    for a, c in zip(got[:3], bat[:3]):
        assert np.array_equal(a.cpu().numpy(), c.cpu().numpy())
    assert got[3] == bat[3]


def _sha(*arrays):
    import hashlib
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_paper_scale_replica_bit_exact(dev, pkg):
    # the 100,000,000-vector uint8 workload at 1/100 scale: 50 Dirichlet-sized
    # sub-indexes, uint8 rows converted on the device to float32 and a
    # float16 search copy, MOS degree bound 8. The oracle's merge of the
    # same replica is stored as digests (tests/golden, written by a script
    # that runs only the oracle): the sub-indexes built here must be the
    # oracle's inputs byte for byte, and the merged graph the oracle's
    import json
    import os
    import torch
    from paper_2602_17099_amd.prepare import knn_l2_exact
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_scale_replica.json")
    gold = json.load(open(path))
    sizes = gold["sizes"]
    U = inputs.paper_scale_u8(sum(sizes))
    assert _sha(U) == gold["inputs_sha256"]
    Ud = _t(U, dev)
    Xd = pkg.convert(Ud, torch.float32)
    H = pkg.convert(Ud, torch.float16)
    del U
    subs, b = [], 0
    for i, n in enumerate(sizes):
        Xi = Xd[b:b + n]
        knn = knn_l2_exact(Xi, None, gold["K"], exclude_self=True)
        off, nb, e = pkg.build_graph(Xi, knn, gold["R"], alpha=gold["alpha"], reverse=True,
                                     alpha_rev=gold["alpha"], repair=True)
        del knn
        assert _sha(off.cpu().numpy(), nb.cpu().numpy(), np.array([e], np.int32)) == \
            gold["subindex_sha256"][i], f"sub-index {i} differs from the oracle's input"
        subs.append((off, nb, e))
        b += n
    off, nb, ds, entry = pkg.merge(subs, Xd, R=gold["R"], L=gold["L"], alpha=gold["alpha"],
                                   mos_degree=gold["mos_degree"], search=H)
    st = pkg.stats()
    assert st["n_ops"] == gold["n_ops"] and entry == gold["entry"]
    off, nb, ds = off.cpu().numpy(), nb.cpu().numpy(), ds.cpu().numpy()
    assert int(off[-1]) == gold["n_edges"]
    for v, row in gold["sample_rows"].items():
        v = int(v)
        assert nb[off[v]:off[v + 1]].tolist() == row, v
    assert _sha(off.astype(np.int64), nb.astype(np.int32), ds.astype(np.float64)) == \
        gold["merged_sha256"]
    print(f"[paper-scale replica] {st['n_ops']} operations, {gold['n_edges']} edges, "
          f"{st['ms_total']:.1f} ms merge, bit-exact")
