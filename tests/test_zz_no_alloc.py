"""rnsm_search_noalloc (the allocation-free beam search) against rnsm_search.

Both entry points run the same kernels; the allocation-free one keeps its
counters, error flag and cosine norms in the library's static device scratch,
which keeps the previous call's contents. Two calls in a row, the second with
a smaller input, must give exactly the results of rnsm_search, through the C
ABI.
"""
import numpy as np
import pytest

from paper_2602_17099_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case(orc):
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    import paper_2602_17099_amd as pkg
    pkg.lib()
    X = inputs.tiny_int(4000, 32, seed=301)
    Q = inputs.tiny_int(400, 32, seed=302)
    off, nb, entry = orc.build_graph(X, 24, 12, alpha=1.2, reverse=True)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return pkg, t(X), t(Q), t(off), t(nb), entry


def _both(pkg, g, Xd, Qd, ef, k, metric, seeds=None, search=None, qsearch=None):
    import torch
    off, nb, entry = g
    q = Qd if qsearch is None else qsearch
    ref = pkg.search(off, nb, entry, Xd, q, ef, k, seeds=seeds, metric=metric,
                     base_search=search)
    got = pkg.search(off, nb, entry, Xd, q, ef, k, seeds=seeds, metric=metric,
                     base_search=search, noalloc=True)
    torch.cuda.synchronize()
    return ref, got


def test_noalloc_search_equals_search_two_calls(case):
    import torch
    pkg, Xd, Qd, off, nb, entry = case
    g = (off, nb, entry)
    # first call: cosine over every query (norms in the scratch)
    ref, got = _both(pkg, g, Xd, Qd, 48, 20, 2)
    assert torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])
    assert (got[0][:, 0] >= 0).all()
    # second call, smaller: 150 queries, other beam, seeds; the scratch still
    # holds the first call's counters and norms
    seeds = torch.randint(-1, Xd.shape[0], (150, 9), dtype=torch.int32,
                          generator=torch.Generator().manual_seed(3)).to(Xd.device)
    ref, got = _both(pkg, g, Xd, Qd[:150], 24, 10, 2, seeds=seeds)
    assert torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])


def test_noalloc_search_l2_and_16bit_copy(case):
    import torch
    pkg, Xd, Qd, off, nb, entry = case
    g = (off, nb, entry)
    ref, got = _both(pkg, g, Xd, Qd, 64, 64, 0)
    assert torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])
    xb = Xd.to(torch.bfloat16)
    ref, got = _both(pkg, g, Xd, Qd[:77], 33, 5, 0, search=xb, qsearch=Qd[:77].to(torch.bfloat16))
    assert torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])
