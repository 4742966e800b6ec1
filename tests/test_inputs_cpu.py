"""Host checks of the seeded input generators (no GPU): determinism, value
ranges and the size draws of the many-sub-index workloads."""
import numpy as np
import pytest

from paper_2602_17099_amd import inputs


def test_generators_are_deterministic_and_in_range():
    a = inputs.tiny_int(500, 32, seed=5)
    assert np.array_equal(a, inputs.tiny_int(500, 32, seed=5))
    assert a.dtype == np.float32 and a.min() >= -8 and a.max() <= 8
    assert np.array_equal(a, np.rint(a))
    u = inputs.mixture_u8(3000, 128, seed=6)
    assert np.array_equal(u, inputs.mixture_u8(3000, 128, seed=6))
    assert u.min() >= 0 and u.max() <= 255 and np.array_equal(u, np.rint(u))
    # queries: the same mixture, an independent draw
    q = inputs.mixture_u8(3000, 128, seed=6, stream=1)
    assert not np.array_equal(u, q)
    assert abs(float(u.mean()) - float(q.mean())) < 2.0
    m = inputs.mixture_unit(2000, 96, comps=32, seed=7)
    assert np.allclose(np.linalg.norm(m.astype(np.float64), axis=1), 1.0, atol=1e-6)
    assert np.array_equal(m, inputs.mixture_unit(2000, 96, comps=32, seed=7))
    d = inputs.mixture_unit(500, 768, comps=16, decay=True, seed=8)
    # with the 1/sqrt(i) scale the leading dimensions carry most of the energy
    e = (d.astype(np.float64) ** 2).mean(0)
    assert e[:64].sum() > e[-64:].sum() * 4


@pytest.mark.parametrize("m,lo,hi,total,seed", [(10, 50_000, 2_000_000, 10_000_000, 0x524E534D + 3),
                                                (10, 300, 2400, 9000, 1101),
                                                (5, 600, 3001, 9000, 3),
                                                (50, 1000, 400_000, 2_000_000, 9)])
def test_uneven_sizes(m, lo, hi, total, seed):
    s = inputs.uneven_sizes(m, lo, hi, total, seed=seed)
    assert len(s) == m and sum(s) == total
    assert all(lo <= x <= hi for x in s)
    assert s == inputs.uneven_sizes(m, lo, hi, total, seed=seed)
    assert len(set(s)) > 1  # uneven


def test_dirichlet_sizes():
    s = inputs.dirichlet_sizes(50, 1_000_000, 4000, seed=12)
    assert len(s) == 50 and sum(s) == 1_000_000 and min(s) >= 4000
    assert s == inputs.dirichlet_sizes(50, 1_000_000, 4000, seed=12)


def test_slab_order_is_a_sorted_permutation():
    X = inputs.mixture_unit(4000, 96, comps=64, seed=13)
    o = inputs.slab_order(X, 14)
    assert np.array_equal(np.sort(o), np.arange(len(X)))
    d = inputs.rng(14).standard_normal(X.shape[1])
    proj = X[o].astype(np.float64) @ (d / np.linalg.norm(d))
    assert np.all(np.diff(proj) >= 0)
    assert np.array_equal(o, inputs.slab_order(X, 14))
