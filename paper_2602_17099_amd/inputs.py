"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only draws random numbers (numpy PCG64): vectors shaped like the
paper's workloads (dataset table, Section 6.1) and small random graphs for
tests. It holds none of the method's arithmetic: no distances, no search, no
pruning. Every workload is fully determined by its seed.

Recipes (the paper's datasets are not available; these stand in for them):

* ``tiny_int``: i.i.d. integers uniform in [-8, 8], dim 32, stored as float32.
  Squared-L2 distances between such vectors are exact small integers.
* ``mixture_u8``: 0..255 integers drawn from an equal-weight Gaussian mixture
  (SIFT-like, 128-d). Component centres are 128 + ``center_sd`` * N(0, I),
  points are centre + ``sigma`` * N(0, I), rounded and clipped to [0, 255],
  stored as float32. The centre spread is chosen so that components overlap:
  with well separated components no exact k-NN edge crosses a component and a
  flat graph built from k-NN lists cannot be navigated between them.
* ``mixture_unit``: L2-normalised Gaussian mixture (DEEP-like / embedding-like),
  optional per-dimension scale decaying as 1/sqrt(i).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 0x524E534D  # "RNSM"


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.PCG64(seed))


def tiny_int(n: int, dim: int = 32, seed: int = SEED_BASE + 1, lo: int = -8, hi: int = 8) -> np.ndarray:
    """Integers uniform in [lo, hi] stored as float32, shape (n, dim)."""
    g = rng(seed)
    return g.integers(lo, hi + 1, size=(n, dim)).astype(np.float32)


def mixture_u8(n: int, dim: int = 128, comps: int = 64, sigma: float = 30.0,
               center_sd: float = 20.0, seed: int = SEED_BASE + 2,
               stream: int = 0, centre_range: tuple[float, float] | None = None) -> np.ndarray:
    """Gaussian-mixture integers in [0, 255] stored as float32, shape (n, dim).

    Centres are 128 + center_sd * N(0, I), or uniform on centre_range per
    coordinate when given. ``stream`` selects an independent draw (0: base
    vectors, 1: queries) from the same mixture: the centres depend on
    ``seed`` only.
    """
    gc = rng(seed)
    if centre_range is None:
        centres = 128.0 + center_sd * gc.standard_normal((comps, dim))
    else:
        centres = gc.uniform(centre_range[0], centre_range[1], (comps, dim))
    g = rng(seed * 1000003 + 17 + stream)
    out = np.empty((n, dim), dtype=np.float32)
    chunk = 1 << 16
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        lab = g.integers(0, comps, size=e - s)
        x = centres[lab] + sigma * g.standard_normal((e - s, dim))
        out[s:e] = np.clip(np.rint(x), 0, 255)
    return out


def mixture_unit(n: int, dim: int = 96, comps: int = 256, noise: float = 0.5,
                 decay: bool = False, seed: int = SEED_BASE + 3,
                 stream: int = 0) -> np.ndarray:
    """L2-normalised Gaussian-mixture vectors, float32, shape (n, dim)."""
    gc = rng(seed)
    scale = (1.0 / np.sqrt(np.arange(1, dim + 1))) if decay else np.ones(dim)
    centres = gc.standard_normal((comps, dim)) * scale
    g = rng(seed * 1000003 + 29 + stream)
    out = np.empty((n, dim), dtype=np.float32)
    chunk = 1 << 16
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        lab = g.integers(0, comps, size=e - s)
        x = centres[lab] + noise * scale * g.standard_normal((e - s, dim))
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[s:e] = x
    return out


def uneven_sizes(m: int, lo: int, hi: int, total: int, seed: int) -> list[int]:
    """m sizes drawn log-uniform on [lo, hi], then scaled by a common factor
    (clamped to [lo, hi], water-filling) so that they sum to ``total``."""
    g = rng(seed)
    s = np.exp(g.uniform(np.log(lo), np.log(hi), size=m))
    fa, fb = 1e-6, 1e6
    for _ in range(200):
        f = np.sqrt(fa * fb)
        t = np.clip(s * f, lo, hi).sum()
        if t < total:
            fa = f
        else:
            fb = f
    sizes = np.floor(np.clip(s * fb, lo, hi)).astype(np.int64)
    # hand the rounding remainder to the largest sizes below the cap
    rem = int(total - sizes.sum())
    order = np.argsort(-sizes, kind="stable")
    i = 0
    while rem != 0 and i < 10 * m:
        j = order[i % m]
        step = 1 if rem > 0 else -1
        if lo <= sizes[j] + step <= hi:
            sizes[j] += step
            rem -= step
        i += 1
    return [int(v) for v in sizes]


def random_graph(n: int, deg: int, seed: int, ring: bool = True) -> tuple[np.ndarray, np.ndarray]:
    """Random directed graph as CSR (int64 offsets, int32 local ids).

    Every row has ``deg`` distinct out-neighbours, no self-loop. With ``ring``
    the first neighbour of v is (v + 1) mod n, so the graph is strongly
    connected. Requires deg < n.
    """
    assert 0 < deg < n
    g = rng(seed)
    nbrs = np.empty((n, deg), dtype=np.int32)
    for v in range(n):
        row = []
        if ring:
            row.append((v + 1) % n)
        while len(row) < deg:
            c = int(g.integers(0, n))
            if c != v and c not in row:
                row.append(c)
        nbrs[v] = row
    offsets = np.arange(0, n * deg + 1, deg, dtype=np.int64)
    return offsets, nbrs.reshape(-1)


def projection_graph(X: np.ndarray, deg: int, n_proj: int = 8, seed: int = SEED_BASE + 50
                     ) -> tuple[np.ndarray, np.ndarray]:
    """Cheap locality-structured graph as CSR (int64 offsets, int32 local ids).

    For each of ``n_proj`` seeded random directions the vertices are ordered
    by their projection, and every vertex is linked to the
    ``deg // (2 n_proj)`` vertices on either side of it in that order. A row
    is the union over directions, ascending ids, without self-loops or
    duplicates (so its degree is at most ``deg``). Used as an input graph at
    sizes where building a proximity graph on the CPU would take too long;
    it computes no distance.
    """
    n = X.shape[0]
    w = max(1, deg // (2 * n_proj))
    g = rng(seed)
    cols = []
    for _ in range(n_proj):
        d = g.standard_normal(X.shape[1])
        order = np.argsort(X.astype(np.float64) @ d, kind="stable")
        pos = np.empty(n, dtype=np.int64)
        pos[order] = np.arange(n)
        for o in list(range(-w, 0)) + list(range(1, w + 1)):
            q = pos + o
            ok = (q >= 0) & (q < n)
            c = np.full(n, -1, dtype=np.int64)
            c[ok] = order[q[ok]]
            cols.append(c)
    C = np.sort(np.stack(cols, axis=1), axis=1)
    dup = np.zeros_like(C, dtype=bool)
    dup[:, 1:] = C[:, 1:] == C[:, :-1]
    C[dup] = -1
    C[C == np.arange(n)[:, None]] = -1
    C = np.sort(np.where(C < 0, np.iinfo(np.int64).max, C), axis=1)
    valid = C != np.iinfo(np.int64).max
    valid[:, deg:] = False
    cnt = valid.sum(axis=1)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=offsets[1:])
    return offsets, C[valid].astype(np.int32)


def dirichlet_sizes(m: int, total: int, min_size: int, seed: int) -> list[int]:
    """m sizes: min_size each plus a Dirichlet(1, ..., 1) share of the rest,
    rounded by largest remainder so that they sum to ``total``."""
    assert total >= m * min_size
    g = rng(seed)
    w = g.dirichlet(np.ones(m))
    extra = w * (total - m * min_size)
    base = np.floor(extra).astype(np.int64)
    rem = int(total - m * min_size - base.sum())
    order = np.argsort(-(extra - base), kind="stable")
    base[order[:rem]] += 1
    return [int(min_size + b) for b in base]


def slab_order(X: np.ndarray, seed: int) -> np.ndarray:
    """Row order by the projection on a seeded random unit direction (a slab
    partition when the rows are then cut into consecutive sub-indexes)."""
    d = rng(seed).standard_normal(X.shape[1])
    return np.argsort(X.astype(np.float64) @ (d / np.linalg.norm(d)), kind="stable")


def paper_scale_u8(n: int, seed: int = SEED_BASE + 5, stream: int = 0) -> np.ndarray:
    """The 100,000,000-vector uint8 workload's distribution (any n): dim 96,
    4,096 components with centres uniform on [40, 215] per coordinate, noise
    sigma 30, rounded and clipped to [0, 255]; uint8."""
    return mixture_u8(n, 96, comps=4096, sigma=30.0, seed=seed, stream=stream,
                      centre_range=(40.0, 215.0)).astype(np.uint8)
