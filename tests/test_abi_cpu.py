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
    names = set(re.findall(r"^\s*(?:rnsm_status|const char\*)\s+(\w+)\s*\(", hdr, re.M))
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
