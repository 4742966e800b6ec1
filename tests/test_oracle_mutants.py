"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a private copy of the oracle's C source (a
flipped comparison, a dropped step, a swapped operand), builds it on the CPU,
and runs the pin suite against it: the suite must fail. No GPU involved.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rnsm_oracle.c")

MUTANTS = {
    "distance_not_squared": ("s += t * t;", "s += fabs(t);"),
    "key_tie_reversed": ("(da == db && ia < ib)", "(da == db && ia > ib)"),
    "beam_no_truncation": ("        if (size > ef) size = ef;\n    }\n    for (int i = 0; i < size; ++i) {",
                           "    }\n    for (int i = 0; i < size; ++i) {"),
    "beam_expands_farthest": ("if (!C[i].expanded) { u = i; break; }", "if (!C[i].expanded) { u = i; }"),
    "prune_not_strict": ("if (a * dwv < c[i].d)", "if (a * dwv <= c[i].d)"),
    "prune_alpha_wrong_side": ("if (a * dwv < c[i].d)", "if (dwv < a * c[i].d)"),
    "pivot_tie_reversed": ("(a.g == b.g && a.x < b.x)", "(a.g == b.g && a.x > b.x)"),
    "mos_relay_costliest": ("(best < 0 || C[c * m + v] < C[best * m + v])",
                            "(best < 0 || C[c * m + v] > C[best * m + v])"),
    "no_reverse_prune": ("        if (rcnt[v + 1] == rcnt[v]) continue;", "        continue;"),
    "ops_order_reversed": ("(c1 == c0 && (i1 > i0 || (i1 == i0 && j1 > j0)))",
                           "(c1 == c0 && (i1 < i0 || (i1 == i0 && j1 < j0)))"),
    "larger_is_source": ("int src = (sizes[j] < sizes[i]) ? j : i;",
                         "int src = (sizes[j] > sizes[i]) ? j : i;"),
    "ops_cost_order_reversed": ("int later = c1 > c0 ||", "int later = c1 < c0 ||"),
    "follower_seeded_from_entry": ("res_ids + (int64_t)p * RES,\n" + " " * 35 + "res_n[p], EL",
                                   "&t->entry,\n" + " " * 35 + "1, EL"),
    "follower_seeded_from_top1": ("res_n[p], EL, &vis", "(res_n[p] > 0 ? 1 : 0), EL, &vis"),
    "follower_beam_ef_naive": ("res_n[p], EL, &vis", "res_n[p], L, &vis"),
    "follower_cosine_query_norm_dropped": ("double qn = S->norms ? S->norms[s->base + y] : 1.0;",
                                           "double qn = 1.0;"),
    "merged_entry_smallest": ("if (sizes[i] > sizes[big]) big = i;",
                              "if (sizes[i] < sizes[big]) big = i;"),
    "knn_queries_no_cosine_norm": ("un = sqrt(s);", "un = 1.0;"),
    "knn_queries_unsorted": ("qsort(c, (size_t)n, sizeof(wkey_t), wkey_cmp);", ""),
    "builder_reverse_with_alpha": ("deg2[w] = prune(&S, w, W2, nw, alpha_rev, R",
                                   "deg2[w] = prune(&S, w, W2, nw, alpha, R"),
    "repair_links_from_farthest": ("if (deg[v] < R && (rf < 0 || key_less(d, v, drf, rf)))",
                                   "if (deg[v] < R && (rf < 0 || key_less(drf, rf, d, v)))"),
    "repair_ignores_free_slots": ("P[np].t = rf >= 0 ? rf : r;", "P[np].t = r;"),
    "repair_replaces_first_entry": ("rows[t * R + R - 1] = (int32_t)P[k].u;",
                                    "rows[t * R] = (int32_t)P[k].u;"),
    "repair_accepts_farthest": ("    if (key_less(x->d, x->u, y->d, y->u)) return -1;",
                                "    if (key_less(x->d, x->u, y->d, y->u)) return 1;"),
    "repair_accepts_one_per_pass": ("const int64_t take = deg[t] < R ? R - deg[t] : 1;",
                                    "const int64_t take = 1;"),
    "repair_every_unreached_proposes": ("if (vis[u] || excl[u]) continue;", "if (vis[u]) continue;"),
    "repair_cycles_by_larger_id": ("if (v < w) ins[w] = 1;", "if (v > w) ins[w] = 1;"),
    "repair_single_pass": ("for (int pass = 0; pass < 4096; ++pass)", "for (int pass = 0; pass < 1; ++pass)"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    with tempfile.TemporaryDirectory() as td:
        csrc = os.path.join(td, "rnsm_oracle.c")
        with open(csrc, "w") as f:
            f.write(src.replace(old, new))
        hdr = os.path.join(ROOT, "oracle", "rnsm_oracle.h")
        with open(os.path.join(td, "rnsm_oracle.h"), "w") as f:
            f.write(open(hdr).read())
        so = os.path.join(td, "libmutant.so")
        subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", so, csrc, "-lm"],
                       check=True)
        env = dict(os.environ, RNSM_ORACLE_LIB=so)
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                           env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
        assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
