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
    "prune_not_strict": ("return r->a * dwv < dpv;", "return r->a * dwv <= dpv;"),
    "prune_alpha_wrong_side": ("return r->a * dwv < dpv;", "return dwv < r->a * dpv;"),
    "angle_factor_four_dropped": ("c * c > 4.0 * r->a * r->a * dpv * dpw",
                                  "c * c > r->a * r->a * dpv * dpw"),
    "angle_obtuse_not_excluded": ("return c > 0.0 && c * c", "return c * c"),
    "tau_without_factor_three": ("r.a = 3.0 * (double)param;", "r.a = (double)param;"),
    "tau_on_squared_distances": ("return t > 0.0 && sqrt(dwv) < t;", "return t > 0.0 && dwv < t;"),
    "rule_ignored_by_merge": ("const rule_t rule = prune_rule_param(P->prune_rule, P->alpha, P->prune_param);",
                              "const rule_t rule = prune_rule_param(0, P->alpha, P->prune_param);"),
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
    "repair_links_from_farthest": ("if (r < 0 || key_less(d, v, dr, r)) {\n                    r = v;\n                    dr = d;\n                }\n            }\n            P[h].t",
                                   "if (r < 0 || key_less(dr, r, d, v)) {\n                    r = v;\n                    dr = d;\n                }\n            }\n            P[h].t"),
    "repair_ignores_free_slots": ("if (vis[v] && deg[v] < R) queue[nc++] = (int32_t)v;",
                                  "if (vis[v]) queue[nc++] = (int32_t)v;"),
    "repair_replaces_first_entry": ("rows[t * R + R - 1] = (int32_t)P[k].u;",
                                    "rows[t * R] = (int32_t)P[k].u;"),
    "repair_accepts_farthest": ("    if (key_less(x->d, x->u, y->d, y->u)) return -1;",
                                "    if (key_less(x->d, x->u, y->d, y->u)) return 1;"),
    "repair_accepts_one_per_pass": ("const int64_t take = deg[t] < R ? R - deg[t] : 1;",
                                    "const int64_t take = 1;"),
    "repair_every_unreached_proposes": ("if (!vis[u] && !excl[u]) P[np++].u = u;",
                                        "if (!vis[u]) P[np++].u = u;"),
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
