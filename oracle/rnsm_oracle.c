/*
 * Plain, slow, obviously correct CPU reference of the RNSM merge path.
 *
 * TEST INFRASTRUCTURE ONLY. The product library never links, calls or
 * executes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do. It shares no code with the HIP path.
 *
 * All distances are computed in double precision from the original float32
 * values. Everything is deterministic. Loops over vertices whose work is
 * independent (one search, or one prune, per vertex) may run on several
 * threads (OpenMP, orc_set_threads); each vertex's arithmetic is the same
 * either way, counts are summed, and everything else is sequential. Functions follow
 * the paper (arXiv 2602.17099) in its own order and notation:
 *
 *   beam search ............ Algorithm 1 (Section 2.2)
 *   edge selection prune ... RNG / heuristic edge selection (Section 2.2,
 *                            Section 4.2 "UpdateGraph", Section 5 execution)
 *   RNSM pairwise merge .... Algorithm 2 (Section 4.2): neighbor expansion,
 *                            reverse inversion, lazy greedy pivots, naive
 *                            search, local sliding, graph update with
 *                            reverse edges
 *   MOS .................... Algorithm 3 (Section 5)
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - key order is (distance, global id), ascending, everywhere;
 *   - the prune drops v when some kept w has alpha*d(w,v) < d(p,v) (strict),
 *     stops at R kept, never backfills; alpha is rounded to float32 first and
 *     the product is formed in double;
 *   - searches keep a visited set (Algorithm 1 says "unexpanded neighbor");
 *   - a follower is seeded with every id of its pivot's final beam;
 *   - searches of every operation read only the input sub-index graphs;
 *   - the source of an operation is the smaller sub-index (ties: lower index).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "rnsm_oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

/* threads for the loops over independent vertices (1: sequential) */
void orc_set_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* distances (the paper's delta; L2 is its default, Section 2.1)       */
/* ------------------------------------------------------------------ */

double orc_dist_vec(const float* a, const float* b, int dim, int metric,
                    double na, double nb) {
    if (metric == ORC_L2SQ) {
        double s = 0.0;
        for (int j = 0; j < dim; ++j) {
            double t = (double)a[j] - (double)b[j];
            s += t * t;
        }
        return s;
    }
    double dot = 0.0;
    for (int j = 0; j < dim; ++j) dot += (double)a[j] * (double)b[j];
    if (metric == ORC_IP) return 1.0 - dot;
    /* cosine */
    return 1.0 - dot / (na * nb);
}

void orc_norms(const float* X, int64_t n, int dim, double* out) {
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < dim; ++j) s += (double)X[i * dim + j] * (double)X[i * dim + j];
        out[i] = sqrt(s);
    }
}

typedef struct {
    const float* X;      /* global rows [N x dim] */
    int dim;
    int metric;
    const double* norms; /* [N], used for cosine only (may be NULL otherwise) */
} space_t;

static double dist_ids(const space_t* S, int64_t a, int64_t b) {
    double na = S->norms ? S->norms[a] : 1.0, nb = S->norms ? S->norms[b] : 1.0;
    return orc_dist_vec(S->X + a * S->dim, S->X + b * S->dim, S->dim, S->metric, na, nb);
}

/* (d, id) ascending */
static int key_less(double da, int64_t ia, double db, int64_t ib) {
    return da < db || (da == db && ia < ib);
}

/* ------------------------------------------------------------------ */
/* Algorithm 1: beam search                                            */
/* ------------------------------------------------------------------ */

typedef struct {
    double d;
    int32_t id;      /* local id in the searched graph */
    int expanded;
} cand_t;

/* visited set with a generation counter, reusable across searches */
typedef struct {
    uint32_t* stamp;
    uint32_t gen;
    int64_t n;
} visited_t;

static int visited_init(visited_t* v, int64_t n) {
    v->stamp = (uint32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    v->gen = 0;
    v->n = n;
    return v->stamp != NULL;
}
static void visited_next(visited_t* v) {
    if (++v->gen == 0) {
        memset(v->stamp, 0, sizeof(uint32_t) * (size_t)v->n);
        v->gen = 1;
    }
}

/* insert keeping C sorted by (d, global id); C has room for cap entries */
static void cand_insert(cand_t* C, int* size, double d, int32_t id, int64_t base) {
    int i = *size;
    while (i > 0 && key_less(d, base + id, C[i - 1].d, base + C[i - 1].id)) {
        C[i] = C[i - 1];
        --i;
    }
    C[i].d = d;
    C[i].id = id;
    C[i].expanded = 0;
    ++*size;
}

/*
 * Beam search on one graph (Algorithm 1).
 * G: n vertices, CSR (offsets, nbrs) with local ids; vertex v is global row
 * base + v of S->X. The query is the vector q (with norm qn for cosine).
 * C starts from the seeds (deduplicated, truncated to the ef best); the loop
 * expands the nearest unexpanded entry, inserts its not-yet-visited
 * out-neighbours, and truncates C back to ef, until every entry of C is
 * expanded. Returns |C| and writes C in key order.
 */
static int beam_search(const space_t* S, int64_t n, const int64_t* offsets, const int32_t* nbrs,
                       int64_t base, const float* q, double qn, const int32_t* seeds, int nseeds,
                       int ef, visited_t* vis, int32_t* out_ids, double* out_d, int64_t* ndc,
                       int64_t* n_expand) {
    int maxdeg = 0;
    (void)n;
    /* capacity: ef + largest degree met; grow on demand */
    int cap = ef + nseeds + 64;
    cand_t* C = (cand_t*)malloc(sizeof(cand_t) * (size_t)cap);
    int size = 0;
    visited_next(vis);
    int64_t nd = 0, ne = 0;

    for (int i = 0; i < nseeds; ++i) {
        int32_t s = seeds[i];
        if (s < 0) continue;
        if (vis->stamp[s] == vis->gen) continue; /* dedupe seeds */
        vis->stamp[s] = vis->gen;
        const float* x = S->X + (base + s) * S->dim;
        double xn = S->norms ? S->norms[base + s] : 1.0;
        double d = orc_dist_vec(q, x, S->dim, S->metric, qn, xn);
        ++nd;
        cand_insert(C, &size, d, s, base);
    }
    if (size > ef) size = ef;

    for (;;) {
        int u = -1;
        for (int i = 0; i < size; ++i)
            if (!C[i].expanded) { u = i; break; }
        if (u < 0) break;
        C[u].expanded = 1;
        ++ne;
        int32_t uid = C[u].id;
        int64_t b = offsets[uid], e = offsets[uid + 1];
        int deg = (int)(e - b);
        if (deg > maxdeg) maxdeg = deg;
        if (size + deg > cap) {
            cap = size + deg + 64;
            C = (cand_t*)realloc(C, sizeof(cand_t) * (size_t)cap);
        }
        for (int64_t j = b; j < e; ++j) {
            int32_t v = nbrs[j];
            if (vis->stamp[v] == vis->gen) continue;
            vis->stamp[v] = vis->gen;
            const float* x = S->X + (base + v) * S->dim;
            double xn = S->norms ? S->norms[base + v] : 1.0;
            double d = orc_dist_vec(q, x, S->dim, S->metric, qn, xn);
            ++nd;
            cand_insert(C, &size, d, v, base);
        }
        if (size > ef) size = ef;
    }
    for (int i = 0; i < size; ++i) {
        out_ids[i] = C[i].id;
        out_d[i] = C[i].d;
    }
    free(C);
    if (ndc) *ndc += nd;
    if (n_expand) *n_expand += ne;
    return size;
}

int orc_beam_search(int64_t n, const int64_t* offsets, const int32_t* nbrs, int64_t base,
                    const float* X, int dim, int metric, const double* norms,
                    const float* q, const int32_t* seeds, int nseeds, int ef,
                    int32_t* out_ids, double* out_d, int64_t* ndc) {
    space_t S = {X, dim, metric, norms};
    visited_t vis;
    if (!visited_init(&vis, n)) return -1;
    double qn = 1.0;
    if (metric == ORC_COSINE) {
        double s = 0.0;
        for (int j = 0; j < dim; ++j) s += (double)q[j] * (double)q[j];
        qn = sqrt(s);
    }
    int r = beam_search(&S, n, offsets, nbrs, base, q, qn, seeds, nseeds, ef, &vis, out_ids, out_d,
                        ndc, NULL);
    free(vis.stamp);
    return r;
}

/* ------------------------------------------------------------------ */
/* Edge selection (RNG rule with alpha)                                */
/* ------------------------------------------------------------------ */

typedef struct {
    double d;
    int32_t id; /* global */
} wkey_t;

static int wkey_cmp(const void* a, const void* b) {
    const wkey_t* x = (const wkey_t*)a;
    const wkey_t* y = (const wkey_t*)b;
    if (key_less(x->d, x->id, y->d, y->id)) return -1;
    if (key_less(y->d, y->id, x->d, x->id)) return 1;
    return 0;
}

/*
 * The rule by which an already kept w removes a later candidate v, from the
 * distances d(p,v), d(p,w), d(w,v) (squared L2 for rules 1 and 2):
 *   0  alpha (the RNG rule with a factor; alpha = 1 is NSG's MRNG):
 *      alpha * d(w, v) < d(p, v);
 *   1  angle (SSG): the angle at p between v and w is below theta, i.e.
 *      cos = (d(p,v) + d(p,w) - d(w,v)) / (2 sqrt(d(p,v) d(p,w))) exceeds
 *      cos(theta), decided as c > 0 and c^2 > 4 cos^2(theta) d(p,v) d(p,w)
 *      with c the numerator (0 < theta <= 90 degrees);
 *   2  tau (tau-MNG): w lies in the tau-lune of (p, v): sqrt(d(w, v)) <
 *      sqrt(d(p, v)) - 3 tau (w precedes v, so d(p, w) <= d(p, v)).
 * a: alpha, cos(theta) or 3 tau, formed once in double (prune_rule_param).
 */
typedef struct {
    int kind;
    double a;
} rule_t;

static int rule_drops(const rule_t* r, double dpv, double dpw, double dwv) {
    if (r->kind == 1) {
        const double c = dpv + dpw - dwv;
        return c > 0.0 && c * c > 4.0 * r->a * r->a * dpv * dpw;
    }
    if (r->kind == 2) {
        const double t = sqrt(dpv) - r->a;
        return t > 0.0 && sqrt(dwv) < t;
    }
    return r->a * dwv < dpv;
}

/* the rule's constant from the user's parameter: alpha as given (float32),
 * cos(theta) for theta in degrees, 3 tau */
static rule_t prune_rule_param(int kind, float alpha, float param) {
    rule_t r;
    r.kind = kind;
    if (kind == 1)
        r.a = cos((double)param * (3.14159265358979323846 / 180.0));
    else if (kind == 2)
        r.a = 3.0 * (double)param;
    else
        r.a = (double)alpha;
    return r;
}

/*
 * Prune(p, W): sort the candidates by (d(p,.), id); walk them in order and
 * keep v unless some already kept w removes it by the rule (alpha: alpha *
 * d(w, v) < d(p, v)); stop once R are kept. Duplicates and p itself are
 * removed first.
 */
static int prune_rule(const space_t* S, int64_t p, const int32_t* W, int nW, const rule_t* rule,
                      int R, int32_t* out_ids, double* out_d);

static int prune(const space_t* S, int64_t p, const int32_t* W, int nW, float alpha, int R,
                 int32_t* out_ids, double* out_d) {
    const rule_t r = prune_rule_param(0, alpha, 0.0f);
    return prune_rule(S, p, W, nW, &r, R, out_ids, out_d);
}

static int prune_rule(const space_t* S, int64_t p, const int32_t* W, int nW, const rule_t* rule,
                      int R, int32_t* out_ids, double* out_d) {
    wkey_t* c = (wkey_t*)malloc(sizeof(wkey_t) * (size_t)(nW > 0 ? nW : 1));
    int nc = 0;
    for (int i = 0; i < nW; ++i) {
        int32_t v = W[i];
        if (v < 0 || v == p) continue;
        int dup = 0;
        for (int j = 0; j < nc; ++j)
            if (c[j].id == v) { dup = 1; break; }
        if (dup) continue;
        c[nc].id = v;
        c[nc].d = dist_ids(S, p, v);
        ++nc;
    }
    qsort(c, (size_t)nc, sizeof(wkey_t), wkey_cmp);
    int nk = 0;
    for (int i = 0; i < nc && nk < R; ++i) {
        int dominated = 0;
        for (int j = 0; j < nk; ++j) {
            double dwv = dist_ids(S, out_ids[j], c[i].id);
            if (rule_drops(rule, c[i].d, out_d[j], dwv)) { dominated = 1; break; }
        }
        if (!dominated) {
            out_ids[nk] = c[i].id;
            out_d[nk] = c[i].d;
            ++nk;
        }
    }
    free(c);
    return nk;
}

int orc_prune_rule(int64_t p, const int32_t* W, int nW, const float* X, int dim, int metric,
                   const double* norms, int rule, float alpha, float param, int R,
                   int32_t* out_ids, double* out_d) {
    space_t S = {X, dim, metric, norms};
    const rule_t r = prune_rule_param(rule, alpha, param);
    return prune_rule(&S, p, W, nW, &r, R, out_ids, out_d);
}

int orc_prune(int64_t p, const int32_t* W, int nW, const float* X, int dim, int metric,
              const double* norms, float alpha, int R, int32_t* out_ids, double* out_d) {
    space_t S = {X, dim, metric, norms};
    return prune(&S, p, W, nW, alpha, R, out_ids, out_d);
}

/* ------------------------------------------------------------------ */
/* Algorithm 2, phase 1: neighbor expansion and reverse inversion      */
/* ------------------------------------------------------------------ */

/*
 * N_k(v): beam search in the source graph from v itself with effort k+,
 * keep the first k results other than v. nk_out is [n x k], -1 padded.
 */
static int expand_neighbors(const space_t* S, int64_t n, const int64_t* offsets,
                            const int32_t* nbrs, int64_t base, int k, int kplus,
                            int32_t* nk_out, int64_t* ndc, int64_t v0, int64_t v1) {
    int64_t nd = 0;
    int fail = 0;
#pragma omp parallel reduction(+ : nd) reduction(| : fail)
    {
        visited_t vis;
        int32_t* ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)kplus);
        double* ds = (double*)malloc(sizeof(double) * (size_t)kplus);
        const int ok = visited_init(&vis, n) && ids && ds;
        fail |= !ok;
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = v0; v < v1; ++v) {
            if (!ok) continue;
            int32_t seed = (int32_t)v;
            const float* q = S->X + (base + v) * S->dim;
            double qn = S->norms ? S->norms[base + v] : 1.0;
            int c = beam_search(S, n, offsets, nbrs, base, q, qn, &seed, 1, kplus, &vis, ids, ds,
                                &nd, NULL);
            int t = 0;
            for (int i = 0; i < c && t < k; ++i)
                if (ids[i] != v) nk_out[v * k + t++] = ids[i];
            for (; t < k; ++t) nk_out[v * k + t] = -1;
        }
        free(ids);
        free(ds);
        free(vis.stamp);
    }
    if (ndc) *ndc += nd;
    return fail ? -1 : 0;
}

int orc_expand(int64_t n, const int64_t* offsets, const int32_t* nbrs, int64_t base,
               const float* X, int dim, int metric, const double* norms, int k, int kplus,
               int32_t* nk_out) {
    space_t S = {X, dim, metric, norms};
    return expand_neighbors(&S, n, offsets, nbrs, base, k, kplus, nk_out, NULL, 0, n);
}

/* rows v0..v1-1 of N_k only (independent per vertex: callers may run ranges
   on separate threads; nk_out is still indexed by vertex) */
int orc_expand_range(int64_t n, const int64_t* offsets, const int32_t* nbrs, int64_t base,
                     const float* X, int dim, int metric, const double* norms, int k, int kplus,
                     int64_t v0, int64_t v1, int32_t* nk_out) {
    space_t S = {X, dim, metric, norms};
    if (v0 < 0 || v1 > n || v0 > v1) return -1;
    return expand_neighbors(&S, n, offsets, nbrs, base, k, kplus, nk_out, NULL, v0, v1);
}

/* R_k(x) = { y : x in N_k(y) }, each list in ascending id order. */
int orc_invert(int64_t n, const int32_t* nk, int k, int64_t* rk_off, int32_t* rk_ids) {
    for (int64_t i = 0; i <= n; ++i) rk_off[i] = 0;
    for (int64_t y = 0; y < n; ++y)
        for (int j = 0; j < k; ++j) {
            int32_t x = nk[y * k + j];
            if (x >= 0) rk_off[x + 1]++;
        }
    for (int64_t i = 0; i < n; ++i) rk_off[i + 1] += rk_off[i];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) fill[i] = rk_off[i];
    for (int64_t y = 0; y < n; ++y) /* y ascending => every list sorted */
        for (int j = 0; j < k; ++j) {
            int32_t x = nk[y * k + j];
            if (x >= 0) rk_ids[fill[x]++] = (int32_t)y;
        }
    free(fill);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2, phase 2: lazy greedy pivot selection                   */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t g;
    int32_t x;
} hent_t;

/* max-heap on gain, ties: smaller id first */
static int hent_above(hent_t a, hent_t b) { return a.g > b.g || (a.g == b.g && a.x < b.x); }

static void heap_push(hent_t* h, int64_t* n, hent_t e) {
    int64_t i = (*n)++;
    h[i] = e;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!hent_above(h[i], h[p])) break;
        hent_t t = h[i]; h[i] = h[p]; h[p] = t;
        i = p;
    }
}

static hent_t heap_pop(hent_t* h, int64_t* n) {
    hent_t top = h[0];
    h[0] = h[--*n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *n && hent_above(h[l], h[m])) m = l;
        if (r < *n && hent_above(h[r], h[m])) m = r;
        if (m == i) break;
        hent_t t = h[i]; h[i] = h[m]; h[m] = t;
        i = m;
    }
    return top;
}

/*
 * Heap of (|R_k(x)|, x). Pop the top; drop it when x is covered; when the
 * gain |R_k(x) \ Covered| fell below the stored key, push it back with the
 * new gain; otherwise x becomes a pivot with followers F_x = R_k(x) \ Covered
 * and Covered grows by {x} and R_k(x).
 * pivot_of[y] = x for a follower y of x, -1 for a pivot.
 * order[0..*n_piv) lists the pivots in selection order.
 */
int orc_pivots(int64_t n, const int64_t* rk_off, const int32_t* rk_ids, int32_t* pivot_of,
               int32_t* order, int64_t* n_piv) {
    hent_t* h = (hent_t*)malloc(sizeof(hent_t) * (size_t)(n > 0 ? n : 1));
    char* covered = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t hn = 0, np = 0;
    for (int64_t x = 0; x < n; ++x) {
        hent_t e = {rk_off[x + 1] - rk_off[x], (int32_t)x};
        heap_push(h, &hn, e);
    }
    for (int64_t i = 0; i < n; ++i) pivot_of[i] = -2; /* unassigned */
    while (hn > 0) {
        hent_t e = heap_pop(h, &hn);
        int32_t x = e.x;
        if (covered[x]) continue;
        int64_t g = 0;
        for (int64_t j = rk_off[x]; j < rk_off[x + 1]; ++j)
            if (!covered[rk_ids[j]]) ++g;
        if (g < e.g) {
            hent_t r = {g, x};
            heap_push(h, &hn, r);
            continue;
        }
        for (int64_t j = rk_off[x]; j < rk_off[x + 1]; ++j) {
            int32_t y = rk_ids[j];
            if (!covered[y]) pivot_of[y] = x;
        }
        pivot_of[x] = -1;
        order[np++] = x;
        covered[x] = 1;
        for (int64_t j = rk_off[x]; j < rk_off[x + 1]; ++j) covered[rk_ids[j]] = 1;
    }
    *n_piv = np;
    free(h);
    free(covered);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 3: merge order selection                                  */
/* ------------------------------------------------------------------ */

#define HOP_INF 0x3fffffff

static void mos_hops(int m, const char* adj, int* H) {
    int* q = (int*)malloc(sizeof(int) * (size_t)m);
    for (int s = 0; s < m; ++s) {
        for (int t = 0; t < m; ++t) H[s * m + t] = HOP_INF;
        H[s * m + s] = 0;
        int qh = 0, qt = 0;
        q[qt++] = s;
        while (qh < qt) {
            int u = q[qh++];
            for (int v = 0; v < m; ++v)
                if (adj[u * m + v] && H[s * m + v] == HOP_INF) {
                    H[s * m + v] = H[s * m + u] + 1;
                    q[qt++] = v;
                }
        }
    }
    free(q);
}

/* cost matrix: Euclidean distance of centroids, or 1 for every pair when
 * centroids is NULL (random partitions) */
void orc_mos_cost(int m, const double* centroids, int dim, double* C) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            if (i == j) { C[i * m + j] = 0.0; continue; }
            if (!centroids) { C[i * m + j] = 1.0; continue; }
            double s = 0.0;
            for (int t = 0; t < dim; ++t) {
                double d = centroids[i * dim + t] - centroids[j * dim + t];
                s += d * d;
            }
            C[i * m + j] = sqrt(s);
        }
}

/*
 * Vertices are visited in ascending order of their mean cost to their
 * min(R, m-1) nearest others (ties: index). For each v, while some x lies
 * more than delta hops away, take the cheapest such x (ties: index):
 * both below the degree bound -> edge (v,x); x saturated -> relay to the
 * cheapest unsaturated neighbour x' of x, edge (v,x'); v saturated -> relay
 * from the cheapest unsaturated neighbour v' of v, edge (v',x); otherwise, or
 * when no relay exists, edge (v,x) as a counted fallback. Hops are recomputed
 * by BFS after each edge. Edges are written in insertion order.
 * Requires delta >= 2 (a relay puts x within two hops of v).
 */
int orc_mos(int m, const double* C, int R, int delta, int32_t* out_edges, int cap,
            int* n_edges, int* n_fallback) {
    if (m < 1 || R < 1 || delta < 2) return -1;
    char* adj = (char*)calloc((size_t)m * m, 1);
    int* H = (int*)malloc(sizeof(int) * (size_t)m * m);
    int* deg = (int*)calloc((size_t)m, sizeof(int));
    int* order = (int*)malloc(sizeof(int) * (size_t)m);
    double* avg = (double*)malloc(sizeof(double) * (size_t)m);
    double* tmp = (double*)malloc(sizeof(double) * (size_t)m);
    int ne = 0, nf = 0;
    int r = R < m - 1 ? R : m - 1;
    for (int i = 0; i < m; ++i) {
        int t = 0;
        for (int j = 0; j < m; ++j)
            if (j != i) tmp[t++] = C[i * m + j];
        /* partial selection sort of the r smallest */
        double s = 0.0;
        for (int a = 0; a < r; ++a) {
            int best = a;
            for (int b = a + 1; b < t; ++b)
                if (tmp[b] < tmp[best]) best = b;
            double x = tmp[a]; tmp[a] = tmp[best]; tmp[best] = x;
            s += tmp[a];
        }
        avg[i] = r > 0 ? s / r : 0.0;
        order[i] = i;
    }
    for (int a = 1; a < m; ++a) { /* stable insertion sort by (avg, index) */
        int v = order[a], b = a;
        while (b > 0 && avg[order[b - 1]] > avg[v]) { order[b] = order[b - 1]; --b; }
        order[b] = v;
    }
    mos_hops(m, adj, H);
    for (int oi = 0; oi < m; ++oi) {
        int v = order[oi];
        for (;;) {
            int x = -1;
            for (int c = 0; c < m; ++c) {
                if (c == v || H[v * m + c] <= delta) continue;
                if (x < 0 || C[v * m + c] < C[v * m + x]) x = c;
            }
            if (x < 0) break;
            int a = v, b = x, fallback = 0;
            if (deg[v] < R && deg[x] < R) {
                /* direct edge */
            } else if (deg[v] < R && deg[x] >= R) {
                int best = -1;
                for (int c = 0; c < m; ++c)
                    if (adj[x * m + c] && c != v && deg[c] < R &&
                        (best < 0 || C[c * m + v] < C[best * m + v]))
                        best = c;
                if (best >= 0) b = best; else fallback = 1;
            } else if (deg[v] >= R && deg[x] < R) {
                int best = -1;
                for (int c = 0; c < m; ++c)
                    if (adj[v * m + c] && c != x && deg[c] < R &&
                        (best < 0 || C[c * m + x] < C[best * m + x]))
                        best = c;
                if (best >= 0) a = best; else fallback = 1;
            } else {
                fallback = 1;
            }
            if (ne >= cap) { ne = -1; break; }
            adj[a * m + b] = adj[b * m + a] = 1;
            deg[a]++; deg[b]++;
            out_edges[2 * ne] = a;
            out_edges[2 * ne + 1] = b;
            ++ne;
            nf += fallback;
            mos_hops(m, adj, H);
        }
        if (ne < 0) break;
    }
    *n_edges = ne;
    *n_fallback = nf;
    free(adj); free(H); free(deg); free(order); free(avg); free(tmp);
    return ne < 0 ? -2 : 0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2, phase 3 + graph update, for one operation s -> t        */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n, base;
    const int64_t* offsets;
    const int32_t* nbrs;
    int32_t entry;
} sub_t;

typedef struct {
    int32_t* rows;  /* [N x R] global ids */
    double* dists;  /* [N x R] */
    int32_t* deg;   /* [N] */
    int R;
} rows_t;

static int64_t g_ndc_expand, g_ndc_naive, g_ndc_slide;

static int pair_op(const space_t* S, const sub_t* s, const sub_t* t, const rows_t* rows,
                   const orc_params_t* P, const int32_t* pivot_of, const int32_t* piv_order,
                   int64_t n_piv, int32_t* trace_res_ids, double* trace_res_d) {
    const int L = P->ef_naive, EL = P->ef_slide, R = P->R;
    const int RES = L > EL ? L : EL;
    const rule_t rule = prune_rule_param(P->prune_rule, P->alpha, P->prune_param);
    int32_t* res_ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)(s->n * RES));
    double* res_d = (double*)malloc(sizeof(double) * (size_t)(s->n * RES));
    int* res_n = (int*)calloc((size_t)s->n, sizeof(int));
    if (!res_ids || !res_d || !res_n) return -1;
    int64_t ndc_naive = 0, ndc_slide = 0;
    int fail = 0;

    /* naive search of every pivot from the target's default entry point
     * (each search is independent: one visited set per thread) */
#pragma omp parallel reduction(+ : ndc_naive) reduction(| : fail)
    {
        visited_t vis;
        const int ok = visited_init(&vis, t->n);
        fail |= !ok;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n_piv; ++i) {
            if (!ok) continue;
            int64_t p = piv_order[i];
            const float* q = S->X + (s->base + p) * S->dim;
            double qn = S->norms ? S->norms[s->base + p] : 1.0;
            res_n[p] = beam_search(S, t->n, t->offsets, t->nbrs, t->base, q, qn, &t->entry, 1, L,
                                   &vis, res_ids + p * RES, res_d + p * RES, &ndc_naive, NULL);
        }
        free(vis.stamp);
    }
    /* local sliding of every follower from its pivot's results (every pivot
     * is done: the loop above has ended) */
#pragma omp parallel reduction(+ : ndc_slide) reduction(| : fail)
    {
        visited_t vis;
        const int ok = visited_init(&vis, t->n);
        fail |= !ok;
#pragma omp for schedule(dynamic, 16)
        for (int64_t y = 0; y < s->n; ++y) {
            int32_t p = pivot_of[y];
            if (p < 0 || !ok) continue;
            const float* q = S->X + (s->base + y) * S->dim;
            double qn = S->norms ? S->norms[s->base + y] : 1.0;
            res_n[y] = beam_search(S, t->n, t->offsets, t->nbrs, t->base, q, qn, res_ids + (int64_t)p * RES,
                                   res_n[p], EL, &vis, res_ids + y * RES, res_d + y * RES,
                                   &ndc_slide, NULL);
        }
        free(vis.stamp);
    }
    g_ndc_naive += ndc_naive;
    g_ndc_slide += ndc_slide;
    if (fail) {
        free(res_ids); free(res_d); free(res_n);
        return -1;
    }
    if (trace_res_ids) {
        for (int64_t y = 0; y < s->n; ++y)
            for (int j = 0; j < RES; ++j) {
                trace_res_ids[y * RES + j] = j < res_n[y] ? res_ids[y * RES + j] : -1;
                trace_res_d[y * RES + j] = j < res_n[y] ? res_d[y * RES + j] : INFINITY;
            }
    }

    /* source update: concatenate with the current row, prune to R (each
     * vertex reads and writes only its own row) */
#pragma omp parallel
    {
        int32_t* W = (int32_t*)malloc(sizeof(int32_t) * (size_t)(R + RES + 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t u = 0; u < s->n; ++u) {
            int64_t gu = s->base + u;
            int nw = 0;
            for (int j = 0; j < rows->deg[gu]; ++j) W[nw++] = rows->rows[gu * R + j];
            for (int j = 0; j < res_n[u]; ++j) W[nw++] = (int32_t)(t->base + res_ids[u * RES + j]);
            rows->deg[gu] = prune_rule(S, gu, W, nw, &rule, R, rows->rows + gu * R,
                                       rows->dists + gu * R);
        }
        free(W);
    }

    /* reverse edges: every kept u -> v with v in the target */
    int64_t* rcnt = (int64_t*)calloc((size_t)(t->n + 1), sizeof(int64_t));
    for (int64_t u = 0; u < s->n; ++u) {
        int64_t gu = s->base + u;
        for (int j = 0; j < rows->deg[gu]; ++j) {
            int64_t v = rows->rows[gu * R + j] - t->base;
            if (v >= 0 && v < t->n) rcnt[v + 1]++;
        }
    }
    for (int64_t v = 0; v < t->n; ++v) rcnt[v + 1] += rcnt[v];
    int32_t* rev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(rcnt[t->n] > 0 ? rcnt[t->n] : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(t->n > 0 ? t->n : 1));
    for (int64_t v = 0; v < t->n; ++v) fill[v] = rcnt[v];
    for (int64_t u = 0; u < s->n; ++u) {
        int64_t gu = s->base + u;
        for (int j = 0; j < rows->deg[gu]; ++j) {
            int64_t v = rows->rows[gu * R + j] - t->base;
            if (v >= 0 && v < t->n) rev[fill[v]++] = (int32_t)gu;
        }
    }
    int maxrev = 0;
    for (int64_t v = 0; v < t->n; ++v)
        if (rcnt[v + 1] - rcnt[v] > maxrev) maxrev = (int)(rcnt[v + 1] - rcnt[v]);
#pragma omp parallel
    {
        int32_t* W2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(R + maxrev + 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < t->n; ++v) {
            if (rcnt[v + 1] == rcnt[v]) continue;
            int64_t gv = t->base + v;
            int nw = 0;
            for (int j = 0; j < rows->deg[gv]; ++j) W2[nw++] = rows->rows[gv * R + j];
            for (int64_t j = rcnt[v]; j < rcnt[v + 1]; ++j) W2[nw++] = rev[j];
            rows->deg[gv] = prune_rule(S, gv, W2, nw, &rule, R, rows->rows + gv * R,
                                       rows->dists + gv * R);
        }
        free(W2);
    }
    free(rev); free(fill); free(rcnt);
    free(res_ids); free(res_d); free(res_n);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Whole merge: MOS plan, operation order, sequential operations        */
/* ------------------------------------------------------------------ */

/*
 * Operation plan: MOS edges (Algorithm 3) executed in ascending order of
 * (cost, min index, max index); each runs from the smaller sub-index to the
 * larger one (ties: the lower index is the source). out_ops: 2*cap int32.
 */
int orc_plan(int m, const int64_t* sizes, const double* centroids, int dim, int R, int delta,
             int32_t* out_ops, int cap, int* n_ops, int* n_fallback) {
    double* C = (double*)malloc(sizeof(double) * (size_t)m * m);
    orc_mos_cost(m, centroids, dim, C);
    int r = orc_plan_cost(m, sizes, C, R, delta, out_ops, cap, n_ops, n_fallback);
    free(C);
    return r;
}

/* the same plan from a given cost matrix C [m x m] */
int orc_plan_cost(int m, const int64_t* sizes, const double* C, int R, int delta,
                  int32_t* out_ops, int cap, int* n_ops, int* n_fallback) {
    int ne = 0, nf = 0;
    int32_t* edges = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(m * m + 1));
    if (m >= 2 && orc_mos(m, C, R, delta, edges, m * m, &ne, &nf) != 0) {
        free(edges);
        return -1;
    }
    if (ne > cap) { free(edges); return -2; }
    /* normalise every edge to (min, max) */
    for (int a = 0; a < ne; ++a) {
        int32_t e0 = edges[2 * a], e1 = edges[2 * a + 1];
        edges[2 * a] = e0 < e1 ? e0 : e1;
        edges[2 * a + 1] = e0 < e1 ? e1 : e0;
    }
    /* stable insertion sort by (cost, min index, max index) */
    for (int a = 1; a < ne; ++a) {
        int32_t i0 = edges[2 * a], j0 = edges[2 * a + 1];
        int b = a;
        while (b > 0) {
            int32_t i1 = edges[2 * (b - 1)], j1 = edges[2 * (b - 1) + 1];
            double c0 = C[i0 * m + j0], c1 = C[i1 * m + j1];
            int later = c1 > c0 || (c1 == c0 && (i1 > i0 || (i1 == i0 && j1 > j0)));
            if (!later) break;
            edges[2 * b] = edges[2 * (b - 1)];
            edges[2 * b + 1] = edges[2 * (b - 1) + 1];
            --b;
        }
        edges[2 * b] = i0;
        edges[2 * b + 1] = j0;
    }
    /* direction: the smaller sub-index is the source; ties: lower index */
    for (int a = 0; a < ne; ++a) {
        int i = edges[2 * a], j = edges[2 * a + 1];
        int src = (sizes[j] < sizes[i]) ? j : i;
        int dst = src == i ? j : i;
        out_ops[2 * a] = src;
        out_ops[2 * a + 1] = dst;
    }
    *n_ops = ne;
    if (n_fallback) *n_fallback = nf;
    free(edges);
    return 0;
}

int orc_merge(int m, const int64_t* sizes, const int64_t* offsets_cat, const int32_t* nbrs_cat,
              const int32_t* entries, const float* X, int dim, const orc_params_t* P,
              int32_t* out_rows, double* out_dists, int32_t* out_deg, int32_t* out_entry,
              int32_t* out_ops, int* out_nops, orc_trace_t* trace) {
    if (m < 1 || P->R < 1 || P->ef_naive < 1 || P->ef_slide < 1 || P->k < 1 || P->kplus < P->k)
        return -1;
    if (P->prune_rule < 0 || P->prune_rule > 2 || (P->prune_rule != 0 && P->metric != ORC_L2SQ))
        return -1;
    if (P->prune_rule == 1 && !(P->prune_param > 0.0f && P->prune_param <= 90.0f)) return -1;
    if (P->prune_rule == 2 && !(P->prune_param >= 0.0f)) return -1;
    const int R = P->R;
    int64_t N = 0;
    sub_t* subs = (sub_t*)malloc(sizeof(sub_t) * (size_t)m);
    int64_t ooff = 0, noff = 0;
    for (int i = 0; i < m; ++i) {
        subs[i].n = sizes[i];
        subs[i].base = N;
        subs[i].offsets = offsets_cat + ooff;
        subs[i].nbrs = nbrs_cat + noff;
        subs[i].entry = entries[i];
        noff += subs[i].offsets[sizes[i]];
        ooff += sizes[i] + 1;
        N += sizes[i];
    }
    double* norms = NULL;
    if (P->metric == ORC_COSINE) {
        norms = (double*)malloc(sizeof(double) * (size_t)N);
        orc_norms(X, N, dim, norms);
    }
    space_t S = {X, dim, P->metric, norms};
    rows_t rows = {out_rows, out_dists, out_deg, R};
    /* rows start as the input rows in global ids */
    for (int i = 0; i < m; ++i)
        for (int64_t v = 0; v < subs[i].n; ++v) {
            int64_t g = subs[i].base + v;
            int64_t b = subs[i].offsets[v], e = subs[i].offsets[v + 1];
            if (e - b > R) { free(subs); free(norms); return -2; }
            out_deg[g] = (int32_t)(e - b);
            for (int64_t j = b; j < e; ++j) {
                out_rows[g * R + (j - b)] = (int32_t)(subs[i].base + subs[i].nbrs[j]);
                out_dists[g * R + (j - b)] = dist_ids(&S, g, subs[i].base + subs[i].nbrs[j]);
            }
        }

    /* plan */
    int cap = m * m, ne = 0;
    double* cent = NULL;
    if (P->use_centroids) {
        cent = (double*)calloc((size_t)m * dim, sizeof(double));
        for (int i = 0; i < m; ++i) {
            for (int64_t v = 0; v < subs[i].n; ++v)
                for (int t = 0; t < dim; ++t)
                    cent[i * dim + t] += (double)X[(subs[i].base + v) * dim + t];
            for (int t = 0; t < dim; ++t) cent[i * dim + t] /= (double)subs[i].n;
        }
    }
    int rmos = P->mos_degree;
    if (rmos <= 0) {
        rmos = (int)ceil(sqrt((double)m));
        if (rmos < 2) rmos = 2;
    }
    int nfb = 0;
    if (orc_plan(m, sizes, cent, dim, rmos, P->mos_diameter, out_ops, cap, &ne, &nfb) != 0) {
        free(subs); free(norms); free(cent);
        return -3;
    }
    *out_nops = ne;

    /* expansion, inversion and pivots, once per source sub-index, from its
     * input graph */
    int32_t** piv_of = (int32_t**)calloc((size_t)m, sizeof(int32_t*));
    int32_t** piv_ord = (int32_t**)calloc((size_t)m, sizeof(int32_t*));
    int64_t* npiv = (int64_t*)calloc((size_t)m, sizeof(int64_t));
    g_ndc_expand = g_ndc_naive = g_ndc_slide = 0;
    int rc = 0;
    for (int a = 0; a < ne && rc == 0; ++a) {
        int si = out_ops[2 * a];
        if (piv_of[si]) continue;
        const sub_t* s = &subs[si];
        int32_t* nk = (int32_t*)malloc(sizeof(int32_t) * (size_t)(s->n * P->k));
        int64_t* rko = (int64_t*)malloc(sizeof(int64_t) * (size_t)(s->n + 1));
        int32_t* rki = (int32_t*)malloc(sizeof(int32_t) * (size_t)(s->n * P->k + 1));
        piv_of[si] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(s->n > 0 ? s->n : 1));
        piv_ord[si] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(s->n > 0 ? s->n : 1));
        if (expand_neighbors(&S, s->n, s->offsets, s->nbrs, s->base, P->k, P->kplus, nk,
                             &g_ndc_expand, 0, s->n) != 0)
            rc = -4;
        orc_invert(s->n, nk, P->k, rko, rki);
        if (P->all_pivots) {
            for (int64_t v = 0; v < s->n; ++v) { piv_of[si][v] = -1; piv_ord[si][v] = (int32_t)v; }
            npiv[si] = s->n;
        } else {
            orc_pivots(s->n, rko, rki, piv_of[si], piv_ord[si], &npiv[si]);
        }
        if (trace && a == 0) {
            if (trace->nk) memcpy(trace->nk, nk, sizeof(int32_t) * (size_t)(s->n * P->k));
            if (trace->pivot_of) memcpy(trace->pivot_of, piv_of[si], sizeof(int32_t) * (size_t)s->n);
        }
        free(nk); free(rko); free(rki);
    }
    for (int a = 0; a < ne && rc == 0; ++a) {
        int si = out_ops[2 * a], ti = out_ops[2 * a + 1];
        int32_t* tri = (trace && a == 0) ? trace->res_ids : NULL;
        double* trd = (trace && a == 0) ? trace->res_d : NULL;
        if (pair_op(&S, &subs[si], &subs[ti], &rows, P, piv_of[si], piv_ord[si], npiv[si], tri,
                    trd) != 0)
            rc = -5;
    }
    /* merged entry: the entry of the largest sub-index (ties: lowest index) */
    int big = 0;
    for (int i = 1; i < m; ++i)
        if (sizes[i] > sizes[big]) big = i;
    *out_entry = (int32_t)(subs[big].base + subs[big].entry);
    if (trace) {
        trace->ndc_expand = g_ndc_expand;
        trace->ndc_naive = g_ndc_naive;
        trace->ndc_slide = g_ndc_slide;
        trace->n_pivots = ne > 0 ? npiv[out_ops[0]] : 0;
    }
    for (int i = 0; i < m; ++i) { free(piv_of[i]); free(piv_ord[i]); }
    free(piv_of); free(piv_ord); free(npiv);
    free(subs); free(norms); free(cent);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Sub-index builder (inputs) and exact k-NN                            */
/* ------------------------------------------------------------------ */

/* exact K nearest neighbours of every row of X (excluding itself) by
 * (d, id), brute force. out [n x K] local ids, -1 padded when n-1 < K */
int orc_knn(int64_t n, const float* X, int dim, int metric, int K, int32_t* out) {
    double* norms = NULL;
    if (metric == ORC_COSINE) {
        norms = (double*)malloc(sizeof(double) * (size_t)n);
        orc_norms(X, n, dim, norms);
    }
    space_t S = {X, dim, metric, norms};
#pragma omp parallel
    {
        wkey_t* c = (wkey_t*)malloc(sizeof(wkey_t) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t v = 0; v < n; ++v) {
            int nc = 0;
            for (int64_t u = 0; u < n; ++u) {
                if (u == v) continue;
                c[nc].id = (int32_t)u;
                c[nc].d = dist_ids(&S, v, u);
                ++nc;
            }
            qsort(c, (size_t)nc, sizeof(wkey_t), wkey_cmp);
            for (int j = 0; j < K; ++j) out[v * K + j] = j < nc ? c[j].id : -1;
        }
        free(c);
    }
    free(norms);
    return 0;
}

/* exact top-K of the rows of X for external queries Q, by (d, id) */
int orc_knn_queries(int64_t n, const float* X, int64_t nq, const float* Q, int dim, int metric,
                    int K, int32_t* out_ids, double* out_d) {
#pragma omp parallel
    {
    wkey_t* c = (wkey_t*)malloc(sizeof(wkey_t) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 4)
    for (int64_t i = 0; i < nq; ++i) {
        const float* q = Q + i * dim;
        double qn = 1.0;
        if (metric == ORC_COSINE) {
            double s = 0.0;
            for (int j = 0; j < dim; ++j) s += (double)q[j] * (double)q[j];
            qn = sqrt(s);
        }
        for (int64_t u = 0; u < n; ++u) {
            double un = 1.0;
            if (metric == ORC_COSINE) {
                double s = 0.0;
                for (int j = 0; j < dim; ++j) s += (double)X[u * dim + j] * (double)X[u * dim + j];
                un = sqrt(s);
            }
            c[u].id = (int32_t)u;
            c[u].d = orc_dist_vec(q, X + u * dim, dim, metric, qn, un);
        }
        qsort(c, (size_t)n, sizeof(wkey_t), wkey_cmp);
        for (int j = 0; j < K; ++j) {
            out_ids[i * K + j] = j < n ? c[j].id : -1;
            out_d[i * K + j] = j < n ? c[j].d : INFINITY;
        }
    }
    free(c);
    }
    return 0;
}

/*
 * Builder: row(v) = Prune(v, kNN(v), alpha, R). With reverse != 0, every
 * kept edge v -> w also offers v to w, and every w that received an offer is
 * pruned again over row(w) + offers, with alpha_rev. Entry: the vertex closest
 * to the centroid (exact integer criterion sum_j (n x_j - S_j)^2 when every
 * value is an integer, double precision otherwise), ties by id.
 * out_nbrs has room for n x R ids; out_offsets n+1.
 */
/* Everything reachable from `start` along the rows (up to R ids per row,
 * deg[v] used) that is not yet marked joins vis; returns how many joined. */
static int64_t reach_from(int64_t n, int R, const int32_t* rows, const int32_t* deg, int64_t start,
                          char* vis, int32_t* queue) {
    if (vis[start]) return 0;
    int64_t head = 0, tail = 0;
    vis[start] = 1;
    queue[tail++] = (int32_t)start;
    while (head < tail) {
        const int64_t v = queue[head++];
        for (int j = 0; j < deg[v]; ++j) {
            const int32_t w = rows[v * R + j];
            if (w >= 0 && w < n && !vis[w]) {
                vis[w] = 1;
                queue[tail++] = w;
            }
        }
    }
    return tail;
}

int64_t orc_reachable(int64_t n, const int64_t* offsets, const int32_t* nbrs, int32_t entry) {
    if (n <= 0 || entry < 0 || entry >= n) return 0;
    char* vis = (char*)calloc((size_t)n, 1);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int64_t head = 0, tail = 0;
    vis[entry] = 1;
    queue[tail++] = entry;
    while (head < tail) {
        const int64_t v = queue[head++];
        for (int64_t j = offsets[v]; j < offsets[v + 1]; ++j) {
            const int32_t w = nbrs[j];
            if (w >= 0 && w < n && !vis[w]) {
                vis[w] = 1;
                queue[tail++] = w;
            }
        }
    }
    free(vis);
    free(queue);
    return tail;
}

/* Reachability repair of a built graph, in passes. A pass takes the
 * vertices the entry reaches and the unreached rest. Its heads are the
 * unreached vertices that no unreached vertex links to; when there are none
 * (only cycles and what hangs off them are left), the unreached vertices
 * that no unreached vertex of smaller id links to (following links backwards
 * to ever smaller ids ends at one of them, so every unreached vertex hangs
 * off a head). Each
 * head proposes to the reached vertex nearest to it ((d, id) order) among
 * those with a free slot in their row, or, when no reached row has one, to
 * the nearest reached vertex. Each vertex with proposals accepts the nearest
 * ((d, head id) order), as many as its row has free slots, each appended; a
 * full row accepts one, which replaces its last entry (its farthest, rows
 * being in (d, id) order). Passes repeat until one starts with every vertex
 * reached (at most 4096). Returns the number of links added. */
typedef struct {
    int64_t t, u;
    double d;
} prop_t;

static int prop_cmp(const void* a, const void* b) {
    const prop_t* x = (const prop_t*)a;
    const prop_t* y = (const prop_t*)b;
    if (x->t != y->t) return x->t < y->t ? -1 : 1;
    if (key_less(x->d, x->u, y->d, y->u)) return -1;
    if (key_less(y->d, y->u, x->d, x->u)) return 1;
    return 0;
}

static int64_t repair_reach(const space_t* S, int64_t n, int R, int32_t* rows, int32_t* deg,
                            int32_t entry) {
    char* vis = (char*)malloc((size_t)n);
    char* inu = (char*)malloc((size_t)n);
    char* ins = (char*)malloc((size_t)n);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    prop_t* P = (prop_t*)malloc(sizeof(prop_t) * (size_t)n);
    int64_t links = 0;
    for (int pass = 0; pass < 4096; ++pass) {
        memset(vis, 0, (size_t)n);
        if (reach_from(n, R, rows, deg, entry, vis, queue) == n) break;
        /* unreached vertices some unreached vertex links to (inu), some
         * unreached vertex of smaller id (ins) */
        memset(inu, 0, (size_t)n);
        memset(ins, 0, (size_t)n);
        for (int64_t v = 0; v < n; ++v) {
            if (vis[v]) continue;
            for (int j = 0; j < deg[v]; ++j) {
                const int32_t w = rows[v * R + j];
                if (w >= 0 && w < n && !vis[w]) {
                    inu[w] = 1;
                    if (v < w) ins[w] = 1;
                }
            }
        }
        int64_t nheads = 0;
        for (int64_t u = 0; u < n; ++u)
            if (!vis[u] && !inu[u]) ++nheads;
        const char* excl = nheads > 0 ? inu : ins;
        int64_t np = 0;
        for (int64_t u = 0; u < n; ++u)
            if (!vis[u] && !excl[u]) P[np++].u = u;
        /* the targets a head may propose to: the reached vertices with a free
         * slot, or every reached vertex when none has one */
        int64_t nc = 0;
        for (int64_t v = 0; v < n; ++v)
            if (vis[v] && deg[v] < R) queue[nc++] = (int32_t)v;
        if (nc == 0)
            for (int64_t v = 0; v < n; ++v)
                if (vis[v]) queue[nc++] = (int32_t)v;
        /* each head's proposal on its own (threads over heads): the nearest
         * target */
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t h = 0; h < np; ++h) {
            const int64_t u = P[h].u;
            int64_t r = -1;
            double dr = 0.0;
            for (int64_t c = 0; c < nc; ++c) {
                const int64_t v = queue[c];
                const double d = dist_ids(S, u, v);
                if (r < 0 || key_less(d, v, dr, r)) {
                    r = v;
                    dr = d;
                }
            }
            P[h].t = r;
            P[h].d = dr;
        }
        qsort(P, (size_t)np, sizeof(prop_t), prop_cmp);
        for (int64_t i = 0; i < np;) {
            const int64_t t = P[i].t;
            int64_t e = i;
            while (e < np && P[e].t == t) ++e;
            const int64_t take = deg[t] < R ? R - deg[t] : 1;
            for (int64_t k = i; k < e && k - i < take; ++k) {
                if (deg[t] < R)
                    rows[t * R + deg[t]++] = (int32_t)P[k].u;
                else
                    rows[t * R + R - 1] = (int32_t)P[k].u;
                ++links;
            }
            i = e;
        }
    }
    free(vis);
    free(inu);
    free(ins);
    free(queue);
    free(P);
    return links;
}

int64_t orc_repair(int64_t n, const float* X, int dim, int metric, int R, int32_t* rows,
                   int32_t* deg, int32_t entry) {
    if (n <= 0 || entry < 0 || entry >= n) return 0;
    double* norms = NULL;
    if (metric == ORC_COSINE) {
        norms = (double*)malloc(sizeof(double) * (size_t)n);
        orc_norms(X, n, dim, norms);
    }
    space_t S = {X, dim, metric, norms};
    const int64_t links = repair_reach(&S, n, R, rows, deg, entry);
    free(norms);
    return links;
}

int orc_build(int64_t n, const float* X, int dim, int metric, const int32_t* knn, int K, int R,
              float alpha, int options, float alpha_rev, int64_t* out_offsets, int32_t* out_nbrs,
              int32_t* out_entry) {
    const int reverse = options & 1;
    double* norms = NULL;
    if (metric == ORC_COSINE) {
        norms = (double*)malloc(sizeof(double) * (size_t)n);
        orc_norms(X, n, dim, norms);
    }
    space_t S = {X, dim, metric, norms};
    int32_t* rows = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n * R + 1));
    double* rd = (double*)malloc(sizeof(double) * (size_t)(n * R + 1));
    int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    /* rows on their own (threads over vertices) */
#pragma omp parallel
    {
        int32_t* W = (int32_t*)malloc(sizeof(int32_t) * (size_t)(K + 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < n; ++v) {
            int nw = 0;
            for (int j = 0; j < K; ++j)
                if (knn[v * K + j] >= 0) W[nw++] = knn[v * K + j];
            deg[v] = prune(&S, v, W, nw, alpha, R, rows + v * R, rd + v * R);
        }
        free(W);
    }
    if (reverse) {
        int64_t* cnt = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
        for (int64_t v = 0; v < n; ++v)
            for (int j = 0; j < deg[v]; ++j) cnt[rows[v * R + j] + 1]++;
        for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
        int32_t* rev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cnt[n] + 1));
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        for (int64_t v = 0; v < n; ++v) fill[v] = cnt[v];
        for (int64_t v = 0; v < n; ++v)
            for (int j = 0; j < deg[v]; ++j) rev[fill[rows[v * R + j]]++] = (int32_t)v;
        int maxr = 0;
        for (int64_t v = 0; v < n; ++v)
            if (cnt[v + 1] - cnt[v] > maxr) maxr = (int)(cnt[v + 1] - cnt[v]);
        /* every offer is read from the rows of the first pass */
        int32_t* rows2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n * R + 1));
        int32_t* deg2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
#pragma omp parallel
        {
            int32_t* W2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(R + maxr + 1));
#pragma omp for schedule(dynamic, 64)
            for (int64_t w = 0; w < n; ++w) {
                if (cnt[w + 1] == cnt[w]) {
                    deg2[w] = deg[w];
                    memcpy(rows2 + w * R, rows + w * R, sizeof(int32_t) * (size_t)deg[w]);
                    continue;
                }
                int nw = 0;
                for (int j = 0; j < deg[w]; ++j) W2[nw++] = rows[w * R + j];
                for (int64_t j = cnt[w]; j < cnt[w + 1]; ++j) W2[nw++] = rev[j];
                deg2[w] = prune(&S, w, W2, nw, alpha_rev, R, rows2 + w * R, rd + w * R);
            }
            free(W2);
        }
        memcpy(rows, rows2, sizeof(int32_t) * (size_t)(n * R));
        memcpy(deg, deg2, sizeof(int32_t) * (size_t)n);
        free(rows2); free(deg2); free(rev); free(fill); free(cnt);
    }
    /* entry */
    int integral = 1;
    for (int64_t i = 0; i < n * dim && integral; ++i)
        if (X[i] != floor(X[i]) || fabs(X[i]) > 1e6) integral = 0;
    int64_t best = 0;
    if (integral) {
        int64_t* Ssum = (int64_t*)calloc((size_t)dim, sizeof(int64_t));
        for (int64_t v = 0; v < n; ++v)
            for (int j = 0; j < dim; ++j) Ssum[j] += (int64_t)X[v * dim + j];
        __int128 bestc = 0;
        for (int64_t v = 0; v < n; ++v) {
            __int128 c = 0;
            for (int j = 0; j < dim; ++j) {
                __int128 t = (__int128)n * (int64_t)X[v * dim + j] - Ssum[j];
                c += t * t;
            }
            if (v == 0 || c < bestc) { bestc = c; best = v; }
        }
        free(Ssum);
    } else {
        double* mean = (double*)calloc((size_t)dim, sizeof(double));
        for (int64_t v = 0; v < n; ++v)
            for (int j = 0; j < dim; ++j) mean[j] += (double)X[v * dim + j];
        for (int j = 0; j < dim; ++j) mean[j] /= (double)n;
        double bestc = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            double c = 0.0;
            for (int j = 0; j < dim; ++j) {
                double t = (double)X[v * dim + j] - mean[j];
                c += t * t;
            }
            if (v == 0 || c < bestc) { bestc = c; best = v; }
        }
        free(mean);
    }
    *out_entry = (int32_t)best;
    int64_t links = 0;
    if (options & 2) links = repair_reach(&S, n, R, rows, deg, (int32_t)best);
    out_offsets[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        out_offsets[v + 1] = out_offsets[v] + deg[v];
        memcpy(out_nbrs + out_offsets[v], rows + v * R, sizeof(int32_t) * (size_t)deg[v]);
    }
    free(rows); free(rd); free(deg); free(norms);
    return (int)links;
}
