// Host-side planning of the RNSM path: merge order selection (Algorithm 3,
// Section 5) with the execution order and direction rules of Section 5, and
// the lazy greedy pivot selection of Algorithm 2 (Section 4.2).
#include "rnsm_plan.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace rnsm {

// ---------------------------------------------------------------- MOS

namespace {

// hop counts from v in the undirected graph adj (INT32_MAX: unreachable)
void bfs_from(int v, const std::vector<std::vector<int>>& adj, std::vector<int>& hop) {
    const int m = (int)adj.size();
    hop.assign(m, INT32_MAX);
    std::vector<int> q;
    q.reserve(m);
    hop[v] = 0;
    q.push_back(v);
    for (size_t h = 0; h < q.size(); ++h) {
        const int u = q[h];
        for (int w : adj[u])
            if (hop[w] == INT32_MAX) {
                hop[w] = hop[u] + 1;
                q.push_back(w);
            }
    }
}

bool has_edge(const std::vector<std::vector<int>>& adj, int a, int b) {
    return std::find(adj[a].begin(), adj[a].end(), b) != adj[a].end();
}

}  // namespace

int mos_edges(int m, const std::vector<double>& cost, int R, int delta,
              std::vector<std::pair<int, int>>& edges, int* fallbacks) {
    edges.clear();
    *fallbacks = 0;
    if (m < 1 || R < 1 || delta < 2 || (int)cost.size() != m * m) return -1;
    auto C = [&](int a, int b) { return cost[(size_t)a * m + b]; };
    // vertices by ascending mean cost to their min(R, m-1) cheapest others
    const int r = std::min(R, m - 1);
    std::vector<double> mean(m, 0.0);
    for (int i = 0; i < m; ++i) {
        std::vector<double> c;
        c.reserve(m);
        for (int j = 0; j < m; ++j)
            if (j != i) c.push_back(C(i, j));
        std::partial_sort(c.begin(), c.begin() + r, c.end());
        double s = 0.0;
        for (int t = 0; t < r; ++t) s += c[t];
        mean[i] = r > 0 ? s / r : 0.0;
    }
    std::vector<int> order(m);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return mean[a] < mean[b]; });

    std::vector<std::vector<int>> adj(m);
    std::vector<int> hop;
    auto deg = [&](int a) { return (int)adj[a].size(); };
    for (int v : order) {
        for (;;) {
            bfs_from(v, adj, hop);
            int x = -1;
            for (int c = 0; c < m; ++c) {
                if (c == v || hop[c] <= delta) continue;
                if (x < 0 || C(v, c) < C(v, x)) x = c;
            }
            if (x < 0) break;
            int a = v, b = x;
            bool fb = false;
            const bool vs = deg(v) >= R, xs = deg(x) >= R;
            if (!vs && xs) {
                // relay to the cheapest unsaturated neighbour of x
                int best = -1;
                for (int c : adj[x])
                    if (c != v && deg(c) < R &&
                        (best < 0 || C(c, v) < C(best, v) || (C(c, v) == C(best, v) && c < best)))
                        best = c;
                if (best >= 0) b = best; else fb = true;
            } else if (vs && !xs) {
                int best = -1;
                for (int c : adj[v])
                    if (c != x && deg(c) < R &&
                        (best < 0 || C(c, x) < C(best, x) || (C(c, x) == C(best, x) && c < best)))
                        best = c;
                if (best >= 0) a = best; else fb = true;
            } else if (vs && xs) {
                fb = true;
            }
            if (has_edge(adj, a, b)) return -2;  // cannot happen for delta >= 2
            adj[a].push_back(b);
            adj[b].push_back(a);
            edges.emplace_back(a, b);
            if (fb) ++*fallbacks;
        }
    }
    return 0;
}

int plan_ops(int m, const int64_t* sizes, const double* centroids, int dim, int R, int delta,
             std::vector<std::pair<int, int>>& ops, int* fallbacks) {
    std::vector<double> cost((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            if (i == j) continue;
            if (!centroids) {
                cost[(size_t)i * m + j] = 1.0;
                continue;
            }
            double s = 0.0;
            for (int t = 0; t < dim; ++t) {
                const double d = centroids[(size_t)i * dim + t] - centroids[(size_t)j * dim + t];
                s += d * d;
            }
            cost[(size_t)i * m + j] = std::sqrt(s);
        }
    std::vector<std::pair<int, int>> e;
    const int rc = mos_edges(m, cost, R, delta, e, fallbacks);
    if (rc != 0) return rc;
    for (auto& p : e)
        if (p.first > p.second) std::swap(p.first, p.second);
    std::stable_sort(e.begin(), e.end(), [&](const std::pair<int, int>& a,
                                             const std::pair<int, int>& b) {
        const double ca = cost[(size_t)a.first * m + a.second];
        const double cb = cost[(size_t)b.first * m + b.second];
        if (ca != cb) return ca < cb;
        return a < b;
    });
    ops.clear();
    for (auto& p : e) {
        const int i = p.first, j = p.second;  // i < j
        if (sizes[j] < sizes[i])
            ops.emplace_back(j, i);
        else
            ops.emplace_back(i, j);
    }
    return 0;
}

// ------------------------------------------------------ lazy greedy pivots

void build_levels(int64_t n, const int32_t* counts, GainLevels& L) {
    L.n = n;
    L.words = (n + 63) / 64;
    int32_t gmax = 0;
    for (int64_t x = 0; x < n; ++x) gmax = std::max(gmax, counts[x]);
    L.nlev = std::min(gmax + 1, GainLevels::LCAP);
    L.ext = nullptr;
    if ((int64_t)L.bits.size() < (int64_t)L.nlev * L.words) L.bits.resize((size_t)L.nlev * L.words);
    L.high.clear();
    // one word of every level at a time: the 64 vertices' bits meet in a
    // small array, then each level's word is stored
    uint64_t loc[GainLevels::LCAP];
    for (int l = 0; l < L.nlev; ++l) loc[l] = 0ull;
    for (int64_t w = 0; w < L.words; ++w) {
        const int64_t x0 = w * 64, x1 = std::min<int64_t>(n, x0 + 64);
        for (int64_t x = x0; x < x1; ++x) {
            const int32_t g = counts[x];
            if (g < GainLevels::LCAP)
                loc[g] |= 1ull << (x - x0);
            else
                L.high.emplace_back((int64_t)g, (int32_t)x);
        }
        for (int l = 0; l < L.nlev; ++l) {
            L.bits[(size_t)l * L.words + w] = loc[l];
            loc[l] = 0ull;
        }
    }
}

// The lazy greedy of Algorithm 2: repeatedly take the vertex with the largest
// stored gain (ties: smallest id); drop it if covered; if its gain
// |R_k(x) minus Covered| fell below the stored one, store it under the new
// gain; otherwise make it a pivot whose followers are its uncovered R_k.
// A vertex is only ever moved to a lower gain while a higher one is
// processed, so every gain level is a bitmap over vertex ids scanned once in
// ascending order (gains of LCAP and more: a heap with the same order);
// Covered is a bitmap too, so covered vertices of a level are dropped 64 at
// a time.
void select_pivots(GainLevels& L, const int64_t* rk_off, const int32_t* rk_ids, int32_t* pivots,
                   int32_t* followers, int32_t* follower_pivot, int64_t chunk, int64_t chunk_max,
                   const Emit& emit, const std::function<void()>& lists_ready) {
    if (lists_ready) lists_ready();
    const int64_t n = L.n, words = L.words;
    uint64_t* lv = L.data();
    std::vector<uint64_t> cov((size_t)words, 0ull);
    int64_t np = 0, nf = 0, sent = 0;
    chunk = std::max<int64_t>(chunk, 1);
    auto mark = [&](int64_t g, int64_t x) {
        if (g < GainLevels::LCAP) {
            lv[(size_t)g * words + (x >> 6)] |= 1ull << (x & 63);
        } else {
            L.high.emplace_back(g, (int32_t)x);
            std::push_heap(L.high.begin(), L.high.end(), [](const std::pair<int64_t, int32_t>& a,
                                                            const std::pair<int64_t, int32_t>& b) {
                return a.first < b.first || (a.first == b.first && a.second > b.second);
            });
        }
    };
    // take x at stored gain g: 0 dropped (covered), 1 moved down, 2 pivot
    auto visit = [&](int32_t x, int64_t g) {
        const int64_t o0 = rk_off[x], o1 = rk_off[x + 1];
        // one pass counts the uncovered members and, for lists of up to BUF,
        // keeps them for the pivot case (the lists hold no repeated id)
        constexpr int64_t BUF = 64;
        int32_t unc[BUF];
        int64_t cur = 0;
        const bool fits = o1 - o0 <= BUF;
        for (int64_t j = o0; j < o1; ++j) {
            const int32_t y = rk_ids[j];
            const int64_t u = (int64_t)(~cov[y >> 6] >> (y & 63) & 1ull);
            if (fits) unc[cur] = y;
            cur += u;
        }
        if (cur < g) {
            mark(cur, x);
            return;
        }
        pivots[np++] = x;
        cov[x >> 6] |= 1ull << (x & 63);
        if (fits) {
            for (int64_t t = 0; t < cur; ++t) {
                const int32_t y = unc[t];
                cov[y >> 6] |= 1ull << (y & 63);
                followers[nf] = y;
                follower_pivot[nf++] = x;
            }
        } else {
            for (int64_t j = o0; j < o1; ++j) {
                const int32_t y = rk_ids[j];
                const uint64_t bit = 1ull << (y & 63);
                if (!(cov[y >> 6] & bit)) {
                    cov[y >> 6] |= bit;
                    followers[nf] = y;
                    follower_pivot[nf++] = x;
                }
            }
        }
        if (np + nf - sent >= chunk) {
            emit(np, nf);
            sent = np + nf;
            chunk = std::max(chunk, std::min(2 * chunk, chunk_max));
        }
    };
    // gains of LCAP and more first, largest gain then smallest id
    auto hcmp = [](const std::pair<int64_t, int32_t>& a, const std::pair<int64_t, int32_t>& b) {
        return a.first < b.first || (a.first == b.first && a.second > b.second);
    };
    std::make_heap(L.high.begin(), L.high.end(), hcmp);
    while (!L.high.empty()) {
        std::pop_heap(L.high.begin(), L.high.end(), hcmp);
        const auto e = L.high.back();
        L.high.pop_back();
        if (!((cov[e.second >> 6] >> (e.second & 63)) & 1ull)) visit(e.second, e.first);
    }
    // A level is scanned in id order, but the lists of its vertices lie all
    // over the offsets and ids, so each visit would wait on memory: the
    // offsets of the vertices a few bitmap words ahead, and then their ids,
    // are fetched early.
    constexpr int64_t PF_OFF = 16, PF_IDS = 8;  // bitmap words ahead
    auto prefetch_word = [&](const uint64_t* b, int64_t w, bool ids) {
        uint64_t m = b[w] & ~cov[w];
        while (m) {
            const int64_t x = w * 64 + __builtin_ctzll(m);
            m &= m - 1;
            if (ids)
                __builtin_prefetch(rk_ids + rk_off[x]);
            else
                __builtin_prefetch(rk_off + x);
        }
    };
    for (int64_t g = L.nlev - 1; g >= 1; --g) {
        uint64_t* b = lv + (size_t)g * words;
        for (int64_t w = 0; w < words; ++w) {
            if (w + PF_OFF < words) prefetch_word(b, w + PF_OFF, false);
            if (w + PF_IDS < words) prefetch_word(b, w + PF_IDS, true);
            uint64_t bits = b[w] & ~cov[w];
            while (bits) {
                const int32_t x = (int32_t)(w * 64 + __builtin_ctzll(bits));
                bits &= bits - 1;
                visit(x, g);
                bits &= ~cov[w];
            }
        }
    }
    // Gain 0 last: a gain never rises, so every vertex still uncovered here
    // is a pivot whose reverse list is all covered (no followers, nothing
    // newly covered), taken in ascending id order without reading its list.
    for (int64_t w = 0; L.nlev > 0 && w < words; ++w) {
        uint64_t bits = lv[w] & ~cov[w];
        while (bits) {
            pivots[np++] = (int32_t)(w * 64 + __builtin_ctzll(bits));
            bits &= bits - 1;
            if (np + nf - sent >= chunk) {
                emit(np, nf);
                sent = np + nf;
                chunk = std::max(chunk, std::min(2 * chunk, chunk_max));
            }
        }
    }
    if (np + nf > sent || sent == 0) emit(np, nf);
    (void)n;
}

}  // namespace rnsm
