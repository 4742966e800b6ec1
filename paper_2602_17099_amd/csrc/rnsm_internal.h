// Internal interface between the host orchestration (rnsm_api.cpp) and the
// device kernels (rnsm_kernels.hip). Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rnsm {

typedef unsigned long long u64;

// counters the search kernel accumulates (one atomic per wavefront)
enum { CNT_NDC = 0, CNT_EXP = 1, CNT_ADJ = 2, CNT_HFULL = 3, CNT_N = 4 };
// copies of the counters, summed on the host: CNT_SLOTS * CNT_N entries per launch
enum { CNT_SLOTS = 64 };

struct SearchArgs {
    const char* base;         // target rows, search storage type, row r at base + r*row_bytes
    int nch;                  // 16-byte chunks per row
    int row_bytes;
    const int64_t* offs;      // target CSR
    const int32_t* nbrs;
    const int32_t* padj;      // optional padded adjacency [n x rp], -1 filled (replaces offs/nbrs)
    int rp;
    int64_t n;                // target size
    const char* qvec;         // query rows (same storage type), row u at qvec + u*row_bytes
    const int32_t* qidx;      // query i uses row qidx[i] (NULL: row i)
    int64_t nq;
    int seed_mode;            // 0: entry, 1: the query's own row id, 2: seed rows
    int32_t entry;
    const int32_t* seed_ids;  // mode 2: row seed_row[i] (NULL: row i) of seed_stride ids, n_seeds used
    int64_t seed_stride;
    const int32_t* seed_row;
    int n_seeds;
    int metric;
    const float* base_norm;   // cosine: norms of target rows
    const float* q_norm;      // cosine: norms of query rows (indexed like the query row)
    int ef;
    int G;                    // lanes per row (power of two)
    int lgG;                  // log2(G)
    int cpl;                  // 16-byte chunks per lane (nch = G * cpl)
    int hbits;                // log2 of the LDS visited-table words (32-bit) per wavefront
    int hash_mode;            // 0: two-way sets of 16-bit tags (forgetful), 1: linear probing
    int out_mode;             // 0: first out_k of the beam, 1: first out_k excluding the query's own id
    int32_t* out_ids;
    float* out_d;
    int64_t out_stride;
    int out_k;
    const int32_t* out_row;   // output row of query i (NULL: i)
    u64* counters;            // CNT_SLOTS x CNT_N entries
    int* err;
    float* row_d;             // optional (seed mode 1): the distances of the query's own
                              // neighbours, from its first expansion, go to
                              // row_d[(row_d_base + u) * row_d_stride + slot]
    int64_t row_d_base;
    int row_d_stride;
};

// One operation of a round in the persistent pivot-group search: its naive
// and sliding search arguments (target graph and rows, beams, outputs; the
// sliding seeds are row p of slide.seed_ids for the group of pivot p), and its
// groups g: pivot gpiv[g], followers fol[fbeg[g] .. fbeg[g+1]) (source-local
// ids). Groups of all operations are numbered from group_base on.
struct GroupOp {
    SearchArgs naive, slide;
    const int32_t* gpiv;
    const int64_t* fbeg;
    const int32_t* fol;
    int64_t group_base, n_groups;
};

struct GroupArgs {
    const GroupOp* ops;   // device array, ascending group_base
    int n_ops;
    int64_t n_groups;     // all operations together
    unsigned* next;       // 8 range counters, zero at launch
    int hbits;            // LDS visited table of every search
    int64_t fmax;         // followers searched in a group's work item (the rest: overflow)
    u64* counters;        // CNT_SLOTS x CNT_N for the pivots, then as many for the followers
};

struct PruneArgs {
    int grid_cap;             // row distances: at most this many blocks (0: one wave a vertex)
    const float* X;           // float32 rows of every vertex (global ids)
    const char* xb;           // bfloat16 copy of X (dim * 2 bytes a row): the MFMA prune in
                              // exact mode (rows exact in bfloat16) reads this one
    int G16, lgG16;           // lanes per row of the copy in the candidate distances
    int64_t n_total;          // number of rows of X (ids >= n_total are rejected)
    int nch;
    int G;                    // lanes per row (power of two)
    int lgG;
    int cpl;                  // 16-byte chunks per lane (nch = G * cpl)
    int metric;
    const float* norms;
    int64_t n_items;
    const int32_t* items;     // item i -> vertex item_base + items[i] (NULL: item_base + i)
    int64_t item_base;
    const int32_t* rows_in;   // [* x R] current rows, indexed by vertex (NULL: empty rows)
    const int32_t* deg_in;
    const float* rows_d;      // their float32 distances (NaN: not known), or NULL
    int extra_mode;           // 0: none, 1: fixed stride, 2: CSR
    const int32_t* extra_ids;
    const float* extra_d;     // float32 distances d(p, extra) in the extra layout, or NULL
    int64_t extra_stride;
    int extra_cnt;
    const int64_t* extra_off;
    int64_t extra_index_base; // extra row of vertex p is p - extra_index_base
    int64_t extra_id_add;     // added to every extra id (-1 entries skipped)
    int skip_empty_extra;     // leave rows without extra candidates untouched
    int extra_sorted;         // mode 1 with extra_d: each extra row is in ascending
                              // (d, id) order, -1 ids last (a search's final beam)
    float alpha;
    // the removal rule (float32 walk only): 0 alpha; 1 angle (SSG), rule_a =
    // cos(theta); 2 tau-MNG, rule_a = 3 tau; 1 and 2 on squared L2
    int rule;
    double rule_a;
    int R;
    int32_t* rows_out;
    int32_t* deg_out;
    float* dist_out;
    int32_t* rev_cnt;         // optional: +1 at rev_cnt[v - rev_lo] for every kept v in
    int64_t rev_lo, rev_n;    // [rev_lo, rev_lo + rev_n) (reverse-edge counts)
    u64* scratch;             // keys of candidate lists longer than wcap (mode 2)
    int wcap;
    int* err;
    // MFMA prune of float rows (hi/lo split): a pair whose estimate lies
    // within band * scale of the alpha boundary is decided again with the
    // float32 walk's own arithmetic (0: no re-decision); rechecks counts them
    double band;
    u64* rechecks;
    // which vertices this launch prunes, by candidate count: 0 all, 1 those
    // with at most LONG_LIST candidates, 2 the others (the float32 walk takes
    // those, 16 at a time in key order, with no full sort)
    int list_filter;
};
constexpr int LONG_LIST = 1024;

// launchers (all asynchronous on `st`)
hipError_t launch_validate(const int64_t* offs, const int32_t* nbrs, int64_t n, int64_t nnz,
                           int R, int* flags, hipStream_t st);
hipError_t launch_pad_adjacency(const int64_t* offs, const int32_t* nbrs, int64_t n, int rp,
                                int32_t* out, hipStream_t st);
hipError_t launch_init_rows(const int64_t* offs, const int32_t* nbrs, int64_t n, int64_t base,
                            int R, int32_t* rows, int32_t* deg, float* rdist, hipStream_t st);
// row norms summed in double; out64 (optional) keeps the double values
hipError_t launch_norms(const float* X, int64_t n, int dim, float* out, hipStream_t st,
                        double* out64 = nullptr);
hipError_t launch_search(int tt, const SearchArgs& a, int waves_per_block, hipStream_t st);
// row norms of 16-bit rows (tt 1: bfloat16, 2: float16), summed in double
hipError_t launch_norms16(const void* X, int tt, int64_t n, int dim, float* out, hipStream_t st);
// zero bytes (a multiple of 4) at p with a kernel (no memset node in a captured graph)
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
// the persistent pivot-group search of a round (every op with the same
// search shape as `shape`: storage type tt, chunks per lane, lanes per row,
// table mode, beam class)
// blocks_out (may be NULL): the grid launched
hipError_t launch_group_search(int tt, const SearchArgs& shape, const GroupArgs& g, int wpb,
                               hipStream_t st, int64_t* blocks_out = nullptr);
// pivot groups of one source from pivot_of (-1 pivots), pivots taken along
// `order` (NULL: id order): gpiv[n_groups], fbeg[n_groups + 1] (offsets into
// fol), fol (followers by group), prune_order (each pivot then its
// followers); flag, gpos (n + 1), group_of, cnt: scratch
hipError_t launch_groups(const int32_t* order, int64_t n, const int32_t* pivot_of, int32_t* flag,
                         int64_t* gpos, int32_t* gpiv, int32_t* group_of, int32_t* cnt,
                         int64_t* fbeg, int32_t* fol, int32_t* prune_order, int64_t* scan_tmp,
                         int64_t n_groups, hipStream_t st);
// followers past the first fmax of their group (the overflow, searched by a
// plain launch after the group search): cnt[g] = excess of group g (scratch,
// n_groups), ooff (n_groups + 1) its scan, ofl / oflp the overflow followers
// and their pivots, group by group; nf followers in all
hipError_t launch_group_overflow(int64_t n_groups, int64_t nf, const int32_t* gpiv,
                                 const int64_t* fbeg, const int32_t* fol, const int32_t* pivot_of,
                                 const int32_t* group_of, int64_t fmax, int32_t* cnt, int64_t* ooff,
                                 int32_t* ofl, int32_t* oflp, int64_t* scan_tmp, hipStream_t st);
hipError_t launch_fill32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
// pivot selection on the device (the lazy greedy in parallel rounds, the same
// pivots and groups): init, then rounds (each a no-op once ctl[0] is 0: a
// round picked nothing); ctl[1] counts pivots, ctl[2] rounds with picks.
// pivot_of: -1 pivot, else the pivot's id
hipError_t launch_check_lists(int64_t n, const int64_t* off, const int32_t* ids, int* flag,
                              hipStream_t st);
hipError_t launch_select_init(int64_t n, const int64_t* off, unsigned char* lose, int32_t* gain,
                              int32_t* pivot_of, int64_t* ctl, hipStream_t st);
// forward lists F(y) = {x : y in R_k(x)} of CSR reverse lists (off, ids):
// cnt, cur n words of scratch, f_off n + 1, f_ids off[n]
// flag (device int) set unless order[0, n) is a permutation of 0..n-1 (cnt:
// n words of scratch)
hipError_t launch_perm_check(const int32_t* order, int64_t n, int32_t* cnt, int* flag,
                             hipStream_t st);
hipError_t launch_select_forward(int64_t n, const int64_t* off, const int32_t* ids, int32_t* cnt,
                                 int32_t* cur, int64_t* f_off, int32_t* f_ids, int64_t* scan_tmp,
                                 hipStream_t st);
// `rounds` rounds over the active vertices act[0, nact) (NULL: all n), the
// reverse lists (off, ids) and the forward lists (f_ids with CSR offsets
// f_off, or f_off NULL: fixed stride fk, -1 padded); items: a round's chunk
// items, at least n + off[n] / 16 + 1 entries
hipError_t launch_select_rounds(int64_t n, const int32_t* act, int64_t nact, const int64_t* off,
                                const int32_t* ids, const int32_t* f_ids, const int64_t* f_off,
                                int fk, unsigned char* lose, int32_t* gain, int32_t* pivot_of,
                                int64_t* items, int64_t* ctl, int rounds, hipStream_t st);
// the remaining rounds over act[0, nact) in one workgroup (few vertices left)
hipError_t launch_select_tail(int64_t n, const int32_t* act, int64_t nact, const int64_t* off,
                              const int32_t* ids, const int32_t* f_ids, const int64_t* f_off,
                              int fk, unsigned char* lose, int32_t* gain, int32_t* pivot_of,
                              int64_t* items, int64_t* ctl, hipStream_t st);
constexpr int64_t SELECT_TAIL_MAX = 8192;  // active vertices for the one-workgroup tail
// the still uncovered active vertices into act_out, their count into ctl[4]
hipError_t launch_select_compact(const int32_t* act, int64_t nact, const int32_t* gain,
                                 int32_t* act_out, int64_t* ctl, hipStream_t st);
// static device scratch of the allocation-free search (bytes per device) and
// its address on the current device (looked up once per device)
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;
hipError_t noalloc_scratch(void** out);
size_t search_lds_bytes(int hbits, int waves_per_block);
hipError_t launch_prune(const PruneArgs& a, hipStream_t st);
// the same rule with the Gram products on bfloat16 MFMA (dims 32, 64, 96,
// 128; R <= 64): nt = 1 for rows exact in bfloat16 with exact float32 sums,
// nt = 3 (hi/lo split) otherwise
bool prune_mfma_supported(int dim);
// default relative band of the float re-decision (2^-10)
constexpr double PRUNE_BAND = 1.0 / 1024.0;
bool prune_mfma_fits(const PruneArgs& a, int nt);  // dimension, R and LDS size
// missing distances of the rows of a prune's vertices, as that prune would
// compute them (b16: the MFMA prune in exact mode, reading the bfloat16 copy)
hipError_t launch_row_dists(const PruneArgs& a, bool b16, hipStream_t st);
hipError_t launch_prune_mfma(const PruneArgs& a, int nt, hipStream_t st);
// out[0] = 1 if every value is an integer, out[1] / out[2] = order-preserving
// bits of min / max (key_to_float gives the value back)
hipError_t launch_value_range(const float* X, int64_t total, unsigned* out, hipStream_t st);
float key_to_float(unsigned k);
// src_type 0: float32, 3: uint8; dst_type 0: float32, 1: bfloat16, 2: float16
hipError_t launch_convert(const void* src, int src_type, void* dst, int dst_type, int64_t count,
                          hipStream_t st);
hipError_t launch_scan(const int32_t* cnt, int64_t n, int64_t* off, int64_t* tmp_blocks,
                       hipStream_t st);
size_t scan_tmp_elems(int64_t n);
// lazy-greedy gain levels from list lengths (lcap levels of (n + 63) / 64
// words, lists of lcap or more as (length, id) in high[0, min(ctl[0], cap)))
hipError_t launch_gain_levels(const int32_t* cnt, int64_t n, int lcap, unsigned long long* bits,
                              int* ctl, int2* high, int64_t cap, hipStream_t st);
// reverse k-NN inversion (R_k) in two halves: list lengths into cnt, then
// offsets and ids (cnt is overwritten)
hipError_t launch_count_ids(const int32_t* nk, int64_t n, int k, int32_t* cnt, hipStream_t st);
hipError_t launch_invert_lists(const int32_t* nk, int64_t n, int k, int32_t* cnt,
                               int64_t* rk_off, int32_t* rk_ids, int64_t* scan_tmp,
                               hipStream_t st);
hipError_t launch_rev_count(const int32_t* rows, const int32_t* deg, int64_t s_base, int64_t n_s,
                            int R, int64_t t_base, int64_t n_t, int32_t* cnt, hipStream_t st);
hipError_t launch_rev_scatter(const int32_t* rows, const int32_t* deg, const float* rdist,
                              int64_t s_base, int64_t n_s, int R, int64_t t_base, int64_t n_t,
                              const int64_t* off, int32_t* cur, int32_t* rev, float* rev_d,
                              hipStream_t st);
// CSR output; for inner product and cosine (norms64 required then) every
// stored distance is recomputed with float64 sums
hipError_t launch_compact(const int32_t* rows, const int32_t* deg, const float* rdist,
                          const int64_t* off, int64_t N, int R, const float* X, int dim,
                          int metric, const float* norms, int32_t* out_nbrs, float* out_dists,
                          hipStream_t st, const double* norms64 = nullptr);
hipError_t launch_copy_rows(const int32_t* rows_a, const int32_t* deg_a, const float* dist_a,
                            const int32_t* cnt, int64_t n, int R, int32_t* rows_b,
                            int32_t* deg_b, float* dist_b, hipStream_t st);
hipError_t launch_entry(const float* X, int64_t n, int dim, int* flag, double* colsum_d,
                        unsigned long long* colsum_i, u64* block_best, int64_t nblocks,
                        hipStream_t st);
int64_t entry_blocks(int64_t n);
// breadth-first vertex order of a padded-adjacency graph from root (a
// processing order only); vis: (n + 31) / 32 words of scratch, ctl: 4 device
// words (order tail, frontier start and end, finished blocks), h_ctl: 4
// pinned host words; synchronises st once per batch of BFS_BATCH levels
#define BFS_BATCH 8
hipError_t launch_bfs_order(const int32_t* padj, int rp, int64_t n, int32_t root, unsigned* vis,
                            int32_t* order, unsigned* ctl, unsigned* h_ctl, hipStream_t st);
// the same in steps: init from root; grow (levels until the frontier is
// empty; h_ctl[0] = vertices reached, order[0, h_ctl[0]) the reached ones)
hipError_t launch_bfs_init(int64_t n, int32_t root, unsigned* vis, int32_t* order, unsigned* ctl,
                           hipStream_t st);
hipError_t launch_bfs_grow(const int32_t* padj, int rp, int64_t n, int32_t* order, unsigned* vis,
                           unsigned* ctl, unsigned* h_ctl, hipStream_t st);
// one pass of the builder's reachability repair over rows of R ids (-1
// padded) and the reached bits `vis` of a search from the entry. heads:
// clears inu (n bytes), cnt and cur (n words each), marks unreached vertices
// an unreached vertex links to, and counts the heads (ctl[0]) and the
// smallest unreached id (ctl[1]); propose: each head (only = 0: no
// unreached vertex links to it; 1: none of smaller id does) proposes
// (target pt[u], key pk[u]) from its k-NN list (knn [n x K],
// exact, sorted by (d, id)) or is listed in fb (ctl[2] of them) for scan;
// cands + scan: the global scan of the listed heads over the reached
// vertices with a free slot (every reached vertex when none has one), 16
// heads a block (dim <= 1024); accept: proposals grouped by target (cnt,
// off: n + 1, seg: n keys), each target taking its nearest ones (as many as
// its free slots, appended; one over a full row's last entry), links
// counted into *links
hipError_t launch_repair_heads(int64_t n, const int32_t* rows, const int32_t* deg, int R,
                               const unsigned* vis, unsigned char* inu, int32_t* cnt, int32_t* cur,
                               unsigned long long* ctl, hipStream_t st);
hipError_t launch_repair_propose(int64_t n, const float* X, int dim, int metric, const float* norms,
                                 const int32_t* knn, int K, const unsigned* vis,
                                 const unsigned char* inu, const int32_t* deg, int R, int64_t only,
                                 int32_t* pt, unsigned long long* pk, int32_t* fb,
                                 unsigned long long* ctl, hipStream_t st);
hipError_t launch_repair_cands(int64_t n, const unsigned* vis, const int32_t* deg, int R,
                               int all_reached, int32_t* cand, unsigned long long* cnt,
                               hipStream_t st);
hipError_t launch_repair_scan(int64_t n, const float* X, int dim, int metric, const float* norms,
                              const int32_t* fb, int64_t nfb, const int32_t* cand, int64_t ncand,
                              int32_t* pt, unsigned long long* pk, hipStream_t st);
hipError_t launch_repair_accept(int64_t n, const unsigned* vis, const unsigned char* inu,
                                int64_t only, const int32_t* pt, const unsigned long long* pk,
                                int32_t* cnt, int32_t* cur, int64_t* off, int64_t* scan_tmp,
                                unsigned long long* seg, int32_t* rows, int32_t* deg, int R,
                                unsigned long long* links, hipStream_t st);
hipError_t launch_pad_tail(int32_t* rows, const int32_t* deg, int64_t n, int R, hipStream_t st);
// largest row length (atomicMax into *maxdeg, zeroed by the caller) and a
// flag for malformed offsets
hipError_t launch_csr_shape(const int64_t* offs, int64_t n, unsigned* maxdeg, int* bad,
                            hipStream_t st);

// lanes per row for rows of nch 16-byte chunks: the smallest power of two G
// with 4*G >= nch that divides nch, so that every lane holds nch/G <= 4 whole
// chunks; -1 when there is none
inline int lanes_per_row(int nch) {
    for (int g = 1; g <= 64; g <<= 1)
        if (4 * g >= nch && nch % g == 0) return g;
    return -1;
}
inline int ilog2i(int g) {
    int b = 0;
    while ((1 << b) < g) ++b;
    return b;
}

}  // namespace rnsm
