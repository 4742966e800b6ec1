/*
 * librnsm: Reverse Neighbor Sliding Merge (RNSM) of proximity-graph indexes
 * on AMD Instinct MI355X (gfx950), after arXiv 2602.17099.
 *
 * The method (Section 4, Algorithm 2): every vertex of the smaller
 * sub-index (the source) finds neighbours in the larger one (the target) by
 * greedy beam search (Algorithm 1). Pivot vertices, picked by a lazy greedy
 * over reverse k-NN lists, start from the target's entry point ("naive
 * search"); their followers start from the pivot's results ("local
 * sliding"). Each source vertex's results are concatenated with its current
 * out-neighbours and pruned by the RNG/alpha edge-selection rule to out-degree
 * R; the kept cross edges are offered back to the target vertices as reverse
 * edges, and every target that received some is pruned again. With more than
 * two sub-indexes, Merge Order Selection (Section 5, Algorithm 3) picks which
 * pairs to merge and in which order.
 *
 * Conventions shared by every entry point:
 *  - Ids: sub-index i's local id v has global id base_i + v, where base_i is
 *    the sum of the sizes of sub-indexes 0..i-1 in the order given.
 *  - Distances: RNSM_L2SQ = sum (x-y)^2, RNSM_IP = 1 - <x,y>,
 *    RNSM_COSINE = 1 - <x,y>/(|x||y|); all accumulate in float32. Every
 *    ordering is by (distance, id) ascending.
 *  - Prune rule: candidates sorted by (d(p,.), id); v is dropped when some
 *    already kept w has alpha * d(w,v) < d(p,v) (strict; alpha as float32,
 *    product formed in double); stop at R kept; no backfill.
 *  - Memory: every pointer marked "device" is HIP device memory (for example
 *    torch.Tensor.data_ptr() of a CUDA/HIP tensor). rnsm_merge, rnsm_search
 *    and rnsm_tune_search also take graphs and vectors in host memory
 *    (mem = RNSM_HOST), which they copy to the device first. Inputs are
 *    borrowed and read only; nothing is retained after a call returns.
 *    Outputs are caller-allocated device buffers, except a merge with
 *    RNSM_FLAG_HOST_OUT, whose host arrays the library allocates and
 *    rnsm_csr_free releases. Work runs on `stream` (NULL: the default stream)
 *    and every call has finished on the device when it returns.
 *  - Errors: every entry point returns rnsm_status; no exception crosses the
 *    boundary. On error the outputs are unspecified and nothing leaks;
 *    rnsm_last_error() describes the failure (thread-local).
 *  - The library is not reentrant per device: calls that overlap on one
 *    device are serialised by an internal lock.
 */
#ifndef RNSM_H
#define RNSM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RNSM_OK = 0,
    RNSM_EINVAL = 1,       /* bad argument or malformed input graph */
    RNSM_ENOMEM = 2,       /* device or host allocation failed */
    RNSM_EDEVICE = 3,      /* a HIP call failed */
    RNSM_EUNSUPPORTED = 4, /* valid but outside what the kernels handle */
    RNSM_EINTERNAL = 5
} rnsm_status;

typedef enum { RNSM_L2SQ = 0, RNSM_IP = 1, RNSM_COSINE = 2 } rnsm_metric;

/* where the memory of an input or output lives */
typedef enum { RNSM_DEVICE = 0, RNSM_HOST = 1 } rnsm_memspace;

/* storage type of the vectors the searches read (RNSM_U8: conversion input only) */
typedef enum { RNSM_F32 = 0, RNSM_BF16 = 1, RNSM_F16 = 2, RNSM_U8 = 3 } rnsm_dtype;

/* flags of rnsm_params */
#define RNSM_FLAG_ALL_PIVOTS 1u     /* every source vertex runs a naive search (cross-query merge) */
#define RNSM_FLAG_CENTROID_COSTS 2u /* MOS costs = centroid distances (default: unit costs) */
#define RNSM_FLAG_AUTOTUNE 4u       /* pick the search shape with rnsm_tune_search's measurement on
                                       the largest sub-index (65,536 of its rows, beam ef_naive),
                                       once per process for each device, storage type, row size,
                                       beam, R, metric and power-of-two size class; ignored when
                                       params fix search_hash_bits / search_waves_per_block */
#define RNSM_FLAG_HOST_OUT 8u       /* the merged graph goes to host arrays that the library
                                       allocates (out->mem = RNSM_HOST; free with rnsm_csr_free);
                                       the caller's out pointers are ignored */
#define RNSM_FLAG_NO_STATS 16u      /* skip the device timing events and counter read-back of
                                       rnsm_get_stats (its times and counts stay zero) */
#define RNSM_FLAG_BATCHED 32u       /* the batched form: operations in rounds of the plan
                                       (operations sharing no sub-index together), pivot selection
                                       on the device, and one persistent launch per round that
                                       searches every pivot group (pivot, then its followers) of
                                       the round's operations; the same merged graph */

/*
 * One input sub-index: a flat proximity graph (Section 2.2) over n vectors.
 * CSR: offsets[n+1] (int64, offsets[0] = 0, non-decreasing), nbrs[offsets[n]]
 * local ids in [0, n), both in device memory, or both in host memory with
 * mem = RNSM_HOST. Rows hold no self-loop and no duplicate, and at most R
 * entries (rnsm_merge rejects others with RNSM_EINVAL); nbrs may be NULL when
 * offsets[n] = 0 (no edges). entry: local id of the default entry point.
 */
typedef struct {
    int64_t n;
    const int64_t* offsets;
    const int32_t* nbrs;
    int32_t entry;
    rnsm_memspace mem;
} rnsm_graph;

/*
 * Vectors of all sub-indexes, concatenated in global-id order.
 * f32: device, row-major [n x dim] float32 original values; the prune, the
 *      output distances and the cosine norms read these.
 * search_dtype / search: the copy the beam searches read. RNSM_F32 reads f32
 *      (search may be NULL). RNSM_BF16 / RNSM_F16 read `search`, a device
 *      row-major [n x dim] array of 16-bit values (the plain FP32 form versus
 *      the reduced-precision form).
 * Rows are read in 16-byte chunks by groups of G lanes, G a power of two,
 * each lane holding 1 to 4 whole chunks: the number of chunks per row
 * (dim * element size / 16, for the 16-bit copy and for the float32 rows)
 * must be 2^k times 1, 2, 3 or 4 and at most 256 (float32: dim 4, 8, 12,
 * 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024); otherwise
 * RNSM_EUNSUPPORTED.
 * row_stride: elements from one row to the next in f32 and in search (0:
 *      dim, rows packed; otherwise >= dim, e.g. a column slice of a wider
 *      matrix). mem: RNSM_DEVICE, or RNSM_HOST for f32 and search in host
 *      memory. Strided or host rows are first copied, packed, to the device
 *      (rnsm_search_noalloc takes packed device rows only).
 */
typedef struct {
    int64_t n;
    int32_t dim;
    const float* f32;
    rnsm_dtype search_dtype;
    const void* search;
    int64_t row_stride;
    rnsm_memspace mem;
} rnsm_vectors;

/*
 * Parameters. Zero means "default" where a default is given.
 * R        max out-degree of the merged graph (1..64)
 * L        beam width; ef_naive and ef_slide default to L (1..128)
 * alpha    prune factor (>= 1)
 * k_reverse (default 5) reverse k-NN size, k_expand (default 16) the
 *          neighbor-expansion beam width k+ (Section 4.2); k_reverse <= k_expand <= 64
 * mos_degree   MOS degree bound (default max(2, ceil(sqrt(m))))
 * mos_diameter MOS diameter bound (default 2, must be >= 2)
 * flags    RNSM_FLAG_*
 * stream   hipStream_t or NULL
 * search_hash_bits, search_waves_per_block  shape of every beam search of
 *          the merge: log2 of the LDS visited table's two-way sets (8..12)
 *          and wavefronts per block (1..4, fewer when a block would need
 *          over 64 KB of LDS); 0 = the library's default for the beam width,
 *          degree and storage type (or, with RNSM_FLAG_AUTOTUNE, the shape
 *          the merge measures itself; its first call of a kind includes the
 *          tuning time). rnsm_tune_search measures them. Results do not
 *          depend on the shape, only the speed does.
 * max_device_bytes  budget of the device memory the merge's own buffers
 *          need (inputs copied from the host or from strided rows included,
 *          the caller's inputs and outputs not); a call that would exceed it
 *          returns RNSM_ENOMEM before allocating. 0: no budget.
 * prune_rule, prune_param  the edge-selection rule of the merge's prunes,
 *          for graphs of other proximity-graph families (Section 6's
 *          applicability experiment): RNSM_PRUNE_ALPHA (0, default; the RNG
 *          rule with factor alpha, NSG's MRNG at alpha = 1): kept w removes
 *          a later candidate v when alpha d(w,v) < d(p,v); RNSM_PRUNE_ANGLE
 *          (SSG): when the angle at p between v and w is below prune_param
 *          degrees (0 < theta <= 90); RNSM_PRUNE_TAU (tau-MNG): when
 *          |w - v| < |p - v| - 3 prune_param (tau >= 0). The angle and tau
 *          rules take RNSM_L2SQ (RNSM_EINVAL otherwise) and run on the
 *          float32 prune; decisions are taken in double from the float32
 *          distances, the rule's constant (cos theta, 3 tau) formed in
 *          double on the host.
 */
#define RNSM_PRUNE_ALPHA 0
#define RNSM_PRUNE_ANGLE 1
#define RNSM_PRUNE_TAU 2
typedef struct {
    int32_t R, L;
    float alpha;
    rnsm_metric metric;
    int32_t k_reverse, k_expand, ef_naive, ef_slide;
    int32_t mos_degree, mos_diameter;
    uint32_t flags;
    void* stream;
    int32_t search_hash_bits, search_waves_per_block;
    int64_t max_device_bytes;
    int32_t prune_rule;
    float prune_param;
} rnsm_params;

/*
 * Merged graph. By default caller-allocated device buffers:
 * offsets [N+1] int64; nbrs [N*R] int32 capacity (global ids, first
 * offsets[N] used); dists [N*R] float32 capacity or NULL (distance of each
 * edge, recomputed in float32 on the original vectors); mem = RNSM_DEVICE.
 * With RNSM_FLAG_HOST_OUT the library allocates host arrays offsets [N+1],
 * nbrs [n_edges] and dists [n_edges], sets mem = RNSM_HOST, and the caller
 * releases them with rnsm_csr_free (on error nothing is left allocated).
 * Written by the call: entry (global id of the entry of the largest
 * sub-index, ties: lowest index) and n_edges.
 * Pruned rows are in (distance, id) order; rows no operation touched keep the
 * input order.
 */
typedef struct {
    int64_t* offsets;
    int32_t* nbrs;
    float* dists;
    int32_t entry;
    int64_t n_edges;
    rnsm_memspace mem;
} rnsm_csr;

/* Releases the host arrays of a merged graph the library allocated
 * (mem = RNSM_HOST) and zeroes the struct; does nothing for NULL or for
 * caller-owned device buffers (mem = RNSM_DEVICE). */
void rnsm_csr_free(rnsm_csr* g);

/*
 * Counters and event timings of the last rnsm_merge on this thread. Arrays
 * indexed [3] are per search phase: 0 neighbor expansion, 1 pivots' naive
 * search, 2 followers' local sliding.
 */
typedef struct {
    double ms_total;        /* host wall time of the call */
    double ms_search[3];    /* search kernels of each phase (device events) */
    double ms_invert;       /* reverse k-NN inversion (device events) */
    double ms_plan;         /* host: MOS, reverse k-NN transfer, lazy greedy (the greedy
                               overlaps the device searches of the pivot groups it has
                               handed over) */
    double ms_prune;        /* source and target prunes with the reverse edges (device events) */
    double ms_compact;      /* CSR compaction (device events) */
    int64_t n_ops, n_source_vertices, n_pivots, n_followers, n_reverse_edges;
    int64_t queries[3];     /* searches run */
    int64_t ndc[3];         /* distance computations (re-evaluations included) */
    int64_t expansions[3];  /* vertices expanded */
    int64_t adjacency[3];   /* adjacency entries read */
    int64_t launches[3];    /* search kernel launches */
    double bytes[3];        /* algorithmic bytes from the counts above: every distance reads
                               one row, every expansion two offsets and its adjacency, every
                               query its row, its seeds and its output */
    int64_t hash_evictions; /* visited-table evictions: a forgotten vertex may be evaluated
                               again, which adds to ndc but never changes a result */
    int32_t row_bytes;      /* bytes of one row of the searched copy */
    int32_t exact_visited;  /* 1 when the searches ran with the probing visited table */
    int32_t prune_path;     /* prune arithmetic: 0 float32 walk, 1 bfloat16 MFMA Gram with
                               exact products (rows exact in bfloat16, integer sums below
                               2^24), 3 MFMA Gram with a hi/lo bfloat16 split of each row,
                               pairs near the alpha boundary decided in float32 as the walk
                               does; the MFMA forms cover dims 32..128 (multiples of 32)
                               and 256..1024 (multiples of 128) */
    double ms_search_span;  /* device time from the first naive search to the last sliding
                               search of each operation, summed over operations: naive and
                               sliding launches overlap on two streams, so this is below
                               ms_search[1] + ms_search[2] */
    int32_t search_hash_bits, search_waves_per_block;  /* shape of the operations' searches */
    int64_t prune_rechecks; /* prune_path 3: vertex pairs whose split-Gram estimate lay near the
                               alpha boundary and were decided with float32 arithmetic on
                               the original rows instead */
    int64_t n_rounds;       /* rounds of operations: the batched form runs the operations that
                               share no sub-index together; the plain form one per round */
    int64_t group_blocks;   /* batched form: blocks of the last round's persistent group search */
    int64_t group_overflow; /* batched form: followers past the first 2 of their pivot's group,
                               searched by a plain launch after the group search */
    double ms_order;        /* batched form: breadth-first orders of the sources (device time) */
    double ms_select;       /* batched form: pivot selection (device time) */
    int64_t select_rounds;  /* batched form: rounds of the parallel pivot selection */
    double ms_groups;       /* batched form: pivot groups, overflow lists and prune order */
} rnsm_stats;

/*
 * Merge m >= 2 sub-indexes into one graph (Algorithm 2 per operation,
 * Algorithm 3 for the operation plan; Section 5 for the order: operations
 * by ascending cost then (min index, max index), the smaller sub-index is the
 * source, ties: the lower index). Searches of every operation read the input
 * graphs only; rows start as the input rows and are updated operation by
 * operation. graphs[m], vecs (N = sum of sizes rows), params, out as above.
 * RNSM_EINVAL: m < 2, NULL pointers, vecs->n != N, R/L/alpha/k out of range,
 * an entry out of range, or a malformed input row (offsets not
 * non-decreasing, id out of range, self-loop, duplicate, degree > R).
 * RNSM_ENOMEM: a device or host allocation failed, or params->max_device_bytes
 * would be exceeded.
 */
rnsm_status rnsm_merge(int32_t m, const rnsm_graph* graphs, const rnsm_vectors* vecs,
                       const rnsm_params* params, rnsm_csr* out);

/* rnsm_merge with L2SQ, float32 search and default k, k+, MOS settings. */
rnsm_status rnsm_merge_simple(int32_t m, const rnsm_graph* graphs, const rnsm_vectors* vecs,
                              int32_t R, int32_t L, float alpha, rnsm_csr* out);

/*
 * Merge order selection (Algorithm 3) plus the execution order and direction
 * of Section 5. Host only: deterministic, thread-safe, no device work.
 * sizes[m]; centroids: NULL for unit costs (random partitions) or host
 * [m x dim] double centroids (costs = Euclidean distances). degree_bound >= 1,
 * diameter >= 2. out_ops receives 2*count int32: (source, target) pairs in
 * execution order; cap = capacity in pairs. out_fallbacks counts edges added
 * beyond the degree bound when no relay exists.
 * RNSM_EINVAL on bad arguments or when cap is too small.
 */
rnsm_status mos_plan(int32_t m, const int64_t* sizes, const double* centroids, int32_t dim,
                     int32_t degree_bound, int32_t diameter, int32_t* out_ops, int32_t cap,
                     int32_t* out_count, int32_t* out_fallbacks);

/*
 * Pivot and follower selection of RNSM (Algorithm 2, phase 2): the lazy
 * greedy over the reverse k-NN lists R_k, the same host code the merge runs
 * while its searches start. Host only: deterministic, thread-safe, no device
 * work. Repeatedly takes the vertex with the largest gain |R_k(x) minus
 * Covered| (ties: the smallest id); it becomes a pivot, and its uncovered
 * R_k members become its followers; it and they are then covered.
 * rk_offsets: host [n+1] int64, rk_offsets[0] = 0, non-decreasing;
 * rk_ids: host [rk_offsets[n]] int32, R_k(x) = rk_ids[rk_offsets[x] ..
 * rk_offsets[x+1]), ids in 0..n-1, not x itself, no repeats (may be NULL
 * when rk_offsets[n] = 0). All borrowed, read-only.
 * Outputs, host, caller-owned, capacity n each: pivots in selection order
 * (*out_n_pivots of them); followers grouped by pivot in selection order,
 * each group in its pivot's list order, with follower_pivot[i] the pivot of
 * followers[i] (*out_n_followers of them). Every vertex is written once,
 * as a pivot or as a follower: *out_n_pivots + *out_n_followers = n.
 * RNSM_EINVAL: n < 0 or n > INT32_MAX, NULL pointers, malformed lists.
 */
rnsm_status rnsm_select_pivots(int64_t n, const int64_t* rk_offsets, const int32_t* rk_ids,
                               int32_t* pivots, int64_t* out_n_pivots, int32_t* followers,
                               int32_t* follower_pivot, int64_t* out_n_followers);

/*
 * The same pivot and follower selection on the device (the batched form's
 * phase 2): the lazy greedy in parallel rounds. Each round, every uncovered
 * vertex whose key (gain, then the smaller id) is the largest at itself and
 * at each of its uncovered followers, among the uncovered vertices listing
 * that position, becomes a pivot and takes its uncovered followers. Such a
 * vertex is also the sequential greedy's pick before any vertex it competes
 * with, with the same followers, so the result equals rnsm_select_pivots'.
 * rk_offsets device [n+1] int64, rk_ids device int32 (as rnsm_select_pivots,
 * repeats not allowed); pivot_of device [n] int32 output: -1 for a pivot,
 * else the follower's pivot; *out_n_pivots (host) the pivot count.
 * Synchronises `stream`. RNSM_EINVAL for NULL pointers, n out of range
 * (0 <= n < 2^30: a gain word also carries the vertex's coverage), or an id
 * out of range or naming its own list's vertex.
 */
rnsm_status rnsm_select_pivots_device(int64_t n, const int64_t* rk_offsets, const int32_t* rk_ids,
                                      int32_t* pivot_of, int64_t* out_n_pivots, void* stream);

/*
 * Beam search (Algorithm 1) of nq queries in one graph.
 * g: the graph (local ids 0..n-1, device CSR), base: its n vectors
 * (search_dtype/search/f32 as in rnsm_vectors; base->n == g->n).
 * queries: device [nq x dim] in the same storage type as the searched copy.
 * seeds: device [nq x n_seeds] local ids (-1 = none) or NULL to start every
 * query from g->entry. ef in 1..128, k in 1..ef.
 * out_ids: device [nq x k] local ids (-1 when fewer than k found);
 * out_dists: device [nq x k] float32 or NULL.
 * Cosine: base norms come from base->f32, query norms from the query rows as
 * given (float32, or the 16-bit values); both summed in double.
 * Synchronises `stream` (NULL: the null stream) before returning.
 * RNSM_EINVAL on bad arguments; RNSM_EINTERNAL if a search exceeded its
 * iteration bound.
 */
rnsm_status rnsm_search(const rnsm_graph* g, const rnsm_vectors* base, const void* queries,
                        int64_t nq, const int32_t* seeds, int32_t n_seeds, int32_t ef, int32_t k,
                        rnsm_metric metric, int32_t* out_ids, float* out_dists, void* stream);

/*
 * rnsm_search for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results, but its counters, error flag and
 * cosine norms live in a static device array of the library (16 MiB per
 * device, held until the process ends) instead of library-allocated memory;
 * it calls no hipMalloc, hipFree or other allocating routine. The caller
 * still passes inputs and outputs. Every call on a device shares that
 * device's array, so calls that overlap on one device (on different
 * streams or threads) race; calls are otherwise serialised by the library's
 * lock. RNSM_EINVAL when cosine norms do not fit the array (4 bytes per base
 * row plus 4 per query, about 4.19 million rows together), besides the
 * argument errors of rnsm_search.
 */
rnsm_status rnsm_search_noalloc(const rnsm_graph* g, const rnsm_vectors* base, const void* queries,
                                int64_t nq, const int32_t* seeds, int32_t n_seeds, int32_t ef,
                                int32_t k, rnsm_metric metric, int32_t* out_ids, float* out_dists,
                                void* stream);

/*
 * Autotuner of the beam-search shape (the batched form's project-written
 * tuner of wavefronts per block and LDS visited-table size; the beam width
 * stays the caller's, since it sets recall). Times Algorithm 1 on the
 * device for min(n_sample, n) of the graph's own rows as queries (ids
 * i * n / n_sample), searched from g->entry with beam ef, under the
 * default shape and every table size 2^8..2^12 sets x 1, 2, 4 wavefronts
 * per block that fits 64 KB of LDS per block; each shape's time is the best
 * of three launches after one untimed launch. g, base as in rnsm_search.
 * Writes the fastest shape (pass it as rnsm_params.search_hash_bits /
 * search_waves_per_block) and the default's, with their times; synchronises
 * `stream` (NULL: the null stream). RNSM_EINVAL on bad arguments.
 */
typedef struct {
    int32_t hash_bits, waves_per_block;     /* fastest shape measured */
    float ms;                               /* its time for the sample */
    int32_t default_hash_bits, default_waves_per_block;
    float default_ms;
    int64_t n_queries;
    int32_t n_tried;                        /* shapes timed, the default included */
} rnsm_search_tuning;
rnsm_status rnsm_tune_search(const rnsm_graph* g, const rnsm_vectors* base, int32_t ef,
                             rnsm_metric metric, int64_t n_sample, rnsm_search_tuning* out,
                             void* stream);

/*
 * Sub-index builder used to make inputs: row(v) = Prune(v, knn(v), alpha, R);
 * with RNSM_BUILD_REVERSE, every kept v -> w offers v to w, and each w that
 * got offers is pruned again over row(w) + offers with alpha_rev. Entry: the
 * vertex closest to the centroid (exact integer criterion when every value
 * is an integer, float64 otherwise), ties by id. With RNSM_BUILD_REPAIR,
 * every vertex the entry cannot reach is linked in (the searches of
 * Algorithm 1 start from the entry alone), in passes: the heads of the
 * unreached part (unreached vertices no unreached vertex links to; when
 * there are none, those no unreached vertex of smaller id links to) each
 * propose to their
 * nearest reached vertex ((distance, id) order, float32 distances) with a
 * free slot in its row, else to their nearest reached vertex; every vertex
 * accepts its nearest proposals, as many as it has free slots, appended (a
 * full row accepts one, over its last, farthest entry); passes repeat (at
 * most 4096) until everything is reached. The nearest free vertex is read from the head's k-NN list when
 * the list holds one (exact for exact lists), else found by a full scan.
 * X: device [n x dim] float32. knn: device [n x K] local ids sorted by
 * (d, id), -1 padded, no self. out_offsets: device [n+1]; out_nbrs: device
 * [n x R] capacity. *out_entry written; *out_links (may be NULL): repair
 * links added. Synchronises `stream`.
 */
#define RNSM_BUILD_REVERSE 1
#define RNSM_BUILD_REPAIR 2
rnsm_status rnsm_build_graph(int64_t n, const float* X, int32_t dim, rnsm_metric metric,
                             const int32_t* knn, int32_t K, int32_t R, float alpha,
                             int32_t options, float alpha_rev, int64_t* out_offsets,
                             int32_t* out_nbrs, int32_t* out_entry, int64_t* out_links,
                             void* stream);

/*
 * Vertices reachable from `entry` along the edges of a CSR graph (entry
 * included): the fraction a search from the entry (Algorithm 1) can reach.
 * offsets: device [n+1] int64, nbrs: device int32 ids (entries outside
 * 0..n-1 are skipped). *out_count written. Synchronises `stream`.
 * RNSM_EINVAL on a NULL pointer, an entry outside 0..n-1 or malformed
 * offsets.
 */
rnsm_status rnsm_reachable(int64_t n, const int64_t* offsets, const int32_t* nbrs, int32_t entry,
                           int64_t* out_count, void* stream);

/*
 * Staging conversion of vectors on the device (the inputs of the merge: the
 * 16-bit search copy of float32 rows, or float32 / float16 rows from uint8
 * data). count elements from src (src_type) to dst (dst_type), both device
 * pointers, caller-owned, not overlapping. Supported:
 *   F32 -> BF16, F32 -> F16: round to nearest, ties to even (the rounding of
 *        the IEEE 754 conversions); NaN stays NaN (quiet), infinities and
 *        values past the largest finite value become infinities;
 *   U8 -> F16, U8 -> F32, U8 -> BF16: exact (every 0..255 is representable).
 * Asynchronous on `stream` (NULL: the null stream). RNSM_EINVAL for NULL
 * pointers with count > 0, count < 0 or an unsupported pair.
 */
rnsm_status rnsm_convert(const void* src, rnsm_dtype src_type, void* dst, rnsm_dtype dst_type,
                         int64_t count, void* stream);

/* Stats of the last rnsm_merge on the calling thread. */
rnsm_status rnsm_get_stats(rnsm_stats* out);

/* Thread-local message of the last failure ("" if none). */
const char* rnsm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RNSM_H */
