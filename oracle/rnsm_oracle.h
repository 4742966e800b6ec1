/*
 * CPU reference of the RNSM merge path (arXiv 2602.17099). Test
 * infrastructure only: used by the test suite, the smoke check and the CPU
 * baseline leg of the benchmark, never by the product library.
 */
#ifndef RNSM_ORACLE_H
#define RNSM_ORACLE_H
#include <stdint.h>

enum { ORC_L2SQ = 0, ORC_IP = 1, ORC_COSINE = 2 };

typedef struct {
    int R;            /* max out-degree of the merged graph */
    int ef_naive;     /* beam width of the pivots' naive search (L) */
    int ef_slide;     /* beam width of the followers' local sliding */
    float alpha;      /* prune factor, compared as (double)alpha * d < d */
    int metric;
    int k;            /* reverse-kNN size */
    int kplus;        /* expansion beam width */
    int mos_degree;   /* <= 0: max(2, ceil(sqrt(m))) */
    int mos_diameter; /* >= 2 */
    int use_centroids;/* MOS costs from centroids (1) or unit costs (0) */
    int all_pivots;   /* every source vertex runs a naive search (CM) */
    int prune_rule;   /* 0 alpha, 1 angle (SSG, prune_param = theta in degrees), 2 tau-MNG
                         (prune_param = tau); 1 and 2 take squared L2 */
    float prune_param;
} orc_params_t;

typedef struct {
    /* first operation only; each pointer may be NULL */
    int32_t* nk;       /* [n_s x k] local ids, -1 padded */
    int32_t* pivot_of; /* [n_s] -1 for pivots, else the pivot's local id */
    int32_t* res_ids;  /* [n_s x max(ef_naive, ef_slide)] target-local ids, -1 padded */
    double* res_d;
    int64_t ndc_expand, ndc_naive, ndc_slide, n_pivots;
} orc_trace_t;

/* threads for the loops over independent vertices (OpenMP builds; 1 = sequential) */
void orc_set_threads(int n);
int orc_get_threads(void);
double orc_dist_vec(const float* a, const float* b, int dim, int metric, double na, double nb);
void orc_norms(const float* X, int64_t n, int dim, double* out);
int orc_beam_search(int64_t n, const int64_t* offsets, const int32_t* nbrs, int64_t base,
                    const float* X, int dim, int metric, const double* norms, const float* q,
                    const int32_t* seeds, int nseeds, int ef, int32_t* out_ids, double* out_d,
                    int64_t* ndc);
int orc_prune(int64_t p, const int32_t* W, int nW, const float* X, int dim, int metric,
              const double* norms, float alpha, int R, int32_t* out_ids, double* out_d);
int orc_prune_rule(int64_t p, const int32_t* W, int nW, const float* X, int dim, int metric,
                   const double* norms, int rule, float alpha, float param, int R,
                   int32_t* out_ids, double* out_d);
int orc_expand(int64_t n, const int64_t* offsets, const int32_t* nbrs, int64_t base,
               const float* X, int dim, int metric, const double* norms, int k, int kplus,
               int32_t* nk_out);
int orc_expand_range(int64_t n, const int64_t* offsets, const int32_t* nbrs, int64_t base,
                     const float* X, int dim, int metric, const double* norms, int k, int kplus,
                     int64_t v0, int64_t v1, int32_t* nk_out);
int orc_invert(int64_t n, const int32_t* nk, int k, int64_t* rk_off, int32_t* rk_ids);
int orc_pivots(int64_t n, const int64_t* rk_off, const int32_t* rk_ids, int32_t* pivot_of,
               int32_t* order, int64_t* n_piv);
void orc_mos_cost(int m, const double* centroids, int dim, double* C);
int orc_mos(int m, const double* C, int R, int delta, int32_t* out_edges, int cap, int* n_edges,
            int* n_fallback);
int orc_plan(int m, const int64_t* sizes, const double* centroids, int dim, int R, int delta,
             int32_t* out_ops, int cap, int* n_ops, int* n_fallback);
int orc_plan_cost(int m, const int64_t* sizes, const double* C, int R, int delta,
                  int32_t* out_ops, int cap, int* n_ops, int* n_fallback);
int orc_merge(int m, const int64_t* sizes, const int64_t* offsets_cat, const int32_t* nbrs_cat,
              const int32_t* entries, const float* X, int dim, const orc_params_t* P,
              int32_t* out_rows, double* out_dists, int32_t* out_deg, int32_t* out_entry,
              int32_t* out_ops, int* out_nops, orc_trace_t* trace);
int orc_knn(int64_t n, const float* X, int dim, int metric, int K, int32_t* out);
int orc_knn_queries(int64_t n, const float* X, int64_t nq, const float* Q, int dim, int metric,
                    int K, int32_t* out_ids, double* out_d);
/* options: 1 reverse edges with an alpha_rev re-prune, 2 reachability repair
 * from the entry; returns the number of repair links added */
int orc_build(int64_t n, const float* X, int dim, int metric, const int32_t* knn, int K, int R,
              float alpha, int options, float alpha_rev, int64_t* out_offsets, int32_t* out_nbrs,
              int32_t* out_entry);
/* the builder's reachability repair on rows of up to R ids (row v at rows +
 * v R, deg[v] used), in place; returns the number of links added */
int64_t orc_repair(int64_t n, const float* X, int dim, int metric, int R, int32_t* rows,
                   int32_t* deg, int32_t entry);
/* vertices reachable from entry along the CSR edges (entry included) */
int64_t orc_reachable(int64_t n, const int64_t* offsets, const int32_t* nbrs, int32_t entry);
#endif
