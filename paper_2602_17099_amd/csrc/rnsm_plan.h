// Host planning of the RNSM path (no device code).
#pragma once
#include <stdint.h>

#include <utility>
#include <vector>

namespace rnsm {

// Algorithm 3 edges in insertion order; 0 on success
int mos_edges(int m, const std::vector<double>& cost, int R, int delta,
              std::vector<std::pair<int, int>>& edges, int* fallbacks);

// MOS edges ordered by (cost, min index, max index), each directed from the
// smaller sub-index (ties: the lower index) to the larger
int plan_ops(int m, const int64_t* sizes, const double* centroids, int dim, int R, int delta,
             std::vector<std::pair<int, int>>& ops, int* fallbacks);

struct Pivots {
    std::vector<int32_t> pivots;          // selection order
    std::vector<int32_t> followers;       // grouped by pivot (selection order), ids ascending
    std::vector<int32_t> follower_pivot;  // pivot of each follower
};

// lazy greedy over reverse k-NN lists R_k (CSR; the order inside a list only
// changes the order of the follower list, not the pivots or their followers)
void select_pivots(int64_t n, const int64_t* rk_off, const int32_t* rk_ids, Pivots& out);

}  // namespace rnsm
