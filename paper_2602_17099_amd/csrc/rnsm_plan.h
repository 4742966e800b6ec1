// Host planning of the RNSM path (no device code).
#pragma once
#include <stdint.h>

#include <functional>
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

// Lazy greedy over reverse k-NN lists R_k (CSR). Writes the pivots in
// selection order, and the followers grouped by pivot (selection order) with
// the pivot of each follower; the order inside an R_k list only changes the
// order of a pivot's followers, not the pivots or their follower sets.
// `emit(np, nf)` is called with the running counts each time at least
// `chunk` vertices (pivots plus followers; the chunk doubles after every call
// up to chunk_max) were added since the last call, and once at the end; a
// caller can start work on every group emitted so far while the selection
// goes on.
// `ids_ready` (optional) is called after the gain levels are built from
// rk_off and before rk_ids is first read, so that the ids may still be in
// transit while the levels are built.
using Emit = std::function<void(int64_t np, int64_t nf)>;
void select_pivots(int64_t n, const int64_t* rk_off, const int32_t* rk_ids, int32_t* pivots,
                   int32_t* followers, int32_t* follower_pivot, int64_t chunk, int64_t chunk_max,
                   const Emit& emit, const std::function<void()>& ids_ready = {});

}  // namespace rnsm
