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

// Gain levels of the lazy greedy: level g holds, as a bitmap over vertex
// ids, the vertices whose stored gain is g (levels up to LCAP - 1; higher
// gains wait in a heap ordered the same way). Built from the R_k list
// lengths alone, so it can be made while the lists are still in transit;
// the storage is kept for the next build.
struct GainLevels {
    static constexpr int LCAP = 32;
    int64_t n = 0, words = 0;
    int nlev = 0;                   // levels held in `bits` (or `ext`)
    std::vector<uint64_t> bits;     // nlev x words
    uint64_t* ext = nullptr;        // the same layout in a caller's buffer, used instead
    std::vector<std::pair<int64_t, int32_t>> high;  // (gain, id) of gains >= LCAP
    uint64_t* data() { return ext ? ext : bits.data(); }
};
void build_levels(int64_t n, const int32_t* counts, GainLevels& L);

// Lazy greedy over reverse k-NN lists R_k (CSR) from levels built on the
// same lists (the levels are consumed). Writes the pivots in selection
// order, and the followers grouped by pivot (selection order) with the
// pivot of each follower; the order inside an R_k list only changes the
// order of a pivot's followers, not the pivots or their follower sets.
// `emit(np, nf)` is called with the running counts each time at least
// `chunk` vertices (pivots plus followers; the chunk doubles after every call
// up to chunk_max) were added since the last call, and once at the end; a
// caller can start work on every group emitted so far while the selection
// goes on. `lists_ready` (optional) is called before rk_off / rk_ids are
// first read, so that they may still be in transit until then.
using Emit = std::function<void(int64_t np, int64_t nf)>;
void select_pivots(GainLevels& L, const int64_t* rk_off, const int32_t* rk_ids, int32_t* pivots,
                   int32_t* followers, int32_t* follower_pivot, int64_t chunk, int64_t chunk_max,
                   const Emit& emit, const std::function<void()>& lists_ready = {});

}  // namespace rnsm
