// C ABI of librnsm (declared in include/rnsm.h): argument checks, device
// workspace, and the orchestration of the RNSM merge (Algorithm 2 per
// operation, Algorithm 3 for the plan).
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <array>
#include <chrono>
#include <cmath>
#include <map>
#include <thread>
#include <deque>
#include <condition_variable>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rnsm.h"
#include "rnsm_internal.h"
#include "rnsm_plan.h"

using namespace rnsm;

namespace {

thread_local std::string g_err;
thread_local rnsm_stats g_stats;
std::mutex g_lock;

rnsm_status fail(rnsm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            return fail(e_ == hipErrorOutOfMemory ? RNSM_ENOMEM : RNSM_EDEVICE, "%s: %s (%s:%d)", \
                        #x, hipGetErrorString(e_), __FILE__, __LINE__);                    \
    } while (0)

// device buffers kept between calls, per device, grown on demand
struct Workspace {
    struct Buf {
        void* p = nullptr;
        size_t bytes = 0;
        uint64_t call = 0;  // the call that last requested it
        size_t need = 0;    // the largest size that call requested
    };
    // Per call (begin_call): the device bytes the call's own buffers need
    // (each named buffer counted once, at the largest size the call asks
    // for), checked against the caller's budget before any allocation; and
    // the allocation-failure injector: with RNSM_FAIL_ALLOC=k the call's k-th
    // buffer request (device or pinned host) fails as out of memory, before
    // anything is allocated (for tests of the error paths).
    uint64_t call_id = 0;
    size_t call_bytes = 0, budget = 0;
    int64_t requests = 0, fail_at = 0;
    void begin_call(int64_t max_device_bytes) {
        ++call_id;
        call_bytes = 0;
        budget = max_device_bytes > 0 ? (size_t)max_device_bytes : 0;
        requests = 0;
        const char* f = getenv("RNSM_FAIL_ALLOC");
        fail_at = f ? atoll(f) : 0;
    }
    bool inject_failure() { return ++requests == fail_at; }
    std::map<std::string, Buf> bufs, hbufs;
    GainLevels levels;  // lazy-greedy gain levels, storage kept between calls
    // second stream (default priority) for the naive searches of the pivot
    // chunks, which then overlap the sliding searches of earlier chunks
    hipStream_t side = nullptr;
    hipError_t side_stream(hipStream_t* out) {
        if (!side) {
            hipError_t e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
            if (e != hipSuccess) {
                side = nullptr;
                return e;
            }
        }
        *out = side;
        return hipSuccess;
    }
    // pinned host staging buffers (hipHostMalloc), kept like the device ones
    hipError_t hget(const std::string& name, size_t bytes, void** out) {
        if (inject_failure()) return hipErrorOutOfMemory;
        Buf& b = hbufs[name];
        if (bytes == 0) bytes = 16;
        if (b.bytes < bytes) {
            if (b.p) {
                hipError_t e = hipHostFree(b.p);
                if (e != hipSuccess) return e;
                b.p = nullptr;
                b.bytes = 0;
            }
            hipError_t e = hipHostMalloc(&b.p, bytes, hipHostMallocDefault);
            if (e != hipSuccess) return e;
            b.bytes = bytes;
        }
        *out = b.p;
        return hipSuccess;
    }
    hipError_t get(const std::string& name, size_t bytes, void** out) {
        if (inject_failure()) return hipErrorOutOfMemory;
        Buf& b = bufs[name];
        if (bytes == 0) bytes = 16;
        const size_t prev = b.call == call_id ? b.need : 0;
        const size_t need = std::max(prev, bytes);
        if (budget && call_bytes - prev + need > budget) return hipErrorOutOfMemory;
        call_bytes = call_bytes - prev + need;
        b.call = call_id;
        b.need = need;
        if (b.bytes < bytes) {
            if (b.p) {
                hipError_t e = hipFree(b.p);
                if (e != hipSuccess) return e;
                b.p = nullptr;
                b.bytes = 0;
            }
            hipError_t e = hipMalloc(&b.p, bytes);
            if (e != hipSuccess) return e;
            b.bytes = bytes;
        }
        *out = b.p;
        return hipSuccess;
    }
};
std::map<int, Workspace> g_ws;

#define WS(ptr, name, bytes) HIPCHK(ws.get(name, (size_t)(bytes), (void**)&(ptr)))
#define HS(ptr, name, bytes) HIPCHK(ws.hget(name, (size_t)(bytes), (void**)&(ptr)))

int elt_size(rnsm_dtype t) { return t == RNSM_F32 ? 4 : 2; }

int ilog2_ceil(int64_t x) {
    int b = 0;
    while ((1ll << b) < x) ++b;
    return b;
}

// LDS visited-table size, wavefronts per block and table mode of a search of
// beam ef over a graph of n vertices with rows of degree <= maxdeg, on the
// copy of type tt. The fast table is lossy (a forgotten vertex is evaluated
// again and dropped by key), so it is sized for occupancy rather than for
// the whole visited set: 8 KB (2048 two-way sets of 16-bit tags) for the L=64, R=32
// searches on float32 rows; 4 KB on 16-bit rows, whose kernels need fewer
// registers, so that LDS does not cap their occupancy below the registers'
// 6 wavefronts per SIMD. RNSM_EXACT_VISITED=1, or a
// graph too large for 16-bit tags, selects an 8192-slot probing table that
// holds every visited vertex (distance counts then equal the method's own).
// RNSM_HASH_BITS / RNSM_WPB override the sizes (diagnostics); a caller's
// hb_req / wpb_req (non-zero: the merge's search_hash_bits and
// search_waves_per_block, say from rnsm_tune_search) override both. Blocks
// are cut to at most 64 KB of LDS by using fewer wavefronts per block.
struct SearchShape {
    int hbits, wpb, mode;
};

// visited-table sizes (log2 of the two-way sets) a caller may ask for
constexpr int TUNE_HB_MIN = 8, TUNE_HB_MAX = 12;

SearchShape search_shape(int ef, int maxdeg, int64_t n, int tt, int hb_req = 0, int wpb_req = 0) {
    SearchShape s;
    const int hmax = tt == 0 ? 11 : 10;
    int hb = ilog2_ceil((int64_t)ef * (maxdeg > 0 ? maxdeg : 16));
    hb = hb < 8 ? 8 : (hb > hmax ? hmax : hb);
    s.mode = 0;
    const char* x = getenv("RNSM_EXACT_VISITED");
    if (x && atoi(x) == 1) {
        s.mode = 1;
        hb = 13;
    }
    const char* e = getenv("RNSM_HASH_BITS");
    if (e && atoi(e) >= 6 && atoi(e) <= 14) hb = atoi(e);
    if (hb_req > 0 && s.mode == 0) hb = hb_req;
    if (s.mode == 0 && n >= ((int64_t)0xffff << hb)) {
        s.mode = 1;  // ids do not fit the 16-bit tags
        hb = 13;
    }
    int w = 1;
    const char* ew = getenv("RNSM_WPB");
    if (ew && atoi(ew) >= 1 && atoi(ew) <= 4) w = atoi(ew);
    if (wpb_req > 0) w = wpb_req;
    while (w > 1 && search_lds_bytes(hb, w) > 64 * 1024) --w;
    s.hbits = hb;
    s.wpb = w;
    return s;
}

struct VecInfo {
    int tt;        // 0 f32, 1 bf16, 2 f16 (search copy)
    int row_bytes; // search copy
    int nch;       // chunks of the search copy
    int G, cpl;
    int nch32, G32, cpl32;  // float32 originals (prune)
    const char* search;
};

rnsm_status vec_info(const rnsm_vectors* v, VecInfo& vi) {
    if (!v->f32) return fail(RNSM_EINVAL, "vectors: f32 is NULL");
    if (v->dim < 1) return fail(RNSM_EINVAL, "vectors: dim < 1");
    if (v->search_dtype != RNSM_F32 && v->search_dtype != RNSM_BF16 &&
        v->search_dtype != RNSM_F16)
        return fail(RNSM_EINVAL, "vectors: unknown search dtype %d", (int)v->search_dtype);
    if (v->search_dtype != RNSM_F32 && !v->search)
        return fail(RNSM_EINVAL, "vectors: search copy is NULL for a 16-bit search dtype");
    const int es = elt_size(v->search_dtype);
    if (((int64_t)v->dim * es) % 16 != 0 || ((int64_t)v->dim * 4) % 16 != 0)
        return fail(RNSM_EUNSUPPORTED, "vectors: dim %d gives rows that are not a multiple of 16 bytes",
                    v->dim);
    vi.tt = v->search_dtype == RNSM_F32 ? 0 : (v->search_dtype == RNSM_BF16 ? 1 : 2);
    vi.row_bytes = v->dim * es;
    vi.nch = vi.row_bytes / 16;
    vi.G = lanes_per_row(vi.nch);
    vi.nch32 = v->dim / 4;
    vi.G32 = lanes_per_row(vi.nch32);
    if (vi.G < 0 || vi.G32 < 0)
        return fail(RNSM_EUNSUPPORTED,
                    "vectors: dim %d does not split into whole 16-byte chunks per lane "
                    "(supported: chunks per row = 2^k x {1,2,3,4}, up to 256)", v->dim);
    vi.cpl = (vi.nch + vi.G - 1) / vi.G;
    vi.cpl32 = (vi.nch32 + vi.G32 - 1) / vi.G32;
    vi.search = v->search_dtype == RNSM_F32 ? (const char*)v->f32 : (const char*)v->search;
    return RNSM_OK;
}

// Staging of inputs (the first step of the path): the kernels read device
// CSR and packed device rows, so graphs in host memory, and rows in host
// memory or with a row stride, are first copied into workspace buffers.
rnsm_status stage_graph(Workspace& ws, const char* fn, int idx, const rnsm_graph& g,
                        hipStream_t st, rnsm_graph& out) {
    out = g;
    out.mem = RNSM_DEVICE;
    if (g.mem == RNSM_DEVICE) return RNSM_OK;
    if (g.mem != RNSM_HOST) return fail(RNSM_EINVAL, "%s: graph %d: unknown memspace", fn, idx);
    if (!g.offsets) return fail(RNSM_EINVAL, "%s: graph %d has a NULL CSR pointer", fn, idx);
    const int64_t nnz = g.offsets[g.n];
    if (g.offsets[0] != 0 || nnz < 0)
        return fail(RNSM_EINVAL, "%s: graph %d: offsets[0] != 0 or offsets[n] < 0", fn, idx);
    if (nnz > 0 && !g.nbrs) return fail(RNSM_EINVAL, "%s: graph %d has a NULL CSR pointer", fn, idx);
    int64_t* o;
    int32_t* nb;
    const std::string tag = std::to_string(idx);
    WS(o, "in_offsets_" + tag, sizeof(int64_t) * (g.n + 1));
    WS(nb, "in_nbrs_" + tag, sizeof(int32_t) * std::max<int64_t>(nnz, 1));
    HIPCHK(hipMemcpyAsync(o, g.offsets, sizeof(int64_t) * (g.n + 1), hipMemcpyHostToDevice, st));
    if (nnz > 0)
        HIPCHK(hipMemcpyAsync(nb, g.nbrs, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st));
    out.offsets = o;
    out.nbrs = nnz > 0 ? nb : nullptr;
    return RNSM_OK;
}

// rows of v packed on the device (out.row_stride = 0, out.mem = device);
// v.dim, v.f32 and the search copy were checked by vec_info
rnsm_status stage_vectors(Workspace& ws, const char* fn, const rnsm_vectors& v, hipStream_t st,
                          rnsm_vectors& out) {
    out = v;
    out.mem = RNSM_DEVICE;
    out.row_stride = 0;
    if (v.mem != RNSM_DEVICE && v.mem != RNSM_HOST)
        return fail(RNSM_EINVAL, "%s: vectors: unknown memspace", fn);
    const int64_t stride = v.row_stride ? v.row_stride : v.dim;
    if (stride < v.dim) return fail(RNSM_EINVAL, "%s: vectors: row_stride < dim", fn);
    if (v.mem == RNSM_DEVICE && stride == v.dim) return RNSM_OK;
    const hipMemcpyKind kind = v.mem == RNSM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    auto copy_rows = [&](void* dst, const void* src, size_t esz) -> hipError_t {
        if (stride == v.dim)
            return hipMemcpyAsync(dst, src, esz * v.dim * v.n, kind, st);
        return hipMemcpy2DAsync(dst, esz * v.dim, src, esz * stride, esz * v.dim, v.n, kind, st);
    };
    float* f;
    WS(f, "in_f32", sizeof(float) * v.n * v.dim);
    HIPCHK(copy_rows(f, v.f32, sizeof(float)));
    out.f32 = f;
    if (v.search_dtype != RNSM_F32) {
        void* sc;
        WS(sc, "in_search", (size_t)2 * v.n * v.dim);
        HIPCHK(copy_rows(sc, v.search, 2));
        out.search = sc;
    }
    return RNSM_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

struct Events {
    std::vector<hipEvent_t> ev;
    bool no_stats = false;  // RNSM_FLAG_NO_STATS: stat() records nothing
    ~Events() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    // an event that only times a phase for rnsm_get_stats (index -1 when skipped)
    hipError_t stat(hipStream_t st, int* idx) {
        if (no_stats) {
            *idx = -1;
            return hipSuccess;
        }
        return record(st, idx);
    }
    hipError_t record(hipStream_t st, int* idx) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        ev.push_back(e);
        *idx = (int)ev.size() - 1;
        return hipEventRecord(e, st);
    }
    float between(int a, int b) {
        float ms = 0.f;
        if (a >= 0 && b >= 0) (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
        return ms;
    }
};

// Value summary of float32 rows X (n x dim): whether every value is an
// integer, the largest magnitude and the spread (max - min).
struct ValueInfo {
    bool integral = false;
    double bound = INFINITY, range = INFINITY;
};
// the summary from launch_value_range's three words
void decode_value_range(const unsigned* h, ValueInfo* out) {
    const double lo = key_to_float(h[1]), hi = key_to_float(h[2]);
    out->integral = h[0] == 1u;
    out->bound = std::max(std::fabs(lo), std::fabs(hi));
    out->range = hi - lo;
    if (!std::isfinite(out->bound)) out->integral = false;
}

hipError_t value_info(const float* X, int64_t n, int dim, unsigned* scratch3, hipStream_t st,
                      ValueInfo* out) {
    hipError_t e = launch_value_range(X, n * dim, scratch3, st);
    if (e != hipSuccess) return e;
    unsigned h[3];
    e = hipMemcpyAsync(h, scratch3, sizeof h, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    decode_value_range(h, out);
    return hipSuccess;
}

// Integer rows of magnitude <= maxmag (exact in a 16-bit float type with
// that many integers) whose distance sums are all exact in float32: every
// inner-product partial sum (dim * bound^2) and every squared-L2 partial sum
// (dim * range^2) below 2^24. Then every distance is the same number in any
// summation order, whichever copy it is computed from.
bool int_exact(const ValueInfo& v, int dim, double maxmag) {
    const double lim = 16777216.0;
    return v.integral && v.bound <= maxmag && (double)dim * v.bound * v.bound < lim &&
           (double)dim * v.range * v.range < lim;
}

// Prune arithmetic: the bfloat16 MFMA Gram when the dimension fits it, with
// exact products (mode 1) on rows exact in bfloat16 with exact sums, the
// hi/lo split (mode 3) otherwise; the float32 walk (mode 0) for other
// dimensions. RNSM_PRUNE=walk|split forces mode 0 / 3 where allowed.
int choose_prune(const ValueInfo& v, int dim, int R) {
    const char* env = getenv("RNSM_PRUNE");
    if (env && !strcmp(env, "walk")) return 0;
    if (!prune_mfma_supported(dim) || R > 64) return 0;
    if (env && !strcmp(env, "split")) return 3;
    return int_exact(v, dim, 256.0) ? 1 : 3;
}

// relative band of the float re-decision in the MFMA prune (RNSM_PRUNE_BAND:
// log2 of the band, e.g. -4; "off" disables it, for measurement)
double prune_band() {
    const char* e = getenv("RNSM_PRUNE_BAND");
    if (!e) return PRUNE_BAND;
    if (!strcmp(e, "off")) return 0.0;
    const int v = atoi(e);
    return v < 0 && v > -60 ? std::ldexp(1.0, v) : PRUNE_BAND;
}

hipError_t run_prune(const PruneArgs& a, int mode, hipStream_t st) {
    if (mode != 0 && prune_mfma_fits(a, mode)) {
        if (a.extra_mode != 2) return launch_prune_mfma(a, mode, st);
        // candidate lists of any length: the MFMA Gram takes those up to
        // LONG_LIST, the float32 walk the longer ones (targets with thousands
        // of reverse edges; the same decisions, see the band re-decision)
        PruneArgs b = a;
        b.list_filter = 1;
        hipError_t e = launch_prune_mfma(b, mode, st);
        if (e != hipSuccess) return e;
        b.list_filter = 2;
        return launch_prune(b, st);
    }
    return launch_prune(a, st);
}

// run_prune(a, mode) takes its candidate distances from the bfloat16 copy
bool prune_reads_b16(const PruneArgs& a, int mode) { return mode == 1 && prune_mfma_fits(a, 1); }

// LDS key capacity of a merge's target prune (longer candidate lists use scratch)
constexpr int TARGET_WCAP = 256;

}  // namespace

const char* rnsm_last_error(void) { return g_err.c_str(); }

static rnsm_status rnsm_convert_impl(const void* src, rnsm_dtype src_type, void* dst, rnsm_dtype dst_type,
                         int64_t count, void* stream) {
    g_err.clear();
    if (count < 0) return fail(RNSM_EINVAL, "rnsm_convert: count < 0");
    if (count > 0 && (!src || !dst)) return fail(RNSM_EINVAL, "rnsm_convert: NULL pointer");
    const bool ok = (src_type == RNSM_F32 && (dst_type == RNSM_BF16 || dst_type == RNSM_F16)) ||
                    (src_type == RNSM_U8 &&
                     (dst_type == RNSM_F16 || dst_type == RNSM_F32 || dst_type == RNSM_BF16));
    if (!ok)
        return fail(RNSM_EINVAL, "rnsm_convert: unsupported conversion %d -> %d", (int)src_type,
                    (int)dst_type);
    HIPCHK(launch_convert(src, (int)src_type, dst, (int)dst_type, count, (hipStream_t)stream));
    return RNSM_OK;
}

static rnsm_status rnsm_get_stats_impl(rnsm_stats* out) {
    if (!out) return fail(RNSM_EINVAL, "rnsm_get_stats: NULL");
    *out = g_stats;
    return RNSM_OK;
}

static rnsm_status mos_plan_impl(int32_t m, const int64_t* sizes, const double* centroids, int32_t dim,
                     int32_t degree_bound, int32_t diameter, int32_t* out_ops, int32_t cap,
                     int32_t* out_count, int32_t* out_fallbacks) {
    g_err.clear();
    if (m < 1 || !sizes || !out_ops || !out_count) return fail(RNSM_EINVAL, "mos_plan: bad arguments");
    if (degree_bound < 1) return fail(RNSM_EINVAL, "mos_plan: degree_bound < 1");
    if (diameter < 2) return fail(RNSM_EINVAL, "mos_plan: diameter < 2");
    if (centroids && dim < 1) return fail(RNSM_EINVAL, "mos_plan: dim < 1 with centroids");
    for (int i = 0; i < m; ++i)
        if (sizes[i] < 1) return fail(RNSM_EINVAL, "mos_plan: size of sub-index %d < 1", i);
    std::vector<std::pair<int, int>> ops;
    int fb = 0;
    if (plan_ops(m, sizes, centroids, dim, degree_bound, diameter, ops, &fb) != 0)
        return fail(RNSM_EINTERNAL, "mos_plan: planner failed");
    if ((int64_t)ops.size() > cap)
        return fail(RNSM_EINVAL, "mos_plan: %d operations exceed cap %d", (int)ops.size(), cap);
    for (size_t i = 0; i < ops.size(); ++i) {
        out_ops[2 * i] = ops[i].first;
        out_ops[2 * i + 1] = ops[i].second;
    }
    *out_count = (int32_t)ops.size();
    if (out_fallbacks) *out_fallbacks = fb;
    return RNSM_OK;
}

static rnsm_status rnsm_select_pivots_impl(int64_t n, const int64_t* rk_offsets, const int32_t* rk_ids,
                               int32_t* pivots, int64_t* out_n_pivots, int32_t* followers,
                               int32_t* follower_pivot, int64_t* out_n_followers) {
    g_err.clear();
    if (n < 0 || n > INT32_MAX) return fail(RNSM_EINVAL, "rnsm_select_pivots: n out of range");
    if (!rk_offsets || !out_n_pivots || !out_n_followers || (n > 0 && (!pivots || !followers ||
                                                                       !follower_pivot)))
        return fail(RNSM_EINVAL, "rnsm_select_pivots: NULL pointer");
    if (rk_offsets[0] != 0) return fail(RNSM_EINVAL, "rnsm_select_pivots: rk_offsets[0] != 0");
    for (int64_t x = 0; x < n; ++x)
        if (rk_offsets[x + 1] < rk_offsets[x])
            return fail(RNSM_EINVAL, "rnsm_select_pivots: rk_offsets decrease at %lld", (long long)x);
    if (rk_offsets[n] > 0 && !rk_ids) return fail(RNSM_EINVAL, "rnsm_select_pivots: NULL rk_ids");
    // a list names other vertices, each once (the gain counts distinct ids)
    std::vector<int32_t> seen((size_t)n, -1);
    std::vector<int32_t> counts((size_t)n);
    for (int64_t x = 0; x < n; ++x) {
        for (int64_t j = rk_offsets[x]; j < rk_offsets[x + 1]; ++j) {
            const int32_t y = rk_ids[j];
            if (y < 0 || y >= n || y == x || seen[(size_t)y] == (int32_t)x)
                return fail(RNSM_EINVAL, "rnsm_select_pivots: list of %lld: id %d out of range, "
                            "itself or repeated", (long long)x, (int)y);
            seen[(size_t)y] = (int32_t)x;
        }
        counts[(size_t)x] = (int32_t)std::min<int64_t>(rk_offsets[x + 1] - rk_offsets[x], INT32_MAX);
    }
    GainLevels levels;
    build_levels(n, counts.data(), levels);
    int64_t np = 0, nf = 0;
    select_pivots(levels, rk_offsets, rk_ids, pivots, followers, follower_pivot,
                  std::max<int64_t>(n, 1), std::max<int64_t>(n, 1),
                  [&](int64_t a, int64_t b) { np = a; nf = b; });
    *out_n_pivots = np;
    *out_n_followers = nf;
    return RNSM_OK;
}

// Pivot selection on the device over reverse lists (off, ids) of n vertices
// and their forward lists (f_ids with CSR offsets f_off, or f_off NULL:
// fixed stride fk, -1 padded, as N_k): rounds of the parallel rule until
// every vertex is covered (the host checks after every `batch` rounds).
// pivot_of receives -1 for pivots, else the pivot. Workspace buffers; the
// caller holds g_lock.
static rnsm_status select_on_device(Workspace& ws, int64_t n, const int64_t* off,
                                    const int32_t* ids, int64_t nnz_bound, const int32_t* f_ids,
                                    const int64_t* f_off, int fk, int32_t* pivot_of, hipStream_t st,
                                    int64_t* n_pivots, int batch = 8, int64_t* rounds = nullptr) {
    // (a gain word holds coverage too: n < 2^30 keeps it from wrapping)
    if (n >= (int64_t)1 << 30) return fail(RNSM_EINVAL, "pivot selection: n >= 2^30");
    unsigned char* lose;
    int32_t* gain;
    int64_t *ctl, *h_ctl;
    WS(lose, "sel_lose", n);
    WS(gain, "sel_gain", sizeof(int32_t) * n);
    WS(ctl, "sel_ctl", sizeof(int64_t) * 8);
    HS(h_ctl, "h_sel_ctl", sizeof(int64_t) * 8);
    int32_t *act_a, *act_b;
    WS(act_a, "sel_act_a", sizeof(int32_t) * std::max<int64_t>(n, 1));
    WS(act_b, "sel_act_b", sizeof(int32_t) * std::max<int64_t>(n, 1));
    // a round's items: every pick's list in chunks of 16 entries
    int64_t* items;
    WS(items, "sel_items", sizeof(int64_t) * (n + nnz_bound / 16 + 1));
    HIPCHK(launch_select_init(n, off, lose, gain, pivot_of, ctl, st));
    // every round with uncovered vertices picks at least the one with the
    // largest key; after each check batch the rounds run over the vertices
    // still uncovered only
    const int32_t* act = nullptr;
    int64_t nact = n;
    int64_t tail_max = SELECT_TAIL_MAX;
    if (const char* c = getenv("RNSM_SELECT_TAIL")) tail_max = atoll(c);
    for (int64_t done = 0; done <= n + batch; done += batch) {
        HIPCHK(launch_select_rounds(n, act, nact, off, ids, f_ids, f_off, fk, lose, gain, pivot_of,
                                    items, ctl, batch, st));
        int32_t* act_next = act == act_a ? act_b : act_a;
        HIPCHK(launch_select_compact(act, nact, gain, act_next, ctl, st));
        HIPCHK(hipMemcpyAsync(h_ctl, ctl, sizeof(int64_t) * 6, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (h_ctl[4] == 0) {
            *n_pivots = h_ctl[1];
            if (rounds) *rounds = h_ctl[2];
            return RNSM_OK;
        }
        if (h_ctl[0] == 0 || h_ctl[4] < 0 || h_ctl[4] > nact)
            return fail(RNSM_EINTERNAL, "pivot selection: inconsistent active counts");
        act = act_next;
        nact = h_ctl[4];
        if (nact <= tail_max) {
            // the last rounds in one workgroup: no launch per round
            HIPCHK(launch_select_tail(n, act, nact, off, ids, f_ids, f_off, fk, lose, gain, pivot_of,
                                      items, ctl, st));
            int32_t* act_fin = act == act_a ? act_b : act_a;
            HIPCHK(launch_select_compact(act, nact, gain, act_fin, ctl, st));
            HIPCHK(hipMemcpyAsync(h_ctl, ctl, sizeof(int64_t) * 6, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (h_ctl[4] != 0)
                return fail(RNSM_EINTERNAL, "pivot selection: vertices left after the last rounds");
            *n_pivots = h_ctl[1];
            if (rounds) *rounds = h_ctl[2];
            return RNSM_OK;
        }
    }
    return fail(RNSM_EINTERNAL, "pivot selection did not cover every vertex");
}

static rnsm_status rnsm_select_pivots_device_impl(int64_t n, const int64_t* rk_offsets,
                                                  const int32_t* rk_ids, int32_t* pivot_of,
                                                  int64_t* out_n_pivots, void* stream) {
    g_err.clear();
    if (n < 0 || n >= ((int64_t)1 << 30))
        return fail(RNSM_EINVAL, "rnsm_select_pivots_device: n out of range (0 <= n < 2^30)");
    if (!out_n_pivots || (n > 0 && (!rk_offsets || !rk_ids || !pivot_of)))
        return fail(RNSM_EINVAL, "rnsm_select_pivots_device: NULL pointer");
    *out_n_pivots = 0;
    if (n == 0) return RNSM_OK;
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    Workspace& ws = g_ws[dev];
    ws.begin_call(0);
    int *flag, hflag = 0;
    WS(flag, "sel_check", sizeof(int));
    HIPCHK(launch_zero(flag, sizeof(int), st));
    HIPCHK(launch_check_lists(n, rk_offsets, rk_ids, flag, st));
    HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hflag)
        return fail(RNSM_EINVAL, "rnsm_select_pivots_device: malformed lists (offsets, an id out "
                    "of range or a list naming its owner)");
    // forward lists of the caller's reverse lists
    int32_t *fcnt, *fcur, *f_ids;
    int64_t *f_off, *stmp;
    int64_t nnz = 0;
    HIPCHK(hipMemcpyAsync(&nnz, rk_offsets + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    WS(fcnt, "sel_fcnt", sizeof(int32_t) * n);
    WS(fcur, "sel_fcur", sizeof(int32_t) * n);
    WS(f_off, "sel_foff", sizeof(int64_t) * (n + 1));
    WS(f_ids, "sel_fids", sizeof(int32_t) * std::max<int64_t>(nnz, 1));
    WS(stmp, "sel_scan", sizeof(int64_t) * scan_tmp_elems(n));
    HIPCHK(launch_select_forward(n, rk_offsets, rk_ids, fcnt, fcur, f_off, f_ids, stmp, st));
    int batch = 8;
    if (const char* c = getenv("RNSM_SELECT_BATCH")) batch = std::max(1, atoi(c));
    return select_on_device(ws, n, rk_offsets, rk_ids, nnz, f_ids, f_off, 0, pivot_of, st,
                            out_n_pivots, batch);
}

static rnsm_status tune_shape_locked(const rnsm_graph* g, const rnsm_vectors* base,
                                     const VecInfo& vi, int32_t ef, rnsm_metric metric,
                                     int64_t n_sample, int maxdeg, rnsm_search_tuning* out,
                                     hipStream_t st);

// shapes picked by the merge's own tuning (RNSM_FLAG_AUTOTUNE), per device,
// storage type, row bytes, beam, degree bound, metric and log2 of the
// largest sub-index; guarded by g_lock
static std::map<std::array<int64_t, 7>, std::pair<int, int>> g_tuned;

static rnsm_status rnsm_merge_impl(int32_t m, const rnsm_graph* graphs, const rnsm_vectors* vecs,
                       const rnsm_params* p, rnsm_csr* out) {
    const auto t0 = std::chrono::steady_clock::now();
    g_err.clear();
    memset(&g_stats, 0, sizeof g_stats);
    // ---------------------------------------------------- host argument checks
    if (m < 2) return fail(RNSM_EINVAL, "rnsm_merge: m = %d < 2", m);
    if (!graphs || !vecs || !p || !out) return fail(RNSM_EINVAL, "rnsm_merge: NULL argument");
    const bool host_out = (p->flags & RNSM_FLAG_HOST_OUT) != 0;
    if (!host_out && (!out->offsets || !out->nbrs))
        return fail(RNSM_EINVAL, "rnsm_merge: NULL output buffer");
    if (p->max_device_bytes < 0) return fail(RNSM_EINVAL, "rnsm_merge: max_device_bytes < 0");
    const int R = p->R;
    if (R < 1 || R > 64) return fail(RNSM_EINVAL, "rnsm_merge: R = %d outside 1..64", R);
    if (p->L < 1 || p->L > 128) return fail(RNSM_EINVAL, "rnsm_merge: L = %d outside 1..128", p->L);
    if (!(p->alpha >= 1.0f) || !std::isfinite(p->alpha))
        return fail(RNSM_EINVAL, "rnsm_merge: alpha must be finite and >= 1");
    if (p->metric < RNSM_L2SQ || p->metric > RNSM_COSINE)
        return fail(RNSM_EINVAL, "rnsm_merge: unknown metric %d", (int)p->metric);
    if (p->prune_rule < RNSM_PRUNE_ALPHA || p->prune_rule > RNSM_PRUNE_TAU)
        return fail(RNSM_EINVAL, "rnsm_merge: unknown prune_rule %d", (int)p->prune_rule);
    if (p->prune_rule != RNSM_PRUNE_ALPHA && p->metric != RNSM_L2SQ)
        return fail(RNSM_EINVAL, "rnsm_merge: the angle and tau rules take squared L2");
    if (p->prune_rule == RNSM_PRUNE_ANGLE && !(p->prune_param > 0.0f && p->prune_param <= 90.0f))
        return fail(RNSM_EINVAL, "rnsm_merge: prune_param (theta) outside (0, 90] degrees");
    if (p->prune_rule == RNSM_PRUNE_TAU && !(p->prune_param >= 0.0f && std::isfinite(p->prune_param)))
        return fail(RNSM_EINVAL, "rnsm_merge: prune_param (tau) must be finite and >= 0");
    // the rule's constant, formed once in double
    const double rule_a = p->prune_rule == RNSM_PRUNE_ANGLE
                              ? cos((double)p->prune_param * (3.14159265358979323846 / 180.0))
                              : 3.0 * (double)p->prune_param;
    const int k = p->k_reverse ? p->k_reverse : 5;
    const int kp = p->k_expand ? p->k_expand : 16;
    if (k < 1 || kp < k || kp > 64)
        return fail(RNSM_EINVAL, "rnsm_merge: need 1 <= k_reverse <= k_expand <= 64 (got %d, %d)", k, kp);
    const int efN = p->ef_naive ? p->ef_naive : p->L;
    const int efS = p->ef_slide ? p->ef_slide : p->L;
    if (efN < 1 || efN > 128 || efS < 1 || efS > 128)
        return fail(RNSM_EINVAL, "rnsm_merge: ef_naive / ef_slide outside 1..128");
    const int diam = p->mos_diameter ? p->mos_diameter : 2;
    if (diam < 2) return fail(RNSM_EINVAL, "rnsm_merge: mos_diameter < 2");
    int rmos = p->mos_degree;
    if (rmos < 0) return fail(RNSM_EINVAL, "rnsm_merge: mos_degree < 0");
    int hb_req = p->search_hash_bits, wpb_req = p->search_waves_per_block;
    if (hb_req != 0 && (hb_req < TUNE_HB_MIN || hb_req > TUNE_HB_MAX))
        return fail(RNSM_EINVAL, "rnsm_merge: search_hash_bits = %d outside %d..%d", hb_req,
                    TUNE_HB_MIN, TUNE_HB_MAX);
    if (wpb_req < 0 || wpb_req > 4)
        return fail(RNSM_EINVAL, "rnsm_merge: search_waves_per_block = %d outside 0..4", wpb_req);
    if (rmos == 0) rmos = std::max(2, (int)std::ceil(std::sqrt((double)m)));
    VecInfo vi;
    rnsm_status vs = vec_info(vecs, vi);
    if (vs != RNSM_OK) return vs;
    std::vector<int64_t> sizes(m), bases(m);
    int64_t N = 0;
    for (int i = 0; i < m; ++i) {
        const rnsm_graph& g = graphs[i];
        if (g.n < 1) return fail(RNSM_EINVAL, "rnsm_merge: sub-index %d is empty", i);
        // nbrs may be NULL for a sub-index without edges (checked with nnz below)
        if (!g.offsets) return fail(RNSM_EINVAL, "rnsm_merge: sub-index %d has a NULL CSR pointer", i);
        if (g.entry < 0 || g.entry >= g.n)
            return fail(RNSM_EINVAL, "rnsm_merge: entry %d of sub-index %d out of range", g.entry, i);
        sizes[i] = g.n;
        bases[i] = N;
        N += g.n;
    }
    if (N != vecs->n) return fail(RNSM_EINVAL, "rnsm_merge: vectors hold %lld rows, graphs %lld",
                                  (long long)vecs->n, (long long)N);
    if (N >= (1ll << 31) - 1) return fail(RNSM_EUNSUPPORTED, "rnsm_merge: more than 2^31-2 vertices");

    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)p->stream;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    Workspace& ws = g_ws[dev];
    ws.begin_call(p->max_device_bytes);
    Events E;
    E.no_stats = (p->flags & RNSM_FLAG_NO_STATS) != 0;

    // ------------------------------------------------------ input staging
    // host or strided inputs to packed device buffers; from here on the
    // graphs and vectors are device memory
    std::vector<rnsm_graph> gstaged(m);
    for (int i = 0; i < m; ++i) {
        const rnsm_status ss = stage_graph(ws, "rnsm_merge", i, graphs[i], st, gstaged[i]);
        if (ss != RNSM_OK) return ss;
    }
    rnsm_vectors vstaged;
    {
        const rnsm_status ss = stage_vectors(ws, "rnsm_merge", *vecs, st, vstaged);
        if (ss != RNSM_OK) return ss;
    }
    graphs = gstaged.data();
    vecs = &vstaged;
    {
        const rnsm_status ss = vec_info(vecs, vi);
        if (ss != RNSM_OK) return ss;
    }

    // ------------------------------------------------ input graph validation
    int* vflags;
    WS(vflags, "vflags", sizeof(int) * m);
    HIPCHK(hipMemsetAsync(vflags, 0, sizeof(int) * m, st));
    std::vector<int64_t> nnz(m), first(m);
    for (int i = 0; i < m; ++i) {
        HIPCHK(hipMemcpyAsync(&first[i], graphs[i].offsets, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(&nnz[i], graphs[i].offsets + graphs[i].n, sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < m; ++i) {
        if (first[i] != 0 || nnz[i] < 0)
            return fail(RNSM_EINVAL, "rnsm_merge: sub-index %d: offsets[0] != 0 or offsets[n] < 0", i);
        if (nnz[i] > 0 && !graphs[i].nbrs)
            return fail(RNSM_EINVAL, "rnsm_merge: sub-index %d has a NULL CSR pointer", i);
        HIPCHK(launch_validate(graphs[i].offsets, graphs[i].nbrs, graphs[i].n, nnz[i], R, vflags + i, st));
    }
    std::vector<int> hflags(m);
    HIPCHK(hipMemcpyAsync(hflags.data(), vflags, sizeof(int) * m, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < m; ++i) {
        const int f = hflags[i];
        if (f & 1) return fail(RNSM_EINVAL, "rnsm_merge: sub-index %d: offsets not non-decreasing", i);
        if (f & 4) return fail(RNSM_EINVAL, "rnsm_merge: sub-index %d: neighbour id out of range", i);
        if (f & 8) return fail(RNSM_EINVAL, "rnsm_merge: sub-index %d: self-loop", i);
        if (f & 16) return fail(RNSM_EINVAL, "rnsm_merge: sub-index %d: duplicate neighbour", i);
        if (f & 2) return fail(RNSM_EINVAL, "rnsm_merge: sub-index %d: degree above R = %d", i, R);
    }
    // the merge's own search-shape tuning: once per kind of input, on the
    // largest sub-index (its own rows as queries, beam ef_naive), unless the
    // caller fixed the shape
    if ((p->flags & RNSM_FLAG_AUTOTUNE) && hb_req == 0 && wpb_req == 0) {
        int big = 0;
        for (int i = 1; i < m; ++i)
            if (sizes[i] > sizes[big]) big = i;
        const std::array<int64_t, 7> key = {dev, vi.tt, vi.row_bytes, efN, R, (int64_t)p->metric,
                                            (int64_t)ilog2_ceil(sizes[big])};
        auto it = g_tuned.find(key);
        if (it == g_tuned.end()) {
            rnsm_vectors vb = *vecs;
            vb.n = sizes[big];
            vb.f32 = vecs->f32 + bases[big] * vecs->dim;
            if (vecs->search_dtype != RNSM_F32)
                vb.search = (const char*)vecs->search + bases[big] * vi.row_bytes;
            VecInfo vib;  // the same layout, rows of sub-index `big`
            rnsm_status ts = vec_info(&vb, vib);
            if (ts != RNSM_OK) return ts;
            rnsm_search_tuning tr;
            ts = tune_shape_locked(&graphs[big], &vb, vib, efN, p->metric, 65536, R, &tr, st);
            if (ts != RNSM_OK) return ts;
            it = g_tuned.emplace(key, std::make_pair((int)tr.hash_bits, (int)tr.waves_per_block)).first;
        }
        hb_req = it->second.first;
        wpb_req = it->second.second;
    }

    // ----------------------------------------------------------------- plan
    const auto tp = std::chrono::steady_clock::now();
    std::vector<std::pair<int, int>> ops;
    int fallbacks = 0;
    std::vector<double> cent;
    if (p->flags & RNSM_FLAG_CENTROID_COSTS) {
        // centroids in float64, summed on the device
        double* cs;
        unsigned long long* csi;
        int* flag;
        u64* bb;
        WS(cs, "centroid_sums", sizeof(double) * vecs->dim);
        WS(csi, "centroid_isums", sizeof(unsigned long long) * vecs->dim);
        WS(flag, "centroid_flag", sizeof(int));
        WS(bb, "entry_best", sizeof(u64) * 3 * entry_blocks(1));
        cent.assign((size_t)m * vecs->dim, 0.0);
        for (int i = 0; i < m; ++i) {
            const int one = 0;  // force the float64 path
            HIPCHK(hipMemcpyAsync(flag, &one, sizeof(int), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemsetAsync(cs, 0, sizeof(double) * vecs->dim, st));
            HIPCHK(launch_entry(vecs->f32 + bases[i] * vecs->dim, sizes[i], vecs->dim, flag, cs, csi,
                                nullptr, 0, st));
            HIPCHK(hipMemcpyAsync(cent.data() + (size_t)i * vecs->dim, cs, sizeof(double) * vecs->dim,
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int t = 0; t < vecs->dim; ++t) cent[(size_t)i * vecs->dim + t] /= (double)sizes[i];
        }
    }
    if (plan_ops(m, sizes.data(), cent.empty() ? nullptr : cent.data(), vecs->dim, rmos, diam, ops,
                 &fallbacks) != 0)
        return fail(RNSM_EINTERNAL, "rnsm_merge: planner failed");
    double ms_plan = ms_since(tp);

    // ------------------------------------------------------------ workspace
    // Order of the set-up: the padded adjacency first, so that the first
    // operation's breadth-first order (side stream, host-paced levels) runs
    // while this stream makes the value summary, row copies, norms and the
    // bfloat16 copy; the summary is read after that.
    int32_t *rows, *deg, *errf;
    float *rdist, *norms = nullptr;
    double* norms64 = nullptr;  // inner product and cosine: for the stored distances
    u64* cnt;
    WS(rows, "rows", sizeof(int32_t) * N * R);
    WS(deg, "deg", sizeof(int32_t) * N);
    WS(rdist, "rdist", sizeof(float) * N * R);
    WS(cnt, "counters", sizeof(u64) * 3 * CNT_SLOTS * CNT_N);
    WS(errf, "errf", sizeof(int));
    // padded adjacency of every input graph (rows of R ids, -1 filled): the
    // searches read a vertex's neighbours with one load, no offsets lookup
    int32_t* padj;
    WS(padj, "padj", sizeof(int32_t) * N * R);
    for (int i = 0; i < m; ++i)
        HIPCHK(launch_pad_adjacency(graphs[i].offsets, graphs[i].nbrs, graphs[i].n, R,
                                    padj + bases[i] * R, st));
    int ev_padj;
    HIPCHK(E.record(st, &ev_padj));
    // value summary, read once the breadth-first order is done
    unsigned *vr, *h_vr;
    WS(vr, "value_range", sizeof(unsigned) * 3);
    HS(h_vr, "h_value_range", sizeof(unsigned) * 3);
    HIPCHK(launch_value_range(vecs->f32, N * vecs->dim, vr, st));
    HIPCHK(hipMemcpyAsync(h_vr, vr, sizeof(unsigned) * 3, hipMemcpyDeviceToHost, st));
    int ev_vr;
    HIPCHK(E.record(st, &ev_vr));
    // bfloat16 copy of the rows for an exact-mode prune (half the bytes for
    // its gathers), made before the summary says whether the rows are exact
    // in it; unused when they are not
    // (above dim 128 the copy is large: made only once the summary asks for it)
    char* xb16 = nullptr;
    if (prune_mfma_supported(vecs->dim) && vecs->dim <= 128 && R <= 64) {
        WS(xb16, "prune_bf16", (size_t)2 * N * vecs->dim);
        HIPCHK(launch_convert(vecs->f32, RNSM_F32, xb16, RNSM_BF16, N * vecs->dim, st));
    }
    u64* rechecks;
    WS(rechecks, "prune_rechecks", sizeof(u64) * CNT_SLOTS);
    HIPCHK(hipMemsetAsync(rechecks, 0, sizeof(u64) * CNT_SLOTS, st));
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(u64) * 3 * CNT_SLOTS * CNT_N, st));
    HIPCHK(hipMemsetAsync(errf, 0, sizeof(int), st));
    if (p->metric == RNSM_COSINE) {
        WS(norms, "norms", sizeof(float) * N);
        WS(norms64, "norms64", sizeof(double) * N);
        HIPCHK(launch_norms(vecs->f32, N, vecs->dim, norms, st, norms64));
    }
    for (int i = 0; i < m; ++i)
        HIPCHK(launch_init_rows(graphs[i].offsets, graphs[i].nbrs, graphs[i].n, bases[i], R, rows,
                                deg, rdist, st));
    // breadth-first order of a source graph from its entry: the expansion
    // runs its queries in that order, and pivot groups are launched by the
    // rank of their pivot in it (locality in L2 only)
    const bool use_bfs = !getenv("RNSM_NO_BFS_ORDER");
    const bool one_stream = getenv("RNSM_ONE_STREAM") && atoi(getenv("RNSM_ONE_STREAM")) == 1;
    int32_t* h_bfs = nullptr;
    // (per_source: the batched form's order buffer of its own per source, no
    // host copy; the plain form's one buffer and its host copy otherwise)
    auto bfs_order_of = [&](int s, hipStream_t strm, int32_t** order_out, int* ev_out,
                            bool per_source = false) -> rnsm_status {
        const int64_t ns = sizes[s];
        int32_t* bfs_order;
        unsigned *bfs_vis, *bfs_tail, *h_tail;
        const std::string oname = per_source ? "bt_bfs_" + std::to_string(s) : "bfs_order";
        WS(bfs_order, oname, sizeof(int32_t) * ns);
        WS(bfs_vis, per_source ? "bt_bfs_visited" : "bfs_visited", sizeof(unsigned) * ((ns + 31) / 32));
        WS(bfs_tail, per_source ? "bt_bfs_ctl" : "bfs_ctl", 4 * sizeof(unsigned));
        HS(h_tail, per_source ? "h_bt_bfs_ctl" : "h_bfs_ctl", 4 * sizeof(unsigned));
        HIPCHK(launch_bfs_order(padj + bases[s] * R, R, ns, graphs[s].entry, bfs_vis, bfs_order,
                                bfs_tail, h_tail, strm));
        if (!per_source) {
            HS(h_bfs, "h_bfs_order", sizeof(int32_t) * ns);
            HIPCHK(hipMemcpyAsync(h_bfs, bfs_order, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, strm));
        } else {
            // the batched form keeps the order on the device: checked there
            // (the host reads the flag at the round's first synchronisation)
            int32_t* pcnt;
            int *pflag, *h_pflag;
            WS(pcnt, "bt_perm_cnt", sizeof(int32_t) * std::max<int64_t>(ns, 1));
            WS(pflag, "bt_perm_flag", sizeof(int) * m);
            HS(h_pflag, "h_bt_perm_flag", sizeof(int) * m);
            HIPCHK(launch_perm_check(bfs_order, ns, pcnt, pflag + s, strm));
            HIPCHK(hipMemcpyAsync(h_pflag + s, pflag + s, sizeof(int), hipMemcpyDeviceToHost, strm));
        }
        HIPCHK(E.record(strm, ev_out));
        *order_out = bfs_order;
        return RNSM_OK;
    };
    hipStream_t sd;
    HIPCHK(ws.side_stream(&sd));
    int32_t* bfs0 = nullptr;
    int ev_bfs0 = -1;
    const bool batched = (p->flags & RNSM_FLAG_BATCHED) != 0;
    const bool bfs_early = use_bfs && !batched && !ops.empty() &&
                           !(p->flags & RNSM_FLAG_ALL_PIVOTS) && sizes[ops[0].first] > 0;
    if (bfs_early) {
        HIPCHK(hipStreamWaitEvent(sd, E.ev[ev_padj], 0));
        const rnsm_status bs = bfs_order_of(ops[0].first, sd, &bfs0, &ev_bfs0);
        if (bs != RNSM_OK) return bs;
    }
    // the batched form: orders of the first round's sources (operations that
    // share no sub-index with an earlier one), made on the side stream during
    // the set-up as well
    std::vector<int> bt_ev_bfs(m, -1), bt_ev_bfs0(m, -1);
    std::vector<int32_t*> bt_bfs(m, nullptr);
    if (batched && use_bfs && !(p->flags & RNSM_FLAG_ALL_PIVOTS)) {
        HIPCHK(hipStreamWaitEvent(sd, E.ev[ev_padj], 0));
        std::vector<char> used(m, 0);
        for (size_t a1 = 0; a1 < ops.size(); ++a1) {
            const int s = ops[a1].first, t = ops[a1].second;
            const bool first_round = !used[s] && !used[t];
            used[s] = used[t] = 1;
            if (!first_round || sizes[s] == 0 || bt_bfs[s]) continue;
            HIPCHK(E.stat(sd, &bt_ev_bfs0[s]));
            const rnsm_status bs = bfs_order_of(s, sd, &bt_bfs[s], &bt_ev_bfs[s], true);
            if (bs != RNSM_OK) return bs;
        }
    }
    ValueInfo vinfo;
    HIPCHK(hipEventSynchronize(E.ev[ev_vr]));
    decode_value_range(h_vr, &vinfo);
    // the angle and tau rules run on the float32 walk
    const int pmode = p->prune_rule != RNSM_PRUNE_ALPHA ? 0 : choose_prune(vinfo, vecs->dim, R);
    if (pmode != 1) xb16 = nullptr;
    if (pmode == 1 && !xb16) {
        WS(xb16, "prune_bf16", (size_t)2 * N * vecs->dim);
        HIPCHK(launch_convert(vecs->f32, RNSM_F32, xb16, RNSM_BF16, N * vecs->dim, st));
    }
    const double band = prune_band();
    // search distances usable as prune keys: a float32 copy computes them
    // with the prune's own lane layout and order; a 16-bit copy only when
    // every distance is exact (integers exact in that type, exact sums)
    const bool search_d_exact =
        vi.tt == 0 || int_exact(vinfo, vecs->dim, vi.tt == 1 ? 256.0 : 2048.0);


    // ------------------------------------------------------- the operations
    // Per operation (source s into target t): neighbour expansion of s in
    // its own graph and the reverse k-NN lists (device); R_k to the host and
    // the lazy greedy there. The greedy hands over pivot groups in chunks;
    // each chunk's naive search (pivots) and local sliding (their followers)
    // are queued at once, so the device searches while the host is still
    // selecting. Then source prune, reverse edges and target prune.
    const int RES = std::max(efN, efS);
    double ms_prune = 0.0;
    std::vector<int> last_use(m, -1);
    for (size_t oi = 0; oi < ops.size(); ++oi) last_use[ops[oi].first] = (int)oi;
    std::vector<std::vector<int32_t>> cached(m);  // lists of a source used again later
    std::vector<int64_t> cached_np(m, 0), cached_nf(m, 0);
    std::vector<std::array<int, 3>> ev_exp;
    std::vector<std::array<int, 4>> ev_chunk;
    std::vector<std::array<int, 2>> ev_span;  // first / last chunk of each operation
    std::vector<std::array<int, 2>> ev_prune;
    int64_t* h_nrev;
    HS(h_nrev, "h_nrev", sizeof(int64_t) * ops.size());
    GainLevels& levels = ws.levels;
    std::vector<char> touched(m, 0);  // rows changed by an earlier operation
    std::vector<int32_t> rank, fbeg, fcnt;
    std::vector<uint64_t> rbits;

    // The batched form (RNSM_FLAG_BATCHED). Operations run in rounds: an
    // operation's round is one past the last earlier operation sharing a
    // sub-index with it, so the operations of a round touch disjoint rows and
    // commute. Per round: for each source not prepared yet, neighbour
    // expansion, reverse inversion, pivot selection on the device (the same
    // pivots and groups as the host greedy) and its pivot groups in
    // breadth-first order; then one persistent launch searches every group of
    // every operation of the round (k_group_search); then each operation's
    // source prune, reverse edges and target prune, as in the plain form.
    std::vector<std::array<int, 4>> ev_rounds;  // group search start / end, overflow end, prunes end
    std::vector<std::array<int, 3>> sel_ev;     // selection start, groups start, groups end
    std::vector<std::array<int, 2>> ord_ev;     // breadth-first order start / end
    int64_t n_rounds_b = 0;
    auto batched_ops = [&]() -> rnsm_status {
        const int nops = (int)ops.size();
        std::vector<int> round_of(nops, 0);
        int nrounds = 0;
        for (int a1 = 0; a1 < nops; ++a1) {
            for (int b1 = 0; b1 < a1; ++b1) {
                const bool share = ops[a1].first == ops[b1].first || ops[a1].first == ops[b1].second ||
                                   ops[a1].second == ops[b1].first || ops[a1].second == ops[b1].second;
                if (share) round_of[a1] = std::max(round_of[a1], round_of[b1] + 1);
            }
            nrounds = std::max(nrounds, round_of[a1] + 1);
        }
        n_rounds_b = nrounds;
        const bool all_piv = (p->flags & RNSM_FLAG_ALL_PIVOTS) != 0;
        std::vector<char> prepared(m, 0);
        std::vector<int64_t> src_np(m, 0), src_nf(m, 0);
        int64_t* gstmp;
        WS(gstmp, "bt_scan_tmp", sizeof(int64_t) * scan_tmp_elems(N));
        // followers per group work item; the rest of a larger group (a hub's
        // reverse list can hold thousands) goes to a plain sliding launch
        // after the group search, so no wavefront runs a long serial tail
        int64_t fmax = 2;  // measured fastest of 2..32 on 2 x 500,000 (dim 128)
        if (const char* c = getenv("RNSM_GROUP_FMAX")) fmax = std::max(1ll, atoll(c));
        int64_t* h_novf;
        HS(h_novf, "h_bt_novf", sizeof(int64_t) * m);
        // rounds of the pivot selection between the host's checks
        int select_batch = 16;
        if (const char* c = getenv("RNSM_SELECT_BATCH")) select_batch = std::max(1, atoi(c));
        // per-source buffers (a source's groups are read by a later round too)
        auto src_buf = [&](const char* what, int s2, size_t bytes, void** out) -> rnsm_status {
            HIPCHK(ws.get(std::string(what) + std::to_string(s2), bytes, out));
            return RNSM_OK;
        };
        int op_slot = 0;
        for (int rr = 0; rr < nrounds; ++rr) {
            std::vector<int> rops;
            for (int oi = 0; oi < nops; ++oi)
                if (round_of[oi] == rr) rops.push_back(oi);
            // ---- the round's untouched targets: their rows' distances (the
            // target prunes read them) on the side stream, queued once the
            // round's first expansion search is (so that they run beside the
            // selection's small kernels, not against the search)
            int ev_rd = -1;
            bool rd_queued = false;
            auto queue_row_dists = [&]() -> rnsm_status {
                if (rd_queued) return RNSM_OK;
                rd_queued = true;
                int ev_go = -1;
                for (int oi : rops) {
                    const int t = ops[oi].second;
                    if (touched[t]) continue;
                    if (ev_go < 0) {
                        HIPCHK(E.record(st, &ev_go));
                        HIPCHK(hipStreamWaitEvent(sd, E.ev[ev_go], 0));
                    }
                    PruneArgs rd = {};
                    rd.X = vecs->f32;
                    rd.xb = xb16;
                    rd.n_total = N;
                    rd.nch = vi.nch32;
                    rd.G = vi.G32;
                    rd.lgG = ilog2i(vi.G32);
                    rd.cpl = vi.cpl32;
                    rd.metric = p->metric;
                    rd.norms = norms;
                    rd.n_items = sizes[t];
                    rd.item_base = bases[t];
                    rd.rows_in = rows;
                    rd.deg_in = deg;
                    rd.rows_d = rdist;
                    rd.R = R;
                    rd.wcap = TARGET_WCAP;
                    rd.err = errf;
                    rd.band = band;
                    rd.rechecks = rechecks;
                    // two blocks a compute unit: the selection's kernels and
                    // the group search run beside it
                    rd.grid_cap = 512;
                    HIPCHK(launch_row_dists(rd, prune_reads_b16(rd, pmode), sd));
                }
                if (ev_go >= 0) HIPCHK(E.record(sd, &ev_rd));
                return RNSM_OK;
            };
            // ---- sources of the round: expansion, inversion, selection, groups
            int ev_novf = -1;
            for (int oi : rops) {
                const int s = ops[oi].first;
                if (prepared[s]) continue;
                const int64_t ns = sizes[s];
                int32_t *pivot_of, *gpiv, *fbeg_d, *fol, *porder;
                int64_t* fbeg64;
                rnsm_status rs;
                if ((rs = src_buf("bt_pivot_of_", s, sizeof(int32_t) * ns, (void**)&pivot_of)) != RNSM_OK) return rs;
                if ((rs = src_buf("bt_gpiv_", s, sizeof(int32_t) * ns, (void**)&gpiv)) != RNSM_OK) return rs;
                if ((rs = src_buf("bt_fbeg_", s, sizeof(int64_t) * (ns + 1), (void**)&fbeg64)) != RNSM_OK) return rs;
                if ((rs = src_buf("bt_fol_", s, sizeof(int32_t) * ns, (void**)&fol)) != RNSM_OK) return rs;
                if ((rs = src_buf("bt_order_", s, sizeof(int32_t) * ns, (void**)&porder)) != RNSM_OK) return rs;
                (void)fbeg_d;
                int32_t* bfs_order = nullptr;
                if (bt_bfs[s]) {  // made on the side stream during the set-up
                    bfs_order = bt_bfs[s];
                    HIPCHK(hipStreamWaitEvent(st, E.ev[bt_ev_bfs[s]], 0));
                    ord_ev.push_back({bt_ev_bfs0[s], bt_ev_bfs[s]});
                } else if (use_bfs && !all_piv) {
                    int ev_a = -1, ev_b = -1;
                    HIPCHK(E.stat(st, &ev_a));
                    const rnsm_status bs = bfs_order_of(s, st, &bfs_order, &ev_b, true);
                    if (bs != RNSM_OK) return bs;
                    ord_ev.push_back({ev_a, ev_b});
                }
                int64_t np = ns;
                int ev_sel0 = -1;
                if (all_piv) {
                    HIPCHK(launch_fill32(pivot_of, ns, -1, st));
                } else {
                    int32_t *nk, *rcnt, *rk_ids;
                    int64_t *rk_off, *stmp;
                    WS(nk, "nk", sizeof(int32_t) * ns * k);
                    WS(rcnt, "rk_cnt", sizeof(int32_t) * ns);
                    WS(rk_off, "rk_off", sizeof(int64_t) * (ns + 1));
                    WS(rk_ids, "rk_ids", sizeof(int32_t) * std::max<int64_t>(ns * k, 1));
                    WS(stmp, "scan_tmp", sizeof(int64_t) * scan_tmp_elems(ns));
                    std::array<int, 3> ex;
                    HIPCHK(E.stat(st, &ex[0]));
                    SearchArgs a = {};
                    a.base = vi.search + bases[s] * vi.row_bytes;
                    a.nch = vi.nch;
                    a.row_bytes = vi.row_bytes;
                    a.offs = graphs[s].offsets;
                    a.nbrs = graphs[s].nbrs;
                    a.padj = padj + bases[s] * R;
                    a.rp = R;
                    a.n = ns;
                    a.qvec = a.base;
                    a.qidx = bfs_order;
                    a.out_row = bfs_order;
                    a.nq = ns;
                    a.seed_mode = 1;
                    a.metric = p->metric;
                    a.base_norm = norms ? norms + bases[s] : nullptr;
                    a.q_norm = a.base_norm;
                    a.ef = kp;
                    a.G = vi.G;
                    a.lgG = ilog2i(vi.G);
                    a.cpl = vi.cpl;
                    const SearchShape sh = search_shape(kp, R, ns, vi.tt, hb_req, wpb_req);
                    a.hbits = sh.hbits;
                    a.hash_mode = sh.mode;
                    a.out_mode = 1;
                    a.out_ids = nk;
                    a.out_stride = k;
                    a.out_k = k;
                    a.counters = cnt + 0 * CNT_SLOTS * CNT_N;
                    a.err = errf;
                    if (!touched[s] && search_d_exact) {
                        a.row_d = rdist;
                        a.row_d_base = bases[s];
                        a.row_d_stride = R;
                    }
                    HIPCHK(launch_search(vi.tt, a, sh.wpb, st));
                    HIPCHK(E.stat(st, &ex[1]));
                    HIPCHK(launch_count_ids(nk, ns, k, rcnt, st));
                    HIPCHK(launch_invert_lists(nk, ns, k, rcnt, rk_off, rk_ids, stmp, st));
                    HIPCHK(E.stat(st, &ex[2]));
                    ev_exp.push_back(ex);
                    g_stats.queries[0] += ns;
                    g_stats.launches[0] += 1;
                    if ((rs = queue_row_dists()) != RNSM_OK) return rs;
                    int64_t nrs = 0;
                    HIPCHK(E.stat(st, &ev_sel0));
                    const rnsm_status ss = select_on_device(ws, ns, rk_off, rk_ids, ns * k, nk,
                                                            nullptr, k, pivot_of, st, &np,
                                                            select_batch, &nrs);
                    if (ss != RNSM_OK) return ss;
                    g_stats.select_rounds += nrs;
                }
                int ev_sel1 = -1;
                HIPCHK(E.stat(st, &ev_sel1));
                int32_t *gflag, *group_of, *gcnt;
                int64_t* gpos;
                WS(gflag, "bt_flag", sizeof(int32_t) * ns);
                WS(gpos, "bt_gpos", sizeof(int64_t) * (ns + 1));
                WS(group_of, "bt_group_of", sizeof(int32_t) * ns);
                WS(gcnt, "bt_gcnt", sizeof(int32_t) * std::max<int64_t>(np, 1));
                HIPCHK(launch_groups(bfs_order, ns, pivot_of, gflag, gpos, gpiv, group_of, gcnt,
                                     fbeg64, fol, porder, gstmp, np, st));
                int32_t *ofl, *oflp;
                int64_t* ooff;
                if ((rs = src_buf("bt_ofl_", s, sizeof(int32_t) * ns, (void**)&ofl)) != RNSM_OK) return rs;
                if ((rs = src_buf("bt_oflp_", s, sizeof(int32_t) * ns, (void**)&oflp)) != RNSM_OK) return rs;
                if ((rs = src_buf("bt_ooff_", s, sizeof(int64_t) * (np + 1), (void**)&ooff)) != RNSM_OK) return rs;
                HIPCHK(launch_group_overflow(np, ns - np, gpiv, fbeg64, fol, pivot_of, group_of, fmax,
                                             gcnt, ooff, ofl, oflp, gstmp, st));
                HIPCHK(hipMemcpyAsync(h_novf + s, ooff + np, sizeof(int64_t), hipMemcpyDeviceToHost, st));
                HIPCHK(E.record(st, &ev_novf));
                sel_ev.push_back({ev_sel0, ev_sel1, ev_novf});
                src_np[s] = np;
                src_nf[s] = ns - np;
                prepared[s] = 1;
            }
            {  // (a round whose sources were all prepared earlier)
                const rnsm_status rs = queue_row_dists();
                if (rs != RNSM_OK) return rs;
            }
            // ---- one persistent search over the round's pivot groups
            std::vector<GroupOp> gops;
            int64_t total_groups = 0;
            int hb_max = 0, mode_max = 0, wpb_min = 4;
            for (int oi : rops) {
                const int s = ops[oi].first, t = ops[oi].second;
                const SearchShape a1 = search_shape(efN, R, sizes[t], vi.tt, hb_req, wpb_req);
                const SearchShape b1 = search_shape(efS, R, sizes[t], vi.tt, hb_req, wpb_req);
                mode_max = std::max({mode_max, a1.mode, b1.mode});
                hb_max = std::max({hb_max, a1.hbits, b1.hbits});
                wpb_min = std::min({wpb_min, a1.wpb, b1.wpb});
                (void)s;
            }
            if (mode_max) hb_max = 13;
            while (wpb_min > 1 && search_lds_bytes(hb_max, wpb_min) > 64 * 1024) --wpb_min;
            std::vector<int32_t*> res_of(rops.size());
            std::vector<float*> resd_of(rops.size());
            for (size_t q = 0; q < rops.size(); ++q) {
                const int oi = rops[q];
                const int s = ops[oi].first, t = ops[oi].second;
                const int64_t ns = sizes[s], nt = sizes[t];
                rnsm_status rs;
                int32_t *gpiv, *fol, *resq;
                int64_t* fbeg64;
                float* resdq;
                if ((rs = src_buf("bt_gpiv_", s, sizeof(int32_t) * ns, (void**)&gpiv)) != RNSM_OK) return rs;
                if ((rs = src_buf("bt_fbeg_", s, sizeof(int64_t) * (ns + 1), (void**)&fbeg64)) != RNSM_OK) return rs;
                if ((rs = src_buf("bt_fol_", s, sizeof(int32_t) * ns, (void**)&fol)) != RNSM_OK) return rs;
                if ((rs = src_buf("bt_res_", s, sizeof(int32_t) * ns * RES, (void**)&resq)) != RNSM_OK) return rs;
                if ((rs = src_buf("bt_resd_", s, sizeof(float) * ns * RES, (void**)&resdq)) != RNSM_OK) return rs;
                res_of[q] = resq;
                resd_of[q] = resdq;
                // beams shorter than RES leave -1 behind them for the prune
                HIPCHK(launch_fill32(resq, ns * RES, -1, st));
                GroupOp go = {};
                SearchArgs a = {};
                a.base = vi.search + bases[t] * vi.row_bytes;
                a.nch = vi.nch;
                a.row_bytes = vi.row_bytes;
                a.offs = graphs[t].offsets;
                a.nbrs = graphs[t].nbrs;
                a.padj = padj + bases[t] * R;
                a.rp = R;
                a.n = nt;
                a.qvec = vi.search + bases[s] * vi.row_bytes;
                a.metric = p->metric;
                a.base_norm = norms ? norms + bases[t] : nullptr;
                a.q_norm = norms ? norms + bases[s] : nullptr;
                a.G = vi.G;
                a.lgG = ilog2i(vi.G);
                a.cpl = vi.cpl;
                a.hbits = hb_max;
                a.hash_mode = mode_max;
                a.out_mode = 0;
                a.out_ids = resq;
                a.out_d = resdq;
                a.out_stride = RES;
                a.err = errf;
                go.naive = a;
                go.naive.seed_mode = 0;
                go.naive.entry = graphs[t].entry;
                go.naive.ef = efN;
                go.naive.out_k = efN;
                go.slide = a;
                go.slide.seed_mode = 2;
                go.slide.seed_ids = resq;
                go.slide.seed_stride = RES;
                go.slide.n_seeds = efN;
                go.slide.ef = efS;
                go.slide.out_k = efS;
                go.gpiv = gpiv;
                go.fbeg = fbeg64;
                go.fol = fol;
                go.group_base = total_groups;
                go.n_groups = src_np[s];
                total_groups += src_np[s];
                gops.push_back(go);
                g_stats.queries[1] += src_np[s];
                g_stats.queries[2] += src_nf[s];
            }
            // each round's op table in slots of its own: the stream may not
            // have copied an earlier round's table yet
            GroupOp *d_ops, *h_ops;
            unsigned* next;
            WS(d_ops, "bt_ops", sizeof(GroupOp) * nops);
            HS(h_ops, "h_bt_ops", sizeof(GroupOp) * nops);
            WS(next, "bt_next", sizeof(unsigned) * 8 * nrounds);
            d_ops += op_slot;
            h_ops += op_slot;
            next += 8 * rr;
            op_slot += (int)gops.size();
            memcpy(h_ops, gops.data(), sizeof(GroupOp) * gops.size());
            HIPCHK(hipMemcpyAsync(d_ops, h_ops, sizeof(GroupOp) * gops.size(), hipMemcpyHostToDevice, st));
            HIPCHK(launch_zero(next, sizeof(unsigned) * 8, st));
            GroupArgs ga = {};
            ga.ops = d_ops;
            ga.n_ops = (int)gops.size();
            ga.n_groups = total_groups;
            ga.next = next;
            ga.hbits = hb_max;
            ga.fmax = fmax;
            ga.counters = cnt + 1 * CNT_SLOTS * CNT_N;
            SearchArgs shape = gops[0].naive;
            shape.ef = std::max(efN, efS);
            std::array<int, 4> er;
            HIPCHK(E.stat(st, &er[0]));
            HIPCHK(launch_group_search(vi.tt, shape, ga, wpb_min, st, &g_stats.group_blocks));
            HIPCHK(E.stat(st, &er[1]));
            g_stats.launches[1] += 1;
            // the overflow followers, one wavefront each, seeded by their
            // pivot's beam (written by the group search)
            if (ev_novf >= 0) HIPCHK(hipEventSynchronize(E.ev[ev_novf]));
            if (use_bfs && !all_piv) {  // (the round's orders were made before ev_novf)
                int* h_pflag;
                HS(h_pflag, "h_bt_perm_flag", sizeof(int) * m);
                for (int oi : rops)
                    if (h_pflag[ops[oi].first])
                        return fail(RNSM_EINTERNAL, "rnsm_merge: breadth-first order is not a permutation");
            }
            for (size_t q = 0; q < rops.size(); ++q) {
                const int s = ops[rops[q]].first, t = ops[rops[q]].second;
                const int64_t novf = h_novf[s];
                if (novf <= 0) continue;
                int32_t *ofl, *oflp;
                rnsm_status rs;
                if ((rs = src_buf("bt_ofl_", s, sizeof(int32_t) * sizes[s], (void**)&ofl)) != RNSM_OK) return rs;
                if ((rs = src_buf("bt_oflp_", s, sizeof(int32_t) * sizes[s], (void**)&oflp)) != RNSM_OK) return rs;
                SearchArgs b = gops[q].slide;
                const SearchShape shB = search_shape(efS, R, sizes[t], vi.tt, hb_req, wpb_req);
                b.hbits = shB.hbits;
                b.hash_mode = shB.mode;
                b.qidx = ofl;
                b.out_row = ofl;
                b.seed_row = oflp;
                b.nq = novf;
                b.counters = cnt + 2 * CNT_SLOTS * CNT_N;
                HIPCHK(launch_search(vi.tt, b, shB.wpb, st));
                g_stats.launches[2] += 1;
                g_stats.group_overflow += novf;
            }
            HIPCHK(E.stat(st, &er[2]));
            g_stats.exact_visited = mode_max;
            g_stats.search_hash_bits = hb_max;
            g_stats.search_waves_per_block = wpb_min;
            // ---- the round's prunes and reverse edges, operation by operation
            if (ev_rd >= 0) HIPCHK(hipStreamWaitEvent(st, E.ev[ev_rd], 0));
            for (size_t q = 0; q < rops.size(); ++q) {
                const int oi = rops[q];
                const int s = ops[oi].first, t = ops[oi].second;
                const int64_t ns = sizes[s], nt = sizes[t];
                int32_t* porder;
                rnsm_status rs;
                if ((rs = src_buf("bt_order_", s, sizeof(int32_t) * ns, (void**)&porder)) != RNSM_OK) return rs;
                PruneArgs qs = {};
                qs.X = vecs->f32;
                qs.xb = xb16;
                qs.n_total = N;
                qs.nch = vi.nch32;
                qs.G = vi.G32;
                qs.lgG = ilog2i(vi.G32);
                qs.cpl = vi.cpl32;
                qs.metric = p->metric;
                qs.norms = norms;
                qs.item_base = bases[s];
                qs.rows_in = rows;
                qs.deg_in = deg;
                qs.rows_d = rdist;
                qs.extra_mode = 1;
                qs.extra_ids = res_of[q];
                qs.extra_d = search_d_exact ? resd_of[q] : nullptr;
                qs.extra_sorted = search_d_exact && RES <= 128;
                qs.extra_stride = RES;
                qs.extra_cnt = RES;
                qs.extra_index_base = bases[s];
                qs.extra_id_add = bases[t];
                qs.alpha = p->alpha;
                qs.rule = p->prune_rule;
                qs.rule_a = rule_a;
                qs.R = R;
                qs.rows_out = rows;
                qs.deg_out = deg;
                qs.dist_out = rdist;
                qs.wcap = R + RES;
                qs.err = errf;
                qs.band = band;
                qs.rechecks = rechecks;
                // (the untouched targets' row distances came from the side stream)
                int32_t *rc, *rcur, *rev;
                int64_t *roff, *stmp2;
                u64* scratch;
                float* rev_d;
                WS(rc, "rev_cnt", sizeof(int32_t) * nt);
                WS(rcur, "rev_cur", sizeof(int32_t) * nt);
                WS(roff, "rev_off", sizeof(int64_t) * (nt + 1));
                WS(rev, "rev_ids", sizeof(int32_t) * std::max<int64_t>(ns * R, 1));
                WS(rev_d, "rev_d", sizeof(float) * std::max<int64_t>(ns * R, 1));
                WS(stmp2, "scan_tmp2", sizeof(int64_t) * scan_tmp_elems(nt));
                WS(scratch, "prune_scratch", sizeof(u64) * 2 * (nt * R + ns * R));
                HIPCHK(launch_zero(rc, sizeof(int32_t) * nt, st));
                HIPCHK(launch_zero(rcur, sizeof(int32_t) * nt, st));
                PruneArgs q1 = qs;
                q1.items = porder;
                q1.n_items = ns;
                q1.rev_cnt = rc;
                q1.rev_lo = bases[t];
                q1.rev_n = nt;
                HIPCHK(run_prune(q1, pmode, st));
                HIPCHK(launch_scan(rc, nt, roff, stmp2, st));
                HIPCHK(launch_rev_scatter(rows, deg, rdist, bases[s], ns, R, bases[t], nt, roff, rcur,
                                          rev, rev_d, st));
                PruneArgs r2 = q1;
                r2.n_items = nt;
                r2.items = nullptr;
                r2.item_base = bases[t];
                r2.extra_mode = 2;
                r2.extra_ids = rev;
                r2.extra_d = rev_d;
                r2.extra_off = roff;
                r2.extra_index_base = bases[t];
                r2.extra_id_add = 0;
                r2.skip_empty_extra = 1;
                r2.extra_sorted = 0;
                r2.scratch = scratch;
                r2.wcap = TARGET_WCAP;
                r2.rev_cnt = nullptr;
                HIPCHK(run_prune(r2, pmode, st));
                HIPCHK(hipMemcpyAsync(h_nrev + oi, roff + nt, sizeof(int64_t), hipMemcpyDeviceToHost, st));
                g_stats.n_followers += src_nf[s];
                g_stats.n_pivots += src_np[s];
                g_stats.n_source_vertices += ns;
                touched[s] = touched[t] = 1;
            }
            HIPCHK(E.stat(st, &er[3]));
            ev_rounds.push_back(er);
            // the next round's groups overwrite nothing this round reads
            // (rows change only through the prunes above, on this stream)
        }
        return RNSM_OK;
    };

    if (batched) {
        const rnsm_status bs = batched_ops();
        if (bs != RNSM_OK) return bs;
    } else
    for (size_t oi = 0; oi < ops.size(); ++oi) {
        const int s = ops[oi].first, t = ops[oi].second;
        const int64_t ns = sizes[s], nt = sizes[t];
        int32_t *d_piv, *d_fol, *d_folp, *res, *h_lists;
        float* res_d;
        WS(d_piv, "pivots", sizeof(int32_t) * ns);
        WS(d_fol, "followers", sizeof(int32_t) * ns);
        WS(d_folp, "follower_pivot", sizeof(int32_t) * ns);
        WS(res, "res", sizeof(int32_t) * ns * RES);
        WS(res_d, "res_d", sizeof(float) * ns * RES);
        // selection lists (the greedy's output) and launch lists (the same
        // groups, each chunk's groups ordered by the pivot's breadth-first rank)
        int32_t* h_launch;
        HS(h_lists, "h_lists", sizeof(int32_t) * 3 * ns);
        HS(h_launch, "h_launch", sizeof(int32_t) * 3 * ns);
        int32_t* h_piv = h_lists;
        int32_t* h_fol = h_lists + ns;
        int32_t* h_folp = h_lists + 2 * ns;
        int32_t* h_lp = h_launch;
        int32_t* h_lf = h_launch + ns;
        int32_t* h_lfp = h_launch + 2 * ns;
        int64_t *h_off = nullptr;
        int32_t* h_ids = nullptr;
        const bool fresh = cached[s].empty() && !(p->flags & RNSM_FLAG_ALL_PIVOTS);
        int ev_rk_off = -1, ev_rk_ids = -1, ev_rk_cnt = -1;
        int ev_go = -1;  // st: result rows cleared; the side stream starts after it
        // gain levels of the greedy, made on the device from the list lengths
        constexpr int LCAP = GainLevels::LCAP;
        const int64_t lv_words = (ns + 63) / 64;
        // long lists (gain >= LCAP) copied with the levels; more are fetched
        // when the greedy starts (RNSM_GAIN_PREFIX sets the count, for tests)
        int64_t hpre = std::min<int64_t>(ns, 1 << 16);
        if (const char* c = getenv("RNSM_GAIN_PREFIX")) hpre = std::min<int64_t>(ns, std::max(1ll, atoll(c)));
        unsigned long long* h_lv = nullptr;
        int* h_lvctl = nullptr;
        int2* h_high = nullptr;
        int2* d_high = nullptr;
        if (fresh) {
            int32_t *nk, *rcnt, *rk_ids;
            int64_t *rk_off, *stmp;
            WS(nk, "nk", sizeof(int32_t) * ns * k);
            WS(rcnt, "rk_cnt", sizeof(int32_t) * ns);
            WS(rk_off, "rk_off", sizeof(int64_t) * (ns + 1));
            WS(rk_ids, "rk_ids", sizeof(int32_t) * ns * k);
            WS(stmp, "scan_tmp", sizeof(int64_t) * scan_tmp_elems(ns));
            // breadth-first order of the source graph from its entry: the
            // expansion runs its queries in that order, and pivot groups are
            // launched by the rank of their pivot in it (locality in L2 only)
            int32_t* bfs_order = nullptr;
            int ev_order = -1;
            if (oi == 0 && bfs_early) {  // made on the side stream during the set-up
                bfs_order = bfs0;
                ev_order = ev_bfs0;
                HIPCHK(hipStreamWaitEvent(st, E.ev[ev_order], 0));
            } else if (use_bfs) {
                const rnsm_status bs = bfs_order_of(s, st, &bfs_order, &ev_order);
                if (bs != RNSM_OK) return bs;
            }
            std::array<int, 3> ex;
            HIPCHK(E.stat(st, &ex[0]));
            SearchArgs a = {};
            a.base = vi.search + bases[s] * vi.row_bytes;
            a.nch = vi.nch;
            a.row_bytes = vi.row_bytes;
            a.offs = graphs[s].offsets;
            a.nbrs = graphs[s].nbrs;
            a.padj = padj + bases[s] * R;
            a.rp = R;
            a.n = ns;
            a.qvec = a.base;
            a.qidx = bfs_order;
            a.out_row = bfs_order;
            a.nq = ns;
            a.seed_mode = 1;
            a.metric = p->metric;
            a.base_norm = norms ? norms + bases[s] : nullptr;
            a.q_norm = a.base_norm;
            a.ef = kp;
            a.G = vi.G;
            a.lgG = ilog2i(vi.G);
            a.cpl = vi.cpl;
            const SearchShape sh = search_shape(kp, R, ns, vi.tt, hb_req, wpb_req);
            a.hbits = sh.hbits;
            a.hash_mode = sh.mode;
            a.out_mode = 1;
            a.out_ids = nk;
            a.out_stride = k;
            a.out_k = k;
            a.counters = cnt + 0 * CNT_SLOTS * CNT_N;
            a.err = errf;
            if (!touched[s] && search_d_exact) {
                // the source rows are still the input rows: the expansion's
                // first step gives their distances, which the prune reuses
                a.row_d = rdist;
                a.row_d_base = bases[s];
                a.row_d_stride = R;
            }
            HIPCHK(launch_search(vi.tt, a, sh.wpb, st));
            HIPCHK(E.stat(st, &ex[1]));
            // the greedy's gain levels, made on the device from the list
            // lengths, go to the host first; offsets and ids follow
            HIPCHK(launch_count_ids(nk, ns, k, rcnt, st));
            {
                unsigned long long* d_lv;
                int* d_lvctl;
                const size_t lv_bytes =
                    sizeof(unsigned long long) * LCAP * (size_t)std::max<int64_t>(lv_words, 1);
                WS(d_lv, "gain_levels", lv_bytes);
                WS(d_lvctl, "gain_ctl", sizeof(int));
                WS(d_high, "gain_high", sizeof(int2) * std::max<int64_t>(ns, 1));
                HS(h_lv, "h_gain_levels", lv_bytes);
                HS(h_lvctl, "h_gain_ctl", sizeof(int));
                HS(h_high, "h_gain_high", sizeof(int2) * std::max<int64_t>(hpre, 1));
                HIPCHK(launch_gain_levels(rcnt, ns, LCAP, d_lv, d_lvctl, d_high, ns, st));
                HIPCHK(hipMemcpyAsync(h_lv, d_lv, sizeof(unsigned long long) * LCAP * lv_words,
                                      hipMemcpyDeviceToHost, st));
                HIPCHK(hipMemcpyAsync(h_lvctl, d_lvctl, sizeof(int), hipMemcpyDeviceToHost, st));
                HIPCHK(hipMemcpyAsync(h_high, d_high, sizeof(int2) * hpre, hipMemcpyDeviceToHost, st));
            }
            HIPCHK(E.record(st, &ev_rk_cnt));
            HIPCHK(launch_invert_lists(nk, ns, k, rcnt, rk_off, rk_ids, stmp, st));
            HIPCHK(E.stat(st, &ex[2]));
            ev_exp.push_back(ex);
            g_stats.queries[0] += ns;
            g_stats.launches[0] += 1;
            // R_k to the host through pinned buffers
            HS(h_off, "h_rk_off", sizeof(int64_t) * (ns + 1));
            HS(h_ids, "h_rk_ids", sizeof(int32_t) * ns * k);
            HIPCHK(hipMemcpyAsync(h_off, rk_off, sizeof(int64_t) * (ns + 1), hipMemcpyDeviceToHost, st));
            HIPCHK(E.record(st, &ev_rk_off));
            HIPCHK(hipMemcpyAsync(h_ids, rk_ids, sizeof(int32_t) * ns * k, hipMemcpyDeviceToHost, st));
            HIPCHK(E.record(st, &ev_rk_ids));
            HIPCHK(hipMemsetAsync(res, 0xff, sizeof(int32_t) * ns * RES, st));
            HIPCHK(E.record(st, &ev_go));
            if (!touched[t]) {
                // the target rows are still the input rows: their distances,
                // which the target prune needs, are computed while the host
                // selects the first pivots (the side stream does not wait)
                PruneArgs rd = {};
                rd.X = vecs->f32;
                rd.xb = xb16;
                rd.n_total = N;
                rd.nch = vi.nch32;
                rd.G = vi.G32;
                rd.lgG = ilog2i(vi.G32);
                rd.cpl = vi.cpl32;
                rd.metric = p->metric;
                rd.norms = norms;
                rd.n_items = nt;
                rd.item_base = bases[t];
                rd.rows_in = rows;
                rd.deg_in = deg;
                rd.rows_d = rdist;
                rd.R = R;
                rd.wcap = TARGET_WCAP;
                rd.err = errf;
                rd.band = band;
                rd.rechecks = rechecks;
                HIPCHK(launch_row_dists(rd, prune_reads_b16(rd, pmode), st));
            }
            if (use_bfs) {
                // ranks on the host while the expansion runs
                HIPCHK(hipEventSynchronize(E.ev[ev_order]));
                rank.assign(ns, -1);
                for (int64_t r = 0; r < ns; ++r) {
                    const int32_t v = h_bfs[r];
                    if (v < 0 || v >= ns || rank[v] >= 0)
                        return fail(RNSM_EINTERNAL, "rnsm_merge: breadth-first order is not a permutation");
                    rank[v] = (int32_t)r;
                }
            }
        }
        // also drains the previous operation, whose copies read h_lists (the
        // stream waited for every one of them before its prunes); a fresh
        // source waits for the R_k offsets only, the ids follow
        const auto th0 = std::chrono::steady_clock::now();
        if (fresh)
            HIPCHK(hipEventSynchronize(E.ev[ev_rk_cnt]));
        else
            HIPCHK(hipStreamSynchronize(st));
        const auto th1 = std::chrono::steady_clock::now();
        if (fresh) {
            levels.n = ns;
            levels.words = lv_words;
            levels.ext = reinterpret_cast<uint64_t*>(h_lv);
            const int64_t nh = h_lvctl[0];
            // levels up to the highest one in use (all of them when some
            // gains went to the heap)
            levels.nlev = nh > 0 ? LCAP : 0;
            for (int g = LCAP - 1; g >= 0 && levels.nlev == 0; --g) {
                const unsigned long long* b = h_lv + (size_t)g * lv_words;
                for (int64_t w = 0; w < lv_words; ++w)
                    if (b[w]) {
                        levels.nlev = g + 1;
                        break;
                    }
            }
            levels.high.resize((size_t)nh);
            for (int64_t i = 0; i < std::min(nh, hpre); ++i)
                levels.high[(size_t)i] = {(int64_t)h_high[i].x, (int32_t)h_high[i].y};
            if (nh > hpre) {  // more long lists than the prefix copied ahead
                std::vector<int2> rest((size_t)(nh - hpre));
                HIPCHK(hipMemcpy(rest.data(), d_high + hpre, sizeof(int2) * (nh - hpre),
                                 hipMemcpyDeviceToHost));
                for (int64_t i = hpre; i < nh; ++i)
                    levels.high[(size_t)i] = {(int64_t)rest[(size_t)(i - hpre)].x,
                                              (int32_t)rest[(size_t)(i - hpre)].y};
            }
        }
        double th_levels = 0, th_ids = 0, th_first_post = -1, th_first_launch = -1;
        if (!fresh) {
            HIPCHK(hipMemsetAsync(res, 0xff, sizeof(int32_t) * ns * RES, st));
            HIPCHK(E.record(st, &ev_go));
        }

        // search arguments shared by the chunks
        SearchArgs a = {};
        a.base = vi.search + bases[t] * vi.row_bytes;
        a.nch = vi.nch;
        a.row_bytes = vi.row_bytes;
        a.offs = graphs[t].offsets;
        a.nbrs = graphs[t].nbrs;
        a.padj = padj + bases[t] * R;
        a.rp = R;
        a.n = nt;
        a.qvec = vi.search + bases[s] * vi.row_bytes;
        a.metric = p->metric;
        a.base_norm = norms ? norms + bases[t] : nullptr;
        a.q_norm = norms ? norms + bases[s] : nullptr;
        a.G = vi.G;
        a.lgG = ilog2i(vi.G);
        a.cpl = vi.cpl;
        a.out_mode = 0;
        a.out_ids = res;
        a.out_d = res_d;
        a.out_stride = RES;
        a.err = errf;
        // wave A: pivots, naive search from the target's entry point
        SearchArgs aA = a;
        aA.seed_mode = 0;
        aA.entry = graphs[t].entry;
        aA.ef = efN;
        aA.out_k = efN;
        aA.counters = cnt + 1 * CNT_SLOTS * CNT_N;
        const SearchShape shA = search_shape(efN, R, nt, vi.tt, hb_req, wpb_req);
        aA.hbits = shA.hbits;
        aA.hash_mode = shA.mode;
        // wave B: followers, local sliding from their pivot's results
        SearchArgs aB = a;
        aB.seed_mode = 2;
        aB.seed_ids = res;
        aB.seed_stride = RES;
        aB.n_seeds = efN;
        aB.ef = efS;
        aB.out_k = efS;
        aB.counters = cnt + 2 * CNT_SLOTS * CNT_N;
        const SearchShape shB = search_shape(efS, R, nt, vi.tt, hb_req, wpb_req);
        aB.hbits = shB.hbits;
        aB.hash_mode = shB.mode;
        g_stats.exact_visited = shB.mode;
        g_stats.search_hash_bits = shB.hbits;
        g_stats.search_waves_per_block = shB.wpb;

        // chunk c: lists and naive search on the side stream, then the
        // sliding search on st after the naive one (event wait); the naive
        // search of chunk c+1 overlaps the sliding search of chunk c
        HIPCHK(hipStreamWaitEvent(sd, E.ev[ev_go], 0));
        // the pivots' copies and naive searches: on the side stream, or (the
        // measurement switch RNSM_ONE_STREAM=1) on st, where every search
        // launch then runs alone and its event time is its own
        const hipStream_t sa = one_stream ? st : sd;
        // source rows: current row + search results, pruned to R after the
        // searches, each pivot group together (order staged with the chunks).
        // (Pruning each chunk on a third stream as soon as its searches end
        // measured no faster: the prune waves take the LDS and CU slots the
        // searches of later chunks would use.)
        int32_t *h_order, *d_order;
        HS(h_order, "h_order", sizeof(int32_t) * ns);
        WS(d_order, "prune_order", sizeof(int32_t) * ns);
        PruneArgs qs = {};
        qs.X = vecs->f32;
        qs.xb = xb16;
        qs.n_total = N;
        qs.nch = vi.nch32;
        qs.G = vi.G32;
        qs.lgG = ilog2i(vi.G32);
        qs.cpl = vi.cpl32;
        qs.metric = p->metric;
        qs.norms = norms;
        qs.item_base = bases[s];
        qs.rows_in = rows;
        qs.deg_in = deg;
        qs.rows_d = rdist;
        qs.extra_mode = 1;
        qs.extra_ids = res;
        qs.extra_d = search_d_exact ? res_d : nullptr;
        qs.extra_sorted = search_d_exact && RES <= 128;  // beams in key order
        qs.extra_stride = RES;
        qs.extra_cnt = RES;
        qs.extra_index_base = bases[s];
        qs.extra_id_add = bases[t];
        qs.alpha = p->alpha;
        qs.rule = p->prune_rule;
        qs.rule_a = rule_a;
        qs.R = R;
        qs.rows_out = rows;
        qs.deg_out = deg;
        qs.dist_out = rdist;
        qs.wcap = R + RES;
        qs.err = errf;
        qs.band = band;
        qs.rechecks = rechecks;
        bool groups_ok = true;
        int64_t pa = 0, fa = 0;  // list prefixes already handed to the device
        int64_t n_launch_a = 0, n_launch_b = 0;
        hipError_t cerr = hipSuccess;
        bool reorder = false;  // set when the lists come from the greedy and ranks exist
        // launch lists for pivots [pa, np) and followers [fa, nf)
        auto stage = [&](int64_t np, int64_t nf) {
            if (!reorder) {
                memcpy(h_lp + pa, h_piv + pa, sizeof(int32_t) * (np - pa));
                memcpy(h_lf + fa, h_fol + fa, sizeof(int32_t) * (nf - fa));
                memcpy(h_lfp + fa, h_folp + fa, sizeof(int32_t) * (nf - fa));
                return;
            }
            // followers of each new pivot: one contiguous run
            for (int64_t i = pa; i < np; ++i) fcnt[h_piv[i]] = 0;
            for (int64_t f = fa; f < nf; ++f) {
                const int32_t pv = h_folp[f];
                if (fcnt[pv]++ == 0) fbeg[pv] = (int32_t)f;
            }
            int64_t lo = INT64_MAX, hi = -1;
            for (int64_t i = pa; i < np; ++i) {
                const int64_t r = rank[h_piv[i]];
                rbits[r >> 6] |= 1ull << (r & 63);
                lo = std::min(lo, r >> 6);
                hi = std::max(hi, r >> 6);
            }
            int64_t o = pa, fo = fa;
            for (int64_t w = lo; w <= hi; ++w) {
                uint64_t b = rbits[w];
                rbits[w] = 0;
                while (b) {
                    const int32_t pv = h_bfs[w * 64 + __builtin_ctzll(b)];
                    b &= b - 1;
                    h_lp[o++] = pv;
                    const int32_t c = fcnt[pv];
                    if (c) {
                        memcpy(h_lf + fo, h_fol + fbeg[pv], sizeof(int32_t) * c);
                        for (int32_t t2 = 0; t2 < c; ++t2) h_lfp[fo + t2] = pv;
                        fo += c;
                    }
                }
            }
        };
        auto emit = [&](int64_t np, int64_t nf) {
            if (cerr != hipSuccess) return;
            stage(np, nf);
            // prune order of the chunk: each pivot followed by its followers,
            // so that neighbouring wavefronts share most candidate rows in L2
            const int64_t o0 = pa + fa;
            {
                int64_t o = o0, f = fa;
                for (int64_t i = pa; i < np; ++i) {
                    const int32_t pv = h_lp[i];
                    h_order[o++] = pv;
                    while (f < nf && h_lfp[f] == pv) h_order[o++] = h_lf[f++];
                }
                if (f != nf) {
                    groups_ok = false;
                    if (cerr == hipSuccess) cerr = hipErrorInvalidValue;
                    return;
                }
            }
            std::array<int, 4> ce;
            auto chk = [&](hipError_t e) {
                if (e != hipSuccess && cerr == hipSuccess) cerr = e;
                return e == hipSuccess;
            };
            if (np > pa && !chk(hipMemcpyAsync(d_piv + pa, h_lp + pa, sizeof(int32_t) * (np - pa),
                                               hipMemcpyHostToDevice, sa)))
                return;
            if (nf > fa) {
                if (!chk(hipMemcpyAsync(d_fol + fa, h_lf + fa, sizeof(int32_t) * (nf - fa),
                                        hipMemcpyHostToDevice, sa)) ||
                    !chk(hipMemcpyAsync(d_folp + fa, h_lfp + fa, sizeof(int32_t) * (nf - fa),
                                        hipMemcpyHostToDevice, sa)))
                    return;
            }
            if (!chk(hipMemcpyAsync(d_order + o0, h_order + o0, sizeof(int32_t) * (np + nf - o0),
                                    hipMemcpyHostToDevice, sa)))
                return;
            if (!chk(E.stat(sa, &ce[0]))) return;
            SearchArgs x = aA;
            x.qidx = d_piv + pa;
            x.out_row = x.qidx;
            x.nq = np - pa;
            if (!chk(launch_search(vi.tt, x, shA.wpb, sa)) || !chk(E.record(sa, &ce[1]))) return;
            if (!chk(hipStreamWaitEvent(st, E.ev[ce[1]], 0))) return;
            if (!chk(E.stat(st, &ce[2]))) return;
            SearchArgs y = aB;
            y.qidx = d_fol + fa;
            y.out_row = y.qidx;
            y.seed_row = d_folp + fa;
            y.nq = nf - fa;
            if (!chk(launch_search(vi.tt, y, shB.wpb, st)) || !chk(E.stat(st, &ce[3]))) return;
            ev_chunk.push_back(ce);
            if (th_first_launch < 0) th_first_launch = ms_since(th1);
            n_launch_a += np > pa;  // the stats are thread-local: added after the join
            n_launch_b += nf > fa;
            pa = np;
            fa = nf;
        };
        const size_t chunk0 = ev_chunk.size();
        const auto tg = std::chrono::steady_clock::now();
        // the greedy (this thread) posts (np, nf) marks; a launcher thread
        // stages each chunk's groups and queues its copies and searches
        std::mutex qm;
        std::condition_variable qcv;
        std::deque<std::pair<int64_t, int64_t>> qmarks;
        bool qdone = false;
        // the greedy thread must not index E.ev while the launcher appends to it
        const hipEvent_t rk_ids_event = ev_rk_ids >= 0 ? E.ev[ev_rk_ids] : nullptr;
        std::thread launcher([&] {
            if (hipSetDevice(dev) != hipSuccess && cerr == hipSuccess) cerr = hipErrorInvalidDevice;
            for (;;) {
                std::pair<int64_t, int64_t> it;
                {
                    std::unique_lock<std::mutex> l(qm);
                    qcv.wait(l, [&] { return !qmarks.empty() || qdone; });
                    if (qmarks.empty()) return;
                    it = qmarks.front();
                    qmarks.pop_front();
                }
                try {
                    emit(it.first, it.second);
                } catch (const std::bad_alloc&) {
                    if (cerr == hipSuccess) cerr = hipErrorOutOfMemory;
                } catch (...) {
                    if (cerr == hipSuccess) cerr = hipErrorUnknown;
                }
            }
        });
        // joins the launcher on every way out of this scope (an exception
        // from the greedy included)
        struct JoinLauncher {
            std::thread& t;
            std::mutex& m;
            std::condition_variable& cv;
            bool& done;
            ~JoinLauncher() {
                if (!t.joinable()) return;
                {
                    std::lock_guard<std::mutex> l(m);
                    done = true;
                }
                cv.notify_one();
                t.join();
            }
        } join_launcher{launcher, qm, qcv, qdone};
        auto post = [&](int64_t a1, int64_t b1) {
            if (th_first_post < 0) th_first_post = ms_since(th1);
            {
                std::lock_guard<std::mutex> l(qm);
                qmarks.emplace_back(a1, b1);
            }
            qcv.notify_one();
        };
        int64_t np = 0, nf = 0;
        hipError_t wait_err = hipSuccess;  // the R_k ids transfer (greedy thread)
        if (p->flags & RNSM_FLAG_ALL_PIVOTS) {
            // every vertex is a pivot (no sliding)
            for (int64_t v = 0; v < ns; ++v) h_piv[v] = (int32_t)v;
            np = ns;
            post(np, 0);
        } else if (fresh) {
            reorder = use_bfs && (int64_t)rank.size() == ns;
            if (reorder) {
                fbeg.resize(ns);
                fcnt.resize(ns);
                rbits.assign((size_t)((ns + 63) / 64), 0ull);
            }
            // chunks double from ns / 16 up to ns / 4 with float32 rows (fewer,
            // longer launches measured faster), from ns / 64 up to ns / 8 with
            // 16-bit rows (their faster searches would otherwise wait on the
            // greedy)
            int64_t chunk = std::max<int64_t>(4096, ns / (vi.tt == 0 ? 16 : 64));
            const int64_t chunk_div = vi.tt == 0 ? 4 : 8;
            if (const char* c = getenv("RNSM_PIVOT_CHUNK")) chunk = std::max(1ll, atoll(c));
            select_pivots(levels, h_off, h_ids, h_piv, h_fol, h_folp, chunk,
                          std::max<int64_t>(chunk, ns / chunk_div),
                          [&](int64_t a1, int64_t b1) {
                              np = a1;
                              nf = b1;
                              post(a1, b1);
                          },
                          [&] {
                              th_levels = ms_since(th1);
                              wait_err = hipEventSynchronize(rk_ids_event);
                              th_ids = ms_since(th1);
                          });  // the ids are copied after the offsets
        } else {
            memcpy(h_lists, cached[s].data(), sizeof(int32_t) * 3 * ns);
            np = cached_np[s];
            nf = cached_nf[s];
            post(np, nf);
        }
        {
            std::lock_guard<std::mutex> l(qm);
            qdone = true;
        }
        qcv.notify_one();
        launcher.join();
        if (wait_err != hipSuccess && cerr == hipSuccess) cerr = wait_err;
        g_stats.launches[1] += n_launch_a;
        g_stats.launches[2] += n_launch_b;
        if (fresh && last_use[s] > (int)oi) {
            cached[s].assign(h_launch, h_launch + 3 * ns);
            cached_np[s] = np;
            cached_nf[s] = nf;
        }
        ms_plan += ms_since(tg);
        if (getenv("RNSM_HOST_TRACE"))
            fprintf(stderr,
                    "[rnsm host] op %zu: wait R_k offsets %.3f ms; after it: levels %.3f, ids %.3f, "
                    "first chunk posted %.3f, first chunk queued %.3f, greedy + queueing %.3f ms\n",
                    oi, std::chrono::duration<double, std::milli>(th1 - th0).count(), th_levels,
                    th_ids, th_first_post, th_first_launch, ms_since(th1));
        if (!ev_chunk.empty() && ev_chunk.size() > chunk0)
            ev_span.push_back({ev_chunk[chunk0][0], ev_chunk.back()[3]});
        if (cerr != hipSuccess) {
            (void)hipStreamSynchronize(sd);
            (void)hipStreamSynchronize(st);
            if (!groups_ok)
                return fail(RNSM_EINTERNAL, "rnsm_merge: pivot groups do not cover the source");
            return fail(cerr == hipErrorOutOfMemory ? RNSM_ENOMEM : RNSM_EDEVICE,
                        "rnsm_merge: queueing searches: %s", hipGetErrorString(cerr));
        }
        if (pa + fa != ns)
            return fail(RNSM_EINTERNAL, "rnsm_merge: pivot groups do not cover the source");
        g_stats.queries[1] += np;
        g_stats.queries[2] += nf;
        // source prune, in the order staged with the chunks (the copies on
        // the side stream precede the last sliding search, which st waited for)
        std::array<int, 2> pe;
        HIPCHK(E.stat(st, &pe[0]));
        // reverse edges into the target (counted by the source prune), then
        // prune every target that got some
        int32_t *rc, *rcur, *rev;
        int64_t *roff, *stmp;
        u64* scratch;
        WS(rc, "rev_cnt", sizeof(int32_t) * nt);
        WS(rcur, "rev_cur", sizeof(int32_t) * nt);
        WS(roff, "rev_off", sizeof(int64_t) * (nt + 1));
        WS(rev, "rev_ids", sizeof(int32_t) * std::max<int64_t>(ns * R, 1));
        float* rev_d;
        WS(rev_d, "rev_d", sizeof(float) * std::max<int64_t>(ns * R, 1));
        WS(stmp, "scan_tmp2", sizeof(int64_t) * scan_tmp_elems(nt));
        WS(scratch, "prune_scratch", sizeof(u64) * 2 * (nt * R + ns * R));
        HIPCHK(hipMemsetAsync(rc, 0, sizeof(int32_t) * nt, st));
        HIPCHK(hipMemsetAsync(rcur, 0, sizeof(int32_t) * nt, st));
        PruneArgs q = qs;
        q.items = d_order;
        q.n_items = ns;
        q.rev_cnt = rc;
        q.rev_lo = bases[t];
        q.rev_n = nt;
        HIPCHK(run_prune(q, pmode, st));
        HIPCHK(launch_scan(rc, nt, roff, stmp, st));
        HIPCHK(launch_rev_scatter(rows, deg, rdist, bases[s], ns, R, bases[t], nt, roff, rcur, rev,
                                  rev_d, st));
        PruneArgs r = q;
        r.n_items = nt;
        r.items = nullptr;
        r.item_base = bases[t];
        r.extra_mode = 2;
        r.extra_ids = rev;
        r.extra_d = rev_d;
        r.extra_off = roff;
        r.extra_index_base = bases[t];
        r.extra_id_add = 0;
        r.skip_empty_extra = 1;
        r.extra_sorted = 0;
        r.scratch = scratch;
        r.wcap = TARGET_WCAP;
        r.rev_cnt = nullptr;
        HIPCHK(run_prune(r, pmode, st));
        HIPCHK(E.stat(st, &pe[1]));
        ev_prune.push_back(pe);
        HIPCHK(hipMemcpyAsync(h_nrev + oi, roff + nt, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        g_stats.n_followers += nf;
        g_stats.n_pivots += np;
        g_stats.n_source_vertices += ns;
        touched[s] = touched[t] = 1;
    }

    // ----------------------------------------------------------- compaction
    // into the caller's device buffers, or (host output) into workspace
    // buffers that are copied to library-allocated host arrays below
    int64_t* o_off = out->offsets;
    int32_t* o_nbrs = out->nbrs;
    float* o_dists = out->dists;
    if (host_out) {
        WS(o_off, "out_offsets", sizeof(int64_t) * (N + 1));
        WS(o_nbrs, "out_nbrs", sizeof(int32_t) * N * R);
        WS(o_dists, "out_dists", sizeof(float) * N * R);
    }
    int c0, c1;
    HIPCHK(E.stat(st, &c0));
    int64_t* stmp3;
    WS(stmp3, "scan_tmp3", sizeof(int64_t) * scan_tmp_elems(N));
    HIPCHK(launch_scan(deg, N, o_off, stmp3, st));
    if (p->metric != RNSM_L2SQ && !norms64) {
        WS(norms64, "norms64", sizeof(double) * N);
        HIPCHK(launch_norms(vecs->f32, N, vecs->dim, nullptr, st, norms64));
    }
    HIPCHK(launch_compact(rows, deg, rdist, o_off, N, R, vecs->f32, vecs->dim, p->metric,
                          norms, o_nbrs, o_dists, st, norms64));
    HIPCHK(E.stat(st, &c1));
    int64_t nedges = 0;
    std::vector<u64> hslots(3 * CNT_SLOTS * CNT_N);
    u64 hc[3 * CNT_N] = {};
    int herr = 0;
    HIPCHK(hipMemcpyAsync(&nedges, o_off + N, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    u64 hrck[CNT_SLOTS] = {};
    if (!E.no_stats) {
        HIPCHK(hipMemcpyAsync(hslots.data(), cnt, sizeof(u64) * hslots.size(),
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hrck, rechecks, sizeof hrck, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipMemcpyAsync(&herr, errf, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (host_out) {
        // host arrays owned by the caller from here on (rnsm_csr_free);
        // released again if anything below fails
        struct HostCsr {
            int64_t* off = nullptr;
            int32_t* nb = nullptr;
            float* d = nullptr;
            ~HostCsr() {
                free(off);
                free(nb);
                free(d);
            }
        } h;
        h.off = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
        h.nb = (int32_t*)malloc(sizeof(int32_t) * std::max<int64_t>(nedges, 1));
        h.d = (float*)malloc(sizeof(float) * std::max<int64_t>(nedges, 1));
        if (!h.off || !h.nb || !h.d)
            return fail(RNSM_ENOMEM, "rnsm_merge: host output allocation failed");
        HIPCHK(hipMemcpyAsync(h.off, o_off, sizeof(int64_t) * (N + 1), hipMemcpyDeviceToHost, st));
        if (nedges > 0) {
            HIPCHK(hipMemcpyAsync(h.nb, o_nbrs, sizeof(int32_t) * nedges, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(h.d, o_dists, sizeof(float) * nedges, hipMemcpyDeviceToHost, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        if (!(herr & 3)) {
            out->offsets = h.off;
            out->nbrs = h.nb;
            out->dists = h.d;
            out->mem = RNSM_HOST;
            h.off = nullptr;
            h.nb = nullptr;
            h.d = nullptr;
        }
    } else {
        out->mem = RNSM_DEVICE;
    }
    for (int ph = 0; ph < 3; ++ph)
        for (int sl = 0; sl < CNT_SLOTS; ++sl)
            for (int c = 0; c < CNT_N; ++c) hc[ph * CNT_N + c] += hslots[(ph * CNT_SLOTS + sl) * CNT_N + c];
    for (auto& ex : ev_exp) {
        g_stats.ms_search[0] += E.between(ex[0], ex[1]);
        g_stats.ms_invert += E.between(ex[1], ex[2]);
    }
    for (auto& ce : ev_chunk) {
        g_stats.ms_search[1] += E.between(ce[0], ce[1]);
        g_stats.ms_search[2] += E.between(ce[2], ce[3]);
    }
    for (auto& pe : ev_prune) ms_prune += E.between(pe[0], pe[1]);
    for (auto& er : ev_rounds) {  // batched form: group searches (naive and sliding together),
                                  // then the overflow followers' sliding
        g_stats.ms_search[1] += E.between(er[0], er[1]);
        g_stats.ms_search[2] += E.between(er[1], er[2]);
        g_stats.ms_search_span += E.between(er[0], er[2]);
        ms_prune += E.between(er[2], er[3]);
    }
    for (auto& oe : ord_ev) g_stats.ms_order += E.between(oe[0], oe[1]);
    for (auto& se : sel_ev) {
        g_stats.ms_select += E.between(se[0], se[1]);
        g_stats.ms_groups += E.between(se[1], se[2]);
    }
    for (auto& sp : ev_span) g_stats.ms_search_span += E.between(sp[0], sp[1]);
    for (size_t oi = 0; oi < ops.size(); ++oi) g_stats.n_reverse_edges += h_nrev[oi];
    if (herr & 1) return fail(RNSM_EINTERNAL, "rnsm_merge: a search exceeded its iteration bound");
    if (herr & 2) return fail(RNSM_EINTERNAL, "rnsm_merge: prune candidate list over capacity");

    // merged entry: entry of the largest sub-index (ties: lowest index)
    int big = 0;
    for (int i = 1; i < m; ++i)
        if (sizes[i] > sizes[big]) big = i;
    out->entry = (int32_t)(bases[big] + graphs[big].entry);
    out->n_edges = nedges;

    rnsm_stats& S = g_stats;
    S.ms_plan = ms_plan;
    S.ms_prune = ms_prune;
    S.ms_compact = E.between(c0, c1);
    S.n_ops = (int64_t)ops.size();
    S.n_rounds = batched ? n_rounds_b : (int64_t)ops.size();
    S.prune_path = pmode;
    for (int sl = 0; sl < CNT_SLOTS; ++sl) S.prune_rechecks += (int64_t)hrck[sl];
    S.row_bytes = vi.row_bytes;
    const double rb = vi.row_bytes;
    for (int ph = 0; ph < 3; ++ph) {
        S.ndc[ph] = (int64_t)hc[ph * CNT_N + CNT_NDC];
        S.expansions[ph] = (int64_t)hc[ph * CNT_N + CNT_EXP];
        S.adjacency[ph] = (int64_t)hc[ph * CNT_N + CNT_ADJ];
        S.hash_evictions += (int64_t)hc[ph * CNT_N + CNT_HFULL];
        // every distance reads one row, every expansion reads two offsets and
        // its adjacency, every query reads its row and writes its result;
        // followers also read their pivot's beam
        const double out_w = ph == 0 ? k : (ph == 1 ? efN : efS);
        S.bytes[ph] = (double)S.ndc[ph] * rb + (double)S.expansions[ph] * 16.0 +
                      (double)S.adjacency[ph] * 4.0 + (double)S.queries[ph] * (rb + 4.0 * out_w) +
                      (ph == 2 ? (double)S.queries[ph] * 4.0 * efN : 0.0);
    }
    S.ms_total = ms_since(t0);
    (void)fallbacks;
    return RNSM_OK;
}

static rnsm_status rnsm_merge_simple_impl(int32_t m, const rnsm_graph* graphs, const rnsm_vectors* vecs,
                              int32_t R, int32_t L, float alpha, rnsm_csr* out) {
    rnsm_params p;
    memset(&p, 0, sizeof p);
    p.R = R;
    p.L = L;
    p.alpha = alpha;
    p.metric = RNSM_L2SQ;
    if (!vecs) return fail(RNSM_EINVAL, "rnsm_merge_simple: NULL vectors");
    rnsm_vectors v = *vecs;
    v.search_dtype = RNSM_F32;
    v.search = nullptr;
    return rnsm_merge(m, graphs, &v, &p, out);
}

// Device buffers of one beam-search call: counters (CNT_SLOTS x CNT_N), the
// error flag, and for cosine the norms of the base rows and of the queries.
struct SearchBufs {
    u64* cnt = nullptr;
    int* errf = nullptr;
    float* bn = nullptr;
    float* qn = nullptr;
};

// Argument checks of rnsm_search and its allocation-free variant.
static rnsm_status search_check(const char* fn, const rnsm_graph* g, const rnsm_vectors* base,
                                const void* queries, int64_t nq, const int32_t* seeds,
                                int32_t n_seeds, int32_t ef, int32_t k, rnsm_metric metric,
                                int32_t* out_ids, VecInfo& vi) {
    if (!g || !base || !out_ids || (nq > 0 && !queries))
        return fail(RNSM_EINVAL, "%s: NULL argument", fn);
    if (nq < 0) return fail(RNSM_EINVAL, "%s: nq < 0", fn);
    if (ef < 1 || ef > 128) return fail(RNSM_EINVAL, "%s: ef outside 1..128", fn);
    if (k < 1 || k > ef) return fail(RNSM_EINVAL, "%s: k outside 1..ef", fn);
    if (metric < RNSM_L2SQ || metric > RNSM_COSINE) return fail(RNSM_EINVAL, "%s: metric", fn);
    if (seeds && n_seeds < 1) return fail(RNSM_EINVAL, "%s: n_seeds < 1", fn);
    if (g->n < 1 || !g->offsets || !g->nbrs || base->n != g->n)
        return fail(RNSM_EINVAL, "%s: graph / base mismatch", fn);
    if (!seeds && (g->entry < 0 || g->entry >= g->n)) return fail(RNSM_EINVAL, "%s: entry", fn);
    return vec_info(base, vi);
}

// Algorithm 1 for nq queries on the given buffers (st ordered): clears the
// counters and the error flag with a kernel, makes the cosine norms (base
// rows from their float32 originals, queries from the rows as given, in the
// searched copy's type), launches, and waits for the error flag.
static rnsm_status search_run(const char* fn, const rnsm_graph* g, const rnsm_vectors* base,
                              const VecInfo& vi, const void* queries, int64_t nq,
                              const int32_t* seeds, int32_t n_seeds, int32_t ef, int32_t k,
                              rnsm_metric metric, int32_t* out_ids, float* out_dists,
                              hipStream_t st, const SearchBufs& b) {
    HIPCHK(launch_zero(b.cnt, sizeof(u64) * CNT_SLOTS * CNT_N, st));
    HIPCHK(launch_zero(b.errf, sizeof(int), st));
    if (metric == RNSM_COSINE) {
        HIPCHK(launch_norms(base->f32, g->n, base->dim, b.bn, st));
        if (vi.tt == 0)
            HIPCHK(launch_norms((const float*)queries, nq, base->dim, b.qn, st));
        else
            HIPCHK(launch_norms16(queries, vi.tt, nq, base->dim, b.qn, st));
    }
    SearchArgs a = {};
    a.base = vi.search;
    a.nch = vi.nch;
    a.row_bytes = vi.row_bytes;
    a.offs = g->offsets;
    a.nbrs = g->nbrs;
    a.n = g->n;
    a.qvec = (const char*)queries;
    a.nq = nq;
    a.seed_mode = seeds ? 2 : 0;
    a.entry = g->entry;
    a.seed_ids = seeds;
    a.seed_stride = n_seeds;
    a.n_seeds = seeds ? n_seeds : 0;
    a.metric = metric;
    a.base_norm = b.bn;
    a.q_norm = b.qn;
    a.ef = ef;
    a.G = vi.G;
    a.lgG = ilog2i(vi.G);
    a.cpl = vi.cpl;
    const SearchShape sh = search_shape(ef, 32, g->n, vi.tt);
    a.hbits = sh.hbits;
    a.hash_mode = sh.mode;
    a.out_mode = 0;
    a.out_ids = out_ids;
    a.out_d = out_dists;
    a.out_stride = k;
    a.out_k = k;
    a.counters = b.cnt;
    a.err = b.errf;
    HIPCHK(launch_search(vi.tt, a, sh.wpb, st));
    int herr = 0;
    HIPCHK(hipMemcpyAsync(&herr, b.errf, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (herr) return fail(RNSM_EINTERNAL, "%s: a search exceeded its iteration bound", fn);
    return RNSM_OK;
}

static rnsm_status rnsm_search_impl(const rnsm_graph* g, const rnsm_vectors* base, const void* queries,
                        int64_t nq, const int32_t* seeds, int32_t n_seeds, int32_t ef, int32_t k,
                        rnsm_metric metric, int32_t* out_ids, float* out_dists, void* stream) {
    g_err.clear();
    VecInfo vi;
    rnsm_status vs = search_check("rnsm_search", g, base, queries, nq, seeds, n_seeds, ef, k,
                                  metric, out_ids, vi);
    if (vs != RNSM_OK || nq == 0) return vs;
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    Workspace& ws = g_ws[dev];
    ws.begin_call(0);
    rnsm_graph gs;
    rnsm_vectors vs2;
    if ((vs = stage_graph(ws, "rnsm_search", 0, *g, st, gs)) != RNSM_OK) return vs;
    if ((vs = stage_vectors(ws, "rnsm_search", *base, st, vs2)) != RNSM_OK) return vs;
    if ((vs = vec_info(&vs2, vi)) != RNSM_OK) return vs;
    g = &gs;
    base = &vs2;
    SearchBufs b;
    WS(b.cnt, "search_counters", sizeof(u64) * CNT_SLOTS * CNT_N);
    WS(b.errf, "search_err", sizeof(int));
    if (metric == RNSM_COSINE) {
        WS(b.bn, "search_bnorm", sizeof(float) * g->n);
        WS(b.qn, "search_qnorm", sizeof(float) * nq);
    }
    return search_run("rnsm_search", g, base, vi, queries, nq, seeds, n_seeds, ef, k, metric,
                      out_ids, out_dists, st, b);
}

// The search-shape autotuner's measurement, with g_lock held: g and base
// already checked, vi their layout. Default shape for rows of degree maxdeg.
static rnsm_status tune_shape_locked(const rnsm_graph* g, const rnsm_vectors* base, const VecInfo& vi,
                              int32_t ef, rnsm_metric metric, int64_t n_sample, int maxdeg,
                              rnsm_search_tuning* out, hipStream_t st) {
    const int64_t nq = std::min<int64_t>(n_sample, g->n);
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    Workspace& ws = g_ws[dev];
    u64* cnt;
    int *errf, *qidx, *oid;
    float* bn = nullptr;
    WS(cnt, "search_counters", sizeof(u64) * CNT_SLOTS * CNT_N);
    WS(errf, "search_err", sizeof(int));
    WS(qidx, "tune_queries", sizeof(int) * nq);
    WS(oid, "tune_ids", sizeof(int) * nq);
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(u64) * CNT_SLOTS * CNT_N, st));
    HIPCHK(hipMemsetAsync(errf, 0, sizeof(int), st));
    if (metric == RNSM_COSINE) {
        WS(bn, "search_bnorm", sizeof(float) * g->n);
        HIPCHK(launch_norms(base->f32, g->n, base->dim, bn, st));
    }
    // queries: the graph's own rows, spread evenly over its ids
    std::vector<int> hq((size_t)nq);
    for (int64_t i = 0; i < nq; ++i) hq[(size_t)i] = (int)(i * g->n / nq);
    HIPCHK(hipMemcpyAsync(qidx, hq.data(), sizeof(int) * nq, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    SearchArgs a = {};
    a.base = vi.search;
    a.nch = vi.nch;
    a.row_bytes = vi.row_bytes;
    a.offs = g->offsets;
    a.nbrs = g->nbrs;
    a.n = g->n;
    a.qvec = vi.search;
    a.qidx = qidx;
    a.nq = nq;
    a.seed_mode = 0;
    a.entry = g->entry;
    a.metric = metric;
    a.base_norm = bn;
    a.q_norm = bn;
    a.ef = ef;
    a.G = vi.G;
    a.lgG = ilog2i(vi.G);
    a.cpl = vi.cpl;
    a.out_mode = 0;
    a.out_ids = oid;
    a.out_stride = 1;
    a.out_k = 1;
    a.counters = cnt;
    a.err = errf;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(RNSM_EDEVICE, "search tuning: hipEventCreate failed");
    }
    // the best of three timed launches of one shape (after one untimed)
    auto time_shape = [&](const SearchShape& sh, float* best) -> hipError_t {
        SearchArgs b = a;
        b.hbits = sh.hbits;
        b.hash_mode = sh.mode;
        hipError_t r = launch_search(vi.tt, b, sh.wpb, st);
        *best = 0.0f;
        for (int rep = 0; rep < 3 && r == hipSuccess; ++rep) {
            float ms = 0.0f;
            if ((r = hipEventRecord(e0, st)) != hipSuccess) break;
            if ((r = launch_search(vi.tt, b, sh.wpb, st)) != hipSuccess) break;
            if ((r = hipEventRecord(e1, st)) != hipSuccess) break;
            if ((r = hipEventSynchronize(e1)) != hipSuccess) break;
            if ((r = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            if (rep == 0 || ms < *best) *best = ms;
        }
        return r;
    };
    const SearchShape def = search_shape(ef, maxdeg, g->n, vi.tt);
    float def_ms = 0.0f;
    hipError_t r = time_shape(def, &def_ms);
    SearchShape best = def;
    float best_ms = def_ms;
    int tried = 1;
    // every table size and block shape the fast table allows (an exact
    // table, forced by the id range or for diagnostics, has one shape)
    for (int hb = TUNE_HB_MIN; hb <= TUNE_HB_MAX && def.mode == 0 && r == hipSuccess; ++hb) {
        for (int w : {1, 2, 4}) {
            const SearchShape sh = search_shape(ef, maxdeg, g->n, vi.tt, hb, w);
            if (sh.mode != 0 || sh.wpb != w || (sh.hbits == def.hbits && sh.wpb == def.wpb))
                continue;
            float ms = 0.0f;
            if ((r = time_shape(sh, &ms)) != hipSuccess) break;
            ++tried;
            if (ms < best_ms) {
                best = sh;
                best_ms = ms;
            }
        }
    }
    int herr = 0;
    if (r == hipSuccess) r = hipMemcpyAsync(&herr, errf, sizeof(int), hipMemcpyDeviceToHost, st);
    if (r == hipSuccess) r = hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != hipSuccess)
        return fail(r == hipErrorOutOfMemory ? RNSM_ENOMEM : RNSM_EDEVICE, "search tuning: %s",
                    hipGetErrorString(r));
    if (herr) return fail(RNSM_EINTERNAL, "search tuning: a search exceeded its iteration bound");
    out->hash_bits = best.hbits;
    out->waves_per_block = best.wpb;
    out->ms = best_ms;
    out->default_hash_bits = def.hbits;
    out->default_waves_per_block = def.wpb;
    out->default_ms = def_ms;
    out->n_queries = nq;
    out->n_tried = tried;
    return RNSM_OK;
}

// Layout of the static scratch in rnsm_search_noalloc: counters, error flag,
// then (cosine) base norms and query norms, each 256-byte aligned.
struct NoallocLayout {
    size_t cnt = 0, err = 0, bn = 0, qn = 0, total = 0;
};
static NoallocLayout noalloc_layout(int64_t n, int64_t nq, rnsm_metric metric) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    NoallocLayout l;
    l.cnt = 0;
    l.err = up(sizeof(u64) * CNT_SLOTS * CNT_N);
    l.bn = l.err + 256;
    l.total = l.bn;
    if (metric == RNSM_COSINE) {
        l.qn = up(l.bn + sizeof(float) * (size_t)n);
        l.total = l.qn + sizeof(float) * (size_t)nq;
    }
    return l;
}

static rnsm_status rnsm_search_noalloc_impl(const rnsm_graph* g, const rnsm_vectors* base,
                                            const void* queries, int64_t nq, const int32_t* seeds,
                                            int32_t n_seeds, int32_t ef, int32_t k,
                                            rnsm_metric metric, int32_t* out_ids, float* out_dists,
                                            void* stream) {
    g_err.clear();
    VecInfo vi;
    rnsm_status vs = search_check("rnsm_search_noalloc", g, base, queries, nq, seeds, n_seeds, ef,
                                  k, metric, out_ids, vi);
    if (vs != RNSM_OK) return vs;
    if (g->mem != RNSM_DEVICE || base->mem != RNSM_DEVICE ||
        (base->row_stride != 0 && base->row_stride != base->dim))
        return fail(RNSM_EUNSUPPORTED,
                    "rnsm_search_noalloc: graph and rows must be packed device memory");
    const NoallocLayout l = noalloc_layout(g->n, nq, metric);
    if (l.total > NOALLOC_SCRATCH_BYTES)
        return fail(RNSM_EINVAL,
                    "rnsm_search_noalloc: cosine norms of %lld base rows and %lld queries need "
                    "%zu bytes of scratch, above its %zu bytes",
                    (long long)g->n, (long long)nq, l.total, NOALLOC_SCRATCH_BYTES);
    if (nq == 0) return RNSM_OK;
    std::lock_guard<std::mutex> lk(g_lock);
    void* sp = nullptr;
    HIPCHK(noalloc_scratch(&sp));
    char* base_p = (char*)sp;
    SearchBufs b;
    b.cnt = (u64*)(base_p + l.cnt);
    b.errf = (int*)(base_p + l.err);
    if (metric == RNSM_COSINE) {
        b.bn = (float*)(base_p + l.bn);
        b.qn = (float*)(base_p + l.qn);
    }
    return search_run("rnsm_search_noalloc", g, base, vi, queries, nq, seeds, n_seeds, ef, k,
                      metric, out_ids, out_dists, (hipStream_t)stream, b);
}

static rnsm_status rnsm_tune_search_impl(const rnsm_graph* g, const rnsm_vectors* base, int32_t ef,
                             rnsm_metric metric, int64_t n_sample, rnsm_search_tuning* out,
                             void* stream) {
    g_err.clear();
    if (!g || !base || !out) return fail(RNSM_EINVAL, "rnsm_tune_search: NULL argument");
    memset(out, 0, sizeof *out);
    if (ef < 1 || ef > 128) return fail(RNSM_EINVAL, "rnsm_tune_search: ef outside 1..128");
    if (metric < RNSM_L2SQ || metric > RNSM_COSINE)
        return fail(RNSM_EINVAL, "rnsm_tune_search: metric");
    if (n_sample < 1) return fail(RNSM_EINVAL, "rnsm_tune_search: n_sample < 1");
    if (g->n < 1 || !g->offsets || !g->nbrs || base->n != g->n)
        return fail(RNSM_EINVAL, "rnsm_tune_search: graph / base mismatch");
    if (g->entry < 0 || g->entry >= g->n) return fail(RNSM_EINVAL, "rnsm_tune_search: entry");
    VecInfo vi;
    rnsm_status vs = vec_info(base, vi);
    if (vs != RNSM_OK) return vs;
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    Workspace& ws = g_ws[dev];
    ws.begin_call(0);
    rnsm_graph gs;
    rnsm_vectors vs2;
    if ((vs = stage_graph(ws, "rnsm_tune_search", 0, *g, st, gs)) != RNSM_OK) return vs;
    if ((vs = stage_vectors(ws, "rnsm_tune_search", *base, st, vs2)) != RNSM_OK) return vs;
    if ((vs = vec_info(&vs2, vi)) != RNSM_OK) return vs;
    return tune_shape_locked(&gs, &vs2, vi, ef, metric, n_sample, 32, out, st);
}

static rnsm_status rnsm_build_graph_impl(int64_t n, const float* X, int32_t dim, rnsm_metric metric,
                             const int32_t* knn, int32_t K, int32_t R, float alpha,
                             int32_t options, float alpha_rev, int64_t* out_offsets,
                             int32_t* out_nbrs, int32_t* out_entry, int64_t* out_links,
                             void* stream) {
    g_err.clear();
    if (out_links) *out_links = 0;
    if (options & ~(RNSM_BUILD_REVERSE | RNSM_BUILD_REPAIR))
        return fail(RNSM_EINVAL, "rnsm_build_graph: unknown option bits");
    const bool reverse = (options & RNSM_BUILD_REVERSE) != 0;
    if (n < 1 || !X || !knn || !out_offsets || !out_nbrs || !out_entry)
        return fail(RNSM_EINVAL, "rnsm_build_graph: bad argument");
    if (K < 1 || R < 1 || R > 64) return fail(RNSM_EINVAL, "rnsm_build_graph: K < 1 or R outside 1..64");
    if (!(alpha >= 1.0f) || (reverse && !(alpha_rev >= 1.0f)))
        return fail(RNSM_EINVAL, "rnsm_build_graph: alpha < 1");
    if (metric < RNSM_L2SQ || metric > RNSM_COSINE) return fail(RNSM_EINVAL, "rnsm_build_graph: metric");
    if (dim < 1 || (dim % 4) != 0) return fail(RNSM_EUNSUPPORTED, "rnsm_build_graph: dim must be a multiple of 4");
    const int nch = dim / 4, G = lanes_per_row(nch);
    if (G < 0) return fail(RNSM_EUNSUPPORTED, "rnsm_build_graph: dim does not split into whole chunks per lane");
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    Workspace& ws = g_ws[dev];
    ws.begin_call(0);
    int32_t *rows1, *deg1, *rows2, *deg2, *rc, *rcur, *rev, *errf;
    float *d1, *d2, *norms = nullptr;
    int64_t *roff, *stmp;
    u64* scratch;
    WS(rows1, "b_rows1", sizeof(int32_t) * n * R);
    WS(deg1, "b_deg1", sizeof(int32_t) * n);
    WS(d1, "b_d1", sizeof(float) * n * R);
    WS(errf, "b_err", sizeof(int));
    ValueInfo vinfo;
    {
        unsigned* vr;
        WS(vr, "value_range", sizeof(unsigned) * 3);
        HIPCHK(value_info(X, n, dim, vr, st, &vinfo));
    }
    const int pmode = choose_prune(vinfo, dim, R);
    char* xb16 = nullptr;
    if (pmode == 1) {
        WS(xb16, "b_prune_bf16", (size_t)2 * n * dim);
        HIPCHK(launch_convert(X, RNSM_F32, xb16, RNSM_BF16, n * (int64_t)dim, st));
    }
    HIPCHK(hipMemsetAsync(errf, 0, sizeof(int), st));
    if (metric == RNSM_COSINE) {
        WS(norms, "b_norms", sizeof(float) * n);
        HIPCHK(launch_norms(X, n, dim, norms, st));
    }
    PruneArgs q = {};
    q.X = X;
    q.xb = xb16;
    q.n_total = n;
    q.nch = nch;
    q.G = G;
    q.lgG = ilog2i(G);
    q.cpl = nch / G;
    q.metric = metric;
    q.norms = norms;
    q.n_items = n;
    q.item_base = 0;
    q.extra_mode = 1;
    q.extra_ids = knn;
    q.extra_stride = K;
    q.extra_cnt = K;
    q.alpha = alpha;
    q.R = R;
    q.rows_out = rows1;
    q.deg_out = deg1;
    q.dist_out = d1;
    q.wcap = K;
    q.err = errf;
    q.band = prune_band();
    HIPCHK(run_prune(q, pmode, st));
    int32_t *rows = rows1, *deg = deg1;
    if (reverse) {
        WS(rows2, "b_rows2", sizeof(int32_t) * n * R);
        WS(deg2, "b_deg2", sizeof(int32_t) * n);
        WS(d2, "b_d2", sizeof(float) * n * R);
        WS(rc, "b_rc", sizeof(int32_t) * n);
        WS(rcur, "b_rcur", sizeof(int32_t) * n);
        WS(roff, "b_roff", sizeof(int64_t) * (n + 1));
        WS(rev, "b_rev", sizeof(int32_t) * n * R);
        WS(stmp, "b_stmp", sizeof(int64_t) * scan_tmp_elems(n));
        WS(scratch, "b_scratch", sizeof(u64) * 4 * n * R);
        HIPCHK(hipMemsetAsync(rc, 0, sizeof(int32_t) * n, st));
        HIPCHK(hipMemsetAsync(rcur, 0, sizeof(int32_t) * n, st));
        HIPCHK(launch_rev_count(rows1, deg1, 0, n, R, 0, n, rc, st));
        HIPCHK(launch_scan(rc, n, roff, stmp, st));
        float* rev_d;
        WS(rev_d, "b_rev_d", sizeof(float) * n * R);
        HIPCHK(launch_rev_scatter(rows1, deg1, d1, 0, n, R, 0, n, roff, rcur, rev, rev_d, st));
        PruneArgs r = q;
        r.rows_in = rows1;
        r.deg_in = deg1;
        r.rows_d = d1;
        r.extra_mode = 2;
        r.extra_ids = rev;
        r.extra_d = rev_d;
        r.extra_off = roff;
        r.extra_index_base = 0;
        r.skip_empty_extra = 1;
        r.extra_sorted = 0;
        r.alpha = alpha_rev;
        r.rows_out = rows2;
        r.deg_out = deg2;
        r.dist_out = d2;
        r.scratch = scratch;
        r.wcap = 256;
        HIPCHK(run_prune(r, pmode, st));
        HIPCHK(launch_copy_rows(rows1, deg1, d1, rc, n, R, rows2, deg2, d2, st));
        rows = rows2;
        deg = deg2;
    }
    // entry: closest to the centroid
    int* flag;
    double* cs;
    unsigned long long* csi;
    u64* bb;
    const int64_t nb = entry_blocks(n);
    WS(flag, "b_flag", sizeof(int));
    WS(cs, "b_cs", sizeof(double) * dim);
    WS(csi, "b_csi", sizeof(unsigned long long) * dim);
    WS(bb, "b_best", sizeof(u64) * 3 * nb);
    const int one = 1;
    HIPCHK(hipMemcpyAsync(flag, &one, sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(cs, 0, sizeof(double) * dim, st));
    HIPCHK(hipMemsetAsync(csi, 0, sizeof(unsigned long long) * dim, st));
    HIPCHK(launch_entry(X, n, dim, flag, cs, csi, bb, nb, st));
    std::vector<u64> hb(3 * nb);
    int herr = 0;
    HIPCHK(hipMemcpyAsync(hb.data(), bb, sizeof(u64) * 3 * nb, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&herr, errf, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (herr & 4) return fail(RNSM_EINVAL, "rnsm_build_graph: a k-NN id is out of range");
    if (herr) return fail(RNSM_EINTERNAL, "rnsm_build_graph: prune candidate list over capacity");
    int64_t best = 0;
    for (int64_t b = 1; b < nb; ++b) {
        const u64* x = &hb[3 * b];
        const u64* y = &hb[3 * best];
        if (x[0] < y[0] || (x[0] == y[0] && (x[1] < y[1] || (x[1] == y[1] && x[2] < y[2])))) best = b;
    }
    const int32_t entry = (int32_t)hb[3 * best + 2];
    *out_entry = entry;
    if (options & RNSM_BUILD_REPAIR) {
        // reachability repair in passes (host-paced: a search from the entry,
        // the heads and their proposals, the acceptances)
        if ((size_t)dim * 16 * sizeof(float) > 64 * 1024)
            return fail(RNSM_EUNSUPPORTED, "rnsm_build_graph: the repair takes dim <= 1024");
        unsigned *vis, *ctl, *h_ctl;
        int32_t *order, *fb, *cand, *pt, *cnt, *cur;
        unsigned char* inu;
        unsigned long long *pk, *seg, *rctl, *h_rctl;
        int64_t *off, *rtmp;
        WS(vis, "b_vis", sizeof(unsigned) * ((n + 31) / 32));
        WS(order, "b_order", sizeof(int32_t) * n);
        WS(ctl, "b_ctl", sizeof(unsigned) * 4);
        WS(inu, "b_inu", ((n + 3) & ~3ll) + 4);  // whole words: k_rep_mark ORs 32-bit words
        WS(fb, "b_fb", sizeof(int32_t) * n);
        WS(cand, "b_cand", sizeof(int32_t) * n);
        WS(pt, "b_pt", sizeof(int32_t) * n);
        WS(cnt, "b_pcnt", sizeof(int32_t) * n);
        WS(cur, "b_pcur", sizeof(int32_t) * n);
        WS(pk, "b_pk", sizeof(unsigned long long) * n);
        WS(seg, "b_seg", sizeof(unsigned long long) * n);
        WS(off, "b_poff", sizeof(int64_t) * (n + 1));
        WS(rtmp, "b_pscan", sizeof(int64_t) * scan_tmp_elems(n));
        WS(rctl, "b_rctl", sizeof(unsigned long long) * 5);
        HS(h_ctl, "h_b_ctl", sizeof(unsigned) * 4);
        HS(h_rctl, "h_b_rctl", sizeof(unsigned long long) * 5);
        HIPCHK(launch_pad_tail(rows, deg, n, R, st));
        HIPCHK(launch_zero(rctl + 3, sizeof(unsigned long long), st));  // links
        for (int pass = 0; pass < 4096; ++pass) {
            HIPCHK(launch_bfs_init(n, entry, vis, order, ctl, st));
            HIPCHK(launch_bfs_grow(rows, R, n, order, vis, ctl, h_ctl, st));
            if ((int64_t)h_ctl[0] >= n) break;
            HIPCHK(launch_repair_heads(n, rows, deg, R, vis, inu, cnt, cur, rctl, st));
            HIPCHK(hipMemcpyAsync(h_rctl, rctl, sizeof(unsigned long long) * 2,
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            // heads: no unreached vertex links to them; when there are none,
            // no unreached vertex of smaller id
            const int64_t only = h_rctl[0] == 0 ? 1 : 0;
            if (h_rctl[1] >= (unsigned long long)n)
                return fail(RNSM_EINTERNAL, "rnsm_build_graph: repair found no unreached vertex");
            HIPCHK(launch_repair_propose(n, X, dim, metric, norms, knn, K, vis, inu, deg, R, only,
                                         pt, pk, fb, rctl, st));
            // heads with no reached free vertex in their list: a scan over
            // the reached vertices with a free slot (all reached ones when
            // no reached row has one)
            HIPCHK(launch_zero(rctl + 4, sizeof(unsigned long long), st));
            HIPCHK(launch_repair_cands(n, vis, deg, R, 0, cand, rctl + 4, st));
            HIPCHK(hipMemcpyAsync(h_rctl + 2, rctl + 2, sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(h_rctl + 4, rctl + 4, sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (h_rctl[2] > 0) {
                if (h_rctl[4] == 0) {
                    HIPCHK(launch_repair_cands(n, vis, deg, R, 1, cand, rctl + 4, st));
                    HIPCHK(hipMemcpyAsync(h_rctl + 4, rctl + 4, sizeof(unsigned long long),
                                          hipMemcpyDeviceToHost, st));
                    HIPCHK(hipStreamSynchronize(st));
                }
                HIPCHK(launch_repair_scan(n, X, dim, metric, norms, fb, (int64_t)h_rctl[2], cand,
                                          (int64_t)h_rctl[4], pt, pk, st));
            }
            HIPCHK(launch_repair_accept(n, vis, inu, only, pt, pk, cnt, cur, off, rtmp, seg, rows,
                                        deg, R, rctl + 3, st));
        }
        HIPCHK(hipMemcpyAsync(h_rctl + 3, rctl + 3, sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (out_links) *out_links = (int64_t)h_rctl[3];
    }
    int64_t* stmp3;
    WS(stmp3, "b_stmp3", sizeof(int64_t) * scan_tmp_elems(n));
    HIPCHK(launch_scan(deg, n, out_offsets, stmp3, st));
    HIPCHK(launch_compact(rows, deg, d1, out_offsets, n, R, X, dim, metric, norms, out_nbrs, nullptr, st));
    HIPCHK(hipStreamSynchronize(st));
    return RNSM_OK;
}

static rnsm_status rnsm_reachable_impl(int64_t n, const int64_t* offsets, const int32_t* nbrs,
                                       int32_t entry, int64_t* out_count, void* stream) {
    g_err.clear();
    if (!out_count || n < 1 || !offsets || !nbrs || entry < 0 || entry >= n || n > INT32_MAX)
        return fail(RNSM_EINVAL, "rnsm_reachable: bad argument");
    *out_count = 0;
    std::lock_guard<std::mutex> lk(g_lock);
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    Workspace& ws = g_ws[dev];
    ws.begin_call(0);
    unsigned *md, *h_md;
    int* bad;
    WS(md, "r_shape", sizeof(unsigned) * 2);
    HS(h_md, "h_r_shape", sizeof(unsigned) * 2);
    bad = reinterpret_cast<int*>(md + 1);
    HIPCHK(launch_zero(md, sizeof(unsigned) * 2, st));
    HIPCHK(launch_csr_shape(offsets, n, md, bad, st));
    HIPCHK(hipMemcpyAsync(h_md, md, sizeof(unsigned) * 2, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h_md[1]) return fail(RNSM_EINVAL, "rnsm_reachable: malformed offsets");
    const int rp = std::max(1u, h_md[0]);
    int32_t *padj, *order;
    unsigned *vis, *ctl, *h_ctl;
    WS(padj, "r_padj", sizeof(int32_t) * n * rp);
    WS(order, "r_order", sizeof(int32_t) * n);
    WS(vis, "r_vis", sizeof(unsigned) * ((n + 31) / 32));
    WS(ctl, "r_ctl", sizeof(unsigned) * 4);
    HS(h_ctl, "h_r_ctl", sizeof(unsigned) * 4);
    HIPCHK(launch_pad_adjacency(offsets, nbrs, n, rp, padj, st));
    HIPCHK(launch_bfs_init(n, entry, vis, order, ctl, st));
    HIPCHK(launch_bfs_grow(padj, rp, n, order, vis, ctl, h_ctl, st));
    *out_count = std::min<int64_t>(n, h_ctl[0]);
    return RNSM_OK;
}

// ------------------------------------------------------------- the C ABI
// Every entry point runs its body under guard(): no C++ exception crosses the
// boundary (std::bad_alloc becomes RNSM_ENOMEM, anything else RNSM_EINTERNAL).
// After a failed merge the device is drained, so that no queued work still
// reads the library's buffers when the next call reuses them.
namespace {
template <class F>
rnsm_status guard(const char* fn, F&& body) {
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return fail(RNSM_ENOMEM, "%s: host allocation failed", fn);
    } catch (const std::exception& e) {
        return fail(RNSM_EINTERNAL, "%s: %s", fn, e.what());
    } catch (...) {
        return fail(RNSM_EINTERNAL, "%s: unexpected exception", fn);
    }
}
}  // namespace

extern "C" {

rnsm_status rnsm_convert(const void* src, rnsm_dtype src_type, void* dst, rnsm_dtype dst_type,
                         int64_t count, void* stream) {
    return guard("rnsm_convert", [&] { return rnsm_convert_impl(src, src_type, dst, dst_type, count, stream); });
}

void rnsm_csr_free(rnsm_csr* g) {
    if (!g || g->mem != RNSM_HOST) return;
    free(g->offsets);
    free(g->nbrs);
    free(g->dists);
    memset(g, 0, sizeof *g);
}

rnsm_status rnsm_get_stats(rnsm_stats* out) {
    return guard("rnsm_get_stats", [&] { return rnsm_get_stats_impl(out); });
}

rnsm_status mos_plan(int32_t m, const int64_t* sizes, const double* centroids, int32_t dim,
                     int32_t degree_bound, int32_t diameter, int32_t* out_ops, int32_t cap,
                     int32_t* out_count, int32_t* out_fallbacks) {
    return guard("mos_plan", [&] { return mos_plan_impl(m, sizes, centroids, dim, degree_bound, diameter, out_ops, cap, out_count, out_fallbacks); });
}

rnsm_status rnsm_select_pivots(int64_t n, const int64_t* rk_offsets, const int32_t* rk_ids,
                               int32_t* pivots, int64_t* out_n_pivots, int32_t* followers,
                               int32_t* follower_pivot, int64_t* out_n_followers) {
    return guard("rnsm_select_pivots", [&] { return rnsm_select_pivots_impl(n, rk_offsets, rk_ids, pivots, out_n_pivots, followers, follower_pivot, out_n_followers); });
}

rnsm_status rnsm_merge(int32_t m, const rnsm_graph* graphs, const rnsm_vectors* vecs,
                       const rnsm_params* p, rnsm_csr* out) {
    const rnsm_status r = guard("rnsm_merge", [&] { return rnsm_merge_impl(m, graphs, vecs, p, out); });
    if (r == RNSM_EDEVICE || r == RNSM_ENOMEM || r == RNSM_EINTERNAL) (void)hipDeviceSynchronize();
    return r;
}

rnsm_status rnsm_merge_simple(int32_t m, const rnsm_graph* graphs, const rnsm_vectors* vecs,
                              int32_t R, int32_t L, float alpha, rnsm_csr* out) {
    return guard("rnsm_merge_simple", [&] { return rnsm_merge_simple_impl(m, graphs, vecs, R, L, alpha, out); });
}

rnsm_status rnsm_search(const rnsm_graph* g, const rnsm_vectors* base, const void* queries,
                        int64_t nq, const int32_t* seeds, int32_t n_seeds, int32_t ef, int32_t k,
                        rnsm_metric metric, int32_t* out_ids, float* out_dists, void* stream) {
    return guard("rnsm_search", [&] { return rnsm_search_impl(g, base, queries, nq, seeds, n_seeds, ef, k, metric, out_ids, out_dists, stream); });
}

rnsm_status rnsm_search_noalloc(const rnsm_graph* g, const rnsm_vectors* base,
                                const void* queries, int64_t nq, const int32_t* seeds,
                                int32_t n_seeds, int32_t ef, int32_t k, rnsm_metric metric,
                                int32_t* out_ids, float* out_dists, void* stream) {
    return guard("rnsm_search_noalloc", [&] {
        return rnsm_search_noalloc_impl(g, base, queries, nq, seeds, n_seeds, ef, k, metric,
                                        out_ids, out_dists, stream);
    });
}

rnsm_status rnsm_select_pivots_device(int64_t n, const int64_t* rk_offsets, const int32_t* rk_ids,
                                      int32_t* pivot_of, int64_t* out_n_pivots, void* stream) {
    return guard("rnsm_select_pivots_device", [&] {
        return rnsm_select_pivots_device_impl(n, rk_offsets, rk_ids, pivot_of, out_n_pivots,
                                              stream);
    });
}

rnsm_status rnsm_tune_search(const rnsm_graph* g, const rnsm_vectors* base, int32_t ef,
                             rnsm_metric metric, int64_t n_sample, rnsm_search_tuning* out,
                             void* stream) {
    return guard("rnsm_tune_search", [&] { return rnsm_tune_search_impl(g, base, ef, metric, n_sample, out, stream); });
}

rnsm_status rnsm_build_graph(int64_t n, const float* X, int32_t dim, rnsm_metric metric,
                             const int32_t* knn, int32_t K, int32_t R, float alpha,
                             int32_t options, float alpha_rev, int64_t* out_offsets,
                             int32_t* out_nbrs, int32_t* out_entry, int64_t* out_links,
                             void* stream) {
    return guard("rnsm_build_graph", [&] { return rnsm_build_graph_impl(n, X, dim, metric, knn, K, R, alpha, options, alpha_rev, out_offsets, out_nbrs, out_entry, out_links, stream); });
}

rnsm_status rnsm_reachable(int64_t n, const int64_t* offsets, const int32_t* nbrs, int32_t entry,
                           int64_t* out_count, void* stream) {
    return guard("rnsm_reachable", [&] { return rnsm_reachable_impl(n, offsets, nbrs, entry, out_count, stream); });
}

}  // extern "C"
