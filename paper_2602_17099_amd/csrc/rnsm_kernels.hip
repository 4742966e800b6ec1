// Device kernels of the RNSM merge path for gfx950 (CDNA4, 64-lane
// wavefronts).
//
//  - k_beam_search: Algorithm 1 (Section 2.2), one wavefront per query. The
//    beam is a sorted array of 64-bit keys (order-preserving float bits of
//    the distance << 32 | id) held one or two per lane; the nearest
//    unexpanded entry is found with a ballot; new entries are placed with a
//    ballot-count and a one-lane shift. The visited set is an open-addressing
//    table in LDS; when a probe sequence is full the vertex is evaluated
//    again and an exact key match in the beam drops the duplicate, which
//    leaves the final beam unchanged (a re-evaluated vertex that is not in
//    the beam has a key above the current worst, because the worst key of a
//    full beam only decreases). Distances: G lanes per row, 16-byte
//    coalesced loads, float32 accumulation, butterfly reduction.
//  - k_prune: the edge-selection rule of Section 2.2 as used by UpdateGraph
//    (Section 4.2): candidates are extracted in (distance, id) order by a
//    wavefront min-reduction; each one is tested against the kept rows,
//    which stay in registers.
//  - reverse-edge count/scatter, reverse k-NN inversion, scans, compaction,
//    input validation and the builder's entry point.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>

#include "rnsm_internal.h"

namespace rnsm {

#define WAVE 64
#define EMPTY_KEY (~0ull)

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ unsigned fkey(float d) {
    d = d + 0.0f;  // -0 -> +0
    unsigned u = __float_as_uint(d);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float fval(unsigned k) {
    unsigned u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}
__device__ __forceinline__ u64 make_key(float d, int id) {
    return ((u64)fkey(d) << 32) | (unsigned)id;
}
__device__ __forceinline__ u64 readlane64(u64 x, int l) {
    unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x & 0xffffffffu), l);
    unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), l);
    return ((u64)hi << 32) | lo;
}
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }
__device__ __forceinline__ u64 lanemask_lt(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}
__device__ __forceinline__ u64 wave_min_u64(u64 x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        u64 o = __shfl_xor(x, off);
        x = o < x ? o : x;
    }
    return x;
}

// blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical blocks so that neighbouring work items share
// one L2
__device__ __forceinline__ int64_t xcd_block() {
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t x = b & 7, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// 16-byte chunk -> floats (f32: 4 values, bf16 / f16: 8 values)
template <int TT>
struct Elt {
    static constexpr int EPC = TT == 0 ? 4 : 8;
};

template <int TT>
__device__ __forceinline__ void cvt_chunk(const uint4 r, float* f) {
    if constexpr (TT == 0) {
        f[0] = __uint_as_float(r.x);
        f[1] = __uint_as_float(r.y);
        f[2] = __uint_as_float(r.z);
        f[3] = __uint_as_float(r.w);
    } else if constexpr (TT == 1) {
        const unsigned w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f[2 * i] = __uint_as_float(w[i] << 16);
            f[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
        }
    } else {
        const unsigned w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            union { unsigned short s; _Float16 h; } lo, hi;
            lo.s = (unsigned short)(w[i] & 0xffffu);
            hi.s = (unsigned short)(w[i] >> 16);
            f[2 * i] = (float)lo.h;
            f[2 * i + 1] = (float)hi.h;
        }
    }
}

__device__ __forceinline__ float finalize_dist(float acc, int metric, float na, float nb) {
    if (metric == 0) return acc;
    if (metric == 1) return 1.0f - acc;
    return 1.0f - acc / (na * nb);
}

// ------------------------------------------------------------ beam search

template <int EFS>
struct Beam {
    u64 k[EFS];
    unsigned e[EFS];  // expanded flag
};

// DPP moves (gfx9 controls): the source lane's value, `old` where there is none
#define DPP_ROW_SHR(n) (0x110 + (n))
#define DPP_WAVE_SHR1 0x138
#define DPP_ROW_BCAST15 0x142
#define DPP_ROW_BCAST31 0x143

template <int CTRL>
__device__ __forceinline__ float dpp_add_src(float v) {
    // value of the DPP source lane, 0 where the source is out of range
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ unsigned wave_shr1(unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_WAVE_SHR1, 0xF, 0xF, false);
}

// sum over each aligned group of G lanes (G a uniform power of two); the
// total is valid in the group's last lane (sub == G-1)
__device__ __forceinline__ float group_sum_last(float v, int G) {
    if (G >= 2) v += dpp_add_src<DPP_ROW_SHR(1)>(v);
    if (G >= 4) v += dpp_add_src<DPP_ROW_SHR(2)>(v);
    if (G >= 8) v += dpp_add_src<DPP_ROW_SHR(4)>(v);
    if (G >= 16) v += dpp_add_src<DPP_ROW_SHR(8)>(v);
    if (G >= 32) v += dpp_add_src<DPP_ROW_BCAST15>(v);
    if (G >= 64) v += dpp_add_src<DPP_ROW_BCAST31>(v);
    return v;
}

template <int EFS>
__device__ __forceinline__ u64 beam_worst(const Beam<EFS>& B, int ef) {
    const int s = ef - 1;
    if constexpr (EFS == 1) {
        return readlane64(B.k[0], s);
    } else {
        return (s >= 64) ? readlane64(B.k[1], s - 64) : readlane64(B.k[0], s);
    }
}

__device__ __forceinline__ u64 shr1_u64(u64 x) {
    return ((u64)wave_shr1((unsigned)(x >> 32)) << 32) | wave_shr1((unsigned)(x & 0xffffffffu));
}

// insert key into the sorted beam of capacity ef; drops exact duplicates
// (a vertex evaluated again after the visited table forgot it)
template <int EFS>
__device__ __forceinline__ void beam_insert(Beam<EFS>& B, u64 key, int ef, int lane) {
    u64 lt = __ballot(B.k[0] < key);
    u64 eq = __ballot(B.k[0] == key);
    int pos = __popcll(lt);
    if constexpr (EFS == 2) {
        lt = __ballot(B.k[1] < key);
        eq |= __ballot(B.k[1] == key);
        pos += __popcll(lt);
    }
    if (eq != 0ull || pos >= ef) return;
    // selects rather than branches: every lane takes its new value with
    // v_cndmask, lanes at or past ef keep their empty slot
    if constexpr (EFS == 1) {
        const u64 up = shr1_u64(B.k[0]);
        const unsigned eup = wave_shr1(B.e[0]);
        const bool sh = lane > pos && lane < ef, at = lane == pos;
        B.k[0] = at ? key : (sh ? up : B.k[0]);
        B.e[0] = at ? 0u : (sh ? eup : B.e[0]);
    } else {
        const u64 a63 = readlane64(B.k[0], 63);
        const unsigned e63 = (unsigned)__builtin_amdgcn_readlane((int)B.e[0], 63);
        const u64 upa = shr1_u64(B.k[0]);
        const unsigned eupa = wave_shr1(B.e[0]);
        const u64 upb = shr1_u64(B.k[1]);
        const unsigned eupb = wave_shr1(B.e[1]);
        const bool sha = lane > pos && lane < ef, ata = lane == pos;
        B.k[0] = ata ? key : (sha ? upa : B.k[0]);
        B.e[0] = ata ? 0u : (sha ? eupa : B.e[0]);
        const int sb = 64 + lane;
        const u64 pb = lane == 0 ? a63 : upb;
        const unsigned peb = lane == 0 ? e63 : eupb;
        const bool shb = sb > pos && sb < ef, atb = sb == pos;
        B.k[1] = atb ? key : (shb ? pb : B.k[1]);
        B.e[1] = atb ? 0u : (shb ? peb : B.e[1]);
    }
}

// Visited set in LDS (4 << hbits bytes). Forgetful form: 2^hbits sets of two
// 16-bit tags in one 32-bit word; vertex v goes to set (v ^ (v >> b)) mod
// 2^b and its tag is v >> b (b = hbits), so (set, tag) identifies v while
// v < 0xffff << b (0xffff marks an empty tag). A new vertex takes the low
// half and moves the earlier one to the high half, whose vertex is
// forgotten. A plain read then a write: two lanes that meet in one set in the
// same instruction may lose one of their tags, which only re-evaluates a
// vertex. Exact form: 32-bit ids with linear probing (up to 64 probes).
// Returns 0 if v was already there, 1 if it went into an empty place, 2 if
// it made the set forget another vertex (or found no slot).
template <bool EXACT>
__device__ __forceinline__ int hash_visit(int* tab, int hbits, int v) {
    if constexpr (!EXACT) {
        const unsigned b = (unsigned)hbits;
        const unsigned hi = (unsigned)v >> b;
        const unsigned set = ((unsigned)v ^ hi) & ((1u << b) - 1u);
        const unsigned old = (unsigned)tab[set];
        if ((old & 0xffffu) == hi || (old >> 16) == hi) return 0;
        tab[set] = (int)((old << 16) | hi);
        return (old >> 16) == 0xffffu ? 1 : 2;
    } else {
        const unsigned h = ((unsigned)v * 2654435761u) >> (32 - hbits);
        const unsigned mask = (1u << hbits) - 1u;
        for (int p = 0; p < 64; ++p) {
            const int old = atomicCAS(&tab[(h + p) & mask], -1, v);
            if (old == -1) return 1;
            if (old == v) return 0;
        }
        return 2;
    }
}

// the query row in the searched copy's layout: float32 values, or the packed
// 16-bit chunks (consumed two at a time by v_dot2)
template <int TT, int CPL>
struct Query {
    float q[CPL][TT == 0 ? 4 : 1];
    uint4 r[TT == 0 ? 1 : CPL];
};

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 halfx2_t __attribute__((ext_vector_type(2)));

// acc + a.lo * b.lo + a.hi * b.hi over two packed 16-bit values
template <int TT>
__device__ __forceinline__ float dot2(unsigned a, unsigned b, float acc) {
    if constexpr (TT == 1)
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a),
                                               __builtin_bit_cast(bf16x2_t, b), acc, false);
    else
        return __builtin_amdgcn_fdot2(__builtin_bit_cast(halfx2_t, a), __builtin_bit_cast(halfx2_t, b),
                                      acc, false);
}
template <int TT>
__device__ __forceinline__ float dot2x4(uint4 a, uint4 b, float acc) {
    acc = dot2<TT>(a.x, b.x, acc);
    acc = dot2<TT>(a.y, b.y, acc);
    acc = dot2<TT>(a.z, b.z, acc);
    return dot2<TT>(a.w, b.w, acc);
}

// per wavefront: the visited table, the compacted candidate list and the
// adjacency slot of each compacted candidate
__host__ __device__ constexpr int search_lds_words(int hbits) { return (1 << hbits) + 128; }

// evaluate the per-lane candidates v (-1: none): visited filter, distances,
// beam insertion. Rows are read by groups of G lanes, CPL 16-byte chunks per
// lane at a stride of G chunks, UNR rows per group per batch.
// Distances: float32 copies sum (q - x)^2 (or q x) per element; 16-bit
// copies use v_dot2 on the packed values, squared L2 as |q|^2 + |x|^2 - 2 q.x
// combined in double (exact whenever the three sums are, e.g. small integers).
// qn: the query's norm (cosine) or squared norm (squared L2, 16-bit copies).
template <int TT, int EFS, int CPL, bool EXACT, int LG>
__device__ __forceinline__ void process_candidates(const SearchArgs& a, Beam<EFS>& B,
                                                   const Query<TT, CPL>& Q, float qn, int* tab,
                                                   int* cl, int v, int lane, u64& ndc,
                                                   u64& nevict, float* rec = nullptr) {
    constexpr int EPC = Elt<TT>::EPC;
    // rows per lane group per batch: two for float32 rows (more loads in
    // flight); one for 16-bit rows, whose 72-78 VGPRs then allow 6 resident
    // wavefronts per SIMD (measured faster for them, slower for float32)
    constexpr int UNR = TT == 0 ? 2 : 1;
    int st = 0;
    if (v >= a.n) v = -1;  // ids from callers are range-checked
    if (v >= 0) st = hash_visit<EXACT>(tab, a.hbits, v);
    nevict += __popcll(__ballot(st == 2));
    const u64 m = __ballot(st != 0);
    const int nc = __popcll(m);
    if (nc == 0) return;
    if (st != 0) {
        const int rk = __popcll(m & lanemask_lt(lane));
        cl[rk] = v;
        cl[WAVE + rk] = lane;  // adjacency slot, for rec
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    ndc += nc;
    // lanes per row: a constant in the instances for the common shapes
    // (LG = log2 G), so that the group sums and indexing fold
    const int lgG = LG >= 0 ? LG : a.lgG, G = 1 << lgG, RPP = WAVE >> lgG;
    const int group = lane >> lgG, sub = lane & (G - 1);
    const int64_t gstride = (int64_t)G * 16;
    for (int c0 = 0; c0 < nc; c0 += RPP * UNR) {
        uint4 raw[UNR][CPL];
        int cid[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int c = c0 + u * RPP + group;
            cid[u] = c < nc ? cl[c] : -1;
            if (cid[u] >= 0) {
                const char* rp = a.base + (int64_t)cid[u] * a.row_bytes + sub * 16;
#pragma unroll
                for (int j = 0; j < CPL; ++j) raw[u][j] = *(const uint4*)(rp + j * gstride);
            }
        }
        float acc[UNR], xx[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            float s = 0.0f, s2 = 0.0f;
            if constexpr (TT == 0) {
#pragma unroll
                for (int j = 0; j < CPL; ++j) {
                    float x[EPC];
                    cvt_chunk<TT>(raw[u][j], x);
                    if (a.metric == 0) {
#pragma unroll
                        for (int t = 0; t < EPC; ++t) {
                            const float d = Q.q[j][t] - x[t];
                            s = fmaf(d, d, s);
                        }
                    } else {
#pragma unroll
                        for (int t = 0; t < EPC; ++t) s = fmaf(Q.q[j][t], x[t], s);
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < CPL; ++j) {
                    s = dot2x4<TT>(Q.r[j], raw[u][j], s);
                    if (a.metric == 0) s2 = dot2x4<TT>(raw[u][j], raw[u][j], s2);
                }
            }
            acc[u] = group_sum_last(s, G);
            xx[u] = (TT != 0 && a.metric == 0) ? group_sum_last(s2, G) : 0.0f;
        }
        const u64 worst = beam_worst(B, a.ef);
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            u64 key = EMPTY_KEY;
            if (sub == G - 1 && cid[u] >= 0) {
                float nb = 1.0f;
                if (a.metric == 2) nb = a.base_norm[cid[u]];
                float d;
                if (TT != 0 && a.metric == 0)
                    d = (float)((double)qn + (double)xx[u] - 2.0 * (double)acc[u]);
                else
                    d = finalize_dist(acc[u], a.metric, qn, nb);
                key = make_key(d, cid[u]);
                if (rec) rec[cl[WAVE + c0 + u * RPP + group]] = d;
            }
            u64 mm = __ballot(key < worst);
            while (mm) {
                const int l = __ffsll((long long)mm) - 1;
                mm &= mm - 1;
                beam_insert(B, readlane64(key, l), a.ef, lane);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// distance counts of a wavefront's searches
struct SearchCounts {
    u64 ndc = 0, nexp = 0, nadj = 0, nevict = 0;
};

// Algorithm 1 for one query, by one wavefront: query row u of a.qvec,
// seeds by seed_mode (0: a.entry, 1: u itself, 2: the n_seeds ids at sp, -1
// and out-of-range ids skipped), the final beam to output row orow. tab / cl:
// this wavefront's LDS visited table and candidate list (the table is
// cleared here).
template <int TT, int EFS, int CPL, bool EXACT, int LG>
__device__ __forceinline__ void search_one(const SearchArgs& a, int u, int seed_mode,
                                           const int32_t* sp, int n_seeds, int64_t orow,
                                           int* tab, int* cl, int lane, SearchCounts& cnt) {
    const int H = 1 << a.hbits;
    for (int t = lane; t < H; t += WAVE) tab[t] = -1;
    __builtin_amdgcn_wave_barrier();

    const int G = LG >= 0 ? (1 << LG) : a.G;
    const int sub = lane & (G - 1);
    const char* qrow = a.qvec + (int64_t)u * a.row_bytes + sub * 16;
    Query<TT, CPL> Q;
    float qn = a.metric == 2 ? a.q_norm[u] : 1.0f;
    if constexpr (TT == 0) {
#pragma unroll
        for (int j = 0; j < CPL; ++j)
            cvt_chunk<TT>(*(const uint4*)(qrow + (int64_t)j * G * 16), Q.q[j]);
    } else {
        float s2 = 0.0f;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            Q.r[j] = *(const uint4*)(qrow + (int64_t)j * G * 16);
            s2 = dot2x4<TT>(Q.r[j], Q.r[j], s2);
        }
        // squared norm of the query (valid in the last lane of each group,
        // the lanes that form the keys)
        const float qq = group_sum_last(s2, G);
        if (a.metric == 0) qn = qq;
    }

    Beam<EFS> B;
#pragma unroll
    for (int s = 0; s < EFS; ++s) {
        B.k[s] = EMPTY_KEY;
        B.e[s] = 0;
    }
    u64 ndc = 0, nexp = 0, nadj = 0, nevict = 0;

    // seeds
    if (seed_mode == 0 || seed_mode == 1) {
        const int s0 = seed_mode == 0 ? a.entry : u;
        process_candidates<TT, EFS, CPL, EXACT, LG>(a, B, Q, qn, tab, cl, lane == 0 ? s0 : -1, lane, ndc,
                                       nevict);
    } else {
        for (int j0 = 0; j0 < n_seeds; j0 += WAVE) {
            const int j = j0 + lane;
            const int v = j < n_seeds ? sp[j] : -1;
            process_candidates<TT, EFS, CPL, EXACT, LG>(a, B, Q, qn, tab, cl, v, lane, ndc, nevict);
        }
    }
    // expand the nearest unexpanded entry until every entry is expanded
    const int64_t maxit = a.n + 2;
    int pf_uid = -1, pf_v = -1;  // adjacency fetched ahead for the runner-up entry
    for (int64_t it = 0;; ++it) {
        u64 m0 = __ballot(B.k[0] != EMPTY_KEY && B.e[0] == 0u);
        int s;
        if (m0) {
            s = __ffsll((long long)m0) - 1;
        } else {
            if constexpr (EFS == 2) {
                u64 m1 = __ballot(B.k[1] != EMPTY_KEY && B.e[1] == 0u);
                if (!m1) break;
                s = 64 + __ffsll((long long)m1) - 1;
            } else {
                break;
            }
        }
        int uid;
        if (s < 64) {
            if (lane == s) B.e[0] = 1u;
            uid = __builtin_amdgcn_readlane((int)(unsigned)(B.k[0] & 0xffffffffu), s);
        } else {
            if constexpr (EFS == 2) {
                if (lane == s - 64) B.e[1] = 1u;
                uid = __builtin_amdgcn_readlane((int)(unsigned)(B.k[1] & 0xffffffffu), s - 64);
            } else {
                uid = 0;
            }
        }
        ++nexp;
        if (a.padj) {
            // padded adjacency: one load, no offsets lookup (already in flight
            // when the entry was the runner-up of the previous expansion)
            const int v = uid == pf_uid ? pf_v : (lane < a.rp ? a.padj[(int64_t)uid * a.rp + lane] : -1);
            // the next unexpanded entry of the sorted beam is expanded next
            // unless this expansion inserts a nearer one: fetch its adjacency
            // now, so that its latency overlaps this expansion's row loads
            pf_uid = -1;
            {
                const u64 mA = __ballot(B.k[0] != EMPTY_KEY && B.e[0] == 0u);
                int s2 = -1;
                if (mA) {
                    s2 = __ffsll((long long)mA) - 1;
                    pf_uid = __builtin_amdgcn_readlane((int)(unsigned)(B.k[0] & 0xffffffffu), s2);
                } else {
                    if constexpr (EFS == 2) {
                        const u64 mB = __ballot(B.k[1] != EMPTY_KEY && B.e[1] == 0u);
                        if (mB) {
                            s2 = __ffsll((long long)mB) - 1;
                            pf_uid = __builtin_amdgcn_readlane((int)(unsigned)(B.k[1] & 0xffffffffu), s2);
                        }
                    }
                }
                if (pf_uid >= 0) pf_v = lane < a.rp ? a.padj[(int64_t)pf_uid * a.rp + lane] : -1;
            }
            nadj += (u64)__popcll(__ballot(v >= 0));
            // the seed's own first expansion evaluates every neighbour of u
            float* rec = (a.row_d && it == 0 && uid == u)
                             ? a.row_d + (a.row_d_base + u) * a.row_d_stride
                             : nullptr;
            process_candidates<TT, EFS, CPL, EXACT, LG>(a, B, Q, qn, tab, cl, v, lane, ndc, nevict, rec);
        } else {
            const int64_t b = a.offs[uid], en = a.offs[uid + 1];
            nadj += (u64)(en - b);
            for (int64_t j0 = b; j0 < en; j0 += WAVE) {
                const int64_t j = j0 + lane;
                const int v = j < en ? a.nbrs[j] : -1;
                process_candidates<TT, EFS, CPL, EXACT, LG>(a, B, Q, qn, tab, cl, v, lane, ndc, nevict);
            }
        }
        if (it > maxit) {
            if (lane == 0) atomicOr(a.err, 1);
            break;
        }
    }

    // write the result
    int32_t* oi = a.out_ids + orow * a.out_stride;
    float* od = a.out_d ? a.out_d + orow * a.out_stride : nullptr;
    if (a.out_mode == 0) {
#pragma unroll
        for (int s = 0; s < EFS; ++s) {
            const int slot = s * 64 + lane;
            if (slot < a.out_k) {
                const u64 kk = B.k[s];
                oi[slot] = kk != EMPTY_KEY ? (int)(unsigned)(kk & 0xffffffffu) : -1;
                if (od) od[slot] = kk != EMPTY_KEY ? fval((unsigned)(kk >> 32)) : INFINITY;
            }
        }
    } else {
        const u64 kk = B.k[0];
        const bool valid = kk != EMPTY_KEY;
        const bool self = valid && (int)(unsigned)(kk & 0xffffffffu) == u;
        const u64 sm = __ballot(self);
        const int cnt = __popcll(__ballot(valid && !self));
        const int pos = lane - __popcll(sm & lanemask_lt(lane));
        if (valid && !self && pos < a.out_k) {
            oi[pos] = (int)(unsigned)(kk & 0xffffffffu);
            if (od) od[pos] = fval((unsigned)(kk >> 32));
        }
        if (lane >= cnt && lane < a.out_k) {
            oi[lane] = -1;
            if (od) od[lane] = INFINITY;
        }
    }
    cnt.ndc += ndc;
    cnt.nexp += nexp;
    cnt.nadj += nadj;
    cnt.nevict += nevict;
}

// one wavefront's counts into a launch's counters, spread over CNT_SLOTS
// copies to keep the atomics of hundreds of thousands of wavefronts from
// meeting on one address
__device__ __forceinline__ void add_counts(u64* counters, const SearchCounts& c, int lane) {
    if (lane == 0) {
        u64* p = counters + (blockIdx.x & (CNT_SLOTS - 1)) * CNT_N;
        atomicAdd(&p[CNT_NDC], c.ndc);
        atomicAdd(&p[CNT_EXP], c.nexp);
        atomicAdd(&p[CNT_ADJ], c.nadj);
        atomicAdd(&p[CNT_HFULL], c.nevict);
    }
}

template <int TT, int EFS, int CPL, bool EXACT, int LG>
__global__ __launch_bounds__(256) void k_beam_search(SearchArgs a) {
    extern __shared__ int smem[];
    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int64_t i = xcd_block() * wpb + wib;
    if (i >= a.nq) return;
    int* tab = smem + (int64_t)wib * search_lds_words(a.hbits);
    int* cl = tab + (1 << a.hbits);
    const int u = a.qidx ? a.qidx[i] : (int)i;
    const int32_t* sp = nullptr;
    if (a.seed_mode == 2) sp = a.seed_ids + (a.seed_row ? a.seed_row[i] : i) * a.seed_stride;
    const int64_t orow = a.out_row ? a.out_row[i] : i;
    SearchCounts c;
    search_one<TT, EFS, CPL, EXACT, LG>(a, u, a.seed_mode, sp, a.n_seeds, orow, tab, cl, lane, c);
    add_counts(a.counters, c, lane);
}

// The searches of a round's operations in one persistent launch. A work item
// is a pivot group: the pivot's naive search from the target's entry, then
// each follower's local sliding seeded with the pivot's final beam, which the
// same wavefront has just written (so no wavefront waits on another). The
// groups (in breadth-first order of the pivots within each operation) are
// cut into 8 contiguous ranges, one per XCD (blocks are dispatched to the
// XCDs in turn): a wavefront takes the groups of its XCD's range, then those
// of the other ranges, through one atomic counter per range. Every
// wavefront ends when all ranges are drained.
// One call site of the search for the pivot and its followers, and the
// wavefront's counts in LDS, keep the registers near the plain search's
// (float32 rows 103 VGPRs, 4 wavefronts per SIMD; 16-bit rows 87). The
// 16-bit instance is held to 6 wavefronts per SIMD (80 VGPRs, 36 bytes a lane
// spilled): 7.0 against 7.5 ms at 5 and 8.5 ms at 4 on 2 x 500,000; a bound
// of 5 on the float32 instance measured no faster.
template <int TT, int EFS, int CPL, bool EXACT, int LG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TT == 0 ? 1 : 6)))
void k_group_search(GroupArgs g) {
    extern __shared__ int smem[];
    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    int* tab = smem + (int64_t)wib * search_lds_words(g.hbits);
    int* cl = tab + (1 << g.hbits);
    const int xcd = blockIdx.x & 7;
    __shared__ u64 wcnt[4][8];  // per wavefront: pivots' counts, followers' counts
    if (lane < 8) wcnt[wib][lane] = 0;
    for (int r = 0; r < 8; ++r) {
        const int rng = (xcd + r) & 7;
        const int64_t lo = g.n_groups * rng / 8, hi = g.n_groups * (rng + 1) / 8;
        for (;;) {
            unsigned t = 0;
            if (lane == 0) t = atomicAdd(&g.next[rng], 1u);
            // wavefront-uniform (scalar) from here on: the op's arguments
            // are then scalar loads
            const int64_t gi = lo + (int64_t)(unsigned)__builtin_amdgcn_readfirstlane((int)t);
            if (gi >= hi) break;
            // the op table through the constant address space: scalar loads
            // (the host pass of this kernel, never run, reads it plainly)
#if defined(__HIP_DEVICE_COMPILE__)
            typedef const __attribute__((address_space(4))) GroupOp CGroupOp;
            CGroupOp* ops = (CGroupOp*)g.ops;
#else
            const GroupOp* ops = g.ops;
#endif
            int k = 0;
            while (k + 1 < g.n_ops && ops[k + 1].group_base <= gi) ++k;
            const int64_t j = gi - ops[k].group_base;
            const int p = ops[k].gpiv[j];
            const int64_t f0 = ops[k].fbeg[j];
            const int64_t f1 = min(ops[k].fbeg[j + 1], f0 + g.fmax);
            const int32_t* fol = ops[k].fol;
            // the pivot's naive search, then its followers' slides, through
            // one call site (one inlined search: fewer live registers)
            for (int64_t f = f0 - 1; f < f1; ++f) {
                const bool piv = f < f0;
                const SearchArgs a = piv ? ops[k].naive : ops[k].slide;
                const int v = piv ? p : fol[f];
                const int32_t* seeds = piv ? nullptr : a.seed_ids + (int64_t)p * a.seed_stride;
                SearchCounts c;
                search_one<TT, EFS, CPL, EXACT, LG>(a, v, piv ? 0 : 2, seeds, piv ? 0 : a.n_seeds, v,
                                                    tab, cl, lane, c);
                // the wavefront's counts wait in LDS (no registers held
                // across the loop)
                if (lane == 0) {
                    u64* w = wcnt[wib] + (piv ? 0 : 4);
                    w[0] += c.ndc;
                    w[1] += c.nexp;
                    w[2] += c.nadj;
                    w[3] += c.nevict;
                }
                // the pivot's beam, just stored by this wavefront, seeds its
                // followers: stores complete before those loads
                if (piv) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            }
        }
    }
    SearchCounts cp, cf;
    if (lane == 0) {
        const u64* w = wcnt[wib];
        cp.ndc = w[0];
        cp.nexp = w[1];
        cp.nadj = w[2];
        cp.nevict = w[3];
        cf.ndc = w[4];
        cf.nexp = w[5];
        cf.nadj = w[6];
        cf.nevict = w[7];
    }
    add_counts(g.counters, cp, lane);
    add_counts(g.counters + CNT_SLOTS * CNT_N, cf, lane);
}

// ------------------------------------------------------------------ prune

// float32 distance between the lane-group layouts of two rows (valid in the
// group's last lane)
template <int CPL>
__device__ __forceinline__ float dist_rows(const float4* a, const float4* b, int metric, int G) {
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const float4 x = a[j], q = b[j];
        if (metric == 0) {
            const float d0 = q.x - x.x, d1 = q.y - x.y, d2 = q.z - x.z, d3 = q.w - x.w;
            acc = fmaf(d0, d0, acc);
            acc = fmaf(d1, d1, acc);
            acc = fmaf(d2, d2, acc);
            acc = fmaf(d3, d3, acc);
        } else {
            acc = fmaf(q.x, x.x, acc);
            acc = fmaf(q.y, x.y, acc);
            acc = fmaf(q.z, x.z, acc);
            acc = fmaf(q.w, x.w, acc);
        }
    }
    return group_sum_last(acc, G);
}

// this lane's CPL chunks of float32 row id (nothing for id < 0)
template <int CPL>
__device__ __forceinline__ void load_row_f32(const float* X, int64_t id, int rowf, int sub, int G,
                                             float4* out) {
    if (id >= 0) {
        const float* r = X + id * rowf + sub * 4;
#pragma unroll
        for (int j = 0; j < CPL; ++j) out[j] = *(const float4*)(r + (int64_t)j * G * 4);
    }
}

// the distances still missing in the keys wk[0, nW) of vertex p (a key with
// the id alone, < 2^32), computed with the lane-group layout: from the
// float32 rows, or (B16) from the bfloat16 copy of rows that are exact in it,
// with v_dot2 and squared L2 as |p|^2 + |w|^2 - 2 p.w in double; every sum is
// then an exact integer, so both give the same float
template <int CPL, bool B16>
__device__ __forceinline__ void collect_dists(const PruneArgs& a, int64_t p, u64* wk, int nW,
                                              int lane) {
    const float pn = a.metric == 2 ? a.norms[p] : 1.0f;
    constexpr int UNR = 2;
    if constexpr (B16) {
        const int G16 = a.G16, RPP16 = WAVE >> a.lgG16;
        const int group16 = lane >> a.lgG16, sub16 = lane & (G16 - 1);
        const int64_t rowb = (int64_t)a.nch * 8;  // bytes of a bfloat16 row
        const int64_t gs = (int64_t)G16 * 16;
        uint4 pq[CPL];
        float pp = 0.0f;
        {
            const char* r = a.xb + p * rowb + sub16 * 16;
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                pq[j] = *(const uint4*)(r + j * gs);
                pp = dot2x4<1>(pq[j], pq[j], pp);
            }
        }
        pp = group_sum_last(pp, G16);
        for (int c0 = 0; c0 < nW; c0 += RPP16 * UNR) {
            uint4 raw[UNR][CPL];
            int cid[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                const int c = c0 + u * RPP16 + group16;
                const u64 kk = c < nW ? wk[c] : EMPTY_KEY;
                cid[u] = kk < (1ull << 32) ? (int)kk : -1;
                if (cid[u] >= 0) {
                    const char* r = a.xb + (int64_t)cid[u] * rowb + sub16 * 16;
#pragma unroll
                    for (int j = 0; j < CPL; ++j) raw[u][j] = *(const uint4*)(r + j * gs);
                }
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                float acc = 0.0f, xx = 0.0f;
                if (cid[u] >= 0) {
#pragma unroll
                    for (int j = 0; j < CPL; ++j) {
                        acc = dot2x4<1>(pq[j], raw[u][j], acc);
                        xx = dot2x4<1>(raw[u][j], raw[u][j], xx);
                    }
                }
                acc = group_sum_last(acc, G16);
                xx = group_sum_last(xx, G16);
                const int c = c0 + u * RPP16 + group16;
                if (sub16 == G16 - 1 && cid[u] >= 0) {
                    const float nb = a.metric == 2 ? a.norms[cid[u]] : 1.0f;
                    const float d = a.metric == 0
                                        ? (float)((double)pp + (double)xx - 2.0 * (double)acc)
                                        : finalize_dist(acc, a.metric, pn, nb);
                    wk[c] = make_key(d, cid[u]);
                }
            }
        }
    }
    const int G = a.G, RPP = WAVE >> a.lgG;
    const int group = lane >> a.lgG, sub = lane & (G - 1);
    const int rowf = a.nch * 4;
    float4 pq[CPL];
    if (!B16) load_row_f32<CPL>(a.X, p, rowf, sub, G, pq);
    for (int c0 = 0; c0 < (B16 ? 0 : nW); c0 += RPP * UNR) {
        float4 raw[UNR][CPL];
        int cid[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int c = c0 + u * RPP + group;
            const u64 kk = c < nW ? wk[c] : EMPTY_KEY;
            cid[u] = kk < (1ull << 32) ? (int)kk : -1;
            load_row_f32<CPL>(a.X, cid[u], rowf, sub, G, raw[u]);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const float acc = dist_rows<CPL>(raw[u], pq, a.metric, G);
            const int c = c0 + u * RPP + group;
            if (sub == G - 1 && cid[u] >= 0) {
                const float nb = a.metric == 2 ? a.norms[cid[u]] : 1.0f;
                wk[c] = make_key(finalize_dist(acc, a.metric, pn, nb), cid[u]);
            }
        }
    }
}

// ws[r] = wk[t] with r = #smaller keys + #equal keys earlier in wk, for
// nW <= KMAX * 64 keys: each lane holds keys t = j * 64 + lane in registers,
// and every key is broadcast once with readlane (no memory reads in the
// O(nW^2) part, which matters when wk is in global scratch)
template <int KMAX>
__device__ __forceinline__ void rank_keys(const u64* wk, u64* ws, int nW, int lane) {
    u64 kv[KMAX];
    int rk[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        const int t = j * WAVE + lane;
        kv[j] = t < nW ? wk[t] : EMPTY_KEY;
        rk[j] = 0;
    }
#pragma unroll
    for (int j2 = 0; j2 < KMAX; ++j2) {
        const int lim = min(WAVE, nW - j2 * WAVE);
        for (int l = 0; l < lim; ++l) {
            const u64 ks = readlane64(kv[j2], l);
            const int s2 = j2 * WAVE + l;
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                rk[j] += (ks < kv[j] || (ks == kv[j] && s2 < j * WAVE + lane)) ? 1 : 0;
        }
    }
#pragma unroll
    for (int j = 0; j < KMAX; ++j)
        if (j * WAVE + lane < nW) ws[rk[j]] = kv[j];
}

// The 16 smallest keys >= lo among wk[0, nW) in ascending order, EMPTY_KEY
// past the last: lane l returns the (l % 16)-th. Each lane keeps the 16
// smallest keys of its share in registers (an insertion network), then 16
// rounds of wavefront minima merge the 64 lists. Equal keys (one vertex twice
// in W) come out next to each other. O(nW / 64) reads per lane.
__device__ __noinline__ u64 next16(const u64* wk, int nW, u64 lo, int lane) {
    u64 s[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) s[i] = EMPTY_KEY;
    for (int t = lane; t < nW; t += WAVE) {
        u64 x = wk[t];
        if (x >= lo && x < s[15]) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const u64 m = s[i] < x ? s[i] : x;
                x = s[i] < x ? x : s[i];
                s[i] = m;
            }
        }
    }
    u64 out = EMPTY_KEY;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const u64 m = wave_min_u64(s[0]);
        if (m == EMPTY_KEY) break;
        const int src = __ffsll((long long)__ballot(s[0] == m)) - 1;
        if (lane == src) {
#pragma unroll
            for (int i = 0; i < 15; ++i) s[i] = s[i + 1];
            s[15] = EMPTY_KEY;
        }
        if ((lane & 15) == r) out = m;
    }
    return out;
}

// a kept edge p -> v into the target range offers p to v: counted here, so
// that the reverse lists need no separate counting pass over the rows
__device__ __forceinline__ void count_reverse(const PruneArgs& a, int64_t v) {
    if (a.rev_cnt && v >= a.rev_lo && v < a.rev_lo + a.rev_n) atomicAdd(&a.rev_cnt[v - a.rev_lo], 1);
}

// Candidate list W of the prune of p (Section 2.2): the current row of p
// plus the extra candidates, minus p itself. Keys (d(p, w), w) go to wk;
// the ones whose float32 distance is already known (search results, reverse
// edges, pruned rows) take it, the others are computed here (collect_dists).
// Then the keys are placed in (d, id) order into *ws_out.
// Returns |W|, or -1 when the wavefront has nothing to do.
template <int CPL, bool B16>
__device__ __forceinline__ int prune_collect(const PruneArgs& a, int64_t p, int64_t e, int lane,
                                             u64* lws, u64* lwk, u64** wk_out, u64** ws_out) {
    const int R = a.R;
    const int G = a.G, RPP = WAVE >> a.lgG;
    const int nrow = a.rows_in ? a.deg_in[p] : 0;
    int next = 0;
    int64_t xo = 0;
    if (a.extra_mode == 1) {
        next = a.extra_cnt;
        xo = e * a.extra_stride;
    } else if (a.extra_mode == 2) {
        xo = a.extra_off[e];
        next = (int)(a.extra_off[e + 1] - xo);
    }
    if (a.skip_empty_extra && next == 0) return -1;
    const int nW = nrow + next;
    // long candidate lists may go to a pass of their own (list_filter)
    if ((a.list_filter == 1 && nW > LONG_LIST) || (a.list_filter == 2 && nW <= LONG_LIST))
        return -1;
    u64* wk = lwk;  // wcap keys each in LDS
    u64* ws = lws;
    if (nW > a.wcap) {
        if (a.extra_mode != 2 || !a.scratch) {
            if (lane == 0) atomicOr(a.err, 2);
            return -1;
        }
        wk = a.scratch + 2 * ((int64_t)R * e + xo);
        ws = wk + nW;
    }
    for (int t = lane; t < nW; t += WAVE) {
        int64_t id;
        float d = __int_as_float(0x7fc00000);
        if (t < nrow) {
            id = a.rows_in[p * R + t];
            if (a.rows_d) d = a.rows_d[p * R + t];
        } else {
            const int32_t x = a.extra_ids[xo + (t - nrow)];
            id = x < 0 ? -1 : (int64_t)x + a.extra_id_add;
            if (a.extra_d) d = a.extra_d[xo + (t - nrow)];
        }
        if (id >= a.n_total) {  // ids from callers are range-checked
            atomicOr(a.err, 4);
            id = -1;
        }
        // a key with the id alone (< 2^32) marks a distance still to compute
        wk[t] = (id < 0 || id == p) ? EMPTY_KEY : (d == d ? make_key(d, (int)id) : (u64)id);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    collect_dists<CPL, B16>(a, p, wk, nW, lane);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // order: position = #smaller keys + #equal keys earlier in W
    if (a.extra_sorted && a.extra_mode == 1 && a.extra_d && nrow <= WAVE && nW <= a.wcap) {
        // the extras (wk[nrow..nW)) are already in key order: rank the row
        // part among itself, then merge the two lists by binary search (row
        // keys before equal extra keys, as their index is lower)
        const int nb = nW - nrow;
        u64 ka = EMPTY_KEY;
        int ra = 0;
        if (lane < nrow) {
            ka = wk[lane];
            for (int s2 = 0; s2 < nrow; ++s2) {
                const u64 ks = wk[s2];
                ra += (ks < ka || (ks == ka && s2 < lane)) ? 1 : 0;
            }
            ws[ra] = ka;  // the row part in order, for the extras' searches
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const u64* xb = wk + nrow;
        int pa = 0;
        if (lane < nrow) {  // extras below ka
            int lo = 0, hi = nb;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (xb[mid] < ka) lo = mid + 1; else hi = mid;
            }
            pa = ra + lo;
        }
        constexpr int XPL = 2;  // extras per lane (nb <= 128)
        u64 kb[XPL];
        int pb[XPL];
#pragma unroll
        for (int x = 0; x < XPL; ++x) {
            const int j = lane + x * WAVE;
            kb[x] = j < nb ? xb[j] : EMPTY_KEY;
            int lo = 0, hi = nrow;  // row keys <= kb
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (ws[mid] <= kb[x]) lo = mid + 1; else hi = mid;
            }
            pb[x] = j + lo;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < nrow) ws[pa] = ka;
#pragma unroll
        for (int x = 0; x < XPL; ++x)
            if (lane + x * WAVE < nb) ws[pb[x]] = kb[x];
    } else if (nW <= 2 * WAVE) {
        rank_keys<2>(wk, ws, nW, lane);
    } else if (nW <= 4 * WAVE) {
        rank_keys<4>(wk, ws, nW, lane);
    } else if (nW <= 8 * WAVE) {
        rank_keys<8>(wk, ws, nW, lane);
    } else if (nW <= LONG_LIST) {
        rank_keys<16>(wk, ws, nW, lane);
    } else {
        // longer lists (targets that collected thousands of reverse edges)
        // are not sorted: the prune takes them 16 at a time in key order
        // (next16), and stops once R are kept
        ws = nullptr;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    *wk_out = wk;
    *ws_out = ws;
    return nW;
}

// distances of the rows of vertices item_base + [0, n_items) to their entries
// (rows_in / deg_in), written to rows_d where it holds NaN, computed by
// collect_dists exactly as a later prune of these vertices would compute
// them (same layout, same arithmetic), so that the prune finds them known.
// One wavefront per vertex, rows of at most 64 entries; a capped grid
// (grid_cap) strides over the vertices, leaving the rest of the device to
// work running beside it.
template <int CPL, bool B16>
__global__ __launch_bounds__(256) void k_row_dists(PruneArgs a) {
    __shared__ u64 keys[4][WAVE];
    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t i = xcd_block() * (blockDim.x >> 6) + wib; i < a.n_items; i += waves) {
        const int64_t p = a.item_base + i;
        const int R = a.R;
        const int nrow = a.deg_in[p];
        float* rd = (float*)a.rows_d + p * R;
        u64* wk = keys[wib];
        bool todo = false;
        if (lane < nrow) {
            const int id = a.rows_in[p * R + lane];
            todo = rd[lane] != rd[lane] && id >= 0 && id < a.n_total && id != p;
            wk[lane] = todo ? (u64)(unsigned)id : EMPTY_KEY;
        }
        if (__ballot(todo) == 0ull) continue;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        collect_dists<CPL, B16>(a, p, wk, nrow, lane);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (todo) rd[lane] = fval((unsigned)(wk[lane] >> 32));
        // the next vertex's keys reuse wk
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Whether kept w removes candidate v under the rule, from d(p,v), d(p,w),
// d(w,v): 0 alpha * d(w,v) < d(p,v); 1 (SSG) the angle at p between v and w
// below theta: c = d(p,v) + d(p,w) - d(w,v) > 0 and c^2 > 4 cos^2(theta)
// d(p,v) d(p,w); 2 (tau-MNG) sqrt(d(w,v)) < sqrt(d(p,v)) - 3 tau. In double,
// each operation rounded on its own in this order (no contraction), so
// exact distances give the same decision on any IEEE double machine.
__device__ __forceinline__ bool rule_drops(int rule, double ra, double alpha, double dpv,
                                           double dpw, double dwv) {
    if (rule == 1) {
        const double c = __dsub_rn(__dadd_rn(dpv, dpw), dwv);
        return c > 0.0 &&
               __dmul_rn(c, c) > __dmul_rn(__dmul_rn(__dmul_rn(__dmul_rn(4.0, ra), ra), dpv), dpw);
    }
    if (rule == 2) {
        const double t = __dsub_rn(__dsqrt_rn(dpv), ra);
        return t > 0.0 && __dsqrt_rn(dwv) < t;
    }
    return alpha * dwv < dpv;
}

// Prune(p, W) with float32 vector arithmetic: candidates are walked in
// (d, id) order; a candidate is kept unless a kept w removes it by the rule
// (alpha: alpha * d(w, v) < d(p, v), strict, in double); stop at R kept.
// Kept rows stay in registers (KS slots per lane group) or are re-read
// (KS == 0); kept distances d(p, w) are read back from the output row.
template <int CPL, int KS>
__global__ __launch_bounds__(256) void k_prune(PruneArgs a) {
    extern __shared__ unsigned char psm[];
    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int64_t i = xcd_block() * wpb + wib;
    if (i >= a.n_items) return;
    // per wavefront: keys[wcap], sorted[wcap], kept ids[R]
    u64* lkeys = (u64*)psm + (int64_t)wib * (2 * a.wcap + a.R);
    int* kept_ids = (int*)(lkeys + 2 * a.wcap);
    const int64_t p = a.item_base + (a.items ? (int64_t)a.items[i] : i);
    const int64_t e = p - a.extra_index_base;
    const int R = a.R;
    const int G = a.G, RPP = WAVE >> a.lgG;
    u64 *wk, *ws;
    const int nW = prune_collect<CPL, false>(a, p, e, lane, lkeys + a.wcap, lkeys, &wk, &ws);
    if (nW < 0) return;
    const int group = lane >> a.lgG, sub = lane & (G - 1);
    const int rowf = a.nch * 4;

    // walk the candidates in (d, id) order
    float4 kept[KS > 0 ? KS : 1][CPL];
    const double alpha = (double)a.alpha;
    int nk = 0;
    u64 prev = EMPTY_KEY;
    float4 vx[CPL], nx[CPL];
    // candidate t in key order: the sorted list, or (long lists, ws NULL)
    // 16 at a time from next16 into a buffer in the then unused LDS keys
    int tbase = -16;
    u64 lo = 0;
    auto key_at = [&](int t) -> u64 {
        if (ws) return t < nW ? ws[t] : EMPTY_KEY;
        if (t >= tbase + 16) {
            const u64 k = next16(wk, nW, lo, lane);
            if (lane < 16) lkeys[lane] = k;
            const u64 last = readlane64(k, 15);
            lo = last == EMPTY_KEY ? EMPTY_KEY : last + 1;
            tbase += 16;
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        return lkeys[t - tbase];
    };
    u64 cur = nW > 0 ? key_at(0) : EMPTY_KEY;
    load_row_f32<CPL>(a.X, cur == EMPTY_KEY ? -1 : (int64_t)(unsigned)(cur & 0xffffffffu), rowf,
                      sub, G, nx);
    for (int t = 0; t < nW && nk < R; ++t) {
        if (cur == EMPTY_KEY) break;
#pragma unroll
        for (int j = 0; j < CPL; ++j) vx[j] = nx[j];
        const u64 kcur = cur;
        // prefetch the next candidate's row
        cur = t + 1 < nW ? key_at(t + 1) : EMPTY_KEY;
        load_row_f32<CPL>(a.X, cur == EMPTY_KEY ? -1 : (int64_t)(unsigned)(cur & 0xffffffffu),
                          rowf, sub, G, nx);
        if (kcur == prev) continue;  // the same vertex twice in W
        prev = kcur;
        const int v = (int)(unsigned)(kcur & 0xffffffffu);
        const float dv = fval((unsigned)(kcur >> 32));
        const float vn = a.metric == 2 ? a.norms[v] : 1.0f;
        bool dom = false;
        const int nslots = (nk + RPP - 1) / RPP;
        if constexpr (KS > 0) {
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                if (s < nslots) {
                    const float acc = dist_rows<CPL>(kept[s], vx, a.metric, G);
                    const int jk = s * RPP + group;
                    if (jk < nk && sub == G - 1) {
                        const float kn = a.metric == 2 ? a.norms[kept_ids[jk]] : 1.0f;
                        const float dkv = finalize_dist(acc, a.metric, kn, vn);
                        const double dpw = a.rule ? (double)a.dist_out[p * R + jk] : 0.0;
                        if (rule_drops(a.rule, a.rule_a, alpha, (double)dv, dpw, (double)dkv))
                            dom = true;
                    }
                }
            }
        } else {
            for (int s = 0; s < nslots; ++s) {
                const int jk = s * RPP + group;
                float4 kx[CPL];
                load_row_f32<CPL>(a.X, jk < nk ? kept_ids[jk] : v, rowf, sub, G, kx);
                const float acc = dist_rows<CPL>(kx, vx, a.metric, G);
                if (jk < nk && sub == G - 1) {
                    const float kn = a.metric == 2 ? a.norms[kept_ids[jk]] : 1.0f;
                    const float dkv = finalize_dist(acc, a.metric, kn, vn);
                    const double dpw = a.rule ? (double)a.dist_out[p * R + jk] : 0.0;
                    if (rule_drops(a.rule, a.rule_a, alpha, (double)dv, dpw, (double)dkv))
                        dom = true;
                }
            }
        }
        if (__ballot(dom) != 0ull) continue;
        if constexpr (KS > 0) {
            const int s = nk / RPP, gsel = nk - s * RPP;
#pragma unroll
            for (int ss = 0; ss < KS; ++ss)
                if (ss == s && group == gsel) {
#pragma unroll
                    for (int j = 0; j < CPL; ++j) kept[ss][j] = vx[j];
                }
        }
        if (lane == 0) {
            kept_ids[nk] = v;
            a.rows_out[p * R + nk] = v;
            a.dist_out[p * R + nk] = dv;
            count_reverse(a, v);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        ++nk;
    }
    if (lane == 0) a.deg_out[p] = nk;
}

// ------------------------------------------------------------ MFMA prune

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

// bfloat16 bits of a finite float, round to nearest even
__device__ __forceinline__ unsigned bf16_bits(float x) {
    const unsigned u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// eight floats -> packed bfloat16 hi = bf16(v) and, with NT == 3, the
// remainder lo = bf16(v - hi), so that hi + lo carries about 16 bits
template <int NT>
__device__ __forceinline__ void split8(const float* v, uint4& hi, uint4& lo) {
    if constexpr (NT == 1) {
        // values exact in bfloat16: the upper halves, two per word
        auto pk = [](float a, float b) {
            return (__float_as_uint(b) & 0xffff0000u) | (__float_as_uint(a) >> 16);
        };
        hi = make_uint4(pk(v[0], v[1]), pk(v[2], v[3]), pk(v[4], v[5]), pk(v[6], v[7]));
        lo = make_uint4(0u, 0u, 0u, 0u);
        return;
    }
    unsigned h[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        h[e] = bf16_bits(v[e]);
        l[e] = NT > 1 ? bf16_bits(v[e] - __uint_as_float(h[e] << 16)) : 0u;
    }
    hi = make_uint4(h[0] | h[1] << 16, h[2] | h[3] << 16, h[4] | h[5] << 16, h[6] | h[7] << 16);
    lo = make_uint4(l[0] | l[1] << 16, l[2] | l[3] << 16, l[4] | l[5] << 16, l[6] | l[7] << 16);
}

// D += A B for 16x32 A and 32x16 B; lane l holds row (A) / column (B) l % 16,
// k = 8 (l / 16) + 0..7; D: lane l, element r is D[4 (l / 16) + r][l % 16]
__device__ __forceinline__ floatx4_t mfma16(uint4 a, uint4 b, floatx4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                  __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
}

// d(w_i, w_j) from the Gram entry g of the two rows: squared L2 as
// u_i + u_j - 2 g, with u = |w|^2 for plain rows or u = |w - p|^2 = d(p, w)
// (the key distance) for rows centred at p; inner product and cosine on the
// rows themselves
__device__ __forceinline__ double gram_dist(float g, int metric, float ui, float uj, float ni,
                                            float nj) {
    if (metric == 0) return (double)ui + (double)uj - 2.0 * (double)g;
    if (metric == 1) return (double)(1.0f - g);
    return (double)(1.0f - g / (ni * nj));
}

// largest integer D with alpha * D < d (double products, exact for |D| < 2^29)
// (the estimate takes the reciprocal of alpha >= 1; the two loops make the
// result exact whatever its rounding)
__device__ __forceinline__ int dom_threshold(double alpha, double inv_alpha, float d) {
    const double dd = (double)d;
    if (!(dd < 1.0e18) || !(dd > -1.0e18)) return dd > 0.0 ? 0x7fffffff : -0x7fffffff;
    double t = floor(dd * inv_alpha);
    if (!(t < 1.0e9)) t = 1.0e9;
    if (t < -1.0e9) t = -1.0e9;
    int ti = (int)t;
    while (alpha * (double)ti >= dd) --ti;
    while (alpha * (double)(ti + 1) < dd) ++ti;
    return ti;
}

// d(w, v) in float32 with the arithmetic of the float32 walk (k_prune): the
// rows in its lane-group layout (G lanes, CPL 16-byte chunks per lane, w as
// the kept row, v as the candidate), the same fma order and group sum, then
// finalize_dist with the norms in the same order. Lane group 0 computes it;
// the value is returned in every lane.
template <int CPL>
__device__ __forceinline__ float walk_pair_dist(const PruneArgs& a, int w, int v, int lane) {
    const int G = a.G, sub = lane & (G - 1), group = lane >> a.lgG;
    const int rowf = a.nch * 4;
    float4 xw[CPL], xv[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        xw[j] = make_float4(0.f, 0.f, 0.f, 0.f);
        xv[j] = xw[j];
    }
    load_row_f32<CPL>(a.X, group == 0 ? (int64_t)w : -1, rowf, sub, G, xw);
    load_row_f32<CPL>(a.X, group == 0 ? (int64_t)v : -1, rowf, sub, G, xv);
    const float acc = dist_rows<CPL>(xw, xv, a.metric, G);
    const float wn = a.metric == 2 ? a.norms[w] : 1.0f, vn = a.metric == 2 ? a.norms[v] : 1.0f;
    const float d = finalize_dist(acc, a.metric, wn, vn);
    return __shfl(d, G - 1);
}

// Whether the alpha test of a pair decided from a hi/lo-split Gram estimate
// dwv may differ from the walk's float32 decision: the estimate lies within
// band * scale of the boundary, scale bounding the pair's distance terms
// (squared L2 centred at p: (sqrt d(p,w) + sqrt d(p,v))^2; inner product:
// |w| |v|; cosine: 1). Outside the band the split's error (about 2^-15 of the
// scale) and the float32 sums' cannot move the decision.
__device__ __forceinline__ bool near_boundary(double alpha, double dwv, float dv, double band,
                                              int metric, float ui, float uj, float si,
                                              float sj) {
    double scale;
    if (metric == 0) {
        const double r = sqrt((double)fmaxf(ui, 0.f)) + sqrt((double)fmaxf(uj, 0.f));
        scale = r * r;
    } else if (metric == 1) {
        scale = sqrt((double)si) * sqrt((double)sj);
    } else {
        scale = 1.0;
    }
    return fabs(alpha * dwv - (double)dv) <= alpha * band * scale;
}

// LDS bytes per wavefront of k_prune_mfma: sorted keys, kept ids, distances,
// key terms and squared norms, then kept-row fragments (R rounded up to whole
// 16-row tiles; hi, then lo with the split), whose space first holds the
// unsorted keys
__host__ __device__ inline int mfma_row_stride(int kd) { return 64 * kd + 16; }
__host__ __device__ inline int mfma_kept_rows(int R) { return (R + 15) & ~15; }
__host__ __device__ inline size_t mfma_kept_bytes(int R) { return ((size_t)R * 16 + 15) / 16 * 16; }
__host__ __device__ inline size_t mfma_prune_lds(int wcap, int R, int kd, int nt) {
    const size_t rows = (size_t)mfma_kept_rows(R) * mfma_row_stride(kd) * (nt > 1 ? 2 : 1);
    const size_t keys = (size_t)wcap * sizeof(u64);
    return keys + mfma_kept_bytes(R) + (rows > keys ? rows : keys);
}

// Prune(p, W) with the candidate x kept-row Gram products on bfloat16 MFMA.
// Candidates are taken 16 at a time in (d, id) order (tile J). Each lane
// holds the 8 KD dimensions [q * 8 KD, (q + 1) * 8 KD) of row l % 16 of the
// tile, q = l / 16, as KD fragments of 8. One MFMA chain gives the 16 x 16
// Gram of the tile with itself; one per 16 kept rows (bfloat16 fragments in
// LDS) gives kept x tile. A pair (w, v) is decided by
// alpha * d(w, v) < d(p, v) as in the walk; then the 16 candidates are
// resolved in order with ballot bit masks, and the kept ones are appended
// to the kept rows.
//  NT == 1: rows exact in bfloat16 and every Gram and squared-norm sum
//           exact in float32 (integers of magnitude <= 256, dim <= 256):
//           every d(w, v) is exact, so every decision equals the walk's.
//           The fragments are read from the bfloat16 copy (half the bytes
//           of the float32 rows, the same values).
//  NT == 3: rows split as hi + lo bfloat16, products hi*hi + hi*lo + lo*hi;
//           squared L2 works on rows centred at p.
template <int KD, int NT, int CPL>
__global__ __launch_bounds__(256, NT == 1 ? 4 : 1) void k_prune_mfma(PruneArgs a) {
    extern __shared__ unsigned char psm[];
    constexpr bool CENTER = NT > 1;
    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int64_t i = xcd_block() * wpb + wib;
    if (i >= a.n_items) return;
    const int R = a.R;
    unsigned char* base = psm + (size_t)wib * mfma_prune_lds(a.wcap, R, KD, NT);
    u64* lkeys = (u64*)base;
    int* kept_ids = (int*)(base + (size_t)a.wcap * sizeof(u64));
    float* kept_d = (float*)(kept_ids + R);
    float* kept_u = kept_d + R;
    float* kept_s = kept_u + R;  // squared norms (float rows: the re-decision band)
    unsigned char* khi = base + (size_t)a.wcap * sizeof(u64) + mfma_kept_bytes(R);
    u64 nrecheck = 0;
    const int rs = mfma_row_stride(KD);
    const size_t klo_off = (size_t)mfma_kept_rows(R) * rs;  // lo fragments follow the hi ones
    const int64_t p = a.item_base + (a.items ? (int64_t)a.items[i] : i);
    const int64_t e = p - a.extra_index_base;
    u64 *wk, *ws;
    // the unsorted keys share the kept rows' space: they are dead once sorted
    const int nW = prune_collect<CPL, NT == 1>(a, p, e, lane, lkeys, (u64*)khi, &wk, &ws);
    if (nW < 0) return;
    (void)wk;
    if (!ws) {  // lists longer than 1024 are the walk's (run with list_filter 2)
        if (lane == 0) atomicOr(a.err, 2);
        return;
    }

    constexpr int DL = 8 * KD;  // dimensions per lane
    const int dim = 32 * KD;
    const int jr = lane & 15, q = lane >> 4;
    const int metric = a.metric;
    const double alpha = (double)a.alpha, inv_alpha = 1.0 / alpha;
    float pf[CENTER ? DL : 1];
    if constexpr (CENTER) {
#pragma unroll
        for (int t = 0; t < DL; ++t) pf[t] = 0.0f;
        if (metric == 0) {
            const float4* pr = (const float4*)(a.X + p * dim + q * DL);
#pragma unroll
            for (int t = 0; t < DL / 4; ++t) {
                const float4 x = pr[t];
                pf[4 * t] = x.x;
                pf[4 * t + 1] = x.y;
                pf[4 * t + 2] = x.z;
                pf[4 * t + 3] = x.w;
            }
        }
    }
    // this lane's DL floats of sorted candidate J * 16 + l % 16 (zeros past the end)
    auto load_tile = [&](int J, float* raw) {
        const int c = J * 16 + jr;
        const u64 kk = c < nW ? ws[c] : EMPTY_KEY;
        if (NT != 1 && kk != EMPTY_KEY) {
            const float4* r = (const float4*)(a.X + (int64_t)(unsigned)(kk & 0xffffffffu) * dim + q * DL);
#pragma unroll
            for (int t = 0; t < DL / 4; ++t) {
                const float4 x = r[t];
                raw[4 * t] = x.x;
                raw[4 * t + 1] = x.y;
                raw[4 * t + 2] = x.z;
                raw[4 * t + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int t = 0; t < DL; ++t) raw[t] = 0.0f;
        }
    };
    // exact mode: the same DL dimensions as KD packed bfloat16 fragments,
    // read from the bfloat16 copy
    const int64_t rowb = (int64_t)dim * 2;
    auto load_frag = [&](int J, uint4* fr) {
        const int c = J * 16 + jr;
        const u64 kk = c < nW ? ws[c] : EMPTY_KEY;
        if (kk != EMPTY_KEY) {
            const uint4* r = (const uint4*)(a.xb + (int64_t)(unsigned)(kk & 0xffffffffu) * rowb +
                                            q * DL * 2);
#pragma unroll
            for (int t = 0; t < KD; ++t) fr[t] = r[t];
        } else {
#pragma unroll
            for (int t = 0; t < KD; ++t) fr[t] = make_uint4(0u, 0u, 0u, 0u);
        }
    };
    // exact mode keeps two tiles of fragments in flight (buffers A and B
    // alternate: tile J reads buffer J % 2, then refills it with tile J + 2)
    float raw[NT == 1 ? 1 : DL];
    uint4 fragA[NT == 1 ? KD : 1], fragB[NT == 1 ? KD : 1];
    int nk = 0;
    u64 prev = EMPTY_KEY;
    const int ntiles = (nW + 15) >> 4;
    if constexpr (NT == 1) {
        load_frag(0, fragA);
        if (ntiles > 1) load_frag(1, fragB);
    } else {
        load_tile(0, raw);
    }
    auto tile = [&](int J, uint4* cur) -> bool {
        const int c = J * 16 + jr;
        const u64 key = c < nW ? ws[c] : EMPTY_KEY;
        const int idj = key == EMPTY_KEY ? -1 : (int)(unsigned)(key & 0xffffffffu);
        const float dj = key == EMPTY_KEY ? INFINITY : fval((unsigned)(key >> 32));
        const float nj = (metric == 2 && idj >= 0) ? a.norms[idj] : 1.0f;
        uint4 hi[KD], lo[KD];
        float sq = 0.0f;  // squared norm of the plain row (exact for NT == 1)
        if constexpr (NT == 1) {
#pragma unroll
            for (int s2 = 0; s2 < KD; ++s2) {
                hi[s2] = cur[s2];
                lo[s2] = make_uint4(0u, 0u, 0u, 0u);
                sq = dot2x4<1>(hi[s2], hi[s2], sq);
            }
        } else {
#pragma unroll
            for (int s2 = 0; s2 < KD; ++s2) {
                float v[8];
#pragma unroll
                for (int e2 = 0; e2 < 8; ++e2) {
                    v[e2] = CENTER ? raw[8 * s2 + e2] - pf[CENTER ? 8 * s2 + e2 : 0] : raw[8 * s2 + e2];
                    sq = fmaf(raw[8 * s2 + e2], raw[8 * s2 + e2], sq);
                }
                split8<NT>(v, hi[s2], lo[s2]);
            }
        }
        float uj = dj;
        sq += __shfl_xor(sq, 16);
        sq += __shfl_xor(sq, 32);
        if constexpr (!CENTER) uj = sq;
        // exact rows, squared L2 or inner product: every d(w, v) is an exact
        // integer, so alpha * d(w, v) < d(p, v) is d(w, v) <= T (integer)
        const bool intd = NT == 1 && metric != 2;
        const int tj = intd ? dom_threshold(alpha, inv_alpha, dj) : 0;
        const int uji = intd && metric == 0 ? (int)uj : 0;
        if constexpr (NT == 1) {  // tile J + 2's rows in flight
            if (J + 2 < ntiles) load_frag(J + 2, cur);
        } else if (J + 1 < ntiles) {  // next tile's rows in flight
            load_tile(J + 1, raw);
        }

        // the tile with itself: pairs (i, j), i = 4 q + r, j = l % 16, i < j
        floatx4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s2 = 0; s2 < KD; ++s2) {
            acc = mfma16(hi[s2], hi[s2], acc);
            if constexpr (NT > 1) {
                acc = mfma16(hi[s2], lo[s2], acc);
                acc = mfma16(lo[s2], hi[s2], acc);
            }
        }
        u64 bt[4], ut[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ii = 4 * q + r;
            bool pred, unc = false;
            if (intd) {
                const int g = (int)acc[r];
                const int dij = metric == 0 ? __shfl(uji, ii) + uji - 2 * g : 1 - g;
                pred = ii < jr && dij <= tj;
            } else {
                const float ui = __shfl(uj, ii);
                const float ni = __shfl(nj, ii);
                const float si = __shfl(sq, ii);
                const double gd = gram_dist(acc[r], metric, ui, uj, ni, nj);
                pred = ii < jr && alpha * gd < (double)dj;
                if constexpr (NT > 1)
                    unc = ii < jr && idj >= 0 && a.band > 0.0 &&
                          near_boundary(alpha, gd, dj, a.band, metric, ui, uj, si, sq);
            }
            bt[r] = __ballot(pred && !unc);
            ut[r] = __ballot(unc);
        }
        if constexpr (NT > 1) {
            // pairs near the boundary: the float32 walk's own decision
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                u64 m = ut[r];
                while (m) {
                    const int l = __ffsll((long long)m) - 1;
                    m &= m - 1;
                    const int ii = 4 * (l >> 4) + r, jj = l & 15;
                    const int w = __builtin_amdgcn_readlane(idj, ii);
                    const int v = __builtin_amdgcn_readlane(idj, jj);
                    const float dv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dj), jj));
                    const float dwv = walk_pair_dist<CPL>(a, w, v, lane);
                    if (alpha * (double)dwv < (double)dv) bt[r] |= 1ull << l;
                    ++nrecheck;
                }
            }
        }
        // kept rows of earlier tiles against the tile
        const int nk0 = nk;
        u64 bk = 0ull;
        for (int kt = 0; kt * 16 < nk0; ++kt) {
            floatx4_t ak = {0.0f, 0.0f, 0.0f, 0.0f};
            const unsigned char* krow = khi + (size_t)(kt * 16 + jr) * rs + q * KD * 16;
#pragma unroll
            for (int s2 = 0; s2 < KD; ++s2) {
                const uint4 kh = *(const uint4*)(krow + s2 * 16);
                ak = mfma16(kh, hi[s2], ak);
                if constexpr (NT > 1) {
                    const uint4 kl = *(const uint4*)(krow + klo_off + s2 * 16);
                    ak = mfma16(kh, lo[s2], ak);
                    ak = mfma16(kl, hi[s2], ak);
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ki = kt * 16 + 4 * q + r;
                bool pred = false, unc = false;
                if (ki < nk0) {
                    if (intd) {
                        const int g = (int)ak[r];
                        const int dkj = metric == 0 ? (int)kept_u[ki] + uji - 2 * g : 1 - g;
                        pred = dkj <= tj;
                    } else {
                        const float nkk = metric == 2 ? a.norms[kept_ids[ki]] : 1.0f;
                        const double gd = gram_dist(ak[r], metric, kept_u[ki], uj, nkk, nj);
                        pred = alpha * gd < (double)dj;
                        if constexpr (NT > 1)
                            unc = idj >= 0 && a.band > 0.0 &&
                                  near_boundary(alpha, gd, dj, a.band, metric, kept_u[ki], uj,
                                                kept_s[ki], sq);
                    }
                }
                bk |= __ballot(pred && !unc);
                if constexpr (NT > 1) {
                    u64 m = __ballot(unc);
                    while (m) {
                        const int l = __ffsll((long long)m) - 1;
                        m &= m - 1;
                        const int w = kept_ids[kt * 16 + 4 * (l >> 4) + r];
                        const int v = __builtin_amdgcn_readlane(idj, l & 15);
                        const float dv =
                            __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dj), l & 15));
                        const float dwv = walk_pair_dist<CPL>(a, w, v, lane);
                        if (alpha * (double)dwv < (double)dv) bk |= 1ull << l;
                        ++nrecheck;
                    }
                }
            }
        }
        const unsigned domk = (unsigned)((bk | (bk >> 16) | (bk >> 32) | (bk >> 48)) & 0xffffull);
        // mask of the earlier tile candidates that would dominate candidate l % 16
        unsigned mj = 0;
#pragma unroll
        for (int ii = 0; ii < 16; ++ii) mj |= (unsigned)((bt[ii & 3] >> (16 * (ii >> 2) + jr)) & 1ull) << ii;
        // resolve the candidates in order (wavefront-uniform). Lanes 0..15
        // hold candidates 0..15 of the tile. Skipped outright: past the end
        // (EMPTY keys sort last), the same vertex as the candidate before it
        // (equal keys are adjacent), dominated by a kept row of an earlier
        // tile; the rest are tested against this tile's kept candidates.
        const unsigned valid16 = (unsigned)(__ballot(key != EMPTY_KEY) & 0xffffull);
        u64 kb = __shfl(key, (jr + 15) & 15);
        if (jr == 0) kb = prev;
        const unsigned dup16 = (unsigned)(__ballot(key == kb) & 0xffffull);
        unsigned cand = valid16 & ~dup16 & ~domk;
        unsigned keptj = 0;
        bool stop = valid16 != 0xffffu;
        while (cand) {
            const int j = __builtin_ctz(cand);
            cand &= cand - 1u;
            const unsigned mjj = (unsigned)__builtin_amdgcn_readlane((int)mj, j);
            if (mjj & keptj) continue;
            keptj |= 1u << j;
            if (nk + __popc(keptj) == R) {
                stop = true;
                break;
            }
        }
        prev = readlane64(key, 15);
        // append the kept candidates (rows, ids, distances, outputs)
        if ((keptj >> jr) & 1u) {
            const int kr = nk + __popc(keptj & ((1u << jr) - 1u));
            unsigned char* dst = khi + (size_t)kr * rs + q * KD * 16;
#pragma unroll
            for (int s2 = 0; s2 < KD; ++s2) {
                *(uint4*)(dst + s2 * 16) = hi[s2];
                if constexpr (NT > 1) *(uint4*)(dst + klo_off + s2 * 16) = lo[s2];
            }
            if (q == 0) {
                kept_ids[kr] = idj;
                kept_d[kr] = dj;
                kept_u[kr] = uj;
                if constexpr (NT > 1) kept_s[kr] = sq;
                a.rows_out[p * R + kr] = idj;
                a.dist_out[p * R + kr] = dj;
                count_reverse(a, idj);
            }
        }
        nk += __popc(keptj);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        return stop;
    };
    if constexpr (NT == 1) {
        for (int J = 0; J < ntiles && nk < R; ++J)
            if ((J & 1) ? tile(J, fragB) : tile(J, fragA)) break;
    } else {
        for (int J = 0; J < ntiles && nk < R; ++J)
            if (tile(J, fragA)) break;
    }
    if (lane == 0) {
        a.deg_out[p] = nk;
        if (nrecheck && a.rechecks)
            atomicAdd(&a.rechecks[blockIdx.x & (CNT_SLOTS - 1)], (u64)nrecheck);
    }
}

// ----------------------------------------------- MFMA prune, K-sliced (dim > 128)

// LDS bytes per wavefront of k_prune_mfma_ks: sorted and unsorted keys, kept
// ids, key terms and squared norms (no row fragments: they are re-read)
__host__ __device__ inline size_t mfma_ks_lds(int wcap, int R) {
    return (size_t)2 * wcap * sizeof(u64) + ((size_t)R * 12 + 15) / 16 * 16;
}

// this lane's 32 dimensions [d0, d0 + 32) of row id as four MFMA fragments:
// NT == 1 the bfloat16 copy's values (exact), NT == 3 the float32 values
// (minus the centre row's when pc >= 0) split as hi + lo; zeros for id < 0.
// sq accumulates the squares of the row's own values.
template <int NT>
__device__ __forceinline__ void load_slice(const PruneArgs& a, int64_t id, int dim, int d0,
                                           const float* pcv, uint4* hi, uint4* lo, float& sq) {
    if (id < 0) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            hi[f] = make_uint4(0u, 0u, 0u, 0u);
            lo[f] = hi[f];
        }
        return;
    }
    if constexpr (NT == 1) {
        const uint4* r = (const uint4*)(a.xb + (id * dim + d0) * 2);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            hi[f] = r[f];
            lo[f] = make_uint4(0u, 0u, 0u, 0u);
            sq = dot2x4<1>(hi[f], hi[f], sq);
        }
    } else {
        const float4* r = (const float4*)(a.X + id * dim + d0);
        float4 x[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) x[t] = r[t];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            float v[8] = {x[2 * f].x, x[2 * f].y, x[2 * f].z, x[2 * f].w,
                          x[2 * f + 1].x, x[2 * f + 1].y, x[2 * f + 1].z, x[2 * f + 1].w};
#pragma unroll
            for (int e2 = 0; e2 < 8; ++e2) {
                sq = fmaf(v[e2], v[e2], sq);
                if (pcv) v[e2] -= pcv[8 * f + e2];
            }
            split8<NT>(v, hi[f], lo[f]);
        }
    }
}

// Prune(p, W) with the Gram products on bfloat16 MFMA for dim = 128 * nsl
// (nsl = 2..8). As k_prune_mfma, but each 16-candidate tile's Grams (with
// itself, then with each 16 kept rows in turn) accumulate in registers over
// slices of 128 dimensions: per slice each lane loads 32 dimensions of its
// row and of a kept row (read again from memory, where they stay in L2), so
// no buffer grows with the dimension. NT == 1: rows exact in bfloat16 with
// exact sums (the bfloat16 copy; every decision exact); NT == 3: hi/lo split
// of the float rows (centred at p for squared L2: CENTER), pairs near the
// boundary decided again with the float32 walk's arithmetic (CPL: the walk's
// chunks per lane).
template <int NT, bool CENTER, int CPL>
__global__ __launch_bounds__(256) void k_prune_mfma_ks(PruneArgs a) {
    extern __shared__ unsigned char psm[];
    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int64_t i = xcd_block() * wpb + wib;
    if (i >= a.n_items) return;
    const int R = a.R;
    unsigned char* base = psm + (size_t)wib * mfma_ks_lds(a.wcap, R);
    u64* lkeys = (u64*)base;
    u64* lraw = lkeys + a.wcap;
    int* kept_ids = (int*)(lraw + a.wcap);
    float* kept_u = (float*)(kept_ids + R);
    float* kept_s = kept_u + R;
    const int64_t p = a.item_base + (a.items ? (int64_t)a.items[i] : i);
    const int64_t e = p - a.extra_index_base;
    u64 *wk, *ws;
    const int nW = prune_collect<CPL, NT == 1>(a, p, e, lane, lkeys, lraw, &wk, &ws);
    if (nW < 0) return;
    (void)wk;
    if (!ws) {  // lists longer than 1024 are the walk's (run with list_filter 2)
        if (lane == 0) atomicOr(a.err, 2);
        return;
    }
    const int dim = a.nch * 4;
    const int nsl = dim >> 7;
    const int jr = lane & 15, q = lane >> 4;
    const int metric = a.metric;
    const double alpha = (double)a.alpha, inv_alpha = 1.0 / alpha;
    int nk = 0;
    u64 prev = EMPTY_KEY, nrecheck = 0;
    const int ntiles = (nW + 15) >> 4;
    // this lane's 32 dimensions of the centre row p in slice sl
    auto centre = [&](int sl, float* pc) {
        const float4* pr = (const float4*)(a.X + p * dim + sl * 128 + q * 32);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const float4 x = pr[t];
            pc[4 * t] = x.x;
            pc[4 * t + 1] = x.y;
            pc[4 * t + 2] = x.z;
            pc[4 * t + 3] = x.w;
        }
    };
    for (int J = 0; J < ntiles && nk < R; ++J) {
        const int c = J * 16 + jr;
        const u64 key = c < nW ? ws[c] : EMPTY_KEY;
        const int idj = key == EMPTY_KEY ? -1 : (int)(unsigned)(key & 0xffffffffu);
        const float dj = key == EMPTY_KEY ? INFINITY : fval((unsigned)(key >> 32));
        const float nj = (metric == 2 && idj >= 0) ? a.norms[idj] : 1.0f;
        const int nk0 = nk, nkt = (nk0 + 15) >> 4;
        // the tile with itself
        floatx4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
        float sq = 0.0f;
        for (int sl = 0; sl < nsl; ++sl) {
            float pc[CENTER ? 32 : 1];
            if constexpr (CENTER) centre(sl, pc);
            uint4 hi[4], lo[4];
            load_slice<NT>(a, idj, dim, sl * 128 + q * 32, CENTER ? pc : nullptr, hi, lo, sq);
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                acc = mfma16(hi[f], hi[f], acc);
                if constexpr (NT > 1) {
                    acc = mfma16(hi[f], lo[f], acc);
                    acc = mfma16(lo[f], hi[f], acc);
                }
            }
        }
        sq += __shfl_xor(sq, 16);
        sq += __shfl_xor(sq, 32);
        // key terms: d(p, v) for float rows, |v|^2 for exact rows
        const float uj = NT > 1 ? dj : sq;
        const bool intd = NT == 1 && metric != 2;
        const int tj = intd ? dom_threshold(alpha, inv_alpha, dj) : 0;
        const int uji = intd && metric == 0 ? (int)uj : 0;
        // pairs (ii, jr), ii = 4 q + r, ii < jr
        u64 bt[4], ut[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ii = 4 * q + r;
            bool pred, unc = false;
            if (intd) {
                const int g = (int)acc[r];
                const int dij = metric == 0 ? __shfl(uji, ii) + uji - 2 * g : 1 - g;
                pred = ii < jr && dij <= tj;
            } else {
                const float ui = __shfl(uj, ii);
                const float ni = __shfl(nj, ii);
                const float si = __shfl(sq, ii);
                const double gd = gram_dist(acc[r], metric, ui, uj, ni, nj);
                pred = ii < jr && alpha * gd < (double)dj;
                if constexpr (NT > 1)
                    unc = ii < jr && idj >= 0 && a.band > 0.0 &&
                          near_boundary(alpha, gd, dj, a.band, metric, ui, uj, si, sq);
            }
            bt[r] = __ballot(pred && !unc);
            ut[r] = __ballot(unc);
        }
        if constexpr (NT > 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                u64 m = ut[r];
                while (m) {
                    const int l = __ffsll((long long)m) - 1;
                    m &= m - 1;
                    const int w = __builtin_amdgcn_readlane(idj, 4 * (l >> 4) + r);
                    const int v = __builtin_amdgcn_readlane(idj, l & 15);
                    const float dv =
                        __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dj), l & 15));
                    const float dwv = walk_pair_dist<CPL>(a, w, v, lane);
                    if (alpha * (double)dwv < (double)dv) bt[r] |= 1ull << l;
                    ++nrecheck;
                }
            }
        }
        // each 16 kept rows against the tile
        u64 bk = 0ull;
        for (int kt = 0; kt < nkt; ++kt) {
            const int kr = kt * 16 + jr;
            const int kid = kr < nk0 ? kept_ids[kr] : -1;
            floatx4_t ak = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int sl = 0; sl < nsl; ++sl) {
                float pc[CENTER ? 32 : 1];
                if constexpr (CENTER) centre(sl, pc);
                float dummy = 0.0f;
                uint4 hi[4], lo[4], khi[4], klo[4];
                load_slice<NT>(a, idj, dim, sl * 128 + q * 32, CENTER ? pc : nullptr, hi, lo,
                               dummy);
                load_slice<NT>(a, kid, dim, sl * 128 + q * 32, CENTER ? pc : nullptr, khi, klo,
                               dummy);
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    ak = mfma16(khi[f], hi[f], ak);
                    if constexpr (NT > 1) {
                        ak = mfma16(khi[f], lo[f], ak);
                        ak = mfma16(klo[f], hi[f], ak);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ki = kt * 16 + 4 * q + r;
                bool pred = false, unc = false;
                if (ki < nk0) {
                    if (intd) {
                        const int g = (int)ak[r];
                        const int dkj = metric == 0 ? (int)kept_u[ki] + uji - 2 * g : 1 - g;
                        pred = dkj <= tj;
                    } else {
                        const float nkk = metric == 2 ? a.norms[kept_ids[ki]] : 1.0f;
                        const double gd = gram_dist(ak[r], metric, kept_u[ki], uj, nkk, nj);
                        pred = alpha * gd < (double)dj;
                        if constexpr (NT > 1)
                            unc = idj >= 0 && a.band > 0.0 &&
                                  near_boundary(alpha, gd, dj, a.band, metric, kept_u[ki], uj,
                                                kept_s[ki], sq);
                    }
                }
                bk |= __ballot(pred && !unc);
                if constexpr (NT > 1) {
                    u64 m = __ballot(unc);
                    while (m) {
                        const int l = __ffsll((long long)m) - 1;
                        m &= m - 1;
                        const int w = kept_ids[kt * 16 + 4 * (l >> 4) + r];
                        const int v = __builtin_amdgcn_readlane(idj, l & 15);
                        const float dv =
                            __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dj), l & 15));
                        const float dwv = walk_pair_dist<CPL>(a, w, v, lane);
                        if (alpha * (double)dwv < (double)dv) bk |= 1ull << l;
                        ++nrecheck;
                    }
                }
            }
        }
        const unsigned domk = (unsigned)((bk | (bk >> 16) | (bk >> 32) | (bk >> 48)) & 0xffffull);
        unsigned mj = 0;
#pragma unroll
        for (int ii = 0; ii < 16; ++ii) mj |= (unsigned)((bt[ii & 3] >> (16 * (ii >> 2) + jr)) & 1ull) << ii;
        // resolve the 16 candidates in order (as k_prune_mfma)
        const unsigned valid16 = (unsigned)(__ballot(key != EMPTY_KEY) & 0xffffull);
        u64 kb = __shfl(key, (jr + 15) & 15);
        if (jr == 0) kb = prev;
        const unsigned dup16 = (unsigned)(__ballot(key == kb) & 0xffffull);
        unsigned cand = valid16 & ~dup16 & ~domk;
        unsigned keptj = 0;
        bool stop = valid16 != 0xffffu;
        while (cand) {
            const int j = __builtin_ctz(cand);
            cand &= cand - 1u;
            const unsigned mjj = (unsigned)__builtin_amdgcn_readlane((int)mj, j);
            if (mjj & keptj) continue;
            keptj |= 1u << j;
            if (nk + __popc(keptj) == R) {
                stop = true;
                break;
            }
        }
        prev = readlane64(key, 15);
        if (((keptj >> jr) & 1u) && q == 0) {
            const int kr = nk + __popc(keptj & ((1u << jr) - 1u));
            kept_ids[kr] = idj;
            kept_u[kr] = uj;
            kept_s[kr] = sq;
            a.rows_out[p * R + kr] = idj;
            a.dist_out[p * R + kr] = dj;
            count_reverse(a, idj);
        }
        nk += __popc(keptj);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (stop) break;
    }
    if (lane == 0) {
        a.deg_out[p] = nk;
        if (nrecheck && a.rechecks)
            atomicAdd(&a.rechecks[blockIdx.x & (CNT_SLOTS - 1)], (u64)nrecheck);
    }
}

// ------------------------------------------------------------ small kernels

// one wavefront per row: offsets, degree, id range, self-loops, duplicates
__global__ __launch_bounds__(256) void k_validate(const int64_t* offs, const int32_t* nbrs,
                                                  int64_t n, int64_t nnz, int R, int* flags) {
    __shared__ int rowbuf[4][WAVE];
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    const int64_t v = (int64_t)blockIdx.x * 4 + w;
    if (v >= n) return;
    const int64_t b = offs[v], e = offs[v + 1];
    if (b > e || b < 0 || e > nnz) {
        if (lane == 0) atomicOr(flags, 1);
        return;
    }
    const int64_t deg = e - b;
    if (deg > R || deg > WAVE) {
        if (lane == 0) atomicOr(flags, 2);
        return;
    }
    const int x = lane < deg ? nbrs[b + lane] : -1;
    int f = 0;
    if (lane < deg) {
        if (x < 0 || x >= n) f |= 4;
        if (x == v) f |= 8;
    }
    rowbuf[w][lane] = x;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < deg)
        for (int t = 0; t < lane; ++t)
            if (rowbuf[w][t] == x) f |= 16;
    int all = 0;
#pragma unroll
    for (int bit = 4; bit <= 16; bit <<= 1)
        if (__ballot((f & bit) != 0) != 0ull) all |= bit;
    if (lane == 0 && all) atomicOr(flags, all);
}

__global__ void k_pad_adjacency(const int64_t* offs, const int32_t* nbrs, int64_t n, int rp,
                                int32_t* out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * rp) return;
    const int64_t v = t / rp;
    const int j = (int)(t - v * rp);
    const int64_t b = offs[v], e = offs[v + 1];
    out[t] = j < e - b ? nbrs[b + j] : -1;
}

// Breadth-first order of a graph given as padded adjacency [n x rp] (-1
// filled) from `root`, used only as a processing order: searches of vertices
// close in the graph then run in neighbouring wavefronts and share L2. Within
// a level the order follows atomics and is not deterministic; no result
// depends on it. order[0..n) receives every vertex once. The visited set is a
// bitmap of n bits (small enough to stay in L2); a plain read filters out
// most visited neighbours before the atomic.
// ctl: [0] order tail, [1] [2] current frontier order[s, e), [3] blocks of
// the running level that have finished
__global__ void k_bfs_init(int64_t n, int32_t root, unsigned* vis, int32_t* order, unsigned* ctl) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t words = (n + 31) >> 5;
    if (t >= words) return;
    vis[t] = t == (root >> 5) ? 1u << (root & 31) : 0u;
    if (t == 0) {
        order[0] = root;
        ctl[0] = 1u;
        ctl[1] = 0u;
        ctl[2] = 1u;
        ctl[3] = 0u;
    }
}

// appends the flagged values of a block to order[tail...]: one global atomic
// per block (BFS_T threads), offsets from wavefront ballots and LDS
#define BFS_T 1024
__device__ __forceinline__ void block_append(bool flag, int32_t val, int32_t* order,
                                             unsigned* tail) {
    __shared__ unsigned wcount[BFS_T / WAVE];
    __shared__ unsigned bbase;
    const int lane = lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const u64 m = __ballot(flag);
    if (lane == 0) wcount[wid] = (unsigned)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned tot = 0;
        for (int w2 = 0; w2 < nw; ++w2) {
            const unsigned c = wcount[w2];
            wcount[w2] = tot;
            tot += c;
        }
        bbase = tot ? atomicAdd(tail, tot) : 0u;
    }
    __syncthreads();
    if (flag) order[bbase + wcount[wid] + __popcll(m & lanemask_lt(lane))] = val;
}

// one level: the frontier order[ctl[1], ctl[2]), one thread per (vertex,
// slot) over a fixed grid (block-uniform strides, so every thread of a block
// takes part in each append). The last block to finish makes the appended
// vertices the next frontier, so levels follow one another on the stream
// without the host; a level with an empty frontier does nothing.
__global__ __launch_bounds__(BFS_T) void k_bfs_level(const int32_t* padj, int rp, int64_t n,
                                                     int32_t* order, unsigned* vis, unsigned* ctl) {
    const int64_t s = ctl[1], e = ctl[2];
    const int64_t total = (e - s) * rp;
    const bool narrow = total <= 0xffffffffll;  // 32-bit division (block-uniform)
    for (int64_t b0 = (int64_t)blockIdx.x * BFS_T; b0 < total; b0 += (int64_t)gridDim.x * BFS_T) {
        const int64_t t = b0 + threadIdx.x;
        bool found = false;
        int32_t w = -1;
        if (t < total) {
            int64_t q;
            if (narrow) q = (int64_t)((uint32_t)t / (uint32_t)rp);
            else q = t / rp;
            const int32_t u = order[s + q];
            w = padj[(int64_t)u * rp + (int)(t - q * rp)];
            if (w >= 0 && w < n) {
                const unsigned bit = 1u << (w & 31);
                if (!(__atomic_load_n(&vis[w >> 5], __ATOMIC_RELAXED) & bit))
                    found = !(atomicOr(&vis[w >> 5], bit) & bit);
            }
        }
        block_append(found, w, order, ctl);
        __syncthreads();  // bbase and wcount are reused by the next stride
    }
    // every wavefront of the block has read the frontier bounds before the
    // block counts as finished: a block whose loop ran no stride has had no
    // barrier yet, and the last block's update of the bounds must not reach
    // one of its wavefronts that has not started
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&ctl[3], 1u) == gridDim.x - 1) {
            // every block has read the bounds and made its appends
            __threadfence();
            const unsigned t = atomicAdd(&ctl[0], 0u);
            atomicExch(&ctl[1], (unsigned)e);
            atomicExch(&ctl[2], t);
            atomicExch(&ctl[3], 0u);
        }
    }
}

// vertices no level reached, after the others
__global__ __launch_bounds__(BFS_T) void k_bfs_rest(int64_t n, const unsigned* vis, int32_t* order,
                                                    unsigned* tail) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool miss = t < n && !((vis[t >> 5] >> (t & 31)) & 1u);
    block_append(miss, (int32_t)t, order, tail);
}

// ------------------------------------------------ reachability and its repair

// One pass of the builder's reachability repair, over rows of R ids (-1
// padded, deg[v] used) and the reached bits of a search from the entry:
// heads are the unreached vertices no unreached vertex links to (or, when
// there are none, those no unreached vertex of smaller id links to); each
// proposes to its
// nearest reached vertex with a free slot, else to its nearest reached
// vertex, and every vertex accepts its nearest proposals. Keys are (float32
// distance key, id); distances summed in index order (exact on integers).
__device__ __forceinline__ bool reached_bit(const unsigned* vis, int64_t v) {
    return (vis[v >> 5] >> (v & 31)) & 1u;
}

__device__ __forceinline__ float row_dist(const float* X, int dim, int metric, const float* norms,
                                          int64_t a, int64_t b) {
    const float* x = X + a * dim;
    const float* y = X + b * dim;
    float acc = 0.0f;
    if (metric == 0) {
        for (int j = 0; j < dim; ++j) {
            const float t = x[j] - y[j];
            acc = fmaf(t, t, acc);
        }
        return acc;
    }
    for (int j = 0; j < dim; ++j) acc = fmaf(x[j], y[j], acc);
    return metric == 1 ? 1.0f - acc : 1.0f - acc / (norms[a] * norms[b]);
}

// ctl: [0] heads, [1] smallest unreached id, [2] heads left to the global scan
// inu: bit 0 when an unreached vertex links to the vertex, bit 1 when one of
// smaller id does
__global__ void k_rep_clear(int64_t n, unsigned char* inu, int32_t* cnt, int32_t* cur,
                            unsigned long long* ctl) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        inu[t] = 0;
        cnt[t] = 0;
        cur[t] = 0;
    }
    if (t == 0) {
        ctl[0] = 0;
        ctl[1] = ~0ull;
        ctl[2] = 0;
    }
}

__global__ void k_rep_mark(const int32_t* rows, const int32_t* deg, int R, int64_t n,
                           const unsigned* vis, unsigned char* inu) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || reached_bit(vis, v)) return;
    for (int j = 0; j < deg[v]; ++j) {
        const int32_t w = rows[v * R + j];
        if (w >= 0 && w < n && !reached_bit(vis, w)) {
            unsigned* word = reinterpret_cast<unsigned*>(inu + (w & ~3ll));
            const unsigned bits = (v < w ? 3u : 1u) << (8 * (w & 3));
            atomicOr(word, bits);
        }
    }
}

__global__ void k_rep_heads(int64_t n, const unsigned* vis, const unsigned char* inu,
                            unsigned long long* ctl) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool un = u < n && !reached_bit(vis, u);
    const bool head = un && !(inu[u] & 1u);
    const u64 m = __ballot(head);
    if (m && lane_id() == __ffsll((long long)m) - 1) atomicAdd(&ctl[0], (unsigned long long)__popcll(m));
    if (un) atomicMin(&ctl[1], (unsigned long long)u);
}

// mode 0: no unreached vertex links to u; mode 1: none of smaller id does
__device__ __forceinline__ bool rep_is_head(int64_t u, const unsigned* vis,
                                            const unsigned char* inu, int64_t mode) {
    if (reached_bit(vis, u)) return false;
    return !(inu[u] & (mode ? 2u : 1u));
}

// a head's proposal from its exact k-NN list (sorted by (d, id)): the first
// reached entry with a free slot is the nearest such vertex of all, since
// every vertex nearer than the list's last lies in the list; heads without
// one go to the global scan. Proposal of head u: target pt[u], key pk[u] =
// (distance key, u)
__global__ void k_rep_propose_knn(int64_t n, const float* X, int dim, int metric,
                                  const float* norms, const int32_t* knn, int K,
                                  const unsigned* vis, const unsigned char* inu,
                                  const int32_t* deg, int R, int64_t only, int32_t* pt,
                                  unsigned long long* pk, int32_t* fb, unsigned long long* ctl) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n || !rep_is_head(u, vis, inu, only)) return;
    int64_t rf = -1;
    for (int j = 0; j < K && rf < 0; ++j) {
        const int32_t w = knn[u * K + j];
        if (w >= 0 && w < n && reached_bit(vis, w) && deg[w] < R) rf = w;
    }
    if (rf < 0) {
        fb[atomicAdd(&ctl[2], 1ull)] = (int32_t)u;
        return;
    }
    const float d = row_dist(X, dim, metric, norms, u, rf);
    pt[u] = (int32_t)rf;
    pk[u] = ((unsigned long long)fkey(d) << 32) | (unsigned long long)u;
}

// the candidates of the global scan: reached vertices with a free slot
// (all_reached: every reached vertex), appended in any order (*cnt of them)
__global__ void k_rep_cands(int64_t n, const unsigned* vis, const int32_t* deg, int R,
                            int all_reached, int32_t* cand, unsigned long long* cnt) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = v < n && reached_bit(vis, v) && (all_reached || deg[v] < R);
    const u64 m = __ballot(in);
    if (m == 0ull) return;
    unsigned long long base = 0;
    const int lead = __ffsll((long long)m) - 1;
    if (lane_id() == lead) base = atomicAdd(cnt, (unsigned long long)__popcll(m));
    base = __shfl(base, lead);
    if (in) cand[base + __popcll(m & lanemask_lt(lane_id()))] = (int32_t)v;
}

// the global scan for REP_TILE heads per block (their rows staged in LDS):
// each thread takes candidate rows in turn and keeps, per head, the least
// (distance key, id); the block's least per head becomes its proposal
constexpr int REP_TILE = 16;
__global__ __launch_bounds__(256) void k_rep_propose_scan(int64_t n, const float* X, int dim,
                                                          int metric, const float* norms,
                                                          const int32_t* fb, int64_t nfb,
                                                          const int32_t* cand, int64_t ncand,
                                                          int32_t* pt, unsigned long long* pk) {
    extern __shared__ float hrow[];  // REP_TILE x dim
    __shared__ unsigned long long sbest[REP_TILE];
    const int64_t h0 = (int64_t)blockIdx.x * REP_TILE;
    const int nh = (int)min<int64_t>(REP_TILE, nfb - h0);
    for (int t = threadIdx.x; t < REP_TILE * dim; t += blockDim.x) {
        const int h = t / dim, j = t - h * dim;
        hrow[t] = h < nh ? X[(int64_t)fb[h0 + h] * dim + j] : 0.0f;
    }
    if (threadIdx.x < REP_TILE) sbest[threadIdx.x] = ~0ull;
    __syncthreads();
    unsigned long long best[REP_TILE];
#pragma unroll
    for (int h = 0; h < REP_TILE; ++h) best[h] = ~0ull;
    for (int64_t c = threadIdx.x; c < ncand; c += blockDim.x) {
        const int64_t v = cand[c];
        const float* y = X + v * dim;
        float acc[REP_TILE];
#pragma unroll
        for (int h = 0; h < REP_TILE; ++h) acc[h] = 0.0f;
        for (int j = 0; j < dim; ++j) {
            const float yj = y[j];
#pragma unroll
            for (int h = 0; h < REP_TILE; ++h) {
                if (metric == 0) {
                    const float t = hrow[h * dim + j] - yj;
                    acc[h] = fmaf(t, t, acc[h]);
                } else {
                    acc[h] = fmaf(hrow[h * dim + j], yj, acc[h]);
                }
            }
        }
#pragma unroll
        for (int h = 0; h < REP_TILE; ++h) {
            if (h >= nh) break;
            float d = acc[h];
            if (metric == 1) d = 1.0f - acc[h];
            if (metric == 2) d = 1.0f - acc[h] / (norms[fb[h0 + h]] * norms[v]);
            const unsigned long long key = ((unsigned long long)fkey(d) << 32) | (unsigned long long)v;
            best[h] = key < best[h] ? key : best[h];
        }
    }
#pragma unroll
    for (int h = 0; h < REP_TILE; ++h)
        if (h < nh && best[h] != ~0ull) atomicMin(&sbest[h], best[h]);
    __syncthreads();
    if (threadIdx.x >= nh) return;
    const unsigned long long t = sbest[threadIdx.x];
    if (t == ~0ull) return;
    const int64_t u = fb[h0 + threadIdx.x];
    pt[u] = (int32_t)(t & 0xffffffffull);
    pk[u] = (t & 0xffffffff00000000ull) | (unsigned long long)u;
}

// proposals grouped by target: counts, then (after a scan into off) the keys
// of each target's proposals in its segment of seg, in any order
__global__ void k_rep_count(int64_t n, const unsigned* vis, const unsigned char* inu, int64_t only,
                            const int32_t* pt, int32_t* cnt) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n && rep_is_head(u, vis, inu, only)) atomicAdd(&cnt[pt[u]], 1);
}

__global__ void k_rep_scatter(int64_t n, const unsigned* vis, const unsigned char* inu,
                              int64_t only, const int32_t* pt, const unsigned long long* pk,
                              const int64_t* off, int32_t* cur, unsigned long long* seg) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n || !rep_is_head(u, vis, inu, only)) return;
    const int32_t t = pt[u];
    seg[off[t] + atomicAdd(&cur[t], 1)] = pk[u];
}

// each target takes its nearest proposals (least keys), as many as its row
// has free slots, appended; a full row takes one, over its last entry
__global__ void k_rep_accept(int64_t n, const int32_t* cnt, const int64_t* off,
                             const unsigned long long* seg, int32_t* rows, int32_t* deg, int R,
                             unsigned long long* links) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int taken = 0;
    if (t < n && cnt[t] > 0) {
        const unsigned long long* sg = seg + off[t];
        const int c = cnt[t];
        const int take = deg[t] < R ? R - deg[t] : 1;
        unsigned long long prev = 0;
        for (int k = 0; k < take && k < c; ++k) {
            // the least key above the previous one (keys are distinct: they hold the head id)
            unsigned long long m = ~0ull;
            for (int i = 0; i < c; ++i) {
                const unsigned long long x = sg[i];
                if ((k == 0 || x > prev) && x < m) m = x;
            }
            prev = m;
            const int32_t u = (int32_t)(m & 0xffffffffull);
            if (deg[t] < R)
                rows[t * R + deg[t]++] = u;
            else
                rows[t * R + R - 1] = u;
            ++taken;
        }
    }
    int64_t tk = taken;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) tk += __shfl_xor(tk, o);
    if (lane_id() == 0 && tk) atomicAdd(links, (unsigned long long)tk);
}

// -1 after each row's used entries (row v: rows + v R, deg[v] used)
__global__ void k_pad_tail(int32_t* rows, const int32_t* deg, int64_t n, int R) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * R) return;
    if ((int)(t % R) >= deg[t / R]) rows[t] = -1;
}

// largest row length of a CSR graph, and whether its offsets are well formed
__global__ void k_csr_shape(const int64_t* offs, int64_t n, unsigned* maxdeg, int* bad) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int64_t d = offs[x + 1] - offs[x];
    if (d < 0 || d > 0x7fffffff || offs[x] < 0) {
        atomicOr(bad, 1);
        return;
    }
    atomicMax(maxdeg, (unsigned)d);
}

// one thread per row slot, so that consecutive threads write consecutive ids
__global__ void k_init_rows(const int64_t* offs, const int32_t* nbrs, int64_t n, int64_t base,
                            int R, int32_t* rows, int32_t* deg, float* rdist) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * R) return;
    const int64_t v = t / R;
    const int j = (int)(t - v * R);
    const int64_t b = offs[v], e = offs[v + 1];
    const int64_t g = base + v;
    if (j == 0) deg[g] = (int32_t)(e - b);
    if (j < e - b) {
        rows[g * R + j] = (int32_t)(base + nbrs[b + j]);
        rdist[g * R + j] = __int_as_float(0x7fc00000);  // NaN: not computed yet
    }
}

// row norms, summed in double (the float32 copy is the double result rounded)
__global__ void k_norms(const float* X, int64_t n, int dim, float* out, double* out64) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double s = 0.0;
    for (int j = 0; j < dim; ++j) {
        const double x = (double)X[v * dim + j];
        s = fma(x, x, s);
    }
    const double r = sqrt(s);
    if (out) out[v] = (float)r;
    if (out64) out64[v] = r;
}

// exclusive scan of int32 counts into int64 offsets (n+1 entries)
#define SCAN_T 256
#define SCAN_PER 4
#define SCAN_BLK (SCAN_T * SCAN_PER)

__global__ __launch_bounds__(SCAN_T) void k_scan_block(const int32_t* cnt, int64_t n,
                                                       int64_t* off, int64_t* bsum) {
    __shared__ int64_t s[SCAN_T];
    const int64_t b0 = (int64_t)blockIdx.x * SCAN_BLK;
    int64_t v[SCAN_PER];
    int64_t t = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
        const int64_t idx = b0 + threadIdx.x * SCAN_PER + j;
        v[j] = idx < n ? cnt[idx] : 0;
        t += v[j];
    }
    s[threadIdx.x] = t;
    __syncthreads();
    for (int o = 1; o < SCAN_T; o <<= 1) {
        int64_t x = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += x;
        __syncthreads();
    }
    int64_t run = s[threadIdx.x] - t;
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
        const int64_t idx = b0 + threadIdx.x * SCAN_PER + j;
        if (idx < n) off[idx] = run;
        run += v[j];
    }
    if (threadIdx.x == SCAN_T - 1) bsum[blockIdx.x] = s[SCAN_T - 1];
}

__global__ __launch_bounds__(SCAN_T) void k_scan_sums(int64_t* bsum, int64_t nb) {
    __shared__ int64_t s[SCAN_T];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += SCAN_T) {
        const int64_t idx = c0 + threadIdx.x;
        const int64_t x = idx < nb ? bsum[idx] : 0;
        s[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < SCAN_T; o <<= 1) {
            int64_t y = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += y;
            __syncthreads();
        }
        if (idx < nb) bsum[idx] = carry + s[threadIdx.x] - x;
        const int64_t tot = s[SCAN_T - 1];
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ void k_scan_add(int64_t* off, int64_t n, const int64_t* bsum, int64_t nb) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) off[idx] += bsum[idx / SCAN_BLK];
    if (idx == 0) off[n] = bsum[nb];
}

__global__ void k_count_ids(const int32_t* ids, int64_t total, int32_t* cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int32_t x = ids[t];
    if (x >= 0) atomicAdd(&cnt[x], 1);
}

__global__ void k_invert_scatter(const int32_t* nk, int64_t n, int k, const int64_t* off,
                                 int32_t* cur, int32_t* out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int32_t x = nk[t];
    if (x < 0) return;
    const int pos = atomicAdd(&cur[x], 1);
    out[off[x] + pos] = (int32_t)(t / k);
}

__global__ void k_sort_segments(const int64_t* off, int64_t n, int32_t* ids) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int64_t b = off[x], e = off[x + 1];
    for (int64_t i = b + 1; i < e; ++i) {
        const int32_t v = ids[i];
        int64_t j = i;
        while (j > b && ids[j - 1] > v) {
            ids[j] = ids[j - 1];
            --j;
        }
        ids[j] = v;
    }
}

__global__ void k_rev_count(const int32_t* rows, const int32_t* deg, int64_t s_base, int64_t n_s,
                            int R, int64_t t_base, int64_t n_t, int32_t* cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_s * R) return;
    const int64_t u = t / R;
    const int j = (int)(t - u * R);
    const int64_t g = s_base + u;
    if (j >= deg[g]) return;
    const int64_t v = (int64_t)rows[g * R + j] - t_base;
    if (v >= 0 && v < n_t) atomicAdd(&cnt[v], 1);
}

__global__ void k_rev_scatter(const int32_t* rows, const int32_t* deg, const float* rdist,
                              int64_t s_base, int64_t n_s, int R, int64_t t_base, int64_t n_t,
                              const int64_t* off, int32_t* cur, int32_t* rev, float* rev_d) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_s * R) return;
    const int64_t u = t / R;
    const int j = (int)(t - u * R);
    const int64_t g = s_base + u;
    if (j >= deg[g]) return;
    const int64_t v = (int64_t)rows[g * R + j] - t_base;
    if (v < 0 || v >= n_t) return;
    const int pos = atomicAdd(&cur[v], 1);
    rev[off[v] + pos] = (int32_t)g;
    if (rev_d) rev_d[off[v] + pos] = rdist[g * R + j];  // d(u, v) = d(v, u), same arithmetic
}

// One wavefront per vertex (R <= 64: one lane per slot). Distances a prune
// did not compute (input edges of rows no operation touched) are computed
// here with the prune's lane-group layout and summation order.
// One wavefront per vertex. With norms64 (inner product, cosine) every
// stored distance is recomputed with float64 sums and norms: 1 - <x, y> and
// 1 - <x, y> / (|x| |y|) lose digits to cancellation in float32 when the
// distance is small.
template <int CPL>
__global__ __launch_bounds__(256) void k_compact(const int32_t* rows, const int32_t* deg,
                                                 const float* rdist, const int64_t* off, int64_t N,
                                                 int R, const float* X, int nch, int G, int lgG,
                                                 int metric, const float* norms, int32_t* out_nbrs,
                                                 float* out_dists, const double* norms64) {
    __shared__ int slots[4][WAVE];
    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    const int64_t v = (int64_t)blockIdx.x * (blockDim.x >> 6) + wib;
    if (v >= N) return;
    const int dg = deg[v];
    const int64_t o = off[v];
    int32_t u = -1;
    float d = 0.0f;
    if (lane < dg) {
        u = rows[v * R + lane];
        d = rdist[v * R + lane];
        out_nbrs[o + lane] = u;
    }
    if (!out_dists) return;
    const bool miss = lane < dg && (d != d || norms64 != nullptr);
    if (lane < dg && !miss) out_dists[o + lane] = d;
    const u64 need = __ballot(miss);
    if (need == 0ull) return;
    const int cnt = __popcll(need);
    if (miss) slots[wib][__popcll(need & lanemask_lt(lane))] = lane;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int group = lane >> lgG, sub = lane & (G - 1), RPP = WAVE >> lgG;
    const int rowf = nch * 4;
    float4 pv[CPL];
    load_row_f32<CPL>(X, v, rowf, sub, G, pv);
    const float vn = metric == 2 ? norms[v] : 1.0f;
    for (int c0 = 0; c0 < cnt; c0 += RPP) {
        const int c = c0 + group;
        const int sl = c < cnt ? slots[wib][c] : 0;
        const int32_t uu = __shfl(u, sl);
        float4 ux[CPL];
        load_row_f32<CPL>(X, c < cnt ? (int64_t)uu : -1, rowf, sub, G, ux);
        if (norms64) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                s = fma((double)ux[j].x, (double)pv[j].x, s);
                s = fma((double)ux[j].y, (double)pv[j].y, s);
                s = fma((double)ux[j].z, (double)pv[j].z, s);
                s = fma((double)ux[j].w, (double)pv[j].w, s);
            }
            for (int off2 = 1; off2 < G; off2 <<= 1) s += __shfl_xor(s, off2);
            if (c < cnt && sub == G - 1) {
                const double dd = metric == 1 ? 1.0 - s : 1.0 - s / (norms64[v] * norms64[uu]);
                out_dists[o + sl] = (float)dd;
            }
        } else {
            const float acc = dist_rows<CPL>(ux, pv, metric, G);
            if (c < cnt && sub == G - 1)
                out_dists[o + sl] = finalize_dist(acc, metric, vn, metric == 2 ? norms[uu] : 1.0f);
        }
    }
}

__global__ void k_copy_rows(const int32_t* rows_a, const int32_t* deg_a, const float* dist_a,
                            const int32_t* cnt, int64_t n, int R, int32_t* rows_b, int32_t* deg_b,
                            float* dist_b) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * R) return;
    const int64_t v = t / R;
    if (cnt[v] != 0) return;  // pruned again: written by the prune
    const int j = (int)(t - v * R);
    if (j == 0) deg_b[v] = deg_a[v];
    if (j < deg_a[v]) {
        rows_b[t] = rows_a[t];
        dist_b[t] = dist_a[t];
    }
}

// value summary of X for the choice of the prune arithmetic: out[0] stays 1
// while every value is an integer, out[1] / out[2] are the order-preserving
// bits (fkey) of the minimum / maximum
__device__ __forceinline__ void value_acc(float x, bool& frac, unsigned& lo, unsigned& hi) {
    frac |= !(x == floorf(x));
    const unsigned k = fkey(x);
    lo = k < lo ? k : lo;
    hi = k > hi ? k : hi;
}

// total4 float4 values (16-byte loads), then the total % 4 tail
__global__ __launch_bounds__(256) void k_value_range(const float* X, int64_t total, unsigned* out) {
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t total4 = total >> 2;
    bool frac = false;
    unsigned lo = ~0u, hi = 0u;
    const float4* X4 = (const float4*)X;
    for (int64_t t = t0; t < total4; t += stride) {
        const float4 x = X4[t];
        value_acc(x.x, frac, lo, hi);
        value_acc(x.y, frac, lo, hi);
        value_acc(x.z, frac, lo, hi);
        value_acc(x.w, frac, lo, hi);
    }
    for (int64_t t = 4 * total4 + t0; t < total; t += stride) value_acc(X[t], frac, lo, hi);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned l2 = __shfl_xor(lo, off), h2 = __shfl_xor(hi, off);
        lo = l2 < lo ? l2 : lo;
        hi = h2 > hi ? h2 : hi;
    }
    // one set of atomics per block: the wavefronts' results meet in LDS
    __shared__ unsigned blo[4], bhi[4], bfr[4];
    const int w = threadIdx.x >> 6;
    const bool anyfrac = __ballot(frac) != 0ull;
    if (lane_id() == 0) {
        blo[w] = lo;
        bhi[w] = hi;
        bfr[w] = anyfrac ? 1u : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned l = blo[0], h = bhi[0], f = bfr[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
            l = blo[i] < l ? blo[i] : l;
            h = bhi[i] > h ? bhi[i] : h;
            f |= bfr[i];
        }
        if (f) atomicAnd(&out[0], 0u);
        atomicMin(&out[1], l);
        atomicMax(&out[2], h);
    }
}

hipError_t launch_value_range(const float* X, int64_t total, unsigned* out, hipStream_t st) {
    const unsigned init[3] = {1u, ~0u, 0u};
    hipError_t e = hipMemcpyAsync(out, init, sizeof init, hipMemcpyHostToDevice, st);
    if (e != hipSuccess || total <= 0) return e;
    int64_t blocks = (total / 4 + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_value_range, dim3((unsigned)blocks), dim3(256), 0, st, X, total, out);
    return hipGetLastError();
}

float key_to_float(unsigned k) {
    const unsigned u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float f;
    memcpy(&f, &u, sizeof f);
    return f;
}

// ------------------------------------------------------------ conversion

// float32 -> bfloat16 / float16 bits, round to nearest, ties to even
__device__ __forceinline__ unsigned short f32_to_bf16_rne(float x) {
    const unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (unsigned short)((u >> 16) | 0x0040u);  // NaN stays a (quiet) NaN
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ unsigned short f32_to_f16_rne(float x) {
    return __half_as_ushort(__float2half_rn(x));
}

// count elements, 4 per thread (src and dst are read / written in 4-element
// groups where the count allows)
__global__ void k_convert(const void* src, int st, void* dst, int dt, int64_t count, int vec) {
    const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (t >= count) return;
    const int m = count - t < 4 ? (int)(count - t) : 4;
    if (vec && m == 4 && st == 0 && dt != 0) {
        // float32 to 16-bit, aligned: one 16-byte load and one 8-byte store
        const float4 x = ((const float4*)src)[t >> 2];
        const bool b = dt == 1;
        const unsigned a0 = b ? f32_to_bf16_rne(x.x) : f32_to_f16_rne(x.x);
        const unsigned a1 = b ? f32_to_bf16_rne(x.y) : f32_to_f16_rne(x.y);
        const unsigned a2 = b ? f32_to_bf16_rne(x.z) : f32_to_f16_rne(x.z);
        const unsigned a3 = b ? f32_to_bf16_rne(x.w) : f32_to_f16_rne(x.w);
        ((uint2*)dst)[t >> 2] = make_uint2(a0 | (a1 << 16), a2 | (a3 << 16));
        return;
    }
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (e >= m) { v[e] = 0.0f; continue; }
        v[e] = st == 0 ? ((const float*)src)[t + e] : (float)((const unsigned char*)src)[t + e];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (e >= m) continue;
        if (dt == 0) ((float*)dst)[t + e] = v[e];
        else if (dt == 1) ((unsigned short*)dst)[t + e] = f32_to_bf16_rne(v[e]);
        else ((unsigned short*)dst)[t + e] = f32_to_f16_rne(v[e]);
    }
}

hipError_t launch_convert(const void* src, int src_type, void* dst, int dst_type, int64_t count,
                          hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int s = src_type == 0 ? 0 : 1;  // 0: float32, 1: uint8
    const int64_t threads = (count + 3) / 4;
    const int vec = ((uintptr_t)src & 15) == 0 && ((uintptr_t)dst & 7) == 0;
    hipLaunchKernelGGL(k_convert, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, src, s,
                       dst, dst_type, count, vec);
    return hipGetLastError();
}

// builder entry point: vertex closest to the centroid
__global__ void k_check_integral(const float* X, int64_t total, int* flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (t < total) {
        const float x = X[t];
        bad = x != floorf(x) || fabsf(x) > 1.0e6f;
    }
    if (__ballot(bad) != 0ull && lane_id() == 0) atomicAnd(flag, 0);
}

// column sums; thread t sums column t % dim over a slab of COLSUM_ROWS rows
#define COLSUM_ROWS 1024
__global__ void k_colsum(const float* X, int64_t n, int dim, const int* flag, double* cs_d,
                         unsigned long long* cs_i) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nslab = (n + COLSUM_ROWS - 1) / COLSUM_ROWS;
    if (t >= nslab * dim) return;
    const int c = (int)(t % dim);
    const int64_t r0 = (t / dim) * COLSUM_ROWS;
    const int64_t r1 = r0 + COLSUM_ROWS < n ? r0 + COLSUM_ROWS : n;
    if (*flag) {
        long long s = 0;
        for (int64_t r = r0; r < r1; ++r) s += (long long)X[r * dim + c];
        atomicAdd(&cs_i[c], (unsigned long long)s);
    } else {
        double s = 0.0;
        for (int64_t r = r0; r < r1; ++r) s += (double)X[r * dim + c];
        atomicAdd(&cs_d[c], s);
    }
}

#define ENTRY_T 256
__global__ __launch_bounds__(ENTRY_T) void k_entry_crit(const float* X, int64_t n, int dim,
                                                        const int* flag, const double* cs_d,
                                                        const unsigned long long* cs_i,
                                                        u64* block_best) {
    // per block: (criterion, id) minimum; integral data -> exact
    // sum_j (n x_j - S_j)^2 in 128-bit; otherwise float64 sum_j (x_j - mean_j)^2
    __shared__ unsigned __int128 sc[ENTRY_T];
    __shared__ double sd[ENTRY_T];
    __shared__ int64_t sid[ENTRY_T];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool integral = *flag != 0;
    unsigned __int128 ci = ~(unsigned __int128)0;
    double cd = INFINITY;
    if (v < n) {
        if (integral) {
            ci = 0;
            for (int c = 0; c < dim; ++c) {
                const __int128 d = (__int128)n * (long long)X[v * dim + c] - (__int128)(long long)cs_i[c];
                ci += (unsigned __int128)(d * d);
            }
        } else {
            cd = 0.0;
            for (int c = 0; c < dim; ++c) {
                const double d = (double)X[v * dim + c] - cs_d[c] / (double)n;
                cd += d * d;
            }
        }
    }
    sc[threadIdx.x] = ci;
    sd[threadIdx.x] = cd;
    sid[threadIdx.x] = v < n ? v : INT64_MAX;
    __syncthreads();
    for (int o = ENTRY_T / 2; o >= 1; o >>= 1) {
        if (threadIdx.x < o) {
            const int a = threadIdx.x, b = threadIdx.x + o;
            bool take;
            if (integral)
                take = sc[b] < sc[a] || (sc[b] == sc[a] && sid[b] < sid[a]);
            else
                take = sd[b] < sd[a] || (sd[b] == sd[a] && sid[b] < sid[a]);
            if (take) {
                sc[a] = sc[b];
                sd[a] = sd[b];
                sid[a] = sid[b];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        u64* o = block_best + blockIdx.x * 3;
        if (integral) {
            o[0] = (u64)(sc[0] >> 64);
            o[1] = (u64)sc[0];
        } else {
            union { double d; u64 u; } c;
            c.d = sd[0];
            o[0] = 0;
            o[1] = c.u;
        }
        o[2] = (u64)sid[0];
    }
}

// ---------------------------------------------------------------- launchers

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_bfs_init(int64_t n, int32_t root, unsigned* vis, int32_t* order, unsigned* ctl,
                           hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (root < 0 || root >= n) root = 0;
    hipLaunchKernelGGL(k_bfs_init, dim3(nblk((n + 31) >> 5, 256)), dim3(256), 0, st, n, root, vis,
                       order, ctl);
    return hipGetLastError();
}

hipError_t launch_bfs_grow(const int32_t* padj, int rp, int64_t n, int32_t* order, unsigned* vis,
                           unsigned* ctl, unsigned* h_ctl, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipError_t e = hipSuccess;
    // at most one thread per (vertex, slot) of the largest possible frontier
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(nblk(n * rp, BFS_T), 512));
    for (;;) {
        for (int l = 0; l < BFS_BATCH; ++l)
            hipLaunchKernelGGL(k_bfs_level, dim3((unsigned)grid), dim3(BFS_T), 0, st, padj, rp, n,
                               order, vis, ctl);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(h_ctl, ctl, 3 * sizeof(unsigned), hipMemcpyDeviceToHost, st)) !=
            hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        // stop once the frontier is empty (every reachable vertex ordered)
        if (h_ctl[2] <= h_ctl[1] || (int64_t)h_ctl[0] > n) break;
    }
    return e;
}

hipError_t launch_bfs_order(const int32_t* padj, int rp, int64_t n, int32_t root, unsigned* vis,
                            int32_t* order, unsigned* ctl, unsigned* h_ctl, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipError_t e = launch_bfs_init(n, root, vis, order, ctl, st);
    if (e != hipSuccess) return e;
    if ((e = launch_bfs_grow(padj, rp, n, order, vis, ctl, h_ctl, st)) != hipSuccess) return e;
    if ((int64_t)h_ctl[0] < n) {
        hipLaunchKernelGGL(k_bfs_rest, dim3(nblk(n, BFS_T)), dim3(BFS_T), 0, st, n, vis, order, ctl);
        e = hipGetLastError();
    }
    return e;
}


// order[0, n) a permutation of 0..n-1: counts per id, then every count one
__global__ void k_perm_count(const int32_t* order, int64_t n, int32_t* cnt, int* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = order[i];
    if (v < 0 || v >= n) atomicOr(flag, 1);
    else atomicAdd(&cnt[v], 1);
}

__global__ void k_perm_check(const int32_t* cnt, int64_t n, int* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && cnt[i] != 1) atomicOr(flag, 1);
}

hipError_t launch_perm_check(const int32_t* order, int64_t n, int32_t* cnt, int* flag,
                             hipStream_t st) {
    hipError_t e = launch_zero(flag, sizeof(int), st);
    if (e != hipSuccess || n <= 0) return e;
    if ((e = launch_zero(cnt, sizeof(int32_t) * (size_t)n, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_perm_count, dim3(nblk(n, 256)), dim3(256), 0, st, order, n, cnt, flag);
    hipLaunchKernelGGL(k_perm_check, dim3(nblk(n, 256)), dim3(256), 0, st, cnt, n, flag);
    return hipGetLastError();
}

hipError_t launch_pad_tail(int32_t* rows, const int32_t* deg, int64_t n, int R, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pad_tail, dim3(nblk(n * R, 256)), dim3(256), 0, st, rows, deg, n, R);
    return hipGetLastError();
}

hipError_t launch_csr_shape(const int64_t* offs, int64_t n, unsigned* maxdeg, int* bad,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_csr_shape, dim3(nblk(n, 256)), dim3(256), 0, st, offs, n, maxdeg, bad);
    return hipGetLastError();
}

hipError_t launch_repair_heads(int64_t n, const int32_t* rows, const int32_t* deg, int R,
                               const unsigned* vis, unsigned char* inu, int32_t* cnt, int32_t* cur,
                               unsigned long long* ctl, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rep_clear, dim3(nblk(n, 256)), dim3(256), 0, st, n, inu, cnt, cur, ctl);
    hipLaunchKernelGGL(k_rep_mark, dim3(nblk(n, 256)), dim3(256), 0, st, rows, deg, R, n, vis, inu);
    hipLaunchKernelGGL(k_rep_heads, dim3(nblk(n, 256)), dim3(256), 0, st, n, vis, inu, ctl);
    return hipGetLastError();
}

hipError_t launch_repair_propose(int64_t n, const float* X, int dim, int metric, const float* norms,
                                 const int32_t* knn, int K, const unsigned* vis,
                                 const unsigned char* inu, const int32_t* deg, int R, int64_t only,
                                 int32_t* pt, unsigned long long* pk, int32_t* fb,
                                 unsigned long long* ctl, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rep_propose_knn, dim3(nblk(n, 256)), dim3(256), 0, st, n, X, dim, metric,
                       norms, knn, K, vis, inu, deg, R, only, pt, pk, fb, ctl);
    return hipGetLastError();
}

hipError_t launch_repair_cands(int64_t n, const unsigned* vis, const int32_t* deg, int R,
                               int all_reached, int32_t* cand, unsigned long long* cnt,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rep_cands, dim3(nblk(n, 256)), dim3(256), 0, st, n, vis, deg, R,
                       all_reached, cand, cnt);
    return hipGetLastError();
}

hipError_t launch_repair_scan(int64_t n, const float* X, int dim, int metric, const float* norms,
                              const int32_t* fb, int64_t nfb, const int32_t* cand, int64_t ncand,
                              int32_t* pt, unsigned long long* pk, hipStream_t st) {
    if (n <= 0 || nfb <= 0 || ncand <= 0) return hipSuccess;
    const size_t lds = sizeof(float) * REP_TILE * (size_t)dim;
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rep_propose_scan, dim3(nblk(nfb, REP_TILE)), dim3(256), lds, st, n, X, dim,
                       metric, norms, fb, nfb, cand, ncand, pt, pk);
    return hipGetLastError();
}

hipError_t launch_repair_accept(int64_t n, const unsigned* vis, const unsigned char* inu,
                                int64_t only, const int32_t* pt, const unsigned long long* pk,
                                int32_t* cnt, int32_t* cur, int64_t* off, int64_t* scan_tmp,
                                unsigned long long* seg, int32_t* rows, int32_t* deg, int R,
                                unsigned long long* links, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rep_count, dim3(nblk(n, 256)), dim3(256), 0, st, n, vis, inu, only, pt, cnt);
    hipError_t e = launch_scan(cnt, n, off, scan_tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rep_scatter, dim3(nblk(n, 256)), dim3(256), 0, st, n, vis, inu, only, pt,
                       pk, off, cur, seg);
    hipLaunchKernelGGL(k_rep_accept, dim3(nblk(n, 256)), dim3(256), 0, st, n, cnt, off, seg, rows,
                       deg, R, links);
    return hipGetLastError();
}

hipError_t launch_validate(const int64_t* offs, const int32_t* nbrs, int64_t n, int64_t nnz,
                           int R, int* flags, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate, dim3(nblk(n, 4)), dim3(256), 0, st, offs, nbrs, n, nnz, R, flags);
    return hipGetLastError();
}

hipError_t launch_pad_adjacency(const int64_t* offs, const int32_t* nbrs, int64_t n, int rp,
                                int32_t* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pad_adjacency, dim3(nblk(n * rp, 256)), dim3(256), 0, st, offs, nbrs, n, rp,
                       out);
    return hipGetLastError();
}

hipError_t launch_init_rows(const int64_t* offs, const int32_t* nbrs, int64_t n, int64_t base,
                            int R, int32_t* rows, int32_t* deg, float* rdist, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_rows, dim3(nblk(n * R, 256)), dim3(256), 0, st, offs, nbrs, n, base,
                       R, rows, deg, rdist);
    return hipGetLastError();
}

hipError_t launch_norms(const float* X, int64_t n, int dim, float* out, hipStream_t st,
                        double* out64) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_norms, dim3(nblk(n, 256)), dim3(256), 0, st, X, n, dim, out, out64);
    return hipGetLastError();
}

// row norms of 16-bit rows (tt 1: bfloat16, 2: float16), summed in double
__global__ void k_norms16(const unsigned short* X, int tt, int64_t n, int dim, float* out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double s = 0.0;
    for (int j = 0; j < dim; ++j) {
        const unsigned short h = X[v * dim + j];
        float x;
        if (tt == 1) {
            x = __uint_as_float((unsigned)h << 16);
        } else {
            union { unsigned short s; _Float16 f; } c;
            c.s = h;
            x = (float)c.f;
        }
        s = fma((double)x, (double)x, s);
    }
    out[v] = (float)sqrt(s);
}

hipError_t launch_norms16(const void* X, int tt, int64_t n, int dim, float* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (tt != 1 && tt != 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_norms16, dim3(nblk(n, 256)), dim3(256), 0, st,
                       (const unsigned short*)X, tt, n, dim, out);
    return hipGetLastError();
}

// zero `bytes` bytes at p (a multiple of 4, p 4-byte aligned): a kernel
// rather than hipMemsetAsync, so that code a caller captures into a HIP
// graph records no memset node
__global__ void k_zero_words(unsigned* p, int64_t words) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < words) p[t] = 0u;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    if ((bytes & 3) != 0 || ((uintptr_t)p & 3) != 0) return hipErrorInvalidValue;
    const int64_t words = (int64_t)(bytes >> 2);
    hipLaunchKernelGGL(k_zero_words, dim3(nblk(words, 256)), dim3(256), 0, st, (unsigned*)p,
                       words);
    return hipGetLastError();
}

template <int TT, int EFS, bool EXACT>
static void launch_search_c(const SearchArgs& a, dim3 grid, dim3 block, size_t lds, hipStream_t st) {
    // dim 128 (512-byte float32 rows over 8 lanes, 256-byte 16-bit rows over
    // 4 lanes): lanes per row fixed at compile time
    constexpr int LG128 = TT == 0 ? 3 : 2;
    if (a.cpl == 4 && a.lgG == LG128) {
        hipLaunchKernelGGL((k_beam_search<TT, EFS, 4, EXACT, LG128>), grid, block, lds, st, a);
        return;
    }
    switch (a.cpl) {
        case 1: hipLaunchKernelGGL((k_beam_search<TT, EFS, 1, EXACT, -1>), grid, block, lds, st, a); break;
        case 2: hipLaunchKernelGGL((k_beam_search<TT, EFS, 2, EXACT, -1>), grid, block, lds, st, a); break;
        case 3: hipLaunchKernelGGL((k_beam_search<TT, EFS, 3, EXACT, -1>), grid, block, lds, st, a); break;
        default: hipLaunchKernelGGL((k_beam_search<TT, EFS, 4, EXACT, -1>), grid, block, lds, st, a); break;
    }
}

template <int TT, int EFS>
static void launch_search_m(const SearchArgs& a, dim3 grid, dim3 block, size_t lds, hipStream_t st) {
    if (a.hash_mode)
        launch_search_c<TT, EFS, true>(a, grid, block, lds, st);
    else
        launch_search_c<TT, EFS, false>(a, grid, block, lds, st);
}

size_t search_lds_bytes(int hbits, int wpb) {
    return (size_t)wpb * search_lds_words(hbits) * sizeof(int);
}

hipError_t launch_search(int tt, const SearchArgs& a, int wpb, hipStream_t st) {
    if (a.nq <= 0) return hipSuccess;
    const size_t lds = search_lds_bytes(a.hbits, wpb);
    const dim3 grid(nblk(a.nq, wpb)), block(wpb * WAVE);
    const int efs = a.ef > 64 ? 2 : 1;
    if (tt == 0) {
        if (efs == 1) launch_search_m<0, 1>(a, grid, block, lds, st);
        else launch_search_m<0, 2>(a, grid, block, lds, st);
    } else if (tt == 1) {
        if (efs == 1) launch_search_m<1, 1>(a, grid, block, lds, st);
        else launch_search_m<1, 2>(a, grid, block, lds, st);
    } else {
        if (efs == 1) launch_search_m<2, 1>(a, grid, block, lds, st);
        else launch_search_m<2, 2>(a, grid, block, lds, st);
    }
    return hipGetLastError();
}

// the persistent pivot-group search: as many blocks as the device holds at
// once (each wavefront loops over the queue), no more than the groups need.
// Resident wavefronts per CU from the kernel's registers (512 VGPRs per SIMD
// lane, 4 SIMDs, at most 8 per SIMD) and its LDS (160 KiB per CU). More
// blocks than fit are harmless: they start as others end and drain the
// queue (no block waits on another).
template <int TT, int EFS, int CPL, bool EXACT, int LG>
static hipError_t launch_group_c(const GroupArgs& g, int wpb, hipStream_t st, int64_t* out) {
    const void* fn = reinterpret_cast<const void*>(&k_group_search<TT, EFS, CPL, EXACT, LG>);
    const size_t lds = search_lds_bytes(g.hbits, wpb);
    int cus = 0, dev = 0;
    hipFuncAttributes fa;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess) return e;
    const int vg = std::max(8, (fa.numRegs + 7) & ~7);
    const int per_simd = std::min(8, 512 / vg);
    int64_t per_cu = std::max(1, 4 * per_simd / wpb);
    if (lds > 0) per_cu = std::min<int64_t>(per_cu, std::max<size_t>(1, (160 * 1024) / lds));
    int64_t blocks = per_cu * std::max(cus, 1);
    if (const char* c = getenv("RNSM_GROUP_BLOCKS")) blocks = std::max(8ll, atoll(c));
    blocks = std::min<int64_t>(blocks, (g.n_groups + wpb - 1) / wpb);
    blocks = std::max<int64_t>(blocks, 8);  // every XCD's range has wavefronts of its own
    if (out) *out = blocks;
    hipLaunchKernelGGL((k_group_search<TT, EFS, CPL, EXACT, LG>), dim3((unsigned)blocks),
                       dim3(wpb * WAVE), lds, st, g);
    return hipGetLastError();
}

template <int TT, int EFS, bool EXACT>
static hipError_t launch_group_m(const SearchArgs& a, const GroupArgs& g, int wpb, hipStream_t st,
                                 int64_t* out) {
    constexpr int LG128 = TT == 0 ? 3 : 2;
    if (a.cpl == 4 && a.lgG == LG128) return launch_group_c<TT, EFS, 4, EXACT, LG128>(g, wpb, st, out);
    switch (a.cpl) {
        case 1: return launch_group_c<TT, EFS, 1, EXACT, -1>(g, wpb, st, out);
        case 2: return launch_group_c<TT, EFS, 2, EXACT, -1>(g, wpb, st, out);
        case 3: return launch_group_c<TT, EFS, 3, EXACT, -1>(g, wpb, st, out);
        default: return launch_group_c<TT, EFS, 4, EXACT, -1>(g, wpb, st, out);
    }
}

template <int TT, int EFS>
static hipError_t launch_group_e(const SearchArgs& a, const GroupArgs& g, int wpb, hipStream_t st,
                                 int64_t* out) {
    return a.hash_mode ? launch_group_m<TT, EFS, true>(a, g, wpb, st, out)
                       : launch_group_m<TT, EFS, false>(a, g, wpb, st, out);
}

hipError_t launch_group_search(int tt, const SearchArgs& shape, const GroupArgs& g, int wpb,
                               hipStream_t st, int64_t* out) {
    if (g.n_groups <= 0) return hipSuccess;
    const bool two = shape.ef > 64;
    if (tt == 0)
        return two ? launch_group_e<0, 2>(shape, g, wpb, st, out) : launch_group_e<0, 1>(shape, g, wpb, st, out);
    if (tt == 1)
        return two ? launch_group_e<1, 2>(shape, g, wpb, st, out) : launch_group_e<1, 1>(shape, g, wpb, st, out);
    return two ? launch_group_e<2, 2>(shape, g, wpb, st, out) : launch_group_e<2, 1>(shape, g, wpb, st, out);
}

// ------------------------------------------------------ pivot groups (batched form)

// pivot groups of one source in breadth-first order of the pivots: flags of
// the pivots along the order (for a scan into their group numbers)
__global__ void k_grp_flags(const int32_t* order, int64_t n, const int32_t* pivot_of,
                            int32_t* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = order ? order[i] : (int32_t)i;
    flag[i] = pivot_of[v] == -1 ? 1 : 0;
}

// group g = gpos of pivot order[i]: gpiv[g] and the pivot's group number
__global__ void k_grp_place(const int32_t* order, int64_t n, const int32_t* flag,
                            const int64_t* gpos, int32_t* gpiv, int32_t* group_of) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const int32_t v = order ? order[i] : (int32_t)i;
    gpiv[gpos[i]] = v;
    group_of[v] = (int32_t)gpos[i];
}

// followers per group
__global__ void k_grp_count(int64_t n, const int32_t* pivot_of, const int32_t* group_of,
                            int32_t* cnt) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= n) return;
    const int32_t p = pivot_of[y];
    if (p >= 0) atomicAdd(&cnt[group_of[p]], 1);
}

// followers into their group's run (order within a run is free: each
// follower's search depends on its pivot's beam only)
__global__ void k_grp_scatter(int64_t n, const int32_t* pivot_of, const int32_t* group_of,
                              const int64_t* fbeg, int32_t* cur, int32_t* fol) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= n) return;
    const int32_t p = pivot_of[y];
    if (p < 0) return;
    const int32_t g = group_of[p];
    fol[fbeg[g] + atomicAdd(&cur[g], 1)] = (int32_t)y;
}

// the prune order of the source: each pivot followed by its followers, group
// after group (group g starts at g + fbeg[g], so follower slot f of group g
// lands at g + 1 + f); one thread per group head, one per follower slot
__global__ void k_grp_order(int64_t ng, int64_t nf, const int32_t* gpiv, const int64_t* fbeg,
                            const int32_t* fol, const int32_t* pivot_of, const int32_t* group_of,
                            int32_t* order) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ng) {
        order[t + fbeg[t]] = gpiv[t];
    } else if (t - ng < nf) {
        const int64_t f = t - ng;
        const int32_t y = fol[f];
        order[(int64_t)group_of[pivot_of[y]] + 1 + f] = y;
    }
}

__global__ void k_grp_excess(int64_t ng, const int64_t* fbeg, int64_t fmax, int32_t* exc) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < ng) exc[g] = (int32_t)max<int64_t>(0, fbeg[g + 1] - fbeg[g] - fmax);
}

// follower slot f of the runs: its group from its pivot, its place in the run
__global__ void k_grp_overflow(int64_t nf, const int32_t* gpiv, const int64_t* fbeg,
                               const int32_t* fol, const int32_t* pivot_of, const int32_t* group_of,
                               int64_t fmax, const int64_t* ooff, int32_t* ofl, int32_t* oflp) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const int32_t y = fol[f];
    const int32_t g = group_of[pivot_of[y]];
    const int64_t r = f - fbeg[g] - fmax;
    if (r < 0) return;
    ofl[ooff[g] + r] = y;
    oflp[ooff[g] + r] = gpiv[g];
}

hipError_t launch_group_overflow(int64_t ng, int64_t nf, const int32_t* gpiv, const int64_t* fbeg,
                                 const int32_t* fol, const int32_t* pivot_of,
                                 const int32_t* group_of, int64_t fmax, int32_t* cnt, int64_t* ooff,
                                 int32_t* ofl, int32_t* oflp, int64_t* scan_tmp, hipStream_t st) {
    if (ng <= 0) return launch_zero(ooff, sizeof(int64_t), st);
    hipLaunchKernelGGL(k_grp_excess, dim3(nblk(ng, 256)), dim3(256), 0, st, ng, fbeg, fmax, cnt);
    hipError_t e = launch_scan(cnt, ng, ooff, scan_tmp, st);
    if (e != hipSuccess) return e;
    if (nf > 0)
        hipLaunchKernelGGL(k_grp_overflow, dim3(nblk(nf, 256)), dim3(256), 0, st, nf, gpiv, fbeg,
                           fol, pivot_of, group_of, fmax, ooff, ofl, oflp);
    return hipGetLastError();
}

__global__ void k_fill32(int32_t* p, int64_t n, int32_t v) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

hipError_t launch_fill32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill32, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_groups(const int32_t* order, int64_t n, const int32_t* pivot_of, int32_t* flag,
                         int64_t* gpos, int32_t* gpiv, int32_t* group_of, int32_t* cnt,
                         int64_t* fbeg, int32_t* fol, int32_t* prune_order, int64_t* scan_tmp,
                         int64_t n_groups, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const dim3 g(nblk(n, 256)), b(256);
    hipLaunchKernelGGL(k_grp_flags, g, b, 0, st, order, n, pivot_of, flag);
    hipError_t e = launch_scan(flag, n, gpos, scan_tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grp_place, g, b, 0, st, order, n, flag, gpos, gpiv, group_of);
    if ((e = launch_zero(cnt, sizeof(int32_t) * (size_t)std::max<int64_t>(n_groups, 1), st)) !=
        hipSuccess)
        return e;
    hipLaunchKernelGGL(k_grp_count, g, b, 0, st, n, pivot_of, group_of, cnt);
    if ((e = launch_scan(cnt, n_groups, fbeg, scan_tmp, st)) != hipSuccess) return e;
    if ((e = launch_zero(cnt, sizeof(int32_t) * (size_t)std::max<int64_t>(n_groups, 1), st)) !=
        hipSuccess)
        return e;
    hipLaunchKernelGGL(k_grp_scatter, g, b, 0, st, n, pivot_of, group_of, fbeg, cnt, fol);
    if (n_groups > 0)
        hipLaunchKernelGGL(k_grp_order, dim3(nblk(n, 256)), b, 0, st, n_groups, n - n_groups, gpiv,
                           fbeg, fol, pivot_of, group_of, prune_order);
    return hipGetLastError();
}

template <int CPL>
static void launch_prune_c(const PruneArgs& a, int need, dim3 grid, dim3 block, size_t lds,
                           hipStream_t st) {
    if (need <= 1)
        hipLaunchKernelGGL((k_prune<CPL, 1>), grid, block, lds, st, a);
    else if (need <= 2)
        hipLaunchKernelGGL((k_prune<CPL, 2>), grid, block, lds, st, a);
    else if (need <= 4)
        hipLaunchKernelGGL((k_prune<CPL, 4>), grid, block, lds, st, a);
    else
        hipLaunchKernelGGL((k_prune<CPL, 0>), grid, block, lds, st, a);
}

template <int KD, int CPL>
static void launch_prune_mfma_c(const PruneArgs& a, int nt, dim3 grid, dim3 block, size_t lds,
                                hipStream_t st) {
    if (nt == 1)
        hipLaunchKernelGGL((k_prune_mfma<KD, 1, CPL>), grid, block, lds, st, a);
    else
        hipLaunchKernelGGL((k_prune_mfma<KD, 3, CPL>), grid, block, lds, st, a);
}

// dims whose Grams the K-sliced kernel takes (slices of 128)
static bool prune_ks_dim(int dim) { return dim % 128 == 0 && dim >= 256 && dim <= 1024; }

bool prune_mfma_supported(int dim) {
    return (dim % 32 == 0 && dim >= 32 && dim <= 128) || prune_ks_dim(dim);
}

bool prune_mfma_fits(const PruneArgs& a, int nt) {
    const int dim = a.nch * 4;
    if (!prune_mfma_supported(dim) || a.R > 64) return false;
    if (prune_ks_dim(dim)) return mfma_ks_lds(a.wcap, a.R) <= 64 * 1024;
    return mfma_prune_lds(a.wcap, a.R, dim / 32, nt) <= 64 * 1024;
}

static hipError_t launch_prune_mfma_ks(const PruneArgs& b, int nt, hipStream_t st) {
    const size_t per = mfma_ks_lds(b.wcap, b.R);
    int wpb = 4;
    while (wpb > 1 && per * wpb > 64 * 1024) --wpb;
    const size_t lds = (size_t)wpb * per;
    const dim3 grid(nblk(b.n_items, wpb)), block(wpb * WAVE);
    // the float32 walk's layout (collect_dists, the re-decided pairs);
    // float rows are centred at p for squared L2
    const bool ctr = nt != 1 && b.metric == 0;
    if (b.cpl == 3) {
        if (nt == 1) hipLaunchKernelGGL((k_prune_mfma_ks<1, false, 3>), grid, block, lds, st, b);
        else if (ctr) hipLaunchKernelGGL((k_prune_mfma_ks<3, true, 3>), grid, block, lds, st, b);
        else hipLaunchKernelGGL((k_prune_mfma_ks<3, false, 3>), grid, block, lds, st, b);
    } else if (b.cpl == 4) {
        if (nt == 1) hipLaunchKernelGGL((k_prune_mfma_ks<1, false, 4>), grid, block, lds, st, b);
        else if (ctr) hipLaunchKernelGGL((k_prune_mfma_ks<3, true, 4>), grid, block, lds, st, b);
        else hipLaunchKernelGGL((k_prune_mfma_ks<3, false, 4>), grid, block, lds, st, b);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_prune_mfma(const PruneArgs& a, int nt, hipStream_t st) {
    if (a.n_items <= 0) return hipSuccess;
    const int dim = a.nch * 4;
    if (!prune_mfma_fits(a, nt) || (nt != 1 && nt != 3)) return hipErrorInvalidValue;
    if (nt == 1 && !a.xb) return hipErrorInvalidValue;
    if (prune_ks_dim(dim)) {
        PruneArgs b = a;
        b.G16 = lanes_per_row(dim / 8);
        b.lgG16 = ilog2i(b.G16);
        // the bfloat16 layout of collect_dists takes as many chunks per lane
        if (b.G16 < 1 || (dim / 8) / b.G16 != a.cpl) return hipErrorInvalidValue;
        return launch_prune_mfma_ks(b, nt, st);
    }
    const int kd = dim / 32;
    PruneArgs b = a;
    // bfloat16 layout of prune_collect: dim / 8 chunks, as many per lane as
    // the float32 layout has (kd = 1, 2, 4: 4; kd = 3: 3)
    b.G16 = lanes_per_row(dim / 8);
    b.lgG16 = ilog2i(b.G16);
    const size_t per = mfma_prune_lds(a.wcap, a.R, kd, nt);
    const int wpb = per <= 32 * 1024 ? 2 : 1;
    const size_t lds = (size_t)wpb * per;
    const dim3 grid(nblk(a.n_items, wpb)), block(wpb * WAVE);
    // the candidate-distance layout of prune_collect for dim = 32 kd
    if (b.G16 < 1 || (dim / 8) / b.G16 != (kd == 3 ? 3 : 4)) return hipErrorInvalidValue;
    switch (kd) {
        case 1: launch_prune_mfma_c<1, 4>(b, nt, grid, block, lds, st); break;
        case 2: launch_prune_mfma_c<2, 4>(b, nt, grid, block, lds, st); break;
        case 3: launch_prune_mfma_c<3, 3>(b, nt, grid, block, lds, st); break;
        default: launch_prune_mfma_c<4, 4>(b, nt, grid, block, lds, st); break;
    }
    return hipGetLastError();
}

template <int CPL>
static void launch_row_dists_c(const PruneArgs& a, bool b16, dim3 grid, dim3 block, hipStream_t st) {
    if (b16)
        hipLaunchKernelGGL((k_row_dists<CPL, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((k_row_dists<CPL, false>), grid, block, 0, st, a);
}

hipError_t launch_row_dists(const PruneArgs& a, bool b16, hipStream_t st) {
    if (a.n_items <= 0) return hipSuccess;
    if (a.R > WAVE || !a.rows_d || (b16 && !a.xb)) return hipErrorInvalidValue;
    PruneArgs b = a;
    b.G16 = lanes_per_row(a.nch / 2);
    b.lgG16 = ilog2i(b.G16);
    // the bfloat16 layout takes as many chunks per lane as the float32 one
    if (b16 && (b.G16 < 1 || (a.nch / 2) / b.G16 != a.cpl)) return hipErrorInvalidValue;
    const int64_t nb = nblk(a.n_items, 4);
    const dim3 grid((unsigned)(a.grid_cap > 0 ? std::min<int64_t>(nb, a.grid_cap) : nb)),
        block(4 * WAVE);
    switch (a.cpl) {
        case 1: launch_row_dists_c<1>(b, b16, grid, block, st); break;
        case 2: launch_row_dists_c<2>(b, b16, grid, block, st); break;
        case 3: launch_row_dists_c<3>(b, b16, grid, block, st); break;
        default: launch_row_dists_c<4>(b, b16, grid, block, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_prune(const PruneArgs& a, hipStream_t st) {
    if (a.n_items <= 0) return hipSuccess;
    const int wpb = 2;
    const size_t lds = (size_t)wpb * ((size_t)(2 * a.wcap + a.R) * sizeof(u64));
    const dim3 grid(nblk(a.n_items, wpb)), block(wpb * WAVE);
    const int rpp = WAVE / a.G;
    const int need = (a.R + rpp - 1) / rpp;
    switch (a.cpl) {
        case 1: launch_prune_c<1>(a, need, grid, block, lds, st); break;
        case 2: launch_prune_c<2>(a, need, grid, block, lds, st); break;
        case 3: launch_prune_c<3>(a, need, grid, block, lds, st); break;
        default: launch_prune_c<4>(a, need, grid, block, lds, st); break;
    }
    return hipGetLastError();
}

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + SCAN_BLK - 1) / SCAN_BLK) + 2; }

hipError_t launch_scan(const int32_t* cnt, int64_t n, int64_t* off, int64_t* tmp, hipStream_t st) {
    const int64_t nb = (n + SCAN_BLK - 1) / SCAN_BLK;
    if (n > 0)
        hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(SCAN_T), 0, st, cnt, n, off, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_T), 0, st, tmp, nb);
    hipLaunchKernelGGL(k_scan_add, dim3(nblk(n > 0 ? n : 1, 256)), dim3(256), 0, st, off, n, tmp,
                       nb);
    return hipGetLastError();
}

hipError_t launch_count_ids(const int32_t* nk, int64_t n, int k, int32_t* cnt, hipStream_t st) {
    hipError_t e = launch_zero(cnt, sizeof(int32_t) * (size_t)n, st);
    if (e != hipSuccess) return e;
    if (n > 0)
        hipLaunchKernelGGL(k_count_ids, dim3(nblk(n * k, 256)), dim3(256), 0, st, nk, n * k, cnt);
    return hipGetLastError();
}

// Gain levels of the lazy greedy from the R_k list lengths, one wavefront
// per 64 vertices: word w of level g (g < lcap <= 64) has bit i set when
// vertex 64 w + i has length g. Longer lists go to high as (length, id)
// pairs (any order: the host orders them in a heap); ctl[0] counts them,
// with one atomic per wavefront that has any (all wavefronts run at once:
// per-lane atomics on one address would queue).
__global__ void k_gain_levels(const int32_t* cnt, int64_t n, int64_t words, int lcap,
                              unsigned long long* bits, int* ctl, int2* high, int64_t cap) {
    const int lane = lane_id();
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (w >= words) return;  // whole wavefronts
    const int64_t x = w * 64 + lane;
    const int g = x < n ? cnt[x] : -1;
    u64 mine = 0ull;
    for (int l = 0; l < lcap; ++l) {
        const u64 b = __ballot(g == l);
        if (lane == l) mine = b;
    }
    if (lane < lcap) bits[(int64_t)lane * words + w] = mine;
    const u64 mh = __ballot(g >= lcap);
    if (mh != 0ull) {
        const int leader = __ffsll((long long)mh) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(&ctl[0], __popcll(mh));
        base = __shfl(base, leader);
        if (g >= lcap) {
            const int64_t i = base + __popcll(mh & lanemask_lt(lane));
            if (i < cap) high[i] = make_int2(g, (int)x);
        }
    }
}

hipError_t launch_gain_levels(const int32_t* cnt, int64_t n, int lcap, unsigned long long* bits,
                              int* ctl, int2* high, int64_t cap, hipStream_t st) {
    if (lcap < 1 || lcap > WAVE) return hipErrorInvalidValue;
    hipError_t e = hipMemsetAsync(ctl, 0, sizeof(int), st);
    if (e != hipSuccess || n <= 0) return e;
    const int64_t words = (n + 63) / 64;
    hipLaunchKernelGGL(k_gain_levels, dim3(nblk(words, 4)), dim3(4 * WAVE), 0, st, cnt, n, words,
                       lcap, bits, ctl, high, cap);
    return hipGetLastError();
}

hipError_t launch_invert_lists(const int32_t* nk, int64_t n, int k, int32_t* cnt,
                               int64_t* rk_off, int32_t* rk_ids, int64_t* scan_tmp,
                               hipStream_t st) {
    hipError_t e = launch_scan(cnt, n, rk_off, scan_tmp, st);
    if (e != hipSuccess) return e;
    e = launch_zero(cnt, sizeof(int32_t) * (size_t)n, st);
    if (e != hipSuccess) return e;
    if (n > 0) {
        hipLaunchKernelGGL(k_invert_scatter, dim3(nblk(n * k, 256)), dim3(256), 0, st, nk, n, k,
                           rk_off, cnt, rk_ids);
    }
    return hipGetLastError();
}

hipError_t launch_rev_count(const int32_t* rows, const int32_t* deg, int64_t s_base, int64_t n_s,
                            int R, int64_t t_base, int64_t n_t, int32_t* cnt, hipStream_t st) {
    if (n_s <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rev_count, dim3(nblk(n_s * R, 256)), dim3(256), 0, st, rows, deg, s_base,
                       n_s, R, t_base, n_t, cnt);
    return hipGetLastError();
}

hipError_t launch_rev_scatter(const int32_t* rows, const int32_t* deg, const float* rdist,
                              int64_t s_base, int64_t n_s, int R, int64_t t_base, int64_t n_t,
                              const int64_t* off, int32_t* cur, int32_t* rev, float* rev_d,
                              hipStream_t st) {
    if (n_s <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rev_scatter, dim3(nblk(n_s * R, 256)), dim3(256), 0, st, rows, deg, rdist,
                       s_base, n_s, R, t_base, n_t, off, cur, rev, rev_d);
    return hipGetLastError();
}

hipError_t launch_compact(const int32_t* rows, const int32_t* deg, const float* rdist,
                          const int64_t* off, int64_t N, int R, const float* X, int dim,
                          int metric, const float* norms, int32_t* out_nbrs, float* out_dists,
                          hipStream_t st, const double* norms64) {
    if (N <= 0) return hipSuccess;
    if (R > WAVE) return hipErrorInvalidValue;
    const int nch = dim / 4, G = lanes_per_row(nch);
    if (dim % 4 != 0 || G < 0) return hipErrorInvalidValue;
    const int cpl = nch / G, lgG = ilog2i(G);
    const double* n64 = metric == 0 ? nullptr : norms64;
    if (metric != 0 && !n64 && out_dists) return hipErrorInvalidValue;
    const dim3 grid(nblk(N, 4)), block(256);
    switch (cpl) {
        case 1: hipLaunchKernelGGL(k_compact<1>, grid, block, 0, st, rows, deg, rdist, off, N, R, X, nch, G, lgG, metric, norms, out_nbrs, out_dists, n64); break;
        case 2: hipLaunchKernelGGL(k_compact<2>, grid, block, 0, st, rows, deg, rdist, off, N, R, X, nch, G, lgG, metric, norms, out_nbrs, out_dists, n64); break;
        case 3: hipLaunchKernelGGL(k_compact<3>, grid, block, 0, st, rows, deg, rdist, off, N, R, X, nch, G, lgG, metric, norms, out_nbrs, out_dists, n64); break;
        default: hipLaunchKernelGGL(k_compact<4>, grid, block, 0, st, rows, deg, rdist, off, N, R, X, nch, G, lgG, metric, norms, out_nbrs, out_dists, n64); break;
    }
    return hipGetLastError();
}

hipError_t launch_copy_rows(const int32_t* rows_a, const int32_t* deg_a, const float* dist_a,
                            const int32_t* cnt, int64_t n, int R, int32_t* rows_b,
                            int32_t* deg_b, float* dist_b, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_rows, dim3(nblk(n * R, 256)), dim3(256), 0, st, rows_a, deg_a,
                       dist_a, cnt, n, R, rows_b, deg_b, dist_b);
    return hipGetLastError();
}

int64_t entry_blocks(int64_t n) { return (n + ENTRY_T - 1) / ENTRY_T; }

hipError_t launch_entry(const float* X, int64_t n, int dim, int* flag, double* cs_d,
                        unsigned long long* cs_i, u64* block_best, int64_t nblocks,
                        hipStream_t st) {
    // flag must hold 1, cs_d / cs_i must hold zeros
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_integral, dim3(nblk(n * dim, 256)), dim3(256), 0, st, X, n * dim,
                       flag);
    const int64_t nslab = (n + COLSUM_ROWS - 1) / COLSUM_ROWS;
    hipLaunchKernelGGL(k_colsum, dim3(nblk(nslab * dim, 256)), dim3(256), 0, st, X, n, dim, flag,
                       cs_d, cs_i);
    if (block_best && nblocks > 0)
        hipLaunchKernelGGL(k_entry_crit, dim3((unsigned)nblocks), dim3(ENTRY_T), 0, st, X, n, dim,
                           flag, cs_d, cs_i, block_best);
    return hipGetLastError();
}

// ------------------------------------------------- pivot selection on the device

// The lazy greedy of Algorithm 2 (phase 2) in parallel rounds. Every
// uncovered vertex x has the key (gain, smaller id first) with gain = |R_k(x)
// minus Covered|; x becomes a pivot in a round when its key is the largest,
// among the uncovered vertices, at x itself and at each of its uncovered
// followers (positions whose best key comes from the vertex there and from
// the vertices listing it). Such an x is also the sequential greedy's pick
// before any vertex it competes with, with the same followers, and picks that
// share no position commute, so the pivots and follower groups are the
// greedy's.
//
// The keys come from gains kept up to date: each newly covered y takes one
// from the gain of every x whose list holds it, i.e. every x in y's forward
// list F(y) = {x : y in R_k(x)} (N_k(y) in the merge). Coverage lives in the
// same word: covering a vertex takes SEL_COVER from its gain, so a vertex is
// covered exactly when its word is negative (an uncovered gain never is, and
// n < 2^30 keeps a covered one from wrapping), and one load gives both.
// A round is three kernels over the active vertices (those uncovered when the
// host last checked): best, each uncovered y finds the largest key of y and
// of the uncovered x in F(y) and marks as losers y and those x whose key it
// is not; pick, each uncovered non-loser becomes a pivot (covered, its gains
// taken) and appends its list to the round's items in chunks of SEL_CHUNK
// entries; take, SEL_CHUNK lanes per item cover the chunk's uncovered entries
// and take them from the gains at once. No two picks share an uncovered
// follower and none is another's, so the coverage read in a round is the
// round's starting one where it matters (other decrements never change a
// word's sign); the claim on pivot_of (-2 while uncovered) keeps the gains
// right even for a list that repeats an id.
// ctl[0]: nonzero until a round picks nothing (every round kernel then
// returns at once), ctl[1]: pivots, ctl[2]: rounds with picks, ctl[4]: active
// vertices after a compaction, ctl[5]: the round's items.
struct SelFwd {
    const int32_t* ids;   // forward lists
    const int64_t* off;   // CSR offsets, or NULL: fixed stride fk, -1 padded
    int fk;
};

constexpr int SEL_CHUNK = 16;           // list entries per take item (lanes per item)
constexpr int32_t SEL_COVER = 1 << 30;  // taken from a gain word on covering

__device__ __forceinline__ void fwd_range(const SelFwd& f, int64_t y, int64_t& b, int64_t& e) {
    if (f.off) {
        b = f.off[y];
        e = f.off[y + 1];
    } else {
        b = y * f.fk;
        e = b + f.fk;
    }
}

// key of an uncovered vertex from its gain word g >= 0
__device__ __forceinline__ u64 sel_key_of(int32_t g, int64_t x) {
    return ((u64)(unsigned)g << 32) | (u64)(0xffffffffu - (unsigned)x);
}

__global__ void k_sel_init(int64_t n, const int64_t* rk_off, unsigned char* lose, int32_t* gain,
                           int32_t* pivot_of, int64_t* ctl) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) {
        lose[x] = 0;
        gain[x] = (int32_t)(rk_off[x + 1] - rk_off[x]);
        pivot_of[x] = -2;
    }
    if (x == 0) {
        ctl[0] = 1;
        ctl[1] = 0;
        ctl[2] = 0;
        ctl[3] = 0;
        ctl[4] = n;
        ctl[5] = 0;
    }
}

// a newly covered vertex z: one less gain for every x listing it
__device__ __forceinline__ void sel_uncount(const SelFwd& f, int64_t n, int64_t z, int32_t* gain) {
    int64_t j0, j1;
    fwd_range(f, z, j0, j1);
    for (int64_t j = j0; j < j1; ++j) {
        const int32_t x = f.ids[j];
        if (x >= 0 && x < n) atomicSub(&gain[x], 1);
    }
}

// best key at y and the losers it makes; a vertex's lose byte is cleared by
// the pick kernel that reads it, so every set here is for this round. The
// keys of up to SEL_KREG forward entries stay in registers between the two
// passes.
constexpr int SEL_KREG = 8;

__device__ __forceinline__ void sel_best_one(int64_t n, int64_t y, const SelFwd& f,
                                             const int32_t* __restrict__ gain,
                                             unsigned char* __restrict__ lose) {
    const int32_t gy = gain[y];
    if (gy < 0) return;
    const u64 ky = sel_key_of(gy, y);
    u64 b = ky;
    int64_t j0, j1;
    fwd_range(f, y, j0, j1);
    if (j1 - j0 <= SEL_KREG) {
        u64 kx[SEL_KREG];
#pragma unroll
        for (int u = 0; u < SEL_KREG; ++u) {
            kx[u] = 0;  // no key: never the best (a real key is > 0 in its id half)
            if (j0 + u < j1) {
                const int32_t x = f.ids[j0 + u];
                if (x >= 0 && x < n) {
                    const int32_t g = gain[x];
                    if (g >= 0) kx[u] = sel_key_of(g, x);
                }
            }
            b = kx[u] > b ? kx[u] : b;
        }
        if (b != ky) lose[y] = 1;
#pragma unroll
        for (int u = 0; u < SEL_KREG; ++u)
            if (kx[u] != 0 && kx[u] != b) lose[f.ids[j0 + u]] = 1;
        return;
    }
    for (int64_t j = j0; j < j1; ++j) {
        const int32_t x = f.ids[j];
        if (x >= 0 && x < n) {
            const int32_t g = gain[x];
            if (g >= 0) {
                const u64 k = sel_key_of(g, x);
                b = k > b ? k : b;
            }
        }
    }
    if (b != ky) lose[y] = 1;
    for (int64_t j = j0; j < j1; ++j) {
        const int32_t x = f.ids[j];
        if (x >= 0 && x < n) {
            const int32_t g = gain[x];
            if (g >= 0 && sel_key_of(g, x) != b) lose[x] = 1;
        }
    }
}

__global__ void k_sel_best(int64_t n, const int32_t* __restrict__ act, int64_t nact, SelFwd f,
                           const int32_t* __restrict__ gain, unsigned char* __restrict__ lose,
                           int64_t* ctl) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) ctl[5] = 0;  // the round's item count (the last reader was the previous take)
    if (i >= nact || ctl[0] == 0) return;
    sel_best_one(n, act ? act[i] : i, f, gain, lose);
}

constexpr int SEL_PICK_THREADS = 1024;

// a pick x (uncovered, no loser): a pivot, covered, its gains taken; returns
// its item count (one at least: a round's picks make items even when their
// lists are empty, and a round without items ends the selection)
__device__ __forceinline__ int64_t sel_pick_one(int64_t n, int64_t x, const int64_t* off,
                                                const SelFwd& f, int32_t* gain,
                                                int32_t* pivot_of) {
    pivot_of[x] = -1;
    atomicSub(&gain[x], SEL_COVER);
    sel_uncount(f, n, x, gain);
    return max((int64_t)1, (off[x + 1] - off[x] + SEL_CHUNK - 1) / SEL_CHUNK);
}

// the round's picks: covered, taken from the gains, their lists appended to
// the items (x << 32 | chunk). The block reserves its items with one atomic
// and writes them together: item q of the block belongs to the last thread
// whose first item is at most q (a search over the block's offsets), so a
// hub's thousands of chunks are not one thread's serial loop.
__global__ void __launch_bounds__(SEL_PICK_THREADS)
k_sel_pick(int64_t n, const int32_t* act, int64_t nact, const int64_t* off, SelFwd f,
           unsigned char* lose, int32_t* gain, int32_t* pivot_of, int64_t* items, int64_t* ctl) {
    if (ctl[0] == 0) return;  // uniform: nothing writes ctl[0] during this kernel
    __shared__ int64_t first[SEL_PICK_THREADS];  // block-local offset of each thread's items
    __shared__ int32_t owner[SEL_PICK_THREADS];
    __shared__ int64_t wtot[SEL_PICK_THREADS / WAVE];
    __shared__ int64_t base, total;
    __shared__ int npk;
    const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    if (tid == 0) npk = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + tid;
    int64_t x = -1, nc = 0;
    bool pick = false;
    if (i < nact) {
        x = act ? act[i] : i;
        if (gain[x] >= 0) {
            pick = !lose[x];
            lose[x] = 0;
        }
    }
    if (pick) nc = sel_pick_one(n, x, off, f, gain, pivot_of);
    const u64 pm = __ballot(pick);
    if (lane == 0 && pm) atomicAdd(&npk, __popcll(pm));
    int64_t inc = nc;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const int64_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == WAVE - 1) wtot[w] = inc;
    __syncthreads();
    if (tid == 0) {
        int64_t sum = 0;
        for (int k = 0; k < SEL_PICK_THREADS / WAVE; ++k) {
            const int64_t t = wtot[k];
            wtot[k] = sum;
            sum += t;
        }
        total = sum;
        base = sum ? (int64_t)atomicAdd((unsigned long long*)&ctl[5], (unsigned long long)sum) : 0;
        if (npk) atomicAdd((unsigned long long*)&ctl[1], (unsigned long long)npk);
    }
    __syncthreads();
    first[tid] = wtot[w] + inc - nc;
    owner[tid] = (int32_t)x;
    __syncthreads();
    for (int64_t q = tid; q < total; q += SEL_PICK_THREADS) {
        int lo = 0, hi = SEL_PICK_THREADS - 1;  // last t with first[t] <= q
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (first[mid] <= q) lo = mid;
            else hi = mid - 1;
        }
        items[base + q] = ((int64_t)owner[lo] << 32) | (q - first[lo]);
    }
}

// entry `sub` of a take item: an uncovered follower joins the item's pick
__device__ __forceinline__ void sel_take_one(int64_t n, int64_t it, int sub, const int64_t* off,
                                             const int32_t* ids, const SelFwd& f, int32_t* gain,
                                             int32_t* pivot_of) {
    const int64_t x = it >> 32, c = it & 0xffffffffll;
    const int64_t j = off[x] + c * SEL_CHUNK + sub;
    if (j >= off[x + 1]) return;
    const int32_t y = ids[j];
    if (gain[y] < 0) return;
    if (atomicCAS(&pivot_of[y], -2, (int32_t)x) != -2) return;
    atomicSub(&gain[y], SEL_COVER);
    sel_uncount(f, n, y, gain);
}

// SEL_CHUNK lanes per item, grid-stride over the round's items; thread 0
// ends the selection's rounds when the round picked nothing
__global__ void k_sel_take(int64_t n, const int64_t* off, const int32_t* ids, SelFwd f,
                           int32_t* gain, int32_t* pivot_of, const int64_t* items, int64_t* ctl) {
    const int64_t cnt = ctl[5];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        if (cnt == 0) ctl[0] = 0;
        else ctl[2] += 1;
    }
    const int sub = threadIdx.x & (SEL_CHUNK - 1);
    const int64_t stride = ((int64_t)gridDim.x * blockDim.x) / SEL_CHUNK;
    for (int64_t w = t / SEL_CHUNK; w < cnt; w += stride)
        sel_take_one(n, items[w], sub, off, ids, f, gain, pivot_of);
}

// block-wide exclusive offset of v (a multiple of 64 threads, at most 1024)
// after one atomic reservation of the block's total in *counter; every
// thread of the block calls it
__device__ __forceinline__ int64_t sel_block_reserve(int64_t v, int64_t* counter) {
    __shared__ int64_t wtot[16];
    __shared__ int64_t base;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    int64_t inc = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const int64_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == WAVE - 1) wtot[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t sum = 0;
        const int nw = (int)(blockDim.x >> 6);
        for (int k = 0; k < nw; ++k) {
            const int64_t t = wtot[k];
            wtot[k] = sum;
            sum += t;
        }
        base = sum ? (int64_t)atomicAdd((unsigned long long*)counter, (unsigned long long)sum) : 0;
    }
    __syncthreads();
    return base + wtot[w] + inc - v;
}

// after a check batch: the still uncovered active vertices into act_out
// (ctl[4] counts them; zero at launch)
__global__ void __launch_bounds__(SEL_PICK_THREADS)
k_sel_compact(const int32_t* act, int64_t nact, const int32_t* gain, int32_t* act_out,
              int64_t* ctl) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t x = i < nact ? (act ? act[i] : i) : -1;
    const bool keep = x >= 0 && gain[x] >= 0;
    const int64_t at = sel_block_reserve(keep ? 1 : 0, &ctl[4]);
    if (keep) act_out[at] = (int32_t)x;
}

// The last rounds in one workgroup, once few vertices are left: the same
// three steps per round over act[0, nact), separated by workgroup barriers
// (the group's waves share one L1, so its global writes are visible to the
// group after a barrier), until a round picks nothing; every round with an
// uncovered vertex picks one, so at most nact + 1 rounds run.
__global__ void __launch_bounds__(SEL_PICK_THREADS)
k_sel_tail(int64_t n, const int32_t* act, int64_t nact, const int64_t* off, const int32_t* ids,
           SelFwd f, unsigned char* lose, int32_t* gain, int32_t* pivot_of, int64_t* items,
           int64_t* ctl) {
    __shared__ unsigned long long nitems;
    __shared__ int npk;
    const int tid = threadIdx.x;
    for (int64_t r = 0; r <= nact; ++r) {
        for (int64_t i = tid; i < nact; i += SEL_PICK_THREADS) sel_best_one(n, act[i], f, gain, lose);
        if (tid == 0) {
            nitems = 0;
            npk = 0;
        }
        __syncthreads();
        for (int64_t i = tid; i < nact; i += SEL_PICK_THREADS) {
            const int64_t x = act[i];
            if (gain[x] < 0) continue;
            const bool pick = !lose[x];
            lose[x] = 0;
            if (!pick) continue;
            const int64_t nc = sel_pick_one(n, x, off, f, gain, pivot_of);
            const int64_t at = (int64_t)atomicAdd(&nitems, (unsigned long long)nc);
            for (int64_t c = 0; c < nc; ++c) items[at + c] = (x << 32) | c;
            atomicAdd(&npk, 1);
        }
        __syncthreads();
        const int64_t cnt = (int64_t)nitems;
        if (cnt == 0) break;  // uniform
        if (tid == 0) {
            ctl[1] += npk;
            ctl[2] += 1;
        }
        for (int64_t w = tid / SEL_CHUNK; w < cnt; w += SEL_PICK_THREADS / SEL_CHUNK)
            sel_take_one(n, items[w], tid & (SEL_CHUNK - 1), off, ids, f, gain, pivot_of);
        __syncthreads();  // nitems and npk are reset by the next round
    }
    if (tid == 0) ctl[0] = 0;
}

// forward lists of reverse lists given as CSR (the caller's R_k): a count per
// vertex, then (after a scan into f_off) placement in any order
__global__ void k_sel_fcount(int64_t n, const int64_t* off, const int32_t* ids, int32_t* cnt) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    for (int64_t j = off[x]; j < off[x + 1]; ++j) atomicAdd(&cnt[ids[j]], 1);
}

__global__ void k_sel_fplace(int64_t n, const int64_t* off, const int32_t* ids,
                             const int64_t* f_off, int32_t* cur, int32_t* f_ids) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    for (int64_t j = off[x]; j < off[x + 1]; ++j) {
        const int32_t y = ids[j];
        f_ids[f_off[y] + atomicAdd(&cur[y], 1)] = (int32_t)x;
    }
}

// reverse lists of a device caller: ids in range and not the list's owner
__global__ void k_check_lists(int64_t n, const int64_t* off, const int32_t* ids, int* flag) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int64_t b = off[x], e = off[x + 1];
    bool bad = b > e || b < 0 || e > off[n];
    for (int64_t j = b; j < e && !bad; ++j) bad = ids[j] < 0 || ids[j] >= n || ids[j] == x;
    if (bad) atomicOr(flag, 1);
}

hipError_t launch_check_lists(int64_t n, const int64_t* off, const int32_t* ids, int* flag,
                              hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_lists, dim3(nblk(n, 256)), dim3(256), 0, st, n, off, ids, flag);
    return hipGetLastError();
}

hipError_t launch_select_init(int64_t n, const int64_t* off, unsigned char* lose, int32_t* gain,
                              int32_t* pivot_of, int64_t* ctl, hipStream_t st) {
    hipLaunchKernelGGL(k_sel_init, dim3(nblk(n > 0 ? n : 1, 256)), dim3(256), 0, st, n, off, lose,
                       gain, pivot_of, ctl);
    return hipGetLastError();
}

hipError_t launch_select_forward(int64_t n, const int64_t* off, const int32_t* ids, int32_t* cnt,
                                 int32_t* cur, int64_t* f_off, int32_t* f_ids, int64_t* scan_tmp,
                                 hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipError_t e = launch_zero(cnt, sizeof(int32_t) * (size_t)n, st);
    if (e == hipSuccess) e = launch_zero(cur, sizeof(int32_t) * (size_t)n, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sel_fcount, dim3(nblk(n, 256)), dim3(256), 0, st, n, off, ids, cnt);
    if ((e = launch_scan(cnt, n, f_off, scan_tmp, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sel_fplace, dim3(nblk(n, 256)), dim3(256), 0, st, n, off, ids, f_off, cur,
                       f_ids);
    return hipGetLastError();
}

hipError_t launch_select_rounds(int64_t n, const int32_t* act, int64_t nact, const int64_t* off,
                                const int32_t* ids, const int32_t* f_ids, const int64_t* f_off,
                                int fk, unsigned char* lose, int32_t* gain, int32_t* pivot_of,
                                int64_t* items, int64_t* ctl, int rounds, hipStream_t st) {
    if (n <= 0 || nact <= 0) return hipSuccess;
    const SelFwd f = {f_ids, f_off, fk};
    const dim3 gb(nblk(nact, 256)), gp(nblk(nact, SEL_PICK_THREADS)), b(256), bp(SEL_PICK_THREADS);
    // take: SEL_CHUNK lanes per item, at most 16 items in flight per active vertex
    const int64_t tb = std::min<int64_t>(std::max<int64_t>(nblk(nact * SEL_CHUNK, 256), 1), 1024);
    for (int r = 0; r < rounds; ++r) {
        hipLaunchKernelGGL(k_sel_best, gb, b, 0, st, n, act, nact, f, gain, lose, ctl);
        hipLaunchKernelGGL(k_sel_pick, gp, bp, 0, st, n, act, nact, off, f, lose, gain, pivot_of,
                           items, ctl);
        hipLaunchKernelGGL(k_sel_take, dim3(tb), b, 0, st, n, off, ids, f, gain, pivot_of, items,
                           ctl);
    }
    return hipGetLastError();
}

hipError_t launch_select_tail(int64_t n, const int32_t* act, int64_t nact, const int64_t* off,
                              const int32_t* ids, const int32_t* f_ids, const int64_t* f_off,
                              int fk, unsigned char* lose, int32_t* gain, int32_t* pivot_of,
                              int64_t* items, int64_t* ctl, hipStream_t st) {
    if (n <= 0 || nact <= 0 || !act) return hipSuccess;
    const SelFwd f = {f_ids, f_off, fk};
    hipLaunchKernelGGL(k_sel_tail, dim3(1), dim3(SEL_PICK_THREADS), 0, st, n, act, nact, off, ids, f,
                       lose, gain, pivot_of, items, ctl);
    return hipGetLastError();
}

hipError_t launch_select_compact(const int32_t* act, int64_t nact, const int32_t* gain,
                                 int32_t* act_out, int64_t* ctl, hipStream_t st) {
    hipError_t e = launch_zero(ctl + 4, sizeof(int64_t), st);
    if (e != hipSuccess || nact <= 0) return e;
    hipLaunchKernelGGL(k_sel_compact, dim3(nblk(nact, SEL_PICK_THREADS)), dim3(SEL_PICK_THREADS), 0,
                       st, act, nact, gain, act_out, ctl);
    return hipGetLastError();
}

// ------------------------------------------- static scratch of rnsm_search_noalloc

// The scratch memory of the allocation-free search entry point (counters,
// error flag, cosine norms): a file-scope device array, so that the entry
// point allocates nothing. Every GPU the library runs on holds its own copy
// until the process ends. Host code must not use the array's name as a
// device address (it names a host-side stand-in): noalloc_scratch() gives
// the copy of the current device, looked up once per device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(void** out) {
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void* ptr[MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return hipSuccess;
}

}  // namespace rnsm
