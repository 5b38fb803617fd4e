// Shared device-side definitions of the gfx950 matcher (not part of the ABI).
//
// HBM layout
//   slot arrays (edge attributes, Section IV-A: "attribute store indexed by
//   edge id"): s_src u32, s_dst u32, s_lab u8, s_ts i64, s_key u64 and the
//   DEBI words s_debi[slot * debi_words + w]. A slot is the recycled internal
//   edge id (Section IV-A, memory recycling); the key is the caller's stable id.
//   adjacency (Section II-A: every vertex keeps its in- and out-edges): two CSR
//   arrays, direction 0 = out-edges, 1 = in-edges. An entry is one u64:
//     high 32 bits  (label << nbr_bits) | neighbour
//     low  32 bits  flag << 31 | slot
//   A parallel array adjk[dir][p] holds the key of the edge at position p, so
//   the enumerator reads an emitted edge's key next to its entry.
//   Each vertex's segment is sorted by the high word, so a label's edges form
//   one run, parallel edges to one neighbour form a contiguous sub-run, and a
//   neighbour lookup is a binary search. The flag marks the edges of the batch
//   the current phase enumerates (insert phase: the inserted edges; delete
//   phase: the deleted ones, which stay in the arrays until the next merge).
//   vertex ids: internally, vertices are numbered in order of their label
//   set (vertices with equal label sets form a class, a contiguous id range),
//   so within one edge label a segment is ordered by neighbour class too, and
//   the neighbours that can satisfy a query vertex's labels are one run.
//   vertex filter VF[v * vf_words + w]: one bit per (query, query vertex).
//   counters cnt[v * n_cnt + c]: per-direction degree, per-direction degree of
//   each edge label the queries use, per-direction count of edges whose far
//   endpoint carries each vertex label the queries use.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define MN_MAXQV 16
#define MN_MAXQE 32
#define MN_MAXLV (MN_MAXQV - 2)
#define MN_FLAG 0x80000000u
#define MN_SLOTMASK 0x7FFFFFFFu
#define MN_INVALID 0xFFFFFFFFu
#define MN_BLOCK 256
#define MN_WAVE 64

#define MN_SEED_A 0x243F6A8885A308D3ULL
#define MN_SEED_B 0x13198A2E03707344ULL

// Error codes written by device validation (same values as the ABI).
#define MN_ERR_VERTEX 3
#define MN_ERR_LABEL 4
#define MN_ERR_TS 5
#define MN_ERR_DELETE 6
#define MN_ERR_INTERNAL 99

#define MN_SEM_ISO 0  // mnemonic_semantics: MNEMONIC_ISO
#define MN_SHARDS 32  // copies of the per-phase digests and work tallies (summed on the host)
#define MN_TALLIES 9  // work tallies per phase (EnumStats)
#define MN_MAXCLOSE 8  // closing edges per start edge (the query's cyclomatic number)
#define MN_NVAR 4      // matching orders per (query, start position): the static one and alternatives

// Order-cost network of the scheduler: 24 features -> 64 -> 64 -> 1 (ReLU),
// weights W1[24][64], b1[64], W2[64][64], b2[64], W3[64], b3 in this order.
#define MN_MLP_IN 24
#define MN_MLP_HIDDEN 64
#define MN_MLP_WEIGHTS (MN_MLP_IN * MN_MLP_HIDDEN + MN_MLP_HIDDEN + MN_MLP_HIDDEN * MN_MLP_HIDDEN + 2 * MN_MLP_HIDDEN + 1)

// Scheduler modes (same values as the ABI): the static order, the order the
// network predicts cheapest, or always variant v (MN_SCHED_FIXED + v).
#define MN_SCHED_STATIC 0
#define MN_SCHED_LEARNED 1
#define MN_SCHED_FIXED 2

// A closing query edge: both of its endpoints are mapped by the time the
// level that adds it is reached; it only has to exist. `other` was mapped
// earlier, `nv` by the level itself (for the start level: other = qa,
// nv = qb). dir 0: the query edge runs other -> nv, so its instances sit in
// the out-list of f(other) under (label, f(nv)); dir 1: nv -> other, in the
// in-list of f(other). The same instances also sit in the opposite list of
// f(nv) under (label, f(other)); the enumerator searches the shorter list.
// 16 bytes, 16-byte aligned: the expansion kernel reads one with one load.
struct alignas(16) CloseDesc {
    uint8_t qe;
    uint8_t other;
    uint8_t nv;
    uint8_t dir;
    uint8_t masked;  // query edge index < start position: batch edges forbidden
    uint8_t pad[3];
    int32_t label;   // -1 = any label
    uint32_t pad2;
};
static_assert(sizeof(CloseDesc) == 16, "one 16-byte load per closing edge");

// One level of the search maps one new query vertex `vtx` through its anchor
// edge: the candidates are the entries of f(from)'s out-list (dir 0, query
// edge from -> vtx) or in-list (dir 1, query edge vtx -> from) whose high
// word lies in [key_lo, key_hi] (one label and the id range of the vertex
// classes that can satisfy vtx's label requirement), or the whole list when
// the anchor label is a wildcard. Closing edges close[c_begin, c_end) join
// vtx to vertices mapped earlier.
// 16 bytes, 16-byte aligned: the expansion kernel reads a level with one load.
struct alignas(16) LevelDesc {
    uint8_t vtx;
    uint8_t qe;
    uint8_t from;
    uint8_t c_begin;
    uint8_t c_end;
    uint8_t n_mapped;     // query vertices mapped before this level (start pair + earlier levels)
    uint8_t dir : 1;
    uint8_t masked : 1;
    uint8_t whole : 1;    // wildcard anchor label: every entry of the list is a candidate
    uint8_t empty : 1;    // no vertex class satisfies vtx's labels: no candidates
    uint8_t need_vf : 1;  // candidates must pass the vertex-filter bit of vtx
    uint8_t pad;
    uint32_t key_lo;      // inclusive bounds of the candidates' high words
    uint32_t key_hi;
};
static_assert(sizeof(LevelDesc) == 16, "one 16-byte load per level");

// Matching order for one (query, start position j) pair (Section VI,
// matching order computation): the start edge maps qa -> qb; closing edges
// between qa and qb come first (close[0, c0_end)), then one level per
// remaining query vertex. Plans [0, n_static) hold the static order of each
// pair; the alternative orders of a pair follow them, and vars[] of every
// plan of the pair lists its n_var distinct orders (vars[0]: the static one).
// All orders of a pair share the start-level closing edges, so a start row
// may take any of them.
// The first 16 bytes (the header) are read with one load by the expansion
// kernel; `mapped` and `close_idx` are 16-byte aligned for the same reason.
struct SeedPlan {
    uint16_t q;        // query index
    uint8_t j;         // start position
    uint8_t n_qe;
    uint8_t qa, qb;
    uint8_t n_levels;
    uint8_t c0_end;
    uint8_t sem;
    uint8_t n_close;
    uint8_t n_var;       // distinct matching orders of this (query, j) pair
    uint8_t temporal;    // some pair of edges is ordered in time
    uint32_t vf_base;    // first vertex-filter bit of the query
    uint8_t mapped[MN_MAXQV];     // query vertices in mapping order: qa, qb, level vtx...
    uint8_t close_idx[MN_MAXQE];  // per query edge: index into close[], or 0xFF for a tree edge
    uint32_t debi_base;  // first edgeMatcher bit of the query
    uint8_t variant;     // which order of the pair this plan is
    uint8_t n_ranked;    // edges with a temporal rank
    uint8_t pad1[10];
    LevelDesc lv[MN_MAXLV];
    CloseDesc close[MN_MAXCLOSE];
    uint16_t vars[MN_NVAR];       // plan index of each order of the pair
    int8_t rank[MN_MAXQE];        // temporal rank per query edge (-1: unordered)
    uint8_t rorder[MN_MAXQE];     // the ranked edges by ascending rank
    float lv_est[MN_MAXLV];       // log2(1 + expected candidates per row) of each level, from the
                                  // initial graph's label degrees and the level's class range
};
static_assert(offsetof(SeedPlan, temporal) == 11 && offsetof(SeedPlan, vf_base) == 12, "plan header");
static_assert(offsetof(SeedPlan, mapped) == 16 && offsetof(SeedPlan, close_idx) == 32, "aligned plan arrays");
static_assert(offsetof(SeedPlan, lv) % 16 == 0 && sizeof(SeedPlan) % 16 == 0, "aligned levels");

// Partial embeddings between levels, stored column-wise (row r of column c at
// col[c * cap + r]): column 0 the plan index, 1 + u the data vertex of query
// vertex u (u < wv), 1 + wv + k for a closing edge k the position of its
// instance run in the adjacency list that was searched (bit 31 set when that
// was the list of f(nv)); kcol[k * cap + r] the key of tree edge k. When
// tracing, column 1 + wv + we holds the trace entry of the row's start row.
// hpre[r] and hpre[cap + r]: for a row whose plan ends at this level with no
// closing edge and no temporal order, both digest chains (seeds A and B) over
// the keys of the query edges before the level's anchor edge; its embeddings
// differ only from the anchor edge on.
struct RowsView {
    uint32_t* col;
    uint64_t* kcol;
    uint64_t* hpre;
    uint32_t cap;
    uint32_t wv;
    uint32_t we;
    uint32_t trace;  // 1: the trace column is present
};

// One local-filter requirement of a query vertex: counter c must be >= need.
struct VfReq {
    uint16_t cnt;
    uint16_t need;
};

struct QueryDev {
    uint32_t n_qv, n_qe, sem;
    uint32_t vf_base;    // first VF bit of this query
    uint32_t debi_base;  // first DEBI bit of this query
    uint32_t plan_base;  // index of the plan for start position 0
    uint32_t out_index;  // index of this query's output slots
    uint32_t pad;
    uint64_t vreq[MN_MAXQV];
    int32_t qlab[MN_MAXQE];
    uint8_t qsrc[MN_MAXQE];
    uint8_t qdst[MN_MAXQE];
    uint16_t req_begin[MN_MAXQV + 1];  // VfReq range of each query vertex
};

// Device view of the graph state used by most kernels.
struct GraphView {
    uint32_t n_vertices;
    uint32_t nbr_bits;
    uint32_t nbr_mask;
    uint32_t n_cnt;
    uint32_t vf_words;
    uint32_t debi_words;
    uint32_t n_queries;
    uint32_t n_vfreq;
    const uint64_t* vmask;
    const uint32_t* off[2];
    const uint64_t* adj[2];
    const uint64_t* adjk[2];   // key of the edge at each adjacency position
    uint32_t* vf;
    uint32_t* cnt;
    uint32_t* s_src;
    uint32_t* s_dst;
    uint8_t* s_lab;
    int64_t* s_ts;
    uint64_t* s_key;
    uint32_t* s_debi;
    const QueryDev* queries;
    const SeedPlan* plans;
    const VfReq* vfreq;
    const int16_t* elab_idx;   // [256] compact index of an edge label, -1 if unused
    const int16_t* vlab_idx;   // [64] compact index of a vertex label bit, -1 if unused
    const uint32_t* ext2int;   // [n_vertices] caller's vertex id -> internal id
    // The arrays of direction d. A select between the two kernel-argument
    // pointers, not an index into the argument struct: a lane-dependent index
    // into a by-value struct makes the compiler load the pointer from memory.
    __device__ const uint32_t* offs(uint32_t d) const { return d ? off[1] : off[0]; }
    __device__ const uint64_t* adjs(uint32_t d) const { return d ? adj[1] : adj[0]; }
    __device__ const uint64_t* keys(uint32_t d) const { return d ? adjk[1] : adjk[0]; }
    uint64_t key_mask;         // key-indexed maps are rings: key k sits at k & key_mask
    int64_t* key_ts;           // key -> timestamp of every edge ever inserted (never invalidated:
                               // a re-run of a phase may still meet edges its batch deleted)
    uint32_t n_elab_c;         // compact edge labels
    uint32_t n_vlab_c;         // compact vertex labels
    uint32_t n_static;         // plans holding the static orders
    // scheduler: which matching order each start row takes
    uint32_t sched_mode;       // MN_SCHED_*
    const uint16_t* sched_w;   // bf16 weights of the order-cost network (learned mode)
    // traces (tr_cap = 0: off): per phase, one entry per start row with the
    // features of every order of its pair and the search work below it
    uint64_t* dec;             // start rows whose order the decision kernel settles (NULL: none)
    uint32_t* dec_n;           // their count
    uint32_t tr_cap;           // entries per phase
    uint32_t tr_base;          // index of the launch's first slot in the phase's slot list
    uint32_t* tr_n;            // [2] entries taken per phase (may exceed tr_cap)
    uint64_t* tr_code;         // [2][tr_cap] phase << 62 | variant << 56 | static plan << 32 | slot index
    float* tr_x;               // [2][tr_cap][MN_NVAR][MN_MLP_IN]
    unsigned long long* tr_work;  // [2][tr_cap] 1 + candidates examined below the start row
};

// Counter layout of one vertex: [dir][0] degree, [dir][1 + e] edge label e,
// [dir][1 + n_elab_c + l] neighbours' vertex label l; n_cnt = 2 * (1 + E + L).
__host__ __device__ inline uint32_t cnt_index(uint32_t dir, uint32_t part, uint32_t n_elab_c,
                                              uint32_t n_vlab_c) {
    return dir * (1 + n_elab_c + n_vlab_c) + part;
}

__device__ inline uint32_t ent_hi(uint64_t e) { return (uint32_t)(e >> 32); }
__device__ inline uint32_t ent_lo(uint64_t e) { return (uint32_t)e; }

// SplitMix64 output finaliser (Steele, Lea, Flood 2014).
__device__ inline uint64_t mn_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__device__ inline uint32_t lane_id() { return __lane_id(); }

__device__ inline uint64_t lanemask_lt() {
    uint32_t l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ inline uint32_t uniform_u32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// First index in [lo, hi) whose entry's high word is >= key.
__device__ inline uint32_t lower_hi(const uint64_t* adj, uint32_t lo, uint32_t hi, uint32_t key) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(adj);
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (w[2 * (size_t)mid + 1] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// First index in [lo, hi) whose entry's high word is > key.
__device__ inline uint32_t upper_hi(const uint64_t* adj, uint32_t lo, uint32_t hi, uint32_t key) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(adj);
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (w[2 * (size_t)mid + 1] <= key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

template <typename T>
__device__ inline uint32_t lower_bound_dev(const T* a, uint32_t lo, uint32_t hi, T key) {
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

template <typename T>
__device__ inline uint32_t upper_bound_dev(const T* a, uint32_t lo, uint32_t hi, T key) {
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}
