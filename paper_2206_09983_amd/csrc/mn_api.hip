// C ABI of the matcher: context state, query preprocessing and the per-snapshot
// kernel sequence (Algorithm 1 loop body = Algorithm 2 batchInserts followed by
// batchDeletes). All device work runs on the context's stream; one host
// synchronisation per snapshot returns the counts and digests.
//
// Snapshot t on the device:
//   validate(I_t, D_t)                     nothing below runs if it fails
//   counters -= edges of D_{t-1}           (removal deferred from snapshot t-1)
//   ingest I_t: slots, attributes, DEBI words, counters += edges of I_t
//   sort I_t entries (out, in) and D_{t-1} positions
//   merge: adjacency' = adjacency - D_{t-1} + I_t (I_t entries flagged)
//   VF refresh for endpoints of D_{t-1} and I_t
//   seeds(I_t) -> enumerate new embeddings on G + I_t
//   unflag I_t, flag D_t; seeds(D_t) -> enumerate expired embeddings on G + I_t
//   retire D_t keys, push D_t slots on the free stack
// D_t's entries stay (flagged) in the adjacency until the next merge, and the
// counters/VF keep counting them until then: the filters stay sound (a
// superset), and an enumeration can be re-run on exactly the same state when
// an output buffer was too small.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mnemonic.h"
#include "mn_internal.h"

namespace {

thread_local std::string g_create_error;

struct HipError {
    hipError_t e;
    const char* what;
};

#define HIPCHK(x)                                  \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) throw HipError{e_, #x}; \
    } while (0)

struct ApiError {
    int code;
    std::string msg;
};

inline uint32_t ceil_log2(uint64_t x) {
    uint32_t b = 0;
    while ((1ull << b) < x) b++;
    return b;
}

// Failure injection for tests (mnemonic_fail_alloc_after): the countdown
// makes the n-th device allocation from the moment it is armed fail as if the
// device were out of memory; 0 means disarmed.
uint64_t g_fail_alloc_in = 0;

// Set while mnemonic_apply_batch_noalloc runs on this thread: the call fits
// its batch into the buffers the context already holds, and a buffer that
// would have to grow refuses instead of allocating.
thread_local bool t_no_alloc = false;
// Device allocations and frees of the calling thread, and the host time they
// took (with the stream waits that precede a regrowth): reported per batch.
thread_local uint64_t t_alloc_n = 0;
thread_local double t_alloc_ms = 0;

struct NoAllocScope {
    NoAllocScope() { t_no_alloc = true; }
    ~NoAllocScope() { t_no_alloc = false; }
};

// The per-batch control words of mnemonic_apply_batch_noalloc (readback block
// of counts, digests, work tallies and overflow notes; error word; row
// counters; candidate total; decision-list count) live in this array instead
// of the context's own: one copy per GPU, shared by every such call on it.
// Host code never passes the array's name to a kernel: it uses the address
// hipGetSymbolAddress returns for the device, looked up once per device when
// the device's first context is created.
constexpr uint64_t MN_NOALLOC_WORDS = 1u << 16;  // 512 KiB
constexpr int MN_MAX_DEVICES = 64;
__device__ __align__(256) uint64_t scratch[MN_NOALLOC_WORDS];
std::mutex g_scratch_mu;
uint64_t* g_scratch_ptr[MN_MAX_DEVICES] = {};

// Looks up the device address of `scratch` on `device` (the current device).
void setup_scratch(int device) {
    if (device < 0 || device >= MN_MAX_DEVICES) return;  // the no-allocation call then reports it
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = static_cast<uint64_t*>(ptr);
}

// Device memory comes from the device's stream-ordered pool, and the pool
// keeps what is freed: a buffer that grows is replaced without a stream
// synchronisation, and a later allocation (in this context or another) reuses
// the pool's memory instead of mapping new pages, which a plain allocation
// after a large free can take tens of milliseconds to do. Set up once per
// device. t_stream is the calling context's stream: allocations and frees
// are ordered on it.
bool g_pool_ready[MN_MAX_DEVICES] = {};
thread_local hipStream_t t_stream = nullptr;

void setup_pool(int device) {
    if (device < 0 || device >= MN_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_pool_ready[device]) return;
    hipMemPool_t pool = nullptr;
    HIPCHK(hipDeviceGetDefaultMemPool(&pool, device));
    uint64_t keep = ~0ull;
    HIPCHK(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
    g_pool_ready[device] = true;
}

uint64_t* scratch_of(int device) {
    if (device < 0 || device >= MN_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

template <typename T>
void dev_alloc(T*& p, size_t n) {
    void* q = nullptr;
    if (n == 0) n = 1;
    if (t_no_alloc)
        throw ApiError{MNEMONIC_E_CAPACITY, "the batch needs a buffer of " + std::to_string(n * sizeof(T)) +
                                                " bytes the context does not hold (no-allocation call)"};
    if (g_fail_alloc_in && --g_fail_alloc_in == 0)
        throw ApiError{MNEMONIC_E_OOM, "device allocation of " + std::to_string(n * sizeof(T)) +
                                           " bytes failed (injected)"};
    const auto t0 = std::chrono::steady_clock::now();
    hipError_t e = hipMallocAsync(&q, n * sizeof(T), t_stream);
    if (e != hipSuccess) {
        // the pool may hold freed memory the request needs: hand it back to
        // the device once the stream's pending frees are done, and try again
        (void)hipGetLastError();
        int dev = 0;
        hipMemPool_t pool = nullptr;
        if (hipStreamSynchronize(t_stream) == hipSuccess && hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && hipMemPoolTrimTo(pool, 0) == hipSuccess)
            e = hipMallocAsync(&q, n * sizeof(T), t_stream);
    }
    t_alloc_n++;
    t_alloc_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw ApiError{MNEMONIC_E_OOM, "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed"};
    }
    p = static_cast<T*>(q);
}

template <typename T>
void dev_free(T*& p) {
    if (p) {  // after the work already queued on the stream, which may still use it
        const auto t0 = std::chrono::steady_clock::now();
        (void)hipFreeAsync(p, t_stream);
        t_alloc_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    p = nullptr;
}

// Grows a device array to hold `need` elements, keeping the first `keep`.
template <typename T>
void dev_grow(T*& p, uint64_t& cap, uint64_t need, uint64_t keep, hipStream_t s) {
    if (need <= cap && p) return;
    // twice the need: a stream that keeps growing regrows rarely, and the
    // device has memory to spare
    uint64_t nc = std::max<uint64_t>(2 * need, 2 * cap);
    nc = std::max<uint64_t>(nc, 256);
    T* np = nullptr;
    dev_alloc(np, nc);
    if (p && keep) HIPCHK(hipMemcpyAsync(np, p, keep * sizeof(T), hipMemcpyDeviceToDevice, s));
    dev_free(p);  // stream-ordered: after the copy
    p = np;
    cap = nc;
}

}  // namespace

struct mnemonic_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t flags = MNEMONIC_F_EMIT;
    uint32_t nV = 0, n_elabels = 256, nbr_bits = 1, hb = 1;
    uint64_t out_cap0 = 1ull << 20;  // initial tuples per result buffer

    // vertex classes: distinct label sets in increasing order; internal ids
    // number the vertices class by class (cls_start[c] = first id of class c)
    std::vector<uint64_t> cls_mask;
    std::vector<uint32_t> cls_start;
    // edges per vertex of each edge label in the initial graph ([256]: all labels)
    std::vector<double> lab_deg;
    uint32_t* d_ext2int = nullptr;

    // queries and their preprocessed tables
    uint32_t n_q = 0;
    uint32_t n_plans = 0, n_static = 0, max_levels = 0, wv = 2, we = 1, max_close = 0;
    uint8_t level_rows[MN_MAXLV] = {0};  // some plan continues past level L
    uint8_t level_emit[MN_MAXLV] = {0};  // some plan ends at level L
    std::vector<QueryDev> hq;
    std::vector<SeedPlan> hplans;
    std::vector<DebiBit> hdebi;
    std::vector<VfBit> hvf;
    std::vector<VfReq> hreq;
    int16_t elab_idx[256];
    int16_t vlab_idx[64];
    uint32_t n_elab_c = 0, n_vlab_c = 0, n_cnt = 2;
    uint32_t vf_words = 1, debi_words = 1, n_vf_bits = 0, n_debi_bits = 0, total_qe = 0;

    // device: static tables and per-vertex state
    uint64_t* d_vmask = nullptr;
    QueryDev* d_q = nullptr;
    SeedPlan* d_plans = nullptr;
    DebiBit* d_debi_bits = nullptr;
    VfBit* d_vf_bits = nullptr;
    VfReq* d_req = nullptr;
    int16_t* d_elab_idx = nullptr;
    int16_t* d_vlab_idx = nullptr;
    uint32_t* d_vf = nullptr;
    uint32_t* d_cnt = nullptr;
    // spanning-tree filter (MNEMONIC_F_TREE_FILTER): its steps round by round
    // (round i = steps [tree_round[i], tree_round[i + 1])) and the filter
    // bits the enumerator then reads: VF with the tree's conditions applied
    std::vector<TreeStep> htree;
    std::vector<uint32_t> tree_round;
    TreeStep* d_tree = nullptr;
    uint32_t* d_vfp = nullptr;
    uint4* d_meta[2] = {nullptr, nullptr};

    // slot arrays
    uint64_t cap_slots = 0;
    uint32_t* d_src = nullptr;
    uint32_t* d_dst = nullptr;
    uint8_t* d_lab = nullptr;
    int64_t* d_ts = nullptr;
    uint64_t* d_key = nullptr;
    uint32_t* d_debi = nullptr;
    uint32_t* d_free = nullptr;
    uint64_t cap_debi = 0, cap_free = 0, cap_lab = 0, cap_ts = 0, cap_key = 0, cap_dst = 0;

    // key-indexed maps, rings of cap_keys (a power of two) places: key k sits
    // at k & (cap_keys - 1). Every key below key_lo is dead, and cap_keys
    // exceeds the span from key_lo to the end of the next batch, so the keys
    // that may still be met never share a place; the maps' size follows the
    // live key span (a sliding window's), not the keys ever inserted.
    uint64_t cap_keys = 0, cap_delbits = 0;
    uint32_t* d_key2slot = nullptr;
    int64_t* d_key_ts = nullptr;  // timestamp by key (kept for deleted keys until they fall below key_lo)
    uint32_t* d_delbits = nullptr;
    uint64_t key_lo = 0;           // host copy, as of the last batch
    uint64_t key_lo_seen = 0;      // the device's value read back with the batch, committed with it
    uint64_t* d_key_lo = nullptr;  // advanced on the device after each batch's deletions

    // adjacency, double-buffered
    uint64_t cap_E = 0, cap_E2 = 0, cap_E3 = 0, cap_E4 = 0;
    uint32_t* d_off[2] = {nullptr, nullptr};
    uint32_t* d_off2[2] = {nullptr, nullptr};
    uint64_t* d_adj[2] = {nullptr, nullptr};
    uint64_t* d_adj2[2] = {nullptr, nullptr};
    uint64_t* d_adjk[2] = {nullptr, nullptr};   // key of the edge at each adjacency position
    uint64_t* d_adjk2[2] = {nullptr, nullptr};

    // batch scratch
    uint64_t cap_ins = 0, cap_del = 0, cap_touch = 0, cap_sort = 0;
    uint32_t* d_in_src = nullptr;
    uint32_t* d_in_dst = nullptr;
    uint8_t* d_in_lab = nullptr;
    int64_t* d_in_ts = nullptr;
    uint64_t* d_del_keys = nullptr;
    uint32_t* d_ins_slot = nullptr;
    // batch sort keys of both directions in one array (direction bit on top),
    // ping-pong pair
    uint64_t* d_skey[2] = {nullptr, nullptr};
    uint32_t* d_sval[2] = {nullptr, nullptr};
    uint32_t* d_inspos[2] = {nullptr, nullptr};
    uint32_t* d_ub[2] = {nullptr, nullptr};  // insertion points of the batch entries in the old adjacency
    uint32_t* d_mlim = nullptr;              // the merge's counts at every tile start, one half per direction
    uint64_t cap_mlim = 0;
    uint32_t* d_touched = nullptr;
    uint32_t* d_del_slot[2] = {nullptr, nullptr};        // [buffer]
    uint32_t* d_delpos[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [buffer][dir]
    uint64_t cap_delbuf[2] = {0, 0};
    uint64_t* d_dkey[2] = {nullptr, nullptr};  // deleted positions of both directions, ping-pong
    uint32_t* d_dval[2] = {nullptr, nullptr};
    uint32_t hb_pos = 32;  // significant bits of an adjacency position
    uint32_t* d_sort_scratch = nullptr;
    uint64_t cap_sort_scratch = 0;

    // level-wise enumeration: rows of partial embeddings per level, their
    // candidate runs and offsets, scan scratch and small control words
    struct LevelBuf {
        uint32_t* rows = nullptr;  // cap x ncol words, column-wise
        uint64_t* keys = nullptr;  // cap x we tree-edge keys, column-wise
        uint32_t* lo = nullptr;
        uint32_t* cnt = nullptr;
        uint64_t* off = nullptr;
        uint64_t* hpre = nullptr;  // 2 x cap digest prefixes of rows whose plan ends at this level
        uint64_t cap = 0;
    };
    std::vector<LevelBuf> lvb;
    uint64_t rows_max = 1ull << 25;  // rows per level buffer, grown on demand (bounds each expansion chunk)
    uint64_t* d_scan64 = nullptr;
    uint64_t cap_scan64 = 0;
    uint32_t* d_tiles = nullptr;     // first row of every expansion tile
    uint64_t cap_tiles = 0;
    uint32_t* d_nrows = nullptr;     // [MN_MAXLV + 1] row counters
    uint64_t* d_total = nullptr;     // candidate total of the last scan
    uint64_t* h_ctl = nullptr;       // pinned: readback of counters
    hipEvent_t ev_x[2] = {nullptr, nullptr};  // around each host-sized expansion launch
    // device-sized launches: event pairs resolved after the batch's final sync
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_phase;
    uint32_t ev_used = 0;
    uint64_t cand_k = 1ull << 24;  // candidates one device-sized expansion may take (sizes d_tiles)
    // observed rates per inserted/deleted slot of the last batches: start rows
    // (index MN_MAXLV) and candidates per level; negative = not seen yet. They
    // size grids and buffers for the next batch, whatever its size.
    double rate[2][MN_MAXLV + 1];
    double row_rate[2][MN_MAXLV + 1];  // largest rows of level L per start slot seen (-1: none yet)
    uint64_t chunk_ns[2] = {1, 1};  // slots of the largest start chunk of the last run of each phase
    uint64_t cover[2][MN_MAXLV];    // candidates each level's launch covered in the last device-sized run
    uint32_t tile_items = 4;       // expansion tile = 256 x tile_items candidates (default_tile_items)
    // autotuning of tile_items: trial batches per setting, time and candidates
    static constexpr uint32_t TUNE_TRIALS = 2;
    uint32_t tune_batch = 0;
    double tune_ms[3] = {0, 0, 0};
    double tune_cand[3] = {0, 0, 0};
    bool tuning() const { return (flags & MNEMONIC_F_AUTOTUNE) && tune_batch < 3 * TUNE_TRIALS; }
    double ms_expand[2] = {0, 0};
    uint64_t n_expand[2] = {0, 0};
    uint64_t reruns[2] = {0, 0}, rerun_causes[2] = {0, 0};  // this batch's phase re-runs

    // scheduler: matching-order choice (MN_SCHED_*) and the network's bf16 weights
    uint32_t sched_mode = MN_SCHED_STATIC;
    uint16_t* d_sched_w = nullptr;
    float* d_sched_f32 = nullptr;
    // lexicographic sort of result tuples (MNEMONIC_F_SORT): scratch
    uint64_t* d_srt_k[2] = {nullptr, nullptr};
    uint32_t* d_srt_v[2] = {nullptr, nullptr};
    uint64_t* d_srt_rows = nullptr;
    uint32_t* d_srt_scr = nullptr;
    uint64_t cap_srt = 0, cap_srt_rows = 0, cap_srt_scr = 0;
    // start rows whose order the decision kernel settles
    uint64_t* d_dec = nullptr;
    uint64_t cap_dec = 0;
    uint32_t* d_dec_n = nullptr;
    bool deciding() const { return sched_mode == MN_SCHED_LEARNED || tr_cap != 0; }
    // traces of the start rows (tr_cap entries per phase, 0: off)
    uint32_t tr_cap = 0;
    uint32_t* d_tr_n = nullptr;
    uint64_t* d_tr_code = nullptr;
    float* d_tr_x = nullptr;
    unsigned long long* d_tr_work = nullptr;

    // control block: err, last_ts, zeroed counters
    uint32_t* d_err = nullptr;
    int64_t* d_last_ts = nullptr;
    unsigned long long* d_zr = nullptr;
    uint32_t n_zr = 0;
    std::vector<unsigned long long> h_zr;
    // pinned staging for the end-of-batch readback: the n_zr words, then the
    // error word (its low half); both copies are queued before one wait
    unsigned long long* h_zr_pin = nullptr;
    uint64_t cap_zr_pin = 0;

    // outputs
    std::vector<OutView> houts;
    // Set while mnemonic_set_queries rebuilds the query-dependent state, and
    // while a batch runs from its first launch that may change the graph
    // until it is complete; left set when either fails part way, after which
    // the context only reports why (broken_why).
    bool broken = false;
    std::string broken_why;
    // The last batch (a no-allocation call) could not fit its enumeration in
    // the buffers the context holds: its results are unavailable.
    bool results_incomplete = false;
    // Largest tuples per phase edge seen, per (query, phase) (-1: none yet):
    // sizes the output buffers before a batch, so that a batch larger than
    // any before does not re-run a phase to grow them.
    std::vector<double> out_rate;
    // Largest tuple count seen per (query, phase): bounds that sizing, since a
    // rate taken on a small batch can overstate a large one by far.
    std::vector<uint64_t> out_max;
    OutView* d_outs = nullptr;

    // host mirrors
    uint64_t next_key = 0, n_live = 0, E = 0, n_pending = 0;
    uint32_t n_free = 0, fresh = 0;
    int pend = 0;  // which delete buffer holds the pending deletions
    bool have_result = false;

    mnemonic_stats stats;
    std::string err;
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};

    bool tree_on() const { return (flags & MNEMONIC_F_TREE_FILTER) != 0; }
    // zero-region layout
    uint32_t zr_nseeds(int p) const { return (uint32_t)p; }
    uint32_t zr_cursor(int p) const { return 2u + (uint32_t)p; }
    uint32_t zr_count(int p) const { return 4u + (uint32_t)p * n_q; }
    uint32_t zr_digest(int p) const { return 4u + 2u * n_q + (uint32_t)p * MN_SHARDS * 2u * n_q; }
    uint32_t zr_stats(int p) const {
        return 4u + 2u * n_q + 4u * MN_SHARDS * n_q + (uint32_t)p * MN_SHARDS * MN_TALLIES;
    }
    // Overflow notes of the device-sized levels, per phase, four words per
    // level L: [candidates exceeded the launch, largest candidate total, rows
    // of level L + 1 exceeded their buffer, largest row count]; after the
    // levels: [start rows exceeded their buffer, largest count, -, -].
    uint32_t zr_note(int p) const {
        return 4u + 2u * n_q + 4u * MN_SHARDS * n_q + 2u * MN_TALLIES * MN_SHARDS + (uint32_t)p * 4u * (MN_MAXLV + 1);
    }
    uint32_t note_cand(int p, uint32_t L) const { return zr_note(p) + 4u * L; }
    uint32_t note_rows(int p, uint32_t L) const { return zr_note(p) + 4u * L + 2u; }
    uint32_t note_seed(int p) const { return zr_note(p) + 4u * MN_MAXLV; }
    uint32_t zr_tree() const { return zr_note(2); }  // filter bits the spanning-tree rounds cleared
    uint32_t zr_words() const { return zr_note(2) + 1u; }
    // shard sums of the last readback: digests [p][q][2], tallies [p][MN_TALLIES]
    std::vector<uint64_t> sum_dig;
    uint64_t sum_st[2][MN_TALLIES] = {{0}};
    void summarize() {
        sum_dig.assign(4 * (size_t)n_q, 0);
        for (int p = 0; p < 2; p++) {
            for (uint32_t sh = 0; sh < MN_SHARDS; sh++) {
                const unsigned long long* d = h_zr.data() + zr_digest(p) + (size_t)sh * 2 * n_q;
                for (uint32_t i = 0; i < 2 * n_q; i++) sum_dig[(size_t)p * 2 * n_q + i] += d[i];
            }
            for (int i = 0; i < MN_TALLIES; i++) {
                uint64_t v = 0;
                for (uint32_t sh = 0; sh < MN_SHARDS; sh++) v += h_zr[zr_stats(p) + sh * MN_TALLIES + i];
                sum_st[p][i] = v;
            }
        }
    }
    uint32_t ncol() const { return 1 + wv + we + (tr_cap ? 1 : 0); }
};

namespace {

// ----------------------------------------------------------------- planning
// Internal id range [id_lo, id_hi) spanning every vertex class whose label set
// contains `req`; `exact` when every class in between does too. Returns false
// when no class qualifies.
bool class_hull(const mnemonic_ctx* c, uint64_t req, uint32_t& id_lo, uint32_t& id_hi, bool& exact) {
    int lo = -1, hi = -1;
    const int n = (int)c->cls_mask.size();
    for (int i = 0; i < n; i++)
        if ((req & ~c->cls_mask[i]) == 0) {
            if (lo < 0) lo = i;
            hi = i;
        }
    if (lo < 0) return false;
    exact = true;
    for (int i = lo; i <= hi; i++)
        if (req & ~c->cls_mask[i]) exact = false;
    id_lo = c->cls_start[lo];
    id_hi = c->cls_start[hi + 1];
    return true;
}

// Whether every local-filter requirement of query vertex u is met by the one
// anchor edge that maps it (need <= 1 on a counter that edge increments), in
// which case testing the vertex-filter bit can prune nothing.
bool filters_trivial(const mnemonic_ctx* c, const QueryDev& Q, uint32_t u, uint32_t anchor, uint32_t from,
                     uint32_t dir) {
    const uint32_t E = c->n_elab_c, Lc = c->n_vlab_c;
    const uint32_t dw = 1u - dir;  // the anchor is an in-edge of f(u) when it leaves f(from)
    std::vector<uint16_t> inc;
    inc.push_back((uint16_t)cnt_index(dw, 0, E, Lc));
    if (Q.qlab[anchor] >= 0) inc.push_back((uint16_t)cnt_index(dw, 1 + c->elab_idx[Q.qlab[anchor]], E, Lc));
    for (int b = 0; b < 64; b++)
        if (((Q.vreq[from] >> b) & 1) && c->vlab_idx[b] >= 0)
            inc.push_back((uint16_t)cnt_index(dw, 1 + E + c->vlab_idx[b], E, Lc));
    for (uint32_t r = Q.req_begin[u]; r < Q.req_begin[u + 1]; r++) {
        const VfReq& q = c->hreq[r];
        if (q.need == 0) continue;
        if (q.need > 1 || std::find(inc.begin(), inc.end(), q.cnt) == inc.end()) return false;
    }
    return true;
}

// Static matching order for start edge j (Section VI): the start edge maps
// both its endpoints; then, repeatedly, the unmapped query vertex with the most
// edges to mapped vertices (ties: lowest index) is mapped through one of those
// edges (a labelled one first, then the lowest index), and its other edges to
// mapped vertices become closing edges checked at that level.
// variant bit 0: among the vertices with the most connections to the mapped
// ones, take the highest index instead of the lowest; bit 1: anchor a level
// at its highest-index connecting edge instead of the lowest (labelled edges
// first either way). Variant 0 is the static order.
void build_plan(const mnemonic_ctx* c, const QueryDev& Q, uint32_t qi, uint32_t j, SeedPlan& P, uint32_t variant = 0) {
    const bool rev_vtx = (variant & 1u) != 0, rev_anchor = (variant & 2u) != 0;
    memset(&P, 0, sizeof(P));
    const uint32_t nqv = Q.n_qv, nqe = Q.n_qe;
    P.q = (uint16_t)qi;
    P.j = (uint8_t)j;
    P.n_qe = (uint8_t)nqe;
    P.sem = (uint8_t)Q.sem;
    P.vf_base = Q.vf_base;
    P.debi_base = Q.debi_base;
    for (uint32_t k = 0; k < MN_MAXQE; k++) P.close_idx[k] = 0xFF;
    bool mapped[MN_MAXQV] = {false};
    bool used[MN_MAXQE] = {false};
    uint32_t qa = Q.qsrc[j], qb = Q.qdst[j];
    P.qa = (uint8_t)qa;
    P.qb = (uint8_t)qb;
    P.mapped[0] = (uint8_t)qa;
    P.mapped[1] = (uint8_t)qb;
    mapped[qa] = mapped[qb] = true;
    used[j] = true;
    uint32_t nc = 0;
    auto add_close = [&](uint32_t k, uint32_t newv) {
        if (nc >= MN_MAXCLOSE)
            throw ApiError{MNEMONIC_E_QUERY, "a query has more than 8 edges beyond a spanning tree"};
        CloseDesc& cd = P.close[nc];
        uint32_t other = Q.qsrc[k] == newv ? Q.qdst[k] : Q.qsrc[k];
        cd.qe = (uint8_t)k;
        cd.other = (uint8_t)other;
        cd.nv = (uint8_t)newv;
        cd.dir = Q.qsrc[k] == other ? 0 : 1;
        cd.masked = k < j ? 1 : 0;
        cd.label = Q.qlab[k];
        P.close_idx[k] = (uint8_t)nc;
        used[k] = true;
        nc++;
    };
    for (uint32_t k = 0; k < nqe; k++) {
        if (used[k]) continue;
        if ((Q.qsrc[k] == qa && Q.qdst[k] == qb) || (Q.qsrc[k] == qb && Q.qdst[k] == qa)) add_close(k, qb);
    }
    P.c0_end = (uint8_t)nc;
    uint32_t L = 0;
    while (L + 2 < nqv) {
        int best = -1, best_conn = -1;
        for (uint32_t u = 0; u < nqv; u++) {
            if (mapped[u]) continue;
            int conn = 0;
            for (uint32_t k = 0; k < nqe; k++)
                if (!used[k] && ((Q.qsrc[k] == u && mapped[Q.qdst[k]]) || (Q.qdst[k] == u && mapped[Q.qsrc[k]])))
                    conn++;
            if (conn > best_conn || (rev_vtx && conn == best_conn)) {
                best_conn = conn;
                best = (int)u;
            }
        }
        uint32_t n = (uint32_t)best;
        int anchor = -1;
        for (int pass = 0; pass < 2 && anchor < 0; pass++)
            for (uint32_t t = 0; t < nqe; t++) {
                const uint32_t k = rev_anchor ? nqe - 1 - t : t;
                if (used[k]) continue;
                bool touches = (Q.qsrc[k] == n && mapped[Q.qdst[k]]) || (Q.qdst[k] == n && mapped[Q.qsrc[k]]);
                if (touches && (pass == 1 || Q.qlab[k] >= 0)) {
                    anchor = (int)k;
                    break;
                }
            }
        LevelDesc& lv = P.lv[L];
        uint32_t ak = (uint32_t)anchor;
        uint32_t from = Q.qsrc[ak] == n ? Q.qdst[ak] : Q.qsrc[ak];
        lv.vtx = (uint8_t)n;
        lv.qe = (uint8_t)ak;
        lv.from = (uint8_t)from;
        lv.dir = Q.qsrc[ak] == from ? 0 : 1;
        lv.masked = ak < j ? 1 : 0;
        lv.n_mapped = (uint8_t)(L + 2);
        used[ak] = true;
        // candidates: the anchor label's run restricted to the classes that
        // can carry n's labels (or the whole list for a wildcard label)
        uint32_t id_lo = 0, id_hi = 0;
        bool exact = false;
        const bool some = class_hull(c, Q.vreq[n], id_lo, id_hi, exact);
        lv.whole = Q.qlab[ak] < 0 ? 1 : 0;
        lv.empty = some ? 0 : 1;
        bool labels_implied = exact;
        if (lv.whole) {
            labels_implied = some && exact && id_lo == 0 && id_hi == c->nV;
        } else if (some) {
            lv.key_lo = ((uint32_t)Q.qlab[ak] << c->nbr_bits) | id_lo;
            lv.key_hi = ((uint32_t)Q.qlab[ak] << c->nbr_bits) | (id_hi - 1);
        }
        lv.need_vf = labels_implied ? 0 : 1;  // refined below once the last level is known
        {  // expected candidates per row: the label's mean degree times the share of the class range
            const double deg = c->lab_deg.empty() ? 0.0 : c->lab_deg[Q.qlab[ak] >= 0 ? Q.qlab[ak] : 256];
            const double share = some ? (double)(id_hi - id_lo) / (double)std::max<uint32_t>(1, c->nV) : 0.0;
            P.lv_est[L] = (float)std::log2(1.0 + deg * share);
        }
        lv.c_begin = (uint8_t)nc;
        for (uint32_t k = 0; k < nqe; k++) {
            if (used[k]) continue;
            if ((Q.qsrc[k] == n && mapped[Q.qdst[k]]) || (Q.qdst[k] == n && mapped[Q.qsrc[k]])) add_close(k, n);
        }
        lv.c_end = (uint8_t)nc;
        mapped[n] = true;
        P.mapped[L + 2] = (uint8_t)n;
        L++;
    }
    P.n_levels = (uint8_t)L;
    P.n_close = (uint8_t)nc;
    // Below the last level the filter bit can also prune by degree; with the
    // spanning-tree filter it can prune at every level.
    for (uint32_t l = 0; l < L; l++) {
        LevelDesc& lv = P.lv[l];
        if (c->tree_on() || (l + 1 < L && !lv.need_vf && !filters_trivial(c, Q, lv.vtx, lv.qe, lv.from, lv.dir)))
            lv.need_vf = 1;
    }
}

// Temporal ranks of the query's edges on a plan (all -1 without qtorder).
void set_ranks(SeedPlan& P, const mnemonic_query& q) {
    P.temporal = 0;
    for (uint32_t k = 0; k < MN_MAXQE; k++) P.rank[k] = -1;
    if (!q.qtorder) return;
    int lo = 1 << 30, hi = -1;
    for (uint32_t k = 0; k < q.n_qe; k++) {
        P.rank[k] = (int8_t)q.qtorder[k];
        if (q.qtorder[k] >= 0) {
            lo = std::min(lo, q.qtorder[k]);
            hi = std::max(hi, q.qtorder[k]);
        }
    }
    P.temporal = hi > lo ? 1 : 0;  // two distinct ranks order some pair
    P.n_ranked = 0;
    for (int r = lo; r <= hi; r++)
        for (uint32_t k = 0; k < q.n_qe; k++)
            if (q.qtorder[k] == r) P.rorder[P.n_ranked++] = (uint8_t)k;
}

void check_query(const mnemonic_query& q) {
    auto bad = [](const std::string& m) { throw ApiError{MNEMONIC_E_QUERY, m}; };
    if (q.n_qv < 2 || q.n_qv > MN_MAXQV) bad("query needs 2..16 vertices");
    if (q.n_qe < 1 || q.n_qe > MN_MAXQE) bad("query needs 1..32 edges");
    if (!q.qv_require || !q.qsrc || !q.qdst || !q.qelabel) bad("query arrays must not be NULL");
    if (q.sem != MNEMONIC_ISO && q.sem != MNEMONIC_HOMO) bad("unknown semantics");
    for (uint32_t i = 0; i < q.n_qe; i++) {
        if (q.qsrc[i] >= q.n_qv || q.qdst[i] >= q.n_qv) bad("query edge endpoint out of range");
        if (q.qsrc[i] == q.qdst[i]) bad("query self-loop");
        if (q.qelabel[i] < -1 || q.qelabel[i] > 255) bad("query edge label out of range");
        if (q.qtorder && (q.qtorder[i] < -1 || q.qtorder[i] > 31)) bad("temporal rank out of -1..31");
        for (uint32_t k = 0; k < i; k++)
            if (q.qsrc[k] == q.qsrc[i] && q.qdst[k] == q.qdst[i]) bad("repeated query edge");
    }
    bool seen[MN_MAXQV] = {false};
    seen[0] = true;
    for (uint32_t it = 0; it < q.n_qv; it++)
        for (uint32_t i = 0; i < q.n_qe; i++)
            if (seen[q.qsrc[i]] || seen[q.qdst[i]]) seen[q.qsrc[i]] = seen[q.qdst[i]] = true;
    for (uint32_t v = 0; v < q.n_qv; v++)
        if (!seen[v]) bad("query not weakly connected");
}

// The spanning-tree filter of Section V-B over each query's BFS tree from
// query vertex 0 (its root; edges taken in index order). Bottom-up (f4), by
// decreasing depth: a vertex keeps its bit for u only with a neighbour, over
// the tree edge to each child c, that keeps its bit for c. Top-down (f1), by
// increasing depth: a vertex keeps its bit for c only with a neighbour over
// the tree edge from the parent u that keeps its bit for u. Each depth is one
// round: its steps test and need disjoint bits.
void build_tree_steps(mnemonic_ctx* c, const mnemonic_query* qs, uint32_t n_q) {
    struct Edge {
        uint32_t depth;
        TreeStep up, down;
    };
    std::vector<Edge> edges;
    uint32_t maxd = 0;
    auto range = [&](TreeStep& st, int32_t lab, uint64_t req) {
        uint32_t lo = 0, hi = 0;
        bool exact = false;
        const bool some = class_hull(c, req, lo, hi, exact);
        st.whole = lab < 0 ? 1u : 0u;
        st.empty = some ? 0u : 1u;
        st.key_lo = st.key_hi = 0;
        if (lab >= 0 && some) {
            st.key_lo = ((uint32_t)lab << c->nbr_bits) | lo;
            st.key_hi = ((uint32_t)lab << c->nbr_bits) | (hi - 1);
        }
    };
    for (uint32_t i = 0; i < n_q; i++) {
        const mnemonic_query& q = qs[i];
        const uint32_t base = c->hq[i].vf_base;
        int depth[MN_MAXQV];
        for (auto& d : depth) d = -1;
        uint32_t queue[MN_MAXQV], head = 0, tail = 0;
        depth[0] = 0;
        queue[tail++] = 0;
        while (head < tail) {
            const uint32_t u = queue[head++];
            for (uint32_t k = 0; k < q.n_qe; k++) {
                uint32_t ch;
                bool out;
                if (q.qsrc[k] == u && depth[q.qdst[k]] < 0) {
                    ch = q.qdst[k];
                    out = true;
                } else if (q.qdst[k] == u && depth[q.qsrc[k]] < 0) {
                    ch = q.qsrc[k];
                    out = false;
                } else {
                    continue;
                }
                depth[ch] = depth[u] + 1;
                queue[tail++] = ch;
                Edge e;
                memset(&e, 0, sizeof(e));
                e.depth = (uint32_t)depth[ch];
                maxd = std::max(maxd, e.depth);
                e.up.test = (uint16_t)(base + u);
                e.up.need = (uint16_t)(base + ch);
                e.up.dir = out ? 0u : 1u;  // from f(u): out-list when the query edge leaves u
                range(e.up, q.qelabel[k], q.qv_require[ch]);
                e.down.test = (uint16_t)(base + ch);
                e.down.need = (uint16_t)(base + u);
                e.down.dir = out ? 1u : 0u;
                range(e.down, q.qelabel[k], q.qv_require[u]);
                edges.push_back(e);
            }
        }
    }
    c->htree.clear();
    c->tree_round.assign(1, 0);
    for (uint32_t d = maxd; d >= 1; d--) {
        for (const Edge& e : edges)
            if (e.depth == d) c->htree.push_back(e.up);
        c->tree_round.push_back((uint32_t)c->htree.size());
    }
    for (uint32_t d = 1; d <= maxd; d++) {
        for (const Edge& e : edges)
            if (e.depth == d) c->htree.push_back(e.down);
        c->tree_round.push_back((uint32_t)c->htree.size());
    }
}

// Expansion tile (256 x items candidates) for a query set whose plans have
// at most max_close closing edges: tiles of 1024 in blocks of 512 threads
// halve the output-place atomics at full occupancy where the kernels' arrays
// are small; with more closing edges those blocks spill registers, and tiles
// of 512 in blocks of 256 measured faster (64-query stream 5.4-5.6 against
// 5.8 ms per batch, serving 3.76 against 3.88 ms of device time).
uint32_t default_tile_items(uint32_t max_close) { return max_close <= 1 ? 4u : 2u; }

void prepare_queries(mnemonic_ctx* c, const mnemonic_query* qs, uint32_t n_q) {
    if (n_q == 0 || n_q > 255 || !qs) throw ApiError{MNEMONIC_E_ARG, "need 1..255 queries"};
    for (uint32_t i = 0; i < n_q; i++) check_query(qs[i]);
    c->n_q = n_q;
    // compact label tables
    for (int i = 0; i < 256; i++) c->elab_idx[i] = -1;
    for (int i = 0; i < 64; i++) c->vlab_idx[i] = -1;
    for (uint32_t i = 0; i < n_q; i++) {
        for (uint32_t k = 0; k < qs[i].n_qe; k++) {
            int l = qs[i].qelabel[k];
            if (l >= 0 && c->elab_idx[l] < 0) c->elab_idx[l] = (int16_t)c->n_elab_c++;
        }
        for (uint32_t u = 0; u < qs[i].n_qv; u++)
            for (int b = 0; b < 64; b++)
                if (((qs[i].qv_require[u] >> b) & 1) && c->vlab_idx[b] < 0) c->vlab_idx[b] = (int16_t)c->n_vlab_c++;
    }
    const uint32_t E = c->n_elab_c, Lc = c->n_vlab_c;
    c->n_cnt = 2 * (1 + E + Lc);
    uint32_t vf_base = 0, debi_base = 0, plan_base = 0;
    std::vector<std::vector<SeedPlan>> alts;  // per static plan: all of its orders
    for (uint32_t i = 0; i < n_q; i++) {
        const mnemonic_query& q = qs[i];
        QueryDev Q;
        memset(&Q, 0, sizeof(Q));
        Q.n_qv = q.n_qv;
        Q.n_qe = q.n_qe;
        Q.sem = (uint32_t)q.sem;
        Q.vf_base = vf_base;
        Q.debi_base = debi_base;
        Q.plan_base = plan_base;
        Q.out_index = i;
        for (uint32_t u = 0; u < q.n_qv; u++) Q.vreq[u] = q.qv_require[u];
        for (uint32_t k = 0; k < q.n_qe; k++) {
            Q.qsrc[k] = (uint8_t)q.qsrc[k];
            Q.qdst[k] = (uint8_t)q.qdst[k];
            Q.qlab[k] = q.qelabel[k];
        }
        const bool iso = q.sem == MNEMONIC_ISO;
        // local filters per query vertex (Section V-A, f2 and f3)
        for (uint32_t u = 0; u < q.n_qv; u++) {
            Q.req_begin[u] = (uint16_t)c->hreq.size();
            VfBit vb;
            vb.vreq = q.qv_require[u];
            vb.req_begin = (uint32_t)c->hreq.size();
            for (uint32_t dir = 0; dir < 2; dir++) {
                uint32_t tot = 0;
                uint32_t per_lab[256] = {0};
                uint32_t per_vl[64] = {0};
                for (uint32_t k = 0; k < q.n_qe; k++) {
                    uint32_t near = dir == 0 ? q.qsrc[k] : q.qdst[k];
                    uint32_t far = dir == 0 ? q.qdst[k] : q.qsrc[k];
                    if (near != u) continue;
                    tot++;
                    if (q.qelabel[k] >= 0) per_lab[q.qelabel[k]]++;
                    for (int b = 0; b < 64; b++)
                        if ((q.qv_require[far] >> b) & 1) per_vl[b]++;
                }
                auto need = [&](uint32_t n) { return (uint16_t)(iso ? n : (n ? 1 : 0)); };
                if (tot) c->hreq.push_back(VfReq{(uint16_t)cnt_index(dir, 0, E, Lc), need(tot)});
                for (int l = 0; l < 256; l++)
                    if (per_lab[l])
                        c->hreq.push_back(VfReq{(uint16_t)cnt_index(dir, 1 + c->elab_idx[l], E, Lc), need(per_lab[l])});
                for (int b = 0; b < 64; b++)
                    if (per_vl[b])
                        c->hreq.push_back(
                            VfReq{(uint16_t)cnt_index(dir, 1 + E + c->vlab_idx[b], E, Lc), need(per_vl[b])});
            }
            vb.req_end = (uint32_t)c->hreq.size();
            c->hvf.push_back(vb);
        }
        Q.req_begin[q.n_qv] = (uint16_t)c->hreq.size();
        for (uint32_t k = 0; k < q.n_qe; k++) {
            DebiBit db;
            db.label = q.qelabel[k];
            db.pad = 0;
            db.req_src = q.qv_require[q.qsrc[k]];
            db.req_dst = q.qv_require[q.qdst[k]];
            c->hdebi.push_back(db);
        }
        for (uint32_t j = 0; j < q.n_qe; j++) {
            // the static order, then the distinct alternatives (kept aside:
            // they follow every static plan)
            SeedPlan P;
            build_plan(c, Q, i, j, P, 0);
            set_ranks(P, q);
            P.n_var = 1;
            P.variant = 0;
            std::vector<SeedPlan> vs(1, P);
            for (uint32_t v : {3u, 1u, 2u}) {
                SeedPlan V;
                build_plan(c, Q, i, j, V, v);
                set_ranks(V, q);
                bool dup = false;
                for (const SeedPlan& W : vs)
                    dup = dup || (memcmp(W.mapped, V.mapped, sizeof(V.mapped)) == 0 &&
                                  memcmp(W.lv, V.lv, sizeof(V.lv)) == 0 && memcmp(W.close, V.close, sizeof(V.close)) == 0);
                if (!dup && vs.size() < MN_NVAR) vs.push_back(V);
            }
            for (uint32_t v = 0; v < vs.size(); v++) {
                SeedPlan& V = vs[v];
                c->max_levels = std::max<uint32_t>(c->max_levels, V.n_levels);
                c->max_close = std::max<uint32_t>(c->max_close, V.n_close);
                for (uint32_t L = 0; L < V.n_levels; L++) {
                    if (L + 1 == V.n_levels)
                        c->level_emit[L] = 1;
                    else
                        c->level_rows[L] = 1;
                }
                V.n_var = (uint8_t)vs.size();
                V.variant = (uint8_t)v;
            }
            c->hplans.push_back(vs[0]);
            alts.push_back(vs);
        }
        vf_base += q.n_qv;
        debi_base += q.n_qe;
        plan_base += q.n_qe;
        c->hq.push_back(Q);
    }
    // alternatives after the static plans; every order of a pair lists all of them
    c->n_static = (uint32_t)c->hplans.size();
    for (uint32_t sp = 0; sp < c->n_static; sp++) {
        std::vector<SeedPlan>& vs = alts[sp];
        uint16_t idx[MN_NVAR] = {0, 0, 0, 0};
        idx[0] = (uint16_t)sp;
        for (uint32_t v = 1; v < vs.size(); v++) idx[v] = (uint16_t)(c->hplans.size() + v - 1);
        if (c->hplans.size() + vs.size() > 65535) throw ApiError{MNEMONIC_E_LIMIT, "too many matching orders"};
        for (uint32_t v = 0; v < vs.size(); v++) memcpy(vs[v].vars, idx, sizeof(idx));
        c->hplans[sp] = vs[0];
        for (uint32_t v = 1; v < vs.size(); v++) c->hplans.push_back(vs[v]);
    }
    c->n_plans = (uint32_t)c->hplans.size();
    for (uint32_t i = 0; i < n_q; i++) {
        c->wv = std::max<uint32_t>(c->wv, qs[i].n_qv);
        c->we = std::max<uint32_t>(c->we, qs[i].n_qe);
    }
    c->n_vf_bits = vf_base;
    c->n_debi_bits = debi_base;
    c->total_qe = debi_base;
    c->vf_words = (vf_base + 31) / 32;
    c->debi_words = (debi_base + 31) / 32;
    build_tree_steps(c, qs, n_q);
}

template <typename T>
void upload(T*& d, const std::vector<T>& h, hipStream_t s) {
    dev_alloc(d, h.size());
    if (!h.empty()) HIPCHK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

GraphView make_view(const mnemonic_ctx* c, bool next) {
    GraphView g;
    memset(&g, 0, sizeof(g));
    g.n_vertices = c->nV;
    g.nbr_bits = c->nbr_bits;
    g.nbr_mask = (1u << c->nbr_bits) - 1u;
    g.n_cnt = c->n_cnt;
    g.vf_words = c->vf_words;
    g.debi_words = c->debi_words;
    g.n_queries = c->n_q;
    g.n_vfreq = (uint32_t)c->hreq.size();
    g.vmask = c->d_vmask;
    for (int d = 0; d < 2; d++) {
        g.off[d] = next ? c->d_off2[d] : c->d_off[d];
        g.adj[d] = next ? c->d_adj2[d] : c->d_adj[d];
        g.adjk[d] = next ? c->d_adjk2[d] : c->d_adjk[d];
    }
    g.vf = c->d_vf;
    g.cnt = c->d_cnt;
    g.s_src = c->d_src;
    g.s_dst = c->d_dst;
    g.s_lab = c->d_lab;
    g.s_ts = c->d_ts;
    g.s_key = c->d_key;
    g.s_debi = c->d_debi;
    g.queries = c->d_q;
    g.plans = c->d_plans;
    g.vfreq = c->d_req;
    g.elab_idx = c->d_elab_idx;
    g.vlab_idx = c->d_vlab_idx;
    g.ext2int = c->d_ext2int;
    g.key_ts = c->d_key_ts;
    g.key_mask = c->cap_keys ? c->cap_keys - 1 : 0;
    g.n_elab_c = c->n_elab_c;
    g.n_vlab_c = c->n_vlab_c;
    g.n_static = c->n_static;
    g.sched_mode = c->sched_mode;
    g.sched_w = c->d_sched_w;
    g.dec = c->deciding() ? c->d_dec : nullptr;
    g.dec_n = c->d_dec_n;
    g.tr_cap = c->tr_cap;
    g.tr_n = c->d_tr_n;
    g.tr_code = c->d_tr_code;
    g.tr_x = c->d_tr_x;
    g.tr_work = c->d_tr_work;
    return g;
}

// Makes every buffer large enough for a snapshot of n_ins insertions and
// n_del deletions.
// Batch scratch starts sized for this many edges (and doubles past it), so
// that batches of up to 2^18 insertions or deletions never stop to allocate.
constexpr uint64_t kScratchMin = 1ull << 18;

void ensure_capacity(mnemonic_ctx* c, uint64_t n_ins, uint64_t n_del) {
    hipStream_t s = c->stream;
    uint64_t need_slots = (uint64_t)c->fresh + (n_ins > c->n_free ? n_ins - c->n_free : 0);
    uint64_t live_slots = c->fresh;
    if (need_slots >= (1ull << 31)) throw ApiError{MNEMONIC_E_LIMIT, "more than 2^31 edge slots"};
    if (need_slots > c->cap_slots) {
        uint64_t cap = c->cap_slots;
        uint64_t t;
        t = cap; dev_grow(c->d_src, t, need_slots, live_slots, s);
        t = cap; dev_grow(c->d_dst, t, need_slots, live_slots, s);
        t = cap; dev_grow(c->d_lab, t, need_slots, live_slots, s);
        t = cap; dev_grow(c->d_ts, t, need_slots, live_slots, s);
        t = cap; dev_grow(c->d_key, t, need_slots, live_slots, s);
        t = cap; dev_grow(c->d_free, t, need_slots, c->n_free, s);
        uint64_t dcap = cap * c->debi_words;
        dev_grow(c->d_debi, dcap, t * c->debi_words, live_slots * c->debi_words, s);
        c->cap_slots = t;
    }
    // the key rings must place every key from key_lo to the end of this batch
    // apart; a larger ring takes the entries of the keys that may still be met
    const uint64_t span = c->next_key + n_ins - c->key_lo;
    if (span >= c->cap_keys) {
        uint64_t nc = 1024;
        while (nc < span + span / 4 + 1) nc *= 2;
        uint32_t* k2s = nullptr;
        int64_t* kts = nullptr;
        uint32_t* bits = nullptr;
        try {
            dev_alloc(k2s, nc);
            dev_alloc(kts, nc);
            dev_alloc(bits, nc / 32);
        } catch (...) {
            dev_free(k2s);
            dev_free(kts);
            dev_free(bits);
            throw;
        }
        mn_launch_fill_u32(bits, 0u, nc / 32, s);
        if (c->cap_keys)
            mn_launch_ring_copy(c->d_key2slot, c->d_key_ts, c->cap_keys - 1, k2s, kts, nc - 1, c->key_lo,
                                c->next_key, s);
        dev_free(c->d_key2slot);  // stream-ordered: after the copy
        dev_free(c->d_key_ts);
        dev_free(c->d_delbits);
        c->d_key2slot = k2s;
        c->d_key_ts = kts;
        c->d_delbits = bits;
        c->cap_keys = nc;
        c->cap_delbits = nc / 32;
    }
    uint64_t need_E = c->E - c->n_pending + n_ins;
    c->hb_pos = std::max<uint32_t>(1, ceil_log2(std::max<uint64_t>(c->E, need_E) + 1));
    // adjacency positions must stay below 2^31 (bit 31 tags closing-edge runs)
    if (need_E >= (1ull << 31) - 1) throw ApiError{MNEMONIC_E_LIMIT, "more than 2^31 adjacency entries"};
    for (int d = 0; d < 2; d++) {
        uint64_t t = c->cap_E;
        dev_grow(c->d_adj[d], t, need_E, c->E, s);
        t = c->cap_E;
        dev_grow(c->d_adjk[d], t, need_E, c->E, s);
        t = c->cap_E;
        dev_grow(c->d_adjk2[d], t, need_E, 0, s);
        t = c->cap_E;
        dev_grow(c->d_adj2[d], t, need_E, 0, s);
        if (d == 1) c->cap_E = t;
    }
    dev_grow(c->d_mlim, c->cap_mlim, 2 * mn_merge_limit_words(c->E), 0, s);
    if (n_ins > c->cap_ins) {
        uint64_t nc = std::max<uint64_t>(std::max<uint64_t>(n_ins, kScratchMin), 2 * c->cap_ins);
        c->cap_ins = 0;  // until every buffer below exists again (an allocation may fail)
        dev_free(c->d_in_src);
        dev_free(c->d_in_dst);
        dev_free(c->d_in_lab);
        dev_free(c->d_in_ts);
        dev_free(c->d_ins_slot);
        dev_alloc(c->d_in_src, nc);
        dev_alloc(c->d_in_dst, nc);
        dev_alloc(c->d_in_lab, nc);
        dev_alloc(c->d_in_ts, nc);
        dev_alloc(c->d_ins_slot, nc);
        for (int k = 0; k < 2; k++) {
            dev_free(c->d_skey[k]);
            dev_free(c->d_sval[k]);
            dev_alloc(c->d_skey[k], 2 * nc);
            dev_alloc(c->d_sval[k], 2 * nc);
        }
        for (int d = 0; d < 2; d++) {
            dev_free(c->d_inspos[d]);
            dev_free(c->d_ub[d]);
            dev_alloc(c->d_inspos[d], nc);
            dev_alloc(c->d_ub[d], nc);
        }
        c->cap_ins = nc;
    }
    if (n_del > c->cap_del) {
        uint64_t nc = std::max<uint64_t>(std::max<uint64_t>(n_del, kScratchMin), 2 * c->cap_del);
        c->cap_del = 0;
        dev_free(c->d_del_keys);
        dev_alloc(c->d_del_keys, nc);
        c->cap_del = nc;
    }
    // the delete buffer that receives this snapshot's deletions
    int cur = 1 - c->pend;
    if (n_del > c->cap_delbuf[cur]) {
        uint64_t nc = std::max<uint64_t>(std::max<uint64_t>(n_del, kScratchMin), 2 * c->cap_delbuf[cur]);
        c->cap_delbuf[cur] = 0;
        dev_free(c->d_del_slot[cur]);
        dev_alloc(c->d_del_slot[cur], nc);
        for (int d = 0; d < 2; d++) {
            dev_free(c->d_delpos[cur][d]);
            dev_alloc(c->d_delpos[cur][d], nc);
        }
        c->cap_delbuf[cur] = nc;
    }
    uint64_t n_sort = std::max<uint64_t>(n_ins, c->n_pending);
    if (n_sort > c->cap_sort) {
        uint64_t nc = std::max<uint64_t>(std::max<uint64_t>(n_sort, kScratchMin), 2 * c->cap_sort);
        c->cap_sort = 0;
        for (int k = 0; k < 2; k++) {
            dev_free(c->d_dkey[k]);
            dev_free(c->d_dval[k]);
            dev_alloc(c->d_dkey[k], 2 * nc);
            dev_alloc(c->d_dval[k], 2 * nc);
        }
        c->cap_sort = nc;
    }
    uint64_t ssw = mn_sort_scratch_words((uint32_t)std::max<uint64_t>(2 * n_sort, 2 * kScratchMin));
    if (ssw > c->cap_sort_scratch) {
        c->cap_sort_scratch = 0;
        dev_free(c->d_sort_scratch);
        dev_alloc(c->d_sort_scratch, ssw);
        c->cap_sort_scratch = ssw;
    }
    uint64_t n_touch = 2 * (c->n_pending + n_ins);
    if (n_touch > c->cap_touch) {
        uint64_t nc = std::max<uint64_t>(std::max<uint64_t>(n_touch, 2 * kScratchMin), 2 * c->cap_touch);
        c->cap_touch = 0;
        dev_free(c->d_touched);
        dev_alloc(c->d_touched, nc);
        c->cap_touch = nc;
    }
}

// Each buffer is replaced only once its successor is allocated, and the
// device's copy of the table follows the host's whenever anything changed,
// also when an allocation fails part way (the error then leaves every buffer
// valid at its recorded capacity).
void grow_outputs(mnemonic_ctx* c, const std::vector<uint64_t>& need) {
    bool changed = false;
    auto upload = [&]() {
        HIPCHK(hipMemcpyAsync(c->d_outs, c->houts.data(), c->houts.size() * sizeof(OutView),
                              hipMemcpyHostToDevice, c->stream));
    };
    try {
        for (uint32_t q = 0; q < c->n_q; q++)
            for (int p = 0; p < 2; p++) {
                uint64_t n = need[2 * q + p];
                if (n <= c->houts[q].cap[p]) continue;
                // a quarter above the need, or up to twice it for a buffer that
                // keeps growing
                uint64_t nc = std::max<uint64_t>(n + n / 4, std::min<uint64_t>(c->houts[q].cap[p] * 2, 2 * n));
                uint64_t* fresh = nullptr;
                dev_alloc(fresh, nc * c->hq[q].n_qe);
                dev_free(c->houts[q].keys[p]);  // stream-ordered: after the launches that wrote it
                c->houts[q].keys[p] = fresh;
                c->houts[q].cap[p] = nc;
                changed = true;
            }
    } catch (...) {
        if (changed) upload();
        throw;
    }
    if (changed) upload();
}

PhaseOut phase_out(mnemonic_ctx* c, int p) {
    PhaseOut po;
    po.count = c->d_zr + c->zr_count(p);
    po.digest = c->d_zr + c->zr_digest(p);
    po.stats = reinterpret_cast<EnumStats*>(c->d_zr + c->zr_stats(p));
    po.n_q = c->n_q;
    po.outs = c->d_outs;
    po.phase = p;
    po.emit = (c->flags & MNEMONIC_F_EMIT) ? 1 : 0;
    return po;
}

void reset_phase(mnemonic_ctx* c, int p) {
    hipStream_t s = c->stream;
    // counts, digests, cursor and stats of one phase (err is 0 whenever this runs)
    mn_launch_reset(c->d_err, c->d_zr + c->zr_count(p), c->n_q, s);
    mn_launch_reset(c->d_err, c->d_zr + c->zr_digest(p), MN_SHARDS * 2 * c->n_q, s);
    mn_launch_reset(c->d_err, c->d_zr + c->zr_stats(p), MN_SHARDS * MN_TALLIES, s);
    mn_launch_reset(c->d_err, c->d_zr + c->zr_note(p), 4 * (MN_MAXLV + 1), s);
    if (c->tr_cap) mn_launch_set_u32(c->d_tr_n + p, 0, s);
}

// Grows level L's buffers to hold `need` rows (contents are not kept: a
// level is only grown while it holds no rows).
void grow_level(mnemonic_ctx* c, uint32_t L, uint64_t need) {
    auto& B = c->lvb[L];
    if (need <= B.cap) return;
    if (t_no_alloc) return;  // the level keeps its rows; a larger need is noted by the kernels
    uint64_t nc = std::min<uint64_t>(c->rows_max, std::max<uint64_t>(need, std::max<uint64_t>(B.cap * 2, 4096)));
    dev_free(B.rows);  // stream-ordered: after the launches that used them
    dev_free(B.keys);
    dev_free(B.lo);
    dev_free(B.cnt);
    dev_free(B.off);
    dev_free(B.hpre);
    B.cap = 0;
    dev_alloc(B.rows, nc * c->ncol());
    dev_alloc(B.keys, nc * c->we);
    dev_alloc(B.lo, nc);
    dev_alloc(B.cnt, nc);
    dev_alloc(B.off, nc);
    dev_alloc(B.hpre, 2 * nc);
    B.cap = nc;
    uint64_t sw = mn_scan64_scratch_words((uint32_t)nc);
    if (sw > c->cap_scan64) {
        c->cap_scan64 = 0;
        dev_free(c->d_scan64);
        dev_alloc(c->d_scan64, sw);
        c->cap_scan64 = sw;
    }
}

RowsView rows_view(const mnemonic_ctx* c, uint32_t L) {
    RowsView R;
    memset(&R, 0, sizeof(R));
    R.wv = c->wv;
    R.we = c->we;
    R.trace = c->tr_cap ? 1u : 0u;
    if (L < c->lvb.size()) {
        R.col = c->lvb[L].rows;
        R.kcol = c->lvb[L].keys;
        R.hpre = c->lvb[L].hpre;
        R.cap = (uint32_t)c->lvb[L].cap;
    }
    return R;
}

// Pinned staging of n_zr + 1 words (the readback block and the error word).
void size_zr_pin(mnemonic_ctx* c) {
    if (c->cap_zr_pin >= c->n_zr + 2) return;
    if (c->h_zr_pin) (void)hipHostFree(c->h_zr_pin);
    c->h_zr_pin = nullptr;
    c->cap_zr_pin = 0;
    HIPCHK(hipHostMalloc((void**)&c->h_zr_pin, (c->n_zr + 2) * 8, hipHostMallocDefault));
    c->cap_zr_pin = c->n_zr + 2;
}

// The readback block into h_zr (and the error word into *err when given):
// both copies land in pinned memory, then one wait.
void read_zr(mnemonic_ctx* c, uint32_t* err) {
    hipStream_t s = c->stream;
    HIPCHK(hipMemcpyAsync(c->h_zr_pin, c->d_zr, c->n_zr * 8, hipMemcpyDeviceToHost, s));
    if (err) {
        c->h_zr_pin[c->n_zr] = 0;
        HIPCHK(hipMemcpyAsync(c->h_zr_pin + c->n_zr, c->d_err, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(c->h_zr_pin + c->n_zr + 1, c->d_key_lo, 8, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    std::memcpy(c->h_zr.data(), c->h_zr_pin, c->n_zr * 8);
    if (err) {
        *err = (uint32_t)c->h_zr_pin[c->n_zr];
        c->key_lo_seen = c->h_zr_pin[c->n_zr + 1];
    }
}

uint64_t read_u32(mnemonic_ctx* c, const uint32_t* d) {
    HIPCHK(hipMemcpyAsync(c->h_ctl, d, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return *reinterpret_cast<uint32_t*>(c->h_ctl);
}

uint64_t read_u64(mnemonic_ctx* c, const uint64_t* d) {
    HIPCHK(hipMemcpyAsync(c->h_ctl, d, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return c->h_ctl[0];
}

// Level L of the search over the n rows of level buffer L: candidate runs,
// their offsets, then the candidate space in chunks no larger than the next
// level's row buffer; each chunk's survivors are searched to the end before
// the next chunk starts (depth first over chunks, breadth first inside one).
void process_level(mnemonic_ctx* c, const GraphView& g, const PhaseOut& po, uint32_t L, uint64_t n) {
    if (n == 0) return;
    hipStream_t s = c->stream;
    auto& B = c->lvb[L];
    mn_launch_level_range(g, rows_view(c, L), (uint32_t)n, nullptr, L, B.lo, B.cnt, po.stats, c->d_err, s);
    mn_scan_exclusive64(B.cnt, B.off, (uint32_t)n, c->d_scan64, c->d_total, s);
    const uint64_t T = read_u64(c, c->d_total);
    if (T == 0) return;
    const bool next = L + 1 < c->max_levels;
    if (next) grow_level(c, L + 1, T);
    // chunks bounded by the next level's rows (each candidate yields <= 1 row),
    // and in a no-allocation call by the tile buffer the context holds
    uint64_t K = next ? c->lvb[L + 1].cap : (1ull << 26);
    if (t_no_alloc) K = std::min<uint64_t>(K, c->cap_tiles >= 2 ? (c->cap_tiles - 1) * MN_BLOCK : 0);
    if (K == 0) throw ApiError{MNEMONIC_E_CAPACITY, "no room for one level of the enumeration"};
    const bool timing = (c->flags & (MNEMONIC_F_TIMING | MNEMONIC_F_AUTOTUNE)) != 0 && !t_no_alloc;
    for (uint64_t c0 = 0; c0 < T; c0 += K) {
        const uint64_t c1 = std::min<uint64_t>(T, c0 + K);
        uint32_t* n_out = c->d_nrows + L + 1;
        mn_launch_set_u32(n_out, 0, s);
        const uint64_t need_tiles = mn_expand_tiles(c0, c1) + 1;
        if (need_tiles > c->cap_tiles) {
            dev_free(c->d_tiles);
            c->cap_tiles = 0;
            dev_alloc(c->d_tiles, need_tiles);
            c->cap_tiles = need_tiles;
        }
        // one event pair serves every launch: the readback below waits for it
        mn_launch_expand(g, rows_view(c, L), (uint32_t)n, nullptr, B.lo, B.off, nullptr, c->d_tiles, c0, c1, nullptr,
                         nullptr, 0,
                         c->tile_items, L, c->max_close, c->level_rows[L] != 0, c->level_emit[L] != 0,
                         rows_view(c, L + 1), n_out, po, c->d_err, s, timing ? c->ev_x[0] : nullptr,
                         timing ? c->ev_x[1] : nullptr);
        c->n_expand[po.phase]++;
        const uint64_t n1 = read_u32(c, n_out);
        if (timing) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, c->ev_x[0], c->ev_x[1]));
            c->ms_expand[po.phase] += ms;
        }
        if (next && n1 > c->lvb[L + 1].cap) throw ApiError{MNEMONIC_E_HIP, "row buffer overflow (internal)"};
        if (next) process_level(c, g, po, L + 1, n1);
    }
}

// Event pair i of the batch (created on first use).
std::pair<hipEvent_t, hipEvent_t> event_pair(mnemonic_ctx* c, int phase) {
    const uint32_t i = c->ev_used++;
    while (c->ev_pool.size() < 2 * (size_t)(i + 1)) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        c->ev_pool.push_back(e);
    }
    if (c->ev_phase.size() < i + 1) c->ev_phase.resize(i + 1);
    c->ev_phase[i] = phase;
    return {c->ev_pool[2 * i], c->ev_pool[2 * i + 1]};
}

// Adds the durations of the recorded device-sized expansions (after a sync).
void resolve_events(mnemonic_ctx* c) {
    for (uint32_t i = 0; i < c->ev_used; i++) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, c->ev_pool[2 * i], c->ev_pool[2 * i + 1]));
        c->ms_expand[c->ev_phase[i]] += ms;
    }
    c->ev_used = 0;
}

// All levels of one chunk of start rows with no host round trip: every
// launch reads its row count and candidate total from device memory and
// each level takes at most as many candidates as the next level's buffer
// holds. A level with more sets its note; the host then grows the buffers
// and runs the phase again.
void device_levels(mnemonic_ctx* c, const GraphView& g, const PhaseOut& po, uint64_t n0_max, uint64_t ns) {
    hipStream_t s = c->stream;
    const bool timing = (c->flags & (MNEMONIC_F_TIMING | MNEMONIC_F_AUTOTUNE)) != 0 && !t_no_alloc;
    // every level takes some rows, so that an overflow always leaves a note;
    // levels and the candidate buffer are sized at the largest rates seen
    // with a margin, so that a batch larger than any before does not re-run
    // the phase to grow them
    for (uint32_t L = 1; L < c->max_levels; L++) {
        const double rr = c->row_rate[po.phase][L];
        const uint64_t want = rr > 0 ? (uint64_t)(1.5 * rr * (double)ns) : 0;
        grow_level(c, L, std::min<uint64_t>(c->rows_max, std::max<uint64_t>(1ull << 16, want)));
    }
    {
        const uint64_t most = MN_EXPAND_MAX_BLOCKS * MN_BLOCK * c->tile_items;
        uint64_t want = 0;
        for (uint32_t L = 0; L < c->max_levels; L++)
            if (c->rate[po.phase][L] > 0) want = std::max<uint64_t>(want, (uint64_t)(1.5 * c->rate[po.phase][L] * (double)ns));
        if (want > c->cand_k && want <= most / 2) c->cand_k = std::min<uint64_t>(most, std::max<uint64_t>(want, 2 * c->cand_k));
    }
    // candidates one launch may take: bounded by the tile buffer (a
    // no-allocation call takes what the buffer it has covers)
    uint64_t K = c->cand_k;
    const uint64_t need_tiles = mn_expand_tiles(0, K) + 1;
    if (need_tiles > c->cap_tiles) {
        if (t_no_alloc) {
            K = c->cap_tiles >= 2 ? (c->cap_tiles - 1) * MN_BLOCK : 0;
        } else {
            dev_free(c->d_tiles);
            c->cap_tiles = 0;
            dev_alloc(c->d_tiles, need_tiles);
            c->cap_tiles = need_tiles;
        }
    }
    uint64_t n_max = std::min<uint64_t>(n0_max, c->lvb[0].cap);
    for (uint32_t L = 0; L < c->max_levels; L++) {
        auto& B = c->lvb[L];
        const uint32_t* n_dev = c->d_nrows + L;
        const bool next = L + 1 < c->max_levels;
        uint32_t* n_out = c->d_nrows + L + 1;
        // the rows level L - 1 made (the start rows at level 0) are noted
        // against this buffer here, and the next level's row counter starts
        // at zero
        mn_launch_level_range(g, rows_view(c, L), (uint32_t)n_max, n_dev, L, B.lo, B.cnt, po.stats, c->d_err, s,
                              next ? n_out : nullptr,
                              c->d_zr + (L ? c->note_rows(po.phase, L - 1) : c->note_seed(po.phase)));
        // candidates are bounded by the tile buffer and the grid only; rows
        // past the next level's buffer are counted and noted
        unsigned long long* note = c->d_zr + c->note_cand(po.phase, L);
        const double rt = c->rate[po.phase][L];
        const uint64_t expect = rt < 0 ? (~0ull >> 8) : (uint64_t)(rt * (double)ns) + 1;
        // offsets, total and partition in two launches where the rows fit
        // MN_SCAN_DIRECT_MAX scan tiles, else the general scan and partition
        const uint32_t nb = (uint32_t)((n_max + MN_SCAN_TILE - 1) / MN_SCAN_TILE);
        const bool fused = n_max > 0 && K > 0 && nb <= MN_SCAN_DIRECT_MAX;
        if (fused) {
            mn_scan64_local(B.cnt, B.off, (uint32_t)n_max, c->d_scan64, s, n_dev);
            mn_launch_offsets_partition(B.cnt, B.off, c->d_scan64, nb, (uint32_t)n_max, n_dev, 0,
                                        mn_expand_end(0, K, expect, c->tile_items), c->d_total, c->tile_items,
                                        c->d_tiles, note, s);
        } else {
            mn_scan_exclusive64(B.cnt, B.off, (uint32_t)n_max, c->d_scan64, nullptr, s, n_dev);
        }
        std::pair<hipEvent_t, hipEvent_t> ev(nullptr, nullptr);
        if (timing) ev = event_pair(c, po.phase);
        c->cover[po.phase][L] =
            mn_launch_expand(g, rows_view(c, L), (uint32_t)n_max, n_dev, B.lo, B.off, B.cnt, c->d_tiles, 0, K,
                             c->d_total, note, expect, c->tile_items, L, c->max_close, c->level_rows[L] != 0,
                             c->level_emit[L] != 0, rows_view(c, L + 1), n_out, po, c->d_err, s, ev.first, ev.second,
                             fused);
        c->n_expand[po.phase]++;
        if (next) n_max = c->lvb[L + 1].cap;
    }
}

// One enumeration phase (p = 0: new embeddings of the inserted slots; 1:
// expired embeddings of the deleted slots) on the current graph view. With
// host_chunks the levels are walked with host round trips and chunked to any
// size; otherwise they run device-sized (device_levels).
void enumerate_phase(mnemonic_ctx* c, int p, const uint32_t* slots, uint64_t n_slots, bool host_chunks = false) {
    hipStream_t s = c->stream;
    const bool timing = (c->flags & (MNEMONIC_F_TIMING | MNEMONIC_F_AUTOTUNE)) != 0 && !t_no_alloc;
    if (timing) HIPCHK(hipEventRecord(c->ev[2 * p], s));
    if (n_slots && c->n_static) {
        GraphView g = make_view(c, false);
        if (c->tree_on()) g.vf = c->d_vfp;
        PhaseOut po = phase_out(c, p);
        // Start rows per slot: the last batches' rate with a margin when known
        // (the seed kernel counts past the buffer and the phase is re-run if
        // that was short), else every (slot, plan) pair; host-walked levels
        // keep the worst case.
        const double r0 = c->rate[p][MN_MAXLV];
        const double per_slot = (host_chunks || r0 < 0) ? (double)c->n_static : std::min<double>(c->n_static, 1.5 * r0 + 0.01);
        // a no-allocation call walks the start rows in chunks its first level holds
        const double room = t_no_alloc && host_chunks && c->max_levels ? (double)c->lvb[0].cap : (double)c->rows_max;
        const uint64_t chunk = std::max<uint64_t>(1, (uint64_t)(room / per_slot));
        c->chunk_ns[p] = std::min<uint64_t>(chunk, n_slots);
        for (uint64_t s0 = 0; s0 < n_slots; s0 += chunk) {
            const uint64_t ns = std::min<uint64_t>(chunk, n_slots - s0);
            if (c->max_levels)  // else every plan emits at once
                grow_level(c, 0, std::min<uint64_t>(c->rows_max, (uint64_t)(per_slot * (double)ns) + 1024));
            // without room for the decision list (no-allocation call) the start
            // rows keep the static order: the results do not depend on it
            const bool decide = c->max_levels && c->deciding() && !(t_no_alloc && c->cap_dec < c->lvb[0].cap);
            if (!decide) g.dec = nullptr;
            if (decide) {
                if (c->cap_dec < c->lvb[0].cap) {
                    dev_free(c->d_dec);
                    c->cap_dec = 0;
                    dev_alloc(c->d_dec, c->lvb[0].cap);
                    c->cap_dec = c->lvb[0].cap;
                }
                mn_launch_set_u32(c->d_dec_n, 0, s);
                g.dec = c->d_dec;
            }
            mn_launch_set_u32(c->d_nrows, 0, s);
            g.tr_base = (uint32_t)s0;
            mn_launch_seed_rows(g, slots + s0, (uint32_t)ns, c->n_static, c->max_close, rows_view(c, 0), c->d_nrows,
                                po, c->d_err, s);
            if (c->max_levels == 0) continue;
            if (decide)
                mn_launch_decide(g, rows_view(c, 0), slots + s0, (uint32_t)c->cap_dec,
                                 (uint32_t)std::min<double>((double)c->cap_dec, per_slot * (double)ns + 1.0), p, s);
            if (host_chunks) {
                mn_launch_note_count(c->d_nrows, c->lvb[0].cap, c->d_zr + c->note_seed(p), s);
                const uint64_t n0 = read_u32(c, c->d_nrows);
                process_level(c, g, po, 0, n0);
            } else {
                device_levels(c, g, po, ns * c->n_static, ns);
            }
        }
    }
    if (timing) HIPCHK(hipEventRecord(c->ev[2 * p + 1], s));
}

// After a device-sized phase: grows what its notes say was too small.
// Returns true when the phase must run again; host_chunks is set when a level
// needs more rows than one buffer may hold.
// cause receives the stats' rerun_causes bits of what was too small.
bool absorb_notes(mnemonic_ctx* c, int p, bool& host_chunks, uint64_t& cause, std::string* why = nullptr) {
    const unsigned long long* z = c->h_zr.data();
    bool again = false;
    auto say = [&](const char* what, uint32_t L, uint64_t got, uint64_t room) {
        if (!why) return;
        char buf[160];
        snprintf(buf, sizeof(buf), " [phase %d level %u: %s %llu > %llu]", p, L, what, (unsigned long long)got,
                 (unsigned long long)room);
        *why += buf;
    };
    const double ns = (double)std::max<uint64_t>(1, c->chunk_ns[p]);
    // A stage that was cut short fed only part of its output to the levels
    // below: their totals are scaled by the parts left out (cut), so that one
    // re-run sizes every level.
    double cut = 1.0;
    auto grow_rows = [&](uint32_t L, uint64_t need) {  // rows of level L
        if (need > c->rows_max)
            host_chunks = true;
        else if (need > c->lvb[L].cap)  // twice the need: batches vary, a re-run costs a whole phase
            grow_level(c, L, std::max<uint64_t>(2 * need, 2 * c->lvb[L].cap));
    };
    const unsigned long long* ns0 = z + c->note_seed(p);
    if (ns0[0]) {  // start rows past their buffer
        again = true;
        cause |= 1u;
        say("start rows", 0, ns0[1], c->max_levels ? c->lvb[0].cap : 0);
        c->rate[p][MN_MAXLV] = std::max<double>(c->rate[p][MN_MAXLV], (double)ns0[1] / ns);
        if (c->max_levels && c->lvb[0].cap) cut = std::max<double>(1.0, (double)ns0[1] / (double)c->lvb[0].cap);
        grow_rows(0, ns0[1]);
    }
    for (uint32_t L = 0; L < c->max_levels; L++) {
        const unsigned long long* nc = z + c->note_cand(p, L);
        const unsigned long long* nr = z + c->note_rows(p, L);
        if (!nc[1]) continue;
        const double T_est = (double)nc[1] * cut;
        if (nc[0] || cut > 1.0) c->rate[p][L] = std::max<double>(c->rate[p][L], T_est / ns);
        if (nc[0]) {  // more candidates than the launch covered
            again = true;
            cause |= 2u;
            say("candidates", L, nc[1], c->cover[p][L]);
            if (c->cover[p][L] > 0) cut *= std::max<double>(1.0, (double)nc[1] / (double)c->cover[p][L]);
            // past what one device-sized launch can cover, the levels are walked in host chunks
            const uint64_t most = MN_EXPAND_MAX_BLOCKS * MN_BLOCK * c->tile_items;
            if ((uint64_t)T_est > most / 2)
                host_chunks = true;
            else if ((uint64_t)T_est > c->cand_k)
                c->cand_k = std::min<uint64_t>(most, std::max<uint64_t>(2 * (uint64_t)T_est, 2 * c->cand_k));
        }
        if (L + 1 < c->max_levels && nr[1]) {
            const double R_est = (double)nr[1] * cut;
            if (nr[0] || cut > 1.0) grow_rows(L + 1, (uint64_t)R_est);
            if (nr[0]) {  // rows past the next level's buffer
                again = true;
                cause |= 4u;
                say("rows", L + 1, nr[1], c->lvb[L + 1].cap);
                cut *= std::max<double>(1.0, (double)nr[1] / (double)std::max<uint64_t>(1, c->lvb[L + 1].cap));
            }
        }
    }
    return again;
}

// Whether sort_outputs finds every scratch buffer it needs already allocated.
bool sort_fits(const mnemonic_ctx* c) {
    for (uint32_t q = 0; q < c->n_q; q++)
        for (int p = 0; p < 2; p++) {
            const uint64_t n = std::min<uint64_t>(c->h_zr[c->zr_count(p) + q], c->houts[q].cap[p]);
            if (n <= 1) continue;
            if (n > c->cap_srt || n * c->hq[q].n_qe > c->cap_srt_rows ||
                mn_tuple_sort_scratch_words((uint32_t)n) > c->cap_srt_scr)
                return false;
        }
    return true;
}

// Puts every query's result tuples of both phases in lexicographic order.
void sort_outputs(mnemonic_ctx* c) {
    hipStream_t s = c->stream;
    const uint32_t key_bits = std::max<uint32_t>(1, ceil_log2(c->next_key + 1));
    for (uint32_t q = 0; q < c->n_q; q++)
        for (int p = 0; p < 2; p++) {
            const uint64_t n = std::min<uint64_t>(c->h_zr[c->zr_count(p) + q], c->houts[q].cap[p]);
            if (n <= 1) continue;
            if (n >= (1ull << 32)) throw ApiError{MNEMONIC_E_LIMIT, "more than 2^32 tuples to sort"};
            const uint32_t m = c->hq[q].n_qe;
            if (n > c->cap_srt) {
                for (int k = 0; k < 2; k++) {
                    dev_free(c->d_srt_k[k]);
                    dev_free(c->d_srt_v[k]);
                }
                c->cap_srt = 0;
                const uint64_t nc = 2 * n;
                for (int k = 0; k < 2; k++) {
                    dev_alloc(c->d_srt_k[k], nc);
                    dev_alloc(c->d_srt_v[k], nc);
                }
                c->cap_srt = nc;
            }
            if (n * m > c->cap_srt_rows) {
                dev_free(c->d_srt_rows);
                c->cap_srt_rows = 0;
                dev_alloc(c->d_srt_rows, 2 * n * m);
                c->cap_srt_rows = 2 * n * m;
            }
            const uint64_t sw = mn_tuple_sort_scratch_words((uint32_t)n);
            if (sw > c->cap_srt_scr) {
                dev_free(c->d_srt_scr);
                c->cap_srt_scr = 0;
                dev_alloc(c->d_srt_scr, 2 * sw);
                c->cap_srt_scr = 2 * sw;
            }
            mn_sort_tuples(c->houts[q].keys[p], (uint32_t)n, m, key_bits, c->d_srt_k[0], c->d_srt_k[1], c->d_srt_v[0],
                           c->d_srt_v[1], c->d_srt_rows, c->d_srt_scr, s);
        }
    HIPCHK(hipGetLastError());
}

// One snapshot; `enumerate` is false only for the initial load.
int run_batch(mnemonic_ctx* c, uint64_t n_ins, const uint32_t* src, const uint32_t* dst,
              const uint8_t* lab, const int64_t* ts, const uint64_t* del_keys, uint64_t n_del,
              bool on_device, bool enumerate, uint64_t* first_new_key) {
    hipStream_t s = c->stream;
    if (n_ins + n_del >= (1ull << 31)) throw ApiError{MNEMONIC_E_ARG, "batch too large"};
    t_alloc_n = 0;
    t_alloc_ms = 0;
    ensure_capacity(c, n_ins, n_del);
    static const uint32_t kItems[3] = {2, 4, 8};
    const bool tune = enumerate && c->tuning() && !t_no_alloc;
    if (tune) c->tile_items = kItems[c->tune_batch % 3];
    const bool timing = (c->flags & (MNEMONIC_F_TIMING | MNEMONIC_F_AUTOTUNE)) != 0 && enumerate && !t_no_alloc;
    for (int p = 0; p < 2; p++) {
        c->ms_expand[p] = 0;
        c->n_expand[p] = 0;
        c->reruns[p] = c->rerun_causes[p] = 0;
    }
    c->ev_used = 0;
    if (timing) HIPCHK(hipEventRecord(c->ev[4], s));

    const uint32_t* in_src = src;
    const uint32_t* in_dst = dst;
    const uint8_t* in_lab = lab;
    const int64_t* in_ts = ts;
    const uint64_t* dk = del_keys;
    if (!on_device) {
        if (n_ins) {
            HIPCHK(hipMemcpyAsync(c->d_in_src, src, n_ins * 4, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(c->d_in_dst, dst, n_ins * 4, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(c->d_in_lab, lab, n_ins, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(c->d_in_ts, ts, n_ins * 8, hipMemcpyHostToDevice, s));
        }
        if (n_del) HIPCHK(hipMemcpyAsync(c->d_del_keys, del_keys, n_del * 8, hipMemcpyHostToDevice, s));
        in_src = c->d_in_src;
        in_dst = c->d_in_dst;
        in_lab = c->d_in_lab;
        in_ts = c->d_in_ts;
        dk = c->d_del_keys;
    }
    const int pend = c->pend, cur = 1 - c->pend;
    const uint32_t n_prev = (uint32_t)c->n_pending;
    BatchView b;
    memset(&b, 0, sizeof(b));
    b.n_ins = (uint32_t)n_ins;
    b.n_del = (uint32_t)n_del;
    b.n_prev_del = n_prev;
    b.n_free = c->n_free;
    b.fresh = c->fresh;
    b.hb = c->hb;
    const uint64_t dirbit = 1ull << (c->hb + c->nbr_bits);  // direction bit of the batch sort keys
    b.dirbit = dirbit;
    b.next_key = c->next_key;
    b.key_lo = c->key_lo;
    b.key_mask = c->cap_keys - 1;
    b.n_elabels = c->n_elabels;
    b.n_debi_bits = c->n_debi_bits;
    b.n_vf_bits = c->n_vf_bits;
    b.in_src = in_src;
    b.in_dst = in_dst;
    b.in_lab = in_lab;
    b.in_ts = in_ts;
    b.del_keys = dk;
    b.free_stack = c->d_free;
    b.key2slot = c->d_key2slot;
    b.delbits = c->d_delbits;
    b.err = c->d_err;
    b.last_ts = c->d_last_ts;
    b.ins_slot = c->d_ins_slot;
    for (int d = 0; d < 2; d++) {
        b.skey[d] = c->d_skey[0] + d * n_ins;
        b.sval[d] = c->d_sval[0] + d * n_ins;
        b.delpos[d] = c->d_delpos[cur][d];
    }
    b.touched = c->d_touched;
    b.prev_del_slot = c->d_del_slot[pend];
    b.del_slot = c->d_del_slot[cur];
    b.debi_bits = c->d_debi_bits;
    b.vf_bits = c->d_vf_bits;

    if (enumerate && (c->flags & MNEMONIC_F_EMIT) && !(c->flags & MNEMONIC_F_INDEX_ONLY) && !t_no_alloc) {
        // outputs sized for this batch at the largest per-edge rates seen,
        // with a margin; at most 4x per batch, so one unusual batch cannot
        // claim a large share of the device
        std::vector<uint64_t> want(2 * (size_t)c->n_q, 0);
        for (uint32_t q = 0; q < c->n_q; q++)
            for (int p = 0; p < 2; p++) {
                const double r = c->out_rate[2 * (size_t)q + p];
                if (r <= 0) continue;
                const double est = 1.5 * r * (double)(p ? n_del : n_ins);
                const double most = 2.0 * (double)c->out_max[2 * (size_t)q + p] + 65536.0;
                want[2 * (size_t)q + p] =
                    (uint64_t)std::min<double>(std::min<double>(est, most), 4.0 * (double)c->houts[q].cap[p]);
            }
        grow_outputs(c, want);
    }
    GraphView g0 = make_view(c, false);
    // From the first launch on, a failure other than the validation's leaves
    // the graph, its index or the results part way through the batch: the
    // context stays unusable unless the batch completes (or validation
    // rejects it, which changes nothing: every kernel after the validation
    // does no work once the error word is set).
    if (enumerate) {
        c->broken = true;
        c->broken_why = "a batch";
        c->results_incomplete = false;
    }
    mn_launch_reset(c->d_err, c->d_zr, c->n_zr, s);
    if (c->tr_cap) {  // the trace holds this batch's start rows only
        mn_launch_set_u32(c->d_tr_n, 0, s);
        mn_launch_set_u32(c->d_tr_n + 1, 0, s);
    }
    mn_launch_validate(g0, b, s);
    mn_launch_prev_del(g0, b, s);
    mn_launch_ingest(g0, b, s);

    const bool merge = n_ins > 0 || n_prev > 0;
    const uint64_t E_new = c->E - n_prev + n_ins;
    if (merge) {
        // one sort of the batch entries of both directions (the direction bit
        // on top keeps them apart) and one of the pending deletion positions
        uint64_t* bk = c->d_skey[0];
        uint32_t* bv = c->d_sval[0];
        uint64_t* tk = c->d_skey[1];
        uint32_t* tv = c->d_sval[1];
        mn_radix_sort(bk, bv, tk, tv, (uint32_t)(2 * n_ins), c->hb + c->nbr_bits + 1, c->d_sort_scratch, s);
        const uint64_t dbit = 1ull << c->hb_pos;
        uint64_t* dk = c->d_dkey[0];
        if (n_prev) {
            uint32_t* v0 = c->d_dval[0];
            uint64_t* k1 = c->d_dkey[1];
            uint32_t* v1 = c->d_dval[1];
            mn_launch_widen(c->d_delpos[pend][0], dk, 0, c->d_delpos[pend][1], dk + n_prev, dbit, n_prev, c->d_err,
                            s);
            mn_radix_sort(dk, v0, k1, v1, 2 * n_prev, c->hb_pos + 1, c->d_sort_scratch, s);
        }
        MergeSide side[2];
        for (int d = 0; d < 2; d++) {
            MergeSide& m = side[d];
            m.off = c->d_off[d];
            m.adj = c->d_adj[d];
            m.adjk = c->d_adjk[d];
            m.bk = bk + d * n_ins;
            m.kbase = d ? dirbit : 0;
            m.bv = bv + d * n_ins;
            m.dpos = n_prev ? dk + d * n_prev : nullptr;
            m.dbase = d ? dbit : 0;
            m.newoff = c->d_off2[d];
            m.meta = c->d_meta[d];
            m.adj_new = c->d_adj2[d];
            m.adjk_new = c->d_adjk2[d];
            m.inspos = c->d_inspos[d];
            m.ub = c->d_ub[d];
            m.lim = c->d_mlim + d * mn_merge_limit_words(c->E);
        }
        mn_launch_merge(side, c->nV, (uint32_t)c->E, c->d_key, (uint32_t)n_ins, n_prev, c->hb, (uint32_t)E_new,
                        c->d_err, s);
    }
    // from here on the kernels work on the merged adjacency
    GraphView g1 = make_view(c, merge);
    mn_launch_vf_refresh(g1, c->d_vf_bits, c->n_vf_bits, enumerate ? c->d_touched : nullptr,
                         enumerate ? (uint32_t)(2 * (n_prev + n_ins)) : c->nV, c->d_err, s);
    if (enumerate && c->tree_on() && !(c->flags & MNEMONIC_F_INDEX_ONLY)) {
        // the spanning-tree filter on G with the batch's insertions (both
        // phases enumerate on it): VF, then the rounds
        HIPCHK(hipMemcpyAsync(c->d_vfp, c->d_vf, (size_t)c->nV * c->vf_words * 4, hipMemcpyDeviceToDevice, s));
        for (size_t i = 0; i + 1 < c->tree_round.size(); i++)
            mn_launch_tree_step(g1, c->d_vfp, c->d_tree + c->tree_round[i], c->tree_round[i + 1] - c->tree_round[i],
                                c->nV, c->d_zr + c->zr_tree(), c->d_err, s);
    }
    uint64_t* adjn[2] = {merge ? c->d_adj2[0] : c->d_adj[0], merge ? c->d_adj2[1] : c->d_adj[1]};
    // the enumerator reads the current view; point it at the merged arrays
    auto swap_in = [&]() {
        if (!merge) return;
        for (int d = 0; d < 2; d++) {
            std::swap(c->d_adj[d], c->d_adj2[d]);
            std::swap(c->d_adjk[d], c->d_adjk2[d]);
            std::swap(c->d_off[d], c->d_off2[d]);
        }
    };
    swap_in();
    uint32_t err = 0;
    const bool enum_on = enumerate && !(c->flags & MNEMONIC_F_INDEX_ONLY);
    try {
        if (enum_on) enumerate_phase(c, 0, c->d_ins_slot, n_ins);
        mn_launch_set_flags(adjn[0], c->d_inspos[0], adjn[1], c->d_inspos[1], (uint32_t)n_ins, 0, c->d_err, s);
        GraphView g2 = make_view(c, false);
        mn_launch_flag_del(g2, adjn[0], adjn[1], b, s);
        if (enum_on) enumerate_phase(c, 1, c->d_del_slot[cur], n_del);
        uint32_t n_free_after = c->n_free - (uint32_t)std::min<uint64_t>(n_ins, c->n_free);
        mn_launch_finalize(b, n_free_after, s);
        mn_launch_advance_lo(c->d_key2slot, c->cap_keys - 1, c->d_key_lo, c->next_key + n_ins, c->d_err, s);
        if (timing) HIPCHK(hipEventRecord(c->ev[5], s));
        read_zr(c, &err);
        c->summarize();
    } catch (...) {
        swap_in();  // a swap is its own inverse: back to the pre-batch arrays
        throw;
    }
    if (err) {
        swap_in();
        c->broken = false;  // nothing changed
        switch (err) {
            case MN_ERR_VERTEX: throw ApiError{MNEMONIC_E_VERTEX, "edge endpoint >= n_vertices"};
            case MN_ERR_LABEL: throw ApiError{MNEMONIC_E_LABEL, "edge label >= n_elabels"};
            case MN_ERR_TS: throw ApiError{MNEMONIC_E_TS_ORDER, "timestamps decrease"};
            case MN_ERR_DELETE: throw ApiError{MNEMONIC_E_BAD_DELETE, "deletion key not live or repeated"};
            default: throw ApiError{MNEMONIC_E_HIP, "internal consistency check failed on the device"};
        }
    }
    // commit the host mirrors
    if (first_new_key) *first_new_key = c->next_key;
    uint32_t took = (uint32_t)std::min<uint64_t>(n_ins, c->n_free);
    c->fresh += (uint32_t)(n_ins - took);
    c->n_free = c->n_free - took + (uint32_t)n_del;
    c->next_key += n_ins;
    c->key_lo = c->key_lo_seen;
    c->n_live = c->n_live + n_ins - n_del;
    c->E = E_new;
    c->n_pending = n_del;
    c->pend = cur;

    if (enum_on) {
        // outputs too small, or a level's buffers too small: grow and
        // enumerate the phase again on the same state (the flags of the
        // phase being re-run are restored first)
        bool emit = (c->flags & MNEMONIC_F_EMIT) != 0;
        bool host_chunks[2] = {false, false};
        // A device-sized run that overflows leaves notes that size the next
        // one; which rows a truncated level kept depends on atomic order, so
        // the estimates converge in a few runs but without a fixed bound.
        // After DEVICE_RUNS of them a phase is walked in host-sized chunks,
        // which completes in one run; one more run may follow to grow
        // outputs to the exact counts.
        constexpr int DEVICE_RUNS = 3;
        const int max_attempts = DEVICE_RUNS + 3;
        for (int attempt = 0; attempt < max_attempts; attempt++) {
            std::vector<uint64_t> need(2 * c->n_q, 0);
            bool redo[2] = {false, false};
            std::string why;
            const bool last = attempt == max_attempts - 1;
            uint64_t cause[2] = {0, 0};
            for (int p = 0; p < 2; p++) {
                redo[p] = absorb_notes(c, p, host_chunks[p], cause[p], last ? &why : nullptr);
                if (redo[p] && attempt + 1 >= DEVICE_RUNS) host_chunks[p] = true;
            }
            for (uint32_t q = 0; q < c->n_q; q++)
                for (int p = 0; p < 2; p++) {
                    need[2 * q + p] = c->h_zr[c->zr_count(p) + q];
                    if (emit && need[2 * q + p] > c->houts[q].cap[p]) {
                        redo[p] = true;
                        cause[p] |= 8u;
                        if (last) why += " [query " + std::to_string(q) + " output " + std::to_string(need[2 * q + p]) + "]";
                    }
                }
            if (t_no_alloc && (redo[0] || redo[1])) {
                // No buffer may grow in this call. Levels that outgrew theirs
                // are walked again in chunks the buffers hold; output lists that
                // are too small cannot be helped: the batch stands, its results
                // are incomplete.
                bool fits = (cause[0] | cause[1]) & 8u ? false : true;
                for (int p = 0; p < 2 && fits; p++)
                    if (redo[p] && c->max_levels && c->lvb[0].cap < c->n_static) fits = false;
                if (!fits) {
                    c->results_incomplete = true;
                    for (int p = 0; p < 2; p++) c->rerun_causes[p] |= cause[p];
                    break;
                }
                for (int p = 0; p < 2; p++) host_chunks[p] = host_chunks[p] || redo[p];
            }
            for (int p = 0; p < 2; p++)
                if (redo[p]) {
                    c->reruns[p]++;
                    c->rerun_causes[p] |= cause[p];
                }
            if (!redo[0] && !redo[1]) break;
            if (last) throw ApiError{MNEMONIC_E_HIP, "enumeration did not settle (internal)" + why};
            if (!t_no_alloc) grow_outputs(c, need);
            if (redo[0]) {
                // per direction: deletion flags cleared before insertion flags are set
                mn_launch_set_flags(c->d_adj[0], c->d_delpos[cur][0], c->d_adj[1], c->d_delpos[cur][1],
                                    (uint32_t)n_del, 0, c->d_err, s);
                mn_launch_set_flags(c->d_adj[0], c->d_inspos[0], c->d_adj[1], c->d_inspos[1], (uint32_t)n_ins, 1,
                                    c->d_err, s);
                reset_phase(c, 0);
                enumerate_phase(c, 0, c->d_ins_slot, n_ins, host_chunks[0]);
                mn_launch_set_flags(c->d_adj[0], c->d_inspos[0], c->d_adj[1], c->d_inspos[1], (uint32_t)n_ins, 0,
                                    c->d_err, s);
                mn_launch_set_flags(c->d_adj[0], c->d_delpos[cur][0], c->d_adj[1], c->d_delpos[cur][1],
                                    (uint32_t)n_del, 1, c->d_err, s);
            }
            if (redo[1]) {
                reset_phase(c, 1);
                enumerate_phase(c, 1, c->d_del_slot[cur], n_del, host_chunks[1]);
            }
            read_zr(c, nullptr);
            c->summarize();
        }
        if (emit && (c->flags & MNEMONIC_F_SORT) && !c->results_incomplete) {
            if (t_no_alloc && !sort_fits(c)) {
                c->results_incomplete = true;
            } else {
                sort_outputs(c);
                HIPCHK(hipStreamSynchronize(s));
            }
        }
        if (timing) resolve_events(c);
        if (tune) {
            const uint32_t k = c->tune_batch % 3;
            c->tune_ms[k] += c->ms_expand[0] + c->ms_expand[1];
            c->tune_cand[k] += (double)(c->sum_st[0][1] + c->sum_st[1][1]);
            if (++c->tune_batch == 3 * mnemonic_ctx::TUNE_TRIALS) {
                int best = 1;
                double best_cost = 1e300;
                for (int i = 0; i < 3; i++) {
                    const double cost = c->tune_cand[i] > 0 ? c->tune_ms[i] / c->tune_cand[i] : 1e300;
                    if (cost < best_cost) {
                        best_cost = cost;
                        best = i;
                    }
                }
                c->tile_items = kItems[best];
            }
        }
        // output rates of this batch for the next one
        for (uint32_t q = 0; q < c->n_q; q++)
            for (int p = 0; p < 2; p++) {
                const uint64_t ne = p ? n_del : n_ins;
                const uint64_t n = c->h_zr[c->zr_count(p) + q];
                double& r = c->out_rate[2 * (size_t)q + p];
                if (ne) r = std::max<double>(r, (double)n / (double)ne);
                c->out_max[2 * (size_t)q + p] = std::max<uint64_t>(c->out_max[2 * (size_t)q + p], n);
            }
        // rates of this batch for the next one (levels that saw candidates)
        for (int p = 0; p < 2; p++) {
            const double ns = (double)std::max<uint64_t>(1, c->chunk_ns[p]);
            for (uint32_t L = 0; L <= MN_MAXLV; L++) {
                if (L < MN_MAXLV && L >= c->max_levels) continue;
                // the largest rate seen: batch sizes and hub hits vary, an
                // estimate that falls short costs a re-run of the phase, and a
                // generous one only idle blocks
                const uint64_t T = c->h_zr[L < MN_MAXLV ? c->note_cand(p, L) + 1 : c->note_seed(p) + 1];
                if (T) c->rate[p][L] = std::max<double>((double)T / ns, c->rate[p][L]);
                // rows of level L (noted when level L's ranges were taken)
                if (L >= 1 && L < c->max_levels) {
                    const uint64_t R = c->h_zr[c->note_rows(p, L - 1) + 1];
                    if (R) c->row_rate[p][L] = std::max<double>((double)R / ns, c->row_rate[p][L]);
                }
            }
        }
        // stats
        mnemonic_stats& st = c->stats;
        st.n_live_edges = c->n_live;
        st.slot_high_water = c->fresh;
        for (int p = 0; p < 2; p++) {
            const uint64_t* z = c->sum_st[p];
            st.seeds[p] = z[0];
            st.entries_scanned[p] = z[1];
            st.probe_words[p] = z[2];
            st.range_probe_words[p] = z[3];
            st.key_reads[p] = z[4];
            st.tuples[p] = z[5];
            st.vf_reads[p] = z[6];
            st.frontier_rows[p] = z[7];
            st.vf_rejects[p] = z[8];
            st.expand_launches[p] = c->n_expand[p];
            st.reruns[p] = c->reruns[p];
            st.rerun_causes[p] = c->rerun_causes[p];
            st.expand_tile = (uint64_t)MN_BLOCK * c->tile_items;
            st.ms_expand[p] = c->ms_expand[p];
            uint64_t words = 0;
            for (uint32_t q = 0; q < c->n_q; q++) words += c->h_zr[c->zr_count(p) + q] * c->hq[q].n_qe;
            st.tuple_words[p] = words;
        }
        if (timing) {
            float ms = 0;
            for (int p = 0; p < 2; p++) {
                HIPCHK(hipEventElapsedTime(&ms, c->ev[2 * p], c->ev[2 * p + 1]));
                st.ms_enumerate[p] = ms;
            }
            HIPCHK(hipEventElapsedTime(&ms, c->ev[4], c->ev[5]));
            st.ms_batch = ms;
        }
        c->have_result = true;
    }
    c->stats.allocations = t_alloc_n;
    c->stats.ms_alloc = t_alloc_ms;
    c->stats.tree_cleared = c->h_zr[c->zr_tree()];
    c->broken = false;
    if (c->results_incomplete)
        throw ApiError{MNEMONIC_E_CAPACITY, "batch applied, but its enumeration needs larger buffers than the context "
                                            "holds (causes " + std::to_string(c->rerun_causes[0]) + ", " +
                                            std::to_string(c->rerun_causes[1]) + "): its results are unavailable"};
    return MNEMONIC_OK;
}

// Points the context's per-batch control words into the device's scratch
// array for the duration of a no-allocation call, and back afterwards.
struct ScratchSwap {
    mnemonic_ctx* c;
    unsigned long long* zr;
    uint32_t* err;
    uint32_t* nrows;
    uint64_t* total;
    uint32_t* dec_n;
    static uint64_t words(const mnemonic_ctx* c) { return c->n_zr + 1 + (MN_MAXLV + 2 + 1) / 2 + 1 + 1; }
    ScratchSwap(mnemonic_ctx* c_, uint64_t* w) : c(c_), zr(c_->d_zr), err(c_->d_err), nrows(c_->d_nrows),
                                                 total(c_->d_total), dec_n(c_->d_dec_n) {
        c->d_zr = reinterpret_cast<unsigned long long*>(w);
        w += c->n_zr;
        c->d_err = reinterpret_cast<uint32_t*>(w);
        w += 1;
        c->d_nrows = reinterpret_cast<uint32_t*>(w);
        w += (MN_MAXLV + 2 + 1) / 2;
        c->d_total = w;
        w += 1;
        c->d_dec_n = reinterpret_cast<uint32_t*>(w);
    }
    ~ScratchSwap() {
        c->d_zr = zr;
        c->d_err = err;
        c->d_nrows = nrows;
        c->d_total = total;
        c->d_dec_n = dec_n;
    }
};

template <typename F>
int guarded(mnemonic_ctx* c, F&& f) {
    try {
        if (c && c->broken) {
            c->err = "context unusable: " + c->broken_why + " failed part way; destroy it";
            return MNEMONIC_E_HIP;
        }
        if (c) {
            c->err.clear();
            t_stream = c->stream;
        }
        return f();
    } catch (const ApiError& e) {
        if (c) c->err = e.msg;
        else g_create_error = e.msg;
        return e.code;
    } catch (const HipError& e) {
        std::string m = std::string(e.what) + ": " + hipGetErrorString(e.e);
        if (c) c->err = m;
        else g_create_error = m;
        return MNEMONIC_E_HIP;
    } catch (const std::bad_alloc&) {
        if (c) c->err = "host allocation failed";
        else g_create_error = "host allocation failed";
        return MNEMONIC_E_OOM;
    }
}

void free_all(mnemonic_ctx* c) {
    dev_free(c->d_vmask);
    dev_free(c->d_q);
    dev_free(c->d_plans);
    dev_free(c->d_debi_bits);
    dev_free(c->d_vf_bits);
    dev_free(c->d_req);
    dev_free(c->d_elab_idx);
    dev_free(c->d_vlab_idx);
    dev_free(c->d_vf);
    dev_free(c->d_vfp);
    dev_free(c->d_tree);
    dev_free(c->d_cnt);
    dev_free(c->d_meta[0]);
    dev_free(c->d_meta[1]);
    dev_free(c->d_src);
    dev_free(c->d_dst);
    dev_free(c->d_lab);
    dev_free(c->d_ts);
    dev_free(c->d_key);
    dev_free(c->d_debi);
    dev_free(c->d_free);
    dev_free(c->d_key2slot);
    dev_free(c->d_key_ts);
    dev_free(c->d_delbits);
    dev_free(c->d_key_lo);
    for (int k = 0; k < 2; k++) {
        dev_free(c->d_skey[k]);
        dev_free(c->d_sval[k]);
        dev_free(c->d_dkey[k]);
        dev_free(c->d_dval[k]);
    }
    for (int d = 0; d < 2; d++) {
        dev_free(c->d_off[d]);
        dev_free(c->d_off2[d]);
        dev_free(c->d_adj[d]);
        dev_free(c->d_adj2[d]);
        dev_free(c->d_adjk[d]);
        dev_free(c->d_adjk2[d]);
        dev_free(c->d_inspos[d]);
        dev_free(c->d_ub[d]);
        dev_free(c->d_del_slot[d]);
        for (int k = 0; k < 2; k++) dev_free(c->d_delpos[d][k]);
    }
    dev_free(c->d_mlim);
    dev_free(c->d_in_src);
    dev_free(c->d_in_dst);
    dev_free(c->d_in_lab);
    dev_free(c->d_in_ts);
    dev_free(c->d_del_keys);
    dev_free(c->d_ins_slot);
    dev_free(c->d_touched);
    dev_free(c->d_sort_scratch);
    dev_free(c->d_err);
    dev_free(c->d_last_ts);
    dev_free(c->d_zr);
    for (auto& o : c->houts)
        for (int p = 0; p < 2; p++) dev_free(o.keys[p]);
    dev_free(c->d_outs);
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : c->ev_x)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : c->ev_pool)
        if (e) (void)hipEventDestroy(e);
    dev_free(c->d_tiles);
    for (auto& B : c->lvb) {
        dev_free(B.keys);
        dev_free(B.rows);
        dev_free(B.lo);
        dev_free(B.cnt);
        dev_free(B.off);
        dev_free(B.hpre);
    }
    dev_free(c->d_scan64);
    dev_free(c->d_nrows);
    dev_free(c->d_total);
    dev_free(c->d_ext2int);
    dev_free(c->d_sched_w);
    dev_free(c->d_sched_f32);
    dev_free(c->d_tr_n);
    dev_free(c->d_tr_code);
    dev_free(c->d_tr_x);
    dev_free(c->d_tr_work);
    dev_free(c->d_dec);
    dev_free(c->d_dec_n);
    for (int k = 0; k < 2; k++) {
        dev_free(c->d_srt_k[k]);
        dev_free(c->d_srt_v[k]);
    }
    dev_free(c->d_srt_rows);
    dev_free(c->d_srt_scr);
    if (c->h_ctl) (void)hipHostFree(c->h_ctl);
    c->h_ctl = nullptr;
    if (c->h_zr_pin) (void)hipHostFree(c->h_zr_pin);
    c->h_zr_pin = nullptr;
    c->cap_zr_pin = 0;
}

}  // namespace

extern "C" {

int mnemonic_create(const mnemonic_graph* g, const mnemonic_query* q, uint32_t n_q,
                    const mnemonic_options* opt, void* hip_stream, mnemonic_ctx** out) {
    g_create_error.clear();
    if (!g || !q || !out) {
        g_create_error = "NULL argument";
        return MNEMONIC_E_ARG;
    }
    mnemonic_ctx* c = new (std::nothrow) mnemonic_ctx();
    if (!c) return MNEMONIC_E_OOM;
    memset(&c->stats, 0, sizeof(c->stats));
    int rc = guarded(nullptr, [&]() -> int {
        if (g->n_vertices == 0 || (g->n_edges && (!g->src || !g->dst || !g->elabel || !g->ts)) || !g->vlabel_mask)
            throw ApiError{MNEMONIC_E_ARG, "graph arrays must not be NULL and n_vertices must be > 0"};
        if (g->n_vertices > (1u << 24)) throw ApiError{MNEMONIC_E_LIMIT, "n_vertices > 2^24"};
        if (g->n_elabels > 256) throw ApiError{MNEMONIC_E_ARG, "n_elabels > 256"};
        HIPCHK(hipGetDevice(&c->device));
        setup_scratch(c->device);
        setup_pool(c->device);
        c->stream = static_cast<hipStream_t>(hip_stream);
        t_stream = c->stream;
        if (opt) c->flags = opt->flags;
        // at most 2^26 rows per level: the kernels index a level's columns in 32 bits
        if (opt && opt->rows_per_level)
            c->rows_max = std::min<uint64_t>(1ull << 26, std::max<uint64_t>(1024, opt->rows_per_level));
        c->nV = g->n_vertices;
        c->n_elabels = g->n_elabels ? g->n_elabels : 256;
        c->nbr_bits = std::max<uint32_t>(1, ceil_log2(c->nV));
        c->hb = c->nbr_bits + std::max<uint32_t>(1, ceil_log2(c->n_elabels));
        // vertex classes (distinct label sets, ascending) and internal ids
        // assigned class by class, caller's order within a class
        std::vector<uint32_t> order(c->nV);
        for (uint32_t v = 0; v < c->nV; v++) order[v] = v;
        std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
            return g->vlabel_mask[a] < g->vlabel_mask[b];
        });
        std::vector<uint32_t> ext2int(c->nV);
        std::vector<uint64_t> vmask_int(c->nV);
        for (uint32_t i = 0; i < c->nV; i++) {
            const uint64_t m = g->vlabel_mask[order[i]];
            ext2int[order[i]] = i;
            vmask_int[i] = m;
            if (c->cls_mask.empty() || c->cls_mask.back() != m) {
                c->cls_mask.push_back(m);
                c->cls_start.push_back(i);
            }
        }
        c->cls_start.push_back(c->nV);
        c->lab_deg.assign(257, 0.0);
        for (uint64_t e = 0; e < g->n_edges; e++) c->lab_deg[g->elabel[e]] += 1.0;
        c->lab_deg[256] = (double)g->n_edges;
        for (double& d : c->lab_deg) d /= (double)c->nV;
        prepare_queries(c, q, n_q);
        c->tile_items = default_tile_items(c->max_close);
        for (uint32_t i = 0; i < n_q; i++)
            for (uint32_t k = 0; k < q[i].n_qe; k++)
                if (q[i].qelabel[k] >= (int32_t)c->n_elabels)
                    throw ApiError{MNEMONIC_E_QUERY, "query edge label >= n_elabels"};
        hipStream_t s = c->stream;
        for (auto& e : c->ev) HIPCHK(hipEventCreate(&e));
        dev_alloc(c->d_vmask, c->nV);
        HIPCHK(hipMemcpyAsync(c->d_vmask, vmask_int.data(), (size_t)c->nV * 8, hipMemcpyHostToDevice, s));
        dev_alloc(c->d_ext2int, c->nV);
        HIPCHK(hipMemcpyAsync(c->d_ext2int, ext2int.data(), (size_t)c->nV * 4, hipMemcpyHostToDevice, s));
        c->lvb.resize(c->max_levels);
        for (int p = 0; p < 2; p++)
            for (int L = 0; L <= MN_MAXLV; L++) c->rate[p][L] = c->row_rate[p][L] = -1.0;  // unknown: size by capacity
        dev_alloc(c->d_nrows, MN_MAXLV + 2);
        dev_alloc(c->d_dec_n, 1);
        dev_alloc(c->d_total, 1);
        HIPCHK(hipHostMalloc((void**)&c->h_ctl, 64, hipHostMallocDefault));
        for (auto& e : c->ev_x) HIPCHK(hipEventCreate(&e));
        upload(c->d_q, c->hq, s);
        upload(c->d_plans, c->hplans, s);
        upload(c->d_debi_bits, c->hdebi, s);
        upload(c->d_vf_bits, c->hvf, s);
        upload(c->d_req, c->hreq, s);
        dev_alloc(c->d_elab_idx, 256);
        dev_alloc(c->d_vlab_idx, 64);
        HIPCHK(hipMemcpyAsync(c->d_elab_idx, c->elab_idx, sizeof(c->elab_idx), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(c->d_vlab_idx, c->vlab_idx, sizeof(c->vlab_idx), hipMemcpyHostToDevice, s));
        dev_alloc(c->d_vf, (size_t)c->nV * c->vf_words);
        dev_alloc(c->d_cnt, (size_t)c->nV * c->n_cnt);
        mn_launch_init_vertices(c->d_vf, c->d_cnt, c->nV, c->vf_words, c->n_cnt, s);
        if (c->tree_on()) {
            upload(c->d_tree, c->htree, s);
            dev_alloc(c->d_vfp, (size_t)c->nV * c->vf_words);
        }
        dev_alloc(c->d_meta[0], c->nV);
        dev_alloc(c->d_meta[1], c->nV);
        for (int d = 0; d < 2; d++) {
            dev_alloc(c->d_off[d], (size_t)c->nV + 1);
            dev_alloc(c->d_off2[d], (size_t)c->nV + 1);
            HIPCHK(hipMemsetAsync(c->d_off[d], 0, ((size_t)c->nV + 1) * 4, s));
        }
        dev_alloc(c->d_err, 1);
        dev_alloc(c->d_last_ts, 1);
        dev_alloc(c->d_key_lo, 1);
        HIPCHK(hipMemsetAsync(c->d_key_lo, 0, 8, s));
        int64_t mn = INT64_MIN;
        HIPCHK(hipMemcpyAsync(c->d_last_ts, &mn, 8, hipMemcpyHostToDevice, s));
        c->n_zr = c->zr_words();
        c->h_zr.assign(c->n_zr, 0);
        size_zr_pin(c);
        dev_alloc(c->d_zr, c->n_zr);
        // output buffers
        uint64_t cap = opt && opt->out_capacity ? opt->out_capacity : (1ull << 20);
        c->out_cap0 = cap;
        c->houts.resize(n_q);
        c->out_rate.assign(2 * (size_t)n_q, -1.0);
        c->out_max.assign(2 * (size_t)n_q, 0);
        for (uint32_t i = 0; i < n_q; i++)
            for (int p = 0; p < 2; p++) {
                c->houts[i].cap[p] = (c->flags & MNEMONIC_F_EMIT) ? cap : 0;
                c->houts[i].keys[p] = nullptr;
                if (c->flags & MNEMONIC_F_EMIT) dev_alloc(c->houts[i].keys[p], cap * c->hq[i].n_qe);
            }
        dev_alloc(c->d_outs, n_q);
        HIPCHK(hipMemcpyAsync(c->d_outs, c->houts.data(), n_q * sizeof(OutView), hipMemcpyHostToDevice, s));
        // initial graph: the same ingest/merge path without enumeration
        run_batch(c, g->n_edges, g->src, g->dst, g->elabel, g->ts, nullptr, 0, false, false, nullptr);
        HIPCHK(hipStreamSynchronize(s));
        return MNEMONIC_OK;
    });
    if (rc != MNEMONIC_OK) {
        free_all(c);
        delete c;
        return rc;
    }
    *out = c;
    return MNEMONIC_OK;
}

int mnemonic_apply_batch(mnemonic_ctx* ctx, const mnemonic_edges* ins, const uint64_t* del_keys,
                         uint64_t n_del, uint64_t* first_new_key) {
    if (!ctx) return MNEMONIC_E_ARG;
    return guarded(ctx, [&]() -> int {
        uint64_t n_ins = ins ? ins->n : 0;
        if (n_ins && (!ins->src || !ins->dst || !ins->elabel || !ins->ts))
            throw ApiError{MNEMONIC_E_ARG, "insertion arrays must not be NULL"};
        if (n_del && !del_keys) throw ApiError{MNEMONIC_E_ARG, "del_keys must not be NULL"};
        bool dev = ins && ins->on_device;
        return run_batch(ctx, n_ins, ins ? ins->src : nullptr, ins ? ins->dst : nullptr,
                         ins ? ins->elabel : nullptr, ins ? ins->ts : nullptr, del_keys, n_del, dev, true,
                         first_new_key);
    });
}

int mnemonic_apply_batch_noalloc(mnemonic_ctx* ctx, const mnemonic_edges* ins, const uint64_t* del_keys,
                                 uint64_t n_del, uint64_t* first_new_key) {
    if (!ctx) return MNEMONIC_E_ARG;
    return guarded(ctx, [&]() -> int {
        uint64_t n_ins = ins ? ins->n : 0;
        if (n_ins && (!ins->src || !ins->dst || !ins->elabel || !ins->ts))
            throw ApiError{MNEMONIC_E_ARG, "insertion arrays must not be NULL"};
        if (n_del && !del_keys) throw ApiError{MNEMONIC_E_ARG, "del_keys must not be NULL"};
        uint64_t* w = scratch_of(ctx->device);
        if (!w) throw ApiError{MNEMONIC_E_HIP, "the device's no-allocation scratch is not set up"};
        const uint64_t need = ScratchSwap::words(ctx);
        if (need > MN_NOALLOC_WORDS)
            throw ApiError{MNEMONIC_E_CAPACITY, "the query set's control block (" + std::to_string(need) +
                                                    " words) exceeds the no-allocation scratch (" +
                                                    std::to_string(MN_NOALLOC_WORDS) + " words)"};
        ScratchSwap swap(ctx, w);
        NoAllocScope no_alloc;
        bool dev = ins && ins->on_device;
        return run_batch(ctx, n_ins, ins ? ins->src : nullptr, ins ? ins->dst : nullptr,
                         ins ? ins->elabel : nullptr, ins ? ins->ts : nullptr, del_keys, n_del, dev, true,
                         first_new_key);
    });
}

int mnemonic_get_result(mnemonic_ctx* ctx, uint32_t query, mnemonic_result* out) {
    if (!ctx || !out || query >= ctx->n_q) return MNEMONIC_E_ARG;
    if (ctx->broken) return MNEMONIC_E_HIP;
    if (ctx->results_incomplete) return MNEMONIC_E_CAPACITY;
    memset(out, 0, sizeof(*out));
    out->n_qe = ctx->hq[query].n_qe;
    if (!ctx->have_result) return MNEMONIC_OK;
    out->n_new = ctx->h_zr[ctx->zr_count(0) + query];
    out->n_expired = ctx->h_zr[ctx->zr_count(1) + query];
    const uint64_t* d = ctx->sum_dig.data();
    const uint32_t nq = ctx->n_q;
    out->dig_new[0] = d[2 * query];
    out->dig_new[1] = d[2 * query + 1];
    out->dig_expired[0] = d[2 * nq + 2 * query];
    out->dig_expired[1] = d[2 * nq + 2 * query + 1];
    if (ctx->flags & MNEMONIC_F_EMIT) {
        out->new_keys = ctx->houts[query].keys[0];
        out->expired_keys = ctx->houts[query].keys[1];
    }
    return MNEMONIC_OK;
}

int mnemonic_copy_keys(mnemonic_ctx* ctx, uint32_t query, int expired, uint64_t* host_buf,
                       uint64_t capacity, uint64_t* needed) {
    if (!ctx || query >= ctx->n_q) return MNEMONIC_E_ARG;
    return guarded(ctx, [&]() -> int {
        if (!(ctx->flags & MNEMONIC_F_EMIT)) throw ApiError{MNEMONIC_E_ARG, "context does not emit tuples"};
        if (ctx->results_incomplete)
            throw ApiError{MNEMONIC_E_CAPACITY, "the last batch's results are unavailable (no-allocation call)"};
        int p = expired ? 1 : 0;
        uint64_t n = ctx->have_result ? ctx->h_zr[ctx->zr_count(p) + query] : 0;
        if (needed) *needed = n;
        if (n > capacity) throw ApiError{MNEMONIC_E_CAPACITY, "host buffer too small"};
        if (n) {
            if (!host_buf) throw ApiError{MNEMONIC_E_ARG, "host_buf must not be NULL"};
            HIPCHK(hipMemcpyAsync(host_buf, ctx->houts[query].keys[p], n * ctx->hq[query].n_qe * 8,
                                  hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
        }
        return MNEMONIC_OK;
    });
}

int mnemonic_get_stats(mnemonic_ctx* ctx, mnemonic_stats* out) {
    if (!ctx || !out) return MNEMONIC_E_ARG;
    if (ctx->broken) return MNEMONIC_E_HIP;
    *out = ctx->stats;
    out->n_live_edges = ctx->n_live;
    out->slot_high_water = ctx->fresh;
    out->key_capacity = ctx->cap_keys;
    out->key_lo = ctx->key_lo;
    return MNEMONIC_OK;
}

const char* mnemonic_last_error(const mnemonic_ctx* ctx) {
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

int mnemonic_set_queries(mnemonic_ctx* ctx, const mnemonic_query* q, uint32_t n_q) {
    if (!ctx || !q) return MNEMONIC_E_ARG;
    return guarded(ctx, [&]() -> int {
        mnemonic_ctx* c = ctx;
        // plan the new set on a scratch context first: a bad query changes nothing
        mnemonic_ctx t;
        t.flags = c->flags;
        t.nV = c->nV;
        t.n_elabels = c->n_elabels;
        t.nbr_bits = c->nbr_bits;
        t.hb = c->hb;
        t.cls_mask = c->cls_mask;
        t.cls_start = c->cls_start;
        t.lab_deg = c->lab_deg;
        prepare_queries(&t, q, n_q);
        for (uint32_t i = 0; i < n_q; i++)
            for (uint32_t k = 0; k < q[i].n_qe; k++)
                if (q[i].qelabel[k] >= (int32_t)c->n_elabels)
                    throw ApiError{MNEMONIC_E_QUERY, "query edge label >= n_elabels"};
        hipStream_t s = c->stream;
        HIPCHK(hipStreamSynchronize(s));
        c->broken = true;  // until every query-dependent part is rebuilt below
        c->broken_why = "a query-set change";
        // query tables
        c->n_q = t.n_q;
        c->n_plans = t.n_plans;
        c->n_static = t.n_static;
        c->max_levels = t.max_levels;
        c->wv = t.wv;
        c->we = t.we;
        c->max_close = t.max_close;
        // the tile follows the new plans; an autotuned context tunes again
        c->tile_items = default_tile_items(c->max_close);
        c->tune_batch = 0;
        for (int i = 0; i < 3; i++) c->tune_ms[i] = c->tune_cand[i] = 0;
        memcpy(c->level_rows, t.level_rows, sizeof(c->level_rows));
        memcpy(c->level_emit, t.level_emit, sizeof(c->level_emit));
        c->hq.swap(t.hq);
        c->hplans.swap(t.hplans);
        c->hdebi.swap(t.hdebi);
        c->hvf.swap(t.hvf);
        c->hreq.swap(t.hreq);
        c->htree.swap(t.htree);
        c->tree_round.swap(t.tree_round);
        memcpy(c->elab_idx, t.elab_idx, sizeof(c->elab_idx));
        memcpy(c->vlab_idx, t.vlab_idx, sizeof(c->vlab_idx));
        c->n_elab_c = t.n_elab_c;
        c->n_vlab_c = t.n_vlab_c;
        c->n_cnt = t.n_cnt;
        c->vf_words = t.vf_words;
        const uint32_t old_words = c->debi_words;
        c->debi_words = t.debi_words;
        c->n_vf_bits = t.n_vf_bits;
        c->n_debi_bits = t.n_debi_bits;
        c->total_qe = t.total_qe;
        dev_free(c->d_q);
        dev_free(c->d_plans);
        dev_free(c->d_debi_bits);
        dev_free(c->d_vf_bits);
        dev_free(c->d_req);
        upload(c->d_q, c->hq, s);
        upload(c->d_plans, c->hplans, s);
        upload(c->d_debi_bits, c->hdebi, s);
        upload(c->d_vf_bits, c->hvf, s);
        upload(c->d_req, c->hreq, s);
        HIPCHK(hipMemcpyAsync(c->d_elab_idx, c->elab_idx, sizeof(c->elab_idx), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(c->d_vlab_idx, c->vlab_idx, sizeof(c->vlab_idx), hipMemcpyHostToDevice, s));
        // per-vertex filters and counters, per-slot edgeMatcher words: rebuilt
        // from the edges present
        dev_free(c->d_vf);
        dev_free(c->d_cnt);
        dev_alloc(c->d_vf, (size_t)c->nV * c->vf_words);
        dev_alloc(c->d_cnt, (size_t)c->nV * c->n_cnt);
        mn_launch_init_vertices(c->d_vf, c->d_cnt, c->nV, c->vf_words, c->n_cnt, s);
        if (c->tree_on()) {
            dev_free(c->d_tree);
            dev_free(c->d_vfp);
            upload(c->d_tree, c->htree, s);
            dev_alloc(c->d_vfp, (size_t)c->nV * c->vf_words);
        }
        if (c->debi_words != old_words && c->cap_slots) {
            dev_free(c->d_debi);
            dev_alloc(c->d_debi, c->cap_slots * c->debi_words);
        }
        GraphView g = make_view(c, false);
        mn_launch_reset(c->d_err, nullptr, 0, s);  // a failed batch may have left its error word set
        mn_launch_reindex(g, c->d_debi_bits, c->n_debi_bits, c->fresh, c->d_key2slot, c->key_lo, c->d_del_slot[c->pend],
                          (uint32_t)c->n_pending, s);
        mn_launch_vf_refresh(g, c->d_vf_bits, c->n_vf_bits, nullptr, c->nV, c->d_err, s);
        // outputs and per-phase tallies for the new count of queries
        for (auto& o : c->houts)
            for (int p = 0; p < 2; p++) dev_free(o.keys[p]);
        dev_free(c->d_outs);
        c->houts.assign(n_q, OutView{});
        c->out_rate.assign(2 * (size_t)n_q, -1.0);
        c->out_max.assign(2 * (size_t)n_q, 0);
        for (uint32_t i = 0; i < n_q; i++)
            for (int p = 0; p < 2; p++) {
                c->houts[i].cap[p] = (c->flags & MNEMONIC_F_EMIT) ? c->out_cap0 : 0;
                c->houts[i].keys[p] = nullptr;
                if (c->flags & MNEMONIC_F_EMIT) dev_alloc(c->houts[i].keys[p], c->out_cap0 * c->hq[i].n_qe);
            }
        dev_alloc(c->d_outs, n_q);
        HIPCHK(hipMemcpyAsync(c->d_outs, c->houts.data(), n_q * sizeof(OutView), hipMemcpyHostToDevice, s));
        dev_free(c->d_zr);
        c->n_zr = c->zr_words();
        c->h_zr.assign(c->n_zr, 0);
        size_zr_pin(c);
        dev_alloc(c->d_zr, c->n_zr);
        // level buffers (their width follows the queries) and the sizing state
        for (auto& B : c->lvb) {
            dev_free(B.keys);
            dev_free(B.rows);
            dev_free(B.lo);
            dev_free(B.cnt);
            dev_free(B.off);
            dev_free(B.hpre);
        }
        c->lvb.assign(c->max_levels, mnemonic_ctx::LevelBuf{});
        for (int p = 0; p < 2; p++)
            for (int L = 0; L <= MN_MAXLV; L++) c->rate[p][L] = c->row_rate[p][L] = -1.0;
        c->have_result = false;
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
        c->broken = false;
        return MNEMONIC_OK;
    });
}

int mnemonic_set_scheduler(mnemonic_ctx* ctx, int mode, const float* weights) {
    if (!ctx) return MNEMONIC_E_ARG;
    return guarded(ctx, [&]() -> int {
        if (mode < 0 || mode >= MN_SCHED_FIXED + MN_NVAR) throw ApiError{MNEMONIC_E_ARG, "bad scheduler mode"};
        if (mode == MN_SCHED_LEARNED) {
            if (!weights) throw ApiError{MNEMONIC_E_ARG, "the learned scheduler needs weights"};
            if (!ctx->d_sched_w) {
                dev_alloc(ctx->d_sched_f32, MN_MLP_WEIGHTS);
                dev_alloc(ctx->d_sched_w, MN_MLP_WEIGHTS);
            }
            HIPCHK(hipMemcpyAsync(ctx->d_sched_f32, weights, MN_MLP_WEIGHTS * sizeof(float), hipMemcpyHostToDevice,
                                  ctx->stream));
            mn_to_bf16(ctx->d_sched_f32, ctx->d_sched_w, MN_MLP_WEIGHTS, ctx->stream);
            HIPCHK(hipGetLastError());
            HIPCHK(hipStreamSynchronize(ctx->stream));
        }
        ctx->sched_mode = (uint32_t)mode;
        return MNEMONIC_OK;
    });
}

int mnemonic_query_orders(mnemonic_ctx* ctx, uint32_t query, uint32_t j, uint32_t* n_orders) {
    if (!ctx || !n_orders) return MNEMONIC_E_ARG;
    if (ctx->broken) return MNEMONIC_E_HIP;
    if (query >= ctx->n_q || j >= ctx->hq[query].n_qe) return MNEMONIC_E_ARG;
    *n_orders = ctx->hplans[ctx->hq[query].plan_base + j].n_var;
    return MNEMONIC_OK;
}

int mnemonic_set_trace(mnemonic_ctx* ctx, uint64_t capacity) {
    if (!ctx) return MNEMONIC_E_ARG;
    return guarded(ctx, [&]() -> int {
        if (capacity > (1u << 28)) throw ApiError{MNEMONIC_E_ARG, "trace capacity > 2^28"};
        HIPCHK(hipStreamSynchronize(ctx->stream));
        // the rows between levels gain or lose the trace column: reallocated on demand
        for (auto& B : ctx->lvb) {
            dev_free(B.keys);
            dev_free(B.rows);
            dev_free(B.lo);
            dev_free(B.cnt);
            dev_free(B.off);
            dev_free(B.hpre);
            B.cap = 0;
        }
        dev_free(ctx->d_tr_n);
        dev_free(ctx->d_tr_code);
        dev_free(ctx->d_tr_x);
        dev_free(ctx->d_tr_work);
        ctx->tr_cap = 0;
        if (capacity) {
            dev_alloc(ctx->d_tr_n, 2);
            dev_alloc(ctx->d_tr_code, 2 * capacity);
            dev_alloc(ctx->d_tr_x, 2 * capacity * MN_NVAR * MN_MLP_IN);
            dev_alloc(ctx->d_tr_work, 2 * capacity);
            mn_launch_set_u32(ctx->d_tr_n, 0, ctx->stream);
            mn_launch_set_u32(ctx->d_tr_n + 1, 0, ctx->stream);
            HIPCHK(hipGetLastError());
            HIPCHK(hipStreamSynchronize(ctx->stream));
            ctx->tr_cap = (uint32_t)capacity;
        }
        return MNEMONIC_OK;
    });
}

int mnemonic_get_trace(mnemonic_ctx* ctx, int phase, uint64_t* n, uint64_t* codes, float* x, uint64_t* work,
                       uint64_t cap) {
    if (!ctx || (phase != 0 && phase != 1) || !n) return MNEMONIC_E_ARG;
    return guarded(ctx, [&]() -> int {
        if (!ctx->tr_cap) throw ApiError{MNEMONIC_E_ARG, "tracing is off"};
        uint32_t cnt[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(cnt, ctx->d_tr_n, sizeof(cnt), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        const uint64_t m = std::min<uint64_t>(cnt[phase], ctx->tr_cap);
        *n = m;
        const uint64_t k = std::min<uint64_t>(m, cap);
        const size_t base = (size_t)phase * ctx->tr_cap;
        if (k && codes)
            HIPCHK(hipMemcpyAsync(codes, ctx->d_tr_code + base, k * 8, hipMemcpyDeviceToHost, ctx->stream));
        if (k && x)
            HIPCHK(hipMemcpyAsync(x, ctx->d_tr_x + base * MN_NVAR * MN_MLP_IN, k * MN_NVAR * MN_MLP_IN * 4,
                                  hipMemcpyDeviceToHost, ctx->stream));
        if (k && work) HIPCHK(hipMemcpyAsync(work, ctx->d_tr_work + base, k * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        return MNEMONIC_OK;
    });
}

void mnemonic_fail_alloc_after(uint64_t n) { g_fail_alloc_in = n; }

int mnemonic_mlp_predict(const float* w, const float* x, uint64_t n, int bf16, float* y, void* hip_stream) {
    if (n && (!w || !x || !y)) return MNEMONIC_E_ARG;
    mn_mlp_predict(w, x, n, bf16, y, static_cast<hipStream_t>(hip_stream));
    return hipGetLastError() == hipSuccess ? MNEMONIC_OK : MNEMONIC_E_HIP;
}

int mnemonic_mlp_grad(const float* w, const float* x, const float* target, const uint32_t* idx, uint64_t off,
                      uint64_t m, float* grad, float* loss, void* hip_stream) {
    if (m && (!w || !x || !target || !grad || !loss)) return MNEMONIC_E_ARG;
    mn_mlp_grad(w, x, target, idx, off, m, grad, loss, static_cast<hipStream_t>(hip_stream));
    return hipGetLastError() == hipSuccess ? MNEMONIC_OK : MNEMONIC_E_HIP;
}

int mnemonic_mlp_adam(float* w, float* m1, float* m2, float* grad, float lr, uint32_t step, void* hip_stream) {
    if (!w || !m1 || !m2 || !grad || step == 0) return MNEMONIC_E_ARG;
    mn_mlp_adam(w, m1, m2, grad, lr, step, static_cast<hipStream_t>(hip_stream));
    return hipGetLastError() == hipSuccess ? MNEMONIC_OK : MNEMONIC_E_HIP;
}

void mnemonic_destroy(mnemonic_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    t_stream = ctx->stream;
    free_all(ctx);
    (void)hipStreamSynchronize(ctx->stream);  // the frees are ordered on the caller's stream
    delete ctx;
}

}  // extern "C"
