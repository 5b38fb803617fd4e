// Work units and the level-wise enumerator (Section VI, "Embedding
// Enumeration").
//
// A work unit is a batch edge at a start position j of a query: its
// edgeMatcher bit for q_j is set and both endpoints pass the vertex filter
// (Section VI, work decomposition; the edgeMatcher word holds a bit for every
// query edge, tree or not, so a non-tree start edge needs no expansion into
// tree-edge units). The static order for (query, j) then maps one new query
// vertex per level through an anchor edge whose candidates are one run of the
// mapped endpoint's sorted adjacency (getCandidates of Section IV-A),
// checks each candidate against the duplicate-removal mask (positions k < j
// may not use batch edges), the vertex filter, injectivity (isomorphism only)
// and the closing edges (verifyNte), and emits at the last level.
//
// The paper gives each work unit to one CPU thread, which backtracks depth
// first. On the GPU the search runs breadth first instead, one level at a
// time over all work units of a phase, so that every candidate entry is one
// lane's work no matter how skewed the subtrees are:
//   k_seed_rows    one row per work unit (start pair mapped, start-level
//                  closing edges found); 2-vertex queries emit here
//   k_decide       (learned scheduler, traces) the matching order of each row
//   k_level_range  per row, the candidate run [lo, lo + cnt) of the level
//   scan           u64 offsets of the runs (flattened candidate space); with
//                  k_offsets_partition the offsets, the candidate total and
//                  the first row of every expansion tile in one more launch
//   k_partition    the first row of every expansion tile (levels too wide
//                  for k_offsets_partition, and host-walked chunks)
//   k_expand       one lane per candidate: filters, closing edges, temporal
//                  order, then a new row for the next level or, at the plan's
//                  last level, the embeddings themselves
// Normally every launch of a phase reads its row count and candidate total
// from device memory (no host round trip); a level that outgrows its buffers
// leaves a note and the host re-runs the phase with larger ones, or walks the
// levels in host-sized chunks, depth first over chunks, so each level's row
// buffer stays bounded whatever the fan-out. Parallel closing-edge instances
// do not multiply rows: a row keeps the start of each closing edge's instance
// run, and emission expands every combination of instances (parallel edges
// are distinct instances, Section I).
#include <hip/hip_ext.h>

#include "mn_internal.h"
#include "mn_sched.h"

namespace {

// candidates per lane in one expansion tile (tile = 256 x items): 1, 2 or 4
constexpr uint32_t EX_TILE_MIN = MN_BLOCK;  // the smallest tile sizes the tile_row buffer
constexpr uint64_t EX_SPARE_TILES = 8192;   // grid margin of a device-sized expansion past the expected tiles
// Waves per SIMD the expansion kernels' registers must allow in blocks of
// 512 and more threads (two or more waves per SIMD each): with no or one
// closing edge, full occupancy (64 VGPRs, a few spill in the emitting
// variants: measured faster than losing a block), with more, as many blocks
// as their larger arrays leave room for. Blocks of 256 keep the compiler's
// choice.
constexpr uint32_t ex_min_waves(uint32_t threads, int nc) {
    return threads < 512 ? 1u : nc <= 1 ? 8u : nc <= 4 ? 6u : 4u;
}
constexpr uint32_t NO_RUN = 0xFFFFFFFFu;
constexpr uint32_t RUN_SWAP = 0x80000000u;
constexpr uint8_t TREE_EDGE = 0xFF;
// The learned choice leaves the static order only for a predicted saving of
// more than this many log2 units of work (0.25: about 16% less work).
constexpr float SCHED_MARGIN = 0.25f;

__device__ inline bool failed(const uint32_t* err) { return *(volatile const uint32_t*)err != 0u; }

__device__ inline void set_err(const uint32_t* err, uint32_t code) {
    atomicCAS(const_cast<uint32_t*>(err), 0u, code);
}

__device__ inline uint64_t shfl64(uint64_t x, int src) {
    uint32_t lo = __shfl((uint32_t)x, src, MN_WAVE);
    uint32_t hi = __shfl((uint32_t)(x >> 32), src, MN_WAVE);
    return ((uint64_t)hi << 32) | lo;
}

// Wave sums through DPP lane moves (no LDS traffic): pairs and quads by quad
// permutes, rows of 16 by the half-row and row mirrors, then row 0's total
// into row 1 and row 2's into row 3 (row_bcast:15), rows 0-1 into rows 2-3
// (row_bcast:31); lane 63 ends with the wave's total, read back uniformly.
// Every lane of the wave must be active.
#define MN_DPP_STEPS(STEP) \
    STEP(0xB1, 0xF)        \
    STEP(0x4E, 0xF)        \
    STEP(0x141, 0xF)       \
    STEP(0x140, 0xF)       \
    STEP(0x142, 0xA)       \
    STEP(0x143, 0xC)

__device__ inline uint32_t wave_sum32(uint32_t x) {
#define MN_STEP32(ctrl, rows) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, ctrl, rows, 0xF, false);
    MN_DPP_STEPS(MN_STEP32)
#undef MN_STEP32
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

__device__ inline uint64_t wave_sum64(uint64_t x) {
#define MN_STEP64(ctrl, rows)                                                                          \
    {                                                                                                  \
        const uint32_t lo_ = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, ctrl, rows, 0xF, false); \
        const uint32_t hi_ = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), ctrl, rows, 0xF, false); \
        x += ((uint64_t)hi_ << 32) | lo_;                                                              \
    }
    MN_DPP_STEPS(MN_STEP64)
#undef MN_STEP64
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

// Exclusive prefix sum over the wave (all 64 lanes must take part).
__device__ inline uint64_t wave_excl_scan64(uint64_t x, uint64_t& total) {
    const uint32_t lane = __lane_id();
    uint64_t incl = x;
#pragma unroll
    for (int d = 1; d < MN_WAVE; d <<= 1) {
        uint32_t lo = __shfl_up((uint32_t)incl, d, MN_WAVE);
        uint32_t hi = __shfl_up((uint32_t)(incl >> 32), d, MN_WAVE);
        if (lane >= (uint32_t)d) incl += ((uint64_t)hi << 32) | lo;
    }
    total = shfl64(incl, MN_WAVE - 1);
    return incl - x;
}

// Vertices < 2^24 and at most 128 filter words (256 queries x 16 vertices)
// keep the index below 2^31.
__device__ inline bool vf_bit(const GraphView& g, uint32_t v, uint32_t bit) {
    return (g.vf[v * g.vf_words + (bit >> 5)] >> (bit & 31)) & 1u;
}

// Column c of row r. The library keeps a level's rows at most 2^26 and its
// columns at most 50, so c * cap + r fits in 32 bits.
__device__ inline uint32_t rcol(const RowsView& R, uint32_t c, uint32_t r) { return R.col[c * R.cap + r]; }

__device__ inline void wcol(const RowsView& R, uint32_t c, uint32_t r, uint32_t v) { R.col[c * R.cap + r] = v; }

__device__ inline uint64_t rkey(const RowsView& R, uint32_t k, uint32_t r) { return R.kcol[k * R.cap + r]; }

__device__ inline void wkey(const RowsView& R, uint32_t k, uint32_t r, uint64_t v) { R.kcol[k * R.cap + r] = v; }

// Per-lane work tallies of one launch (32 bits suffice per lane and launch).
struct Cnt {
    uint32_t seeds, entries, probes, range_probes, keys, tuples, vf, rows, vfrej;
};

constexpr uint32_t MAXQ = 256;

// Per-block accumulators in LDS: work tallies and per-query digests are
// summed here and reach global memory once per block, into shard
// b % MN_SHARDS, so that no address sees more than a few atomics per launch.
struct BlockAcc {
    unsigned long long st[MN_TALLIES];
    unsigned long long dig[2 * MAXQ];
    uint32_t dead;  // the error word was set before this block started
};

__device__ inline uint32_t block_linear() { return blockIdx.x + blockIdx.y * gridDim.x; }

// Zeroes the accumulators and reads the error word once for the whole block.
__device__ void acc_init(BlockAcc& A, uint32_t n_dig, const uint32_t* err) {
    for (uint32_t i = threadIdx.x; i < MN_TALLIES + n_dig; i += blockDim.x) {
        if (i < MN_TALLIES)
            A.st[i] = 0;
        else
            A.dig[i - MN_TALLIES] = 0;
    }
    if (threadIdx.x == 0) A.dead = failed(err) ? 1u : 0u;
    __syncthreads();
}

// Adds the lanes' tallies and the block's digests to this block's shard.
// Every thread of the block must call it.
__device__ void acc_flush(BlockAcc& A, const Cnt& K, uint32_t n_dig, EnumStats* stats,
                          unsigned long long* digest) {
    // a lane's tallies of one launch fit in 32 bits, and so do a wave's
    const uint32_t v[MN_TALLIES] = {wave_sum32(K.seeds), wave_sum32(K.entries), wave_sum32(K.probes),
                                    wave_sum32(K.range_probes), wave_sum32(K.keys), wave_sum32(K.tuples),
                                    wave_sum32(K.vf), wave_sum32(K.rows), wave_sum32(K.vfrej)};
    if (__lane_id() == 0) {
#pragma unroll
        for (int i = 0; i < MN_TALLIES; i++)
            if (v[i]) atomicAdd(&A.st[i], (unsigned long long)v[i]);
    }
    __syncthreads();
    const uint32_t shard = block_linear() % MN_SHARDS;
    unsigned long long* gst = reinterpret_cast<unsigned long long*>(stats + shard);
    unsigned long long* gdig = digest ? digest + (size_t)shard * n_dig : nullptr;
    if (threadIdx.x < MN_TALLIES && A.st[threadIdx.x]) atomicAdd(&gst[threadIdx.x], A.st[threadIdx.x]);
    for (uint32_t i = threadIdx.x; i < n_dig; i += blockDim.x)
        if (A.dig[i]) atomicAdd(&gdig[i], A.dig[i]);
}

// Lower bound over the high words of a sorted segment, counting the words
// it reads.
__device__ inline uint32_t lower_hi_c(const uint64_t* adj, uint32_t lo, uint32_t hi, uint32_t key,
                                      uint32_t& probes) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(adj);
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        probes++;
        if (w[2 * (size_t)mid + 1] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Both ends of the run of high words in [key_lo, key_hi] of a sorted
// segment: the lower and the upper bound advance in lockstep, so each step
// issues its two loads together and the chain of dependent loads is one
// search long instead of two.
__device__ inline void run_bounds_c(const uint64_t* adj, uint32_t s0, uint32_t s1, uint32_t key_lo, uint32_t key_hi,
                                    uint32_t& a, uint32_t& b, uint32_t& probes) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(adj);
    uint32_t la = s0, ha = s1, lb = s0, hb = s1;
    while (la < ha || lb < hb) {
        const bool ga = la < ha, gb = lb < hb;
        const uint32_t ma = (la + ha) >> 1, mb = (lb + hb) >> 1;
        const uint32_t va = ga ? w[2 * (size_t)ma + 1] : 0u;
        const uint32_t vb = gb ? w[2 * (size_t)mb + 1] : 0u;
        if (ga) {
            probes++;
            if (va < key_lo)
                la = ma + 1;
            else
                ha = ma;
        }
        if (gb) {
            probes++;
            if (vb <= key_hi)
                lb = mb + 1;
            else
                hb = mb;
        }
    }
    a = la;
    b = max(la, lb);  // an empty key range gives an empty run
}

// Where the images of query vertices come from while a candidate is tested:
// the row of the partial embedding (or, at the start level, the start edge's
// endpoints) plus the level's new vertex.
struct Bind {
    RowsView R;
    bool row;  // false at the start level
    uint32_t r;
    uint32_t qa, fa, qb, fb;  // start level: f(qa), f(qb)
    uint64_t skey;            // start level: key of the start edge
    uint32_t cv, fw;          // the level's new vertex (0xFF: none) and its image

    __device__ uint32_t f(uint32_t u) const {
        if (u == cv) return fw;
        if (!row) return u == qa ? fa : fb;
        return rcol(R, 1 + u, r);
    }
    // key of a tree edge mapped before the current level
    __device__ uint64_t tree_key(uint32_t k) const {
        if (!row) return skey;  // at the start level the start edge is the only tree edge
        return rkey(R, k, r);
    }
};

// Instances of closing edge c between f(other) = fo and f(nv) = fn: searches
// the shorter of the two adjacency lists that hold them. Returns the first
// accepted instance (labelled edge: in the (label, neighbour) run;
// unlabelled edge: in the whole list), with RUN_SWAP set when the list of fn
// was used, or NO_RUN when no instance passes the mask. Walks over the
// instances start there.
__device__ uint32_t close_find(const GraphView& g, const CloseDesc& c, uint32_t fo, uint32_t fn,
                               uint32_t& probes) {
    const uint32_t d0 = c.dir, d1 = 1u - c.dir;
    const uint32_t* oa = g.offs(d0);
    const uint32_t* ob = g.offs(d1);
    const uint32_t a0 = oa[fo], a1 = oa[fo + 1];
    const uint32_t b0 = ob[fn], b1 = ob[fn + 1];
    probes += 4;
    const bool sw = (b1 - b0) < (a1 - a0);
    const uint32_t dir = sw ? d1 : d0;
    const uint32_t s0 = sw ? b0 : a0, s1 = sw ? b1 : a1, tgt = sw ? fo : fn;
    const uint64_t* adj = g.adjs(dir);
    const uint32_t flag = sw ? RUN_SWAP : 0u;
    if (c.label >= 0) {
        const uint32_t key = ((uint32_t)c.label << g.nbr_bits) | tgt;
        const uint32_t lb = lower_hi_c(adj, s0, s1, key, probes);
        for (uint32_t p = lb; p < s1; p++) {
            const uint64_t e = adj[p];
            probes += 2;
            if (ent_hi(e) != key) break;
            if (!(c.masked && (ent_lo(e) & MN_FLAG))) return p | flag;
        }
        return NO_RUN;
    }
    for (uint32_t p = s0; p < s1; p++) {
        const uint64_t e = adj[p];
        probes += 2;
        if ((ent_hi(e) & g.nbr_mask) == tgt && !(c.masked && (ent_lo(e) & MN_FLAG))) return p | flag;
    }
    return NO_RUN;
}

// Iterator over the accepted instances of a closing edge from its run start.
struct RunIt {
    const uint64_t* adj;
    const uint64_t* adjk;
    uint32_t p, end, key, tgt, nbr_mask;
    bool lab, masked;
};

__device__ inline RunIt run_open(const GraphView& g, const CloseDesc& c, uint32_t st, uint32_t fo,
                                 uint32_t fn) {
    RunIt it;
    const bool sw = (st & RUN_SWAP) != 0;
    const uint32_t dir = sw ? 1u - c.dir : (uint32_t)c.dir;
    const uint32_t x = sw ? fn : fo;
    it.adj = g.adjs(dir);
    it.adjk = g.keys(dir);
    it.p = st & ~RUN_SWAP;
    it.end = g.offs(dir)[x + 1];
    it.tgt = sw ? fo : fn;
    it.lab = c.label >= 0;
    it.key = it.lab ? (((uint32_t)c.label << g.nbr_bits) | it.tgt) : 0u;
    it.nbr_mask = g.nbr_mask;
    it.masked = c.masked != 0;
    return it;
}

// First accepted instance at or after p, or it.end.
__device__ inline uint32_t run_next(const RunIt& it, uint32_t p, uint32_t& probes) {
    for (; p < it.end; p++) {
        const uint64_t e = it.adj[p];
        probes += 2;
        if (it.lab) {
            if (ent_hi(e) != it.key) return it.end;
        } else if ((ent_hi(e) & it.nbr_mask) != it.tgt) {
            continue;
        }
        if (it.masked && (ent_lo(e) & MN_FLAG)) continue;
        return p;
    }
    return it.end;
}

// A closing edge's instances as a row keeps them once the edge is resolved:
// the key of the instance when there is exactly one, else CK_MULTI | their
// number (edge keys stay below 2^63). st is the first accepted instance, as
// close_find returns it. Later levels then need no walk over the instances
// for a mapping whose closing edges each have one.
constexpr uint64_t CK_MULTI = 1ull << 63;

__device__ inline uint64_t close_word(const GraphView& g, const CloseDesc& c, uint32_t st, uint32_t fo, uint32_t fn,
                                      uint32_t& probes) {
    const RunIt it = run_open(g, c, st, fo, fn);
    const uint32_t q = run_next(it, it.p + 1, probes);
    if (q >= it.end) return it.adjk[it.p];
    uint32_t n = 2;
    for (uint32_t x = run_next(it, q + 1, probes); x < it.end; x = run_next(it, x + 1, probes)) n++;
    return CK_MULTI | n;
}

// Set on a candidate's neighbour (vertices stay below 2^24) between the two
// passes of an expansion: its mapping's closing edges each have one instance.
constexpr uint32_t CK_ONE = 0x80000000u;

// Instances of a closing edge from the row's word (close_word).
__device__ inline uint32_t close_word_count(uint64_t w) { return (w & CK_MULTI) ? (uint32_t)w : 1u; }

// Lanes with `active` set reserve v consecutive places in the per-query
// counters[q]; lanes with the same q share one atomic. All lanes of the wave
// must call this together. Returns the lane's first place.
__device__ uint64_t grouped_reserve(bool active, uint32_t q, uint64_t v, unsigned long long* counters) {
    uint64_t pending = __ballot(active);
    const uint32_t lane = __lane_id();
    uint64_t mine = 0;
    while (pending) {
        const uint32_t leader = (uint32_t)__ffsll((unsigned long long)pending) - 1;
        const uint32_t k = __shfl(q, leader, MN_WAVE);
        const uint64_t grp = __ballot(active && q == k) & pending;
        const bool in = (grp >> lane) & 1ull;
        uint64_t tot;
        const uint64_t ex = wave_excl_scan64(in ? v : 0ull, tot);
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(&counters[k], (unsigned long long)tot);
        base = shfl64(base, leader);
        if (in) mine = base + ex;
        pending &= ~grp;
    }
    return mine;
}

// Adds (a, b) of the active lanes to the block's LDS digests dig[2q],
// dig[2q + 1], one atomic pair per distinct q in the wave. All lanes must call
// this together.
__device__ void grouped_digest(bool active, uint32_t q, uint64_t a, uint64_t b, unsigned long long* digest) {
    uint64_t pending = __ballot(active);
    const uint32_t lane = __lane_id();
    while (pending) {
        const uint32_t leader = (uint32_t)__ffsll((unsigned long long)pending) - 1;
        const uint32_t k = __shfl(q, leader, MN_WAVE);
        const uint64_t grp = __ballot(active && q == k) & pending;
        const bool in = (grp >> lane) & 1ull;
        const uint64_t sa = wave_sum64(in ? a : 0ull), sb = wave_sum64(in ? b : 0ull);
        if (lane == leader) {
            atomicAdd(&digest[2 * k], (unsigned long long)sa);
            atomicAdd(&digest[2 * k + 1], (unsigned long long)sb);
        }
        pending &= ~grp;
    }
}

// Whether instance `key` of closing edge ci can take part in a temporally
// ordered embedding with the mapping's fixed edges (tree edges and the
// anchor aqe, whose key is akey): its timestamp must exceed theirs of lower
// rank and stay below theirs of higher rank. Always true for an unranked
// edge; the other closing edges are checked per combination.
__device__ inline bool inst_in_window(const GraphView& g, const SeedPlan& P, const Bind& B, uint32_t ci, uint64_t key,
                                      uint32_t aqe, uint64_t akey) {
    const int r = P.rank[P.close[ci].qe];
    if (r < 0) return true;
    const int64_t t = g.key_ts[key & g.key_mask];
    for (uint32_t x = 0; x < P.n_ranked; x++) {
        const uint32_t k = P.rorder[x];
        const int rk = P.rank[k];
        if (rk == r || (k != aqe && P.close_idx[k] != TREE_EDGE)) continue;
        const int64_t tk = g.key_ts[(k == aqe ? akey : B.tree_key(k)) & g.key_mask];
        if (rk < r ? !(tk < t) : !(t < tk)) return false;
    }
    return true;
}

// The combinations of the closing edges' instances, stepped through like an
// odometer: digit i is the position of close[i]'s current accepted instance
// in its run, digit 0 moves fastest. A step walks only the digits that move
// (one run step each, plus a wrap to the run's first instance on a carry),
// so a combination costs O(1) run steps on average instead of a walk from
// every run's start. st[i] is close[i]'s first accepted instance (as
// close_find returns it), RUN_SWAP marking the list of f(nv). Under a
// temporal order (`win`) each digit runs only over the instances that fit
// the fixed edges' timestamps (inst_in_window): combinations outside those
// windows cannot be embeddings, and only the windows' product is visited.

// Digit i's first instance at or after p (in its window when `win`), or the
// run's end.
__device__ inline uint32_t odo_seek(const GraphView& g, const SeedPlan& P, const Bind& B, const RunIt& it, uint32_t i,
                                    uint32_t p, bool win, uint32_t aqe, uint64_t akey) {
    uint32_t unused = 0;
    uint32_t q = run_next(it, p, unused);
    while (win && q < it.end && !inst_in_window(g, P, B, i, it.adjk[q], aqe, akey)) q = run_next(it, q + 1, unused);
    return q;
}

// Puts every digit at its first instance; false when some digit has none (no
// combination).
template <int NC>
__device__ inline bool odo_first(const GraphView& g, const SeedPlan& P, const Bind& B, const uint32_t* st,
                                 uint32_t* pos, bool win, uint32_t aqe, uint64_t akey) {
    constexpr int NA = NC > 0 ? NC : 1;
#pragma unroll
    for (uint32_t i = 0; i < NA; i++) pos[i] = st[i] & ~RUN_SWAP;
    if (!win) return true;
#pragma unroll 1
    for (uint32_t i = 0; i < (uint32_t)NC && i < P.n_close; i++) {
        uint32_t s_st = 0;
#pragma unroll
        for (uint32_t k = 0; k < NA; k++)
            if (k == i) s_st = st[k];
        const CloseDesc c = P.close[i];
        const RunIt it = run_open(g, c, s_st, B.f(c.other), B.f(c.nv));
        const uint32_t q = odo_seek(g, P, B, it, i, it.p, true, aqe, akey);
        if (q >= it.end) return false;
#pragma unroll
        for (uint32_t k = 0; k < NA; k++)
            if (k == i) pos[k] = q;
    }
    return true;
}

// Advances to the next combination; false after the last one (every digit
// back at its first instance).
template <int NC>
__device__ inline bool odo_next(const GraphView& g, const SeedPlan& P, const Bind& B, const uint32_t* st,
                                uint32_t* pos, bool win, uint32_t aqe, uint64_t akey) {
    constexpr int NA = NC > 0 ? NC : 1;
    // one digit per step of a rolled loop: the run walk is compiled once,
    // and the digit's state is picked from and put back into the arrays
#pragma unroll 1
    for (uint32_t i = 0; i < (uint32_t)NC && i < P.n_close; i++) {
        uint32_t s_st = 0, s_pos = 0;
#pragma unroll
        for (uint32_t k = 0; k < NA; k++)
            if (k == i) {
                s_st = st[k];
                s_pos = pos[k];
            }
        const CloseDesc c = P.close[i];
        const RunIt it = run_open(g, c, s_st, B.f(c.other), B.f(c.nv));
        // the next instance; past the last one, a carry puts the digit back at
        // its first instance (one exists: odo_first found it)
        uint32_t from = s_pos + 1, v = it.end;
        bool moved = true;
#pragma unroll 1
        for (int pass = 0; pass < 2; pass++) {
            v = odo_seek(g, P, B, it, i, from, win, aqe, akey);
            if (v < it.end) break;
            moved = false;
            from = it.p;
        }
#pragma unroll
        for (uint32_t k = 0; k < NA; k++)
            if (k == i) pos[k] = v;
        if (moved) return true;
    }
    return false;
}

// Key of close[ci]'s current instance (pos[ci] in the list st[ci] names).
template <int NC>
__device__ inline uint64_t odo_key(const GraphView& g, const SeedPlan& P, const uint32_t* st, const uint32_t* pos,
                                   uint32_t ci) {
    constexpr int NA = NC > 0 ? NC : 1;
    uint32_t s_st = 0, s_pos = 0;
#pragma unroll
    for (uint32_t i = 0; i < NA; i++)
        if (i == ci) {
            s_st = st[i];
            s_pos = pos[i];
        }
    const CloseDesc c = P.close[ci];
    const uint32_t dir = (s_st & RUN_SWAP) ? 1u - c.dir : (uint32_t)c.dir;
    return g.keys(dir)[s_pos];
}

// Timestamp of the edge that query edge k maps to in the current combination.
template <int NC>
__device__ inline int64_t edge_ts(const GraphView& g, const SeedPlan& P, const Bind& B, const uint32_t* st,
                                  const uint32_t* pos, uint32_t k, uint32_t aqe, uint64_t akey) {
    const uint32_t ci = P.close_idx[k];
    if (k == aqe || ci == TREE_EDGE) return g.key_ts[(k == aqe ? akey : B.tree_key(k)) & g.key_mask];
    return g.key_ts[odo_key<NC>(g, P, st, pos, ci) & g.key_mask];
}

// Temporal order of one complete embedding: walking the ranked edges by
// ascending rank, every edge's timestamp exceeds the largest timestamp of
// all lower ranks.
template <int NC>
__device__ bool in_time_order(const GraphView& g, const SeedPlan& P, const Bind& B, const uint32_t* st,
                              const uint32_t* pos, uint32_t aqe, uint64_t akey) {
    int64_t below = INT64_MIN, level = INT64_MIN;
    int cur = -1;
    for (uint32_t x = 0; x < P.n_ranked; x++) {
        const uint32_t k = P.rorder[x];
        if (P.rank[k] != cur) {  // a new rank level: the previous one joins the ranks below
            below = max(below, level);
            level = INT64_MIN;
            cur = P.rank[k];
        }
        const int64_t t = edge_ts<NC>(g, P, B, st, pos, k, aqe, akey);
        if (!(below < t)) return false;
        level = max(level, t);
    }
    return true;
}

// Number of embeddings of a complete mapping: the product over the
// closing edges of their accepted instances (st[i] is the first accepted
// instance of close[i]), or, for a plan with a temporal order, the
// combinations of instances that satisfy it. aqe/akey: the anchor query edge
// of the level and its edge (0xFF: none).
template <int NC>
__device__ uint64_t close_mult(const GraphView& g, const SeedPlan& P, const Bind& B, const uint32_t* st,
                               uint32_t& probes, uint32_t aqe, uint64_t akey) {
    constexpr int NA = NC > 0 ? NC : 1;
    uint64_t mult = 1;
#pragma unroll
    for (uint32_t i = 0; i < NA; i++) {
        if (i < (uint32_t)NC && i < P.n_close) {
            const CloseDesc c = P.close[i];
            const RunIt it = run_open(g, c, st[i], B.f(c.other), B.f(c.nv));
            uint32_t n = 0;
            for (uint32_t p = run_next(it, it.p, probes); p < it.end; p = run_next(it, p + 1, probes)) n++;
            mult *= n;
        }
    }
    if (P.temporal && mult) {
        uint32_t pos[NA];
        uint64_t ok = 0;
        if constexpr (NC == 1) {  // one closing edge: a plain walk over its run
            const CloseDesc c = P.close[0];
            const RunIt it = run_open(g, c, st[0], B.f(c.other), B.f(c.nv));
            uint32_t unused = 0;
            for (uint32_t p = it.p; p < it.end; p = run_next(it, p + 1, unused)) {
                pos[0] = p;
                ok += in_time_order<NC>(g, P, B, st, pos, aqe, akey) ? 1u : 0u;
            }
        } else if (odo_first<NC>(g, P, B, st, pos, true, aqe, akey)) {
            do {
                ok += in_time_order<NC>(g, P, B, st, pos, aqe, akey) ? 1u : 0u;
            } while (odo_next<NC>(g, P, B, st, pos, true, aqe, akey));
        }
        mult = ok;
    }
    return mult;
}

// Writes the mult embeddings of one complete mapping at rows pos.. of the
// query's output (when emitting) and returns their digest sums: each tuple
// lists its edges' keys in query-edge order, the anchor query edge aqe
// (0xFF: none) mapping to the edge with key akey, and is folded as
// h_s = mix(...mix(mix(s ^ q) + k_0)... + k_{m-1}), mix = SplitMix64's
// finaliser. Combinations come in odometer order; under a temporal order
// only those that satisfy it (close_mult counted exactly those: mult).
template <int NC>
__device__ void emit_tuples(const GraphView& g, const SeedPlan& P, const Bind& B, const uint32_t* st,
                            uint64_t mult, uint32_t aqe, uint64_t akey, uint64_t pos0, const PhaseOut& po, Cnt& K,
                            uint64_t& dA, uint64_t& dB) {
    constexpr int NA = NC > 0 ? NC : 1;
    const uint32_t q = P.q;
    const OutView& ov = po.outs[q];
    uint64_t* out = ov.keys[po.phase];
    const uint64_t cap = ov.cap[po.phase];
    const uint32_t nqe = P.n_qe;
    const uint64_t s0A = mn_mix64(MN_SEED_A ^ (uint64_t)q);
    const uint64_t s0B = mn_mix64(MN_SEED_B ^ (uint64_t)q);
    uint32_t pos[NA];
    uint64_t j = 0;
    auto one = [&]() {  // the current combination, when it is an embedding
        if (P.temporal && !in_time_order<NC>(g, P, B, st, pos, aqe, akey)) return;
        uint64_t hA = s0A, hB = s0B;
        const bool write = po.emit && (pos0 + j) < cap;
        uint64_t* row = out + (pos0 + j) * nqe;
        j++;
        for (uint32_t k = 0; k < nqe; k++) {
            uint64_t key;
            const uint32_t ci = P.close_idx[k];
            if (k == aqe) {
                key = akey;
            } else if (ci == TREE_EDGE) {
                key = B.tree_key(k);
            } else {
                key = odo_key<NC>(g, P, st, pos, ci);
            }
            K.keys++;
            hA = mn_mix64(hA + key);
            hB = mn_mix64(hB + key);
            if (write) row[k] = key;
        }
        dA += hA;
        dB += hB;
        K.tuples++;
    };
    if constexpr (NC <= 1) {  // at most one closing edge: a plain walk over its run
        pos[0] = 0;
        if (NC == 0 || P.n_close == 0) {
            one();
        } else {
            const CloseDesc c = P.close[0];
            const RunIt it = run_open(g, c, st[0], B.f(c.other), B.f(c.nv));
            uint32_t unused = 0;
            for (uint32_t p = it.p; p < it.end && j < mult; p = run_next(it, p + 1, unused)) {
                pos[0] = p;
                one();
            }
        }
    } else if (odo_first<NC>(g, P, B, st, pos, false, aqe, akey)) {
        // every combination, in_time_order deciding: the windows pay off in
        // close_mult, which meets every complete mapping, while only mappings
        // with embeddings get here
        do {
            one();
        } while (j < mult && odo_next<NC>(g, P, B, st, pos, false, aqe, akey));
    }
}

// Emits every embedding of a complete vertex mapping, reserving its places
// with one global atomic per query and wave. All lanes of the wave must call
// this together (used where complete mappings are rare: 2-vertex queries).
template <int NC>
__device__ void emit_complete(const GraphView& g, const SeedPlan& P, const Bind& B, const uint32_t* st,
                              uint32_t aqe, uint64_t akey, bool active, const PhaseOut& po, BlockAcc& A,
                              Cnt& K) {
    const uint64_t mult = active ? close_mult<NC>(g, P, B, st, K.probes, aqe, akey) : 0u;
    const uint32_t q = P.q;
    const uint64_t pos = grouped_reserve(mult != 0, q, mult, po.count);
    uint64_t dA = 0, dB = 0;
    if (mult) emit_tuples<NC>(g, P, B, st, mult, aqe, akey, pos, po, K, dA, dB);
    grouped_digest(mult != 0, q, dA, dB, A.dig);
}

// Block b of nb -> tile index, so that consecutive tiles run on one XCD
// (workgroups are dealt to the 8 XCDs round robin; each XCD has its own L2).
__device__ inline uint32_t xcd_tile(uint32_t b, uint32_t nb) {
    const uint32_t x = b & 7u, i = b >> 3;
    const uint32_t q = nb >> 3, rmd = nb & 7u;
    return x * q + min(x, rmd) + i;
}

// Largest r in [a, b) with off[r] <= t (off[a] <= t is required).
__device__ inline uint32_t row_of(const uint64_t* off, uint32_t a, uint32_t b, uint64_t t) {
    while (a + 1 < b) {
        const uint32_t m = (a + b) >> 1;
        if (off[m] <= t)
            a = m;
        else
            b = m;
    }
    return a;
}

// Start rows. Each row takes the static order, or the fixed variant; rows
// whose order the decision kernel settles (learned choice, traces) are
// listed in g.dec as (row << 32 | index into slots).
// Block (x, y) takes slots [256x, 256x + 256) against plans [ppb * y, ppb * y
// + ppb), ppb <= SR_MAX_PPB. Few (slot, plan) pairs pass the edgeMatcher bit,
// and they are spread thinly over the waves, so the block works in two
// passes: the first tests the bit of every pair (the slot's matcher word is
// re-read only when the plan moves to another word) and lists the passing
// pairs in LDS; the second runs the dependent loads (endpoints, filters,
// start-level closing edges, row writes) over that list, 256 pairs per step,
// each lane with its own plan.
constexpr uint32_t SR_MAX_PPB = 32;

template <int NC>
__global__ __launch_bounds__(MN_BLOCK) void k_seed_rows(GraphView g, const uint32_t* __restrict__ slots,
                                                        uint32_t n, uint32_t n_plans, uint32_t ppb, RowsView R,
                                                        uint32_t* n_rows, PhaseOut po, const uint32_t* err) {
    __shared__ BlockAcc A;
    __shared__ uint32_t s_slot[MN_BLOCK];
    __shared__ uint16_t s_pair[MN_BLOCK * SR_MAX_PPB];  // lane | plan offset << 8, grouped by plan
    __shared__ uint32_t s_cnt[SR_MAX_PPB];
    __shared__ uint32_t s_n;
    if (threadIdx.x < SR_MAX_PPB) s_cnt[threadIdx.x] = 0;
    acc_init(A, 2 * po.n_q, err);  // ends with a barrier
    const uint32_t i = blockIdx.x * MN_BLOCK + threadIdx.x;
    const bool live = i < n && !A.dead;
    const uint32_t slot = live ? slots[i] : 0u;
    s_slot[threadIdx.x] = slot;
    const uint32_t p0 = blockIdx.y * ppb, p1 = min(n_plans, p0 + min(ppb, SR_MAX_PPB));
    // pass 1: the edgeMatcher bit of every (slot, plan) pair, counted per plan
    uint32_t word = 0, word_at = 0xFFFFFFFFu, hits = 0;
    for (uint32_t pi = p0; pi < p1; pi++) {  // block-uniform
        const SeedPlan& P = g.plans[pi];
        const uint32_t bit = P.debi_base + P.j;
        if ((bit >> 5) != word_at) {  // uniform
            word_at = bit >> 5;
            word = live ? g.s_debi[(size_t)slot * g.debi_words + word_at] : 0u;
        }
        const bool hit = (word >> (bit & 31)) & 1u;
        hits |= (uint32_t)hit << (pi - p0);
        const uint64_t bal = __ballot(hit);
        if (bal && __lane_id() == 0) atomicAdd(&s_cnt[pi - p0], (uint32_t)__popcll(bal));
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // at most 32 plans: exclusive offsets, serially
        uint32_t run = 0;
        for (uint32_t k = 0; k < p1 - p0; k++) {
            const uint32_t c = s_cnt[k];
            s_cnt[k] = run;
            run += c;
        }
        s_n = run;
    }
    __syncthreads();
    // the passing pairs, plan by plan, so that rows of one plan stay together
    for (uint32_t pi = p0; pi < p1; pi++) {  // block-uniform
        const bool hit = (hits >> (pi - p0)) & 1u;
        const uint64_t bal = __ballot(hit);
        if (bal) {
            uint32_t base = 0;
            if (__lane_id() == 0) base = atomicAdd(&s_cnt[pi - p0], (uint32_t)__popcll(bal));
            base = __shfl(base, 0, MN_WAVE);
            if (hit)
                s_pair[base + (uint32_t)__popcll(bal & lanemask_lt())] =
                    (uint16_t)(threadIdx.x | ((pi - p0) << 8));
        }
    }
    __syncthreads();
    const uint32_t m = s_n;
    Cnt K = {};
    constexpr int NA = NC > 0 ? NC : 1;
    // pass 2: the listed pairs, densely
    for (uint32_t k0 = 0; k0 < m; k0 += MN_BLOCK) {  // block-uniform
        const uint32_t k = k0 + threadIdx.x;
        bool ok = k < m;
        const uint32_t e = ok ? s_pair[k] : 0u;
        const uint32_t lane = e & 0xFFu, pslot = s_slot[lane];
        const SeedPlan& P = g.plans[p0 + (e >> 8)];
        uint32_t s = 0, d = 0;
        if (ok) {
            s = g.s_src[pslot];
            d = g.s_dst[pslot];
            K.vf += 2;
            const bool loop_ok = !(P.sem == MN_SEM_ISO && s == d);
            const bool vf_ok = vf_bit(g, s, P.vf_base + P.qa) && vf_bit(g, d, P.vf_base + P.qb);
            K.vfrej += loop_ok && !vf_ok ? 1u : 0u;
            ok = loop_ok && vf_ok;
        }
        Bind B;
        B.R = R;
        B.row = false;
        B.r = 0;
        B.qa = P.qa;
        B.fa = s;
        B.qb = P.qb;
        B.fb = d;
        B.skey = ok ? g.s_key[pslot] : 0ull;
        B.cv = 0xFF;
        B.fw = 0;
        uint32_t st[NA];
#pragma unroll
        for (uint32_t c = 0; c < NA; c++) {
            st[c] = 0;
            if (ok && c < (uint32_t)NC && c < P.c0_end) {
                const CloseDesc cd = P.close[c];
                st[c] = close_find(g, cd, B.f(cd.other), B.f(cd.nv), K.probes);
                if (st[c] == NO_RUN) ok = false;
            }
        }
        if (ok) K.seeds++;
        // 2-vertex queries: the pair is already a complete mapping (every
        // lane of the wave takes part in the call)
        emit_complete<NC>(g, P, B, st, 0xFF, 0ull, ok && P.n_levels == 0, po, A, K);
        const bool to_row = ok && P.n_levels != 0;
        // does the decision kernel settle this pair's rows?
        const bool decide = g.dec && (g.tr_cap || (g.sched_mode == MN_SCHED_LEARNED && P.n_var > 1));
        uint32_t var = 0;
        if (!decide && g.sched_mode >= MN_SCHED_FIXED && g.sched_mode - MN_SCHED_FIXED < P.n_var)
            var = g.sched_mode - MN_SCHED_FIXED;
        const uint64_t bal = __ballot(to_row);
        uint32_t base = 0;
        if (__lane_id() == 0 && bal) base = atomicAdd(n_rows, (uint32_t)__popcll(bal));
        base = __shfl(base, 0, MN_WAVE);
        uint32_t r = MN_INVALID;
        if (to_row) {
            r = base + (uint32_t)__popcll(bal & lanemask_lt());
            if (r < R.cap) {
                wcol(R, 0, r, P.vars[var]);
                wcol(R, 1 + P.qa, r, s);
                wcol(R, 1 + P.qb, r, d);
                wkey(R, P.j, r, B.skey);
#pragma unroll
                for (uint32_t c = 0; c < NA; c++)
                    if (c < (uint32_t)NC && c < P.c0_end) {
                        const CloseDesc cd = P.close[c];
                        wcol(R, 1 + R.wv + cd.qe, r, st[c]);
                        wkey(R, cd.qe, r, close_word(g, cd, st[c], B.f(cd.other), B.f(cd.nv), K.probes));
                    }
                if (R.trace) wcol(R, 1 + R.wv + R.we, r, MN_INVALID);
                K.rows++;
            } else {
                r = MN_INVALID;  // rows past the buffer are counted, not written: the host grows it and runs again
            }
        }
        const bool listed = decide && r != MN_INVALID;
        const uint64_t lb = __ballot(listed);
        if (lb) {
            uint32_t lbase = 0;
            if (__lane_id() == 0) lbase = atomicAdd(g.dec_n, (uint32_t)__popcll(lb));
            lbase = __shfl(lbase, 0, MN_WAVE);
            if (listed)
                g.dec[lbase + (uint32_t)__popcll(lb & lanemask_lt())] =
                    ((uint64_t)r << 32) | (blockIdx.x * MN_BLOCK + lane);
        }
    }
    acc_flush(A, K, 2 * po.n_q, po.stats, po.digest);
}

// Settles the order of the listed start rows (four lanes per row, lane v for
// order v): features of each order, the network's prediction in learned
// mode, the trace entry when tracing. Rows hold their static plan on entry.
// The grid strides over min(*dec_n, cap) rows.
template <bool LEARN>
__global__ __launch_bounds__(MN_BLOCK) void k_decide(GraphView g, RowsView R, const uint32_t* __restrict__ slots,
                                                     uint32_t cap, int phase) {
    __shared__ sched::NetVec V;
    __shared__ __align__(16) uint16_t s_xs[LEARN ? MN_BLOCK / MN_WAVE : 1][MN_WAVE * sched::XS_STRIDE];
    sched::NetFrag F;
    if (LEARN) {
        const uint16_t* w = g.sched_w;
        auto W = [w](uint32_t i) { return w[i]; };
        sched::load_frag(F, W);
        sched::load_vec(V, W);
        __syncthreads();
    }
    const uint32_t total = min(*g.dec_n, cap);
    constexpr uint32_t RPB = MN_BLOCK / MN_NVAR;  // rows per block and pass
    const uint32_t v = threadIdx.x % MN_NVAR;
    for (uint32_t k0 = blockIdx.x * RPB; k0 < total; k0 += gridDim.x * RPB) {  // uniform per block
        const uint32_t k = k0 + threadIdx.x / MN_NVAR;
        const bool on = k < total;
        uint32_t r = 0, i = 0;
        const SeedPlan* P = g.plans;
        if (on) {
            const uint64_t e = g.dec[k];
            r = (uint32_t)(e >> 32);
            i = (uint32_t)e;
            P = &g.plans[rcol(R, 0, r)];
        }
        const bool has = on && v < P->n_var;
        float x[MN_MLP_IN];
#pragma unroll
        for (int f = 0; f < MN_MLP_IN; f++) x[f] = 0.0f;
        if (has) {
            const uint32_t slot = slots[i];
            sched::features(g, g.plans[P->vars[v]], rcol(R, 1 + P->qa, r), rcol(R, 1 + P->qb, r), g.s_lab[slot], x);
        }
        float y = has ? 0.0f : 3.4e38f;
        if (LEARN) {  // the whole block evaluates together (the loop is uniform per block)
            const float p = sched::eval_wave(F, V, x, s_xs[threadIdx.x / MN_WAVE]);
            if (has) y = p;
        }
        // the order of the row: smallest prediction (lowest order on ties),
        // or the fixed variant, or the static order
        uint32_t best = v;
        float by = y;
#pragma unroll
        for (int m = 1; m < MN_NVAR; m <<= 1) {
            const float oy = __shfl_xor(by, m, MN_NVAR);
            const uint32_t ob = __shfl_xor(best, m, MN_NVAR);
            if (oy < by || (oy == by && ob < best)) {
                by = oy;
                best = ob;
            }
        }
        uint32_t var = 0;
        if (LEARN) {  // another order must promise clearly less work than the static one
            const float y0 = __shfl(y, (int)(__lane_id() & ~(MN_NVAR - 1u)), MN_WAVE);
            var = by < y0 - SCHED_MARGIN ? best : 0u;
        }
        else if (g.sched_mode >= MN_SCHED_FIXED && on && g.sched_mode - MN_SCHED_FIXED < P->n_var)
            var = g.sched_mode - MN_SCHED_FIXED;
        // trace entry: one per row, taken by its lane 0
        uint32_t te = MN_INVALID;
        if (g.tr_cap) {
            const bool lead = on && v == 0;
            const uint64_t tb = __ballot(lead);
            uint32_t tbase = 0;
            if (__lane_id() == 0 && tb) tbase = atomicAdd(g.tr_n + phase, (uint32_t)__popcll(tb));
            tbase = __shfl(tbase, 0, MN_WAVE);
            const uint32_t e = tbase + (uint32_t)__popcll(tb & lanemask_lt());
            if (lead && e < g.tr_cap) te = (uint32_t)phase * g.tr_cap + e;
            te = __shfl(te, (int)(__lane_id() & ~(MN_NVAR - 1u)), MN_WAVE);
            if (on && te != MN_INVALID) {
                float* dst = g.tr_x + ((size_t)te * MN_NVAR + v) * MN_MLP_IN;
#pragma unroll
                for (int f = 0; f < MN_MLP_IN; f++) dst[f] = x[f];
            }
        }
        if (on && v == 0) {
            if (te != MN_INVALID) {
                g.tr_code[te] = ((uint64_t)phase << 62) | ((uint64_t)var << 56) |
                                ((uint64_t)P->vars[0] << 32) | (uint64_t)(g.tr_base + i);
                g.tr_work[te] = 1ull;
                wcol(R, 1 + R.wv + R.we, r, te);
            }
            wcol(R, 0, r, P->vars[var]);
        }
    }
}

// The fields of a plan the expansion reads for every candidate, from one
// 16-byte load of the plan's header.
struct PlanHead {
    uint32_t q, n_qe, n_levels, sem, n_close, temporal, vf_base;
};

__device__ inline PlanHead plan_head_of(const uint4& h) {
    PlanHead H;
    H.q = h.x & 0xFFFFu;
    H.n_qe = h.x >> 24;
    H.n_levels = (h.y >> 16) & 0xFFu;
    H.sem = h.z & 0xFFu;
    H.n_close = (h.z >> 8) & 0xFFu;
    H.temporal = h.z >> 24;
    H.vf_base = h.w;
    return H;
}

__device__ inline PlanHead plan_head(const SeedPlan* P) { return plan_head_of(*reinterpret_cast<const uint4*>(P)); }

// 16 bytes of a plan read with one load. Left alone, the compiler splits
// such a load into one narrow load per field the caller uses, and the
// expansion's time goes with its count of load instructions; the empty asm
// takes every word, so the load stays whole.
__device__ inline uint4 load_whole16(const void* p) {
    uint4 v = *reinterpret_cast<const uint4*>(p);
    asm("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w));
    return v;
}

// Level L of plan P, one 16-byte load.
__device__ inline LevelDesc load_level(const SeedPlan* P, uint32_t L) {
    return __builtin_bit_cast(LevelDesc, load_whole16(&P->lv[L]));
}

// 16 bytes at an address every active lane of the wave shares, read by the
// scalar unit: the vector memory path, which bounds the expansion by the
// data it returns per lane, is left out. Plans are not written while a
// kernel that reads them runs.
__device__ inline uint4 load_uniform16(const void* p) {
    const __attribute__((address_space(4))) uint32_t* q = (const __attribute__((address_space(4))) uint32_t*)p;
    return make_uint4(q[0], q[1], q[2], q[3]);
}

// 16 bytes at byte `at` (the same for every lane) of plan pl: by the scalar
// unit when every active lane of the wave takes the same plan, else one
// vector load per lane.
__device__ inline uint4 plan_words(const SeedPlan* plans, uint32_t pl, uint32_t at) {
    const uint32_t pl0 = __builtin_amdgcn_readfirstlane(pl);
    if (__ballot(pl != pl0) == 0) return load_uniform16(reinterpret_cast<const char*>(plans + pl0) + at);
    return load_whole16(reinterpret_cast<const char*>(plans + pl) + at);
}

// Level L and header of plan P. When every active lane of the wave takes the
// same plan (the rows of one parent sit next to each other, so most waves
// do), both come from scalar loads; otherwise each lane loads its own.
__device__ inline void plan_level(const SeedPlan* plans, uint32_t pl, uint32_t L, LevelDesc& lv, PlanHead& H) {
    const uint32_t pl0 = __builtin_amdgcn_readfirstlane(pl);
    if (__ballot(pl != pl0) == 0) {
        const SeedPlan* P = plans + pl0;
        lv = __builtin_bit_cast(LevelDesc, load_uniform16(&P->lv[L]));
        H = plan_head_of(load_uniform16(P));
    } else {
        // both loads issued before either is waited for: one asm takes all
        // their words, so each stays one 16-byte load (see load_whole16)
        uint4 a = *reinterpret_cast<const uint4*>(&plans[pl].lv[L]);
        uint4 h = *reinterpret_cast<const uint4*>(plans + pl);
        asm("" : "+v"(a.x), "+v"(a.y), "+v"(a.z), "+v"(a.w), "+v"(h.x), "+v"(h.y), "+v"(h.z), "+v"(h.w));
        lv = __builtin_bit_cast(LevelDesc, a);
        H = plan_head_of(h);
    }
}

// Closing edge c of plan pl, one 16-byte load (scalar when the wave's
// active lanes share the plan).
__device__ inline CloseDesc load_close(const SeedPlan* plans, uint32_t pl, uint32_t c) {
    return __builtin_bit_cast(CloseDesc, plan_words(plans, pl, offsetof(SeedPlan, close) + c * sizeof(CloseDesc)));
}

// Byte i (< 16) of a 16-byte vector.
__device__ inline uint32_t byte_of(const uint4& v, uint32_t i) {
    const uint32_t w = i < 8 ? (i < 4 ? v.x : v.y) : (i < 12 ? v.z : v.w);
    return (w >> (8 * (i & 3))) & 0xFFu;
}

// Exclusive count of the set bits of `mask` below this lane.
__device__ inline uint32_t lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Stores a key of an emitted embedding: a global-memory store marked
// non-temporal (the tuples stream out and are not read again here).
__device__ inline void store_key(uint64_t* p, uint64_t v) {
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) uint64_t*)p);
}

// Both digest chains over the keys of query edges [0, aqe) of row r (all tree
// edges of a plan with no closing edge), from query q's seeds.
__device__ inline void digest_prefix(const RowsView& R, uint32_t r, uint32_t q, uint32_t aqe, uint64_t& hA,
                                     uint64_t& hB) {
    hA = mn_mix64(MN_SEED_A ^ (uint64_t)q);
    hB = mn_mix64(MN_SEED_B ^ (uint64_t)q);
    for (uint32_t k0 = 0; k0 < aqe; k0 += 8) {
        uint64_t kv[8];
#pragma unroll
        for (uint32_t i = 0; i < 8; i++) kv[i] = k0 + i < aqe ? rkey(R, k0 + i, r) : 0ull;
#pragma unroll
        for (uint32_t i = 0; i < 8; i++)
            if (k0 + i < aqe) {
                hA = mn_mix64(hA + kv[i]);
                hB = mn_mix64(hB + kv[i]);
            }
    }
}

// Device-sized levels fold two bookkeeping steps in here: thread 0 compares
// the row count with the buffer (note[0] = 1 when *n_dev > n, note[1] = the
// largest count seen) and zeroes the next level's row counter (zero_next).
__global__ __launch_bounds__(MN_BLOCK) void k_level_range(GraphView g, RowsView R, uint32_t n,
                                                          const uint32_t* n_dev, uint32_t L,
                                                          uint32_t* __restrict__ lo, uint32_t* __restrict__ cnt,
                                                          EnumStats* stats, uint32_t* zero_next,
                                                          unsigned long long* note, const uint32_t* err) {
    __shared__ BlockAcc A;
    if (n_dev) {
        const uint32_t nd = *n_dev;
        if (note && blockIdx.x == 0 && threadIdx.x == 0) {
            if (nd > n) note[0] = 1ull;
            atomicMax(note + 1, (unsigned long long)nd);
        }
        n = min(n, nd);
    }
    if (zero_next && blockIdx.x == 0 && threadIdx.x == 0) *zero_next = 0u;
    if (blockIdx.x * MN_BLOCK >= n) return;  // the same for the whole block
    acc_init(A, 0, err);
    Cnt K = {};
    // the grid is bounded (the row count may be known on the device only):
    // it strides over the rows
    for (uint32_t r = blockIdx.x * MN_BLOCK + threadIdx.x; r < n && !A.dead; r += gridDim.x * MN_BLOCK) {
        const uint32_t pl = rcol(R, 0, r);
        const LevelDesc lv =
            __builtin_bit_cast(LevelDesc, plan_words(g.plans, pl, offsetof(SeedPlan, lv) + L * sizeof(LevelDesc)));
        if (R.hpre) {
            // a row whose embeddings end at this level and are all tree edges:
            // its digest chains up to the anchor edge, once for all its candidates
            const PlanHead H = plan_head_of(plan_words(g.plans, pl, 0));
            if (L + 1 == H.n_levels && H.n_close == 0 && !H.temporal) {
                uint64_t hA, hB;
                digest_prefix(R, r, H.q, lv.qe, hA, hB);
                R.hpre[r] = hA;
                R.hpre[R.cap + r] = hB;
            }
        }
        uint32_t a = 0, b = 0;
        if (!lv.empty) {
            const uint32_t x = rcol(R, 1 + lv.from, r);
            const uint32_t* of = g.offs(lv.dir);
            const uint32_t s0 = of[x], s1 = of[x + 1];
            K.range_probes += 2;
            if (lv.whole) {
                a = s0;
                b = s1;
            } else {
                run_bounds_c(g.adjs(lv.dir), s0, s1, lv.key_lo, lv.key_hi, a, b, K.range_probes);
            }
        }
        lo[r] = a;
        cnt[r] = b - a;
        if (R.trace) {  // search work below the row's start row
            const uint32_t e = rcol(R, 1 + R.wv + R.we, r);
            if (e != MN_INVALID && b > a) atomicAdd(g.tr_work + e, (unsigned long long)(b - a));
        }
    }
    acc_flush(A, K, 0, stats, nullptr);
}

// Records a device count against a capacity: note[0] = 1 when *count > cap,
// note[1] = the largest count seen.
__global__ void k_note_count(const uint32_t* count, uint64_t cap, unsigned long long* note) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const unsigned long long n = *count;
        if (n > cap) note[0] = 1ull;
        atomicMax(note + 1, n);
    }
}

// Candidates [c0, cend) of one expansion, cend = min(c1, *T_dev) when the
// total is on the device, and the number of tiles that cover them.
__device__ inline uint64_t expand_end(uint64_t c1, const uint64_t* T_dev) { return T_dev ? min(c1, *T_dev) : c1; }

__host__ __device__ inline uint32_t expand_tiles(uint64_t c0, uint64_t cend, uint32_t tile) {
    return cend > c0 ? (uint32_t)((cend - c0 + tile - 1) / tile) : 0u;
}

// First row of every expansion tile: tile_row[i] = row of candidate
// c0 + i * tile for i < nt, tile_row[nt] = row of candidate cend - 1.
// In the device-sized form (n_dev, cnt and T_dev given) every thread derives
// the candidate total from the last row's offset and count, thread 0 stores
// it in *T_dev for the expansion and records it in `note` (note[0] = 1 when
// it exceeds c1, the candidates the next level's rows can take; note[1] = the
// largest total seen), so the host can grow and re-run.
__global__ __launch_bounds__(MN_BLOCK) void k_partition(const uint64_t* __restrict__ off,
                                                        const uint32_t* __restrict__ cnt, uint32_t n,
                                                        const uint32_t* n_dev, uint64_t c0, uint64_t c1,
                                                        uint64_t* T_dev, uint32_t tile,
                                                        uint32_t* __restrict__ tile_row, unsigned long long* note) {
    if (n_dev) n = min(n, *n_dev);
    const uint32_t i = blockIdx.x * MN_BLOCK + threadIdx.x;
    uint64_t cend = c1;
    if (T_dev) {
        const uint64_t T = n ? off[n - 1] + cnt[n - 1] : 0ull;
        cend = min(c1, T);
        if (i == 0) {
            *T_dev = T;
            if (note) {
                if (T > c1) note[0] = 1ull;
                atomicMax(note + 1, (unsigned long long)T);
            }
        }
    }
    const uint32_t nt = expand_tiles(c0, cend, tile);
    if (nt == 0 || i > nt) return;
    const uint64_t t = i < nt ? c0 + (uint64_t)i * tile : cend - 1;
    tile_row[i] = row_of(off, 0, n, t);
}

// Completes a level's candidate offsets and partitions them in one launch.
// off holds exclusive sums within tiles of MN_SCAN_TILE rows and sums[b] the
// total of tile b (nb tiles): every block adds the totals in front of it and
// sums all of them for the level's total T. Each row with candidates [o, o +
// cnt) inside [c0, cend), cend = min(c1, T), writes tile_row[i] for every
// expansion tile i whose first candidate c0 + i * tile it holds, and
// tile_row[nt] if it holds cend - 1 (nt tiles cover [c0, cend)): the row of a
// candidate is the one that contains it, as k_partition finds by search.
// Block 0 stores T and notes it against c1.
__global__ __launch_bounds__(MN_BLOCK) void k_offsets_partition(const uint32_t* __restrict__ cnt,
                                                                uint64_t* __restrict__ off,
                                                                const uint64_t* __restrict__ sums, uint32_t nb,
                                                                uint32_t n, const uint32_t* n_dev, uint64_t c0,
                                                                uint64_t c1, uint64_t* T_dev, uint32_t tile,
                                                                uint32_t* __restrict__ tile_row,
                                                                unsigned long long* note) {
    __shared__ uint64_t s_pre[MN_BLOCK / MN_WAVE], s_tot[MN_BLOCK / MN_WAVE];
    if (n_dev) n = min(n, *n_dev);
    // the grid follows the buffer's capacity; only tiles that hold rows count,
    // and blocks past them leave (block 0 stores the total)
    const uint32_t nbu = min(nb, (uint32_t)(((uint64_t)n + MN_SCAN_TILE - 1) / MN_SCAN_TILE));
    if (blockIdx.x > 0 && blockIdx.x >= nbu) return;  // the same for the whole block
    uint64_t pre = 0, tot = 0;
    for (uint32_t i = threadIdx.x; i < nbu; i += MN_BLOCK) {
        const uint64_t v = sums[i];
        tot += v;
        if (i < blockIdx.x) pre += v;
    }
    pre = wave_sum64(pre);
    tot = wave_sum64(tot);
    if (__lane_id() == 0) {
        s_pre[threadIdx.x / MN_WAVE] = pre;
        s_tot[threadIdx.x / MN_WAVE] = tot;
    }
    __syncthreads();
    uint64_t add = 0, T = 0;
    for (uint32_t w = 0; w < MN_BLOCK / MN_WAVE; w++) {
        add += s_pre[w];
        T += s_tot[w];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *T_dev = T;
        if (note) {
            if (T > c1) note[0] = 1ull;
            atomicMax(note + 1, (unsigned long long)T);
        }
    }
    const uint64_t cend = min(c1, T);
    const uint32_t nt = expand_tiles(c0, cend, tile);
    const size_t base = (size_t)blockIdx.x * MN_SCAN_TILE;
    for (uint32_t k = threadIdx.x; k < MN_SCAN_TILE; k += MN_BLOCK) {
        const size_t r = base + k;
        if (r >= n) break;
        const uint64_t o = off[r] + add;
        off[r] = o;
        const uint32_t m = cnt[r];
        const uint64_t a = max(o, c0), b = min(o + m, cend);
        if (a >= b) continue;  // no candidates in the window
        for (uint64_t i = (a - c0 + tile - 1) / tile; c0 + i * tile < b; i++) tile_row[i] = (uint32_t)r;
        if (b == cend) tile_row[nt] = (uint32_t)r;
    }
}

constexpr uint32_t NO_LOC = 0xFFFFFFFFu;

// Largest a in [0, span) with rel[a] <= i (rel[0] = 0), searched in LDS over
// the rows' first candidates relative to the tile's first (32 bits).
__device__ inline uint32_t row_in_lds(const uint32_t* rel, uint32_t span, uint32_t i) {
    uint32_t a = 0, b = span;
    while (a + 1 < b) {
        const uint32_t m = (a + b) >> 1;
        if (rel[m] <= i)
            a = m;
        else
            b = m;
    }
    return a;
}

// The same over global offsets [lo, hi) (tiles whose rows do not fit in LDS).
__device__ inline uint32_t row_in_global(const uint64_t* off, uint32_t a, uint32_t b, uint64_t t, uint64_t& o) {
    uint64_t oa = off[a];
    while (a + 1 < b) {
        const uint32_t m = (a + b) >> 1;
        const uint64_t om = off[m];
        if (om <= t) {
            a = m;
            oa = om;
        } else {
            b = m;
        }
    }
    o = oa;
    return a;
}

// One complete mapping with a single embedding whose query edges other than
// the anchor aqe are all tree edges (no closing edge, no temporal order): the
// tuple is the row's tree keys with akey at aqe. Both digest chains continue
// from the row's prefix (the edges before aqe); the tuple is written at `row`
// when emitting.
__device__ inline void emit_tree_tuple(const RowsView& R, uint32_t r, uint32_t nqe, uint32_t aqe, uint64_t akey,
                                       uint64_t* row, bool write, Cnt& K, uint64_t& dA, uint64_t& dB) {
    uint64_t hA = R.hpre[r], hB = R.hpre[R.cap + r];
    for (uint32_t k0 = 0; k0 < nqe; k0 += 8) {  // one pass for up to 8 edges
        uint64_t kv[8];
#pragma unroll
        for (uint32_t i = 0; i < 8; i++) {
            const uint32_t k = k0 + i;
            kv[i] = k < nqe && k != aqe ? rkey(R, k, r) : akey;
        }
#pragma unroll
        for (uint32_t i = 0; i < 8; i++) {
            const uint32_t k = k0 + i;
            if (k >= aqe && k < nqe) {
                hA = mn_mix64(hA + kv[i]);
                hB = mn_mix64(hB + kv[i]);
            }
        }
        if (write) {
#pragma unroll
            for (uint32_t i = 0; i < 8; i++)
                if (k0 + i < nqe) store_key(row + k0 + i, kv[i]);
        }
    }
    K.keys += nqe;
    K.tuples++;
    dA += hA;
    dB += hB;
}

// Embeddings of a complete mapping at the last level of a plan with closing
// edges and no temporal order: the product of each closing edge's instances,
// from the row's words for edges resolved at earlier levels (close_word) and
// by a walk for those this level resolves (st[c], its new vertex mapped to w).
template <int NC>
__device__ inline uint64_t closed_mult(const GraphView& g, uint32_t pl, const RowsView& R, uint32_t r,
                                       const LevelDesc& lv, uint32_t n_close, const uint32_t* st, uint32_t w,
                                       uint32_t& probes) {
    constexpr int NA = NC > 0 ? NC : 1;
    uint64_t mult = 1;
#pragma unroll
    for (uint32_t c = 0; c < NA; c++) {
        if (c < (uint32_t)NC && c < n_close) {
            const CloseDesc cd = load_close(g.plans, pl, c);
            uint32_t n;
            if (c >= lv.c_begin && c < lv.c_end) {
                const RunIt it = run_open(g, cd, st[c], rcol(R, 1 + cd.other, r), w);
                n = 1;
                for (uint32_t x = run_next(it, it.p + 1, probes); x < it.end; x = run_next(it, x + 1, probes)) n++;
            } else {
                n = close_word_count(rkey(R, cd.qe, r));
            }
            mult *= n;
        }
    }
    return mult;
}

// The one embedding of a complete mapping whose closing edges each have one
// instance (no temporal order): the row's keys, the closing edges this level
// resolves at their first accepted instances and akey at the anchor aqe;
// both digest chains from query q's seeds. Written at `row` when emitting.
template <int NC>
__device__ inline void emit_closed_tuple(const GraphView& g, uint32_t pl, const RowsView& R, uint32_t r,
                                         uint32_t q, uint32_t nqe, const LevelDesc& lv, const uint32_t* st,
                                         uint64_t akey, uint64_t* row, bool write, Cnt& K, uint64_t& dA,
                                         uint64_t& dB) {
    constexpr int NA = NC > 0 ? NC : 1;
    uint32_t hq[NA];
    uint64_t hk[NA];
#pragma unroll
    for (uint32_t c = 0; c < NA; c++) {
        hq[c] = 0xFFu;
        hk[c] = 0;
        if (c < (uint32_t)NC && c >= lv.c_begin && c < lv.c_end) {
            const CloseDesc cd = load_close(g.plans, pl, c);
            const bool sw = (st[c] & RUN_SWAP) != 0;
            hq[c] = cd.qe;
            hk[c] = g.keys(sw ? 1u - cd.dir : (uint32_t)cd.dir)[st[c] & ~RUN_SWAP];
        }
    }
    uint64_t hA = mn_mix64(MN_SEED_A ^ (uint64_t)q), hB = mn_mix64(MN_SEED_B ^ (uint64_t)q);
    for (uint32_t k0 = 0; k0 < nqe; k0 += 8) {  // one pass for up to 8 edges
        uint64_t kv[8];
#pragma unroll
        for (uint32_t i = 0; i < 8; i++) {
            const uint32_t k = k0 + i;
            kv[i] = k < nqe && k != lv.qe ? rkey(R, k, r) : akey;
#pragma unroll
            for (uint32_t c = 0; c < NA; c++)
                if (hq[c] == k) kv[i] = hk[c];
        }
#pragma unroll
        for (uint32_t i = 0; i < 8; i++)
            if (k0 + i < nqe) {
                hA = mn_mix64(hA + kv[i]);
                hB = mn_mix64(hB + kv[i]);
            }
        if (write) {
#pragma unroll
            for (uint32_t i = 0; i < 8; i++)
                if (k0 + i < nqe) store_key(row + k0 + i, kv[i]);
        }
    }
    K.keys += nqe;
    K.tuples++;
    dA += hA;
    dB += hB;
}

// One block of BT threads tests a tile of BT x ITEMS candidates in two
// passes. Pass 1 runs the filters and gives every survivor a place inside the
// block (LDS counters per query for embeddings, one for new rows); one global
// atomic per query and block then reserves the block's places; pass 2 writes
// rows and embeddings. Contended device-scope atomics (they serialise across
// the XCDs) drop from one per wave and item to one per block.
// What pass 1 learns about a candidate (its row, entry position, neighbour
// and closing-run starts) waits in LDS for pass 2. Each lane keeps the
// digests of the embeddings it emits in registers and the block reduces them
// once; waves whose survivors each have one embedding of one query take their
// places with a ballot count instead of a scan.
template <int NC, bool ROWS, bool EMIT, uint32_t ITEMS, uint32_t BT>
__global__ __launch_bounds__(BT, ex_min_waves(BT, NC)) void k_expand(GraphView g, RowsView in, uint32_t n_in,
                                                     const uint32_t* __restrict__ lo,
                                                     const uint64_t* __restrict__ off,
                                                     const uint32_t* __restrict__ tile_row, uint64_t c0,
                                                     uint64_t c1, const uint64_t* T_dev, uint32_t L,
                                                     RowsView out, uint32_t* n_out, PhaseOut po,
                                                     const uint32_t* err) {
    constexpr int NA = NC > 0 ? NC : 1;
    constexpr uint32_t EX_TILE = BT * ITEMS;
    constexpr uint32_t EX_LDS_ROWS = EX_TILE + 1;
    // the tile's rows when they fit: first candidate relative to the tile's
    // (the first row's is 0; d0 = how far it starts before the tile), first
    // adjacency position of the run, plan
    __shared__ uint32_t s_rel[EX_LDS_ROWS], s_lo[EX_LDS_ROWS];
    __shared__ uint16_t s_pl[EX_LDS_ROWS];
    __shared__ BlockAcc A;
    __shared__ uint32_t s_r[EX_TILE], s_p[EX_TILE], s_loc[EX_TILE], s_w[EX_TILE];
    __shared__ uint32_t s_st[NA][EX_TILE];
    __shared__ unsigned long long s_qn[MAXQ];  // places per query: counts, then global bases
    __shared__ uint32_t s_nrows, s_rbase;
    // one tile per block; the grid covers [c0, c1) (the host sizes c1 to the
    // grid), and blocks past the candidates present leave at once
    const uint64_t cend = expand_end(c1, T_dev);
    const uint32_t nt = expand_tiles(c0, cend, EX_TILE);
    if (blockIdx.x >= nt) return;  // the same for every thread of the block
    acc_init(A, EMIT ? 2 * po.n_q : 0, err);
    // the first nt blocks are dealt to the XCDs round robin; consecutive tiles
    // go to blocks of one XCD
    const uint32_t tile = xcd_tile(blockIdx.x, nt);
    const uint32_t ncol = 1 + in.wv + in.we + in.trace;
    Cnt K = {};
    const uint64_t t0 = c0 + (uint64_t)tile * EX_TILE;
    const uint64_t t1 = min(t0 + (uint64_t)EX_TILE, cend);
    const uint32_t rlo = tile_row[tile], rhi = tile_row[tile + 1] + 1;  // rows of this tile lie in [rlo, rhi)
    const uint32_t span = rhi - rlo;
    const bool staged = span <= EX_LDS_ROWS;
    const uint32_t d0 = (uint32_t)(t0 - off[rlo]);  // the runs' positions fit in 32 bits
    if (staged)
        for (uint32_t x = threadIdx.x; x < span; x += BT) {
            const uint32_t rr = rlo + x;
            const uint64_t o = off[rr];
            s_rel[x] = x ? (uint32_t)(o - t0) : 0u;  // rows after the first start inside the tile or past it
            s_lo[x] = lo[rr];
            s_pl[x] = (uint16_t)rcol(in, 0, rr);
        }
    if (EMIT)
        for (uint32_t x = threadIdx.x; x < po.n_q; x += BT) s_qn[x] = 0;
    if (threadIdx.x == 0) s_nrows = 0;
    __syncthreads();

    // ---- pass 1: filters and places inside the block
    for (uint32_t it = 0; it < ITEMS; it++) {
        const uint32_t idx = it * BT + threadIdx.x;
        const uint64_t t = t0 + idx;
        bool ok = t < t1 && !A.dead;
        uint32_t r = 0, w = 0, p = 0;
        LevelDesc lv = {};
        PlanHead H = {};
        uint32_t st[NA];
#pragma unroll
        for (uint32_t c = 0; c < NA; c++) st[c] = 0;
        const SeedPlan* P = g.plans;
        uint32_t pl = 0;  // plan of the candidate's row
        if (ok) {
            uint32_t base;
            if (staged) {
                const uint32_t a = row_in_lds(s_rel, span, idx);
                r = rlo + a;
                base = s_lo[a] + (a ? idx - s_rel[a] : idx + d0);  // position of the candidate in its run
                pl = s_pl[a];
            } else {
                uint64_t o;
                r = row_in_global(off, rlo, rhi, t, o);
                base = lo[r] + (uint32_t)(t - o);
                pl = rcol(in, 0, r);
            }
            P = &g.plans[pl];
            plan_level(g.plans, pl, L, lv, H);
            p = base;
            const uint64_t e = g.adjs(lv.dir)[p];
            K.entries++;
            w = ent_hi(e) & g.nbr_mask;
            if (lv.masked && (ent_lo(e) & MN_FLAG)) ok = false;
            if (ok && lv.need_vf) {
                K.vf++;
                ok = vf_bit(g, w, H.vf_base + lv.vtx);
                K.vfrej += ok ? 0u : 1u;
            }
            if (ok && H.sem == MN_SEM_ISO) {
                // the images of the L + 2 mapped query vertices, loaded together
                // (the trip count is the launch's, the same for every lane)
                const uint4 mv = plan_words(g.plans, pl, offsetof(SeedPlan, mapped));
                uint32_t img[MN_MAXQV];
#pragma unroll
                for (uint32_t m = 0; m < MN_MAXQV; m++)
                    if (m < L + 2) img[m] = rcol(in, 1 + byte_of(mv, m), r);
                bool clash = false;
#pragma unroll
                for (uint32_t m = 0; m < MN_MAXQV; m++)
                    if (m < L + 2) clash |= img[m] == w;
                ok = !clash;
            }
            if (ok && H.temporal && P->rank[lv.qe] >= 0) {
                // timestamps never decrease with keys, so the order of two
                // tree edges' keys must agree with the order of their ranks
                const uint64_t nk = g.keys(lv.dir)[p];
                const int rn = P->rank[lv.qe];
                for (uint32_t l = 0; l <= L && ok; l++) {
                    const uint32_t k = l == 0 ? P->j : P->lv[l - 1].qe;
                    const int rk = P->rank[k];
                    if (rk < 0 || rk == rn) continue;
                    const uint64_t kk = rkey(in, k, r);
                    if (rk < rn ? !(kk < nk) : !(nk < kk)) ok = false;
                }
            }
#pragma unroll
            for (uint32_t c = 0; c < NA; c++) {
                if (ok && c < (uint32_t)NC && c >= lv.c_begin && c < lv.c_end) {
                    const CloseDesc cd = load_close(g.plans, pl, c);
                    st[c] = close_find(g, cd, rcol(in, 1 + cd.other, r), w, K.probes);
                    if (st[c] == NO_RUN) ok = false;
                }
            }
        }
        const bool last = ok && (L + 1 == H.n_levels);
        const bool to_row = ok && !last;
        uint32_t loc = NO_LOC;
        if (ROWS) {
            const uint64_t bal = __ballot(to_row);
            uint32_t base = 0;
            if (__lane_id() == 0 && bal) base = atomicAdd(&s_nrows, (uint32_t)__popcll(bal));
            base = __shfl(base, 0, MN_WAVE);
            if (to_row) loc = base + lane_rank(bal);
        } else if (to_row) {
            set_err(err, MN_ERR_INTERNAL);  // the host launches ROWS wherever a plan continues
        }
        if (EMIT) {
            uint64_t mult = 0;
            if (last) {
                if (!H.temporal && (NC == 0 || H.n_close == 0)) {
                    mult = 1;
                } else if (NC <= 4 && !H.temporal) {
                    // (plans with more closing edges keep the general path's registers)
                    mult = closed_mult<NC>(g, pl, in, r, lv, H.n_close, st, w, K.probes);
                    if (mult == 1) w |= CK_ONE;  // pass 2 writes the one embedding from the row
                } else {
                    Bind B;
                    B.R = in;
                    B.row = true;
                    B.r = r;
                    B.qa = B.fa = B.qb = B.fb = 0;
                    B.skey = 0;
                    B.cv = lv.vtx;
                    B.fw = w;
#pragma unroll
                    for (uint32_t c = 0; c < NA; c++)
                        if (c < (uint32_t)NC && c < H.n_close && !(c >= lv.c_begin && c < lv.c_end))
                            st[c] = rcol(in, 1 + in.wv + load_close(g.plans, pl, c).qe, r);
                    mult = close_mult<NC>(g, *P, B, st, K.probes, lv.qe, H.temporal ? g.keys(lv.dir)[p] : 0ull);
                }
            }
            const bool has = mult != 0;
            const uint64_t hb = __ballot(has);
            if (hb) {  // uniform
                const uint32_t lead = (uint32_t)__ffsll((unsigned long long)hb) - 1;
                const uint32_t qlead = (uint32_t)__builtin_amdgcn_readlane((int)H.q, (int)lead);
                if (__ballot(has && (mult != 1 || H.q != qlead)) == 0) {
                    // one embedding per survivor, one query: a ballot count
                    unsigned long long b0 = 0;
                    if (__lane_id() == lead) b0 = atomicAdd(&s_qn[qlead], (unsigned long long)__popcll(hb));
                    const uint32_t basel = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b0, (int)lead);
                    if (has) loc = basel + lane_rank(hb);
                } else {
                    const uint64_t lpos = grouped_reserve(has, H.q, mult, s_qn);
                    if (has) loc = (uint32_t)lpos;
                }
            }
        } else if (last) {
            set_err(err, MN_ERR_INTERNAL);  // the host launches EMIT wherever a plan ends
        }
        if (t < t1) {
            s_loc[idx] = loc;
            s_r[idx] = r;
            s_p[idx] = p;
            s_w[idx] = w;
#pragma unroll
            for (uint32_t c = 0; c < NA; c++) s_st[c][idx] = st[c];
        }
    }
    __syncthreads();
    // ---- one global reservation per query (and one for rows) per block
    if (ROWS && threadIdx.x == 0 && s_nrows) s_rbase = atomicAdd(n_out, s_nrows);
    if (EMIT)
        for (uint32_t x = threadIdx.x; x < po.n_q; x += BT)
            if (s_qn[x]) s_qn[x] = atomicAdd(&po.count[x], s_qn[x]);
    __syncthreads();

    // ---- pass 2: write rows and embeddings at their places
    uint32_t dq = MAXQ;  // query of the lane's digest sums
    uint64_t dA = 0, dB = 0;
    for (uint32_t it = 0; it < ITEMS; it++) {
        const uint32_t idx = it * BT + threadIdx.x;
        const uint64_t t = t0 + idx;
        const uint32_t loc = t < t1 ? s_loc[idx] : NO_LOC;
        if (loc == NO_LOC) continue;
        const uint32_t r = s_r[idx], w = s_w[idx], p = s_p[idx];
        const uint32_t pl = staged ? (uint32_t)s_pl[r - rlo] : rcol(in, 0, r);
        const SeedPlan* P = &g.plans[pl];
        LevelDesc lv;
        PlanHead H;
        plan_level(g.plans, pl, L, lv, H);
        const uint64_t akey = g.keys(lv.dir)[p];
        const bool last = L + 1 == H.n_levels;
        uint32_t st[NA];
#pragma unroll
        for (uint32_t c = 0; c < NA; c++) st[c] = s_st[c][idx];
        if (ROWS && !last) {
            const uint32_t dst = s_rbase + loc;
            if (dst < out.cap) {
                // the row's columns and keys, eight loads in flight at a time
                for (uint32_t c0 = 0; c0 < ncol; c0 += 8) {
                    uint32_t v[8];
#pragma unroll
                    for (uint32_t i = 0; i < 8; i++) v[i] = c0 + i < ncol ? rcol(in, c0 + i, r) : 0u;
#pragma unroll
                    for (uint32_t i = 0; i < 8; i++)
                        if (c0 + i < ncol) wcol(out, c0 + i, dst, v[i]);
                }
                for (uint32_t k0 = 0; k0 < in.we; k0 += 8) {
                    uint64_t v[8];
#pragma unroll
                    for (uint32_t i = 0; i < 8; i++) v[i] = k0 + i < in.we ? rkey(in, k0 + i, r) : 0ull;
#pragma unroll
                    for (uint32_t i = 0; i < 8; i++)
                        if (k0 + i < in.we) wkey(out, k0 + i, dst, v[i]);
                }
                wcol(out, 1 + lv.vtx, dst, w);
                wkey(out, lv.qe, dst, akey);
                K.keys++;
#pragma unroll
                for (uint32_t c = 0; c < NA; c++)
                    if (c < (uint32_t)NC && c >= lv.c_begin && c < lv.c_end) {
                        const CloseDesc cd = load_close(g.plans, pl, c);
                        wcol(out, 1 + out.wv + cd.qe, dst, st[c]);
                        wkey(out, cd.qe, dst, close_word(g, cd, st[c], rcol(in, 1 + cd.other, r), w, K.probes));
                    }
                K.rows++;
            }  // rows past the buffer are counted, not written: the host grows it and runs again
        }
        if (EMIT && last) {
            const uint32_t q = H.q;
            if (q != dq) {  // the lane's sums so far belong to another query
                if (dq != MAXQ) {
                    atomicAdd(&A.dig[2 * dq], (unsigned long long)dA);
                    atomicAdd(&A.dig[2 * dq + 1], (unsigned long long)dB);
                }
                dq = q;
                dA = dB = 0;
            }
            const uint64_t pos = s_qn[q] + loc;
            if (!H.temporal && (NC == 0 || H.n_close == 0)) {
                const OutView& ov = po.outs[q];
                const bool write = po.emit && pos < ov.cap[po.phase];
                emit_tree_tuple(in, r, H.n_qe, lv.qe, akey, ov.keys[po.phase] + pos * H.n_qe, write, K, dA, dB);
            } else if (NC > 0 && NC <= 4 && (w & CK_ONE)) {
                const OutView& ov = po.outs[q];
                const bool write = po.emit && pos < ov.cap[po.phase];
                emit_closed_tuple<NC>(g, pl, in, r, q, H.n_qe, lv, st, akey, ov.keys[po.phase] + pos * H.n_qe, write, K,
                                      dA, dB);
            } else {
                Bind B;
                B.R = in;
                B.row = true;
                B.r = r;
                B.qa = B.fa = B.qb = B.fb = 0;
                B.skey = 0;
                B.cv = lv.vtx;
                B.fw = w;
#pragma unroll
                for (uint32_t c = 0; c < NA; c++)
                    if (c < (uint32_t)NC && c < H.n_close && !(c >= lv.c_begin && c < lv.c_end))
                        st[c] = rcol(in, 1 + in.wv + load_close(g.plans, pl, c).qe, r);
                uint32_t unused = 0;
                const uint64_t mult = close_mult<NC>(g, *P, B, st, unused, lv.qe, akey);
                emit_tuples<NC>(g, *P, B, st, mult, lv.qe, akey, pos, po, K, dA, dB);
            }
        }
    }
    if (EMIT) grouped_digest(dq != MAXQ, dq, dA, dB, A.dig);
    acc_flush(A, K, EMIT ? 2 * po.n_q : 0, po.stats, po.digest);
}

inline uint32_t nblocks(uint64_t n) { return (uint32_t)((n + MN_BLOCK - 1) / MN_BLOCK); }

}  // namespace

// Closing-edge arrays sized to the context's largest plan: 0, 1, 2, 4 or 8.
inline int nc_bucket(uint32_t nc) { return nc == 0 ? 0 : nc == 1 ? 1 : nc == 2 ? 2 : nc <= 4 ? 4 : 8; }

void mn_launch_seed_rows(const GraphView& g, const uint32_t* slots, uint32_t n, uint32_t n_plans, uint32_t max_close,
                         RowsView rows, uint32_t* n_rows, PhaseOut po, const uint32_t* err, hipStream_t s) {
    if (!n || !n_plans) return;
    // as many plans per block as bring the grid near 256 blocks (up to 32):
    // a block's set-up, its plan loop and the dense second pass cost less
    // than launching a block per plan (measured: 53 against 34 us per batch
    // on the six-query stream, 81 against 59 on the 64-query one)
    const uint32_t nbx = nblocks(n);
    const uint32_t ppb =
        (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(SR_MAX_PPB, (uint64_t)n_plans * nbx / 256));
    dim3 grid(nbx, (n_plans + ppb - 1) / ppb);
#define MN_SEED_ARGS g, slots, n, n_plans, ppb, rows, n_rows, po, err
    switch (nc_bucket(max_close)) {
        case 0: k_seed_rows<0><<<grid, MN_BLOCK, 0, s>>>(MN_SEED_ARGS); break;
        case 1: k_seed_rows<1><<<grid, MN_BLOCK, 0, s>>>(MN_SEED_ARGS); break;
        case 2: k_seed_rows<2><<<grid, MN_BLOCK, 0, s>>>(MN_SEED_ARGS); break;
        case 4: k_seed_rows<4><<<grid, MN_BLOCK, 0, s>>>(MN_SEED_ARGS); break;
        default: k_seed_rows<8><<<grid, MN_BLOCK, 0, s>>>(MN_SEED_ARGS); break;
    }
#undef MN_SEED_ARGS
}

void mn_launch_decide(const GraphView& g, RowsView rows, const uint32_t* slots, uint32_t cap, uint32_t expect,
                      int phase, hipStream_t s) {
    if (!cap) return;
    constexpr uint32_t RPB = MN_BLOCK / MN_NVAR;
    // enough blocks for the expected rows in one pass, at most two per CU
    const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(512, (expect + RPB - 1) / RPB));
    if (g.sched_mode == MN_SCHED_LEARNED)
        k_decide<true><<<blocks, MN_BLOCK, 0, s>>>(g, rows, slots, cap, phase);
    else
        k_decide<false><<<blocks, MN_BLOCK, 0, s>>>(g, rows, slots, cap, phase);
}

void mn_launch_note_count(const uint32_t* count, uint64_t cap, unsigned long long* note, hipStream_t s) {
    k_note_count<<<1, 64, 0, s>>>(count, cap, note);
}

void mn_launch_level_range(const GraphView& g, RowsView rows, uint32_t n, const uint32_t* n_dev, uint32_t L,
                           uint32_t* lo, uint32_t* cnt, EnumStats* st, const uint32_t* err, hipStream_t s,
                           uint32_t* zero_next, unsigned long long* note) {
    // at most 16 blocks per CU: a device-sized level passes its buffer's
    // capacity as n, most of it unused
    const uint32_t blocks = std::min<uint32_t>(nblocks(n ? n : 1), 4096u);
    k_level_range<<<blocks, MN_BLOCK, 0, s>>>(g, rows, n, n_dev, L, lo, cnt, st, zero_next, note, err);
}

uint64_t mn_expand_tiles(uint64_t c0, uint64_t c1) { return expand_tiles(c0, c1, EX_TILE_MIN); }

// k_expand launches go through hipExtLaunchKernel so that the optional
// events are stamped by the dispatch itself: they time the kernel, not the
// queue around it.
template <int NC, uint32_t ITEMS, uint32_t BT>
void launch_expand_nc(bool rows, bool emit, dim3 grid, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                      const GraphView& g, RowsView in, uint32_t n_in, const uint32_t* lo, const uint64_t* off,
                      const uint32_t* tile_row, uint64_t c0, uint64_t c1, const uint64_t* T_dev, uint32_t L,
                      RowsView out, uint32_t* n_out, PhaseOut po, const uint32_t* err) {
    auto k = rows && emit ? k_expand<NC, true, true, ITEMS, BT>
                          : rows ? k_expand<NC, true, false, ITEMS, BT> : k_expand<NC, false, true, ITEMS, BT>;
    hipExtLaunchKernelGGL(k, grid, dim3(BT), 0, s, ev0, ev1, 0, g, in, n_in, lo, off, tile_row, c0, c1, T_dev, L,
                          out, n_out, po, err);
}

// Tiles of 256 x T candidates: two per thread, in blocks of 128 x T threads
// (T = 2, 4, 8). Larger blocks take their places in the output with fewer
// device atomics on the shared counters, whose memory-side throughput (about
// one per 12 ns and word) bounds the expansion's largest launches; their LDS
// per wave, and so the occupancy, stay the same.
template <uint32_t T>
void launch_expand_items(uint32_t max_close, bool rows, bool emit, dim3 grid, hipStream_t s, hipEvent_t ev0,
                         hipEvent_t ev1, const GraphView& g, RowsView in, uint32_t n_in, const uint32_t* lo,
                         const uint64_t* off, const uint32_t* tile_row, uint64_t c0, uint64_t c1, const uint64_t* T_dev,
                         uint32_t L, RowsView out, uint32_t* n_out, PhaseOut po, const uint32_t* err) {
#define MN_EXPAND_ARGS rows, emit, grid, s, ev0, ev1, g, in, n_in, lo, off, tile_row, c0, c1, T_dev, L, out, n_out, po, err
    constexpr uint32_t BT = 128 * T, ITEMS = 2;
    switch (nc_bucket(max_close)) {
        case 0: launch_expand_nc<0, ITEMS, BT>(MN_EXPAND_ARGS); break;
        case 1: launch_expand_nc<1, ITEMS, BT>(MN_EXPAND_ARGS); break;
        case 2: launch_expand_nc<2, ITEMS, BT>(MN_EXPAND_ARGS); break;
        case 4: launch_expand_nc<4, ITEMS, BT>(MN_EXPAND_ARGS); break;
        default: launch_expand_nc<8, ITEMS, BT>(MN_EXPAND_ARGS); break;
    }
#undef MN_EXPAND_ARGS
}

inline uint32_t expand_items(uint32_t items) { return items == 4 || items == 8 ? items : 2u; }

uint64_t mn_expand_end(uint64_t c0, uint64_t c1, uint64_t expect, uint32_t items) {
    const uint32_t tile = MN_BLOCK * expand_items(items);
    const uint64_t want = expand_tiles(0, expect + expect / 2, tile) + EX_SPARE_TILES;
    return std::min<uint64_t>(c1, c0 + std::min<uint64_t>(want, MN_EXPAND_MAX_BLOCKS) * tile);
}

void mn_launch_offsets_partition(const uint32_t* cnt, uint64_t* off, const uint64_t* sums, uint32_t nb, uint32_t n,
                                 const uint32_t* n_dev, uint64_t c0, uint64_t c1, uint64_t* T_dev, uint32_t items,
                                 uint32_t* tile_row, unsigned long long* note, hipStream_t s) {
    if (!nb) return;
    k_offsets_partition<<<nb, MN_BLOCK, 0, s>>>(cnt, off, sums, nb, n, n_dev, c0, c1, T_dev,
                                                MN_BLOCK * expand_items(items), tile_row, note);
}

uint64_t mn_launch_expand(const GraphView& g, RowsView in, uint32_t n_in, const uint32_t* n_dev, const uint32_t* lo,
                          const uint64_t* off, const uint32_t* cnt, uint32_t* tile_row, uint64_t c0, uint64_t c1,
                          uint64_t* T_dev,
                          unsigned long long* note, uint64_t expect, uint32_t items, uint32_t L, uint32_t max_close,
                          bool rows, bool emit, RowsView out, uint32_t* n_out, PhaseOut po, const uint32_t* err,
                          hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, bool partitioned) {
    if (c1 <= c0 || !n_in) {
        if (ev0) {  // an empty pair keeps the caller's bookkeeping simple
            (void)hipEventRecord(ev0, s);
            (void)hipEventRecord(ev1, s);
        }
        return c1;
    }
    items = expand_items(items);
    const uint32_t tile = MN_BLOCK * items;
    // With the total on the device, the grid follows the expected candidate
    // count with a margin, and the candidates it can cover bound c1: a larger
    // total leaves a note and the host runs the phase again with more blocks.
    // The margin is relative (batches vary) plus a fixed EX_SPARE_TILES:
    // blocks past the candidates present leave at once, so spare blocks cost
    // little, while a re-run costs the whole phase (a deletion phase that
    // meets a hub can take several times its usual candidates).
    if (T_dev) c1 = mn_expand_end(c0, c1, expect, items);
    const uint64_t tiles = expand_tiles(c0, c1, tile);
    if (!partitioned)
        k_partition<<<nblocks(tiles + 1), MN_BLOCK, 0, s>>>(off, cnt, n_in, n_dev, c0, c1, T_dev, tile, tile_row,
                                                            note);
    const dim3 grid((uint32_t)tiles);
#define MN_ITEMS_ARGS max_close, rows, emit, grid, s, ev0, ev1, g, in, n_in, lo, off, tile_row, c0, c1, T_dev, L, out, n_out, po, err
    if (items == 8)
        launch_expand_items<8>(MN_ITEMS_ARGS);
    else if (items == 4)
        launch_expand_items<4>(MN_ITEMS_ARGS);
    else
        launch_expand_items<2>(MN_ITEMS_ARGS);
#undef MN_ITEMS_ARGS
    return c1;
}
