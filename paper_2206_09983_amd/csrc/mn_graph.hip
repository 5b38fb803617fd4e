// Graph update kernels for one snapshot (Algorithm 2, batchInserts and
// batchDeletes; Section IV-A, DEBI updating and memory recycling).
//
//   k_validate     endpoint/label/timestamp checks and deletion-key liveness,
//                  before anything changes (a failing batch changes nothing:
//                  every later kernel returns at once when the error word is set)
//   k_prev_del     deferred removal bookkeeping of the previous snapshot's
//                  deletions (counter decrements)
//   k_ingest       slot allocation (recycled slots first), attribute writes,
//                  edgeMatcher -> DEBI words, counter increments, sort keys
//   k_vertex_meta  per-vertex new offsets of the merged adjacency
//   k_merge_new/limits/old  merged, sorted adjacency: the batch entries
//                  (flagged) at their insertion points, the counts at every
//                  tile start of the old array, then the old entries minus
//                  the deleted ones (both directions in each launch)
//   k_vf_refresh   per-vertex local filters (f2/f3 of Section V-A) as VF bits
//   k_flag_del     locate and flag the deletion batch's adjacency entries
//   k_finalize     retire deleted keys, push their slots on the free stack
#include "mn_internal.h"

namespace {

__device__ inline bool failed(const uint32_t* err) { return *(volatile const uint32_t*)err != 0u; }

__device__ inline void set_err(uint32_t* err, uint32_t code) { atomicCAS(err, 0u, code); }

// Adds delta (+1 / -1 as u32) to the local-filter counters touched by one edge.
__device__ void count_edge(const GraphView& g, uint32_t s, uint32_t d, uint32_t lab, uint32_t delta) {
    const uint32_t E = g.n_elab_c, L = g.n_vlab_c;
    uint32_t* cs = g.cnt + (size_t)s * g.n_cnt;
    uint32_t* cd = g.cnt + (size_t)d * g.n_cnt;
    atomicAdd(cs + cnt_index(0, 0, E, L), delta);
    atomicAdd(cd + cnt_index(1, 0, E, L), delta);
    int32_t e = g.elab_idx[lab];
    if (e >= 0) {
        atomicAdd(cs + cnt_index(0, 1 + e, E, L), delta);
        atomicAdd(cd + cnt_index(1, 1 + e, E, L), delta);
    }
    if (L) {
        uint64_t md = g.vmask[d], ms = g.vmask[s];
        while (md) {
            uint32_t b = __ffsll((unsigned long long)md) - 1;
            md &= md - 1;
            int32_t l = g.vlab_idx[b];
            if (l >= 0) atomicAdd(cs + cnt_index(0, 1 + E + l, E, L), delta);
        }
        while (ms) {
            uint32_t b = __ffsll((unsigned long long)ms) - 1;
            ms &= ms - 1;
            int32_t l = g.vlab_idx[b];
            if (l >= 0) atomicAdd(cd + cnt_index(1, 1 + E + l, E, L), delta);
        }
    }
}

// edgeMatcher (Section III) of one slot: per query edge, the edge label is
// equal or the query label empty, and both endpoint label sets contain the
// query vertices' required sets. Writes the slot's DEBI words.
__device__ void match_edge(const GraphView& g, const DebiBit* __restrict__ bits, uint32_t n_bits, uint32_t slot,
                           uint32_t s, uint32_t d, uint32_t l) {
    const uint64_t ms = g.vmask[s], md = g.vmask[d];
    for (uint32_t w = 0; w < g.debi_words; w++) {
        uint32_t word = 0;
        const uint32_t lo = w * 32, hi = min(lo + 32, n_bits);
        for (uint32_t bit = lo; bit < hi; bit++) {
            const DebiBit db = bits[bit];
            const bool m = (db.label < 0 || (uint32_t)db.label == l) && (db.req_src & ~ms) == 0 &&
                           (db.req_dst & ~md) == 0;
            word |= (uint32_t)m << (bit - lo);
        }
        g.s_debi[(size_t)slot * g.debi_words + w] = word;
    }
}

__global__ __launch_bounds__(MN_BLOCK) void k_reset(uint32_t* err, unsigned long long* a, uint32_t n) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *err = 0;
    if (i < n) a[i] = 0ull;
}

__global__ __launch_bounds__(MN_BLOCK) void k_validate(GraphView g, BatchView b) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < b.n_ins) {
        uint32_t s = b.in_src[i], d = b.in_dst[i], l = b.in_lab[i];
        if (s >= g.n_vertices || d >= g.n_vertices) set_err(b.err, MN_ERR_VERTEX);
        if (l >= b.n_elabels) set_err(b.err, MN_ERR_LABEL);
        int64_t prev = i ? b.in_ts[i - 1] : *b.last_ts;
        if (b.in_ts[i] < prev) set_err(b.err, MN_ERR_TS);
    } else if (i < b.n_ins + b.n_del) {
        uint64_t k = b.del_keys[i - b.n_ins];
        uint64_t lim = b.next_key + b.n_ins;
        if (k >= lim || k < b.key_lo) {  // never inserted, or long dead
            set_err(b.err, MN_ERR_DELETE);
        } else if (k < b.next_key && b.key2slot[k & b.key_mask] == MN_INVALID) {
            set_err(b.err, MN_ERR_DELETE);
        } else {
            const uint64_t rk = k & b.key_mask;
            uint32_t bit = 1u << (uint32_t)(rk & 31);
            uint32_t old = atomicOr(&b.delbits[rk >> 5], bit);
            if (old & bit) set_err(b.err, MN_ERR_DELETE);
        }
    }
}

__global__ __launch_bounds__(MN_BLOCK) void k_prev_del(GraphView g, BatchView b) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.n_prev_del || failed(b.err)) return;
    uint32_t slot = b.prev_del_slot[i];
    uint32_t s = g.s_src[slot], d = g.s_dst[slot];
    count_edge(g, s, d, g.s_lab[slot], 0xFFFFFFFFu);
    b.touched[2 * i] = s;
    b.touched[2 * i + 1] = d;
}

__global__ __launch_bounds__(MN_BLOCK) void k_ingest(GraphView g, BatchView b) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.n_ins || failed(b.err)) return;
    uint32_t slot = i < b.n_free ? b.free_stack[b.n_free - 1 - i] : b.fresh + (i - b.n_free);
    // caller's vertex ids (validated above) -> internal ids
    uint32_t s = g.ext2int[b.in_src[i]], d = g.ext2int[b.in_dst[i]], l = b.in_lab[i];
    uint64_t key = b.next_key + i;
    g.s_src[slot] = s;
    g.s_dst[slot] = d;
    g.s_lab[slot] = (uint8_t)l;
    g.s_ts[slot] = b.in_ts[i];
    g.key_ts[key & b.key_mask] = b.in_ts[i];
    g.s_key[slot] = key;
    b.key2slot[key & b.key_mask] = slot;
    match_edge(g, b.debi_bits, b.n_debi_bits, slot, s, d, l);
    count_edge(g, s, d, l, 1u);
    uint64_t hs = ((uint64_t)l << g.nbr_bits) | d;  // out-entry high word
    uint64_t hd = ((uint64_t)l << g.nbr_bits) | s;  // in-entry high word
    b.skey[0][i] = ((uint64_t)s << b.hb) | hs;
    b.skey[1][i] = b.dirbit | ((uint64_t)d << b.hb) | hd;
    b.sval[0][i] = slot;
    b.sval[1][i] = slot;
    b.ins_slot[i] = slot;
    b.touched[2 * b.n_prev_del + 2 * i] = s;
    b.touched[2 * b.n_prev_del + 2 * i + 1] = d;
}

// After the query set changed: edgeMatcher words of every live slot, and the
// local-filter counters of every edge the counters hold: the live ones and
// those deleted by the last batch (the next batch decrements them).
__global__ __launch_bounds__(MN_BLOCK) void k_reindex(GraphView g, const DebiBit* __restrict__ bits, uint32_t n_bits,
                                                      uint32_t n_slots, const uint32_t* __restrict__ key2slot,
                                                      uint64_t key_lo, const uint32_t* __restrict__ pend,
                                                      uint32_t n_pend) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_slots) {
        const uint32_t slot = i;
        const uint64_t key = g.s_key[slot];
        // retired (a key below key_lo is dead, and another key may hold its
        // ring place), or recycled under another key
        if (key < key_lo || key2slot[key & g.key_mask] != slot) return;
        const uint32_t s = g.s_src[slot], d = g.s_dst[slot], l = g.s_lab[slot];
        match_edge(g, bits, n_bits, slot, s, d, l);
        count_edge(g, s, d, l, 1u);
    } else if (i < n_slots + n_pend) {
        const uint32_t slot = pend[i - n_slots];
        count_edge(g, g.s_src[slot], g.s_dst[slot], g.s_lab[slot], 1u);
    }
}

// Lower bounds of k1 <= k2 in sorted a[lo, hi), searched in lockstep: each
// step issues both loads before either is used.
__device__ inline void lower_bounds2(const uint64_t* __restrict__ a, uint32_t lo, uint32_t hi, uint64_t k1,
                                     uint64_t k2, uint32_t& r1, uint32_t& r2) {
    uint32_t l1 = lo, h1 = hi, l2 = lo, h2 = hi;
    while (l1 < h1 || l2 < h2) {
        const bool g1 = l1 < h1, g2 = l2 < h2;
        const uint32_t m1 = (l1 + h1) >> 1, m2 = (l2 + h2) >> 1;
        const uint64_t v1 = g1 ? a[m1] : 0ull, v2 = g2 ? a[m2] : 0ull;
        if (g1) {
            if (v1 < k1)
                l1 = m1 + 1;
            else
                h1 = m1;
        }
        if (g2) {
            if (v2 < k2)
                l2 = m2 + 1;
            else
                h2 = m2;
        }
    }
    r1 = l1;
    r2 = l2;
}

// Per vertex: its run of batch entries [bs, be) in bk and of deleted positions
// [ds, de) in dpos, and its offset in the merged adjacency. Four threads first
// bound the block's 256 vertices in both sorted arrays, so that every
// vertex searches only its block's window. blockIdx.y is the direction.
// First i in [lo, hi) with a[i] >= key (hi if none), by a whole wave (all
// lanes call it with the same arguments): each round the 64 lanes probe 64
// evenly spaced places of the range and keep the 1/65 between the last probe
// below key and the first not below it, so 2^18 values take three rounds of
// dependent loads instead of eighteen.
template <typename T>
__device__ uint32_t wave_lower_bound(const T* __restrict__ a, uint32_t lo, uint32_t hi, T key) {
    const uint32_t lane = __lane_id();
    while (hi - lo > MN_WAVE) {  // the answer lies in [lo, hi]
        const uint64_t n = hi - lo;
        const uint32_t c = (uint32_t)__popcll(__ballot(a[lo + (uint32_t)(n * (lane + 1) / 65)] < key));
        // a is sorted, so the c probes below key are the first c
        const uint32_t nlo = c ? lo + (uint32_t)(n * c / 65) + 1 : lo;
        hi = c < MN_WAVE ? lo + (uint32_t)(n * (c + 1) / 65) : hi;
        lo = nlo;
    }
    const uint32_t p = lo + lane;
    return lo + (uint32_t)__popcll(__ballot(p < hi && a[p] < key));
}

__global__ __launch_bounds__(MN_BLOCK) void k_vertex_meta(MergeSide m0, MergeSide m1, uint32_t nv, uint32_t e_old,
                                                          uint32_t n_b, uint32_t n_d, uint32_t hb,
                                                          const uint32_t* err) {
    const MergeSide& m = blockIdx.y ? m1 : m0;
    const uint32_t* __restrict__ off = m.off;
    const uint64_t* __restrict__ bk = m.bk;
    const uint64_t* __restrict__ dpos = m.dpos;
    const uint64_t kbase = m.kbase, dbase = m.dbase;
    __shared__ uint32_t s_w[4];
    const uint32_t v0 = blockIdx.x * MN_BLOCK, v1 = min(v0 + MN_BLOCK, nv);
    const uint32_t tid = threadIdx.x;
    // the block's windows of the sorted batch entries and deletion positions,
    // one wave per bound
    static_assert(MN_BLOCK / MN_WAVE == 4, "one wave per window bound");
    {
        const uint32_t wv = tid / MN_WAVE;
        const uint32_t u = wv & 1u ? v1 : v0;
        const uint32_t x = wv < 2 ? wave_lower_bound<uint64_t>(bk, 0, n_b, kbase + ((uint64_t)u << hb))
                                  : wave_lower_bound<uint64_t>(dpos, 0, n_d, dbase + off[u]);
        if (__lane_id() == 0) s_w[wv] = x;
    }
    __syncthreads();
    const uint32_t v = v0 + tid;
    if (v >= nv || failed(err)) return;
    uint32_t bs = s_w[0], be = s_w[0], ds = s_w[2], de = s_w[2];
    const uint32_t o0 = off[v], o1 = off[v + 1];
    if (s_w[0] < s_w[1])
        lower_bounds2(bk, s_w[0], s_w[1], kbase + ((uint64_t)v << hb), kbase + ((uint64_t)(v + 1) << hb), bs, be);
    if (s_w[2] < s_w[3]) lower_bounds2(dpos, s_w[2], s_w[3], dbase + o0, dbase + o1, ds, de);
    m.newoff[v] = o0 - ds + bs;
    // k_merge_new reads meta only for vertices with batch entries: most
    // vertices write none (16 of the 20 bytes a vertex would write)
    if (be > bs) m.meta[v] = make_uint4(bs, be - bs, ds, de - ds);
    if (v == nv - 1) m.newoff[nv] = e_old - n_d + n_b;
}

constexpr uint32_t MG_ITEMS = 8;
constexpr uint32_t MG_TILE = MN_BLOCK * MG_ITEMS;

// Batch entries: placed after every kept old entry of their vertex with a high
// word <= theirs. ub[r] records that insertion point (the first old position
// after the batch entry), which places the old entries in k_merge_old.
__global__ __launch_bounds__(MN_BLOCK) void k_merge_new(MergeSide m0, MergeSide m1,
                                                        const uint64_t* __restrict__ s_key, uint32_t n_b,
                                                        uint32_t hb, uint32_t e_new, uint32_t* err) {
    const MergeSide& m = blockIdx.y ? m1 : m0;
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_b || failed(err)) return;
    uint64_t key = m.bk[r] - m.kbase;
    uint32_t v = (uint32_t)(key >> hb);
    uint32_t h = (uint32_t)(key & ((1ull << hb) - 1));
    uint32_t o0 = m.off[v], o1 = m.off[v + 1];
    uint32_t ub = upper_hi(m.adj, o0, o1, h);
    m.ub[r] = ub;
    uint4 mt = m.meta[v];
    uint32_t kept = ub - o0;
    if (mt.w) kept -= lower_bound_dev<uint64_t>(m.dpos, mt.z, mt.z + mt.w, m.dbase + ub) - mt.z;
    uint32_t out = m.newoff[v] + kept + (r - mt.x);
    if (out >= e_new) {  // never expected; refuse rather than write out of bounds
        set_err(err, MN_ERR_INTERNAL);
        m.inspos[r] = 0;
        return;
    }
    const uint32_t slot = m.bv[r];
    m.adj_new[out] = ((uint64_t)h << 32) | MN_FLAG | slot;
    m.adjk_new[out] = s_key[slot];
    m.inspos[r] = out;
}

// Both counts at every tile start of the old array: lim[t] = insertion points
// below t * MG_TILE and lim[nt + 1 + t] = deletions below it, t in [0, nt].
// Thread i owns the boundary before sorted value i and writes the tiles whose
// start falls between values i - 1 and i, so the limits cost one pass over
// the batch instead of a binary search per tile. A side with no values is not
// written (k_merge_old reads zero for it). blockIdx.y is the direction.
__global__ __launch_bounds__(MN_BLOCK) void k_merge_limits(MergeSide m0, MergeSide m1, uint32_t n_b, uint32_t n_d,
                                                           uint32_t nt) {
    const MergeSide& m = blockIdx.y ? m1 : m0;
    const uint32_t* __restrict__ ub = m.ub;
    const uint64_t* __restrict__ dpos = m.dpos;
    const uint64_t dbase = m.dbase;
    uint32_t* __restrict__ lim = m.lim;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (n_b && i <= n_b) {
        const uint32_t t0 = i ? ub[i - 1] / MG_TILE + 1 : 0u;
        const uint32_t t1 = i < n_b ? min(nt, ub[i] / MG_TILE) : nt;
        for (uint32_t t = t0; t <= t1; t++) lim[t] = i;
    }
    if (n_d && i <= n_d) {
        const uint32_t t0 = i ? (uint32_t)(dpos[i - 1] - dbase) / MG_TILE + 1 : 0u;
        const uint32_t t1 = i < n_d ? min(nt, (uint32_t)(dpos[i] - dbase) / MG_TILE) : nt;
        for (uint32_t t = t0; t <= t1; t++) lim[nt + 1 + t] = i;
    }
}

// Old entries keep their order: the kept entry at old position p moves to
// p - (deleted entries before p) + (batch entries whose insertion point is
// <= p), whatever its vertex. Each block takes a tile of the old array; both
// counts at the tile's start and end come from k_merge_limits, the deletions
// and insertion points inside the tile are marked in LDS and prefix-summed,
// and every entry then costs one LDS read between its loads and its stores.
// ub (n_b, sorted) comes from k_merge_new, which must run first. blockIdx.y
// is the direction.
__global__ __launch_bounds__(MN_BLOCK) void k_merge_old(MergeSide m0, MergeSide m1, uint32_t e_old, uint32_t n_b,
                                                        uint32_t n_d, uint32_t e_new, uint32_t* err) {
    const MergeSide& m = blockIdx.y ? m1 : m0;
    const uint64_t* __restrict__ adj = m.adj;
    const uint64_t* __restrict__ adjk = m.adjk;
    const uint32_t* __restrict__ ub = m.ub;
    const uint64_t* __restrict__ dpos = m.dpos;
    const uint64_t dbase = m.dbase;
    const uint32_t* __restrict__ lim = m.lim;
    uint64_t* __restrict__ adj_new = m.adj_new;
    uint64_t* __restrict__ adjk_new = m.adjk_new;
    __shared__ __align__(16) int32_t s_m[MG_TILE];
    __shared__ int32_t s_wsum[MN_BLOCK / MN_WAVE];
    __shared__ uint32_t s_dead;
    const uint32_t tid = threadIdx.x;
    const uint32_t p0 = blockIdx.x * MG_TILE;
    const uint32_t p1 = min(p0 + MG_TILE, e_old);
    // the tile's entries are requested before anything waits on them
    uint64_t e[MG_ITEMS], ek[MG_ITEMS];
#pragma unroll
    for (uint32_t k = 0; k < MG_ITEMS; k++) {
        const uint32_t p = p0 + k * MN_BLOCK + tid;
        e[k] = p < p1 ? adj[p] : 0ull;
        ek[k] = p < p1 ? adjk[p] : 0ull;
    }
    // insertion points and deletions below the tile's start and end (at the
    // last tile the end limit counts up to nt * MG_TILE: insertion points at
    // e_old or beyond mark places past p1, which nothing reads)
    const uint32_t nt = gridDim.x, t = blockIdx.x;
    const uint32_t uA = n_b ? lim[t] : 0u, uB = n_b ? lim[t + 1] : 0u;
    const uint32_t dA = n_d ? lim[nt + 1 + t] : 0u, dB = n_d ? lim[nt + 2 + t] : 0u;
    if (tid == 0) s_dead = failed(err) ? 1u : 0u;
#pragma unroll
    for (uint32_t k = 0; k < MG_ITEMS; k++) s_m[k * MN_BLOCK + tid] = 0;
    __syncthreads();
    if (s_dead) return;
    const bool marks = uA < uB || dA < dB;  // the same for every thread of the block
    if (marks) {
        for (uint32_t r = uA + tid; r < uB; r += MN_BLOCK) {
            const uint32_t i = ub[r] - p0;
            if (i < MG_TILE) atomicAdd(&s_m[i], 1);
        }
        for (uint32_t k = dA + tid; k < dB; k += MN_BLOCK) {
            const uint32_t i = (uint32_t)(dpos[k] - dbase) - p0 + 1;  // counts for the entries after it
            if (i < MG_TILE) atomicAdd(&s_m[i], -1);
        }
        __syncthreads();
        // inclusive scan over the tile: eight consecutive marks per thread,
        // then across the lanes and the waves
        int4* q = reinterpret_cast<int4*>(s_m + tid * MG_ITEMS);
        const int4 a = q[0], b = q[1];
        int32_t v[MG_ITEMS] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (uint32_t k = 1; k < MG_ITEMS; k++) v[k] += v[k - 1];
        const int32_t run = v[MG_ITEMS - 1];
        const uint32_t lane = __lane_id(), wave = tid / MN_WAVE;
        int32_t incl = run;
#pragma unroll
        for (int d = 1; d < MN_WAVE; d <<= 1) {
            const int32_t y = __shfl_up(incl, d, MN_WAVE);
            if (lane >= (uint32_t)d) incl += y;
        }
        if (lane == MN_WAVE - 1) s_wsum[wave] = incl;
        __syncthreads();
        int32_t pre = incl - run;
        for (uint32_t w = 0; w < wave; w++) pre += s_wsum[w];
        q[0] = make_int4(v[0] + pre, v[1] + pre, v[2] + pre, v[3] + pre);
        q[1] = make_int4(v[4] + pre, v[5] + pre, v[6] + pre, v[7] + pre);
        __syncthreads();
    }
    const int64_t base = (int64_t)uA - (int64_t)dA;
#pragma unroll
    for (uint32_t k = 0; k < MG_ITEMS; k++) {
        const uint32_t p = p0 + k * MN_BLOCK + tid;
        if (p >= p1 || (ent_lo(e[k]) & MN_FLAG)) continue;  // past the end, or deleted by the previous snapshot
        const int64_t dst = (int64_t)p + base + (marks ? s_m[k * MN_BLOCK + tid] : 0);
        if (dst < 0 || dst >= (int64_t)e_new) {  // never expected; refuse rather than write out of bounds
            set_err(err, MN_ERR_INTERNAL);
            continue;
        }
        adj_new[dst] = e[k];
        adjk_new[dst] = ek[k];
    }
}

// Spanning-tree filter step (Section V-B): f4 bottom-up, a vertex stays a
// candidate for query vertex u only if, for the tree child c, some
// neighbour over the tree edge's label and direction is still a candidate
// for c; f1 top-down, a candidate for c needs a neighbour that is still a
// candidate for its tree parent. Both are the one rule of TreeStep, applied
// to bit `test` with `need` on the other side. Block row y takes step y; the
// grid strides over the vertices. The first entry of the range is found by
// binary search and the run is walked until a supporting neighbour turns up.
__global__ __launch_bounds__(MN_BLOCK) void k_tree_step(GraphView g, uint32_t* vf, const TreeStep* __restrict__ steps,
                                                        uint32_t n_v, unsigned long long* cleared,
                                                        const uint32_t* err) {
    if (failed(err)) return;
    const TreeStep st = steps[blockIdx.y];
    const uint32_t W = g.vf_words;
    const uint32_t tw = st.test >> 5, tb = 1u << (st.test & 31);
    const uint32_t nw = st.need >> 5, nb = 1u << (st.need & 31);
    uint32_t n_clear = 0;
    for (uint32_t v = blockIdx.x * MN_BLOCK + threadIdx.x; v < n_v; v += gridDim.x * MN_BLOCK) {
        uint32_t* word = vf + (size_t)v * W + tw;
        if (!(*word & tb)) continue;
        bool found = false;
        if (!st.empty) {
            const uint32_t* of = st.dir ? g.off[1] : g.off[0];
            const uint64_t* adj = st.dir ? g.adj[1] : g.adj[0];
            const uint32_t* w32 = reinterpret_cast<const uint32_t*>(adj);
            uint32_t a = of[v], b = of[v + 1];
            if (!st.whole) {
                while (a < b) {  // first entry with high word >= key_lo
                    const uint32_t m = (a + b) >> 1;
                    if (w32[2 * (size_t)m + 1] < st.key_lo)
                        a = m + 1;
                    else
                        b = m;
                }
                b = of[v + 1];
            }
            for (uint32_t p = a; p < b && !found; p++) {
                const uint32_t hi = w32[2 * (size_t)p + 1];
                if (!st.whole && hi > st.key_hi) break;
                const uint32_t x = hi & g.nbr_mask;
                found = (vf[(size_t)x * W + nw] & nb) != 0u;
            }
        }
        if (!found) {
            atomicAnd(word, ~tb);
            n_clear++;
        }
    }
    if (cleared) {
        uint32_t tot = n_clear;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) tot += __shfl_xor(tot, d, 64);
        if (__lane_id() == 0 && tot) atomicAdd(cleared, (unsigned long long)tot);
    }
}

// VF bit of (query, vertex u) at data vertex v: label requirement plus the
// counting filters of Section V-A (f2: edges per direction and label; f3:
// edges per direction towards each neighbour label), thresholds prepared on
// the host per semantics. A half-wave of 32 lanes serves one vertex: lane j
// tests bit 32w + j of word w, and one wave-wide ballot assembles the words
// of the wave's two vertices, so no lane walks the bits one by one. The loop
// runs over vertex pairs with a wave-uniform bound, which the ballot needs.
__global__ __launch_bounds__(MN_BLOCK) void k_vf_refresh(GraphView g, const VfBit* __restrict__ bits,
                                                         uint32_t n_bits, const uint32_t* __restrict__ list,
                                                         uint32_t n, const uint32_t* err) {
    if (failed(err)) return;  // the same word for every lane: whole waves leave
    constexpr uint32_t WPB = MN_BLOCK / 64;
    const uint32_t lane = threadIdx.x & 63, half = lane >> 5, j = lane & 31;
    const uint64_t n_pairs = ((uint64_t)n + 1) / 2, stride = (uint64_t)gridDim.x * WPB;
    // the lane's bit of the first word and its first four requirements are
    // the same for every vertex: loaded once, ahead of the vertex loads
    const VfBit vb0 = j < n_bits ? bits[j] : VfBit{0, 0, 0};
    VfReq q0[4];
#pragma unroll
    for (uint32_t k = 0; k < 4; k++)
        q0[k] = vb0.req_begin + k < vb0.req_end ? g.vfreq[vb0.req_begin + k] : VfReq{0, 0};
    for (uint64_t pair = (uint64_t)blockIdx.x * WPB + threadIdx.x / 64; pair < n_pairs; pair += stride) {
        const uint64_t i = 2 * pair + half;
        const bool live = i < n;
        const uint32_t v = live ? (list ? list[i] : (uint32_t)i) : 0u;
        const uint64_t mv = live ? g.vmask[v] : 0ull;
        const uint32_t* c = g.cnt + (size_t)v * g.n_cnt;
        for (uint32_t w = 0; w < g.vf_words; w++) {
            const uint32_t bit = w * 32 + j;
            bool ok = false;
            if (live && bit < n_bits) {
                const VfBit vb = w ? bits[bit] : vb0;
                ok = (vb.vreq & ~mv) == 0;
                // four requirements per step, their loads issued together
                for (uint32_t r = vb.req_begin; ok && r < vb.req_end; r += 4) {
                    const bool first = w == 0 && r == vb.req_begin;
                    VfReq q[4];
                    uint32_t have[4];
#pragma unroll
                    for (uint32_t k = 0; k < 4; k++)
                        q[k] = first ? q0[k] : r + k < vb.req_end ? g.vfreq[r + k] : VfReq{0, 0};
#pragma unroll
                    for (uint32_t k = 0; k < 4; k++) have[k] = r + k < vb.req_end ? c[q[k].cnt] : 0u;
#pragma unroll
                    for (uint32_t k = 0; k < 4; k++) ok = ok && have[k] >= q[k].need;
                }
            }
            const uint64_t m = __ballot(ok);
            if (live && j == 0) g.vf[(size_t)v * g.vf_words + w] = (uint32_t)(m >> (32 * half));
        }
    }
}

// blockIdx.y picks the direction: (adj0, pos0) or (adj1, pos1).
__global__ __launch_bounds__(MN_BLOCK) void k_set_flags(uint64_t* adj0, const uint32_t* __restrict__ pos0,
                                                        uint64_t* adj1, const uint32_t* __restrict__ pos1,
                                                        uint32_t n, int set, const uint32_t* err) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || failed(err)) return;
    uint64_t* adj = blockIdx.y ? adj1 : adj0;
    const uint32_t* pos = blockIdx.y ? pos1 : pos0;
    uint32_t* lo = reinterpret_cast<uint32_t*>(adj) + 2 * (size_t)pos[i];
    *lo = set ? (*lo | MN_FLAG) : (*lo & MN_SLOTMASK);
}

// blockIdx.y is the direction: both directions' searches run side by side.
__global__ __launch_bounds__(MN_BLOCK) void k_flag_del(GraphView g, uint64_t* adj_out, uint64_t* adj_in,
                                                       BatchView b) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t dir = blockIdx.y;
    if (i >= b.n_del || failed(b.err)) return;
    const uint64_t k = b.del_keys[i];
    const uint32_t slot = b.key2slot[k & b.key_mask];
    if (dir == 0) b.del_slot[i] = slot;
    const uint32_t s = g.s_src[slot], d = g.s_dst[slot], l = g.s_lab[slot];
    const uint32_t v = dir ? d : s;
    const uint32_t h = (l << g.nbr_bits) | (dir ? s : d);
    uint64_t* adj = dir ? adj_in : adj_out;
    const uint32_t end = g.off[dir][v + 1];
    uint32_t pos = lower_hi(adj, g.off[dir][v], end, h);
    uint32_t* w = reinterpret_cast<uint32_t*>(adj);
    while (pos < end && (w[2 * (size_t)pos] & MN_SLOTMASK) != slot) pos++;  // the run holds this slot
    if (pos == end) {  // internal inconsistency: never expected
        set_err(b.err, MN_ERR_INTERNAL);
        return;
    }
    w[2 * (size_t)pos] |= MN_FLAG;
    b.delpos[dir][i] = pos;
}

__global__ __launch_bounds__(MN_BLOCK) void k_finalize(BatchView b, uint32_t n_free_after) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = !failed(b.err);
    if (i < b.n_del) {
        uint64_t k = b.del_keys[i];
        if (k < b.next_key + b.n_ins && k >= b.key_lo) {
            const uint64_t rk = k & b.key_mask;
            atomicAnd(&b.delbits[rk >> 5], ~(1u << (uint32_t)(rk & 31)));
        }
        if (ok) {
            b.key2slot[k & b.key_mask] = MN_INVALID;
            b.free_stack[n_free_after + i] = b.del_slot[i];
        }
    }
    if (i == 0 && ok && b.n_ins) *b.last_ts = b.in_ts[b.n_ins - 1];
}

__global__ __launch_bounds__(MN_BLOCK) void k_init_vertices(uint32_t* vf, uint32_t* cnt, uint32_t nv,
                                                            uint32_t vf_words, uint32_t n_cnt) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (size_t)nv * vf_words) vf[i] = 0;
    if (i < (size_t)nv * n_cnt) cnt[i] = 0;
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// blockIdx.y picks the direction: (in0, out0, add0) or (in1, out1, add1).
__global__ __launch_bounds__(MN_BLOCK) void k_widen(const uint32_t* __restrict__ in0, uint64_t* __restrict__ out0,
                                                    uint64_t add0, const uint32_t* __restrict__ in1,
                                                    uint64_t* __restrict__ out1, uint64_t add1, uint32_t n,
                                                    const uint32_t* err) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || failed(err)) return;
    if (blockIdx.y)
        out1[i] = add1 + in1[i];
    else
        out0[i] = add0 + in0[i];
}

inline uint32_t nblocks(uint64_t n) { return (uint32_t)((n + MN_BLOCK - 1) / MN_BLOCK); }

}  // namespace


void mn_launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s) { k_set_u32<<<1, 64, 0, s>>>(p, v); }

void mn_launch_widen(const uint32_t* in0, uint64_t* out0, uint64_t add0, const uint32_t* in1, uint64_t* out1,
                     uint64_t add1, uint32_t n, const uint32_t* err, hipStream_t s) {
    if (n) k_widen<<<dim3(nblocks(n), 2), MN_BLOCK, 0, s>>>(in0, out0, add0, in1, out1, add1, n, err);
}

void mn_launch_reset(uint32_t* err, unsigned long long* zero_a, uint32_t n_a, hipStream_t s) {
    k_reset<<<nblocks(n_a ? n_a : 1), MN_BLOCK, 0, s>>>(err, zero_a, n_a);
}

void mn_launch_validate(const GraphView& g, const BatchView& b, hipStream_t s) {
    uint32_t n = b.n_ins + b.n_del;
    if (n) k_validate<<<nblocks(n), MN_BLOCK, 0, s>>>(g, b);
}

void mn_launch_prev_del(const GraphView& g, const BatchView& b, hipStream_t s) {
    if (b.n_prev_del) k_prev_del<<<nblocks(b.n_prev_del), MN_BLOCK, 0, s>>>(g, b);
}

void mn_launch_ingest(const GraphView& g, const BatchView& b, hipStream_t s) {
    if (b.n_ins) k_ingest<<<nblocks(b.n_ins), MN_BLOCK, 0, s>>>(g, b);
}

void mn_launch_merge(const MergeSide* side, uint32_t n_vertices, uint32_t e_old, const uint64_t* s_key,
                     uint32_t n_b, uint32_t n_d, uint32_t hb, uint32_t e_new, uint32_t* err, hipStream_t s) {
    const MergeSide m0 = side[0], m1 = side[1];
    k_vertex_meta<<<dim3(nblocks(n_vertices), 2), MN_BLOCK, 0, s>>>(m0, m1, n_vertices, e_old, n_b, n_d, hb, err);
    if (n_b) k_merge_new<<<dim3(nblocks(n_b), 2), MN_BLOCK, 0, s>>>(m0, m1, s_key, n_b, hb, e_new, err);
    if (e_old) {
        const uint32_t nt = (e_old + MG_TILE - 1) / MG_TILE;
        if (n_b || n_d)
            k_merge_limits<<<dim3(nblocks((uint64_t)std::max(n_b, n_d) + 1), 2), MN_BLOCK, 0, s>>>(m0, m1, n_b, n_d,
                                                                                                  nt);
        k_merge_old<<<dim3(nt, 2), MN_BLOCK, 0, s>>>(m0, m1, e_old, n_b, n_d, e_new, err);
    }
}

uint64_t mn_merge_limit_words(uint64_t e_old) { return 2 * ((e_old + MG_TILE - 1) / MG_TILE + 1); }

void mn_launch_reindex(const GraphView& g, const DebiBit* bits, uint32_t n_bits, uint32_t n_slots,
                       const uint32_t* key2slot, uint64_t key_lo, const uint32_t* pend, uint32_t n_pend,
                       hipStream_t s) {
    const uint64_t n = (uint64_t)n_slots + n_pend;
    if (n) k_reindex<<<nblocks(n), MN_BLOCK, 0, s>>>(g, bits, n_bits, n_slots, key2slot, key_lo, pend, n_pend);
}

void mn_launch_vf_refresh(const GraphView& g, const VfBit* bits, uint32_t n_bits,
                          const uint32_t* list, uint32_t n, const uint32_t* err, hipStream_t s) {
    // two vertices per wave, a grid of at most 65,536 blocks looping over the rest
    constexpr uint32_t VPB = 2 * (MN_BLOCK / 64);
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(65536, ((uint64_t)n + VPB - 1) / VPB);
    if (n) k_vf_refresh<<<blocks, MN_BLOCK, 0, s>>>(g, bits, n_bits, list, n, err);
}

void mn_launch_tree_step(const GraphView& g, uint32_t* vf, const TreeStep* steps, uint32_t n, uint32_t n_v,
                         unsigned long long* cleared, const uint32_t* err, hipStream_t s) {
    if (!n || !n_v) return;
    const uint32_t bx = (uint32_t)std::min<uint64_t>(4096, nblocks(n_v));
    for (uint32_t s0 = 0; s0 < n; s0 += 65535)
        k_tree_step<<<dim3(bx, std::min<uint32_t>(65535, n - s0)), MN_BLOCK, 0, s>>>(g, vf, steps + s0, n_v, cleared,
                                                                                  err);
}

void mn_launch_set_flags(uint64_t* adj0, const uint32_t* pos0, uint64_t* adj1, const uint32_t* pos1, uint32_t n,
                         int set, const uint32_t* err, hipStream_t s) {
    if (n) k_set_flags<<<dim3(nblocks(n), 2), MN_BLOCK, 0, s>>>(adj0, pos0, adj1, pos1, n, set, err);
}

void mn_launch_flag_del(const GraphView& g, uint64_t* adj_out, uint64_t* adj_in, const BatchView& b,
                        hipStream_t s) {
    if (b.n_del) k_flag_del<<<dim3(nblocks(b.n_del), 2), MN_BLOCK, 0, s>>>(g, adj_out, adj_in, b);
}

void mn_launch_finalize(const BatchView& b, uint32_t n_free_after, hipStream_t s) {
    uint32_t n = b.n_del ? b.n_del : 1;
    k_finalize<<<nblocks(n), MN_BLOCK, 0, s>>>(b, n_free_after);
}

// One block moves *lo past dead keys: 4,096 keys per step (16 per thread),
// stopping at the first live one or at `end`. A windowed stream retires its
// oldest keys each batch, so a step or two suffice.
__global__ __launch_bounds__(MN_BLOCK) void k_advance_lo(const uint32_t* __restrict__ key2slot, uint64_t key_mask,
                                                         uint64_t* lo_dev, uint64_t end, const uint32_t* err) {
    __shared__ uint32_t s_first;
    if (failed(err)) return;  // the same for the whole block
    uint64_t lo = *lo_dev;
    constexpr uint32_t PER = 32, STEP = PER * MN_BLOCK;
    while (lo < end) {  // uniform: every thread holds the same lo
        if (threadIdx.x == 0) s_first = STEP;
        __syncthreads();
        for (uint32_t j = 0; j < PER; j++) {
            const uint32_t o = j * MN_BLOCK + threadIdx.x;
            const uint64_t k = lo + o;
            // one LDS atomic per wave: its first live key (past the first one
            // most keys are live, and an atomic each serialised on one word)
            const uint64_t live = __ballot(k < end && key2slot[k & key_mask] != MN_INVALID);
            if (live && __lane_id() == (uint32_t)__ffsll((unsigned long long)live) - 1) atomicMin(&s_first, o);
        }
        __syncthreads();
        const uint32_t f = s_first;
        __syncthreads();
        if (f < STEP) {
            lo += f;
            break;
        }
        lo = min(end, lo + STEP);
    }
    if (threadIdx.x == 0) *lo_dev = lo;
}

void mn_launch_advance_lo(const uint32_t* key2slot, uint64_t key_mask, uint64_t* lo, uint64_t end,
                          const uint32_t* err, hipStream_t s) {
    k_advance_lo<<<1, MN_BLOCK, 0, s>>>(key2slot, key_mask, lo, end, err);
}

__global__ __launch_bounds__(MN_BLOCK) void k_ring_copy(const uint32_t* __restrict__ k2s_old,
                                                        const int64_t* __restrict__ ts_old, uint64_t m_old,
                                                        uint32_t* __restrict__ k2s_new, int64_t* __restrict__ ts_new,
                                                        uint64_t m_new, uint64_t lo, uint64_t hi) {
    const uint64_t k = lo + (uint64_t)blockIdx.x * MN_BLOCK + threadIdx.x;
    if (k >= hi) return;
    k2s_new[k & m_new] = k2s_old[k & m_old];
    ts_new[k & m_new] = ts_old[k & m_old];
}

void mn_launch_ring_copy(const uint32_t* k2s_old, const int64_t* ts_old, uint64_t m_old, uint32_t* k2s_new,
                         int64_t* ts_new, uint64_t m_new, uint64_t lo, uint64_t hi, hipStream_t s) {
    if (hi <= lo) return;
    k_ring_copy<<<(uint32_t)((hi - lo + MN_BLOCK - 1) / MN_BLOCK), MN_BLOCK, 0, s>>>(k2s_old, ts_old, m_old,
                                                                                       k2s_new, ts_new, m_new, lo, hi);
}

__global__ __launch_bounds__(MN_BLOCK) void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * MN_BLOCK + threadIdx.x;
    if (i < n) p[i] = v;
}

void mn_launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
    if (n) k_fill_u32<<<(uint32_t)((n + MN_BLOCK - 1) / MN_BLOCK), MN_BLOCK, 0, s>>>(p, v, n);
}

void mn_launch_init_vertices(uint32_t* vf, uint32_t* cnt, uint32_t n_vertices, uint32_t vf_words,
                             uint32_t n_cnt, hipStream_t s) {
    uint64_t n = (uint64_t)n_vertices * (vf_words > n_cnt ? vf_words : n_cnt);
    k_init_vertices<<<nblocks(n), MN_BLOCK, 0, s>>>(vf, cnt, n_vertices, vf_words, n_cnt);
}
