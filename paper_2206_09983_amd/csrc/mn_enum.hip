// Work units and the enumerator (Section VI, "Embedding Enumeration").
//
// k_seed: every batch edge whose DEBI word says it satisfies edgeMatcher for
// query edge q_j, and whose endpoints pass the vertex filter, becomes one work
// unit (slot, query, j) (Section VI, "work decomposition"). The DEBI word holds
// a bit for every query edge, tree or not, so a non-tree start edge needs no
// expansion into tree-edge seeds.
//
// k_enumerate: one 64-lane wavefront backtracks one work unit at a time,
// pulling units from a global counter (the paper's pull-based distribution).
// The static order for (query, j) maps one new query vertex per level through
// an anchor edge; the anchor's candidates are a label run of the mapped
// endpoint's sorted adjacency (getCandidates, Section IV-A), tested 64 at a
// time, one per lane: duplicate-removal mask (positions k < j may not use
// batch edges, Section VI), vertex filter bit, injectivity (isomorphism
// only), and each closing edge (verifyNte) by binary search for the
// (label, neighbour) run in the already-mapped endpoint's adjacency. Survivors
// are compacted by ballot into the level's LDS buffer and expanded one at a
// time; at the last level every surviving lane emits its embeddings directly.
// Parallel closing edges multiply embeddings (each instance is distinct).
#include "mn_internal.h"

namespace {

constexpr uint32_t EN_WAVES = MN_BLOCK / MN_WAVE;
constexpr uint32_t MN_MAXCL = 8;  // closing edges per level (checked at creation)

__device__ inline bool failed(const uint32_t* err) { return *(volatile const uint32_t*)err != 0u; }

__device__ inline uint64_t shfl64(uint64_t x, int src) {
    uint32_t lo = __shfl((uint32_t)x, src, MN_WAVE);
    uint32_t hi = __shfl((uint32_t)(x >> 32), src, MN_WAVE);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t wave_sum64(uint64_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t lo = __shfl_xor((uint32_t)x, d, MN_WAVE);
        uint32_t hi = __shfl_xor((uint32_t)(x >> 32), d, MN_WAVE);
        x += ((uint64_t)hi << 32) | lo;
    }
    return x;
}

__device__ inline uint32_t wave_excl_scan(uint32_t x, uint32_t& total) {
    uint32_t lane = __lane_id();
    uint32_t incl = x;
#pragma unroll
    for (int d = 1; d < MN_WAVE; d <<= 1) {
        uint32_t y = __shfl_up(incl, d, MN_WAVE);
        if (lane >= (uint32_t)d) incl += y;
    }
    total = __shfl(incl, MN_WAVE - 1, MN_WAVE);
    return incl - x;
}

__device__ inline bool vf_bit(const GraphView& g, uint32_t v, uint32_t bit) {
    return (g.vf[(size_t)v * g.vf_words + (bit >> 5)] >> (bit & 31)) & 1u;
}

struct Counters {
    uint64_t entries, probes, keys, tuples, seeds;
};

// Binary searches that also count the adjacency words they read.
__device__ inline uint32_t lower_hi_c(const uint64_t* adj, uint32_t lo, uint32_t hi, uint32_t key,
                                      uint64_t& probes) {
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

__device__ inline uint32_t upper_hi_c(const uint64_t* adj, uint32_t lo, uint32_t hi, uint32_t key,
                                      uint64_t& probes) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(adj);
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        probes++;
        if (w[2 * (size_t)mid + 1] <= key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Range of possible instances of closing edge c whose new endpoint is w.
// A labelled closing edge is one (label, w) run; an unlabelled one scans the
// whole segment and filters by neighbour.
__device__ inline void close_range(const GraphView& g, const CloseDesc& c, uint32_t x, uint32_t w,
                                   uint32_t& lo, uint32_t& hi, uint64_t& probes) {
    const uint64_t* adj = g.adj[c.dir];
    uint32_t s0 = g.off[c.dir][x], s1 = g.off[c.dir][x + 1];
    if (c.label >= 0) {
        uint32_t h = ((uint32_t)c.label << g.nbr_bits) | w;
        lo = lower_hi_c(adj, s0, s1, h, probes);
        hi = upper_hi_c(adj, lo, s1, h, probes);
    } else {
        lo = s0;
        hi = s1;
    }
}

__device__ inline bool close_accept(const GraphView& g, const CloseDesc& c, uint32_t p, uint32_t w) {
    uint64_t e = g.adj[c.dir][p];
    if (c.label < 0 && (ent_hi(e) & g.nbr_mask) != w) return false;
    if (c.masked && (ent_lo(e) & MN_FLAG)) return false;
    return true;
}

__device__ inline uint32_t close_count(const GraphView& g, const CloseDesc& c, uint32_t lo, uint32_t hi,
                                       uint32_t w, uint64_t& probes) {
    uint32_t n = 0;
    for (uint32_t p = lo; p < hi; p++) n += close_accept(g, c, p, w);
    probes += hi - lo;
    return n;
}

// Position of the first acceptable instance at or after p, or hi.
__device__ inline uint32_t close_next(const GraphView& g, const CloseDesc& c, uint32_t p, uint32_t hi,
                                      uint32_t w) {
    while (p < hi && !close_accept(g, c, p, w)) p++;
    return p;
}

struct WaveLds {
    uint64_t ekey[MN_MAXQE];  // key of each query edge mapped above the current level
    uint32_t map[MN_MAXQV];   // data vertex of each mapped query vertex
    uint32_t cur[MN_MAXLV], end[MN_MAXLV];
    uint32_t bn[MN_MAXLV], bi[MN_MAXLV], has[MN_MAXLV];
    uint32_t od_pos[MN_MAXQE], od_hi[MN_MAXQE], od_lo[MN_MAXQE];
    uint32_t buf[MN_MAXLV][MN_WAVE];
};

struct Ctx {
    const GraphView* g;
    const QueryDev* Q;
    const SeedPlan* P;
    WaveLds* S;
    uint32_t q;
    uint32_t lane;
};

// Odometer over the closing edges [cb, ce) of a level whose new vertex is the
// (wave-uniform) data vertex w: first combination / next combination. Every
// lane computes the same values; lane 0 stores them.
__device__ bool od_first(Ctx& C, uint32_t cb, uint32_t ce, uint32_t w, Counters& K) {
    const GraphView& g = *C.g;
    for (uint32_t c = cb; c < ce; c++) {
        const CloseDesc cd = C.P->close[c];
        uint32_t x = C.S->map[cd.other];
        uint32_t lo, hi;
        close_range(g, cd, x, w, lo, hi, K.probes);
        uint32_t p = close_next(g, cd, lo, hi, w);
        if (p >= hi) return false;
        uint32_t slot = ent_lo(g.adj[cd.dir][p]) & MN_SLOTMASK;
        uint64_t key = g.s_key[slot];
        K.keys++;
        if (C.lane == 0) {
            C.S->od_lo[c] = lo;
            C.S->od_hi[c] = hi;
            C.S->od_pos[c] = p;
            C.S->ekey[cd.qe] = key;
        }
    }
    wave_lds_sync();
    return true;
}

__device__ bool od_next(Ctx& C, uint32_t cb, uint32_t ce, uint32_t w, Counters& K) {
    const GraphView& g = *C.g;
    for (uint32_t cc = ce; cc > cb; cc--) {
        uint32_t c = cc - 1;
        const CloseDesc cd = C.P->close[c];
        uint32_t hi = uniform_u32(C.S->od_hi[c]);
        uint32_t p = close_next(g, cd, uniform_u32(C.S->od_pos[c]) + 1, hi, w);
        K.probes++;
        if (p < hi) {
            uint32_t slot = ent_lo(g.adj[cd.dir][p]) & MN_SLOTMASK;
            uint64_t key = g.s_key[slot];
            K.keys++;
            if (C.lane == 0) {
                C.S->od_pos[c] = p;
                C.S->ekey[cd.qe] = key;
            }
            // reset the later closing edges to their first instance
            for (uint32_t c2 = c + 1; c2 < ce; c2++) {
                const CloseDesc d2 = C.P->close[c2];
                uint32_t lo2 = uniform_u32(C.S->od_lo[c2]), hi2 = uniform_u32(C.S->od_hi[c2]);
                uint32_t p2 = close_next(g, d2, lo2, hi2, w);
                if (p2 >= hi2) p2 = lo2;  // never expected: the first instance existed before
                uint32_t s2 = ent_lo(g.adj[d2.dir][p2]) & MN_SLOTMASK;
                uint64_t k2 = g.s_key[s2];
                K.keys++;
                if (C.lane == 0) {
                    C.S->od_pos[c2] = p2;
                    C.S->ekey[d2.qe] = k2;
                }
            }
            wave_lds_sync();
            return true;
        }
    }
    return false;
}

// Tests the anchor entry at position p for level L. Returns the number of
// closing-edge instance combinations (0 = rejected) and, for the last level,
// the per-closing ranges and counts.
__device__ inline uint32_t filter_candidate(Ctx& C, const LevelDesc& lv, uint32_t p, uint32_t& w_out,
                                            uint32_t& slot_out, uint32_t* clo, uint32_t* chi,
                                            uint32_t* ccnt, Counters& K) {
    const GraphView& g = *C.g;
    uint64_t e = g.adj[lv.dir][p];
    K.entries++;
    uint32_t w = ent_hi(e) & g.nbr_mask;
    w_out = w;
    slot_out = ent_lo(e) & MN_SLOTMASK;
    if (lv.masked && (ent_lo(e) & MN_FLAG)) return 0;
    if (!vf_bit(g, w, C.Q->vf_base + lv.vtx)) return 0;
    if (C.Q->sem == 0) {
        for (uint32_t t = 0; t < lv.n_mapped; t++)
            if (C.S->map[C.P->mapped[t]] == w) return 0;
    }
    uint32_t mult = 1;
    uint32_t ncl = lv.c_end - lv.c_begin;
#pragma unroll
    for (uint32_t i = 0; i < MN_MAXCL; i++) {
        if (i < ncl) {
            const CloseDesc cd = C.P->close[lv.c_begin + i];
            uint32_t x = C.S->map[cd.other];
            uint32_t lo, hi;
            close_range(g, cd, x, w, lo, hi, K.probes);
            uint32_t n = close_count(g, cd, lo, hi, w, K.probes);
            clo[i] = lo;
            chi[i] = hi;
            ccnt[i] = n;
            mult *= n;
            if (!n) return 0;
        }
    }
    return mult;
}

// Emits the mult embeddings of one lane at the last level (or of the seed
// level when the query has two vertices). pos is this lane's first output row.
__device__ void emit_lane(Ctx& C, const LevelDesc* lv, uint32_t mult, uint32_t slot, const uint32_t* clo,
                          const uint32_t* chi, const uint32_t* ccnt, uint32_t w, uint64_t pos,
                          uint64_t* out, uint64_t cap, int emit, uint64_t& dA, uint64_t& dB,
                          Counters& K) {
    const GraphView& g = *C.g;
    const uint32_t nqe = C.Q->n_qe;
    uint64_t akey = 0;
    if (lv) {
        akey = g.s_key[slot];
        K.keys++;
    }
    uint32_t ncl = lv ? (uint32_t)(lv->c_end - lv->c_begin) : 0u;
    const uint64_t s0A = mn_mix64(MN_SEED_A ^ (uint64_t)C.q);
    const uint64_t s0B = mn_mix64(MN_SEED_B ^ (uint64_t)C.q);
    for (uint32_t t = 0; t < mult; t++) {
        uint64_t ckey[MN_MAXCL];
        uint32_t rem = t;
#pragma unroll
        for (uint32_t i = 0; i < MN_MAXCL; i++) {
            ckey[i] = 0;
            if (i < ncl) {
                const CloseDesc cd = C.P->close[lv->c_begin + i];
                uint32_t dig = rem % ccnt[i];
                rem /= ccnt[i];
                uint32_t p = close_next(g, cd, clo[i], chi[i], w);
                for (uint32_t k = 0; k < dig && p < chi[i]; k++) p = close_next(g, cd, p + 1, chi[i], w);
                if (p < chi[i]) {  // always true: the instances were counted
                    uint32_t s = ent_lo(g.adj[cd.dir][p]) & MN_SLOTMASK;
                    ckey[i] = g.s_key[s];
                    K.keys++;
                }
            }
        }
        uint64_t hA = s0A, hB = s0B;
        bool write = emit && (pos + t) < cap;
        uint64_t* row = out + (pos + t) * nqe;
        for (uint32_t k = 0; k < nqe; k++) {
            uint32_t src = C.P->last_src[k];
            uint64_t key;
            if (src == 0xFF)
                key = C.S->ekey[k];
            else if (src == 0xFE)
                key = akey;
            else {
                key = 0;
#pragma unroll
                for (uint32_t i = 0; i < MN_MAXCL; i++)
                    if (i == src) key = ckey[i];
            }
            hA = mn_mix64(hA + key);
            hB = mn_mix64(hB + key);
            if (write) row[k] = key;
        }
        dA += hA;
        dB += hB;
        K.tuples++;
    }
}

// Processes the candidates of the last level in chunks of 64 and emits.
__device__ void run_last_level(Ctx& C, uint32_t L, const PhaseOut& po, int phase, int emit,
                               uint64_t& dA, uint64_t& dB, Counters& K) {
    const LevelDesc lv = C.P->lv[L];
    uint64_t* out = po.outs[C.Q->out_index].keys[phase];
    uint64_t cap = po.outs[C.Q->out_index].cap[phase];
    uint32_t cur = uniform_u32(C.S->cur[L]);
    const uint32_t end = uniform_u32(C.S->end[L]);
    for (; cur < end; cur += MN_WAVE) {
        uint32_t p = cur + C.lane;
        uint32_t clo[MN_MAXCL], chi[MN_MAXCL], ccnt[MN_MAXCL];
        uint32_t mult = 0, w = 0, slot = 0;
        if (p < end) mult = filter_candidate(C, lv, p, w, slot, clo, chi, ccnt, K);
        uint32_t total;
        uint32_t excl = wave_excl_scan(mult, total);
        total = uniform_u32(total);
        if (!total) continue;
        unsigned long long base = 0;
        if (C.lane == 0) base = atomicAdd(&po.count[C.q], (unsigned long long)total);
        base = shfl64(base, 0);
        if (mult) emit_lane(C, &lv, mult, slot, clo, chi, ccnt, w, base + excl, out, cap, emit, dA, dB, K);
    }
}

// Sets up level L's anchor range from the mapped endpoint's sorted adjacency.
__device__ void setup_level(Ctx& C, uint32_t L, Counters& K) {
    const GraphView& g = *C.g;
    const LevelDesc lv = C.P->lv[L];
    uint32_t x = uniform_u32(C.S->map[lv.from]);
    const uint64_t* adj = g.adj[lv.dir];
    uint32_t lo = g.off[lv.dir][x], hi = g.off[lv.dir][x + 1];
    if (lv.label >= 0) {
        uint32_t l = (uint32_t)lv.label << g.nbr_bits;
        lo = lower_hi_c(adj, lo, hi, l, K.probes);
        hi = upper_hi_c(adj, lo, hi, l | g.nbr_mask, K.probes);
    }
    if (C.lane == 0) {
        C.S->cur[L] = lo;
        C.S->end[L] = hi;
        C.S->bn[L] = 0;
        C.S->bi[L] = 0;
        C.S->has[L] = 0;
    }
    wave_lds_sync();
}

// Moves level L (not the last) to its next mapping; false when exhausted.
__device__ bool advance_level(Ctx& C, uint32_t L, Counters& K) {
    const GraphView& g = *C.g;
    const LevelDesc lv = C.P->lv[L];
    if (uniform_u32(C.S->has[L])) {
        uint32_t w = uniform_u32(C.S->map[lv.vtx]);
        if (od_next(C, lv.c_begin, lv.c_end, w, K)) return true;
        if (C.lane == 0) C.S->has[L] = 0;
        wave_lds_sync();
    }
    while (true) {
        uint32_t bi = uniform_u32(C.S->bi[L]);
        uint32_t bn = uniform_u32(C.S->bn[L]);
        if (bi < bn) {
            uint32_t p = uniform_u32(C.S->buf[L][bi]);
            uint64_t e = g.adj[lv.dir][p];
            uint32_t w = ent_hi(e) & g.nbr_mask;
            uint32_t slot = ent_lo(e) & MN_SLOTMASK;
            uint64_t key = g.s_key[slot];
            K.keys++;
            if (C.lane == 0) {
                C.S->bi[L] = bi + 1;
                C.S->map[lv.vtx] = w;
                C.S->ekey[lv.qe] = key;
            }
            wave_lds_sync();
            if (!od_first(C, lv.c_begin, lv.c_end, w, K)) continue;
            if (C.lane == 0) C.S->has[L] = 1;
            wave_lds_sync();
            return true;
        }
        uint32_t cur = uniform_u32(C.S->cur[L]);
        uint32_t end = uniform_u32(C.S->end[L]);
        if (cur >= end) return false;
        uint32_t p = cur + C.lane;
        uint32_t clo[MN_MAXCL], chi[MN_MAXCL], ccnt[MN_MAXCL];
        uint32_t w, slot, mult = 0;
        if (p < end) mult = filter_candidate(C, lv, p, w, slot, clo, chi, ccnt, K);
        uint64_t bal = __ballot(mult != 0);
        if (mult) C.S->buf[L][__popcll(bal & lanemask_lt())] = p;
        if (C.lane == 0) {
            C.S->bn[L] = (uint32_t)__popcll(bal);
            C.S->bi[L] = 0;
            C.S->cur[L] = cur + MN_WAVE;
        }
        wave_lds_sync();
    }
}

__global__ __launch_bounds__(MN_BLOCK) void k_enumerate(GraphView g, const uint64_t* __restrict__ seeds,
                                                        const uint32_t* n_seeds_p, uint32_t* cursor,
                                                        PhaseOut po, int phase, int emit,
                                                        const uint32_t* err) {
    __shared__ WaveLds lds[EN_WAVES];
    if (failed(err)) return;
    Ctx C;
    C.g = &g;
    C.S = &lds[threadIdx.x / MN_WAVE];
    C.lane = __lane_id();
    const uint32_t n_seeds = *n_seeds_p;
    Counters K = {0, 0, 0, 0, 0};
    while (true) {
        uint32_t sidx = 0;
        if (C.lane == 0) sidx = atomicAdd(cursor, 1u);
        sidx = uniform_u32(__shfl(sidx, 0, MN_WAVE));
        if (sidx >= n_seeds) break;
        const uint64_t sd = seeds[sidx];
        const uint32_t slot = (uint32_t)sd;
        const uint32_t q = (uint32_t)(sd >> 32) & 0xFFFFu;
        const uint32_t j = (uint32_t)(sd >> 48);
        C.q = q;
        C.Q = &g.queries[q];
        C.P = &g.plans[C.Q->plan_base + j];
        if (C.lane == 0) K.seeds++;
        const uint32_t qa = C.P->qa, qb = C.P->qb;
        const uint32_t vs = g.s_src[slot], vd = g.s_dst[slot];
        const uint64_t skey = g.s_key[slot];
        if (C.lane == 0) {
            C.S->map[qa] = vs;
            C.S->map[qb] = vd;
            C.S->ekey[j] = skey;
        }
        wave_lds_sync();
        uint64_t dA = 0, dB = 0;
        const uint32_t nl = C.P->n_levels;
        if (od_first(C, 0, C.P->c0_end, vd, K)) {
            do {
                if (nl == 0) {
                    uint64_t* out = po.outs[C.Q->out_index].keys[phase];
                    uint64_t cap = po.outs[C.Q->out_index].cap[phase];
                    if (C.lane == 0) {
                        unsigned long long base = atomicAdd(&po.count[q], 1ull);
                        emit_lane(C, nullptr, 1, 0, nullptr, nullptr, nullptr, 0, base, out, cap, emit,
                                  dA, dB, K);
                    }
                    continue;
                }
                uint32_t L = 0;
                setup_level(C, 0, K);
                while (true) {
                    if (L == nl - 1) {
                        run_last_level(C, L, po, phase, emit, dA, dB, K);
                        if (L == 0) break;
                        L--;
                        continue;
                    }
                    if (advance_level(C, L, K)) {
                        L++;
                        setup_level(C, L, K);
                    } else {
                        if (L == 0) break;
                        L--;
                    }
                }
            } while (od_next(C, 0, C.P->c0_end, vd, K));
        }
        uint64_t sA = wave_sum64(dA), sB = wave_sum64(dB);
        if (C.lane == 0 && (sA | sB)) {
            atomicAdd(&po.digest[2 * q], (unsigned long long)sA);
            atomicAdd(&po.digest[2 * q + 1], (unsigned long long)sB);
        }
    }
    uint64_t e = wave_sum64(K.entries), p = wave_sum64(K.probes), k = wave_sum64(K.keys);
    uint64_t t = wave_sum64(K.tuples), s = wave_sum64(K.seeds);
    if (C.lane == 0) {
        EnumStats* st = po.stats + phase;
        atomicAdd(&st->seeds, (unsigned long long)s);
        atomicAdd(&st->entries, (unsigned long long)e);
        atomicAdd(&st->probe_words, (unsigned long long)p);
        atomicAdd(&st->key_reads, (unsigned long long)k);
        atomicAdd(&st->tuples, (unsigned long long)t);
    }
}

__global__ __launch_bounds__(MN_BLOCK) void k_seed(GraphView g, const uint32_t* __restrict__ slots,
                                                   uint32_t n, uint64_t* __restrict__ seeds,
                                                   uint32_t* n_seeds, const uint32_t* err) {
    if (failed(err)) return;
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool valid = i < n;
    uint32_t slot = valid ? slots[i] : 0;
    uint32_t s = valid ? g.s_src[slot] : 0, d = valid ? g.s_dst[slot] : 0;
    uint32_t c = 0;
    for (int pass = 0; pass < 2; pass++) {
        uint32_t base_l = 0;
        if (pass == 1) {
            uint32_t total;
            uint32_t excl = wave_excl_scan(c, total);
            uint32_t base = 0;
            if (__lane_id() == 0 && total) base = atomicAdd(n_seeds, total);
            base = __shfl(base, 0, MN_WAVE);
            base_l = base + excl;
        }
        uint32_t k = 0;
        if (valid) {
            for (uint32_t q = 0; q < g.n_queries; q++) {
                const QueryDev& Q = g.queries[q];
                for (uint32_t j = 0; j < Q.n_qe; j++) {
                    uint32_t bit = Q.debi_base + j;
                    if (!((g.s_debi[(size_t)slot * g.debi_words + (bit >> 5)] >> (bit & 31)) & 1u)) continue;
                    if (Q.sem == 0 && s == d) continue;
                    if (!vf_bit(g, s, Q.vf_base + Q.qsrc[j]) || !vf_bit(g, d, Q.vf_base + Q.qdst[j])) continue;
                    if (pass == 1)
                        seeds[base_l + k] = (uint64_t)slot | ((uint64_t)q << 32) | ((uint64_t)j << 48);
                    k++;
                }
            }
        }
        c = k;
    }
}

}  // namespace

void mn_launch_seed(const GraphView& g, const DebiBit*, const uint32_t* slots, uint32_t n,
                    uint64_t* seeds, uint32_t* n_seeds, const uint32_t* err, hipStream_t s) {
    if (n) k_seed<<<(n + MN_BLOCK - 1) / MN_BLOCK, MN_BLOCK, 0, s>>>(g, slots, n, seeds, n_seeds, err);
}

void mn_launch_enumerate(const GraphView& g, const uint64_t* seeds, const uint32_t* n_seeds,
                         uint32_t max_seeds, uint32_t* cursor, PhaseOut po, int phase, int emit,
                         const uint32_t* err, hipStream_t s) {
    if (!max_seeds) return;
    uint32_t waves = max_seeds;
    uint32_t blocks = (waves + EN_WAVES - 1) / EN_WAVES;
    if (blocks > 2048) blocks = 2048;
    k_enumerate<<<blocks, MN_BLOCK, 0, s>>>(g, seeds, n_seeds, cursor, po, phase, emit, err);
}
