// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mn_common.h"

// ------------------------------------------------------------------ sorting
// Exclusive prefix sum of n u32 values (in may equal out). `scratch` must hold
// mn_scan_scratch_words(n) words.
size_t mn_scan_scratch_words(uint32_t n);
void mn_scan_exclusive(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* scratch,
                       hipStream_t s);

// Exclusive prefix sum of n u32 values into u64 offsets; *total (when given)
// receives the sum. `scratch` must hold mn_scan64_scratch_words(n) u64 words. With n_dev,
// the count is min(n, *n_dev), read on the device (n sizes the launch).
size_t mn_scan64_scratch_words(uint32_t n);
// The per-tile pass alone: out holds exclusive sums within tiles of
// MN_SCAN_TILE values, sums[b] the total of tile b; returns the tile count.
constexpr uint32_t MN_SCAN_TILE = 2048;
constexpr uint32_t MN_SCAN_DIRECT_MAX = 2048;  // tiles a block may sum in front of itself
uint32_t mn_scan64_local(const uint32_t* in, uint64_t* out, uint32_t n, uint64_t* sums, hipStream_t s,
                         const uint32_t* n_dev);
void mn_scan_exclusive64(const uint32_t* in, uint64_t* out, uint32_t n, uint64_t* scratch,
                         uint64_t* total, hipStream_t s, const uint32_t* n_dev = nullptr);

// Stable LSD radix sort of (u64 key, u32 value) pairs on bits [0, nbits).
// Ping-pongs between (keys, vals) and (ktmp, vtmp); on return keys/vals point
// at the sorted arrays (the pointers may have been swapped).
size_t mn_sort_scratch_words(uint32_t n);
void mn_radix_sort(uint64_t*& keys, uint32_t*& vals, uint64_t*& ktmp, uint32_t*& vtmp, uint32_t n,
                   uint32_t nbits, uint32_t* scratch, hipStream_t s);

// Sorts n rows of m u64 keys (row-major, keys < 2^key_bits) into
// lexicographic order in place. Scratch: k0, k1 (n u64 each), v0, v1 (n u32
// each), tmp_rows (n * m u64), scratch (mn_tuple_sort_scratch_words(n) u32).
size_t mn_tuple_sort_scratch_words(uint32_t n);
void mn_sort_tuples(uint64_t* rows, uint32_t n, uint32_t m, uint32_t key_bits, uint64_t* k0, uint64_t* k1,
                    uint32_t* v0, uint32_t* v1, uint64_t* tmp_rows, uint32_t* scratch, hipStream_t s);

// ------------------------------------------------------------------ batches
// Per-bit descriptors precomputed on the host.
struct DebiBit {  // one edgeMatcher bit: query edge label and endpoint requirements
    int32_t label;
    uint32_t pad;
    uint64_t req_src;
    uint64_t req_dst;
};
struct VfBit {  // one vertex-filter bit: label requirement and count requirements
    uint64_t vreq;
    uint32_t req_begin;
    uint32_t req_end;
};

// One step of the spanning-tree filter (Section V-B, f1 top-down and f4
// bottom-up) for one query tree edge: a vertex keeps bit `test` only if its
// adjacency in direction `dir` holds, inside the high-word range [key_lo,
// key_hi] (the tree edge's label and the other end's vertex classes; every
// entry when `whole`), a neighbour with bit `need`.
struct TreeStep {
    uint16_t test;
    uint16_t need;
    uint32_t dir;
    uint32_t key_lo;
    uint32_t key_hi;
    uint32_t whole;
    uint32_t empty;  // no vertex class can carry the other end: the bit is cleared everywhere
};

struct BatchView {
    uint32_t n_ins, n_del, n_prev_del;
    uint32_t n_free;        // free-slot stack height before this batch
    uint32_t fresh;         // first never-used slot
    uint32_t hb;            // composite sort key = (vertex << hb) | high word
    uint64_t dirbit;        // direction bit of in-list sort keys (above every vertex/high-word bit)
    uint64_t next_key;      // key of the first inserted edge
    uint64_t key_lo;        // every key below it is dead (deleted)
    uint64_t key_mask;      // ring mask of the key-indexed maps (capacity - 1; the capacity exceeds the
                            // span of keys from key_lo to the end of the batch)
    uint32_t n_elabels;
    uint32_t n_debi_bits;
    uint32_t n_vf_bits;
    uint32_t pad;
    const uint32_t* in_src;
    const uint32_t* in_dst;
    const uint8_t* in_lab;
    const int64_t* in_ts;
    const uint64_t* del_keys;
    uint32_t* free_stack;
    uint32_t* key2slot;
    uint32_t* delbits;
    uint32_t* err;
    int64_t* last_ts;
    uint32_t* ins_slot;
    uint64_t* skey[2];
    uint32_t* sval[2];
    uint32_t* touched;
    const uint32_t* prev_del_slot;
    uint32_t* del_slot;
    uint32_t* delpos[2];
    const DebiBit* debi_bits;
    const VfBit* vf_bits;
};

void mn_launch_reset(uint32_t* err, unsigned long long* zero_a, uint32_t n_a, hipStream_t s);
void mn_launch_validate(const GraphView& g, const BatchView& b, hipStream_t s);
void mn_launch_prev_del(const GraphView& g, const BatchView& b, hipStream_t s);
void mn_launch_ingest(const GraphView& g, const BatchView& b, hipStream_t s);
// One direction of the per-batch adjacency merge. Old arrays: off (nv + 1),
// adj and adjk (e_old). Batch: bk (n_b sorted keys, kbase + vertex << hb |
// high word) with their slots bv; dpos (n_d sorted deleted positions plus
// dbase, or null); kbase and dbase are the direction bit of the combined sort.
// Outputs: newoff (nv + 1), meta (nv), adj_new and adjk_new (e_new), inspos
// and ub (n_b), lim (mn_merge_limit_words(e_old)).
struct MergeSide {
    const uint32_t* off;
    const uint64_t* adj;
    const uint64_t* adjk;
    const uint64_t* bk;
    uint64_t kbase;
    const uint32_t* bv;
    const uint64_t* dpos;
    uint64_t dbase;
    uint32_t* newoff;
    uint4* meta;
    uint64_t* adj_new;
    uint64_t* adjk_new;
    uint32_t* inspos;
    uint32_t* ub;
    uint32_t* lim;
};
// Merged adjacency of both directions (side[0], side[1]) in one launch per
// step: vertex runs and offsets, batch entries at their insertion points,
// the tile limits, then the kept old entries.
void mn_launch_merge(const MergeSide* side, uint32_t n_vertices, uint32_t e_old, const uint64_t* s_key,
                     uint32_t n_b, uint32_t n_d, uint32_t hb, uint32_t e_new, uint32_t* err, hipStream_t s);
// Words of the merge's tile-limit buffer for an old adjacency of e_old entries.
uint64_t mn_merge_limit_words(uint64_t e_old);
// Query-dependent state of the present edges after a change of the query
// set: edgeMatcher words of the live slots among [0, n_slots) and counter
// increments for them and for the n_pend slots deleted by the last batch.
// The counters must be zero before.
void mn_launch_reindex(const GraphView& g, const DebiBit* bits, uint32_t n_bits, uint32_t n_slots,
                       const uint32_t* key2slot, uint64_t key_lo, const uint32_t* pend, uint32_t n_pend,
                       hipStream_t s);
void mn_launch_vf_refresh(const GraphView& g, const VfBit* bits, uint32_t n_bits,
                          const uint32_t* list, uint32_t n, const uint32_t* err, hipStream_t s);
// One round of the spanning-tree filter over the n_v vertices of g: for each
// of the n steps, vertices whose bit `test` lacks a neighbour with bit `need`
// (TreeStep) lose it in vf (n_v x g.vf_words words). Steps of one launch
// must not test a bit another of them needs. cleared (optional) counts the
// bits cleared.
void mn_launch_tree_step(const GraphView& g, uint32_t* vf, const TreeStep* steps, uint32_t n, uint32_t n_v,
                         unsigned long long* cleared, const uint32_t* err, hipStream_t s);
// Sets (set != 0) or clears the flag bit of the entries at pos0[i] of adj0
// and pos1[i] of adj1 (both directions, i < n) in one launch.
void mn_launch_set_flags(uint64_t* adj0, const uint32_t* pos0, uint64_t* adj1, const uint32_t* pos1, uint32_t n,
                         int set, const uint32_t* err, hipStream_t s);
void mn_launch_flag_del(const GraphView& g, uint64_t* adj_out, uint64_t* adj_in, const BatchView& b,
                        hipStream_t s);
void mn_launch_finalize(const BatchView& b, uint32_t n_free_after, hipStream_t s);
// Moves *lo past the dead keys (key2slot INVALID) below the first live one,
// at most up to `end` (one block; no-op once err is set).
void mn_launch_advance_lo(const uint32_t* key2slot, uint64_t key_mask, uint64_t* lo, uint64_t end,
                          const uint32_t* err, hipStream_t s);
// Key-map ring growth: copies the entries of keys [lo, hi) from the rings of
// mask m_old to those of mask m_new.
void mn_launch_ring_copy(const uint32_t* k2s_old, const int64_t* ts_old, uint64_t m_old, uint32_t* k2s_new,
                         int64_t* ts_new, uint64_t m_new, uint64_t lo, uint64_t hi, hipStream_t s);
// p[i] = v for i < n.
void mn_launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
void mn_launch_init_vertices(uint32_t* vf, uint32_t* cnt, uint32_t n_vertices, uint32_t vf_words,
                             uint32_t n_cnt, hipStream_t s);

// ------------------------------------------------------------- enumeration
struct OutView {
    uint64_t* keys[2];            // [phase] base of this query's tuple buffer
    uint64_t cap[2];              // tuples
};

struct EnumStats {  // per phase, accumulated by the enumeration kernels
    unsigned long long seeds;         // start rows (work units) that passed the filters
    unsigned long long entries;       // candidate entries tested by k_expand
    unsigned long long probes;        // adjacency words read by closing-edge lookups in k_expand
    unsigned long long range_probes;  // adjacency words read by the candidate-range searches
    unsigned long long keys;          // edge keys gathered for emission
    unsigned long long tuples;
    unsigned long long vf_reads;
    unsigned long long rows;          // partial embeddings written between levels
    unsigned long long vf_rejects;    // work units and candidates the vertex filter eliminated
};
static_assert(sizeof(EnumStats) == MN_TALLIES * 8, "tallies");

// Per-phase outputs. Digests and tallies have MN_SHARDS copies so that
// blocks spread their atomics over many addresses: block b adds into copy
// b % MN_SHARDS, the host sums the copies.
struct PhaseOut {
    unsigned long long* count;    // [n_queries]
    unsigned long long* digest;   // [MN_SHARDS][n_queries][2]
    EnumStats* stats;             // [MN_SHARDS]
    uint32_t n_q;
    const OutView* outs;          // [n_queries]
    int phase;                    // 0 new, 1 expired: which buffer of outs[q]
    int emit;                     // write tuples (else counts and digests only)
};

// Start rows: one per (batch slot, start position) whose edgeMatcher bit and
// endpoint filters pass and whose start-level closing edges exist. Plans with
// no further level emit their embeddings directly. *n_rows counts every row,
// also those past rows.cap, which are not written. n_plans: the static plans
// (one per pair); each row takes the order g.sched_mode selects.
// max_close: the most closing edges any plan has (sizes the kernels' arrays).
void mn_launch_seed_rows(const GraphView& g, const uint32_t* slots, uint32_t n, uint32_t n_plans, uint32_t max_close,
                         RowsView rows, uint32_t* n_rows, PhaseOut po, const uint32_t* err, hipStream_t s);
// Settles the order of the start rows the seed kernel listed in g.dec
// (learned choice and/or trace entries); cap bounds the list, expect (the
// rows the host expects) sizes the grid.
void mn_launch_decide(const GraphView& g, RowsView rows, const uint32_t* slots, uint32_t cap, uint32_t expect,
                      int phase, hipStream_t s);
// note[0] = 1 when *count > cap; note[1] = max(note[1], *count).
void mn_launch_note_count(const uint32_t* count, uint64_t cap, unsigned long long* note, hipStream_t s);

// Candidate range of every row at level L: lo[r] and cnt[r]. With n_dev the
// row count is min(n, *n_dev), read on the device (n sizes the launch), and
// note (optional) records it against n: note[0] = 1 when it is larger,
// note[1] = the largest count seen. zero_next (optional) is set to 0.
void mn_launch_level_range(const GraphView& g, RowsView rows, uint32_t n, const uint32_t* n_dev, uint32_t L,
                           uint32_t* lo, uint32_t* cnt, EnumStats* st, const uint32_t* err, hipStream_t s,
                           uint32_t* zero_next = nullptr, unsigned long long* note = nullptr);
// Grid cap of a device-sized expansion (its candidate total is only known on
// the device): one launch covers at most this many tiles.
constexpr uint64_t MN_EXPAND_MAX_BLOCKS = 1u << 20;

// Tests the candidates [c0, c1) of level L (flattened over rows by the
// offsets `off`); survivors become rows of `out` or, at a plan's last level,
// emitted embeddings.
// tile_row must hold mn_expand_tiles(c0, c1) + 1 words (enough for any tile size).
uint64_t mn_expand_tiles(uint64_t c0, uint64_t c1);
// rows: some plan continues past level L; emit: some plan ends at level L.
// Host-sized form: n_dev = cnt = T_dev = note = NULL, candidates exactly
// [c0, c1). Device-sized form: the row count is min(n_in, *n_dev), the
// candidate total T = off[n-1] + cnt[n-1] is stored in *T_dev and the
// candidates are [c0, min(c1, T)); note[0] is set when T > c1 and note[1]
// keeps the largest T (the host grows buffers and re-runs); `expect`,
// the candidates the host expects, only sizes the grid. items (1, 2 or 4)
// sets the tile: 256 x items candidates per block.
// Returns the end of the candidates the launch covers (c1, lowered to what
// the grid covers in the device-sized form). ev0/ev1, when given, are
// recorded right before and after the k_expand launch itself.
uint64_t mn_launch_expand(const GraphView& g, RowsView in, uint32_t n_in, const uint32_t* n_dev, const uint32_t* lo,
                      const uint64_t* off, const uint32_t* cnt, uint32_t* tile_row, uint64_t c0, uint64_t c1,
                      uint64_t* T_dev,
                      unsigned long long* note, uint64_t expect, uint32_t items, uint32_t L, uint32_t max_close,
                      bool rows, bool emit, RowsView out, uint32_t* n_out, PhaseOut po, const uint32_t* err,
                      hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, bool partitioned = false);
// The device-sized form of a level in fewer launches: after mn_scan64_local
// over the row counts (nb tiles, nb <= MN_SCAN_DIRECT_MAX), completes off,
// stores the candidate total in *T_dev (noted against c1) and writes the
// tile_row partition that mn_launch_expand(..., partitioned = true) then
// uses. c1 must be mn_expand_end(c0, c1, expect, items), the end that launch
// covers.
uint64_t mn_expand_end(uint64_t c0, uint64_t c1, uint64_t expect, uint32_t items);
void mn_launch_offsets_partition(const uint32_t* cnt, uint64_t* off, const uint64_t* sums, uint32_t nb, uint32_t n,
                                 const uint32_t* n_dev, uint64_t c0, uint64_t c1, uint64_t* T_dev, uint32_t items,
                                 uint32_t* tile_row, unsigned long long* note, hipStream_t s);

// Stores v into *p (a device word) in stream order.
void mn_launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s);

// out[i] = add + in[i] as u64 (sort keys).
// out0[i] = add0 + in0[i] and out1[i] = add1 + in1[i] for i < n, in one launch.
void mn_launch_widen(const uint32_t* in0, uint64_t* out0, uint64_t add0, const uint32_t* in1, uint64_t* out1,
                     uint64_t add1, uint32_t n, const uint32_t* err, hipStream_t s);

// ------------------------------------------------------------ order network
// The scheduler's 24 -> 64 -> 64 -> 1 network (weights as in mn_common.h).
// y[i] = net(x[i]) for n samples of 24 floats. bf16 != 0: bf16 inference on
// the matrix cores (weights, inputs and first hidden layer rounded to
// bfloat16, fp32 sums), as the decision kernel evaluates; else fp32 throughout.
void mn_mlp_predict(const float* w, const float* x, uint64_t n, int bf16, float* y, hipStream_t s);
// Adds to grad the gradient of mean((net(x[k]) - target[k])^2) over the m
// samples k = idx[off + t] (t < m; idx NULL: k = off + t), and that mean to *loss.
void mn_mlp_grad(const float* w, const float* x, const float* target, const uint32_t* idx, uint64_t off,
                 uint64_t m, float* grad, float* loss, hipStream_t s);
// One Adam step (step >= 1) on all weights; clears grad.
void mn_mlp_adam(float* w, float* m1, float* m2, float* grad, float lr, uint32_t step, hipStream_t s);
void mn_fill_f32(float* p, float v, uint32_t n, hipStream_t s);
// out[i] = bfloat16 of in[i] (nearest, ties to even).
void mn_to_bf16(const float* in, uint16_t* out, uint32_t n, hipStream_t s);
