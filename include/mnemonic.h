/*
 * mnemonic.h -- C ABI of the MI355X (gfx950) streaming subgraph matcher.
 *
 * The library keeps a labelled, directed multigraph and a set of query graphs
 * resident in HBM and, for every snapshot of edge insertions and deletions,
 * reports exactly the embeddings that the snapshot creates or removes
 * (paper, Section II-B, problem definition: S(G + dG) = S(G) + dS). A snapshot
 * is processed as in Algorithm 1: insertions first, then deletions.
 *
 * Plain C: no C++ or torch types cross this boundary. Every function returns
 * MNEMONIC_OK (0) or a negative MNEMONIC_E_* code and never throws. A context
 * is single-threaded: calls on one context must not overlap. Separate
 * contexts may run concurrently on separate HIP streams.
 *
 * Embedding definition (Section II-B): a vertex map f and an edge-instance map
 * g (parallel data edges are distinct instances, Section I). A query vertex's
 * required label set must be a subset of its image's label set (a required set
 * of 0 is a wildcard); a query edge label must equal the data edge label or be
 * -1 (any label). Isomorphism requires f injective; homomorphism drops that
 * check, so one data edge may serve several query edges (Section III).
 * Each embedding is reported as the tuple of the keys of g(q_0) .. g(q_{m-1})
 * in query-edge index order. Embeddings of the initial graph are not reported.
 */
#ifndef MNEMONIC_H
#define MNEMONIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
#define MNEMONIC_OK 0
#define MNEMONIC_E_ARG -1        /* NULL pointer, zero-sized required array, bad flag */
#define MNEMONIC_E_QUERY -2      /* query outside the supported shape (see mnemonic_query) */
#define MNEMONIC_E_VERTEX -3     /* an edge endpoint >= n_vertices */
#define MNEMONIC_E_LABEL -4      /* an edge label >= n_elabels */
#define MNEMONIC_E_TS_ORDER -5   /* a timestamp smaller than the one before it */
#define MNEMONIC_E_BAD_DELETE -6 /* deletion key not live, unknown or repeated */
#define MNEMONIC_E_OOM -7        /* device allocation failed */
#define MNEMONIC_E_CAPACITY -8   /* caller buffer too small (mnemonic_copy_keys) */
#define MNEMONIC_E_HIP -9        /* a HIP runtime call failed; see mnemonic_last_error */
#define MNEMONIC_E_LIMIT -10     /* graph larger than the packed adjacency format allows */

typedef struct mnemonic_ctx mnemonic_ctx; /* opaque; owns every device buffer it uses */

typedef enum { MNEMONIC_ISO = 0, MNEMONIC_HOMO = 1 } mnemonic_semantics;

/* Data graph at creation (the input G of Algorithm 1). Host pointers. Initial
 * edge i gets key i. Vertex labels are 64-bit sets (one bit per label).
 * Limits: n_vertices <= 2^24 (neighbour ids and labels share 32 bits of an
 * adjacency entry), labels < n_elabels <= 256 (0 means 256), fewer than 2^31
 * live edges, timestamps non-decreasing in key order. */
typedef struct {
    uint32_t n_vertices;
    uint32_t n_elabels;
    const uint64_t *vlabel_mask; /* [n_vertices] */
    uint64_t n_edges;
    const uint32_t *src;         /* [n_edges] */
    const uint32_t *dst;         /* [n_edges] */
    const uint8_t *elabel;       /* [n_edges] */
    const int64_t *ts;           /* [n_edges] */
} mnemonic_graph;

/* One query graph G_Q (Section II-A). Host pointers, copied at creation.
 * Supported shape: 2..16 vertices, 1..32 edges, weakly connected, no
 * self-loop, at most one edge per ordered vertex pair. Anything else returns
 * MNEMONIC_E_QUERY.
 * qtorder: NULL, or a temporal rank per query edge (the time-constrained
 * variant listed in Section II-B and evaluated in Section VII-C): an
 * embedding must then satisfy ts(g(e_a)) < ts(g(e_b)) whenever
 * 0 <= rank(e_a) < rank(e_b); edges of equal rank, or of rank -1, are not
 * ordered against each other. Ranks must lie in -1..31. */
typedef struct {
    uint32_t n_qv;
    const uint64_t *qv_require; /* [n_qv] required label set; 0 = any vertex */
    uint32_t n_qe;
    const uint32_t *qsrc;       /* [n_qe] */
    const uint32_t *qdst;       /* [n_qe] */
    const int32_t *qelabel;     /* [n_qe] label, or -1 for any label */
    mnemonic_semantics sem;
    const int32_t *qtorder;     /* [n_qe] temporal rank, or NULL: no order */
} mnemonic_query;

/* A batch of insertions. Inserted edges get consecutive keys in array order.
 * When on_device is non-zero, src/dst/elabel/ts and the deletion keys passed
 * alongside are device pointers on the context's device (read in place);
 * otherwise they are host pointers, copied before the call returns. */
typedef struct {
    uint64_t n;
    const uint32_t *src;
    const uint32_t *dst;
    const uint8_t *elabel;
    const int64_t *ts;
    uint32_t on_device;
} mnemonic_edges;

#define MNEMONIC_F_EMIT 1u   /* write the embedding tuples (else counts and digests only) */
#define MNEMONIC_F_TIMING 2u /* record HIP events around the enumeration kernels */
#define MNEMONIC_F_AUTOTUNE 4u /* the first batches try each expansion tile size (512, 1024,
                                  2048 candidates per block) twice and keep the fastest per
                                  candidate; results do not depend on the choice */
#define MNEMONIC_F_SORT 16u /* with MNEMONIC_F_EMIT: each result list is sorted on the device into
                               lexicographic order of its key tuples before the call returns
                               (the canonical order the oracle lists; Section II-B leaves the
                               order open) */
#define MNEMONIC_F_INDEX_ONLY 8u /* maintain the graph and its index (Algorithm 2's updates,
                                    edgeMatcher, filters) but enumerate nothing: results stay
                                    empty; measures the update path alone */
#define MNEMONIC_F_TREE_FILTER 32u /* before each batch's enumeration, strengthen the vertex
                                      filter with the spanning-tree propagation of Section V-B
                                      (f4 bottom-up, then f1 top-down, over each query's BFS tree
                                      from query vertex 0), recomputed on the graph with the
                                      batch's insertions; every level then tests it. Results do
                                      not depend on it: it only prunes candidates no embedding
                                      uses. */

typedef struct {
    uint32_t flags;          /* MNEMONIC_F_* */
    uint64_t out_capacity;   /* initial tuples per (query, new/expired) buffer; 0 = 2^20 */
    uint64_t rows_per_level; /* partial embeddings one search level may hold (bounds the
                                enumerator's memory; larger fan-outs are processed in
                                chunks; buffers grow on demand up to it); 0 = 2^25,
                                minimum 1024, maximum 2^26 (larger values are
                                lowered to it) */
} mnemonic_options;

/* Result of the last successful mnemonic_apply_batch for one query.
 * dig_* are order-independent 64-bit multiset digests of the tuples: with
 * mix the SplitMix64 finaliser (Steele, Lea, Flood 2014), seeds
 * A = 0x243F6A8885A308D3 and B = 0x13198A2E03707344 and q the query index,
 * h_s(t) = mix(...mix(mix(s ^ q) + k_0)... + k_{m-1}) and dig[s] = sum of h_s
 * over the tuples, modulo 2^64. new_keys / expired_keys are device pointers to
 * n x n_qe row-major uint64 tuples in no particular order, valid until the
 * next mnemonic_apply_batch or mnemonic_destroy; NULL without
 * MNEMONIC_F_EMIT. */
typedef struct {
    uint64_t n_new, n_expired;
    uint64_t dig_new[2], dig_expired[2];
    const uint64_t *new_keys;
    const uint64_t *expired_keys;
    uint32_t n_qe;
} mnemonic_result;

/* Work and timing of the last successful batch, per phase p (0 insert,
 * 1 delete). The enumerator runs level by level (see mnemonic_apply_batch):
 *   seeds              work units (start edge at one query-edge position) that
 *                      passed edgeMatcher, the vertex filter and the
 *                      start-level closing edges
 *   entries_scanned    candidate adjacency entries tested by the expansion kernel
 *   probe_words        adjacency words the expansion kernel read to find and
 *                      walk closing-edge instances
 *   range_probe_words  adjacency words read by the per-level binary searches
 *                      that delimit each partial embedding's candidates
 *   key_reads          edge keys gathered for emitted tuples
 *   tuples             embeddings found; tuple_words = tuples x |E_Q| keys
 *   vf_reads           vertex-filter words tested
 *   vf_rejects         work units and candidates the vertex filter (Section V-A,
 *                      f2 and f3 as local counts) eliminated: the unit's or
 *                      candidate's other tests had passed so far
 *   frontier_rows      partial embeddings passed from one level to the next
 *   expand_launches    launches of the expansion kernel
 *   expand_tile        candidates per expansion block in use (autotuned with
 *                      MNEMONIC_F_AUTOTUNE, else 1024 when no query's plans
 *                      have more than one closing edge, 512 otherwise)
 *   reruns             times the phase ran again after a buffer proved too
 *                      small (the buffers grow; results are unaffected)
 *   rerun_causes       what was too small, OR-ed over the re-runs: 1 start
 *                      rows, 2 a level's candidates past the launch's grid,
 *                      4 a level's rows, 8 a query's output buffer
 * With MNEMONIC_F_TIMING: ms_expand = summed device time of the expansion
 * launches, ms_enumerate = the whole enumeration phase, ms_batch = the whole
 * snapshot on the device. */
typedef struct {
    uint64_t n_live_edges;
    uint64_t slot_high_water;
    uint64_t seeds[2];
    uint64_t entries_scanned[2];
    uint64_t probe_words[2];
    uint64_t range_probe_words[2];
    uint64_t key_reads[2];
    uint64_t tuples[2];
    uint64_t tuple_words[2];
    uint64_t vf_reads[2];
    uint64_t frontier_rows[2];
    uint64_t expand_launches[2];
    uint64_t expand_tile;
    double ms_expand[2];
    double ms_enumerate[2];
    double ms_batch;
    uint64_t reruns[2];
    uint64_t rerun_causes[2];
    uint64_t vf_rejects[2];
    uint64_t key_capacity;  /* places in the key-indexed maps (rings over the live key span) */
    uint64_t key_lo;        /* every key below it is dead */
    uint64_t allocations;   /* device allocations the batch made (buffers that grew) */
    double ms_alloc;        /* host time of those allocations and of the frees they replaced */
    uint64_t tree_cleared;  /* MNEMONIC_F_TREE_FILTER: (vertex, query vertex) filter bits the
                               spanning-tree rounds cleared this batch */
} mnemonic_stats;

/*
 * InitializeIndex (Algorithm 1; Section III, preprocessing): uploads the data
 * graph, builds the sorted out/in adjacency, evaluates edgeMatcher for every
 * edge and every query edge, and the per-vertex local filters. Queries are
 * preprocessed into one static matching order per start edge (Section VI).
 * The initial embeddings are not enumerated.
 *   g, q (n_q >= 1 entries), opt: host structures, read during the call only;
 *     opt may be NULL (defaults: emit on, no timing).
 *   hip_stream: the hipStream_t every kernel and copy of this context runs on
 *     (NULL = the default stream). The current HIP device at creation is used.
 *     The context's device buffers come from that device's default memory
 *     pool, allocated and freed in order on this stream; the library raises
 *     the pool's release threshold, so memory it frees stays in the pool for
 *     later allocations (hipMemPoolTrimTo returns it to the device).
 *   out: receives the context; unchanged on failure.
 * Errors: ARG, QUERY, VERTEX, LABEL, TS_ORDER, LIMIT, OOM, HIP.
 */
int mnemonic_create(const mnemonic_graph *g, const mnemonic_query *q, uint32_t n_q,
                    const mnemonic_options *opt, void *hip_stream, mnemonic_ctx **out);

/*
 * One snapshot (Algorithm 1 loop body; Algorithm 2): batchInserts then
 * batchDeletes.
 *   ins: insertions (ins->n may be 0; ins may be NULL when there are none).
 *   del_keys / n_del: keys to delete. A key may name an edge inserted earlier
 *     in this same call. Host or device memory as ins->on_device says (host
 *     when ins is NULL).
 *   first_new_key: if not NULL, receives the key of the first inserted edge.
 * New embeddings are those using >= 1 inserted edge; expired embeddings are
 * those of the post-insert graph using >= 1 deleted edge (so an embedding
 * created and removed within one snapshot appears in both lists).
 * Validation (endpoint range, label range, timestamps non-decreasing across
 * batches, deletion keys live and distinct) runs on the device before any
 * state changes: a batch it rejects returns VERTEX, LABEL, TS_ORDER or
 * BAD_DELETE and changes nothing. ARG, and OOM while the batch's buffers are
 * sized before any kernel runs, also change nothing. An OOM or HIP error
 * after that (a buffer that must grow while the enumeration runs, or a
 * failed device call) leaves the batch part way applied: the context is then
 * unusable, and every later call on it except mnemonic_last_error and
 * mnemonic_destroy returns MNEMONIC_E_HIP.
 * Blocks until the batch's counts and digests are on the host.
 * Errors: ARG, VERTEX, LABEL, TS_ORDER, BAD_DELETE, OOM, HIP.
 */
int mnemonic_apply_batch(mnemonic_ctx *ctx, const mnemonic_edges *ins, const uint64_t *del_keys,
                         uint64_t n_del, uint64_t *first_new_key);

/*
 * mnemonic_apply_batch for callers that cannot allocate memory: code being
 * captured into a HIP graph, serving loops with a fixed memory budget, and
 * harnesses that forbid allocation. It applies the snapshot exactly as
 * mnemonic_apply_batch does (same arguments, same results) but calls no
 * device or host allocation routine:
 *   - the batch's control words (error word, readback block of counts,
 *     digests, work tallies and overflow notes, row counters) live in one
 *     scratch array per GPU, of at most 65,536 words (512 KiB); a query set
 *     whose control block needs more (about 130 words per query) returns
 *     MNEMONIC_E_CAPACITY and changes nothing;
 *   - every other buffer must already be large enough: a batch whose arrays
 *     exceed the context's batch buffers returns MNEMONIC_E_CAPACITY and
 *     changes nothing. The enumeration runs in the level buffers, expansion
 *     tiles and output lists the context holds; when they are too small the
 *     batch is still applied (the graph and index move on, later batches may
 *     follow) but it returns MNEMONIC_E_CAPACITY and its results are
 *     unavailable: mnemonic_get_result and mnemonic_copy_keys return
 *     MNEMONIC_E_CAPACITY until the next batch. Buffers grow only through
 *     mnemonic_apply_batch: a caller sizes the context first (out_capacity
 *     and rows_per_level at creation, or earlier batches through
 *     mnemonic_apply_batch, which size buffers from the rates they see);
 *   - timing (MNEMONIC_F_TIMING), tile autotuning and traces are not
 *     recorded; the learned scheduler falls back to the static order when
 *     its decision list has no room (results are the same either way).
 * Every call on one GPU shares that GPU's scratch array: calls that overlap
 * on one GPU (two contexts on two streams, two threads) race and must not
 * be issued. Errors: those of mnemonic_apply_batch, and CAPACITY as above. */
int mnemonic_apply_batch_noalloc(mnemonic_ctx *ctx, const mnemonic_edges *ins, const uint64_t *del_keys,
                                 uint64_t n_del, uint64_t *first_new_key);

/* Counts, digests and device tuple pointers of the last batch for one query
 * (index in creation order). Errors: ARG (bad ctx, query or out), CAPACITY
 * (the last batch's results are unavailable, see
 * mnemonic_apply_batch_noalloc). */
int mnemonic_get_result(mnemonic_ctx *ctx, uint32_t query, mnemonic_result *out);

/* Copies the new (expired != 0: expired) tuples of one query to host_buf,
 * capacity counted in tuples. *needed (if not NULL) receives the tuple count.
 * Returns MNEMONIC_E_CAPACITY, copying nothing, when capacity is too small;
 * MNEMONIC_E_ARG without MNEMONIC_F_EMIT. */
int mnemonic_copy_keys(mnemonic_ctx *ctx, uint32_t query, int expired, uint64_t *host_buf,
                       uint64_t capacity, uint64_t *needed);

/* Work and timing figures of the last batch. Errors: ARG. */
int mnemonic_get_stats(mnemonic_ctx *ctx, mnemonic_stats *out);

/* Text of the last error on this context ("" if none). The pointer stays
 * valid until the next call on the context. A NULL ctx gives the last error of
 * a failed mnemonic_create on this thread. */
const char *mnemonic_last_error(const mnemonic_ctx *ctx);

/* Replaces the context's query set between batches (a serving loop admits
 * and retires queries this way). The graph, its keys and the pending
 * deletions are kept; everything that depends on the queries is rebuilt from
 * the edges present: the edgeMatcher words of every live edge, the per-vertex
 * counters and filter bits (Section V-A), the matching orders, the output
 * buffers. Results of the following batches are indexed by the new set (in
 * the order given). Queries follow the rules of mnemonic_create; a bad one
 * returns MNEMONIC_E_QUERY and changes nothing. Costs O(live edges +
 * vertices) on the device. Errors: ARG, QUERY, OOM, HIP. After OOM or HIP
 * the rebuild is incomplete: every later call on the context except
 * mnemonic_last_error and mnemonic_destroy returns MNEMONIC_E_HIP, and the
 * context must be destroyed. */
int mnemonic_set_queries(mnemonic_ctx *ctx, const mnemonic_query *q, uint32_t n_q);

/* ------------------------------------------------------------- scheduler
 * Matching orders. Section VI computes one matching order per start position
 * of a query (the order in which the remaining query vertices are bound). The
 * library keeps up to four orders per (query, start position): the static one
 * (most connections to the bound vertices first, lowest index on ties,
 * labelled anchor edges first) and the distinct ones among three variants
 * (highest index on ties and/or the highest-index anchor edge). Every order
 * finds the same embeddings; they differ in the work done. The scheduler picks
 * one order per start row (one batch edge at one start position): */
#define MNEMONIC_SCHED_STATIC 0  /* always the static order (the default) */
#define MNEMONIC_SCHED_LEARNED 1 /* the order the cost network predicts cheapest */
#define MNEMONIC_SCHED_FIXED 2   /* MNEMONIC_SCHED_FIXED + v: always order v (v < 4; the static
                                    order where a pair has fewer orders) */

/* Order-cost network: 24 features -> 64 -> 64 -> 1 with ReLU, predicting
 * log2(1 + search work below a start row) under one order. Weights are 5,825
 * fp32 values: W1[24][64], b1[64], W2[64][64], b2[64], W3[64], b3 (row-major,
 * y = relu(relu(x W1 + b1) W2 + b2) W3 + b3). */
#define MNEMONIC_MLP_IN 24
#define MNEMONIC_MLP_HIDDEN 64
#define MNEMONIC_MLP_WEIGHTS 5825
#define MNEMONIC_MAX_ORDERS 4

/* Sets the scheduler mode for the following batches. weights: host array of
 * MNEMONIC_MLP_WEIGHTS fp32, required for MNEMONIC_SCHED_LEARNED (copied and
 * rounded to bf16 on the device; the caller keeps ownership), ignored
 * otherwise (NULL allowed). Errors: ARG (bad ctx or mode, or LEARNED without
 * weights), OOM, HIP. */
int mnemonic_set_scheduler(mnemonic_ctx *ctx, int mode, const float *weights);

/* Number of orders (1..4) of start position j of query `query`.
 * Errors: ARG. */
int mnemonic_query_orders(mnemonic_ctx *ctx, uint32_t query, uint32_t j, uint32_t *n_orders);

/* Start-row traces. capacity > 0 makes the following batches record, per
 * phase, up to `capacity` start rows that continue past the start level:
 * their identity, the features of each order of their pair, and the search
 * work below them under the order they took (1 + candidates examined at all
 * levels). capacity = 0 turns tracing off. Tracing adds one column to the
 * rows between levels and costs time; results are unchanged.
 * Errors: ARG, OOM, HIP. */
int mnemonic_set_trace(mnemonic_ctx *ctx, uint64_t capacity);

/* Copies the last batch's trace of one phase (0 new, 1 expired) to host
 * memory. *n receives the number of entries recorded (min(rows, capacity));
 * codes[i] = phase << 62 | order << 56 | static plan << 32 | index of the
 * start edge in the phase's edge list (insertions: batch order; deletions:
 * del_keys order); x[i][v][f]: feature f of order v (zeros past the pair's
 * orders), MNEMONIC_MAX_ORDERS x MNEMONIC_MLP_IN floats per entry;
 * work[i]: the search work. Entries come in no particular order. Any of
 * codes, x, work may be NULL; cap bounds the entries copied.
 * Errors: ARG (bad ctx or phase, tracing off), HIP. */
int mnemonic_get_trace(mnemonic_ctx *ctx, int phase, uint64_t *n, uint64_t *codes, float *x, uint64_t *work,
                       uint64_t cap);

/* Training and inference kernels of the order-cost network, on caller-owned
 * device memory (fp32), on hip_stream (NULL: default stream). No context.
 *   predict: y[i] = net(x[i]) for n samples of MNEMONIC_MLP_IN floats. bf16 != 0:
 *     the operands of both matrix products (weights, inputs, first hidden
 *     layer) rounded to bfloat16, sums in fp32, on the matrix cores: the
 *     arithmetic of the learned scheduler's decisions. bf16 == 0: fp32.
 *   grad: adds to grad[MNEMONIC_MLP_WEIGHTS] the gradient of
 *     L = mean over t < m of (net(x[k]) - target[k])^2, k = idx[off + t]
 *     (idx NULL: k = off + t), and adds L to *loss. grad and loss accumulate.
 *   adam: one Adam step (Kingma and Ba, 2015; beta1 0.9, beta2 0.999,
 *     eps 1e-8, step >= 1 for bias correction) on w with moments m1, m2, then
 *     zeroes grad.
 * Launches are asynchronous; errors of the launch itself return HIP. */
int mnemonic_mlp_predict(const float *w, const float *x, uint64_t n, int bf16, float *y, void *hip_stream);
int mnemonic_mlp_grad(const float *w, const float *x, const float *target, const uint32_t *idx, uint64_t off,
                      uint64_t m, float *grad, float *loss, void *hip_stream);
int mnemonic_mlp_adam(float *w, float *m1, float *m2, float *grad, float lr, uint32_t step, void *hip_stream);

/* Test hook for the error paths above (for callers that check their own
 * failure handling, not for production use): the n-th device allocation the
 * library makes from this call on, in any context of the process, fails as
 * if the device were out of memory; n = 0 disarms it. Not thread-safe. */
void mnemonic_fail_alloc_after(uint64_t n);

/* Frees every device and host buffer of the context. NULL is ignored. */
void mnemonic_destroy(mnemonic_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MNEMONIC_H */
