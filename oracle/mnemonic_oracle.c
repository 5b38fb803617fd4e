/*
 * Oracle for the streaming subgraph matcher -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded C implementation of what the GPU path must
 * compute. Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product library never does. It shares no
 * code, header or table with the HIP path.
 *
 * What it computes (paper, Section II-B "Problem Definition"): for a snapshot
 * with insert set I and delete set D, applied in the order of Algorithm 1
 * (insertions, then deletions),
 *     new     = S(G u I) \ S(G)          (embeddings that use >= 1 edge of I)
 *     expired = S(G u I) \ S(G u I \ D)  (embeddings that use >= 1 edge of D)
 * An embedding is a vertex map f plus an edge-instance map g (Section I:
 * parallel edges are distinct instances). Conditions (Section II-B):
 *   - vertex labels: required set of u is a subset of the label set of f(u)
 *   - edge labels: equal, or the query edge label is empty (matches any;
 *     caption of the example figure in Section I)
 *   - isomorphism: f injective; homomorphism: no injectivity, one data edge
 *     may serve several query edges (Section III, homomorphism paragraph).
 *   - temporal order, when the query gives ranks (the time-constrained
 *     variant listed among the matching variants of Section II-B, evaluated
 *     in Section VII-C):
 *     ts(g(e_a)) < ts(g(e_b)) whenever rank(e_a) < rank(e_b); edges of equal
 *     rank, or of rank -1, are unconstrained against each other. Checked on
 *     each complete embedding.
 *
 * How (Section VI "Embedding Enumeration"): every edge of the batch that
 * matches query edge q_j is a work unit; the enumerator backtracks from it in
 * a fixed order, and the duplicate-removal mask forbids batch edges at every
 * query position k < j, so an embedding that uses several batch edges is
 * produced exactly once, from its smallest batch-using position. The prose
 * example of that section is followed for the mask direction (earlier
 * positions masked); the result set does not depend on that choice.
 *
 * Adjacency lists hold live keys in arrival order; removal swaps with the
 * last entry (Section IV-A, "Memory recycling"). Nothing is sorted or indexed.
 *
 * Digest of a result list (order independent): for seed s and query index q,
 *   h_s(t) = mix(... mix(mix(s ^ q) + k_0) ... + k_{m-1})
 *   dig_s  = sum over tuples of h_s(t)  (mod 2^64)
 * where mix is the SplitMix64 output finaliser (Steele, Lea, Flood, OOPSLA
 * 2014; constants as published by Vigna).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXQV 16
#define ORC_MAXQE 32
#define ORC_MAXQ 256

#define ORC_SEED_A 0x243F6A8885A308D3ULL
#define ORC_SEED_B 0x13198A2E03707344ULL

typedef struct {
    uint64_t *a;
    size_t n, cap;
} vec64;

static int vec_push(vec64 *v, uint64_t x) {
    if (v->n == v->cap) {
        size_t nc = v->cap ? v->cap * 2 : 4;
        uint64_t *na = (uint64_t *)realloc(v->a, nc * sizeof(uint64_t));
        if (!na) return -1;
        v->a = na;
        v->cap = nc;
    }
    v->a[v->n++] = x;
    return 0;
}

static void vec_remove_value(vec64 *v, uint64_t x) {
    for (size_t i = 0; i < v->n; i++) {
        if (v->a[i] == x) {
            v->a[i] = v->a[v->n - 1];
            v->n--;
            return;
        }
    }
}

typedef struct {
    uint32_t n_qv, n_qe;
    uint64_t vreq[ORC_MAXQV];
    uint32_t qsrc[ORC_MAXQE], qdst[ORC_MAXQE];
    int32_t qlab[ORC_MAXQE];
    int sem; /* 0 iso, 1 homo */
    int temporal;                /* ranks given */
    int32_t rank[ORC_MAXQE];     /* temporal rank per query edge, -1 = none */
    vec64 res[2];  /* [0] new, [1] expired; flat tuples of n_qe keys */
    uint64_t overflow[2];
} orc_query;

typedef struct {
    uint32_t n_vertices;
    uint64_t *vmask;
    /* edge store indexed by key */
    uint64_t n_keys, cap_keys;
    uint32_t *esrc, *edst;
    uint8_t *elab;
    int64_t *ets;
    uint8_t *live;
    uint8_t *dmark; /* marked for deletion in the current delete phase */
    vec64 *out, *in;
    int64_t last_ts;
    uint32_t n_q;
    orc_query q[ORC_MAXQ];
    /* mask mode for the running enumeration */
    int mask_mode;          /* 0 none, 1 keys >= ins_first, 2 dmark */
    uint64_t ins_first;     /* first key of the last inserted batch */
    uint64_t limit;         /* max tuples kept per list (0 = unlimited) */
    /* scratch used by the backtracking */
    uint32_t order[ORC_MAXQE];
    int64_t f[ORC_MAXQV];
    uint64_t g[ORC_MAXQE];
    uint32_t start_j;
    vec64 *sink;
    uint64_t *sink_overflow;
    uint32_t sink_nqe;
    /* static / per-seed list */
    vec64 aux;
    uint64_t aux_overflow;
} orc_ctx;

uint64_t orc_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t orc_tuple_hash(uint64_t seed, uint32_t qidx, const uint64_t *keys, uint32_t n) {
    uint64_t h = orc_mix64(seed ^ (uint64_t)qidx);
    for (uint32_t i = 0; i < n; i++) h = orc_mix64(h + keys[i]);
    return h;
}

static int grow_keys(orc_ctx *c, uint64_t need) {
    if (need <= c->cap_keys) return 0;
    uint64_t nc = c->cap_keys ? c->cap_keys : 16;
    while (nc < need) nc *= 2;
#define GROW(p, T)                                              \
    do {                                                        \
        T *np_ = (T *)realloc(c->p, nc * sizeof(T));            \
        if (!np_) return -1;                                    \
        c->p = np_;                                             \
    } while (0)
    GROW(esrc, uint32_t);
    GROW(edst, uint32_t);
    GROW(elab, uint8_t);
    GROW(ets, int64_t);
    GROW(live, uint8_t);
    GROW(dmark, uint8_t);
#undef GROW
    memset(c->dmark + c->cap_keys, 0, nc - c->cap_keys);
    memset(c->live + c->cap_keys, 0, nc - c->cap_keys);
    c->cap_keys = nc;
    return 0;
}

static int add_edge(orc_ctx *c, uint32_t s, uint32_t d, uint8_t l, int64_t t) {
    uint64_t k = c->n_keys;
    if (grow_keys(c, k + 1)) return -1;
    c->esrc[k] = s;
    c->edst[k] = d;
    c->elab[k] = l;
    c->ets[k] = t;
    c->live[k] = 1;
    c->dmark[k] = 0;
    c->n_keys = k + 1;
    if (vec_push(&c->out[s], k) || vec_push(&c->in[d], k)) return -1;
    if (t > c->last_ts) c->last_ts = t;
    return 0;
}

void *orc_create(uint32_t n_vertices, const uint64_t *vmask, uint64_t n_edges,
                 const uint32_t *src, const uint32_t *dst, const uint8_t *lab,
                 const int64_t *ts) {
    orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    if (!c) return NULL;
    c->n_vertices = n_vertices;
    c->vmask = (uint64_t *)malloc((n_vertices ? n_vertices : 1) * sizeof(uint64_t));
    c->out = (vec64 *)calloc(n_vertices ? n_vertices : 1, sizeof(vec64));
    c->in = (vec64 *)calloc(n_vertices ? n_vertices : 1, sizeof(vec64));
    if (!c->vmask || !c->out || !c->in) return NULL;
    memcpy(c->vmask, vmask, n_vertices * sizeof(uint64_t));
    c->last_ts = INT64_MIN;
    if (grow_keys(c, n_edges + 1)) return NULL;
    for (uint64_t i = 0; i < n_edges; i++)
        if (add_edge(c, src[i], dst[i], lab[i], ts[i])) return NULL;
    return c;
}

void orc_destroy(void *vc) {
    orc_ctx *c = (orc_ctx *)vc;
    if (!c) return;
    for (uint32_t v = 0; v < c->n_vertices; v++) {
        free(c->out[v].a);
        free(c->in[v].a);
    }
    for (uint32_t i = 0; i < c->n_q; i++) {
        free(c->q[i].res[0].a);
        free(c->q[i].res[1].a);
    }
    free(c->aux.a);
    free(c->out);
    free(c->in);
    free(c->vmask);
    free(c->esrc);
    free(c->edst);
    free(c->elab);
    free(c->ets);
    free(c->live);
    free(c->dmark);
    free(c);
}

void orc_set_limit(void *vc, uint64_t max_tuples) { ((orc_ctx *)vc)->limit = max_tuples; }

/* Returns the query index or -1 when the query is outside the supported
 * shape: 1..16 vertices, 1..32 edges, no self-loop, at most one edge per
 * ordered vertex pair, weakly connected. */
int orc_add_query(void *vc, uint32_t n_qv, const uint64_t *vreq, uint32_t n_qe,
                  const uint32_t *qsrc, const uint32_t *qdst, const int32_t *qlab, int sem) {
    orc_ctx *c = (orc_ctx *)vc;
    if (c->n_q >= ORC_MAXQ || n_qv < 1 || n_qv > ORC_MAXQV || n_qe < 1 || n_qe > ORC_MAXQE)
        return -1;
    if (sem != 0 && sem != 1) return -1;
    for (uint32_t i = 0; i < n_qe; i++) {
        if (qsrc[i] >= n_qv || qdst[i] >= n_qv || qsrc[i] == qdst[i]) return -1;
        for (uint32_t k = 0; k < i; k++)
            if (qsrc[k] == qsrc[i] && qdst[k] == qdst[i]) return -1;
    }
    /* weak connectivity by repeated relaxation */
    uint8_t seen[ORC_MAXQV] = {0};
    seen[0] = 1;
    for (uint32_t it = 0; it < n_qv; it++)
        for (uint32_t i = 0; i < n_qe; i++)
            if (seen[qsrc[i]] || seen[qdst[i]]) seen[qsrc[i]] = seen[qdst[i]] = 1;
    for (uint32_t v = 0; v < n_qv; v++)
        if (!seen[v]) return -1;
    orc_query *q = &c->q[c->n_q];
    memset(q, 0, sizeof(*q));
    q->n_qv = n_qv;
    q->n_qe = n_qe;
    memcpy(q->vreq, vreq, n_qv * sizeof(uint64_t));
    memcpy(q->qsrc, qsrc, n_qe * sizeof(uint32_t));
    memcpy(q->qdst, qdst, n_qe * sizeof(uint32_t));
    memcpy(q->qlab, qlab, n_qe * sizeof(int32_t));
    q->sem = sem;
    return (int)c->n_q++;
}

/* Gives query qi temporal ranks (n_qe values, -1 = unconstrained edge).
 * Returns 0, or -1 for a bad query index. */
int orc_set_temporal(void *vc, uint32_t qi, const int32_t *rank) {
    orc_ctx *c = (orc_ctx *)vc;
    if (qi >= c->n_q) return -1;
    orc_query *q = &c->q[qi];
    q->temporal = 1;
    for (uint32_t k = 0; k < q->n_qe; k++) q->rank[k] = rank[k] < 0 ? -1 : rank[k];
    return 0;
}

/* ---------------------------------------------------------------- matching */

static int label_ok(int32_t ql, uint8_t dl) { return ql < 0 || (uint32_t)ql == dl; }

static int vertex_ok(const orc_ctx *c, const orc_query *q, uint32_t u, uint32_t v) {
    return (q->vreq[u] & ~c->vmask[v]) == 0;
}

static int image_has(const orc_ctx *c, const orc_query *q, uint32_t v) {
    for (uint32_t u = 0; u < q->n_qv; u++)
        if (c->f[u] == (int64_t)v) return 1;
    return 0;
}

static int in_batch(const orc_ctx *c, uint64_t key) {
    if (c->mask_mode == 1) return key >= c->ins_first;
    if (c->mask_mode == 2) return c->dmark[key] != 0;
    return 0;
}

/* Order for a start edge: repeatedly take the lowest-index remaining query
 * edge that touches an already mapped vertex (a breadth-first growth from the
 * start edge; any such order gives the same result set). */
static void make_order(orc_ctx *c, const orc_query *q, uint32_t j) {
    uint8_t vis[ORC_MAXQV] = {0}, used[ORC_MAXQE] = {0};
    vis[q->qsrc[j]] = vis[q->qdst[j]] = 1;
    used[j] = 1;
    uint32_t n = 0;
    while (n + 1 < q->n_qe) {
        for (uint32_t k = 0; k < q->n_qe; k++) {
            if (used[k]) continue;
            if (vis[q->qsrc[k]] || vis[q->qdst[k]]) {
                used[k] = 1;
                vis[q->qsrc[k]] = vis[q->qdst[k]] = 1;
                c->order[n++] = k;
                break;
            }
        }
    }
}

/* Temporal order of a complete embedding: every pair of ranked edges with
 * rank a < rank b has strictly increasing timestamps. */
static int temporal_ok(const orc_ctx *c, const orc_query *q) {
    for (uint32_t a = 0; a < q->n_qe; a++)
        for (uint32_t b = 0; b < q->n_qe; b++)
            if (q->rank[a] >= 0 && q->rank[b] >= 0 && q->rank[a] < q->rank[b] &&
                !(c->ets[c->g[a]] < c->ets[c->g[b]]))
                return 0;
    return 1;
}

static void emit(orc_ctx *c, const orc_query *q) {
    if (q->temporal && !temporal_ok(c, q)) return;
    if (c->limit && c->sink->n >= c->limit * q->n_qe) {
        (*c->sink_overflow)++;
        return;
    }
    for (uint32_t k = 0; k < q->n_qe; k++) vec_push(c->sink, c->g[k]);
}

static void extend(orc_ctx *c, const orc_query *q, uint32_t depth) {
    if (depth + 1 == q->n_qe) {
        emit(c, q);
        return;
    }
    uint32_t k = c->order[depth];
    uint32_t x = q->qsrc[k], y = q->qdst[k];
    int masked = k < c->start_j;
    int64_t fx = c->f[x], fy = c->f[y];
    if (fx >= 0) {
        const vec64 *lst = &c->out[fx];
        for (size_t i = 0; i < lst->n; i++) {
            uint64_t e = lst->a[i];
            if (!label_ok(q->qlab[k], c->elab[e])) continue;
            if (masked && in_batch(c, e)) continue;
            uint32_t w = c->edst[e];
            if (fy >= 0) {
                if ((int64_t)w != fy) continue;
                c->g[k] = e;
                extend(c, q, depth + 1);
            } else {
                if (!vertex_ok(c, q, y, w)) continue;
                if (q->sem == 0 && image_has(c, q, w)) continue;
                c->f[y] = w;
                c->g[k] = e;
                extend(c, q, depth + 1);
                c->f[y] = -1;
            }
        }
    } else {
        const vec64 *lst = &c->in[fy];
        for (size_t i = 0; i < lst->n; i++) {
            uint64_t e = lst->a[i];
            if (!label_ok(q->qlab[k], c->elab[e])) continue;
            if (masked && in_batch(c, e)) continue;
            uint32_t w = c->esrc[e];
            if (!vertex_ok(c, q, x, w)) continue;
            if (q->sem == 0 && image_has(c, q, w)) continue;
            c->f[x] = w;
            c->g[k] = e;
            extend(c, q, depth + 1);
            c->f[x] = -1;
        }
    }
}

/* One work unit: data edge `key` placed at query position j. */
static void run_seed(orc_ctx *c, const orc_query *q, uint64_t key, uint32_t j) {
    uint32_t a = q->qsrc[j], b = q->qdst[j];
    uint32_t s = c->esrc[key], d = c->edst[key];
    if (!label_ok(q->qlab[j], c->elab[key])) return;
    if (!vertex_ok(c, q, a, s) || !vertex_ok(c, q, b, d)) return;
    if (q->sem == 0 && s == d) return;
    for (uint32_t u = 0; u < ORC_MAXQV; u++) c->f[u] = -1;
    c->f[a] = s;
    c->f[b] = d;
    c->g[j] = key;
    c->start_j = j;
    make_order(c, q, j);
    extend(c, q, 0);
}

static const orc_query *g_sort_q;
static int cmp_tuple(const void *x, const void *y) {
    const uint64_t *a = (const uint64_t *)x, *b = (const uint64_t *)y;
    for (uint32_t i = 0; i < g_sort_q->n_qe; i++) {
        if (a[i] < b[i]) return -1;
        if (a[i] > b[i]) return 1;
    }
    return 0;
}

static void sort_list(const orc_query *q, vec64 *v) {
    g_sort_q = q;
    qsort(v->a, v->n / q->n_qe, q->n_qe * sizeof(uint64_t), cmp_tuple);
}

/* Insert phase: add the edges (keys continue the arrival order), then, when
 * `enumerate` is set, list the new embeddings of every query. Returns the
 * first key of the batch, or -1 when an endpoint is out of range or a
 * timestamp decreases. */
int64_t orc_insert(void *vc, uint64_t n, const uint32_t *src, const uint32_t *dst,
                   const uint8_t *lab, const int64_t *ts, int enumerate) {
    orc_ctx *c = (orc_ctx *)vc;
    int64_t prev = c->last_ts;
    for (uint64_t i = 0; i < n; i++) {
        if (src[i] >= c->n_vertices || dst[i] >= c->n_vertices) return -1;
        if (ts[i] < prev) return -1;
        prev = ts[i];
    }
    uint64_t first = c->n_keys;
    for (uint64_t i = 0; i < n; i++)
        if (add_edge(c, src[i], dst[i], lab[i], ts[i])) return -1;
    c->ins_first = first;
    if (!enumerate) return (int64_t)first;
    c->mask_mode = 1;
    for (uint32_t qi = 0; qi < c->n_q; qi++) {
        orc_query *q = &c->q[qi];
        q->res[0].n = 0;
        q->overflow[0] = 0;
        c->sink = &q->res[0];
        c->sink_overflow = &q->overflow[0];
        for (uint64_t e = first; e < first + n; e++)
            for (uint32_t j = 0; j < q->n_qe; j++) run_seed(c, q, e, j);
        sort_list(q, &q->res[0]);
    }
    c->mask_mode = 0;
    return (int64_t)first;
}

/* Marks keys for deletion (no removal). Returns -1 for a key that is not
 * live or repeats. */
int orc_mark(void *vc, uint64_t n, const uint64_t *keys) {
    orc_ctx *c = (orc_ctx *)vc;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t k = keys[i];
        if (k >= c->n_keys || !c->live[k] || c->dmark[k]) {
            for (uint64_t t = 0; t < i; t++) c->dmark[keys[t]] = 0;
            return -1;
        }
        c->dmark[k] = 1;
    }
    return 0;
}

void orc_unmark(void *vc, uint64_t n, const uint64_t *keys) {
    orc_ctx *c = (orc_ctx *)vc;
    for (uint64_t i = 0; i < n; i++)
        if (keys[i] < c->n_keys) c->dmark[keys[i]] = 0;
}

/* Delete phase: list the expired embeddings on the current graph (which
 * still holds D), then remove D. */
int orc_delete(void *vc, uint64_t n, const uint64_t *keys, int enumerate) {
    orc_ctx *c = (orc_ctx *)vc;
    if (orc_mark(vc, n, keys)) return -1;
    if (enumerate) {
        c->mask_mode = 2;
        for (uint32_t qi = 0; qi < c->n_q; qi++) {
            orc_query *q = &c->q[qi];
            q->res[1].n = 0;
            q->overflow[1] = 0;
            c->sink = &q->res[1];
            c->sink_overflow = &q->overflow[1];
            for (uint64_t i = 0; i < n; i++)
                for (uint32_t j = 0; j < q->n_qe; j++) run_seed(c, q, keys[i], j);
            sort_list(q, &q->res[1]);
        }
        c->mask_mode = 0;
    }
    for (uint64_t i = 0; i < n; i++) {
        uint64_t k = keys[i];
        vec_remove_value(&c->out[c->esrc[k]], k);
        vec_remove_value(&c->in[c->edst[k]], k);
        c->live[k] = 0;
        c->dmark[k] = 0;
    }
    return 0;
}

/* Algorithm 1, one snapshot: insertions then deletions. */
int orc_apply_batch(void *vc, uint64_t n_ins, const uint32_t *src, const uint32_t *dst,
                    const uint8_t *lab, const int64_t *ts, uint64_t n_del,
                    const uint64_t *del_keys) {
    orc_ctx *c = (orc_ctx *)vc;
    /* validate the deletions against the post-insert key range first, so a
     * failing batch leaves the state untouched */
    uint64_t lim = c->n_keys + n_ins;
    for (uint64_t i = 0; i < n_del; i++) {
        uint64_t k = del_keys[i];
        if (k >= lim) return -1;
        if (k < c->n_keys && !c->live[k]) return -1;
        for (uint64_t t = 0; t < i; t++)
            if (del_keys[t] == k) return -1;
    }
    int64_t prev = c->last_ts;
    for (uint64_t i = 0; i < n_ins; i++) {
        if (src[i] >= c->n_vertices || dst[i] >= c->n_vertices) return -1;
        if (ts[i] < prev) return -1;
        prev = ts[i];
    }
    if (orc_insert(vc, n_ins, src, dst, lab, ts, 1) < 0) return -1;
    return orc_delete(vc, n_del, del_keys, 1);
}

uint64_t orc_count(void *vc, uint32_t qi, int phase) {
    orc_ctx *c = (orc_ctx *)vc;
    return c->q[qi].res[phase].n / c->q[qi].n_qe;
}

const uint64_t *orc_keys(void *vc, uint32_t qi, int phase) {
    return ((orc_ctx *)vc)->q[qi].res[phase].a;
}

uint64_t orc_overflow(void *vc, uint32_t qi, int phase) {
    return ((orc_ctx *)vc)->q[qi].overflow[phase];
}

static void digest_list(uint32_t qi, uint32_t n_qe, const vec64 *v, uint64_t out[2]) {
    uint64_t da = 0, db = 0;
    for (size_t t = 0; t + n_qe <= v->n; t += n_qe) {
        da += orc_tuple_hash(ORC_SEED_A, qi, v->a + t, n_qe);
        db += orc_tuple_hash(ORC_SEED_B, qi, v->a + t, n_qe);
    }
    out[0] = da;
    out[1] = db;
}

void orc_digest(void *vc, uint32_t qi, int phase, uint64_t out[2]) {
    orc_ctx *c = (orc_ctx *)vc;
    digest_list(qi, c->q[qi].n_qe, &c->q[qi].res[phase], out);
}

/* Static mode: S(G) of the current graph. Every embedding has exactly one
 * image of query edge 0, so seeding every live edge at position 0 with no
 * mask lists each embedding once. Result in the auxiliary list. */
uint64_t orc_static(void *vc, uint32_t qi) {
    orc_ctx *c = (orc_ctx *)vc;
    orc_query *q = &c->q[qi];
    c->aux.n = 0;
    c->aux_overflow = 0;
    c->sink = &c->aux;
    c->sink_overflow = &c->aux_overflow;
    c->mask_mode = 0;
    for (uint64_t e = 0; e < c->n_keys; e++)
        if (c->live[e]) run_seed(c, q, e, 0);
    sort_list(q, &c->aux);
    return c->aux.n / q->n_qe;
}

/* One work unit on its own: data edge `key` at position j, masked by
 * mode 0 (nothing), 1 (the last inserted batch) or 2 (marked deletions).
 * Result in the auxiliary list. */
uint64_t orc_seed(void *vc, uint32_t qi, uint64_t key, uint32_t j, int mode) {
    orc_ctx *c = (orc_ctx *)vc;
    orc_query *q = &c->q[qi];
    c->aux.n = 0;
    c->aux_overflow = 0;
    c->sink = &c->aux;
    c->sink_overflow = &c->aux_overflow;
    c->mask_mode = mode;
    if (key < c->n_keys && c->live[key] && j < q->n_qe) run_seed(c, q, key, j);
    c->mask_mode = 0;
    sort_list(q, &c->aux);
    return c->aux.n / q->n_qe;
}

const uint64_t *orc_aux_keys(void *vc) { return ((orc_ctx *)vc)->aux.a; }
uint64_t orc_aux_overflow(void *vc) { return ((orc_ctx *)vc)->aux_overflow; }

void orc_aux_digest(void *vc, uint32_t qi, uint64_t out[2]) {
    orc_ctx *c = (orc_ctx *)vc;
    digest_list(qi, c->q[qi].n_qe, &c->aux, out);
}

uint64_t orc_n_keys(void *vc) { return ((orc_ctx *)vc)->n_keys; }
uint64_t orc_n_live(void *vc) {
    orc_ctx *c = (orc_ctx *)vc;
    uint64_t n = 0;
    for (uint64_t k = 0; k < c->n_keys; k++) n += c->live[k];
    return n;
}
