// Device side of the learned scheduler: the features of a start row under one
// matching order, and the order-cost network evaluated in bf16.
//
// Every order of a (query, start position) pair finds the same embeddings
// (the order only decides which query vertex each level binds), so the choice
// changes the work, never the result. The network predicts log2 of the work
// below a start row (1 + the candidates examined at every level) under one
// order; the decision kernel takes the order with the smallest prediction.
#pragma once

#include "mn_common.h"

namespace sched {

constexpr int NI = MN_MLP_IN, NH = MN_MLP_HIDDEN;
constexpr int OFF_W1 = 0, OFF_B1 = NI * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH;
static_assert(OFF_B3 + 1 == MN_MLP_WEIGHTS, "weight layout");

__device__ inline float log2p1(uint32_t v) { return __log2f(1.0f + (float)v); }

// Edges of vertex x in direction dir carrying edge label lab (any label when
// lab < 0), from the per-vertex counters: one load, no search. For a level
// this is its candidate run before the restriction to the vertex classes
// that can carry the new vertex's labels.
__device__ inline uint32_t label_degree(const GraphView& g, uint32_t x, uint32_t dir, int32_t lab) {
    if (lab < 0) return g.off[dir][x + 1] - g.off[dir][x];
    const int16_t e = g.elab_idx[lab];
    if (e < 0) return 0;
    return g.cnt[(size_t)x * g.n_cnt + cnt_index(dir, 1 + (uint32_t)e, g.n_elab_c, g.n_vlab_c)];
}

// Candidates per row of level l of plan V when its anchor is one of the
// start edge's endpoints (f(qa) = s, f(qb) = d); false when the anchor is
// mapped later, so that only the plan's estimate is known at the start row.
__device__ inline bool level_run(const GraphView& g, const SeedPlan& V, uint32_t l, uint32_t s, uint32_t d,
                                 uint32_t& n) {
    n = 0;
    if (l >= V.n_levels) return true;
    const LevelDesc& lv = V.lv[l];
    if (lv.from != V.qa && lv.from != V.qb) return false;
    if (lv.empty) return true;
    const int32_t lab = lv.whole ? -1 : (int32_t)(lv.key_lo >> g.nbr_bits);
    n = label_degree(g, lv.from == V.qa ? s : d, lv.dir, lab);
    return true;
}

// The 24 features of start edge s -> d (label lab) under plan V, all from
// offsets, per-vertex counters and the plan (no adjacency searches):
//   0-3   log2(1 + degree): out and in of s, out and in of d
//   4     log2(1 + candidates of level 0) (its anchor is always s or d)
//   5, 6  the same for level 1 when its anchor is s or d (and 1), else the
//         plan's estimate from mean label degrees (and 0)
//   7, 8  the same for level 2
//   9-11  closing edges checked at levels 0, 1, 2
//   12    levels / 8      13  1 under isomorphism      14  query edges / 8
//   15    the estimates of levels 3 and deeper, summed
//   16    log2(1 + in-edges of d with the start edge's label)
//   17    1 when level 0 grows from s
//   18-23 start position one-hot (positions past 5 share the last)
__device__ inline void features(const GraphView& g, const SeedPlan& V, uint32_t s, uint32_t d, uint32_t lab,
                                float* x) {
    x[0] = log2p1(g.off[0][s + 1] - g.off[0][s]);
    x[1] = log2p1(g.off[1][s + 1] - g.off[1][s]);
    x[2] = log2p1(g.off[0][d + 1] - g.off[0][d]);
    x[3] = log2p1(g.off[1][d + 1] - g.off[1][d]);
    uint32_t n = 0;
    level_run(g, V, 0, s, d, n);
    x[4] = log2p1(n);
    for (uint32_t l = 1; l < 3; l++) {
        const bool exact = level_run(g, V, l, s, d, n);
        x[3 + 2 * l] = exact ? log2p1(n) : (l < V.n_levels ? V.lv_est[l] : 0.0f);
        x[4 + 2 * l] = exact ? 1.0f : 0.0f;
    }
    for (uint32_t l = 0; l < 3; l++)
        x[9 + l] = l < V.n_levels ? (float)(V.lv[l].c_end - V.lv[l].c_begin) : 0.0f;
    x[12] = (float)V.n_levels * 0.125f;
    x[13] = V.sem == MN_SEM_ISO ? 1.0f : 0.0f;
    x[14] = (float)V.n_qe * 0.125f;
    float tail = 0.0f;
    for (uint32_t l = 3; l < V.n_levels; l++) tail += V.lv_est[l];
    x[15] = tail;
    x[16] = log2p1(label_degree(g, d, 1, (int32_t)lab));
    x[17] = (V.n_levels > 0 && V.lv[0].from == V.qa) ? 1.0f : 0.0f;
    for (uint32_t k = 0; k < 6; k++) x[18 + k] = (min((uint32_t)V.j, 5u) == k) ? 1.0f : 0.0f;
}

__device__ inline float bf(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// bfloat16 rounding (nearest, ties to even) of a finite float.
__device__ inline float bf16_round(float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7F800000u) == 0x7F800000u) return v;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

// LDS image of the network: the bf16 weights, widened to fp32 once per block
// (exact: a bf16 value is an fp32 value with a zero low half), W2 transposed
// (W2t[u2][u]) so that the second layer's inner products read contiguous
// words. Widening once spares every evaluation two ALU operations per weight.
struct __align__(16) NetLds {
    float w1[NI * NH];
    float b1[NH];
    float w2t[NH * NH];
    float b2[NH];
    float w3[NH];
    float b3[4];
};

__device__ inline void load_net(NetLds& N, const uint16_t* __restrict__ w) {
    for (int i = threadIdx.x; i < NI * NH; i += blockDim.x) N.w1[i] = bf(w[OFF_W1 + i]);
    for (int i = threadIdx.x; i < NH * NH; i += blockDim.x) {  // consecutive LDS words per wave
        const int u2 = i / NH, u = i % NH;
        N.w2t[i] = bf(w[OFF_W2 + u * NH + u2]);
    }
    for (int i = threadIdx.x; i < NH; i += blockDim.x) {
        N.b1[i] = bf(w[OFF_B1 + i]);
        N.b2[i] = bf(w[OFF_B2 + i]);
        N.w3[i] = bf(w[OFF_W3 + i]);
    }
    if (threadIdx.x == 0) N.b3[0] = bf(w[OFF_B3]);
}

// One lane, one sample: inputs rounded to bf16, bf16 weights, fp32 sums. The
// hidden layer stays in registers; weights stream from LDS four at a time
// (every lane of a wave reads the same words, a broadcast).
__device__ inline float eval(const NetLds& N, const float* x) {
    float h[NH];
#pragma unroll
    for (int u = 0; u < NH; u++) h[u] = N.b1[u];
#pragma unroll 1
    for (int i = 0; i < NI; i++) {
        const float xi = bf16_round(x[i]);
        const float4* row = reinterpret_cast<const float4*>(N.w1 + i * NH);
#pragma unroll
        for (int u = 0; u < NH / 4; u++) {
            const float4 w = row[u];
            h[4 * u] = fmaf(xi, w.x, h[4 * u]);
            h[4 * u + 1] = fmaf(xi, w.y, h[4 * u + 1]);
            h[4 * u + 2] = fmaf(xi, w.z, h[4 * u + 2]);
            h[4 * u + 3] = fmaf(xi, w.w, h[4 * u + 3]);
        }
    }
#pragma unroll
    for (int u = 0; u < NH; u++) h[u] = fmaxf(h[u], 0.0f);
    float y = N.b3[0];
#pragma unroll 1
    for (int u2 = 0; u2 < NH; u2++) {
        float z = N.b2[u2];
        const float4* col = reinterpret_cast<const float4*>(N.w2t + u2 * NH);
#pragma unroll
        for (int u = 0; u < NH / 4; u++) {
            const float4 w = col[u];
            z = fmaf(h[4 * u], w.x, z);
            z = fmaf(h[4 * u + 1], w.y, z);
            z = fmaf(h[4 * u + 2], w.z, z);
            z = fmaf(h[4 * u + 3], w.w, z);
        }
        y = fmaf(fmaxf(z, 0.0f), N.w3[u2], y);
    }
    return y;
}

}  // namespace sched
