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
    if (lab < 0) return g.offs(dir)[x + 1] - g.offs(dir)[x];
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

// bfloat16 bits of a float, rounded to nearest, ties to even (inf and nan
// keep their top half).
__device__ inline uint16_t bf16_bits(float v) {
    const uint32_t u = __float_as_uint(v);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// ---- matrix-core evaluation (v_mfma_f32_16x16x32_bf16)
//
// One wave evaluates 64 samples, four tiles of 16. Both layers are computed
// transposed, units x samples, so that the first layer's accumulators already
// sit where the second layer's B operand needs them:
//   A (16 units x 32 k): lane i + 16 g holds unit i, k-slots 8 g .. 8 g + 7
//   B (32 k x 16 samples): lane j + 16 g holds sample j, the same k-slots
//   D (16 units x 16 samples): lane j + 16 g holds sample j, units 4 g .. 4 g + 3
// Layer 1: k-slot = input (24 used, 8 zero). Layer 2 contracts over the 64
// hidden units in two K-slices; slot t of group g in slice kc is hidden unit
// 32 kc + 16 (t / 4) + 4 g + t % 4, exactly the unit the lane holds in
// element t % 4 of layer-1 tile 2 kc + t / 4. The A fragments use the same
// slot order, so the hidden layer never leaves the registers. Every operand
// of every product is bf16: the first hidden layer is rounded for the second
// product, the second hidden layer for the output's dot product with W3;
// every sum is fp32.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int XS_STRIDE = 40;  // bf16 per sample row in LDS (32 used; 80 bytes keeps rows 16-byte aligned)

__device__ inline __bf16 as_bf16(uint16_t h) { return __builtin_bit_cast(__bf16, h); }

__device__ inline uint32_t hidden_of_slot(uint32_t kc, uint32_t g, uint32_t t) {
    return 32u * kc + 16u * (t / 4u) + 4u * g + (t % 4u);
}

// The lane's A fragments, loaded once per wave.
struct NetFrag {
    bf16x8 a1[4];     // layer 1, unit tile mt
    bf16x8 a2[4][2];  // layer 2, unit tile mt, K-slice kc
};

// Biases and output weights (fp32 widenings of the bf16 values), shared by
// the block in LDS.
struct NetVec {
    float b1[NH], b2[NH], w3[NH], b3;
};

// W(i) returns the bf16 bits of flat weight i.
template <typename WF>
__device__ inline void load_frag(NetFrag& F, WF W) {
    const uint32_t lane = __lane_id(), i = lane % 16u, g = lane / 16u;
#pragma unroll
    for (uint32_t mt = 0; mt < 4; mt++) {
#pragma unroll
        for (uint32_t t = 0; t < 8; t++) {
            const uint32_t in = 8u * g + t;
            F.a1[mt][t] = as_bf16(in < (uint32_t)NI ? W(OFF_W1 + in * NH + 16u * mt + i) : (uint16_t)0);
#pragma unroll
            for (uint32_t kc = 0; kc < 2; kc++)
                F.a2[mt][kc][t] = as_bf16(W(OFF_W2 + hidden_of_slot(kc, g, t) * NH + 16u * mt + i));
        }
    }
}

template <typename WF>
__device__ inline void load_vec(NetVec& V, WF W) {
    for (int u = threadIdx.x; u < NH; u += blockDim.x) {
        V.b1[u] = bf(W(OFF_B1 + u));
        V.b2[u] = bf(W(OFF_B2 + u));
        V.w3[u] = bf(W(OFF_W3 + u));
    }
    if (threadIdx.x == 0) V.b3 = bf(W(OFF_B3));
}

// Prediction for the lane's sample x (24 features; rounded to bf16 here).
// xs is the wave's LDS staging area (64 x XS_STRIDE bf16). Every lane of the
// wave must call this, and the wave's LDS traffic is ordered by the caller's
// barriers: the call waits on the block at entry and at exit, so the whole
// block must call it together.
__device__ inline float eval_wave(const NetFrag& F, const NetVec& V, const float* x, uint16_t* xs) {
    const uint32_t lane = __lane_id(), i = lane % 16u, g = lane / 16u;
    uint32_t* row = reinterpret_cast<uint32_t*>(xs + lane * XS_STRIDE);
#pragma unroll
    for (int p = 0; p < NI / 2; p++) row[p] = (uint32_t)bf16_bits(x[2 * p]) | ((uint32_t)bf16_bits(x[2 * p + 1]) << 16);
#pragma unroll
    for (int p = NI / 2; p < 16; p++) row[p] = 0u;
    __syncthreads();
    float mine = 0.0f;
#pragma unroll
    for (uint32_t nt = 0; nt < 4; nt++) {
        const bf16x8 xb = *reinterpret_cast<const bf16x8*>(xs + (16u * nt + i) * XS_STRIDE + 8u * g);
        f32x4 h[4];
#pragma unroll
        for (uint32_t mt = 0; mt < 4; mt++) {
            const f32x4 c = {V.b1[16 * mt + 4 * g], V.b1[16 * mt + 4 * g + 1], V.b1[16 * mt + 4 * g + 2],
                             V.b1[16 * mt + 4 * g + 3]};
            h[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a1[mt], xb, c, 0, 0, 0);
        }
        bf16x8 hb[2];
#pragma unroll
        for (uint32_t kc = 0; kc < 2; kc++)
#pragma unroll
            for (uint32_t t = 0; t < 8; t++) hb[kc][t] = as_bf16(bf16_bits(fmaxf(h[2 * kc + t / 4][t % 4], 0.0f)));
        float part = 0.0f;
#pragma unroll
        for (uint32_t mt = 0; mt < 4; mt++) {
            f32x4 z = {V.b2[16 * mt + 4 * g], V.b2[16 * mt + 4 * g + 1], V.b2[16 * mt + 4 * g + 2],
                       V.b2[16 * mt + 4 * g + 3]};
            z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a2[mt][0], hb[0], z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a2[mt][1], hb[1], z, 0, 0, 0);
#pragma unroll
            for (uint32_t r = 0; r < 4; r++)  // the second hidden layer enters its product as bf16 too
                part = fmaf(bf(bf16_bits(fmaxf(z[r], 0.0f))), V.w3[16 * mt + 4 * g + r], part);
        }
        part += __shfl_xor(part, 16, MN_WAVE);
        part += __shfl_xor(part, 32, MN_WAVE);
        if (nt == g) mine = part + V.b3;  // lane 16 g + j holds sample 16 g + j: its own
    }
    __syncthreads();
    return mine;
}

}  // namespace sched
