// The scheduler's network: a 24 -> 64 -> 64 -> 1 ReLU perceptron that
// predicts log2 of a work unit's search work under one matching order
// (see the seed kernel in mn_enum.hip). Training runs here, on the GPU:
// mean squared error, Adam, minibatches gathered through a permutation.
//
// Weights (5,825 fp32, this order): W1[24][64], b1[64], W2[64][64], b2[64],
// W3[64], b3. Each block handles 64 samples with every weight and activation
// in LDS; thread t works on sample t / 4 and a quarter of its units.
// Backward forms the weight gradients of the block as small products over
// its 64 samples in LDS, then adds them to the global gradient once per
// block. The sizes are tiny next to the matcher, so the training products are
// plain FMA loops. Inference in bf16 runs on the matrix cores instead, through
// the same wave-level evaluator the decision kernel uses (mn_sched.h).
#include "mn_internal.h"
#include "mn_sched.h"

namespace {

constexpr int NI = MN_MLP_IN, NH = MN_MLP_HIDDEN;
constexpr int OFF_W1 = 0, OFF_B1 = NI * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH;
static_assert(OFF_B3 + 1 == MN_MLP_WEIGHTS, "weight layout");
constexpr int SPB = 64;  // samples per block
constexpr int PAD = NH + 1;

// Round to bfloat16 (nearest, ties to even) and back.
__device__ inline float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u) return x;  // inf / nan unchanged
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

struct MlpLds {
    float w[MN_MLP_WEIGHTS];
    float x[SPB][NI];
    float h1[SPB][PAD];
    float h2[SPB][PAD];
    float d1[SPB][PAD];
    float d2[SPB][PAD];
    float dy[SPB];
};

// Forward pass of the block's samples into L.h1, L.h2; returns y of sample
// tid / 4 (valid in every lane of that sample's group of four).
__device__ float forward(MlpLds& L) {
    const int t = threadIdx.x, s = t >> 2, part = t & 3;
    for (int u = part * 16; u < part * 16 + 16; u++) {
        float z = L.w[OFF_B1 + u];
        for (int i = 0; i < NI; i++) z = fmaf(L.x[s][i], L.w[OFF_W1 + i * NH + u], z);
        L.h1[s][u] = fmaxf(z, 0.0f);
    }
    __syncthreads();
    float y = 0.0f;
    for (int u2 = part * 16; u2 < part * 16 + 16; u2++) {
        float z = L.w[OFF_B2 + u2];
        for (int u = 0; u < NH; u++) z = fmaf(L.h1[s][u], L.w[OFF_W2 + u * NH + u2], z);
        const float h = fmaxf(z, 0.0f);
        L.h2[s][u2] = h;
        y = fmaf(h, L.w[OFF_W3 + u2], y);
    }
    y += __shfl_xor(y, 1, 4);
    y += __shfl_xor(y, 2, 4);
    return y + L.w[OFF_B3];
}

// Copies the weights (optionally rounded to bf16) and the block's samples
// x[idx[base + s]] (or x[base + s]) into LDS; rows past n are zero.
__device__ void load_block(MlpLds& L, const float* __restrict__ w, const float* __restrict__ x,
                           const uint32_t* __restrict__ idx, uint64_t base, uint64_t n, bool bf16) {
    for (int i = threadIdx.x; i < MN_MLP_WEIGHTS; i += blockDim.x) L.w[i] = bf16 ? bf16_round(w[i]) : w[i];
    for (int i = threadIdx.x; i < SPB * NI; i += blockDim.x) {
        const int s = i / NI, f = i % NI;
        const uint64_t k = base + s;
        float v = 0.0f;
        if (k < n) v = x[(size_t)(idx ? idx[k] : k) * NI + f];
        L.x[s][f] = bf16 ? bf16_round(v) : v;
    }
    __syncthreads();
}

__global__ __launch_bounds__(MN_BLOCK) void k_mlp_predict(const float* __restrict__ w, const float* __restrict__ x,
                                                          uint64_t n, int bf16, float* __restrict__ y) {
    __shared__ MlpLds L;
    const uint64_t base = (uint64_t)blockIdx.x * SPB;
    load_block(L, w, x, nullptr, base, n, bf16 != 0);
    const float v = forward(L);
    const int s = threadIdx.x >> 2;
    if ((threadIdx.x & 3) == 0 && base + s < n) y[base + s] = v;
}

// bf16 inference: weights, inputs and hidden activations rounded to bf16,
// fp32 sums, one sample per lane on the matrix cores.
__global__ __launch_bounds__(MN_BLOCK) void k_mlp_predict_mm(const float* __restrict__ w, const float* __restrict__ x,
                                                             uint64_t n, float* __restrict__ y) {
    __shared__ sched::NetVec V;
    __shared__ __align__(16) uint16_t s_xs[MN_BLOCK / MN_WAVE][MN_WAVE * sched::XS_STRIDE];
    auto W = [w](uint32_t i) { return sched::bf16_bits(w[i]); };
    sched::NetFrag F;
    sched::load_frag(F, W);
    sched::load_vec(V, W);
    __syncthreads();
    const uint64_t s = (uint64_t)blockIdx.x * MN_BLOCK + threadIdx.x;
    float xv[NI];
#pragma unroll
    for (int f = 0; f < NI; f++) xv[f] = s < n ? x[s * NI + f] : 0.0f;
    const float v = sched::eval_wave(F, V, xv, s_xs[threadIdx.x / MN_WAVE]);
    if (s < n) y[s] = v;
}

// Gradient of the mean squared error over the m samples idx[off .. off + m)
// (scaled by 1 / m), added into grad; loss receives the sum of squared errors / m.
__global__ __launch_bounds__(MN_BLOCK) void k_mlp_grad(const float* __restrict__ w, const float* __restrict__ x,
                                                       const float* __restrict__ target,
                                                       const uint32_t* __restrict__ idx, uint64_t off, uint64_t m,
                                                       float* __restrict__ grad, float* __restrict__ loss) {
    __shared__ MlpLds L;
    const uint64_t base = off + (uint64_t)blockIdx.x * SPB;
    const uint64_t end = off + m;
    load_block(L, w, x, idx, base, end, false);
    const int t = threadIdx.x, s = t >> 2, part = t & 3;
    const float y = forward(L);
    const bool valid = base + s < end;
    const float tgt = valid ? target[idx ? idx[base + s] : base + s] : 0.0f;
    const float err = valid ? y - tgt : 0.0f;
    const float inv = 1.0f / (float)m;
    if (part == 0) {
        L.dy[s] = 2.0f * err * inv;
        if (valid) atomicAdd(loss, err * err * inv);
    }
    __syncthreads();
    // dH2 = dy * W3 masked by ReLU; dH1 = (dH2 W2^T) masked by ReLU
    for (int u2 = part * 16; u2 < part * 16 + 16; u2++)
        L.d2[s][u2] = L.h2[s][u2] > 0.0f ? L.dy[s] * L.w[OFF_W3 + u2] : 0.0f;
    __syncthreads();
    for (int u = part * 16; u < part * 16 + 16; u++) {
        float a = 0.0f;
        if (L.h1[s][u] > 0.0f)
            for (int u2 = 0; u2 < NH; u2++) a = fmaf(L.d2[s][u2], L.w[OFF_W2 + u * NH + u2], a);
        L.d1[s][u] = a;
    }
    __syncthreads();
    // weight gradients of this block: sums over its samples
    for (int e = t; e < NH * NH; e += blockDim.x) {  // W2[u][u2]
        const int u = e / NH, u2 = e % NH;
        float a = 0.0f;
        for (int k = 0; k < SPB; k++) a = fmaf(L.h1[k][u], L.d2[k][u2], a);
        if (a != 0.0f) atomicAdd(grad + OFF_W2 + e, a);
    }
    for (int e = t; e < NI * NH; e += blockDim.x) {  // W1[i][u]
        const int i = e / NH, u = e % NH;
        float a = 0.0f;
        for (int k = 0; k < SPB; k++) a = fmaf(L.x[k][i], L.d1[k][u], a);
        if (a != 0.0f) atomicAdd(grad + OFF_W1 + e, a);
    }
    if (t < NH) {
        float b1 = 0.0f, b2 = 0.0f, w3 = 0.0f;
        for (int k = 0; k < SPB; k++) {
            b1 += L.d1[k][t];
            b2 += L.d2[k][t];
            w3 = fmaf(L.h2[k][t], L.dy[k], w3);
        }
        atomicAdd(grad + OFF_B1 + t, b1);
        atomicAdd(grad + OFF_B2 + t, b2);
        atomicAdd(grad + OFF_W3 + t, w3);
    }
    if (t == 0) {
        float b3 = 0.0f;
        for (int k = 0; k < SPB; k++) b3 += L.dy[k];
        atomicAdd(grad + OFF_B3, b3);
    }
}

// Adam (Kingma & Ba 2015) on every weight; clears grad. The constants come
// from the host in double precision rounded once: 1 - beta formed in fp32
// from an fp32 beta would carry a relative error of ~1e-5.
__global__ __launch_bounds__(MN_BLOCK) void k_mlp_adam(float* __restrict__ w, float* __restrict__ m1,
                                                       float* __restrict__ m2, float* __restrict__ grad, float lr,
                                                       float b1, float ob1, float b2, float ob2, float eps, float c1,
                                                       float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MN_MLP_WEIGHTS) return;
    const float g = grad[i];
    const float a = b1 * m1[i] + ob1 * g;
    const float v = b2 * m2[i] + ob2 * g * g;
    m1[i] = a;
    m2[i] = v;
    w[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
    grad[i] = 0.0f;
}

__global__ void k_to_bf16(const float* __restrict__ in, uint16_t* __restrict__ out, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (uint16_t)(__float_as_uint(bf16_round(in[i])) >> 16);
}

__global__ void k_fill_f32(float* p, float v, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline uint32_t mlp_blocks(uint64_t n) { return (uint32_t)((n + SPB - 1) / SPB); }

}  // namespace

void mn_mlp_predict(const float* w, const float* x, uint64_t n, int bf16, float* y, hipStream_t s) {
    if (!n) return;
    if (bf16)
        k_mlp_predict_mm<<<(uint32_t)((n + MN_BLOCK - 1) / MN_BLOCK), MN_BLOCK, 0, s>>>(w, x, n, y);
    else
        k_mlp_predict<<<mlp_blocks(n), MN_BLOCK, 0, s>>>(w, x, n, 0, y);
}

void mn_mlp_grad(const float* w, const float* x, const float* target, const uint32_t* idx, uint64_t off,
                 uint64_t m, float* grad, float* loss, hipStream_t s) {
    if (m) k_mlp_grad<<<mlp_blocks(m), MN_BLOCK, 0, s>>>(w, x, target, idx, off, m, grad, loss);
}

void mn_mlp_adam(float* w, float* m1, float* m2, float* grad, float lr, uint32_t step, hipStream_t s) {
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    k_mlp_adam<<<(MN_MLP_WEIGHTS + MN_BLOCK - 1) / MN_BLOCK, MN_BLOCK, 0, s>>>(
        w, m1, m2, grad, lr, (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), (float)eps, (float)c1,
        (float)c2);
}

void mn_fill_f32(float* p, float v, uint32_t n, hipStream_t s) {
    if (n) k_fill_f32<<<(n + MN_BLOCK - 1) / MN_BLOCK, MN_BLOCK, 0, s>>>(p, v, n);
}

void mn_to_bf16(const float* in, uint16_t* out, uint32_t n, hipStream_t s) {
    if (n) k_to_bf16<<<(n + MN_BLOCK - 1) / MN_BLOCK, MN_BLOCK, 0, s>>>(in, out, n);
}
