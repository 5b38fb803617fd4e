// Device-wide exclusive scan and stable LSD radix sort for gfx950.
//
// Both work on 256-thread blocks (four 64-lane waves). The radix sort's
// scatter ranks keys stably inside a tile with wave ballots: eight ballots on
// the digit bits give each lane the mask of lanes holding the same digit, and
// per-wave digit counts in LDS order the four waves of a round.
#include <algorithm>
#include <utility>

#include "mn_internal.h"

namespace {

constexpr uint32_t SC_ITEMS = 8;
constexpr uint32_t SC_TILE = MN_BLOCK * SC_ITEMS;  // 2048
static_assert(SC_TILE == MN_SCAN_TILE, "scan tile");
// A radix tile is 256 x ROUNDS keys. Small inputs take short tiles so that a
// pass still spreads over many blocks (a tile's rounds run one after another).
constexpr uint32_t RS_ROUNDS_MAX = 16;
constexpr uint32_t RS_TILE_MAX = MN_BLOCK * RS_ROUNDS_MAX;  // 4096
constexpr uint32_t RS_TILE_MIN = MN_BLOCK * 4;             // 1024
constexpr uint32_t RS_WAVES = MN_BLOCK / MN_WAVE;
constexpr uint32_t RS_FUSE_BLOCKS = 128;  // inputs up to 128 tiles scan their histograms in the scatter

__device__ inline uint32_t wave_incl_scan(uint32_t x) {
    uint32_t lane = __lane_id();
#pragma unroll
    for (int d = 1; d < MN_WAVE; d <<= 1) {
        uint32_t y = __shfl_up(x, d, MN_WAVE);
        if (lane >= (uint32_t)d) x += y;
    }
    return x;
}

// in and out may be the same array (the block sums are scanned in place).
__global__ __launch_bounds__(MN_BLOCK) void k_scan_local(const uint32_t* in, uint32_t* out,
                                                         uint32_t* __restrict__ sums, uint32_t n) {
    __shared__ uint32_t wsum[RS_WAVES];
    uint32_t tid = threadIdx.x;
    size_t base = (size_t)blockIdx.x * SC_TILE + (size_t)tid * SC_ITEMS;
    uint32_t v[SC_ITEMS];
    uint32_t tsum = 0;
#pragma unroll
    for (uint32_t i = 0; i < SC_ITEMS; i++) {
        size_t idx = base + i;
        v[i] = idx < n ? in[idx] : 0u;
        tsum += v[i];
    }
    uint32_t incl = wave_incl_scan(tsum);
    uint32_t wave = tid / MN_WAVE;
    if (__lane_id() == MN_WAVE - 1) wsum[wave] = incl;
    __syncthreads();
    uint32_t wpre = 0;
    for (uint32_t w = 0; w < wave; w++) wpre += wsum[w];
    uint32_t run = wpre + incl - tsum;
#pragma unroll
    for (uint32_t i = 0; i < SC_ITEMS; i++) {
        size_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    if (tid == MN_BLOCK - 1) sums[blockIdx.x] = wpre + incl;
}

__global__ __launch_bounds__(MN_BLOCK) void k_scan_add(uint32_t* __restrict__ out,
                                                       const uint32_t* __restrict__ sums, uint32_t n) {
    uint32_t add = sums[blockIdx.x];
    size_t base = (size_t)blockIdx.x * SC_TILE;
    for (uint32_t i = threadIdx.x; i < SC_TILE; i += MN_BLOCK) {
        size_t idx = base + i;
        if (idx < n) out[idx] += add;
    }
}

template <uint32_t ROUNDS>
__global__ __launch_bounds__(MN_BLOCK) void k_rs_hist(const uint64_t* __restrict__ keys, uint32_t n,
                                                      uint32_t shift, uint32_t* __restrict__ hist,
                                                      uint32_t nblk) {
    __shared__ uint32_t h[256];
    uint32_t tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    size_t base = (size_t)blockIdx.x * (MN_BLOCK * ROUNDS);
    uint64_t k[ROUNDS];
#pragma unroll
    for (uint32_t r = 0; r < ROUNDS; r++) {
        const size_t idx = base + (size_t)r * MN_BLOCK + tid;
        k[r] = idx < n ? keys[idx] : 0ull;
    }
#pragma unroll
    for (uint32_t r = 0; r < ROUNDS; r++)
        if (base + (size_t)r * MN_BLOCK + tid < n) atomicAdd(&h[(uint32_t)(k[r] >> shift) & 255u], 1u);
    __syncthreads();
    hist[(size_t)tid * nblk + blockIdx.x] = h[tid];
}

// Stable scatter of one tile by digit, starting at base_off[digit] (LDS).
template <uint32_t ROUNDS>
__device__ void rs_scatter_tile(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, uint32_t n,
                                uint32_t shift, uint32_t* base_off, uint32_t (*wcnt)[256]) {
    uint32_t tid = threadIdx.x;
    uint32_t wave = tid / MN_WAVE;
    for (uint32_t w = 0; w < RS_WAVES; w++) wcnt[w][tid] = 0;
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    size_t base = (size_t)blockIdx.x * (MN_BLOCK * ROUNDS);
    // every round's keys and values are requested before the first round
    // waits on them
    uint64_t keys[ROUNDS];
    uint32_t vals[ROUNDS];
#pragma unroll
    for (uint32_t r = 0; r < ROUNDS; r++) {
        const size_t idx = base + (size_t)r * MN_BLOCK + tid;
        keys[r] = idx < n ? kin[idx] : 0ull;
        vals[r] = idx < n ? vin[idx] : 0u;
    }
#pragma unroll
    for (uint32_t r = 0; r < ROUNDS; r++) {
        size_t idx = base + (size_t)r * MN_BLOCK + tid;
        bool valid = idx < n;
        uint64_t key = keys[r];
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (uint32_t b = 0; b < 8; b++) {
            uint32_t bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        if (!valid) peers = 0;
        bool leader = valid && (peers & lt) == 0;
        if (leader) wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t rank = base_off[d] + (uint32_t)__popcll(peers & lt);
            for (uint32_t w = 0; w < wave; w++) rank += wcnt[w][d];
            if (rank < n) {  // always true for a consistent histogram
                kout[rank] = key;
                vout[rank] = vals[r];
            }
        }
        __syncthreads();
        uint32_t tot = 0;
        for (uint32_t w = 0; w < RS_WAVES; w++) {
            tot += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        base_off[tid] += tot;
        __syncthreads();
    }
}

template <uint32_t ROUNDS>
__global__ __launch_bounds__(MN_BLOCK) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                         const uint32_t* __restrict__ vin,
                                                         uint64_t* __restrict__ kout,
                                                         uint32_t* __restrict__ vout, uint32_t n,
                                                         uint32_t shift,
                                                         const uint32_t* __restrict__ hist,
                                                         uint32_t nblk) {
    __shared__ uint32_t base_off[256];
    __shared__ uint32_t wcnt[RS_WAVES][256];
    base_off[threadIdx.x] = hist[(size_t)threadIdx.x * nblk + blockIdx.x];
    rs_scatter_tile<ROUNDS>(kin, vin, kout, vout, n, shift, base_off, wcnt);
}

// Scatter for small inputs (nblk <= RS_FUSE_BLOCKS): each block derives its
// digit offsets from the unscanned per-block histograms itself (column sums
// scanned over digits, plus the counts of earlier blocks), saving the
// device-wide scan launches.
template <uint32_t ROUNDS>
__global__ __launch_bounds__(MN_BLOCK) void k_rs_scatter_fused(const uint64_t* __restrict__ kin,
                                                               const uint32_t* __restrict__ vin,
                                                               uint64_t* __restrict__ kout,
                                                               uint32_t* __restrict__ vout, uint32_t n,
                                                               uint32_t shift,
                                                               const uint32_t* __restrict__ hist,
                                                               uint32_t nblk) {
    __shared__ uint32_t base_off[256];
    __shared__ uint32_t wcnt[RS_WAVES][256];
    __shared__ uint32_t wsum[RS_WAVES];
    const uint32_t d = threadIdx.x;
    uint32_t col = 0, before = 0;
    const uint32_t* row = hist + (size_t)d * nblk;
    uint32_t b = 0;
    if ((nblk & 3u) == 0) {  // rows of 16-byte words: independent wide loads
        const uint4* row4 = reinterpret_cast<const uint4*>(row);
#pragma unroll 8
        for (; b < nblk; b += 4) {
            const uint4 h = row4[b >> 2];
            col += h.x + h.y + h.z + h.w;
            before += (b < blockIdx.x ? h.x : 0u) + (b + 1 < blockIdx.x ? h.y : 0u) +
                      (b + 2 < blockIdx.x ? h.z : 0u) + (b + 3 < blockIdx.x ? h.w : 0u);
        }
    }
    for (; b < nblk; b++) {
        const uint32_t h = row[b];
        col += h;
        if (b < blockIdx.x) before += h;
    }
    const uint32_t incl = wave_incl_scan(col);
    if (__lane_id() == MN_WAVE - 1) wsum[d / MN_WAVE] = incl;
    __syncthreads();
    uint32_t wpre = 0;
    for (uint32_t w = 0; w < d / MN_WAVE; w++) wpre += wsum[w];
    base_off[d] = wpre + incl - col + before;
    rs_scatter_tile<ROUNDS>(kin, vin, kout, vout, n, shift, base_off, wcnt);
}

__device__ inline uint64_t wave_incl_scan64(uint64_t x) {
    uint32_t lane = __lane_id();
#pragma unroll
    for (int d = 1; d < MN_WAVE; d <<= 1) {
        uint32_t lo = __shfl_up((uint32_t)x, d, MN_WAVE);
        uint32_t hi = __shfl_up((uint32_t)(x >> 32), d, MN_WAVE);
        if (lane >= (uint32_t)d) x += ((uint64_t)hi << 32) | lo;
    }
    return x;
}

// Block-local exclusive scan into u64 (input u32 counts or u64 block sums).
// n_dev (optional) holds the element count on the device; the grid covers n.
template <typename TI>
__global__ __launch_bounds__(MN_BLOCK) void k_scan64_local(const TI* in, uint64_t* out,
                                                           uint64_t* __restrict__ sums, uint32_t n,
                                                           const uint32_t* n_dev) {
    __shared__ uint64_t wsum[RS_WAVES];
    if (n_dev) n = min(n, *n_dev);
    uint32_t tid = threadIdx.x;
    if ((size_t)blockIdx.x * SC_TILE >= n) {  // the same for the whole block: a tile past the values
        if (tid == 0) sums[blockIdx.x] = 0;
        return;
    }
    size_t base = (size_t)blockIdx.x * SC_TILE + (size_t)tid * SC_ITEMS;
    uint64_t v[SC_ITEMS];
    uint64_t tsum = 0;
#pragma unroll
    for (uint32_t i = 0; i < SC_ITEMS; i++) {
        size_t idx = base + i;
        v[i] = idx < n ? (uint64_t)in[idx] : 0ull;
        tsum += v[i];
    }
    uint64_t incl = wave_incl_scan64(tsum);
    uint32_t wave = tid / MN_WAVE;
    if (__lane_id() == MN_WAVE - 1) wsum[wave] = incl;
    __syncthreads();
    uint64_t wpre = 0;
    for (uint32_t w = 0; w < wave; w++) wpre += wsum[w];
    uint64_t run = wpre + incl - tsum;
#pragma unroll
    for (uint32_t i = 0; i < SC_ITEMS; i++) {
        size_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    if (tid == MN_BLOCK - 1) sums[blockIdx.x] = wpre + incl;
}

__global__ __launch_bounds__(MN_BLOCK) void k_scan64_add(uint64_t* __restrict__ out,
                                                         const uint64_t* __restrict__ sums, uint32_t n,
                                                         const uint32_t* n_dev) {
    if (n_dev) n = min(n, *n_dev);
    size_t base = (size_t)blockIdx.x * SC_TILE;
    if (base >= n) return;  // past the elements present
    uint64_t add = sums[blockIdx.x];
    for (uint32_t i = threadIdx.x; i < SC_TILE; i += MN_BLOCK) {
        size_t idx = base + i;
        if (idx < n) out[idx] += add;
    }
}

// As k_scan64_add, for few blocks: each block first sums the block totals
// before it (at most SC_DIRECT_MAX of them, a few loads per thread), which
// saves scanning the totals in launches of their own.
constexpr uint32_t SC_DIRECT_MAX = MN_SCAN_DIRECT_MAX;

__global__ __launch_bounds__(MN_BLOCK) void k_scan64_add_direct(uint64_t* __restrict__ out,
                                                                const uint64_t* __restrict__ sums, uint32_t n,
                                                                const uint32_t* n_dev) {
    __shared__ uint64_t wsum[RS_WAVES];
    if (n_dev) n = min(n, *n_dev);
    const size_t base = (size_t)blockIdx.x * SC_TILE;
    if (base >= n) return;  // past the elements present: the same for the whole block
    uint64_t part = 0;
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += MN_BLOCK) part += sums[i];
    part = wave_incl_scan64(part);  // the last lane holds the wave's total
    if (__lane_id() == MN_WAVE - 1) wsum[threadIdx.x / MN_WAVE] = part;
    __syncthreads();
    uint64_t add = 0;
    for (uint32_t w = 0; w < RS_WAVES; w++) add += wsum[w];
    for (uint32_t i = threadIdx.x; i < SC_TILE; i += MN_BLOCK) {
        const size_t idx = base + i;
        if (idx < n) out[idx] += add;
    }
}

__global__ void k_scan64_total(const uint32_t* __restrict__ in, const uint64_t* __restrict__ out,
                               uint32_t n, const uint32_t* n_dev, uint64_t* total) {
    if (n_dev) n = min(n, *n_dev);
    if (threadIdx.x == 0 && blockIdx.x == 0) *total = n ? out[n - 1] + in[n - 1] : 0ull;
}

inline uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

template <typename TI>
void scan64_rec(const TI* in, uint64_t* out, uint32_t n, const uint32_t* n_dev, uint64_t* scratch,
                hipStream_t s) {
    uint32_t nb = ceil_div(n, SC_TILE);
    uint64_t* sums = scratch;
    k_scan64_local<TI><<<nb, MN_BLOCK, 0, s>>>(in, out, sums, n, n_dev);
    if (nb == 1) return;
    if (nb <= SC_DIRECT_MAX) {
        k_scan64_add_direct<<<nb, MN_BLOCK, 0, s>>>(out, sums, n, n_dev);
        return;
    }
    scan64_rec<uint64_t>(sums, sums, nb, nullptr, scratch + nb + 1, s);
    k_scan64_add<<<nb, MN_BLOCK, 0, s>>>(out, sums, n, n_dev);
}

}  // namespace

uint32_t mn_scan64_local(const uint32_t* in, uint64_t* out, uint32_t n, uint64_t* sums, hipStream_t s,
                         const uint32_t* n_dev) {
    const uint32_t nb = ceil_div(n, SC_TILE);
    if (nb) k_scan64_local<uint32_t><<<nb, MN_BLOCK, 0, s>>>(in, out, sums, n, n_dev);
    return nb;
}

size_t mn_scan64_scratch_words(uint32_t n) {
    size_t words = 4;
    uint64_t m = n;
    while (m > 1) {
        m = (m + SC_TILE - 1) / SC_TILE;
        words += m + 1;
    }
    return words;
}

void mn_scan_exclusive64(const uint32_t* in, uint64_t* out, uint32_t n, uint64_t* scratch,
                         uint64_t* total, hipStream_t s, const uint32_t* n_dev) {
    if (n) scan64_rec<uint32_t>(in, out, n, n_dev, scratch, s);
    if (total) k_scan64_total<<<1, 64, 0, s>>>(in, out, n, n_dev, total);
}

size_t mn_scan_scratch_words(uint32_t n) {
    size_t words = 4;
    uint64_t m = n;
    while (m > 1) {
        m = (m + SC_TILE - 1) / SC_TILE;
        words += m + 1;
    }
    return words;
}

void mn_scan_exclusive(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* scratch,
                       hipStream_t s) {
    if (n == 0) return;
    uint32_t nb = ceil_div(n, SC_TILE);
    uint32_t* sums = scratch;
    k_scan_local<<<nb, MN_BLOCK, 0, s>>>(in, out, sums, n);
    if (nb == 1) return;
    mn_scan_exclusive(sums, sums, nb, scratch + nb + 1, s);
    k_scan_add<<<nb, MN_BLOCK, 0, s>>>(out, sums, n);
}

namespace {

// Rounds per tile for n keys: the shortest tile that keeps the histogram scan
// inside the scatter, else the longest.
uint32_t rs_rounds(uint32_t n) {
    for (uint32_t r = RS_TILE_MIN / MN_BLOCK; r < RS_ROUNDS_MAX; r *= 2)
        if (ceil_div(n, MN_BLOCK * r) <= RS_FUSE_BLOCKS) return r;
    return RS_ROUNDS_MAX;
}

template <uint32_t ROUNDS>
void rs_passes(uint64_t*& keys, uint32_t*& vals, uint64_t*& ktmp, uint32_t*& vtmp, uint32_t n, uint32_t nbits,
               uint32_t* scratch, hipStream_t s) {
    const uint32_t nblk = ceil_div(n, MN_BLOCK * ROUNDS);
    uint32_t* hist = scratch;
    uint32_t* sscr = scratch + (size_t)256 * nblk;
    for (uint32_t shift = 0; shift < nbits; shift += 8) {
        k_rs_hist<ROUNDS><<<nblk, MN_BLOCK, 0, s>>>(keys, n, shift, hist, nblk);
        if (nblk <= RS_FUSE_BLOCKS) {
            k_rs_scatter_fused<ROUNDS><<<nblk, MN_BLOCK, 0, s>>>(keys, vals, ktmp, vtmp, n, shift, hist, nblk);
        } else {
            mn_scan_exclusive(hist, hist, 256 * nblk, sscr, s);
            k_rs_scatter<ROUNDS><<<nblk, MN_BLOCK, 0, s>>>(keys, vals, ktmp, vtmp, n, shift, hist, nblk);
        }
        std::swap(keys, ktmp);
        std::swap(vals, vtmp);
    }
}

}  // namespace

size_t mn_sort_scratch_words(uint32_t n) {
    // a smaller input may take shorter tiles, hence more of them: size for
    // the most tiles any input up to n can use
    const uint32_t m = n ? n : 1;
    const uint32_t nblk = std::max(std::min(ceil_div(m, RS_TILE_MIN), RS_FUSE_BLOCKS), ceil_div(m, RS_TILE_MAX));
    size_t hist = (size_t)256 * nblk;
    return hist + mn_scan_scratch_words((uint32_t)hist);
}

void mn_radix_sort(uint64_t*& keys, uint32_t*& vals, uint64_t*& ktmp, uint32_t*& vtmp, uint32_t n,
                   uint32_t nbits, uint32_t* scratch, hipStream_t s) {
    if (n <= 1 || nbits == 0) return;
    switch (rs_rounds(n)) {
        case 4: rs_passes<4>(keys, vals, ktmp, vtmp, n, nbits, scratch, s); break;
        case 8: rs_passes<8>(keys, vals, ktmp, vtmp, n, nbits, scratch, s); break;
        default: rs_passes<16>(keys, vals, ktmp, vtmp, n, nbits, scratch, s); break;
    }
}

// ------------------------------------------------------ tuple canonical order
// Lexicographic order of result tuples (rows of m u64 keys): an index
// permutation sorted column by column from the last (LSD, each pass a stable
// radix sort of (key, index) pairs), then the rows gathered in that order.
namespace {

__global__ __launch_bounds__(MN_BLOCK) void k_iota(uint32_t* __restrict__ v, uint32_t n) {
    const uint32_t i = blockIdx.x * MN_BLOCK + threadIdx.x;
    if (i < n) v[i] = i;
}

__global__ __launch_bounds__(MN_BLOCK) void k_gather_col(const uint64_t* __restrict__ rows, uint32_t m, uint32_t col,
                                                         const uint32_t* __restrict__ idx, uint32_t n,
                                                         uint64_t* __restrict__ out) {
    const uint32_t i = blockIdx.x * MN_BLOCK + threadIdx.x;
    if (i < n) out[i] = rows[(size_t)idx[i] * m + col];
}

__global__ __launch_bounds__(MN_BLOCK) void k_permute_rows(const uint64_t* __restrict__ src, uint32_t m,
                                                           const uint32_t* __restrict__ idx, uint32_t n,
                                                           uint64_t* __restrict__ dst) {
    const uint64_t t = (uint64_t)blockIdx.x * MN_BLOCK + threadIdx.x;  // one key per thread
    if (t >= (uint64_t)n * m) return;
    const uint64_t r = t / m, k = t % m;
    dst[t] = src[(size_t)idx[r] * m + k];
}

}  // namespace

size_t mn_tuple_sort_scratch_words(uint32_t n) { return mn_sort_scratch_words(n); }

void mn_sort_tuples(uint64_t* rows, uint32_t n, uint32_t m, uint32_t key_bits, uint64_t* k0, uint64_t* k1,
                    uint32_t* v0, uint32_t* v1, uint64_t* tmp_rows, uint32_t* scratch, hipStream_t s) {
    if (n <= 1 || m == 0) return;
    const uint32_t nb = (n + MN_BLOCK - 1) / MN_BLOCK;
    k_iota<<<nb, MN_BLOCK, 0, s>>>(v0, n);
    uint64_t *ka = k0, *kb = k1;
    uint32_t *va = v0, *vb = v1;
    for (uint32_t c = m; c-- > 0;) {
        k_gather_col<<<nb, MN_BLOCK, 0, s>>>(rows, m, c, va, n, ka);
        mn_radix_sort(ka, va, kb, vb, n, key_bits, scratch, s);
    }
    const uint64_t tot = (uint64_t)n * m;
    k_permute_rows<<<(uint32_t)((tot + MN_BLOCK - 1) / MN_BLOCK), MN_BLOCK, 0, s>>>(rows, m, va, n, tmp_rows);
    (void)hipMemcpyAsync(rows, tmp_rows, tot * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
}
