// Stable least-significant-digit radix sort of (key, value) pairs on the
// device, with 8-bit digits: per pass, a digit histogram per tile of 4096
// elements, an exclusive scan of every digit's tile counts (a digit's tiles
// in order), and a stable scatter.  Used for the priority order of the
// Fenwick tree (Section 5, Algorithm 2) and for the level-by-level build of
// the priority-search k-d tree (Section 4.2).
#include "dpc_internal.hpp"

#include <utility>

namespace dpc {
namespace {

constexpr int kThreads = 256;
constexpr int kRsBits = 8;
constexpr int kRsBins = 1 << kRsBits;
constexpr int kRsItems = 16;                   // elements per thread
constexpr int kRsTile = kRsItems * kThreads;   // 4096 elements per tile
static_assert(kRsBins == kThreads, "one bin per thread");

// Digit counts of one tile: hist[digit * tiles + tile].
template <typename K>
__global__ __launch_bounds__(kThreads) void k_rs_hist(const K *__restrict__ key, int64_t n, int shift,
                                                      int64_t tiles, uint32_t *__restrict__ hist) {
    __shared__ uint32_t s_h[kRsBins];
    const int64_t tile = blockIdx.x;
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t e0 = tile * kRsTile;
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        const int64_t e = e0 + (int64_t)r * kThreads + threadIdx.x;
        if (e < n)
            atomicAdd(&s_h[(uint32_t)(key[e] >> shift) & (kRsBins - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * tiles + tile] = s_h[threadIdx.x];
}

// One workgroup per digit: exclusive scan of the digit's tile counts (in
// place) and the digit's total.
__global__ __launch_bounds__(kThreads) void k_rs_scan(uint32_t *__restrict__ hist, int64_t tiles,
                                                      uint32_t *__restrict__ total) {
    __shared__ uint32_t s_w[kThreads / kWave];
    uint32_t *h = hist + (int64_t)blockIdx.x * tiles;
    uint32_t carry = 0;
    const int lane = __lane_id(), w = threadIdx.x / kWave;
    for (int64_t t0 = 0; t0 < tiles; t0 += kThreads) {
        const int64_t t = t0 + threadIdx.x;
        const uint32_t v = t < tiles ? h[t] : 0u;
        uint32_t x = v;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, kWave);
            if (lane >= o)
                x += y;
        }
        if (lane == kWave - 1)
            s_w[w] = x;
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int q = 0; q < kThreads / kWave; ++q) {
            before += q < w ? s_w[q] : 0u;
            all += s_w[q];
        }
        if (t < tiles)
            h[t] = carry + before + x - v;
        carry += all;
        __syncthreads();
    }
    if (threadIdx.x == 0)
        total[blockIdx.x] = carry;
}

// Stable scatter of one tile.  The tile is taken in rounds of kThreads
// elements in order; within a round an element's rank among the equal digits
// before it comes from its wave (lanes with the same digit found by one
// ballot per digit bit) and the counts of the waves before it.
template <typename K>
__global__ __launch_bounds__(kThreads) void k_rs_scatter(const K *__restrict__ kin,
                                                         const uint32_t *__restrict__ vin, int64_t n, int shift,
                                                         int64_t tiles, const uint32_t *__restrict__ hist,
                                                         const uint32_t *__restrict__ total,
                                                         K *__restrict__ kout, uint32_t *__restrict__ vout) {
    constexpr int kW = kThreads / kWave;
    __shared__ uint32_t s_off[kRsBins];     // next output slot of each digit
    __shared__ uint32_t s_cnt[kW][kRsBins];  // this round's count of each digit per wave
    __shared__ uint32_t s_w[kW];
    const int64_t tile = blockIdx.x;
    const int lane = __lane_id(), w = threadIdx.x / kWave;
    // digit bases: exclusive scan of the totals
    {
        const uint32_t v = total[threadIdx.x];
        uint32_t x = v;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, kWave);
            if (lane >= o)
                x += y;
        }
        if (lane == kWave - 1)
            s_w[w] = x;
        __syncthreads();
        uint32_t before = 0;
        for (int q = 0; q < w; ++q)
            before += s_w[q];
        s_off[threadIdx.x] = before + x - v + hist[(int64_t)threadIdx.x * tiles + tile];
    }
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t e0 = tile * kRsTile;
    for (int r = 0; r < kRsItems; ++r) {
        __syncthreads();  // the previous round's counts are read before they are cleared
#pragma unroll
        for (int q = 0; q < kW; ++q)
            s_cnt[q][threadIdx.x] = 0;
        __syncthreads();
        const int64_t e = e0 + (int64_t)r * kThreads + threadIdx.x;
        const bool valid = e < n;
        const K k = valid ? kin[e] : (K)0;
        const uint32_t v = valid ? vin[e] : 0u;
        const uint32_t dg = (uint32_t)(k >> shift) & (kRsBins - 1);
        uint64_t same = __builtin_amdgcn_ballot_w64(valid);
#pragma unroll
        for (int b = 0; b < kRsBits; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t m = __builtin_amdgcn_ballot_w64(bit);
            same &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(same & below);
        if (valid && rank == 0)
            s_cnt[w][dg] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t pre = 0;
            for (int q = 0; q < w; ++q)
                pre += s_cnt[q][dg];
            const uint32_t dst = s_off[dg] + pre + rank;
            kout[dst] = k;
            vout[dst] = v;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int q = 0; q < kW; ++q)
            add += s_cnt[q][threadIdx.x];
        s_off[threadIdx.x] += add;
    }
}


}  // namespace

template <typename K>
dpc_status radix_sort_pairs(K *keys, uint32_t *vals, K *keys_alt, uint32_t *vals_alt, int64_t n, int bits,
                            Workspace &ws, K **keys_out, uint32_t **vals_out) {
    hipStream_t s = ws.stream;
    K *kin = keys, *kout = keys_alt;
    uint32_t *vin = vals, *vout = vals_alt;
    if (n > 0) {
        const int64_t tiles = (n + kRsTile - 1) / kRsTile;
        uint32_t *hist, *total;
        DPC_TRY(ws.alloc(&hist, (size_t)tiles * kRsBins));
        DPC_TRY(ws.alloc(&total, (size_t)kRsBins));
        for (int shift = 0; shift < bits; shift += kRsBits) {
            launch(k_rs_hist<K>, dim3((unsigned)tiles), dim3(kThreads), 0, s, (const K *)kin, n, shift, tiles, hist);
            launch(k_rs_scan, dim3(kRsBins), dim3(kThreads), 0, s, hist, tiles, total);
            launch(k_rs_scatter<K>, dim3((unsigned)tiles), dim3(kThreads), 0, s, (const K *)kin, (const uint32_t *)vin,
                   n, shift, tiles, (const uint32_t *)hist, (const uint32_t *)total, kout, vout);
            std::swap(kin, kout);
            std::swap(vin, vout);
        }
        DPC_HIP(hipGetLastError());
    }
    *keys_out = kin;
    *vals_out = vin;
    return DPC_OK;
}

template dpc_status radix_sort_pairs<uint32_t>(uint32_t *, uint32_t *, uint32_t *, uint32_t *, int64_t, int,
                                               Workspace &, uint32_t **, uint32_t **);
template dpc_status radix_sort_pairs<uint64_t>(uint64_t *, uint32_t *, uint64_t *, uint32_t *, int64_t, int,
                                               Workspace &, uint64_t **, uint32_t **);

}  // namespace dpc
