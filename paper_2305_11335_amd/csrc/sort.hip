// Stable LSD radix sort of (uint64 key, uint32 value) pairs, 8 bits a pass.
//
// The spatial index is built by sorting points on their Morton codes: the
// paper's radix-sort primitive (Section 3.2, "Other parallel primitives").
//
// One pass = three kernels:
//   k_rs_hist     per-tile digit histogram (tile = 4096 keys, 16 per thread);
//                 equal digits within a wave are counted once through a
//                 ballot-based match, so LDS atomics see one update per
//                 distinct digit per wave;
//   k_rs_rowscan  one block per digit scans that digit's counts over tiles;
//   k_rs_scatter  each wave ranks its 1024 keys stably (ballot match +
//                 popcount of lower lanes), the block places the tile in LDS
//                 sorted by digit, then writes runs of equal digits to their
//                 global positions so the stores are contiguous.
#include "dpc_internal.hpp"

namespace dpc {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kItems = 16;
constexpr int kWaveItems = kItems * kWave;  // 1024 keys per wave
constexpr int kTile = kThreads * kItems;     // 4096 keys per block
constexpr int kBits = 8;
constexpr int kBins = 1 << kBits;
static_assert(kThreads == kBins, "one thread per digit");

__device__ inline uint64_t lanes_below() { return (1ull << __lane_id()) - 1ull; }

// Lanes (among `valid` ones) holding the same 8-bit digit as this lane.
__device__ inline uint64_t match_digit(uint32_t dg, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kBits; ++b) {
        const bool bit = (dg >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, kWave);
        if (lane >= o)
            v += t;
    }
    return v;
}

// Inclusive scan over a 256-thread block; s_w holds kWaves entries.
__device__ inline uint32_t block_incl_scan(uint32_t v, uint32_t *s_w) {
    const int w = threadIdx.x / kWave;
    const uint32_t x = wave_incl_scan(v);
    if ((threadIdx.x & (kWave - 1)) == kWave - 1)
        s_w[w] = x;
    __syncthreads();
    uint32_t add = 0;
    for (int j = 0; j < w; ++j)
        add += s_w[j];
    __syncthreads();
    return x + add;
}

__global__ __launch_bounds__(kThreads) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                      uint32_t *__restrict__ hist, int nblocks) {
    __shared__ uint32_t h[kBins];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int w = threadIdx.x / kWave;
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)w * kWaveItems + __lane_id();
#pragma unroll 4
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + (int64_t)r * kWave;
        const bool valid = i < n;
        const uint32_t dg = valid ? (uint32_t)(keys[i] >> shift) & (kBins - 1) : 0u;
        const uint64_t peers = match_digit(dg, valid);
        if (valid && (peers & lanes_below()) == 0)
            atomicAdd(&h[dg], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kThreads) void k_rs_rowscan(const uint32_t *__restrict__ hist,
                                                         uint32_t *__restrict__ hoff,
                                                         uint32_t *__restrict__ bin_total, int nblocks) {
    __shared__ uint32_t s_w[kWaves];
    __shared__ uint32_t s_total;
    const uint32_t *row = hist + (int64_t)blockIdx.x * nblocks;
    uint32_t *orow = hoff + (int64_t)blockIdx.x * nblocks;
    uint32_t carry = 0;  // identical in every thread
    for (int c = 0; c < nblocks; c += kThreads) {
        const int j = c + threadIdx.x;
        const uint32_t v = j < nblocks ? row[j] : 0u;
        const uint32_t incl = block_incl_scan(v, s_w);
        if (j < nblocks)
            orow[j] = carry + incl - v;
        if (threadIdx.x == kThreads - 1)
            s_total = incl;
        __syncthreads();
        carry += s_total;
        __syncthreads();
    }
    if (threadIdx.x == 0)
        bin_total[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kThreads) void k_rs_scatter(const uint64_t *__restrict__ kin,
                                                         const uint32_t *__restrict__ vin,
                                                         uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                         int64_t n, int shift, const uint32_t *__restrict__ hoff,
                                                         const uint32_t *__restrict__ bin_total, int nblocks) {
    __shared__ uint64_t s_k[kTile];
    __shared__ uint32_t s_v[kTile];
    __shared__ uint32_t s_run[kWaves][kBins];
    __shared__ uint32_t s_gbase[kBins];
    __shared__ uint32_t s_w[kWaves];

    const int tid = threadIdx.x;
    const int w = tid / kWave;
    for (int j = tid; j < kWaves * kBins; j += kThreads)
        (&s_run[0][0])[j] = 0;
    __syncthreads();

    const int64_t tile = (int64_t)blockIdx.x * kTile;
    const int64_t base = tile + (int64_t)w * kWaveItems + __lane_id();
    uint64_t kk[kItems];
    uint32_t vv[kItems];
    uint32_t lr[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + (int64_t)r * kWave;
        const bool valid = i < n;
        const uint64_t k = valid ? kin[i] : 0ull;
        const uint32_t dg = (uint32_t)(k >> shift) & (kBins - 1);
        const uint64_t peers = match_digit(dg, valid);
        const uint32_t rank = (uint32_t)__popcll(peers & lanes_below());
        const uint32_t before = s_run[w][dg];
        if (valid && rank == 0)
            s_run[w][dg] = before + (uint32_t)__popcll(peers);
        kk[r] = k;
        vv[r] = valid ? vin[i] : 0u;
        lr[r] = before + rank;
    }
    __syncthreads();

    // Per digit (one per thread): its offset within the tile and per wave.
    const int dgt = tid;
    const uint32_t c0 = s_run[0][dgt], c1 = s_run[1][dgt], c2 = s_run[2][dgt], c3 = s_run[3][dgt];
    const uint32_t tot = c0 + c1 + c2 + c3;
    const uint32_t excl = block_incl_scan(tot, s_w) - tot;
    const uint32_t bt = bin_total[dgt];
    const uint32_t bin_start = block_incl_scan(bt, s_w) - bt;
    s_run[0][dgt] = excl;
    s_run[1][dgt] = excl + c0;
    s_run[2][dgt] = excl + c0 + c1;
    s_run[3][dgt] = excl + c0 + c1 + c2;
    // output position of tile slot j holding digit g is s_gbase[g] + j
    s_gbase[dgt] = bin_start + hoff[(int64_t)dgt * nblocks + blockIdx.x] - excl;
    __syncthreads();

#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + (int64_t)r * kWave;
        if (i < n) {
            const uint32_t dg = (uint32_t)(kk[r] >> shift) & (kBins - 1);
            const uint32_t pos = s_run[w][dg] + lr[r];
            s_k[pos] = kk[r];
            s_v[pos] = vv[r];
        }
    }
    __syncthreads();

    const int64_t left = n - tile;
    const int cnt = left < kTile ? (int)left : kTile;
    for (int j = tid; j < cnt; j += kThreads) {
        const uint64_t k = s_k[j];
        const uint32_t g = s_gbase[(uint32_t)(k >> shift) & (kBins - 1)] + (uint32_t)j;
        kout[g] = k;
        vout[g] = s_v[j];
    }
}

}  // namespace

dpc_status radix_sort_pairs(uint64_t *keys, uint32_t *vals, int64_t n, int key_bits, Workspace &ws,
                            uint64_t **keys_out, uint32_t **vals_out) {
    *keys_out = keys;
    *vals_out = vals;
    const int passes = (key_bits + kBits - 1) / kBits;
    if (n <= 1 || passes == 0)
        return DPC_OK;
    const int nblocks = (int)blocks_for(n, kTile);
    uint64_t *k2;
    uint32_t *v2, *hist, *hoff, *bin_total;
    DPC_TRY(ws.alloc(&k2, n));
    DPC_TRY(ws.alloc(&v2, n));
    DPC_TRY(ws.alloc(&hist, (size_t)kBins * nblocks));
    DPC_TRY(ws.alloc(&hoff, (size_t)kBins * nblocks));
    DPC_TRY(ws.alloc(&bin_total, kBins));
    uint64_t *ka = keys, *kb = k2;
    uint32_t *va = vals, *vb = v2;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kBits;
        hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(kThreads), 0, ws.stream, ka, n, shift, hist, nblocks);
        hipLaunchKernelGGL(k_rs_rowscan, dim3(kBins), dim3(kThreads), 0, ws.stream, hist, hoff, bin_total,
                           nblocks);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(kThreads), 0, ws.stream, ka, va, kb, vb, n, shift,
                           hoff, bin_total, nblocks);
        DPC_HIP(hipGetLastError());
        uint64_t *tk = ka;
        ka = kb;
        kb = tk;
        uint32_t *tv = va;
        va = vb;
        vb = tv;
    }
    *keys_out = ka;
    *vals_out = va;
    return DPC_OK;
}

}  // namespace dpc
