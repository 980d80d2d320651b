// Spatial index set-up: coordinate bounds (the one host read-back), the
// choice of exact arithmetic, the tree shape, and after the density step the
// priority keys and per-node maximum keys.  The k-d tree itself is built in
// kdtree.hip.
#include "dpc_internal.hpp"

#include <limits>

namespace dpc {
namespace {

constexpr int kThreads = 256;

// ---------------------------------------------------------------------------
// bounds

__global__ void k_bounds_init(int32_t *mm) {
    const int t = threadIdx.x;
    if (t < kMaxDim) {
        mm[t] = std::numeric_limits<int32_t>::max();
        mm[kMaxDim + t] = std::numeric_limits<int32_t>::min();
    }
}

__device__ inline int32_t wave_min(int32_t v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1)
        v = min(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ inline int32_t wave_max(int32_t v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1)
        v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

template <int D>
__global__ __launch_bounds__(kThreads) void k_bounds(const int32_t *__restrict__ P, int64_t n, int32_t *mm) {
    int32_t lmin[D], lmax[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lmin[k] = std::numeric_limits<int32_t>::max();
        lmax[k] = std::numeric_limits<int32_t>::min();
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int32_t v = P[i * D + k];
            lmin[k] = min(lmin[k], v);
            lmax[k] = max(lmax[k], v);
        }
    }
    __shared__ int32_t s_min[kThreads / kWave][D], s_max[kThreads / kWave][D];
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int32_t a = wave_min(lmin[k]), b = wave_max(lmax[k]);
        if (__lane_id() == 0) {
            s_min[w][k] = a;
            s_max[w][k] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x < D) {
        const int k = threadIdx.x;
        int32_t a = s_min[0][k], b = s_max[0][k];
        for (int j = 1; j < kThreads / kWave; ++j) {
            a = min(a, s_min[j][k]);
            b = max(b, s_max[j][k]);
        }
        atomicMin(&mm[k], a);
        atomicMax(&mm[kMaxDim + k], b);
    }
}

// ---------------------------------------------------------------------------
// priority keys: the high word is rho with its sign bit flipped (so unsigned
// order is signed order), the low word 2^32 - 1 - original index.  A larger
// key means higher density, or equal density and a lower index: the priority
// (rho, -index).  No real key is 0, which marks padding.

__device__ inline uint64_t pack_key(int32_t rho, int32_t orig) {
    return ((uint64_t)((uint32_t)rho ^ 0x80000000u) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)orig);
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int o) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = __shfl_xor(lo, o, kWave);
    hi = __shfl_xor(hi, o, kWave);
    return ((uint64_t)hi << 32) | lo;
}

// Keys of the sorted positions plus the leaf maxima.  rho comes either in
// sorted order (srho) or in input order (rho_orig, gathered through sidx).
__global__ __launch_bounds__(kThreads) void k_keys_leaf(const int32_t *__restrict__ srho,
                                                        const int32_t *__restrict__ rho_orig,
                                                        const int32_t *__restrict__ sidx, int64_t n,
                                                        int64_t n_leaves, uint64_t *__restrict__ skey,
                                                        uint64_t *__restrict__ maxkey) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_leaves * kLeafSize)
        return;
    uint64_t key = 0;
    if (i < n) {
        const int32_t o = sidx[i];
        const int32_t r = srho ? srho[i] : rho_orig[o];
        key = pack_key(r, o);
        skey[i] = key;
    }
#pragma unroll
    for (int o = kLeafSize / 2; o > 0; o >>= 1) {
        const uint64_t b = shfl_xor_u64(key, o);
        key = b > key ? b : key;
    }
    if ((i & (kLeafSize - 1)) == 0)
        maxkey[n_leaves + i / kLeafSize] = key;
}

// Up to 8 levels of maxima above 256 consecutive nodes of one depth.
__global__ __launch_bounds__(kThreads) void k_key_up(uint64_t *__restrict__ maxkey, int depth_in, int levels) {
    __shared__ uint64_t s[kThreads];
    const int64_t level_base = 1ll << depth_in;
    const int width = level_base < kThreads ? (int)level_base : kThreads;
    const int t = threadIdx.x;
    const int64_t first = level_base + (int64_t)blockIdx.x * kThreads;
    if (t < width)
        s[t] = maxkey[first + t];
    __syncthreads();
    for (int l = 1; l <= levels; ++l) {
        const int cnt = width >> l;
        uint64_t m = 0;
        if (t < cnt)
            m = s[2 * t] > s[2 * t + 1] ? s[2 * t] : s[2 * t + 1];
        __syncthreads();
        if (t < cnt) {
            s[t] = m;
            maxkey[(level_base >> l) + (int64_t)blockIdx.x * (kThreads >> l) + t] = m;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// host side

}  // namespace

dpc_status build_index(const int32_t *points, int64_t n, int d, int64_t T, Workspace &ws, Index &ix) {
    (void)T;
    hipStream_t s = ws.stream;
    ix.n = n;
    ix.d = d;
    // 1. bounds, read back to the host (the one synchronisation point)
    int32_t *mm;
    DPC_TRY(ws.alloc(&mm, 2 * kMaxDim));
    hipLaunchKernelGGL(k_bounds_init, dim3(1), dim3(kWave), 0, s, mm);
    const unsigned grid = blocks_for(n, kThreads) < 1024u ? blocks_for(n, kThreads) : 1024u;
    switch (d) {
#define DPC_BOUNDS_CASE(DD)                                                                  \
    case DD:                                                                                 \
        hipLaunchKernelGGL((k_bounds<DD>), dim3(grid), dim3(kThreads), 0, s, points, n, mm); \
        break;
        DPC_BOUNDS_CASE(1)
        DPC_BOUNDS_CASE(2)
        DPC_BOUNDS_CASE(3)
        DPC_BOUNDS_CASE(4)
        DPC_BOUNDS_CASE(5)
        DPC_BOUNDS_CASE(6)
        DPC_BOUNDS_CASE(7)
        DPC_BOUNDS_CASE(8)
#undef DPC_BOUNDS_CASE
    default:
        return DPC_ERR_INVALID_ARG;
    }
    DPC_HIP(hipGetLastError());
    int32_t host_mm[2 * kMaxDim];
    DPC_HIP(hipMemcpyAsync(host_mm, mm, sizeof(host_mm), hipMemcpyDeviceToHost, s));
    DPC_HIP(hipStreamSynchronize(s));
    unsigned __int128 sum = 0;
    for (int k = 0; k < d; ++k) {
        ix.lo[k] = host_mm[k];
        ix.hi[k] = host_mm[kMaxDim + k];
        const unsigned __int128 w = (unsigned __int128)((int64_t)ix.hi[k] - (int64_t)ix.lo[k]);
        sum += w * w;
    }
    // 2. every squared distance must fit in int64; below 2^53 doubles are exact
    if (sum > (unsigned __int128)std::numeric_limits<int64_t>::max())
        return DPC_ERR_RANGE;
    ix.arith = sum < ((unsigned __int128)1 << 53) ? Arith::F64 : Arith::I64;
    // 3. tree shape
    const int64_t leaves = (n + kLeafSize - 1) / kLeafSize;
    int h = 0;
    while ((1ll << h) < leaves)
        ++h;
    ix.height = h;
    ix.n_leaves = 1ll << h;
    return build_kdtree(points, ws, ix);
}

dpc_status build_priority(const int32_t *srho, const int32_t *rho_orig, Workspace &ws, Index &ix) {
    hipStream_t s = ws.stream;
    DPC_TRY(ws.alloc(&ix.skey, ix.n));
    DPC_TRY(ws.alloc(&ix.maxkey, 2 * ix.n_leaves));
    hipLaunchKernelGGL(k_keys_leaf, dim3(blocks_for(ix.n_leaves * kLeafSize, kThreads)), dim3(kThreads), 0, s, srho,
                       rho_orig, ix.sidx, ix.n, ix.n_leaves, ix.skey, ix.maxkey);
    for (int depth = ix.height; depth > 0;) {
        const int lv = depth < 8 ? depth : 8;
        const int64_t nodes = 1ll << depth;
        const unsigned grid = nodes < kThreads ? 1u : (unsigned)(nodes / kThreads);
        hipLaunchKernelGGL(k_key_up, dim3(grid), dim3(kThreads), 0, s, ix.maxkey, depth, lv);
        depth -= lv;
    }
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

}  // namespace dpc
