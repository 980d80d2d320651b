// Spatial index: coordinate bounds, Morton keys, sort, sorted coordinates,
// and the implicit tree of boxes and maximum priority keys.
//
// The paper indexes points with k-d trees whose nodes keep their cell (tight
// bounding box) for pruning (Section 3.2) and, for the dependent search, the
// highest priority below them (the priority search k-d tree of Section 4.2).
// Here the tree is a complete binary tree over the Morton-sorted points,
// built bottom-up with no pointers: sibling nodes cover adjacent ranges of
// the sorted array, so the tree is fixed by n and the leaf size alone.
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
// Morton codes: axis k of bit level t lands on key bit t*d + k.

__device__ __host__ inline uint64_t spread2(uint64_t x) {
    x &= 0xFFFFFFFFull;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}
__device__ __host__ inline uint64_t compact2(uint64_t x) {
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    return x;
}
__device__ __host__ inline uint64_t spread3(uint64_t x) {
    x &= 0x1FFFFFull;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}
__device__ __host__ inline uint64_t compact3(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x | (x >> 2)) & 0x10C30C30C30C30C3ull;
    x = (x | (x >> 4)) & 0x100F00F00F00F00Full;
    x = (x | (x >> 8)) & 0x001F0000FF0000FFull;
    x = (x | (x >> 16)) & 0x001F00000000FFFFull;
    x = (x | (x >> 32)) & 0x1FFFFFull;
    return x;
}

struct KeyParams {
    int32_t lo[kMaxDim];
    int shift;
    int bits;  // per axis
};

template <int D>
__device__ inline uint64_t morton(const uint32_t (&c)[D], int bits) {
    if constexpr (D == 1) {
        return c[0];
    } else if constexpr (D == 2) {
        return spread2(c[0]) | (spread2(c[1]) << 1);
    } else if constexpr (D == 3) {
        return spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
    } else {
        uint64_t key = 0;
        for (int t = 0; t < bits; ++t)
#pragma unroll
            for (int k = 0; k < D; ++k)
                key |= (uint64_t)((c[k] >> t) & 1u) << (t * D + k);
        return key;
    }
}

template <int D>
__global__ __launch_bounds__(kThreads) void k_keys(const int32_t *__restrict__ P, int64_t n, KeyParams kp,
                                                   uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint32_t c[D];
#pragma unroll
    for (int k = 0; k < D; ++k)
        c[k] = (uint32_t)((int64_t)P[i * D + k] - (int64_t)kp.lo[k]) >> kp.shift;
    keys[i] = morton<D>(c, kp.bits);
    vals[i] = (uint32_t)i;
}

// Sorted coordinates straight from full-precision Morton keys (d <= 3).
template <typename C, int D>
__global__ __launch_bounds__(kThreads) void k_decode(const uint64_t *__restrict__ keys,
                                                     const uint32_t *__restrict__ vals, int64_t n, KeyParams kp,
                                                     C *__restrict__ coords, int32_t *__restrict__ sidx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint64_t key = keys[i];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        uint64_t c;
        if constexpr (D == 1)
            c = key;
        else if constexpr (D == 2)
            c = compact2(key >> k);
        else
            c = compact3(key >> k);
        coords[i * D + k] = (C)((int64_t)kp.lo[k] + (int64_t)c);
    }
    sidx[i] = (int32_t)vals[i];
}

// Sorted coordinates gathered from the input rows.
template <typename C, int D>
__global__ __launch_bounds__(kThreads) void k_gather(const int32_t *__restrict__ P, const uint32_t *__restrict__ vals,
                                                     int64_t n, C *__restrict__ coords, int32_t *__restrict__ sidx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t o = vals[i];
#pragma unroll
    for (int k = 0; k < D; ++k)
        coords[i * D + k] = (C)P[(int64_t)o * D + k];
    sidx[i] = (int32_t)o;
}

// ---------------------------------------------------------------------------
// tree boxes

template <typename C>
__device__ inline C c_max_value() { return std::numeric_limits<C>::max(); }
template <typename C>
__device__ inline C c_lowest_value() { return std::numeric_limits<C>::lowest(); }

template <typename C>
__device__ inline C shfl_xor_c(C v, int o) {
    if constexpr (sizeof(C) == 8) {
        int64_t b = __builtin_bit_cast(int64_t, v);
        int lo = (int)(b & 0xFFFFFFFF), hi = (int)(b >> 32);
        lo = __shfl_xor(lo, o, kWave);
        hi = __shfl_xor(hi, o, kWave);
        return __builtin_bit_cast(C, ((int64_t)hi << 32) | (uint32_t)lo);
    } else {
        return __shfl_xor(v, o, kWave);
    }
}

// One thread per leaf slot; groups of kLeafSize lanes reduce to the leaf box.
template <typename C, int D>
__global__ __launch_bounds__(kThreads) void k_leaf_box(const C *__restrict__ coords, int64_t n, int64_t n_leaves,
                                                       C *__restrict__ box) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_leaves * kLeafSize)
        return;
    const bool have = i < n;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        C mn = have ? coords[i * D + k] : c_max_value<C>();
        C mx = have ? coords[i * D + k] : c_lowest_value<C>();
#pragma unroll
        for (int o = kLeafSize / 2; o > 0; o >>= 1) {
            const C a = shfl_xor_c(mn, o), b = shfl_xor_c(mx, o);
            mn = a < mn ? a : mn;
            mx = b > mx ? b : mx;
        }
        if ((i & (kLeafSize - 1)) == 0) {
            const int64_t v = n_leaves + i / kLeafSize;
            box[(v * D + k) * 2 + 0] = mn;
            box[(v * D + k) * 2 + 1] = mx;
        }
    }
}

// Up to 8 levels of internal nodes above 256 consecutive nodes of one depth.
template <typename C, int D>
__global__ __launch_bounds__(kThreads) void k_box_up(C *__restrict__ box, int depth_in, int levels) {
    __shared__ C s[kThreads][2 * D];
    const int64_t level_base = 1ll << depth_in;
    const int width = level_base < kThreads ? (int)level_base : kThreads;
    const int t = threadIdx.x;
    const int64_t first = level_base + (int64_t)blockIdx.x * kThreads;
    if (t < width) {
#pragma unroll
        for (int j = 0; j < 2 * D; ++j)
            s[t][j] = box[(first + t) * 2 * D + j];
    }
    __syncthreads();
    for (int l = 1; l <= levels; ++l) {
        const int cnt = width >> l;
        C tmp[2 * D];
        if (t < cnt) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const C a0 = s[2 * t][2 * k], b0 = s[2 * t + 1][2 * k];
                const C a1 = s[2 * t][2 * k + 1], b1 = s[2 * t + 1][2 * k + 1];
                tmp[2 * k] = a0 < b0 ? a0 : b0;
                tmp[2 * k + 1] = a1 > b1 ? a1 : b1;
            }
        }
        __syncthreads();
        if (t < cnt) {
            const int64_t node = (level_base >> l) + (int64_t)blockIdx.x * (kThreads >> l) + t;
#pragma unroll
            for (int j = 0; j < 2 * D; ++j) {
                s[t][j] = tmp[j];
                box[node * 2 * D + j] = tmp[j];
            }
        }
        __syncthreads();
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

template <typename C, int D>
dpc_status build_tree_boxes(Index &ix, hipStream_t s) {
    C *coords = static_cast<C *>(ix.coords);
    C *box = static_cast<C *>(ix.box);
    hipLaunchKernelGGL((k_leaf_box<C, D>), dim3(blocks_for(ix.n_leaves * kLeafSize, kThreads)), dim3(kThreads), 0,
                       s, coords, ix.n, ix.n_leaves, box);
    for (int depth = ix.height; depth > 0;) {
        const int lv = depth < 8 ? depth : 8;
        const int64_t nodes = 1ll << depth;
        const unsigned grid = nodes < kThreads ? 1u : (unsigned)(nodes / kThreads);
        hipLaunchKernelGGL((k_box_up<C, D>), dim3(grid), dim3(kThreads), 0, s, box, depth, lv);
        depth -= lv;
    }
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

template <typename C, int D>
dpc_status build_typed(const int32_t *points, const KeyParams &kp, bool decode, uint64_t *keys, uint32_t *vals,
                       Workspace &ws, Index &ix) {
    hipStream_t s = ws.stream;
    C *coords;
    C *box;
    DPC_TRY(ws.alloc(&coords, (size_t)ix.n * D));
    DPC_TRY(ws.alloc(&box, (size_t)2 * ix.n_leaves * 2 * D));
    ix.coords = coords;
    ix.box = box;
    const unsigned grid = blocks_for(ix.n, kThreads);
    if (decode) {
        if constexpr (D <= 3)
            hipLaunchKernelGGL((k_decode<C, D>), dim3(grid), dim3(kThreads), 0, s, keys, vals, ix.n, kp, coords,
                               ix.sidx);
    } else {
        hipLaunchKernelGGL((k_gather<C, D>), dim3(grid), dim3(kThreads), 0, s, points, vals, ix.n, coords, ix.sidx);
    }
    DPC_HIP(hipGetLastError());
    return build_tree_boxes<C, D>(ix, s);
}

template <int D>
dpc_status build_dim(const int32_t *points, Workspace &ws, Index &ix) {
    hipStream_t s = ws.stream;
    // Morton parameters: as many bits per axis as fit in 64 bits, dropping
    // low bits of wide coordinates.
    uint32_t maxspan = 0;
    for (int k = 0; k < D; ++k) {
        const uint32_t sp = (uint32_t)((int64_t)ix.hi[k] - (int64_t)ix.lo[k]);
        maxspan = sp > maxspan ? sp : maxspan;
    }
    const int need = maxspan ? 32 - __builtin_clz(maxspan) : 0;
    const int cap = D == 1 ? 32 : (D == 2 ? 32 : 64 / D);
    KeyParams kp{};
    for (int k = 0; k < D; ++k)
        kp.lo[k] = ix.lo[k];
    kp.bits = need < cap ? need : cap;
    kp.shift = need - kp.bits;
    ix.bits_per_dim = kp.bits;
    ix.shift = kp.shift;
    const bool decode = D <= 3 && kp.shift == 0;

    uint64_t *keys;
    uint32_t *vals;
    DPC_TRY(ws.alloc(&keys, ix.n));
    DPC_TRY(ws.alloc(&vals, ix.n));
    DPC_TRY(ws.alloc(&ix.sidx, ix.n));
    hipLaunchKernelGGL((k_keys<D>), dim3(blocks_for(ix.n, kThreads)), dim3(kThreads), 0, s, points, ix.n, kp, keys,
                       vals);
    DPC_HIP(hipGetLastError());
    uint64_t *sk;
    uint32_t *sv;
    DPC_TRY(radix_sort_pairs(keys, vals, ix.n, kp.bits * D, ws, &sk, &sv));
    if (ix.arith == Arith::F64)
        return build_typed<double, D>(points, kp, decode, sk, sv, ws, ix);
    return build_typed<int64_t, D>(points, kp, decode, sk, sv, ws, ix);
}

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
    switch (d) {
    case 1: return build_dim<1>(points, ws, ix);
    case 2: return build_dim<2>(points, ws, ix);
    case 3: return build_dim<3>(points, ws, ix);
    case 4: return build_dim<4>(points, ws, ix);
    case 5: return build_dim<5>(points, ws, ix);
    case 6: return build_dim<6>(points, ws, ix);
    case 7: return build_dim<7>(points, ws, ix);
    case 8: return build_dim<8>(points, ws, ix);
    default: return DPC_ERR_INVALID_ARG;
    }
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
