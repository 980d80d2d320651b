// Spatial index set-up: coordinate bounds (the host read-back), the choice
// of exact arithmetic, the layout of a group of instances, the tree shape,
// and after the density step the priority keys and per-node maximum keys.
// The k-d trees themselves are built in kdtree.hip.
#include "dpc_internal.hpp"

#include <atomic>

#include <limits>

namespace dpc {
namespace {

constexpr int kThreads = 256;

// ---------------------------------------------------------------------------
// bounds

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

// Workgroup minimum and maximum per axis of per-thread values (valid in
// out_min / out_max, shared memory, after the call).
template <int D>
__device__ inline void block_bounds(const int32_t (&lmin)[D], const int32_t (&lmax)[D], int32_t *out_min,
                                    int32_t *out_max) {
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
        for (int q = 1; q < kThreads / kWave; ++q) {
            a = min(a, s_min[q][k]);
            b = max(b, s_max[q][k]);
        }
        out_min[k] = a;
        out_max[k] = b;
    }
    __syncthreads();
}

// A planned replay's check: the points' bounds (mm, just computed) must lie
// inside the bounds the plan was made for.
struct Box {
    int32_t lo[kMaxDim];
    int32_t hi[kMaxDim];
};

// (A replay clears the status word first; a check only ever sets the range
// error, so the checks of several dimensions add up.)
__global__ void k_bounds_check(const int32_t *__restrict__ mm, Box planned, int d, int32_t *status) {
    if (threadIdx.x == 0) {
        bool ok = true;
        for (int k = 0; k < d; ++k)
            ok = ok && mm[k] >= planned.lo[k] && mm[kMaxDim + k] <= planned.hi[k];
        if (!ok)
            status[0] = (int32_t)DPC_ERR_RANGE;
    }
}

// The same for every instance of a group: mm and planned are
// [count][lo[kMaxDim], hi[kMaxDim]].
__global__ void k_bounds_check_group(const int32_t *__restrict__ mm, const int32_t *__restrict__ planned, int count,
                                     int d, int32_t *status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count)
        return;
    const int32_t *m = mm + (int64_t)i * 2 * kMaxDim;
    const int32_t *p = planned + (int64_t)i * 2 * kMaxDim;
    bool ok = true;
    for (int k = 0; k < d; ++k)
        ok = ok && m[k] >= p[k] && m[kMaxDim + k] <= p[kMaxDim + k];
    if (!ok)
        status[0] = (int32_t)DPC_ERR_RANGE;
}

__global__ void k_bounds_init(int32_t *mm) {
    const int t = threadIdx.x;
    if (t < kMaxDim) {
        mm[t] = std::numeric_limits<int32_t>::max();
        mm[kMaxDim + t] = std::numeric_limits<int32_t>::min();
    }
}

// One instance: a grid-stride pass, combined with atomics.
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
    __shared__ int32_t s_out[2 * D];
    block_bounds<D>(lmin, lmax, s_out, s_out + D);
    if (threadIdx.x < D) {
        atomicMin(&mm[threadIdx.x], s_out[threadIdx.x]);
        atomicMax(&mm[kMaxDim + threadIdx.x], s_out[D + threadIdx.x]);
    }
}

// The same pass four points at a time, as D aligned 16-byte loads (P 16-byte
// aligned): word l, component c holds flat value 4l + c of the four points,
// which belongs to axis (4l + c) mod D.  The n mod 4 points left over are
// read one by one.
template <int D>
__global__ __launch_bounds__(kThreads) void k_bounds_x4(const int32_t *__restrict__ P, int64_t n, int32_t *mm) {
    int32_t lmin[D], lmax[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lmin[k] = std::numeric_limits<int32_t>::max();
        lmax[k] = std::numeric_limits<int32_t>::min();
    }
    const int4 *Q = reinterpret_cast<const int4 *>(P);
    const int64_t groups = n / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t g = t; g < groups; g += stride) {
        int4 w[D];
#pragma unroll
        for (int l = 0; l < D; ++l)
            w[l] = Q[g * D + l];
#pragma unroll
        for (int l = 0; l < D; ++l) {
            const int32_t v[4] = {w[l].x, w[l].y, w[l].z, w[l].w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int k = (4 * l + c) % D;
                lmin[k] = min(lmin[k], v[c]);
                lmax[k] = max(lmax[k], v[c]);
            }
        }
    }
    if (t < n - groups * 4) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int32_t v = P[(groups * 4 + t) * D + k];
            lmin[k] = min(lmin[k], v);
            lmax[k] = max(lmax[k], v);
        }
    }
    __shared__ int32_t s_out[2 * D];
    block_bounds<D>(lmin, lmax, s_out, s_out + D);
    if (threadIdx.x < D) {
        atomicMin(&mm[threadIdx.x], s_out[threadIdx.x]);
        atomicMax(&mm[kMaxDim + threadIdx.x], s_out[D + threadIdx.x]);
    }
}

// A group: every workgroup takes one tile of one instance and writes its
// bounds to the tile's slot; k_bounds_reduce combines each instance's tiles.
template <int D>
__global__ __launch_bounds__(kThreads) void k_bounds_tiles(const Inst *__restrict__ inst,
                                                           const uint32_t *__restrict__ tile_inst,
                                                           int32_t *__restrict__ tmm) {
    const int64_t tile = blockIdx.x;
    const Inst &I = inst_of_tile(inst, tile_inst, tile);
    const int64_t e0 = (tile - I.P / kTile) * kTile;
    int32_t lmin[D], lmax[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lmin[k] = std::numeric_limits<int32_t>::max();
        lmax[k] = std::numeric_limits<int32_t>::min();
    }
    for (int64_t i = e0 + threadIdx.x; i < e0 + kTile && i < I.n; i += kThreads) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int32_t v = I.points[i * D + k];
            lmin[k] = min(lmin[k], v);
            lmax[k] = max(lmax[k], v);
        }
    }
    __shared__ int32_t s_out[2 * D];
    block_bounds<D>(lmin, lmax, s_out, s_out + D);
    if (threadIdx.x < 2 * D)
        tmm[tile * 2 * D + threadIdx.x] = s_out[threadIdx.x];
}

template <int D>
__global__ __launch_bounds__(kThreads) void k_bounds_reduce(const Inst *__restrict__ inst,
                                                            const int32_t *__restrict__ tmm, int32_t *__restrict__ mm) {
    const Inst &I = inst[blockIdx.x];
    const int64_t t0 = I.P / kTile, t1 = t0 + (I.n + kTile - 1) / kTile;
    int32_t lmin[D], lmax[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lmin[k] = std::numeric_limits<int32_t>::max();
        lmax[k] = std::numeric_limits<int32_t>::min();
    }
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kThreads) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            lmin[k] = min(lmin[k], tmm[t * 2 * D + k]);
            lmax[k] = max(lmax[k], tmm[t * 2 * D + D + k]);
        }
    }
    __shared__ int32_t s_out[2 * D];
    block_bounds<D>(lmin, lmax, s_out, s_out + D);
    if (threadIdx.x < D) {
        mm[(int64_t)blockIdx.x * 2 * kMaxDim + threadIdx.x] = s_out[threadIdx.x];
        mm[(int64_t)blockIdx.x * 2 * kMaxDim + kMaxDim + threadIdx.x] = s_out[D + threadIdx.x];
    }
}

// ---------------------------------------------------------------------------
// priority keys (pack_key) and the per-node maxima

__global__ void k_fill_u64(uint64_t *__restrict__ a, int64_t m, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m)
        a[i] = v;
}

// Keys of the sorted positions plus the maxima of non-empty leaves (the
// others stay 0).  rho comes in sorted order (srho, position-indexed) or in
// each instance's input order (its rho array, through sidx).
__global__ __launch_bounds__(kThreads) void k_keys_leaf(const Inst *__restrict__ inst,
                                                        const uint32_t *__restrict__ tile_inst,
                                                        const int32_t *__restrict__ srho,
                                                        const int32_t *__restrict__ sidx,
                                                        uint64_t *__restrict__ skey, uint64_t *__restrict__ maxkey) {
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const Inst &I = inst_of_tile(inst, tile_inst, ((int64_t)blockIdx.x * blockDim.x) / kTile);
    const int64_t i = pos - I.P;
    uint64_t key = 0;
    if (i < I.n) {
        const int32_t o = sidx[pos];
        const int32_t r = srho ? srho[pos] : I.rho[o];
        key = pack_key(r, o);
        skey[pos] = key;
    }
    // the leaf's maximum, by DPP lane moves, lands in its last lane
    const int lsh = I.lsh;
    key = lsh == 6 ? group_max_u64<6>(key) : (lsh == 5 ? group_max_u64<5>(key) : group_max_u64<4>(key));
    const int64_t first = i - ((1 << lsh) - 1);  // the leaf's first position
    if ((i & ((1 << lsh) - 1)) == (1 << lsh) - 1 && first < I.n)
        maxkey[I.N + (1ll << I.height) + (i >> lsh)] = key;
}

// One instance: up to 8 levels of maxima above 256 consecutive nodes of one
// depth.
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

// A group: the maxima of one depth of every instance (blockIdx.y) from the
// depth below.
__global__ __launch_bounds__(kThreads) void k_key_level(const Inst *__restrict__ inst, int depth,
                                                        uint64_t *__restrict__ maxkey) {
    const Inst &I = inst[blockIdx.y];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (depth >= I.height || k >= (1ll << depth))
        return;
    const int64_t v = (1ll << depth) + k;
    const uint64_t a = maxkey[I.N + 2 * v], b = maxkey[I.N + 2 * v + 1];
    maxkey[I.N + v] = a > b ? a : b;
}

// log2 of the LDS subtree size (2048 points up to three dimensions, else
// 1024) over the leaf size
int bottom_levels(int d, int lsh) { return (d <= 3 ? 11 : 10) - lsh; }

int tree_height(int64_t n, int lsh) {
    const int64_t leaves = (n + (1ll << lsh) - 1) >> lsh;
    int h = 0;
    while ((1ll << h) < leaves)
        ++h;
    return h;
}

int64_t padded(int64_t n) { return (n + kTile - 1) / kTile * kTile; }

}  // namespace

// ---------------------------------------------------------------------------
// host side

int64_t isqrt64(int64_t v) {
    int64_t r = (int64_t)__builtin_sqrt((double)v);
    while (r > 0 && (__int128)r * r > v)
        --r;
    while ((__int128)(r + 1) * (r + 1) <= v)
        ++r;
    return r;
}

dpc_status job_bounds(std::vector<Job> &jobs, int d, Workspace &ws, std::vector<int> *bad) {
    hipStream_t s = ws.stream;
    const int count = (int)jobs.size();
    std::vector<int32_t> host_mm((size_t)count * 2 * kMaxDim);
    if (count == 1) {
        int32_t *mm;
        DPC_TRY(ws.alloc(&mm, 2 * kMaxDim));
        launch(k_bounds_init, dim3(1), dim3(kWave), 0, s, mm);
        const unsigned grid = blocks_for(jobs[0].n, kThreads) < 1024u ? blocks_for(jobs[0].n, kThreads) : 1024u;
        const bool aligned = (reinterpret_cast<uintptr_t>(jobs[0].points) & 15u) == 0;
        switch (d) {
#define DPC_BOUNDS_CASE(DD)                                                                                   \
    case DD:                                                                                                  \
        if (aligned)                                                                                          \
            launch((k_bounds_x4<DD>), dim3(grid), dim3(kThreads), 0, s, jobs[0].points, jobs[0].n, mm);       \
        else                                                                                                  \
            launch((k_bounds<DD>), dim3(grid), dim3(kThreads), 0, s, jobs[0].points, jobs[0].n, mm);          \
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
        DPC_HIP(hipMemcpyAsync(host_mm.data(), mm, 2 * kMaxDim * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (t_record && t_plan_status) {
            // a plan's replays check the points against the bounds read now
            DPC_HIP(hipStreamSynchronize(s));
            Box planned{};
            for (int k = 0; k < kMaxDim; ++k) {
                planned.lo[k] = host_mm[k];
                planned.hi[k] = host_mm[kMaxDim + k];
            }
            launch(k_bounds_check, dim3(1), dim3(kWave), 0, s, (const int32_t *)mm, planned, d, t_plan_status);
            DPC_HIP(hipGetLastError());
        }
    } else {
        // instances laid out tile by tile, bounds per tile, then per instance
        std::vector<Inst> pre(count);
        std::vector<uint32_t> tiles;
        int64_t P = 0;
        for (int i = 0; i < count; ++i) {
            Inst I = {};
            I.n = jobs[i].n;
            I.P = P;
            I.points = jobs[i].points;
            pre[i] = I;
            for (int64_t t = 0; t < padded(I.n) / kTile; ++t)
                tiles.push_back((uint32_t)i);
            P += padded(I.n);
        }
        Inst *d_inst;
        uint32_t *d_tiles;
        int32_t *tmm, *mm;
        DPC_TRY(ws.alloc(&d_inst, (size_t)count));
        DPC_TRY(ws.alloc(&d_tiles, tiles.size()));
        DPC_TRY(ws.alloc(&tmm, tiles.size() * 2 * kMaxDim));
        DPC_TRY(ws.alloc(&mm, (size_t)count * 2 * kMaxDim));
        DPC_HIP(hipMemcpyAsync(d_inst, pre.data(), count * sizeof(Inst), hipMemcpyHostToDevice, s));
        DPC_HIP(hipMemcpyAsync(d_tiles, tiles.data(), tiles.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
        const unsigned nt = (unsigned)tiles.size();
        switch (d) {
#define DPC_BOUNDS_CASE(DD)                                                                                     \
    case DD:                                                                                                    \
        launch((k_bounds_tiles<DD>), dim3(nt), dim3(kThreads), 0, s, d_inst, d_tiles, tmm);          \
        launch((k_bounds_reduce<DD>), dim3((unsigned)count), dim3(kThreads), 0, s, d_inst, tmm, mm); \
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
        DPC_HIP(hipMemcpyAsync(host_mm.data(), mm, host_mm.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (t_record && t_plan_status) {
            // a plan's replays check every instance against the bounds read now
            DPC_HIP(hipStreamSynchronize(s));
            int32_t *planned;
            DPC_TRY(ws.alloc(&planned, host_mm.size()));
            DPC_HIP(hipMemcpyAsync(planned, host_mm.data(), host_mm.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                   s));
            launch(k_bounds_check_group, dim3(blocks_for(count, kThreads)), dim3(kThreads), 0, s,
                   (const int32_t *)mm, (const int32_t *)planned, count, d, t_plan_status);
            DPC_HIP(hipGetLastError());
        }
    }
    DPC_HIP(hipStreamSynchronize(s));
    dpc_status st = DPC_OK;
    for (int i = 0; i < count; ++i) {
        Job &J = jobs[i];
        unsigned __int128 sum = 0;
        for (int k = 0; k < d; ++k) {
            J.lo[k] = host_mm[(size_t)i * 2 * kMaxDim + k];
            J.hi[k] = host_mm[(size_t)i * 2 * kMaxDim + kMaxDim + k];
            const unsigned __int128 w = (unsigned __int128)((int64_t)J.hi[k] - (int64_t)J.lo[k]);
            sum += w * w;
        }
        // every squared distance must fit in int64
        if (sum > (unsigned __int128)std::numeric_limits<int64_t>::max()) {
            st = DPC_ERR_RANGE;
            if (bad)
                bad->push_back(i);
        }
    }
    return st;
}

Arith job_arith(const Job &J, int d) {
    unsigned __int128 sum = 0;
    for (int k = 0; k < d; ++k) {
        const unsigned __int128 w = (unsigned __int128)((int64_t)J.hi[k] - (int64_t)J.lo[k]);
        sum += w * w;
    }
    // below 2^53 doubles are exact
    return sum < ((unsigned __int128)1 << 53) ? Arith::F64 : Arith::I64;
}

void density_params(Inst &I, int64_t T, int d) {
    // the clamped integer comparisons need M <= R, where d * R^2 < 2^31 and
    // R < 2^15
    I.T = T;
    I.r = isqrt64(T);
    const int64_t R0 = isqrt64((int64_t)std::numeric_limits<int32_t>::max() / d);
    const int64_t R = R0 < 32767 ? R0 : 32767;
    const int64_t M = I.r + 1;
    I.R = (int32_t)R;
    I.M = (int32_t)(M <= R ? M : R + 1);
    I.limit = M <= R ? (int32_t)(R - M) : -1;
    I.Tn = M <= R ? (int32_t)T : 0;
}

// Leaf size per dimension (log2).  Smaller leaves prune more point tests but
// visit more nodes; on the stand-in workloads 64 points were the fastest in
// 2-D, 3-D and 8-D, so it is the default (dpc_autotune measures an
// instance).  Any choice gives the same outputs.
namespace {
#ifndef DPC_DEFAULT_LSH
#define DPC_DEFAULT_LSH 6
#endif
std::atomic<int> g_leaf_log2[kMaxDim + 1] = {DPC_DEFAULT_LSH, DPC_DEFAULT_LSH, DPC_DEFAULT_LSH,
                                             DPC_DEFAULT_LSH, DPC_DEFAULT_LSH, DPC_DEFAULT_LSH,
                                             DPC_DEFAULT_LSH, DPC_DEFAULT_LSH, DPC_DEFAULT_LSH};
}  // namespace

int leaf_log2(int d) { return d >= 1 && d <= kMaxDim ? g_leaf_log2[d].load(std::memory_order_relaxed) : kMaxLeafLog2; }

void set_leaf_log2(int d, int lsh) {
    if (d >= 1 && d <= kMaxDim && lsh >= kMinLeafLog2 && lsh <= kMaxLeafLog2)
        g_leaf_log2[d].store(lsh, std::memory_order_relaxed);
}

uint64_t workspace_bound(int64_t n, int d) {
    if (n <= 0)
        return 0;
    const uint64_t D = (uint64_t)d, W = (D + 1) / 2;
    const uint64_t Pn = (uint64_t)padded(n), tiles = Pn / kTile;
    // the smaller leaf size has more nodes and leaves: the bound holds for both
    const int lsh = kMinLeafLog2;
    const int h = tree_height(n, lsh);
    const uint64_t leaves = 1ull << h, nodes = 2 * leaves;
    const int jb = h > bottom_levels(d, lsh) ? h - bottom_levels(d, lsh) : 0;
    uint64_t b = 0;
    // per position: coords (8 bytes per axis), the two relative-coordinate
    // and index buffers of the build, the original index, the packed leaf
    // offsets, the key, the sorted density and the label parents
    b += Pn * (8 * D + 2 * 4 * D + 2 * 4 + 4 + 4 * W + 8 + 4 + 4);
    // per node: box, relative box, split hint, maximum key; per leaf: corner and width
    b += nodes * (16 * D + 8 * D + 8 + 8) + leaves * (4 * D + 4);
    // top levels: node boxes, histograms (widest coordinates: 32 bits), select records
    b += (2ull << jb) * 2 * D * 4;
    for (int l = 0; l < jb; ++l) {
        const int bits = top_level_bits(l);
        b += (uint64_t)((32 + bits - 1) / bits) * (1ull << l) * (1ull << bits) * 4;
    }
    b += (jb > 0 ? 1ull << (jb - 1) : 0) * 32;
    // per tile: partition counts, tile boxes, the tile table and tile bounds
    b += tiles * (4 + 4 + 16 * D + 4 + 2 * kMaxDim * 4);
    // descriptor, bounds, work tables of the top levels and subtrees
    b += sizeof(Inst) + 2 * kMaxDim * 4 + 4 * (uint64_t)jb * (tiles + 1) + 8 * 2 * ((1ull << jb) + 1);
    // the instrumented kernels' counters and the labels' flag
    b += kCounters * 8 + 8;
    // rounding of every allocation
    b += (uint64_t)Workspace::kCap * 256;
    return b;
}

dpc_status build_group(const std::vector<Job> &jobs, int d, Arith arith, int lsh, Workspace &ws, Index &ix) {
    if (lsh < kMinLeafLog2 || lsh > kMaxLeafLog2)
        return DPC_ERR_INVALID_ARG;
    ix.lsh = lsh;
    hipStream_t s = ws.stream;
    ix.d = d;
    ix.arith = arith;
    ix.count = (int)jobs.size();
    ix.host.assign(jobs.size(), Inst{});
    ix.intbox = arith == Arith::F64;
    int64_t P = 0, N = 0, L = 0, H = 0, S = 0, B = 0;
    for (int i = 0; i < ix.count; ++i) {
        const Job &J = jobs[i];
        Inst &I = ix.host[i];
        I.n = J.n;
        I.height = tree_height(J.n, lsh);
        I.lsh = lsh;
        I.jb = I.height > bottom_levels(d, lsh) ? I.height - bottom_levels(d, lsh) : 0;
        uint32_t widest = 0;
        for (int k = 0; k < kMaxDim; ++k) {
            I.lo[k] = k < d ? J.lo[k] : 0;
            I.span[k] = k < d ? (uint32_t)((int64_t)J.hi[k] - (int64_t)J.lo[k]) : 0u;
            widest = I.span[k] > widest ? I.span[k] : widest;
        }
        I.wbits = widest ? 32 - __builtin_clz(widest) : 0;
        I.P = P;
        I.N = N;
        I.L = L;
        I.H = H;
        I.S = S;
        I.B = B;
        P += padded(J.n);
        N += 2ll << I.height;
        L += 1ll << I.height;
        // shared histograms for the levels above those split one workgroup per node
        int64_t hw = 0;
        for (int l = 0; l < top_owned_from(I.height, lsh, I.jb); ++l) {
            const int bits = top_level_bits(l);
            hw += (int64_t)((I.wbits + bits - 1) / bits) * (1ll << l) * (1ll << bits);
        }
        H += hw;
        S += I.jb > 0 ? 1ll << (I.jb - 1) : 0;
        B += I.jb > 0 ? (2ll << I.jb) * 2 * d : 0;
        density_params(I, J.T, d);
        if (I.limit < 0)
            ix.intbox = false;
        I.dep_rho_min = J.dep_rho_min;
        I.dep_rho_max = J.dep_rho_max;
        I.rho_min = J.rho_min;
        I.Td = J.Td;
        I.points = J.points;
        I.rho = J.rho;
        I.dep = J.dep;
        I.delta2 = J.delta2;
        I.label = J.label;
        ix.max_height = I.height > ix.max_height ? I.height : ix.max_height;
        ix.max_jb = I.jb > ix.max_jb ? I.jb : ix.max_jb;
        ix.max_wbits = I.wbits > ix.max_wbits ? I.wbits : ix.max_wbits;
    }
    ix.positions = P;
    ix.nodes = N;
    ix.leaves = L;
    (void)s;
    return build_kdtree(ws, ix);
}

dpc_status upload_group(Workspace &ws, Index &ix) {
    hipStream_t s = ws.stream;
    DPC_TRY(ws.alloc(&ix.inst, (size_t)ix.count));
    DPC_HIP(hipMemcpyAsync(ix.inst, ix.host.data(), ix.count * sizeof(Inst), hipMemcpyHostToDevice, s));
    std::vector<uint32_t> tiles;
    if (ix.count > 1) {
        for (int i = 0; i < ix.count; ++i)
            for (int64_t t = 0; t < padded(ix.host[i].n) / kTile; ++t)
                tiles.push_back((uint32_t)i);
        DPC_TRY(ws.alloc(&ix.tile_inst, tiles.size()));
        DPC_HIP(hipMemcpyAsync(ix.tile_inst, tiles.data(), tiles.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    }
    DPC_HIP(hipStreamSynchronize(s));  // the host copies go out of scope
    return DPC_OK;
}

dpc_status build_priority(const int32_t *srho, bool rho_orig, Workspace &ws, Index &ix) {
    hipStream_t s = ws.stream;
    (void)rho_orig;  // without srho the keys read each instance's rho array
    DPC_TRY(ws.alloc(&ix.skey, (size_t)ix.positions));
    DPC_TRY(ws.alloc(&ix.maxkey, (size_t)ix.nodes));
    launch(k_fill_u64, dim3(blocks_for(ix.nodes, kThreads)), dim3(kThreads), 0, s, ix.maxkey, ix.nodes,
                       (uint64_t)0);
    launch(k_keys_leaf, dim3(blocks_for(ix.positions, kThreads)), dim3(kThreads), 0, s, ix.inst,
                       ix.tile_inst, srho, ix.sidx, ix.skey, ix.maxkey);
    return priority_levels(ix, s);
}

dpc_status priority_levels(Index &ix, hipStream_t s) {
    if (ix.count == 1) {
        for (int depth = ix.host[0].height; depth > 0;) {
            const int lv = depth < 8 ? depth : 8;
            const int64_t nodes = 1ll << depth;
            const unsigned grid = nodes < kThreads ? 1u : (unsigned)(nodes / kThreads);
            launch(k_key_up, dim3(grid), dim3(kThreads), 0, s, ix.maxkey, depth, lv);
            depth -= lv;
        }
    } else {
        for (int depth = ix.max_height - 1; depth >= 0; --depth) {
            const unsigned gx = blocks_for(1ll << depth, kThreads);
            launch(k_key_level, dim3(gx, (unsigned)ix.count), dim3(kThreads), 0, s, ix.inst, depth,
                               ix.maxkey);
        }
    }
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

}  // namespace dpc
