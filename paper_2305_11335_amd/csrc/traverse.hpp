// Device helpers shared by the density and dependent-point kernels.
//
// Both kernels give one wavefront 64 consecutive sorted points as queries and
// walk the implicit tree together: the walk is wave-uniform (node index and
// depth live in scalar registers), and each lane keeps its own per-query
// state.  The walk is stackless: in heap numbering the sibling of v is v ^ 1
// and the parent v >> 1, so a depth-first order only needs the current node
// and, when children may be visited in either order, a second "virtual"
// index u whose low bit says whether v was the first or second child taken.
#pragma once

#include "dpc_internal.hpp"

#include <type_traits>

namespace dpc {

// Squared distance from a point to a box (0 inside) and to the box's
// farthest corner.  Exact for both coordinate types on the chosen path.
// max of two values; on the double path (never NaN here) one v_max_f64
template <typename C>
__device__ inline C max2(C a, C b) {
    if constexpr (std::is_same<C, double>::value)
        return __builtin_fmax(a, b);
    else
        return a > b ? a : b;
}

template <typename C, int D>
__device__ inline void box_dist2(const C (&x)[D], const C *__restrict__ b, C &dmin2, C &dmax2) {
    C mn = 0, mx = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const C lo = b[2 * k], hi = b[2 * k + 1];
        const C a = lo - x[k];
        const C c = x[k] - hi;
        const C near = max2<C>(max2<C>(a, c), C(0));
        const C far = max2<C>(-a, -c);
        mn += near * near;
        mx += far * far;
    }
    dmin2 = mn;
    dmax2 = mx;
}

template <typename C, int D>
__device__ inline C box_min_dist2(const C (&x)[D], const C *__restrict__ b) {
    C mn = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const C a = b[2 * k] - x[k];
        const C c = x[k] - b[2 * k + 1];
        const C near = max2<C>(max2<C>(a, c), C(0));
        mn += near * near;
    }
    return mn;
}

template <typename C, int D>
__device__ inline C dist2(const C (&x)[D], const C (&p)[D]) {
    C s = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const C t = x[k] - p[k];
        s += t * t;
    }
    return s;
}

template <typename C, int D>
__device__ inline C point_dist2(const C (&x)[D], const C *__restrict__ p) {
    C s = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const C t = x[k] - p[k];
        s += t * t;
    }
    return s;
}

// The workgroups of a launch go to the 8 XCDs in turn (workgroup i to XCD
// i mod 8), and each XCD has an L2 of its own.  This maps workgroup i to the
// chunk of work it takes so that each XCD takes runs of RUN consecutive
// chunks: neighbouring queries walk the same nodes and leaves, which then
// stay in one L2, while the runs still alternate between XCDs so that dense
// regions are shared out.  A bijection of [0, nb) for any nb (the last,
// partial round of runs keeps the plain order).
template <uint32_t RUN>
__device__ inline uint32_t xcd_chunk(uint32_t b, uint32_t nb) {
    constexpr uint32_t kXcds = 8;
    if (RUN <= 1)
        return b;
    const uint32_t full = nb - nb % (kXcds * RUN);
    if (b >= full)
        return b;
    const uint32_t x = b % kXcds, r = b / kXcds;
    return ((r / RUN) * kXcds + x) * RUN + r % RUN;
}

// First query position of this wavefront (a value the compiler knows is
// uniform across the wave, so state derived from it stays scalar).
template <uint32_t RUN>
__device__ inline int64_t wave_base(int block_threads) {
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    return (int64_t)xcd_chunk<RUN>(blockIdx.x, gridDim.x) * block_threads + (int64_t)w * kWave;
}

// First sorted position and number of points below node v at `depth` of a
// tree with 2^height leaves of 2^lsh points.  Computed in 32 bits (scalar
// instructions; there is no 64-bit scalar compare): n < 2^31 and a tree's
// leaves hold fewer than 2^32 positions, so every position and node capacity
// fits.
__device__ inline void node_range(uint32_t v, int depth, int height, int lsh, int64_t n, int64_t &start,
                                  int64_t &count) {
    const int sh = height - depth + lsh;
    const uint32_t st = (v - (1u << depth)) << sh;
    const uint32_t cap = 1u << sh;
    // (signed: st and n are below 2^31, and a signed max stays on the scalar
    // unit where an unsigned saturating subtraction would not)
    int32_t left = (int32_t)n - (int32_t)st;
    left = left > 0 ? left : 0;
    start = st;
    count = (uint32_t)left < cap ? (uint32_t)left : cap;
}

// Orders a wavefront's LDS writes before its later LDS reads (and the reads
// before later writes): a leaf staged by some lanes is read by all.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Adds a per-lane count into counters[slot] with one atomic per wavefront.
__device__ inline void add_wave_count(int64_t *counters, int slot, uint64_t v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, o, kWave);
        const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, kWave);
        v += ((uint64_t)hi << 32) | lo;
    }
    if (__lane_id() == 0)
        atomicAdd(reinterpret_cast<unsigned long long *>(counters + slot), (unsigned long long)v);
}

}  // namespace dpc
