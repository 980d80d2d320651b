// Density (Section 3, Definition 1): rho_i = #{ j : D^2(i, j) <= T }.
//
// Each wavefront takes 64 consecutive sorted points and walks the tree.  For
// every node a lane classifies the node's box against its own ball:
//   outside  (nearest corner beyond the radius)   -> nothing to count;
//   inside   (farthest corner within the radius)  -> add the node's point
//            count without visiting its points (Section 6.1);
//   partial  -> the wave descends (a leaf's points are tested one by one).
// A lane that settled a node skips that node's subtree; it remembers the
// depth at which it settled, which stays valid while the walk is below it.
#include "traverse.hpp"

#include <climits>

namespace dpc {
namespace {

constexpr int kThreads = 256;

// Points of one leaf within distance^2 T of x.  The leaf's coordinates are
// wave-uniform (scalar loads); a batch of kBatch points is loaded before any
// is used so that the loads overlap.
template <typename C, int D>
__device__ inline int32_t count_within(const C (&x)[D], const C *__restrict__ p, int count, C T) {
    constexpr int kBatch = 8;
    int32_t c = 0;
    int t = 0;
    for (; t + kBatch <= count; t += kBatch) {
        C q[kBatch][D];
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
#pragma unroll
            for (int k = 0; k < D; ++k)
                q[b][k] = p[(t + b) * D + k];
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
            c += dist2<C, D>(x, q[b]) <= T ? 1 : 0;
    }
    for (; t < count; ++t)
        c += point_dist2<C, D>(x, p + t * D) <= T ? 1 : 0;
    return c;
}

template <typename C, int D, bool STATS>
__global__ __launch_bounds__(kThreads) void k_density(const C *__restrict__ coords, const C *__restrict__ box,
                                                      int64_t n, int height, C T, int32_t *__restrict__ srho,
                                                      const int32_t *__restrict__ sidx, int32_t *__restrict__ rho_out,
                                                      int64_t *counters) {
    uint64_t n_pairs = 0, n_nodes = 0, n_contained = 0;
    const int lane = __lane_id();
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t q0 = q - lane;
    if (q0 >= n)
        return;  // the whole wave lies past the end
    const bool valid = q < n;
    const int64_t qq = valid ? q : q0;
    C x[D];
#pragma unroll
    for (int k = 0; k < D; ++k)
        x[k] = coords[qq * D + k];

    int32_t cnt = 0;
    int settled = valid ? INT_MAX : -1;  // depth at which this lane settled the current path
    const uint32_t first_leaf = 1u << height;
    uint32_t v = 1;
    int depth = 0;
    for (;;) {
        int64_t start, count;
        node_range(v, depth, height, n, start, count);
        bool descend = false;
        if (count > 0) {
            bool partial = false;
            if (settled >= depth) {
                settled = INT_MAX;
                if (STATS)
                    ++n_nodes;
                C dmin2, dmax2;
                box_dist2<C, D>(x, box + (size_t)v * 2 * D, dmin2, dmax2);
                if (dmin2 > T) {
                    settled = depth;
                } else if (dmax2 <= T) {
                    cnt += (int32_t)count;
                    settled = depth;
                    if (STATS)
                        n_contained += (uint64_t)count;
                } else {
                    partial = true;
                }
            }
            if (v >= first_leaf) {
                if (partial) {
                    if (STATS)
                        n_pairs += (uint64_t)count;
                    cnt += count_within<C, D>(x, coords + start * D, (int)count, T);
                }
            } else {
                descend = __ballot(partial) != 0;
            }
        }
        if (descend) {
            v <<= 1;
            ++depth;
            continue;
        }
        while (v & 1u) {
            v >>= 1;
            --depth;
        }
        if (v == 0)
            break;
        v += 1;
    }
    if (valid) {
        srho[q] = cnt;
        rho_out[sidx[q]] = cnt;
    }
    if (STATS) {
        add_wave_count(counters, kDensityPairs, n_pairs);
        add_wave_count(counters, kDensityNodes, n_nodes);
        add_wave_count(counters, kDensityContained, n_contained);
    }
}

template <typename C, bool STATS>
dpc_status launch_typed(const Index &ix, C T, int32_t *srho, int32_t *rho_out, int64_t *counters, hipStream_t s) {
    const C *coords = static_cast<const C *>(ix.coords);
    const C *box = static_cast<const C *>(ix.box);
    const dim3 grid(blocks_for(ix.n, kThreads)), block(kThreads);
    switch (ix.d) {
#define DPC_DENSITY_CASE(DD)                                                                                    \
    case DD:                                                                                                    \
        hipLaunchKernelGGL((k_density<C, DD, STATS>), grid, block, 0, s, coords, box, ix.n, ix.height, T, srho,    \
                           ix.sidx, rho_out, counters);                                                         \
        break;
        DPC_DENSITY_CASE(1)
        DPC_DENSITY_CASE(2)
        DPC_DENSITY_CASE(3)
        DPC_DENSITY_CASE(4)
        DPC_DENSITY_CASE(5)
        DPC_DENSITY_CASE(6)
        DPC_DENSITY_CASE(7)
        DPC_DENSITY_CASE(8)
#undef DPC_DENSITY_CASE
    default:
        return DPC_ERR_INVALID_ARG;
    }
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

}  // namespace

dpc_status launch_density(const Index &ix, int64_t T, int32_t *srho, int32_t *rho_out, int64_t *counters,
                          hipStream_t s) {
    if (ix.arith == Arith::F64) {
        // every squared distance is below 2^53, so a larger threshold acts like 2^53
        const double t = T >= (1ll << 53) ? 9007199254740992.0 : (double)T;
        return counters ? launch_typed<double, true>(ix, t, srho, rho_out, counters, s)
                        : launch_typed<double, false>(ix, t, srho, rho_out, nullptr, s);
    }
    return counters ? launch_typed<int64_t, true>(ix, T, srho, rho_out, counters, s)
                    : launch_typed<int64_t, false>(ix, T, srho, rho_out, nullptr, s);
}

}  // namespace dpc
