// Dependent points through a Fenwick tree of k-d trees (Section 5,
// Algorithm 2): the paper's second dependent-point method.  Its results are
// those of the priority-search k-d tree (Definitions 2-3 fix them).
//
// The points are put in decreasing priority order (rho, then the lower index
// first).  In that order the candidates of position p are exactly the
// positions before it, and the Fenwick decomposition (Section 2) splits the
// prefix [0, p) into aligned blocks, one per set bit b of p:
// [h, h + 2^b) with h = p with bits 0..b cleared.  Each such block is the
// Fenwick range B[j] of the j with LSB(j) = 2^b, and every range B[j] is an
// even-numbered block of its size.  A query takes the nearest point of each
// of its ranges and keeps the lexicographic minimum of (D^2, index), the
// write-min of Algorithm 2.
//
// GPU form, one block size b at a time:
//   * ranges of at least 2^kScanLog2 points: range 2k and block 2k + 1 (the
//     positions that search it) form one instance of the batched k-d tree
//     build.  The range's points get keys above every query's, so the
//     dependent kernel's maximum-key pruning searches exactly the range, and
//     queries near each other in space share a wave's walk.  The key's low
//     word carries the input index, so equal distances go to the lower index.
//   * the smaller ranges, which together are the (p mod 2^kScanLog2)
//     positions just before p: a direct scan, staged through LDS.
// The per-size results are merged into a running minimum (one query has one
// result per size, so the merge needs no atomics) and scattered to input
// order at the end.
#include "dpc_internal.hpp"

#include <limits>
#include <vector>

namespace dpc {
namespace {

constexpr int kThreads = 256;
constexpr int kScanLog2 = 10;             // ranges below 2^10 points are scanned
constexpr int64_t kMaxInstances = 32768;  // instances per batched build (grid y)

// ---------------------------------------------------------------------------
// The radix sort of Algorithm 2: the points in decreasing priority.  The
// input is in index order, so a stable sort by decreasing density alone
// leaves equal densities in increasing index order, which is exactly the
// priority order (rho, -index).  Sort key: the density with its sign bit
// flipped, complemented (increasing key = decreasing density); value: the
// index (radix_sort_pairs, radix.hip).

__global__ __launch_bounds__(kThreads) void k_rs_init(const int32_t *__restrict__ rho, int64_t n,
                                                      uint32_t *__restrict__ key, uint32_t *__restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        key[i] = ~((uint32_t)rho[i] ^ 0x80000000u);
        idx[i] = (uint32_t)i;
    }
}

// ord: the indices 0 .. n-1 in decreasing priority (rho, -index).
dpc_status priority_order(const int32_t *rho, int64_t n, uint32_t *ord, Workspace &ws) {
    hipStream_t s = ws.stream;
    uint32_t *ka, *kb, *vb;
    DPC_TRY(ws.alloc(&ka, (size_t)n));
    DPC_TRY(ws.alloc(&kb, (size_t)n));
    DPC_TRY(ws.alloc(&vb, (size_t)n));
    launch(k_rs_init, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, rho, n, ka, ord);
    DPC_HIP(hipGetLastError());
    uint32_t *kout, *vout;
    DPC_TRY(radix_sort_pairs<uint32_t>(ka, ord, kb, vb, n, 32, ws, &kout, &vout));
    // four passes: the result is back in (ka, ord)
    (void)kout;
    return vout == ord ? DPC_OK : DPC_ERR_HIP;
}

// Points in priority order, and whether each is a query (rho >= rho_min).
template <int D>
__global__ __launch_bounds__(kThreads) void k_fw_gather(const int32_t *__restrict__ P,
                                                        const uint32_t *__restrict__ ord,
                                                        const int32_t *__restrict__ rho, int32_t rho_min, int64_t n,
                                                        int32_t *__restrict__ Q, uint8_t *__restrict__ act) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    const int64_t o = ord[p];
#pragma unroll
    for (int k = 0; k < D; ++k)
        Q[p * D + k] = P[o * D + k];
    act[p] = rho[o] >= rho_min ? 1 : 0;
}

// The ranges below 2^kScanLog2 points: each query scans the positions of its
// 2^kScanLog2-aligned chunk that come before it.  A workgroup takes kThreads
// consecutive queries of one chunk and stages the candidates kThreads at a
// time; every lane reads the same candidate at once (an LDS broadcast).
// Exact: differences of int32 values are exact in double, and the double
// path is taken only when every squared distance is below 2^53.
template <typename C, int D>
__global__ __launch_bounds__(kThreads) void k_fw_scan(const int32_t *__restrict__ Q, const uint32_t *__restrict__ ord,
                                                      const uint8_t *__restrict__ act, int64_t n,
                                                      int64_t *__restrict__ bd2, int32_t *__restrict__ bj) {
    __shared__ C s_x[kThreads * D];
    __shared__ int32_t s_j[kThreads];
    const int64_t p0 = (int64_t)blockIdx.x * kThreads;
    const int64_t p = p0 + threadIdx.x;
    const int64_t cs = p0 & ~(((int64_t)1 << kScanLog2) - 1);
    const bool on = p < n && act[p] != 0;
    C x[D];
#pragma unroll
    for (int k = 0; k < D; ++k)
        x[k] = p < n ? (C)Q[p * D + k] : C(0);
    C best = std::numeric_limits<C>::max();
    int32_t bestj = -1;
    for (int64_t t0 = cs; t0 <= p0; t0 += kThreads) {
        __syncthreads();
        const int64_t t = t0 + threadIdx.x;
        if (t < n) {
#pragma unroll
            for (int k = 0; k < D; ++k)
                s_x[threadIdx.x * D + k] = (C)Q[t * D + k];
            s_j[threadIdx.x] = (int32_t)ord[t];
        }
        __syncthreads();
        if (on) {
            // candidates t0 + i < p (all staged: p < n)
            const int64_t left = p - t0;
            const int lim = left < kThreads ? (int)left : kThreads;
            for (int i = 0; i < lim; ++i) {
                C s = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const C dd = x[k] - s_x[i * D + k];
                    s += dd * dd;
                }
                const int32_t j = s_j[i];
                const bool better = s < best || (s == best && (uint32_t)j < (uint32_t)bestj);
                best = better ? s : best;
                bestj = better ? j : bestj;
            }
        }
    }
    if (p < n) {
        bd2[p] = bestj >= 0 ? (int64_t)best : std::numeric_limits<int64_t>::max();
        bj[p] = bestj;
    }
}

// Keys of one block size's instances: the range's points (local index below
// 2^b) rank above every query; a query that is skipped ranks below them all
// and is not searched for (the group runs with rho window [1, 1]).
__global__ __launch_bounds__(kThreads) void k_fw_level_keys(const Inst *__restrict__ inst,
                                                            const uint32_t *__restrict__ tile_inst,
                                                            const int32_t *__restrict__ Q, int d,
                                                            const uint32_t *__restrict__ ord,
                                                            const uint8_t *__restrict__ act, int b,
                                                            const int32_t *__restrict__ sidx,
                                                            uint64_t *__restrict__ skey, uint64_t *__restrict__ maxkey) {
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const Inst &I = inst_of_tile(inst, tile_inst, ((int64_t)blockIdx.x * blockDim.x) / kTile);
    const int64_t i = pos - I.P;
    uint64_t key = 0;
    if (i < I.n) {
        const int32_t o = sidx[pos];
        const int64_t p = (I.points - Q) / d + o;
        key = (int64_t)o < ((int64_t)1 << b) ? pack_key(2, (int32_t)ord[p]) : pack_key(act[p] ? 1 : 0, -1);
        skey[pos] = key;
    }
    // the leaf's maximum, by DPP lane moves, lands in its last lane
    const int lsh = I.lsh;
    key = lsh == 6 ? group_max_u64<6>(key) : (lsh == 5 ? group_max_u64<5>(key) : group_max_u64<4>(key));
    const int64_t first = i - ((1 << lsh) - 1);  // the leaf's first position
    if ((i & ((1 << lsh) - 1)) == (1 << lsh) - 1 && first < I.n)
        maxkey[I.N + (1ll << I.height) + (i >> lsh)] = key;
}

__global__ __launch_bounds__(kThreads) void k_fw_zero(uint64_t *__restrict__ a, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m)
        a[i] = 0;
}

// Write-min of one block size's results into the running minimum.
__global__ __launch_bounds__(kThreads) void k_fw_merge(int64_t n, int b, const uint8_t *__restrict__ act,
                                                       const int32_t *__restrict__ ldep,
                                                       const int64_t *__restrict__ ld2, int64_t *__restrict__ bd2,
                                                       int32_t *__restrict__ bj) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || ((p >> b) & 1) == 0 || act[p] == 0)
        return;
    const int32_t j = ldep[p];
    if (j < 0)
        return;
    const int64_t d2 = ld2[p];
    const int32_t cj = bj[p];
    const int64_t cd = bd2[p];
    if (cj < 0 || d2 < cd || (d2 == cd && j < cj)) {
        bd2[p] = d2;
        bj[p] = j;
    }
}

__global__ __launch_bounds__(kThreads) void k_fw_out(int64_t n, const uint32_t *__restrict__ ord,
                                                     const int64_t *__restrict__ bd2, const int32_t *__restrict__ bj,
                                                     int32_t *__restrict__ dep, int64_t *__restrict__ delta2) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    const int64_t o = ord[p];
    const int32_t j = bj[p];
    dep[o] = j;
    delta2[o] = j >= 0 ? bd2[p] : std::numeric_limits<int64_t>::max();
}

template <int D>
dpc_status gather_and_scan(const Job &J, Arith arith, const uint32_t *ord, int32_t *Q, uint8_t *act, int64_t *bd2,
                           int32_t *bj, hipStream_t s) {
    const dim3 grid(blocks_for(J.n, kThreads)), block(kThreads);
    launch(k_fw_gather<D>, grid, block, 0, s, J.points, ord, (const int32_t *)J.rho, J.dep_rho_min, J.n, Q, act);
    if (arith == Arith::F64)
        launch(k_fw_scan<double, D>, grid, block, 0, s, (const int32_t *)Q, ord, (const uint8_t *)act, J.n, bd2,
               bj);
    else
        launch(k_fw_scan<int64_t, D>, grid, block, 0, s, (const int32_t *)Q, ord, (const uint8_t *)act, J.n, bd2,
               bj);
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

}  // namespace

dpc_status fenwick_dependent(const Job &J, int d, Arith arith, int lsh, Workspace &ws) {
    hipStream_t s = ws.stream;
    const int64_t n = J.n;
    if (n <= 0)
        return DPC_OK;
    const dim3 grid(blocks_for(n, kThreads)), block(kThreads);

    // priority order (the radix sort of Algorithm 2)
    uint32_t *ord;
    DPC_TRY(ws.alloc(&ord, (size_t)n));
    DPC_TRY(priority_order((const int32_t *)J.rho, n, ord, ws));

    // points in that order; the scanned small ranges start the minimum
    int32_t *Q, *bj, *ldep;
    uint8_t *act;
    int64_t *bd2, *ld2;
    DPC_TRY(ws.alloc(&Q, (size_t)n * d));
    DPC_TRY(ws.alloc(&act, (size_t)n));
    DPC_TRY(ws.alloc(&bd2, (size_t)n));
    DPC_TRY(ws.alloc(&bj, (size_t)n));
    DPC_TRY(ws.alloc(&ld2, (size_t)n));
    DPC_TRY(ws.alloc(&ldep, (size_t)n));
    switch (d) {
#define DPC_FW_CASE(DD)                                                    \
    case DD:                                                               \
        DPC_TRY(gather_and_scan<DD>(J, arith, ord, Q, act, bd2, bj, s)); \
        break;
        DPC_FW_CASE(1)
        DPC_FW_CASE(2)
        DPC_FW_CASE(3)
        DPC_FW_CASE(4)
        DPC_FW_CASE(5)
        DPC_FW_CASE(6)
        DPC_FW_CASE(7)
        DPC_FW_CASE(8)
#undef DPC_FW_CASE
    default:
        return DPC_ERR_INVALID_ARG;
    }

    // the k-d tree ranges, one block size at a time
    for (int b = kScanLog2; ((int64_t)1 << b) < n; ++b) {
        const int64_t half = (int64_t)1 << b;
        std::vector<Job> level;
        for (int64_t start = 0; start + half < n; start += 2 * half) {
            Job L;
            L.points = Q + start * d;
            L.n = (2 * half < n - start) ? 2 * half : n - start;
            L.dep_rho_min = 1;
            L.dep_rho_max = 1;
            L.dep = ldep + start;
            L.delta2 = ld2 + start;
            for (int k = 0; k < kMaxDim; ++k) {
                L.lo[k] = J.lo[k];
                L.hi[k] = J.hi[k];
            }
            level.push_back(L);
        }
        for (size_t first = 0; first < level.size(); first += (size_t)kMaxInstances) {
            const size_t last = first + (size_t)kMaxInstances < level.size() ? first + (size_t)kMaxInstances
                                                                              : level.size();
            const std::vector<Job> part(level.begin() + (std::ptrdiff_t)first, level.begin() + (std::ptrdiff_t)last);
            Workspace lw(s);
            Index ix;
            DPC_TRY(build_group(part, d, arith, lsh, lw, ix));
            DPC_TRY(lw.alloc(&ix.skey, (size_t)ix.positions));
            DPC_TRY(lw.alloc(&ix.maxkey, (size_t)ix.nodes));
            launch(k_fw_zero, dim3(blocks_for(ix.nodes, kThreads)), dim3(kThreads), 0, s, ix.maxkey, ix.nodes);
            launch(k_fw_level_keys, dim3(blocks_for(ix.positions, kThreads)), dim3(kThreads), 0, s,
                   (const Inst *)ix.inst, (const uint32_t *)ix.tile_inst, (const int32_t *)Q, d,
                   (const uint32_t *)ord, (const uint8_t *)act, b, (const int32_t *)ix.sidx, ix.skey, ix.maxkey);
            DPC_HIP(hipGetLastError());
            DPC_TRY(priority_levels(ix, s));
            DPC_TRY(launch_dependent(ix, nullptr, s));
            // lw's memory goes back to the pool stream-ordered, after these kernels
        }
        launch(k_fw_merge, grid, block, 0, s, n, b, (const uint8_t *)act, (const int32_t *)ldep,
               (const int64_t *)ld2, bd2, bj);
        DPC_HIP(hipGetLastError());
    }
    launch(k_fw_out, grid, block, 0, s, n, (const uint32_t *)ord, (const int64_t *)bd2, (const int32_t *)bj, J.dep,
           J.delta2);
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

}  // namespace dpc
