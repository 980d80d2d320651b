// Internal declarations of libdpc (not installed; the public interface is
// include/libdpc.h).
//
// The spatial index is a balanced k-d tree in an implicit layout: the points
// are permuted so that leaf c holds positions [c*LS, (c+1)*LS) and node v
// (heap numbering, root 1, children 2v and 2v+1) covers the union of its
// leaves; each node's points are split evenly across the longest side of its
// box.  Nodes store their tight bounding box and the highest priority key
// below them: the boxes give the containment count of Section 6.1 and the
// pruning of Section 3.2, the keys the priority pruning of Section 4.2.2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/libdpc.h"

namespace dpc {

constexpr int kWave = 64;
constexpr int kMaxDim = 8;
constexpr int kLeafSize = 32;  // points per tree leaf

// Coordinates and squared distances are exact in double when every squared
// distance stays below 2^53 (the "f64" path); otherwise 64-bit integers.
enum class Arith { F64, I64 };

struct Index {
    int64_t n = 0;
    int d = 0;
    Arith arith = Arith::F64;
    int32_t lo[kMaxDim] = {0};
    int32_t hi[kMaxDim] = {0};
    int height = 0;         // tree height: 2^height leaves
    int64_t n_leaves = 0;   // 2^height
    // device arrays (owned by the workspace)
    void *coords = nullptr;     // sorted coordinates [n][d], double or int64
    int32_t *sidx = nullptr;    // original index of each sorted position [n]
    void *box = nullptr;        // node boxes [2*n_leaves][d][2] (min, max), like coords
    uint32_t *rbox = nullptr;   // the same boxes relative to lo, as uint32
    uint64_t *skey = nullptr;   // priority key of each sorted position [n]
    uint64_t *maxkey = nullptr; // per-node maximum key [2*n_leaves]
    // Split of each internal node v < n_leaves: axis << 32 | median offset
    // from lo along that axis (points below go left).  Only a hint for the
    // order in which children are searched.
    uint64_t *split = nullptr;
    // Leaf records: the leaf box's lower corner relative to lo [n_leaves][d],
    // its widest side [n_leaves], and every point's offsets from that corner
    // as 16-bit halves, two axes per word [n][(d+1)/2] (meaningful only when
    // the widest side is below 2^16).
    uint32_t *leaf_org = nullptr;
    uint32_t *leaf_ext = nullptr;
    uint32_t *leaf_pack = nullptr;
};

// The library's stream-ordered memory pool on the current device (created on
// first use).  Unlike the device's default pool it keeps freed memory
// instead of returning it at every synchronisation, so repeated calls do not
// map their workspace again.  Returns nullptr if no pool could be created.
hipMemPool_t workspace_pool();

// Stream-ordered device workspace: every allocation is released together.
struct Workspace {
    hipStream_t stream;
    static constexpr int kCap = 128;
    void *ptrs[kCap];
    int count = 0;
    hipMemPool_t pool;
    explicit Workspace(hipStream_t s) : stream(s), pool(workspace_pool()) {}
    ~Workspace() { release(); }
    template <class T>
    dpc_status alloc(T **out, size_t elems) {
        *out = nullptr;
        if (count >= kCap)
            return DPC_ERR_OOM;
        void *p = nullptr;
        size_t bytes = elems * sizeof(T);
        if (bytes == 0)
            bytes = 256;
        const hipError_t e = pool ? hipMallocFromPoolAsync(&p, bytes, pool, stream) : hipMallocAsync(&p, bytes, stream);
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return DPC_ERR_OOM;
        }
        ptrs[count++] = p;
        *out = static_cast<T *>(p);
        return DPC_OK;
    }
    void release() {
        for (int i = 0; i < count; ++i)
            (void)hipFreeAsync(ptrs[i], stream);
        count = 0;
    }
};

#define DPC_HIP(call)                                      \
    do {                                                   \
        if ((call) != hipSuccess) {                        \
            (void)hipGetLastError();                       \
            return DPC_ERR_HIP;                            \
        }                                                  \
    } while (0)

#define DPC_TRY(call)                                      \
    do {                                                   \
        dpc_status _st = (call);                           \
        if (_st != DPC_OK)                                 \
            return _st;                                    \
    } while (0)

// Work counters of the instrumented kernels (DPC_COUNT_WORK), in the order of
// the dpc_stats fields.
enum Counter {
    kDensityPairs = 0,
    kDensityNodes,
    kDensityContained,
    kDependentPairs,
    kDependentNodes,
    kDensityWaveNodes,
    kDensityWavePoints,
    kDependentWaveNodes,
    kDependentWavePoints,
    kCounters
};

// Exact thresholds (host).
dpc_status square_threshold(double r, bool round_up, int64_t *out);

// index.hip
dpc_status build_index(const int32_t *points, int64_t n, int d, int64_t T, Workspace &ws, Index &ix);
dpc_status build_priority(const int32_t *rho_sorted_or_null, const int32_t *rho_orig_or_null,
                          Workspace &ws, Index &ix);

// kdtree.hip: the balanced k-d tree over ix.n points (ix.lo/hi/height/arith
// set); fills ix.coords, ix.sidx and ix.box.
dpc_status build_kdtree(const int32_t *points, Workspace &ws, Index &ix);

// density.hip; counters (or nullptr) selects the instrumented kernel
dpc_status launch_density(const Index &ix, int64_t T, int32_t *srho, int32_t *rho_out, int64_t *counters,
                          hipStream_t s);

// dependent.hip; points whose density is below rho_min are skipped
dpc_status launch_dependent(const Index &ix, int32_t rho_min, int32_t *dep, int64_t *delta2, int64_t *counters,
                            hipStream_t s);

// cluster.hip
dpc_status launch_cluster(int64_t n, const int32_t *rho, const int32_t *dep, const int64_t *delta2,
                          int32_t rho_min, int64_t Td, bool validate, int32_t *label, Workspace &ws);

// Kernel-launch geometry helpers.
inline unsigned blocks_for(int64_t items, int per_block) {
    return static_cast<unsigned>((items + per_block - 1) / per_block);
}

}  // namespace dpc
