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
//
// Every kernel works on a group of instances (independent clustering
// problems) that share the dimension and the arithmetic: a single call is a
// group of one.  The instances' arrays are concatenated; instance i's points
// occupy positions [P_i, P_i + n_i) of the group's point arrays with P_i a
// multiple of kTile, so that every tile of kTile positions, and every
// workgroup or wavefront of consecutive positions, belongs to one instance.
// Positions are instance-local inside the kernels (array pointers are offset
// by P_i), and so are node and leaf numbers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <limits>
#include <vector>

#include "../../include/libdpc.h"

namespace dpc {

constexpr int kWave = 64;
constexpr int kMaxDim = 8;
constexpr int kMaxLeaf = 64;   // most points per tree leaf (a group's leaves hold 16, 32 or 64)
constexpr int kMinLeafLog2 = 4;
constexpr int kMaxLeafLog2 = 6;
constexpr int kTile = 2048;    // positions per tile (the unit of the top-level build passes)

// A DPP lane move (dpp_ctrl CTRL) within the rows selected by ROWS: each
// lane of those rows takes v from its source lane; other lanes, and lanes
// whose source lies outside their row, return keep.  DPP moves run on the
// vector ALU, where __shfl_* goes through the LDS crossbar.
template <int CTRL, int ROWS>
__device__ inline uint32_t dpp_move(uint32_t v, uint32_t keep) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)keep, (int)v, CTRL, ROWS, 0xF, false);
}

// Minimum and maximum over groups of 2^G consecutive lanes (G = 4, 5 or 6)
// with DPP lane moves, which run on the vector ALU instead of the LDS
// crossbar: pairs and quads within a quad, then the mirrored halves of each
// 8- and 16-lane row; rows then pass their last lane's value on (row 1 from
// row 0, row 3 from row 2, then rows 2 and 3 from lane 31).  The result is in
// every lane of a 16-lane group and in the last lane of a 32- or 64-lane one.
template <int G>
__device__ inline void group_min_max(uint32_t &mn, uint32_t &mx) {
    static_assert(G >= 4 && G <= 6, "groups of 16, 32 or 64 lanes");
    uint32_t t;
#define DPC_MINMAX_STEP(CTRL, ROWS)                                      \
    t = dpp_move<CTRL, ROWS>(mn, 0xFFFFFFFFu);                           \
    mn = t < mn ? t : mn;                                                \
    t = dpp_move<CTRL, ROWS>(mx, 0u);                                    \
    mx = t > mx ? t : mx;
    DPC_MINMAX_STEP(0xB1, 0xF)   // quad_perm [1,0,3,2]
    DPC_MINMAX_STEP(0x4E, 0xF)   // quad_perm [2,3,0,1]
    DPC_MINMAX_STEP(0x141, 0xF)  // row_half_mirror
    DPC_MINMAX_STEP(0x140, 0xF)  // row_mirror
    if constexpr (G >= 5) {
        DPC_MINMAX_STEP(0x142, 0xA)  // row_bcast:15 into rows 1 and 3
    }
    if constexpr (G >= 6) {
        DPC_MINMAX_STEP(0x143, 0xC)  // row_bcast:31 into rows 2 and 3
    }
#undef DPC_MINMAX_STEP
}

// One step of group_max_u64: v against the value DPP move CTRL brings in.
template <int CTRL, int ROWS>
__device__ inline uint64_t max_step_u64(uint64_t v) {
    const uint32_t lo = dpp_move<CTRL, ROWS>((uint32_t)v, 0u), hi = dpp_move<CTRL, ROWS>((uint32_t)(v >> 32), 0u);
    const uint64_t o = ((uint64_t)hi << 32) | lo;
    return o > v ? o : v;
}

// Maximum over groups of 2^G lanes (G = 4: every lane of a 16-lane row holds
// it; G = 5 or 6: the last lane of each 32-lane half, or of the wave), with
// the same DPP steps as group_min_max.
template <int G>
__device__ inline uint64_t group_max_u64(uint64_t v) {
    static_assert(G >= 4 && G <= 6, "groups of 16, 32 or 64 lanes");
    v = max_step_u64<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v = max_step_u64<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v = max_step_u64<0x141, 0xF>(v);  // row_half_mirror
    v = max_step_u64<0x140, 0xF>(v);  // row_mirror
    if constexpr (G >= 5)
        v = max_step_u64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    if constexpr (G >= 6)
        v = max_step_u64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Digit width of the radix select of top build level j (whose 2^j nodes each
// keep one histogram of 2^bits counts per pass): 11 bits while a level has
// at most 256 nodes, 10 up to 4096 nodes (two passes for coordinates of up to
// 20 bits), 8 below (small histograms for many nodes).
__host__ __device__ inline int top_level_bits(int j) { return j <= 8 ? 11 : (j <= 12 ? 10 : 8); }

// Top levels whose nodes hold at most 2^kOwnLog2 points are split by one
// workgroup per node, which keeps its histograms in LDS; the shared
// histograms exist for the levels above only.
constexpr int kOwnLog2 = 15;

// First top level of an instance split one workgroup per node (at most jb,
// its first level built in LDS).
__host__ __device__ inline int top_owned_from(int height, int lsh, int jb) {
    const int f = height + lsh - kOwnLog2;
    return f < 0 ? 0 : (f > jb ? jb : f);
}

// Coordinates and squared distances are exact in double when every squared
// distance stays below 2^53 (the "f64" path); otherwise 64-bit integers.
enum class Arith { F64, I64 };

// One instance as the kernels see it (device memory).
struct Inst {
    int64_t n;         // points
    int64_t P;         // first position in the group's point arrays (a multiple of kTile)
    int64_t N;         // first node in the group's node arrays (2 * n_leaves nodes)
    int64_t L;         // first leaf in the group's leaf arrays (n_leaves leaves)
    int64_t H;         // first word of the instance's top-level histograms
    int64_t S;         // first entry of its per-node select records (2^(jb-1))
    int64_t B;         // first word of its top-level relative boxes (2^(jb+1) nodes)
    int32_t height;    // 2^height leaves
    int32_t lsh;       // log2 of the points per leaf (4 or 5, the same for a whole group)
    int32_t jb;        // first level built in LDS (the top levels are 0 .. jb-1)
    int32_t wbits;     // bits of the widest coordinate span
    int32_t lo[kMaxDim];
    uint32_t span[kMaxDim];
    // density: the threshold, r = floor(sqrt(T)), and the clamped integer
    // parameters of the narrow-leaf and integer-box comparisons
    int64_t T;
    int64_t r;
    int32_t M, R, limit, Tn;
    // dependent points and labels
    int32_t dep_rho_min;  // dependents of points below it are skipped
    int32_t dep_rho_max;  // and of points above it
    int32_t rho_min;
    int64_t Td;
    // caller's arrays (input order)
    const int32_t *points;
    int32_t *rho;
    int32_t *dep;
    int64_t *delta2;
    int32_t *label;
};

// Host view of one instance before planning.
struct Job {
    const int32_t *points = nullptr;
    int64_t n = 0;
    int64_t T = 0;          // density threshold (unused by dpc_dependent)
    int32_t dep_rho_min = 0;
    int32_t dep_rho_max = std::numeric_limits<int32_t>::max();
    int32_t rho_min = 0;
    int64_t Td = 0;
    int32_t *rho = nullptr;
    int32_t *dep = nullptr;
    int64_t *delta2 = nullptr;
    int32_t *label = nullptr;
    // set by the bounds pass
    int32_t lo[kMaxDim] = {0};
    int32_t hi[kMaxDim] = {0};
};

// A group of instances and its device arrays (owned by a Workspace).
struct Index {
    int d = 0;
    Arith arith = Arith::F64;
    int lsh = kMaxLeafLog2;     // log2 of the points per leaf
    bool intbox = false;        // every instance can use the clamped integer comparisons
    int count = 0;              // instances
    std::vector<Inst> host;     // descriptors (host copy)
    Inst *inst = nullptr;       // descriptors (device)
    // Instance of each tile (nullptr when the group has one instance).
    uint32_t *tile_inst = nullptr;
    int64_t positions = 0;      // padded positions of all instances (a multiple of kTile)
    int64_t nodes = 0;          // node slots of all instances
    int64_t leaves = 0;         // leaf slots of all instances
    int max_height = 0;
    int max_jb = 0;
    int max_wbits = 0;
    // device arrays (owned by the workspace), indexed by position, node or leaf
    void *coords = nullptr;     // sorted coordinates [pos][d], double or int64
    int32_t *sidx = nullptr;    // instance-local original index of each sorted position
    void *box = nullptr;        // node boxes [node][d][2] (min, max), like coords
    uint32_t *rbox = nullptr;   // the same boxes relative to the instance's lo, as uint32
    uint64_t *skey = nullptr;   // priority key of each sorted position
    uint64_t *maxkey = nullptr; // per-node maximum key
    // Split of each internal node: axis << 32 | median offset from lo along
    // that axis (points below go left).  Only a hint for the order in which
    // children are searched.
    uint64_t *split = nullptr;
    // Leaf records: the leaf box's lower corner relative to lo [leaf][d], its
    // widest side [leaf], and every point's offsets from that corner as
    // 16-bit halves, two axes per word [pos][(d+1)/2] (meaningful only when
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
// A call's workspace holds at most kCap allocations (the workspace bound
// counts on it); a plan's, which keeps every call it records, is unlimited.
// Given a reserve (a bound on what the call will take), the first
// allocation takes that much from the pool at once and later ones are carved
// from it: one pool allocation and one free per call instead of one per
// array (each costs tens of microseconds of host time).  Anything beyond the
// reserve is allocated on its own.
//
// A workspace over an external buffer (the allocation-free entry point's
// scratch) carves every array from that buffer and never touches the pool:
// a request beyond it fails with DPC_ERR_OOM.
struct Workspace {
    hipStream_t stream;
    static constexpr int kCap = 160;
    std::vector<void *> ptrs;  // pool allocations, released together
    int count = 0;             // arrays handed out
    int cap = kCap;
    size_t bytes = 0;  // handed out so far, each array rounded up to 256 bytes
    size_t reserve = 0;
    char *chunk = nullptr;  // the reserve, once allocated
    size_t used = 0;        // bytes of the reserve handed out
    hipMemPool_t pool = nullptr;
    bool external = false;  // chunk is a caller's buffer of `reserve` bytes
    explicit Workspace(hipStream_t s, size_t reserve_bytes = 0)
        : stream(s), reserve(reserve_bytes), pool(workspace_pool()) {
        ptrs.reserve(8);
    }
    // buffer: device memory of buffer_bytes (a multiple of 256), 256-byte aligned
    Workspace(hipStream_t s, void *buffer, size_t buffer_bytes)
        : stream(s), reserve(buffer_bytes), chunk(static_cast<char *>(buffer)), external(true) {}
    ~Workspace() { release(); }
    void *pool_alloc(size_t b) {
        void *p = nullptr;
        const hipError_t e = pool ? hipMallocFromPoolAsync(&p, b, pool, stream) : hipMallocAsync(&p, b, stream);
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        ptrs.push_back(p);
        return p;
    }
    template <class T>
    dpc_status alloc(T **out, size_t elems) {
        *out = nullptr;
        if (count >= cap)
            return DPC_ERR_OOM;
        const size_t want = bytes_rounded(elems * sizeof(T));
        void *p = nullptr;
        if (external) {
            if (want > reserve - used)
                return DPC_ERR_OOM;
            *out = reinterpret_cast<T *>(chunk + used);
            used += want;
            ++count;
            bytes += want;
            return DPC_OK;
        }
        if (reserve > 0 && chunk == nullptr) {
            chunk = static_cast<char *>(pool_alloc(bytes_rounded(reserve)));
            if (chunk == nullptr)
                reserve = 0;  // fall back to one allocation per array
        }
        if (chunk != nullptr && used + want <= bytes_rounded(reserve)) {
            p = chunk + used;
            used += want;
        } else {
            p = pool_alloc(want);
            if (p == nullptr)
                return DPC_ERR_OOM;
        }
        ++count;
        bytes += want;
        *out = static_cast<T *>(p);
        return DPC_OK;
    }
    void release() {
        for (void *p : ptrs)
            (void)hipFreeAsync(p, stream);
        ptrs.clear();
        count = 0;
        used = 0;
        if (!external)
            chunk = nullptr;
    }
    static size_t bytes_rounded(size_t b) { return ((b == 0 ? 256 : b) + 255) & ~(size_t)255; }
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

// A caller's array named in a descriptor, as a global-memory pointer (the
// compiler cannot tell the address space of a pointer loaded from memory,
// and would otherwise emit flat accesses).
template <typename T>
__device__ inline __attribute__((address_space(1))) T *global_ptr(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

// The instance that owns a tile, and the instance-local position of the
// tile's first element.
// Priority keys: the high word is rho with its sign bit flipped (so unsigned
// order is signed order), the low word 2^32 - 1 - original index.  A larger
// key means higher density, or equal density and a lower index: the priority
// (rho, -index).  No real key is 0, which marks padding.
__host__ __device__ inline uint64_t pack_key(int32_t rho, int32_t orig) {
    return ((uint64_t)((uint32_t)rho ^ 0x80000000u) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)orig);
}

__device__ inline const Inst &inst_of_tile(const Inst *__restrict__ inst, const uint32_t *__restrict__ tile_inst,
                                           int64_t tile) {
    return inst[tile_inst ? tile_inst[tile] : 0u];
}

// The density threshold T of an instance and the clamped integer parameters
// derived from it (M, R, limit: limit < 0 when the integer comparisons do
// not apply).
void density_params(Inst &I, int64_t T, int d);

// Upper bound on the workspace bytes (as Workspace::bytes counts them) of one
// instance of n points in d dimensions, alone or as part of a group: a
// group's workspace is at most the sum of its instances' bounds.
uint64_t workspace_bound(int64_t n, int d);

// Exact thresholds (host).
dpc_status square_threshold(double r, bool round_up, int64_t *out);

// floor(sqrt(v)) for v >= 0 (host)
int64_t isqrt64(int64_t v);

// index.hip
// Bounds of every job (one read-back for all), then the range check and
// the arithmetic of each.  Fails with DPC_ERR_RANGE if one is out of range
// (bad[] then marks which, if given).
dpc_status job_bounds(std::vector<Job> &jobs, int d, Workspace &ws, std::vector<int> *bad);
Arith job_arith(const Job &j, int d);
// Plans a group (descriptors, offsets, tile table), allocates its arrays and
// builds every instance's tree with 2^lsh points per leaf.
dpc_status build_group(const std::vector<Job> &jobs, int d, Arith arith, int lsh, Workspace &ws, Index &ix);
// The leaf size used for groups of dimension d (log2; a tuning choice that
// never changes results) and its setter.
int leaf_log2(int d);
void set_leaf_log2(int d, int lsh);
// Priority keys and per-node maxima; rho in sorted order (srho) or in each
// instance's input order (rho_orig: use the instances' rho arrays).
dpc_status build_priority(const int32_t *srho, bool rho_orig, Workspace &ws, Index &ix);
// The per-node maximum keys above the leaf maxima already in ix.maxkey.
dpc_status priority_levels(Index &ix, hipStream_t s);
// Dependent points of one instance through a Fenwick tree of k-d trees
// (Section 5, Algorithm 2), from the rho array the job holds (input order);
// writes the job's dep and delta2.  Results equal launch_dependent's.
dpc_status fenwick_dependent(const Job &J, int d, Arith arith, int lsh, Workspace &ws);

// radix.hip: stable sort of n (key, value) pairs by key bits [0, bits),
// ascending, ping-ponging between (keys, vals) and (keys_alt, vals_alt);
// *keys_out / *vals_out receive whichever pair holds the result.  Takes its
// histograms from ws.  K is uint32_t or uint64_t.
template <typename K>
dpc_status radix_sort_pairs(K *keys, uint32_t *vals, K *keys_alt, uint32_t *vals_alt, int64_t n, int bits,
                            Workspace &ws, K **keys_out, uint32_t **vals_out);

// Dependent points of one instance through the priority-search k-d tree of
// Section 4.2 (one point stored per node), from the rho array the job holds
// (input order); writes the job's dep and delta2.  Results equal
// launch_dependent's.
dpc_status pst_dependent(const Job &J, int d, Workspace &ws);

// Allocates the group's descriptors (and tile table) and copies them to the
// device (synchronising the stream).
dpc_status upload_group(Workspace &ws, Index &ix);

// kdtree.hip: the balanced k-d trees of the group's instances (descriptors
// planned); allocates the group's arrays, uploads the descriptors and fills
// coords, sidx, box, rbox, split and the leaf records.
dpc_status build_kdtree(Workspace &ws, Index &ix);

// density.hip; srho: sorted-order densities (position-indexed); counters (or
// nullptr) selects the instrumented kernel
dpc_status launch_density(const Index &ix, int32_t *srho, int64_t *counters, hipStream_t s);

// dependent.hip
dpc_status launch_dependent(const Index &ix, int64_t *counters, hipStream_t s);

// cluster.hip: labels of a single instance from arrays in input order
dpc_status launch_cluster(int64_t n, const int32_t *rho, const int32_t *dep, const int64_t *delta2,
                          int32_t rho_min, int64_t Td, bool validate, int32_t *label, Workspace &ws);
// labels of every instance of a group (the edges come from its own outputs)
dpc_status launch_group_labels(const Index &ix, Workspace &ws);
// labels of one instance for count parameter pairs (rows of label), with
// every followed edge checked
dpc_status launch_cluster_sweep(int64_t n, const int32_t *rho, const int32_t *dep, const int64_t *delta2, int count,
                                const int32_t *rho_mins, const int64_t *Tds, int32_t *label, Workspace &ws);

// api.hip: every step for a list of instances, each with its own flags (0 or
// DPC_SKIP_NOISE_DEPENDENTS); sets each record's status and returns the first
// failure.  peak_bytes (optional) receives the largest workspace held at once.
dpc_status run_instances(dpc_instance *instances, const uint32_t *flags, int count, hipStream_t stream,
                         size_t *peak_bytes,
                         Workspace *persist = nullptr);

// The argument checks of dpc_run for one instance (host only).
dpc_status check_instance(const dpc_instance &q, uint32_t flags);

// Kernel launches.  Every launch of the method goes through launch(), which
// also appends it (kernel, geometry and argument values) to the calling
// thread's record when one is active: a plan (dpc_plan_create) records its
// first run and later replays the same launches, with no host work, or
// captures them into a HIP graph.
using LaunchRecord = std::vector<std::function<void(hipStream_t)>>;
extern thread_local LaunchRecord *t_record;
// While a plan records: the device word its replays set to DPC_ERR_RANGE when
// the points no longer lie inside the bounds the plan was made for (else 0).
extern thread_local int32_t *t_plan_status;

template <typename... KArgs, typename... Args>
inline void launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t shmem, hipStream_t s, Args... args) {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
    if (t_record)
        t_record->push_back(
            [=](hipStream_t st) { hipLaunchKernelGGL(kernel, grid, block, shmem, st, args...); });
}

// Kernel-launch geometry helpers.
inline unsigned blocks_for(int64_t items, int per_block) {
    return static_cast<unsigned>((items + per_block - 1) / per_block);
}

}  // namespace dpc
