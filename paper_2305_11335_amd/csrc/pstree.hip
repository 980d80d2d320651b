// Dependent points through the priority-search k-d tree as Section 4.2
// defines it (the third dependent-point backend): every node stores the
// point of highest priority among the points of its subtree, and the other
// points of the subtree are split in two across the longest side of their
// box, one part per child.  The stored points thus form a heap in priority
// order.  The query is the priority nearest-neighbour search of Section
// 4.2.2 (Algorithm 1): a subtree whose stored point does not rank above the
// query holds no candidate and is pruned, as is one whose box is farther
// than the best distance so far; every other visited node's stored point is
// a candidate.  Results equal the other backends' (Definitions 2-3 fix
// them); equal distances go to the smaller index.
//
// Layout.  Node v (heap numbering: root 1, children 2v and 2v + 1) exists for
// v <= n, so every level is full but the last, which fills from the left;
// subtree sizes and the place of each subtree's points in a level's array
// follow from n alone (sub_size, seg_start).  The split is by rank: the left
// child takes the first sub_size(2v) of the remaining points in order along
// the axis (ties by position), the right child the rest.
//
// Build, one level at a time.  The points of all subtrees rooted at depth l
// lie in one array, subtree after subtree in node order, each point
// carrying its node.  Per level: (1) each node's highest key and bounding
// box (one workgroup, wavefront or thread per node, by subtree size); (2)
// a sort key per point: node, whether it is the node's stored point, and its
// coordinate along the node's longest side; (3) a stable radix sort; (4) each
// node's stored point goes to the node's slot, and every other point moves to
// its child's subtree in the next level's array (the stored point sorts last
// in its subtree, so a point's place there is its sorted place minus the
// stored points of the subtrees before it).
#include "dpc_internal.hpp"

#include <limits>
#include <utility>

namespace dpc {
namespace {

constexpr int kThreads = 256;

// Tree shape: n nodes; h is the depth of node n.
struct Shape {
    int64_t n;
    int h;
};

// Nodes in the subtree of node v at depth l.
__host__ __device__ inline int64_t sub_size(const Shape &s, int64_t v, int l) {
    const int64_t K = 1ll << (s.h - l);
    int64_t last = s.n - v * K + 1;  // its nodes on the last level
    last = last < 0 ? 0 : (last > K ? K : last);
    return K - 1 + last;
}

// First slot of node v's subtree (v at depth l) in level l's array.
__host__ __device__ inline int64_t seg_start(const Shape &s, int64_t v, int l) {
    const int64_t i = v - (1ll << l), K = 1ll << (s.h - l);
    const int64_t L = s.n + 1 - (1ll << s.h);  // nodes on the last level
    return i * (K - 1) + (i * K < L ? i * K : L);
}

// A level's points (structure of arrays): original index, priority key,
// coordinates relative to the minimum corner, node.
struct Level {
    uint32_t *idx;
    uint64_t *key;
    uint32_t *x;  // [D][cap]
    uint32_t *node;
};

// The tree (indexed by node, 1 .. n): stored point, its key (the subtree's
// highest), its original index, and the subtree's bounding box.
struct Tree {
    uint32_t *pt;   // [node][D]
    uint64_t *key;
    uint32_t *idx;
    uint32_t *box;  // [node][D][2]
};

// The minimum corner (a kernel argument).
struct Corner {
    int32_t v[kMaxDim];
};

__global__ __launch_bounds__(kThreads) void k_pst_init(const int32_t *__restrict__ points, int d, Corner lo,
                                                       const int32_t *__restrict__ rho, int64_t n, int64_t cap,
                                                       Level L0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    L0.idx[i] = (uint32_t)i;
    L0.key[i] = pack_key(rho[i], (int32_t)i);
    for (int k = 0; k < d; ++k)
        L0.x[(int64_t)k * cap + i] = (uint32_t)((int64_t)points[i * d + k] - (int64_t)lo.v[k]);
    L0.node[i] = 1u;
}

// Highest key and box of node v from its points [s, s + m) of the level
// array, accumulated by `lanes` cooperating threads (lane t takes every
// lanes-th point).
template <int D>
__device__ inline void node_scan(const Level &A, int64_t cap, int64_t s, int64_t m, int t, int lanes, uint64_t &kmax,
                                 uint32_t (&mn)[D], uint32_t (&mx)[D]) {
    kmax = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        mn[k] = 0xFFFFFFFFu;
        mx[k] = 0u;
    }
    for (int64_t p = s + t; p < s + m; p += lanes) {
        const uint64_t kk = A.key[p];
        kmax = kk > kmax ? kk : kmax;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const uint32_t v = A.x[(int64_t)k * cap + p];
            mn[k] = v < mn[k] ? v : mn[k];
            mx[k] = v > mx[k] ? v : mx[k];
        }
    }
}

template <int D>
__device__ inline void store_node(const Tree &T, int64_t v, uint64_t kmax, const uint32_t (&mn)[D],
                                  const uint32_t (&mx)[D]) {
    T.key[v] = kmax;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        T.box[(v * D + k) * 2 + 0] = mn[k];
        T.box[(v * D + k) * 2 + 1] = mx[k];
    }
}

// Step (1) for the nodes of depth l whose subtrees are small.  MODE 1: one
// wavefront per node; 2: one thread per node.
template <int D, int MODE>
__global__ __launch_bounds__(kThreads) void k_pst_reduce(Level A, int64_t cap, Shape sh, int l, Tree T) {
    const int64_t first = 1ll << l;
    const int64_t count = (l == sh.h ? sh.n + 1 : 2 * first) - first;
    if constexpr (MODE == 1) {
        const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
        if (i >= count)
            return;
        const int64_t v = first + i;
        uint64_t kmax;
        uint32_t mn[D], mx[D];
        node_scan<D>(A, cap, seg_start(sh, v, l), sub_size(sh, v, l), __lane_id(), kWave, kmax, mn, mx);
        kmax = group_max_u64<6>(kmax);
#pragma unroll
        for (int k = 0; k < D; ++k)
            group_min_max<6>(mn[k], mx[k]);
        if (__lane_id() == kWave - 1)
            store_node<D>(T, v, kmax, mn, mx);
    } else {
        const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (i >= count)
            return;
        const int64_t v = first + i;
        uint64_t kmax;
        uint32_t mn[D], mx[D];
        node_scan<D>(A, cap, seg_start(sh, v, l), sub_size(sh, v, l), 0, 1, kmax, mn, mx);
        store_node<D>(T, v, kmax, mn, mx);
    }
}

// Step (1) for depths whose subtrees are large: each wavefront reduces one
// chunk of kChunk consecutive points of one node (a node's points are
// consecutive in the level's array, so chunks never straddle two), with the
// cross-lane steps done by DPP moves, into one partial per chunk; then one
// wavefront per node combines the node's partials.  cpn chunks per node
// (enough for the largest subtree of the depth; chunks past a smaller
// subtree's end are empty).
constexpr int kChunk = 1024;

template <int D>
struct Partial {
    uint64_t key;
    uint32_t mn[D], mx[D];
};

template <int D>
__global__ __launch_bounds__(kThreads) void k_pst_part(Level A, int64_t cap, Shape sh, int l, int64_t cpn,
                                                       Partial<D> *__restrict__ part) {
    const int64_t first = 1ll << l;
    const int64_t count = (l == sh.h ? sh.n + 1 : 2 * first) - first;
    const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;  // wave-uniform
    if (g >= count * cpn)
        return;
    const int64_t v = first + g / cpn;
    const int64_t s0 = seg_start(sh, v, l), m = sub_size(sh, v, l);
    const int64_t b = (g % cpn) * kChunk;
    const int64_t e = b + kChunk < m ? b + kChunk : m;
    uint64_t kmax = 0;
    uint32_t mn[D], mx[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        mn[k] = 0xFFFFFFFFu;
        mx[k] = 0u;
    }
    for (int64_t p = s0 + b + __lane_id(); p < s0 + e; p += kWave) {
        const uint64_t kk = A.key[p];
        kmax = kk > kmax ? kk : kmax;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const uint32_t x = A.x[(int64_t)k * cap + p];
            mn[k] = x < mn[k] ? x : mn[k];
            mx[k] = x > mx[k] ? x : mx[k];
        }
    }
    kmax = group_max_u64<6>(kmax);
#pragma unroll
    for (int k = 0; k < D; ++k)
        group_min_max<6>(mn[k], mx[k]);
    if (__lane_id() == kWave - 1) {
        Partial<D> r;
        r.key = kmax;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            r.mn[k] = mn[k];
            r.mx[k] = mx[k];
        }
        part[g] = r;
    }
}

template <int D>
__global__ __launch_bounds__(kThreads) void k_pst_combine(Shape sh, int l, int64_t cpn,
                                                          const Partial<D> *__restrict__ part, Tree T) {
    const int64_t first = 1ll << l;
    const int64_t count = (l == sh.h ? sh.n + 1 : 2 * first) - first;
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;  // wave-uniform
    if (i >= count)
        return;
    uint64_t kmax = 0;
    uint32_t mn[D], mx[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        mn[k] = 0xFFFFFFFFu;
        mx[k] = 0u;
    }
    for (int64_t c = __lane_id(); c < cpn; c += kWave) {
        const Partial<D> &r = part[i * cpn + c];
        kmax = r.key > kmax ? r.key : kmax;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            mn[k] = r.mn[k] < mn[k] ? r.mn[k] : mn[k];
            mx[k] = r.mx[k] > mx[k] ? r.mx[k] : mx[k];
        }
    }
    kmax = group_max_u64<6>(kmax);
#pragma unroll
    for (int k = 0; k < D; ++k)
        group_min_max<6>(mn[k], mx[k]);
    if (__lane_id() == kWave - 1)
        store_node<D>(T, first + i, kmax, mn, mx);
}

// Longest side of node v's box (the lowest axis on a tie).
template <int D>
__device__ inline int longest(const Tree &T, int64_t v) {
    int axis = 0;
    uint32_t widest = T.box[(v * D) * 2 + 1] - T.box[(v * D) * 2];
#pragma unroll
    for (int k = 1; k < D; ++k) {
        const uint32_t e = T.box[(v * D + k) * 2 + 1] - T.box[(v * D + k) * 2];
        if (e > widest) {
            widest = e;
            axis = k;
        }
    }
    return axis;
}

// Step (2): sort key = node offset within the level, then 1 for the node's
// stored point, then the coordinate along the node's longest side.
template <int D>
__global__ __launch_bounds__(kThreads) void k_pst_keys(Level A, int64_t cap, int64_t m, int l, int wbits, Tree T,
                                                       uint64_t *__restrict__ skey, uint32_t *__restrict__ sval) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m)
        return;
    const int64_t v = A.node[p];
    const int axis = longest<D>(T, v);
    const uint64_t stored = A.key[p] == T.key[v] ? 1ull : 0ull;
    skey[p] = ((uint64_t)(v - (1ll << l)) << (wbits + 1)) | (stored << wbits) | (uint64_t)A.x[(int64_t)axis * cap + p];
    sval[p] = (uint32_t)p;
}

// Step (4): the stored points to their nodes, the others to their child's
// subtree in the next level's array.
template <int D>
__global__ __launch_bounds__(kThreads) void k_pst_move(Level A, Level B, int64_t cap, int64_t m, Shape sh, int l,
                                                       int wbits, const uint64_t *__restrict__ skey,
                                                       const uint32_t *__restrict__ sval, Tree T) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m)
        return;
    const uint64_t sk = skey[q];
    const int64_t p = sval[q];
    const int64_t i = (int64_t)(sk >> (wbits + 1));
    const int64_t v = (1ll << l) + i;
    if ((sk >> wbits) & 1ull) {
        T.idx[v] = A.idx[p];
#pragma unroll
        for (int k = 0; k < D; ++k)
            T.pt[v * D + k] = A.x[(int64_t)k * cap + p];
        return;
    }
    const int64_t r = q - seg_start(sh, v, l);
    const int64_t child = 2 * v + (r >= sub_size(sh, 2 * v, l + 1) ? 1 : 0);
    const int64_t dst = q - i;
    B.idx[dst] = A.idx[p];
    B.key[dst] = A.key[p];
#pragma unroll
    for (int k = 0; k < D; ++k)
        B.x[(int64_t)k * cap + dst] = A.x[(int64_t)k * cap + p];
    B.node[dst] = (uint32_t)child;
}

// The last level: every subtree is a single point, the node's own.
template <int D>
__global__ __launch_bounds__(kThreads) void k_pst_last(Level A, int64_t cap, Shape sh, Tree T) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t first = 1ll << sh.h;
    if (p >= sh.n + 1 - first)
        return;
    const int64_t v = A.node[p];
    T.idx[v] = A.idx[p];
    T.key[v] = A.key[p];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t c = A.x[(int64_t)k * cap + p];
        T.pt[v * D + k] = c;
        T.box[(v * D + k) * 2 + 0] = c;
        T.box[(v * D + k) * 2 + 1] = c;
    }
}

template <int D>
__device__ inline uint64_t box_gap2(const uint32_t (&x)[D], const uint32_t *__restrict__ b) {
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint64_t g = x[k] < b[2 * k] ? b[2 * k] - x[k] : (x[k] > b[2 * k + 1] ? x[k] - b[2 * k + 1] : 0u);
        s += g * g;
    }
    return s;
}

// The priority nearest-neighbour query of every stored point (one thread
// per node, in heap order: neighbouring threads of the deep levels query
// neighbouring points).  Depth-first, the nearer child first; a node is
// skipped when its stored key (the subtree's highest) does not rank above the
// query, or when its box is farther than the best so far (a node at exactly
// the best distance is still visited: it may hold an equally near smaller
// index).  Squared distances are exact in 64 bits (the range check bounds
// their sum).
template <int D>
__global__ __launch_bounds__(kThreads) void k_pst_query(Shape sh, Tree T, int32_t rho_min, int32_t rho_max,
                                                        int32_t *__restrict__ dep, int64_t *__restrict__ delta2) {
    const int64_t u = 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u > sh.n)
        return;
    const uint64_t kq = T.key[u];
    const int32_t rho_q = (int32_t)((uint32_t)(kq >> 32) ^ 0x80000000u);
    const uint32_t o = T.idx[u];
    if (rho_q < rho_min || rho_q > rho_max) {
        dep[o] = -1;
        delta2[o] = std::numeric_limits<int64_t>::max();
        return;
    }
    uint32_t x[D];
#pragma unroll
    for (int k = 0; k < D; ++k)
        x[k] = T.pt[u * D + k];
    uint64_t best = ~0ull;
    uint32_t best_low = 0;  // low key word of the best point; 0 = none yet
    constexpr int kStack = 2 * 40;
    uint32_t stack[kStack];
    int sp = 0;
    stack[sp++] = 1u;
    while (sp > 0) {
        const int64_t v = stack[--sp];
        const uint64_t kv = T.key[v];
        if (kv <= kq)
            continue;
        if (box_gap2<D>(x, T.box + v * 2 * D) > best)
            continue;
        uint64_t s = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const uint32_t c = T.pt[v * D + k];
            const uint64_t g = x[k] > c ? x[k] - c : c - x[k];
            s += g * g;
        }
        const uint32_t low = (uint32_t)kv;
        if (s < best || (s == best && low > best_low)) {
            best = s;
            best_low = low;
        }
        const int64_t c0 = 2 * v;
        if (c0 > sh.n)
            continue;
        if (c0 + 1 > sh.n) {
            stack[sp++] = (uint32_t)c0;
            continue;
        }
        const uint64_t g0 = box_gap2<D>(x, T.box + c0 * 2 * D), g1 = box_gap2<D>(x, T.box + (c0 + 1) * 2 * D);
        // the farther child goes on the stack first, so the nearer one is searched first
        stack[sp++] = (uint32_t)(g0 <= g1 ? c0 + 1 : c0);
        stack[sp++] = (uint32_t)(g0 <= g1 ? c0 : c0 + 1);
    }
    dep[o] = best_low != 0 ? (int32_t)(0xFFFFFFFFu - best_low) : -1;
    delta2[o] = best_low != 0 ? (int64_t)best : std::numeric_limits<int64_t>::max();
}

int bit_length(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

template <int D>
dpc_status pst_typed(const Job &J, Workspace &ws) {
    hipStream_t s = ws.stream;
    const int64_t n = J.n;
    Shape sh{n, bit_length((uint64_t)n) - 1};
    uint32_t widest = 0;
    for (int k = 0; k < D; ++k) {
        const uint32_t e = (uint32_t)((int64_t)J.hi[k] - (int64_t)J.lo[k]);
        widest = e > widest ? e : widest;
    }
    const int wbits = bit_length(widest) > 0 ? bit_length(widest) : 1;
    const int64_t cap = n;
    Level A{}, B{};
    Tree T{};
    DPC_TRY(ws.alloc(&A.idx, (size_t)cap));
    DPC_TRY(ws.alloc(&A.key, (size_t)cap));
    DPC_TRY(ws.alloc(&A.x, (size_t)cap * D));
    DPC_TRY(ws.alloc(&A.node, (size_t)cap));
    DPC_TRY(ws.alloc(&B.idx, (size_t)cap));
    DPC_TRY(ws.alloc(&B.key, (size_t)cap));
    DPC_TRY(ws.alloc(&B.x, (size_t)cap * D));
    DPC_TRY(ws.alloc(&B.node, (size_t)cap));
    DPC_TRY(ws.alloc(&T.pt, (size_t)(n + 1) * D));
    DPC_TRY(ws.alloc(&T.key, (size_t)(n + 1)));
    DPC_TRY(ws.alloc(&T.idx, (size_t)(n + 1)));
    DPC_TRY(ws.alloc(&T.box, (size_t)(n + 1) * 2 * D));
    uint64_t *ka, *kb;
    uint32_t *va, *vb;
    DPC_TRY(ws.alloc(&ka, (size_t)cap));
    DPC_TRY(ws.alloc(&kb, (size_t)cap));
    DPC_TRY(ws.alloc(&va, (size_t)cap));
    DPC_TRY(ws.alloc(&vb, (size_t)cap));
    // chunk partials of the depths with large subtrees: nodes x chunks per
    // node at each such depth (the launches below index exactly that many)
    int64_t part_entries = 1;
    for (int l = 0; l < sh.h; ++l) {
        const int64_t seg = sub_size(sh, 1ll << l, l);
        if (seg >= 4096) {
            const int64_t need = (1ll << l) * ((seg + kChunk - 1) / kChunk);
            part_entries = need > part_entries ? need : part_entries;
        }
    }
    Partial<D> *part;
    DPC_TRY(ws.alloc(&part, (size_t)part_entries));
    Corner lo{};
    for (int k = 0; k < kMaxDim; ++k)
        lo.v[k] = J.lo[k];
    launch(k_pst_init, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, J.points, D, lo, (const int32_t *)J.rho,
           n, cap, A);
    for (int l = 0; l < sh.h; ++l) {
        const int64_t m = n - ((1ll << l) - 1);
        const int64_t nodes = 1ll << l;
        const int64_t seg = sub_size(sh, 1ll << l, l);  // the largest subtree of this depth
        if (seg >= 4096) {
            const int64_t cpn = (seg + kChunk - 1) / kChunk;
            launch((k_pst_part<D>), dim3(blocks_for(nodes * cpn * kWave, kThreads)), dim3(kThreads), 0, s, A, cap,
                   sh, l, cpn, part);
            launch((k_pst_combine<D>), dim3(blocks_for(nodes * kWave, kThreads)), dim3(kThreads), 0, s, sh, l, cpn,
                   (const Partial<D> *)part, T);
        } else if (seg >= 64)
            launch((k_pst_reduce<D, 1>), dim3(blocks_for(nodes * kWave, kThreads)), dim3(kThreads), 0, s, A, cap,
                   sh, l, T);
        else
            launch((k_pst_reduce<D, 2>), dim3(blocks_for(nodes, kThreads)), dim3(kThreads), 0, s, A, cap, sh, l, T);
        launch((k_pst_keys<D>), dim3(blocks_for(m, kThreads)), dim3(kThreads), 0, s, A, cap, m, l, wbits, T, ka, va);
        uint64_t *ks;
        uint32_t *vs;
        DPC_TRY(radix_sort_pairs<uint64_t>(ka, va, kb, vb, m, l + 1 + wbits, ws, &ks, &vs));
        launch((k_pst_move<D>), dim3(blocks_for(m, kThreads)), dim3(kThreads), 0, s, A, B, cap, m, sh, l, wbits,
               (const uint64_t *)ks, (const uint32_t *)vs, T);
        DPC_HIP(hipGetLastError());
        std::swap(A, B);
    }
    launch((k_pst_last<D>), dim3(blocks_for(n + 1 - (1ll << sh.h), kThreads)), dim3(kThreads), 0, s, A, cap, sh, T);
    launch((k_pst_query<D>), dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, sh, T, J.dep_rho_min,
           J.dep_rho_max, J.dep, J.delta2);
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

}  // namespace

dpc_status pst_dependent(const Job &J, int d, Workspace &ws) {
    if (J.n <= 0)
        return DPC_OK;
    switch (d) {
#define DPC_PST_CASE(DD) \
    case DD:             \
        return pst_typed<DD>(J, ws);
        DPC_PST_CASE(1)
        DPC_PST_CASE(2)
        DPC_PST_CASE(3)
        DPC_PST_CASE(4)
        DPC_PST_CASE(5)
        DPC_PST_CASE(6)
        DPC_PST_CASE(7)
        DPC_PST_CASE(8)
#undef DPC_PST_CASE
    default:
        return DPC_ERR_INVALID_ARG;
    }
}

}  // namespace dpc
