// Balanced k-d tree build (the split rule of Sections 3.2 and 4.2: each
// node's points are divided evenly by a hyperplane across the longest side of
// the node's box), producing the implicit layout described in
// dpc_internal.hpp: sorted coordinates, original ids and one box per node.
//
// Top levels (nodes of at least 2 * subtree-size points): all workgroups
// share a level.  Points live in structure-of-arrays form (coordinate minus
// the global minimum, as uint32, plus the id).  A node's median along its
// split axis is found exactly by most-significant-digit radix select: each
// pass histograms one digit of the points that still match the digits found
// so far (11-bit digits while a level has few nodes, 8-bit below).  The node
// is then partitioned stably: "less than the median" and "equal to the
// median" flags are scanned, and the first equal points in array order fill
// the left half.  The same pass reduces the children's boxes.
//
// Bottom levels: one workgroup owns a subtree of at most 2048 (d <= 3) or
// 1024 points and keeps it in LDS.  On each level every wavefront takes whole
// nodes: it finds the node's median by radix select over a wave-private
// histogram and computes every point's destination with a stable ballot
// scan; the workgroup then permutes the subtree through registers.  It
// writes the subtree's boxes, coordinates and ids straight into the final
// arrays.
//
// Every 2048-point tile of the top levels lies inside a single node, because
// node sizes there are multiples of the tile.
#include "dpc_internal.hpp"

#include <limits>

namespace dpc {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kTile = 2048;
constexpr int kItems = kTile / kThreads;    // 8
constexpr int kWaveItems = kItems * kWave;  // 512

template <int BITS>
struct Digit {
    static constexpr int kBits = BITS;
    static constexpr int kBins = 1 << BITS;
    static constexpr int kPerThread = kBins / kThreads;
    static_assert(kPerThread >= 1, "at least one bin per thread");
};

template <int D>
struct Bottom {
    // points per bottom subtree: what fits in LDS next to the scratch arrays
    static constexpr int kSize = D <= 3 ? 2048 : 1024;
    static constexpr int kLevels = D <= 3 ? 6 : 5;    // log2(kSize / kLeafSize)
    static constexpr int kNodes = kSize / kLeafSize;  // most nodes on one level
    static_assert((kLeafSize << kLevels) == kSize, "subtree size");
};

struct Origin {
    int32_t v[kMaxDim];  // global coordinate minimum per axis
};

struct Spans {
    uint32_t v[kMaxDim];  // max - min per axis
};

__device__ inline uint64_t lanes_below() { return (1ull << __lane_id()) - 1ull; }

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

__device__ inline uint32_t block_incl_scan(uint32_t v, uint32_t *s_w) {
    const int w = threadIdx.x / kWave;
    const uint32_t x = wave_incl_scan(v);
    if (__lane_id() == kWave - 1)
        s_w[w] = x;
    __syncthreads();
    uint32_t add = 0;
    for (int q = 0; q < w; ++q)
        add += s_w[q];
    __syncthreads();
    return x + add;
}

__device__ inline uint32_t bit_length(uint32_t x) { return x ? 32u - (uint32_t)__clz(x) : 0u; }

__device__ inline uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const uint32_t t = __shfl_xor(v, o, kWave);
        v = t < v ? t : v;
    }
    return v;
}
__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const uint32_t t = __shfl_xor(v, o, kWave);
        v = t > v ? t : v;
    }
    return v;
}

// Orders the LDS accesses of the lanes of one wavefront: everything a lane
// did before is visible to every lane of the wave after.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lanes (among `valid` ones) whose NBITS-bit digit equals this lane's.
template <int NBITS>
__device__ inline uint64_t match_digit(uint32_t dg, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < NBITS; ++b) {
        const bool bit = (dg >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// Longest side of a box given as [D][lo, hi] relative coordinates; the lowest
// axis wins a tie.
template <int D>
__device__ inline int longest_axis(const uint32_t *__restrict__ b) {
    int axis = 0;
    uint32_t widest = b[1] - b[0];
#pragma unroll
    for (int k = 1; k < D; ++k) {
        const uint32_t ext = b[2 * k + 1] - b[2 * k];
        if (ext > widest) {
            widest = ext;
            axis = k;
        }
    }
    return axis;
}

// ---------------------------------------------------------------------------
// top levels

struct NodeGeom {
    int64_t start, count, half;
};

__device__ inline NodeGeom node_geom(int64_t t, int64_t S, int64_t n) {
    NodeGeom g;
    g.start = t * S;
    const int64_t left = n - g.start;
    g.count = left < S ? left : S;
    g.half = g.count < S / 2 ? g.count : S / 2;
    return g;
}

struct NodeSelect {
    int axis;
    uint32_t base;  // the box minimum along the axis; select works on x - base
    int passes;     // digits of the axis extent
};

template <int D, int BITS>
__device__ inline NodeSelect node_select(const uint32_t *__restrict__ nbox) {
    NodeSelect s;
    s.axis = longest_axis<D>(nbox);
    s.base = nbox[2 * s.axis];
    s.passes = (int)((bit_length(nbox[2 * s.axis + 1] - s.base) + BITS - 1) / BITS);
    return s;
}

// Replays the digit choices of passes [0, upto) from their histograms: the
// digits of the median found so far (prefix), how many of the node's points
// lie below the prefix range (less), and the median's rank among the points
// matching the prefix (rank).
struct SelectState {
    uint32_t prefix, less, rank;
};

template <int BITS>
__device__ inline SelectState replay(const uint32_t *__restrict__ hist_node, int64_t pass_stride, int upto,
                                     uint32_t half, uint32_t *s_w, uint32_t *s_pick) {
    using Dg = Digit<BITS>;
    SelectState st{0u, 0u, half};
    for (int p = 0; p < upto; ++p) {
        const uint32_t *hp = hist_node + (int64_t)p * pass_stride + threadIdx.x * Dg::kPerThread;
        uint32_t c[Dg::kPerThread];
        uint32_t mine = 0;
#pragma unroll
        for (int b = 0; b < Dg::kPerThread; ++b) {
            c[b] = hp[b];
            mine += c[b];
        }
        uint32_t cum = block_incl_scan(mine, s_w) - mine;
#pragma unroll
        for (int b = 0; b < Dg::kPerThread; ++b) {
            if (cum <= st.rank && st.rank < cum + c[b]) {
                s_pick[0] = threadIdx.x * Dg::kPerThread + b;
                s_pick[1] = cum;
            }
            cum += c[b];
        }
        __syncthreads();
        const uint32_t dg = s_pick[0], below = s_pick[1];
        __syncthreads();
        st.prefix = (st.prefix << BITS) | dg;
        st.less += below;
        st.rank -= below;
    }
    return st;
}

template <int D, int BITS>
__global__ __launch_bounds__(kThreads) void k_sel_hist(const uint32_t *__restrict__ X, int64_t n, int j, int h,
                                                       const uint32_t *__restrict__ boxes, uint32_t *__restrict__ hist,
                                                       int pass) {
    using Dg = Digit<BITS>;
    __shared__ uint32_t s_h[Dg::kBins];
    __shared__ uint32_t s_w[kWaves];
    __shared__ uint32_t s_pick[2];
    const int64_t e0 = (int64_t)blockIdx.x * kTile;
    if (e0 >= n)
        return;
    const int64_t S = (int64_t)kLeafSize << (h - j);
    const int64_t t = e0 / S;
    const NodeGeom g = node_geom(t, S, n);
    const NodeSelect ns = node_select<D, BITS>(boxes + t * 2 * D);
    if (pass >= ns.passes || g.half == g.count)
        return;  // this node's median is already known (or it has no right half)
    const int64_t pass_stride = (1ll << j) * Dg::kBins;
    const SelectState st = replay<BITS>(hist + t * Dg::kBins, pass_stride, pass, (uint32_t)g.half, s_w, s_pick);
    const int shift = (ns.passes - 1 - pass) * BITS;
    for (int b = threadIdx.x; b < Dg::kBins; b += kThreads)
        s_h[b] = 0;
    __syncthreads();
    const uint32_t *x = X + (int64_t)ns.axis * n;
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t e = e0 + (int64_t)w * kWaveItems + (int64_t)r * kWave + __lane_id();
        bool match = false;
        uint32_t dg = 0;
        if (e < n) {
            const uint64_t v = (uint64_t)(x[e] - ns.base);
            match = (v >> (shift + BITS)) == (uint64_t)st.prefix;
            dg = (uint32_t)(v >> shift) & (Dg::kBins - 1);
        }
        // one LDS update per distinct digit in the wave
        const uint64_t peers = match_digit<BITS>(dg, match);
        if (match && (peers & lanes_below()) == 0)
            atomicAdd(&s_h[dg], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    for (int b = threadIdx.x; b < Dg::kBins; b += kThreads) {
        const uint32_t c = s_h[b];
        if (c)
            atomicAdd(&hist[(int64_t)pass * pass_stride + t * Dg::kBins + b], c);
    }
}

struct NodeSplit {
    uint32_t base;     // box minimum along the axis
    uint32_t median;   // relative to base
    uint32_t need_eq;  // points equal to the median that go left (the first ones in array order)
    int32_t axis;
    int32_t all_left;  // the node has no right half
};

template <typename C, int D, int BITS>
__global__ __launch_bounds__(kThreads) void k_part_count(const uint32_t *__restrict__ X, int64_t n, int j, int h,
                                                         const uint32_t *__restrict__ boxes,
                                                         uint32_t *__restrict__ child_boxes,
                                                         const uint32_t *__restrict__ hist, NodeSplit *__restrict__ split,
                                                         uint32_t *__restrict__ cnt_less, uint32_t *__restrict__ cnt_eq,
                                                         C *__restrict__ tree_box, Origin origin) {
    using Dg = Digit<BITS>;
    __shared__ uint32_t s_w[kWaves];
    __shared__ uint32_t s_pick[2];
    __shared__ uint32_t s_c[2][kWaves];
    const int64_t e0 = (int64_t)blockIdx.x * kTile;
    if (e0 >= n)
        return;
    const int64_t S = (int64_t)kLeafSize << (h - j);
    const int64_t t = e0 / S;
    const NodeGeom g = node_geom(t, S, n);
    const uint32_t *nb = boxes + t * 2 * D;
    const NodeSelect ns = node_select<D, BITS>(nb);
    const bool all_left = g.half == g.count;
    SelectState st{0u, 0u, 0u};
    if (!all_left)
        st = replay<BITS>(hist + t * Dg::kBins, (1ll << j) * Dg::kBins, ns.passes, (uint32_t)g.half, s_w, s_pick);
    // with every digit chosen, prefix is the exact median and rank its rank
    // among the points equal to it
    if (e0 == g.start && threadIdx.x == 0) {
        NodeSplit sp;
        sp.base = ns.base;
        sp.median = st.prefix;
        sp.need_eq = st.rank;
        sp.axis = ns.axis;
        sp.all_left = all_left ? 1 : 0;
        split[t] = sp;
        const int64_t v = (1ll << j) + t;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            tree_box[(v * D + k) * 2 + 0] = (C)((int64_t)origin.v[k] + (int64_t)nb[2 * k]);
            tree_box[(v * D + k) * 2 + 1] = (C)((int64_t)origin.v[k] + (int64_t)nb[2 * k + 1]);
        }
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int k = 0; k < D; ++k) {
                child_boxes[((2 * t + c) * D + k) * 2 + 0] = 0xFFFFFFFFu;
                child_boxes[((2 * t + c) * D + k) * 2 + 1] = 0u;
            }
    }
    const uint32_t *x = X + (int64_t)ns.axis * n;
    const int w = threadIdx.x / kWave;
    uint32_t nl = 0, ne = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t e = e0 + (int64_t)w * kWaveItems + (int64_t)r * kWave + __lane_id();
        bool less = false, eq = false;
        if (e < n) {
            const uint32_t v = x[e] - ns.base;
            less = all_left || v < st.prefix;
            eq = !all_left && v == st.prefix;
        }
        nl += (uint32_t)__popcll(__ballot(less));
        ne += (uint32_t)__popcll(__ballot(eq));
    }
    if (__lane_id() == 0) {
        s_c[0][w] = nl;
        s_c[1][w] = ne;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, b = 0;
        for (int q = 0; q < kWaves; ++q) {
            a += s_c[0][q];
            b += s_c[1][q];
        }
        cnt_less[blockIdx.x] = a;
        cnt_eq[blockIdx.x] = b;
    }
}

// Exclusive scans of the per-tile counts (block 0: less, block 1: equal).
__global__ __launch_bounds__(kThreads) void k_part_scan(uint32_t *__restrict__ cnt_less, uint32_t *__restrict__ cnt_eq,
                                                        int m) {
    __shared__ uint32_t s_w[kWaves];
    __shared__ uint32_t s_total;
    uint32_t *a = blockIdx.x == 0 ? cnt_less : cnt_eq;
    uint32_t carry = 0;
    for (int c = 0; c < m; c += kThreads) {
        const int i = c + threadIdx.x;
        const uint32_t v = i < m ? a[i] : 0u;
        const uint32_t incl = block_incl_scan(v, s_w);
        if (i < m)
            a[i] = carry + incl - v;
        if (threadIdx.x == kThreads - 1)
            s_total = incl;
        __syncthreads();
        carry += s_total;
        __syncthreads();
    }
}

template <int D>
__global__ __launch_bounds__(kThreads) void k_part_scatter(const uint32_t *__restrict__ Xin,
                                                           const uint32_t *__restrict__ Iin,
                                                           uint32_t *__restrict__ Xout, uint32_t *__restrict__ Iout,
                                                           int64_t n, int j, int h,
                                                           const NodeSplit *__restrict__ split,
                                                           const uint32_t *__restrict__ scan_less,
                                                           const uint32_t *__restrict__ scan_eq,
                                                           uint32_t *__restrict__ child_boxes) {
    __shared__ uint32_t s_w[2][kWaves];
    __shared__ uint32_t s_box[2][D][2];
    const int64_t e0 = (int64_t)blockIdx.x * kTile;
    if (e0 >= n)
        return;
    const int64_t S = (int64_t)kLeafSize << (h - j);
    const int64_t t = e0 / S;
    const NodeGeom g = node_geom(t, S, n);
    const NodeSplit sp = split[t];
    const int64_t tile0 = g.start / kTile;
    // points of this node before this tile that are below / equal to the median
    const uint32_t less_base = scan_less[blockIdx.x] - scan_less[tile0];
    const uint32_t eq_base = scan_eq[blockIdx.x] - scan_eq[tile0];
    if (threadIdx.x < 2 * D) {
        const int c = threadIdx.x / D, k = threadIdx.x % D;
        s_box[c][k][0] = 0xFFFFFFFFu;
        s_box[c][k][1] = 0u;
    }
    const int w = threadIdx.x / kWave;
    const uint32_t *xa = Xin + (int64_t)sp.axis * n;
    uint32_t lb[kItems], eb[kItems];
    uint32_t less_bits = 0, eq_bits = 0;
    uint32_t run_l = 0, run_e = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t e = e0 + (int64_t)w * kWaveItems + (int64_t)r * kWave + __lane_id();
        bool less = false, eq = false;
        if (e < n) {
            const uint32_t v = xa[e] - sp.base;
            less = sp.all_left || v < sp.median;
            eq = !sp.all_left && v == sp.median;
        }
        const uint64_t ml = __ballot(less), me = __ballot(eq);
        lb[r] = run_l + (uint32_t)__popcll(ml & lanes_below());
        eb[r] = run_e + (uint32_t)__popcll(me & lanes_below());
        run_l += (uint32_t)__popcll(ml);
        run_e += (uint32_t)__popcll(me);
        less_bits |= (less ? 1u : 0u) << r;
        eq_bits |= (eq ? 1u : 0u) << r;
    }
    if (__lane_id() == 0) {
        s_w[0][w] = run_l;
        s_w[1][w] = run_e;
    }
    __syncthreads();
    uint32_t off_l = less_base, off_e = eq_base;
    for (int q = 0; q < w; ++q) {
        off_l += s_w[0][q];
        off_e += s_w[1][q];
    }
    // box accumulators of the two children (l: left, r: right)
    uint32_t lmin[D], lmax[D], rmin[D], rmax[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lmin[k] = rmin[k] = 0xFFFFFFFFu;
        lmax[k] = rmax[k] = 0u;
    }
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t e = e0 + (int64_t)w * kWaveItems + (int64_t)r * kWave + __lane_id();
        if (e >= n)
            continue;
        const bool less = (less_bits >> r) & 1u, eq = (eq_bits >> r) & 1u;
        const uint32_t lbefore = off_l + lb[r];
        const uint32_t ebefore = off_e + eb[r];
        const bool left = less || (eq && ebefore < sp.need_eq);
        const uint32_t eq_left_before = ebefore < sp.need_eq ? ebefore : sp.need_eq;
        const int64_t left_before = (int64_t)lbefore + (int64_t)eq_left_before;
        const int64_t pos = e - g.start;
        const int64_t dst = left ? g.start + left_before : g.start + g.half + (pos - left_before);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const uint32_t v = Xin[(int64_t)k * n + e];
            Xout[(int64_t)k * n + dst] = v;
            if (left) {
                lmin[k] = v < lmin[k] ? v : lmin[k];
                lmax[k] = v > lmax[k] ? v : lmax[k];
            } else {
                rmin[k] = v < rmin[k] ? v : rmin[k];
                rmax[k] = v > rmax[k] ? v : rmax[k];
            }
        }
        Iout[dst] = Iin[e];
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t a = wave_min_u32(lmin[k]), b = wave_max_u32(lmax[k]);
        const uint32_t c = wave_min_u32(rmin[k]), d = wave_max_u32(rmax[k]);
        if (__lane_id() == 0) {
            if (a <= b) {
                atomicMin(&s_box[0][k][0], a);
                atomicMax(&s_box[0][k][1], b);
            }
            if (c <= d) {
                atomicMin(&s_box[1][k][0], c);
                atomicMax(&s_box[1][k][1], d);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * D) {
        const int c = threadIdx.x / D, k = threadIdx.x % D;
        if (s_box[c][k][0] <= s_box[c][k][1]) {
            atomicMin(&child_boxes[((2 * t + c) * D + k) * 2 + 0], s_box[c][k][0]);
            atomicMax(&child_boxes[((2 * t + c) * D + k) * 2 + 1], s_box[c][k][1]);
        }
    }
}

__global__ void k_fill_u32(uint32_t *__restrict__ a, int64_t m, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m)
        a[i] = v;
}

// the root's box in relative coordinates: [0, span] on every axis
template <int D>
__global__ void k_root_box(uint32_t *__restrict__ nb, Spans spans) {
    const int k = threadIdx.x;
    if (k < D) {
        nb[2 * k] = 0u;
        nb[2 * k + 1] = spans.v[k];
    }
}

template <int D>
__global__ __launch_bounds__(kThreads) void k_soa_init(const int32_t *__restrict__ P, int64_t n, Origin origin,
                                                       uint32_t *__restrict__ X, uint32_t *__restrict__ I) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
#pragma unroll
    for (int k = 0; k < D; ++k)
        X[(int64_t)k * n + i] = (uint32_t)((int64_t)P[i * D + k] - (int64_t)origin.v[k]);
    I[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// bottom levels: one workgroup per subtree, in LDS

template <typename C, int D>
__global__ __launch_bounds__(kThreads) void k_bottom(const uint32_t *__restrict__ X, const uint32_t *__restrict__ I,
                                                     int64_t n, int jb, int h, Origin origin, C *__restrict__ tree_box,
                                                     C *__restrict__ coords, int32_t *__restrict__ sidx,
                                                     uint32_t *__restrict__ leaf_org, uint32_t *__restrict__ leaf_ext,
                                                     uint32_t *__restrict__ leaf_pack) {
    constexpr int M = Bottom<D>::kSize;
    constexpr int NB = Bottom<D>::kNodes;
    constexpr int PER = M / kThreads;
    constexpr int kB = 8;  // digit bits of the in-LDS select
    constexpr int kNB = 1 << kB;
    constexpr int kLaneBins = kNB / kWave;  // 4
    __shared__ uint32_t s_x[D][M];
    __shared__ uint32_t s_id[M];
    __shared__ uint16_t s_dst[M];
    __shared__ uint32_t s_hist[kWaves][kNB];
    __shared__ uint32_t s_box[NB][D][2];

    const int64_t S0 = (int64_t)kLeafSize << (h - jb);  // at most M
    const int64_t s0 = (int64_t)blockIdx.x * S0;
    if (s0 >= n)
        return;
    const int cnt0 = (int)(n - s0 < S0 ? n - s0 : S0);
    for (int i = threadIdx.x; i < cnt0; i += kThreads) {
#pragma unroll
        for (int k = 0; k < D; ++k)
            s_x[k][i] = X[(int64_t)k * n + s0 + i];
        s_id[i] = I[s0 + i];
    }
    const int w = threadIdx.x / kWave;
    const int lane = __lane_id();
    for (int l = jb; l <= h; ++l) {
        const int S = kLeafSize << (h - l);  // node size on this level
        const int nsub = (cnt0 + S - 1) / S;
        for (int u = threadIdx.x; u < nsub; u += kThreads)
#pragma unroll
            for (int k = 0; k < D; ++k) {
                s_box[u][k][0] = 0xFFFFFFFFu;
                s_box[u][k][1] = 0u;
            }
        __syncthreads();
        // boxes: every 32-point group lies inside one node (S >= 32)
        for (int base = w * kWave; base < cnt0; base += kThreads) {
            const int i = base + lane;
            const bool have = i < cnt0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                uint32_t a = have ? s_x[k][i] : 0xFFFFFFFFu;
                uint32_t b = have ? s_x[k][i] : 0u;
#pragma unroll
                for (int o = kLeafSize / 2; o > 0; o >>= 1) {
                    const uint32_t ta = __shfl_xor(a, o, kWave), tb = __shfl_xor(b, o, kWave);
                    a = ta < a ? ta : a;
                    b = tb > b ? tb : b;
                }
                if ((i & (kLeafSize - 1)) == 0 && have) {
                    atomicMin(&s_box[i / S][k][0], a);
                    atomicMax(&s_box[i / S][k][1], b);
                }
            }
        }
        __syncthreads();
        for (int u = threadIdx.x; u < nsub; u += kThreads) {
            const int64_t v = (1ll << l) + s0 / S + u;
            uint32_t ext = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                tree_box[(v * D + k) * 2 + 0] = (C)((int64_t)origin.v[k] + (int64_t)s_box[u][k][0]);
                tree_box[(v * D + k) * 2 + 1] = (C)((int64_t)origin.v[k] + (int64_t)s_box[u][k][1]);
                const uint32_t e = s_box[u][k][1] - s_box[u][k][0];
                ext = e > ext ? e : ext;
            }
            if (l == h) {
                // leaf record: corner (relative to the global minimum) and widest extent
                const int64_t c = s0 / kLeafSize + u;
#pragma unroll
                for (int k = 0; k < D; ++k)
                    leaf_org[c * D + k] = s_box[u][k][0];
                leaf_ext[c] = ext;
            }
        }
        if (l == h)
            break;
        // each wave splits whole nodes: exact median, then stable destinations
        for (int u = w; u < nsub; u += kWaves) {
            const int base = u * S;
            const int cnt = cnt0 - base < S ? cnt0 - base : S;
            const int half = cnt < S / 2 ? cnt : S / 2;
            if (half == cnt) {
                for (int i = lane; i < cnt; i += kWave)
                    s_dst[base + i] = (uint16_t)(base + i);
                continue;
            }
            const int a = longest_axis<D>(&s_box[u][0][0]);
            const uint32_t lo = s_box[u][a][0];
            const int passes = (int)((bit_length(s_box[u][a][1] - lo) + kB - 1) / kB);
            uint32_t prefix = 0, rank = (uint32_t)half;
            for (int p = 0; p < passes; ++p) {
                const int shift = (passes - 1 - p) * kB;
                // The histogram is shared by the lanes of this wave: every
                // access is atomic and the phases are fenced at wavefront
                // scope, so no lane's own store can stand in for what the
                // other lanes added.
#pragma unroll
                for (int b = 0; b < kLaneBins; ++b)
                    __hip_atomic_store(&s_hist[w][lane * kLaneBins + b], 0u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WAVEFRONT);
                wave_sync();
                for (int i = lane; i < cnt; i += kWave) {
                    const uint64_t v = (uint64_t)(s_x[a][base + i] - lo);
                    if ((v >> (shift + kB)) == (uint64_t)prefix)
                        __hip_atomic_fetch_add(&s_hist[w][(uint32_t)(v >> shift) & (kNB - 1)], 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WAVEFRONT);
                }
                wave_sync();
                // lane owns bins [4*lane, 4*lane + 4)
                uint32_t c[kLaneBins];
                uint32_t mine = 0;
#pragma unroll
                for (int b = 0; b < kLaneBins; ++b) {
                    c[b] = __hip_atomic_load(&s_hist[w][lane * kLaneBins + b], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WAVEFRONT);
                    mine += c[b];
                }
                wave_sync();
                uint32_t cum = wave_incl_scan(mine) - mine;
                uint32_t pick = 0, below = 0;
                bool found = false;
#pragma unroll
                for (int b = 0; b < kLaneBins; ++b) {
                    if (cum <= rank && rank < cum + c[b]) {
                        pick = (uint32_t)(lane * kLaneBins + b);
                        below = cum;
                        found = true;
                    }
                    cum += c[b];
                }
                const uint64_t fm = __ballot(found);
                const int src = __ffsll((unsigned long long)fm) - 1;
                pick = (uint32_t)__builtin_amdgcn_readlane((int)pick, src);
                below = (uint32_t)__builtin_amdgcn_readlane((int)below, src);
                prefix = (prefix << kB) | pick;
                rank -= below;
            }
            const uint32_t median = prefix, need_eq = rank;
            uint32_t run_l = 0, run_e = 0;
            for (int i0 = 0; i0 < cnt; i0 += kWave) {
                const int i = i0 + lane;
                const bool valid = i < cnt;
                uint32_t v = 0;
                if (valid)
                    v = s_x[a][base + i] - lo;
                const bool less = valid && v < median;
                const bool eq = valid && v == median;
                const uint64_t ml = __ballot(less), me = __ballot(eq);
                const uint32_t lbefore = run_l + (uint32_t)__popcll(ml & lanes_below());
                const uint32_t ebefore = run_e + (uint32_t)__popcll(me & lanes_below());
                run_l += (uint32_t)__popcll(ml);
                run_e += (uint32_t)__popcll(me);
                if (valid) {
                    const bool left = less || (eq && ebefore < need_eq);
                    const uint32_t left_before = lbefore + (ebefore < need_eq ? ebefore : need_eq);
                    const uint32_t dst = left ? left_before : (uint32_t)half + ((uint32_t)i - left_before);
                    s_dst[base + i] = (uint16_t)(base + dst);
                }
            }
        }
        __syncthreads();
        // apply the permutation through registers
        uint32_t tx[PER][D], tid[PER];
        uint32_t td[PER];
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int i = r * kThreads + threadIdx.x;
            if (i < cnt0) {
#pragma unroll
                for (int k = 0; k < D; ++k)
                    tx[r][k] = s_x[k][i];
                tid[r] = s_id[i];
                td[r] = s_dst[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int i = r * kThreads + threadIdx.x;
            if (i < cnt0) {
#pragma unroll
                for (int k = 0; k < D; ++k)
                    s_x[k][td[r]] = tx[r][k];
                s_id[td[r]] = tid[r];
            }
        }
        __syncthreads();
    }
    __syncthreads();
    constexpr int W = (D + 1) / 2;
    for (int i = threadIdx.x; i < cnt0; i += kThreads) {
#pragma unroll
        for (int k = 0; k < D; ++k)
            coords[(s0 + i) * D + k] = (C)((int64_t)origin.v[k] + (int64_t)s_x[k][i]);
        sidx[s0 + i] = (int32_t)s_id[i];
        // offsets from the leaf corner, two 16-bit halves per word (read only
        // for leaves narrow enough that every offset fits)
        const int u = i / kLeafSize;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint32_t a = s_x[2 * w][i] - s_box[u][2 * w][0];
            const uint32_t b = 2 * w + 1 < D ? s_x[2 * w + 1][i] - s_box[u][2 * w + 1][0] : 0u;
            leaf_pack[(s0 + i) * W + w] = (a & 0xFFFFu) | (b << 16);
        }
    }
}

// Digit width of a top level: 11 bits while the level has at most 256 nodes
// (fewer passes), 8 bits below (small histograms for many nodes).
constexpr int kWideLevels = 8;

inline int level_bits(int j) { return j <= kWideLevels ? 11 : 8; }

template <typename C, int D, int BITS>
void launch_level(const uint32_t *Xin, const uint32_t *Iin, uint32_t *Xout, uint32_t *Iout, int64_t n, int j, int h,
                  int passes, const uint32_t *bj, uint32_t *bj1, uint32_t *hj, NodeSplit *split, uint32_t *cnt_less,
                  uint32_t *cnt_eq, C *box, Origin origin, unsigned grid, unsigned tiles, hipStream_t s) {
    for (int p = 0; p < passes; ++p)
        hipLaunchKernelGGL((k_sel_hist<D, BITS>), dim3(grid), dim3(kThreads), 0, s, Xin, n, j, h, bj, hj, p);
    hipLaunchKernelGGL((k_part_count<C, D, BITS>), dim3(grid), dim3(kThreads), 0, s, Xin, n, j, h, bj, bj1, hj, split,
                       cnt_less, cnt_eq, box, origin);
    hipLaunchKernelGGL(k_part_scan, dim3(2), dim3(kThreads), 0, s, cnt_less, cnt_eq, (int)tiles);
    hipLaunchKernelGGL((k_part_scatter<D>), dim3(grid), dim3(kThreads), 0, s, Xin, Iin, Xout, Iout, n, j, h, split,
                       cnt_less, cnt_eq, bj1);
}

template <typename C, int D>
dpc_status build_kd(const int32_t *points, Workspace &ws, Index &ix) {
    hipStream_t s = ws.stream;
    const int64_t n = ix.n;
    const int h = ix.height;
    const int jb = h > Bottom<D>::kLevels ? h - Bottom<D>::kLevels : 0;  // first bottom level
    Origin origin{};
    Spans spans{};
    uint32_t widest = 0;
    for (int k = 0; k < D; ++k) {
        origin.v[k] = ix.lo[k];
        spans.v[k] = (uint32_t)((int64_t)ix.hi[k] - (int64_t)ix.lo[k]);
        widest = spans.v[k] > widest ? spans.v[k] : widest;
    }
    C *coords, *box;
    DPC_TRY(ws.alloc(&coords, (size_t)n * D));
    DPC_TRY(ws.alloc(&box, (size_t)2 * ix.n_leaves * 2 * D));
    DPC_TRY(ws.alloc(&ix.sidx, n));
    DPC_TRY(ws.alloc(&ix.leaf_org, (size_t)ix.n_leaves * D));
    DPC_TRY(ws.alloc(&ix.leaf_ext, (size_t)ix.n_leaves));
    DPC_TRY(ws.alloc(&ix.leaf_pack, (size_t)n * ((D + 1) / 2)));
    ix.coords = coords;
    ix.box = box;

    uint32_t *XA, *XB, *IA, *IB;
    DPC_TRY(ws.alloc(&XA, (size_t)D * n));
    DPC_TRY(ws.alloc(&IA, n));
    hipLaunchKernelGGL((k_soa_init<D>), dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, points, n, origin, XA,
                       IA);
    DPC_HIP(hipGetLastError());
    if (jb > 0) {
        DPC_TRY(ws.alloc(&XB, (size_t)D * n));
        DPC_TRY(ws.alloc(&IB, n));
        const int64_t tiles = (n + kTile - 1) / kTile;
        const int wbits = widest ? 32 - __builtin_clz(widest) : 0;
        // histogram words of every top level: passes x nodes x bins
        int64_t hist_off[64];
        int64_t hist_words = 0;
        for (int j = 0; j < jb; ++j) {
            const int bits = level_bits(j);
            hist_off[j] = hist_words;
            hist_words += (int64_t)((wbits + bits - 1) / bits) * (1ll << j) * (1ll << bits);
        }
        uint32_t *nboxes, *hist, *cnt_less, *cnt_eq;
        NodeSplit *split;
        DPC_TRY(ws.alloc(&nboxes, (size_t)(2ll << jb) * 2 * D));
        DPC_TRY(ws.alloc(&hist, (size_t)(hist_words > 0 ? hist_words : 1)));
        DPC_TRY(ws.alloc(&split, (size_t)1 << (jb - 1)));
        DPC_TRY(ws.alloc(&cnt_less, (size_t)tiles));
        DPC_TRY(ws.alloc(&cnt_eq, (size_t)tiles));
        if (hist_words > 0)
            hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(hist_words, kThreads)), dim3(kThreads), 0, s, hist,
                               hist_words, 0u);
        hipLaunchKernelGGL((k_root_box<D>), dim3(1), dim3(kWave), 0, s, nboxes + 2 * D, spans);
        const unsigned grid = (unsigned)tiles;
        uint32_t *Xin = XA, *Xout = XB, *Iin = IA, *Iout = IB;
        for (int j = 0; j < jb; ++j) {
            const uint32_t *bj = nboxes + (1ll << j) * 2 * D;  // level j boxes start at heap index 2^j
            uint32_t *bj1 = nboxes + (2ll << j) * 2 * D;
            const int bits = level_bits(j);
            const int passes = (wbits + bits - 1) / bits;
            if (bits == 11)
                launch_level<C, D, 11>(Xin, Iin, Xout, Iout, n, j, h, passes, bj, bj1, hist + hist_off[j], split,
                                       cnt_less, cnt_eq, box, origin, grid, (unsigned)tiles, s);
            else
                launch_level<C, D, 8>(Xin, Iin, Xout, Iout, n, j, h, passes, bj, bj1, hist + hist_off[j], split,
                                      cnt_less, cnt_eq, box, origin, grid, (unsigned)tiles, s);
            DPC_HIP(hipGetLastError());
            uint32_t *t = Xin;
            Xin = Xout;
            Xout = t;
            t = Iin;
            Iin = Iout;
            Iout = t;
        }
        XA = Xin;
        IA = Iin;
    }
    hipLaunchKernelGGL((k_bottom<C, D>), dim3((unsigned)(1ll << jb)), dim3(kThreads), 0, s, XA, IA, n, jb, h, origin,
                       box, coords, ix.sidx, ix.leaf_org, ix.leaf_ext, ix.leaf_pack);
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

}  // namespace

dpc_status build_kdtree(const int32_t *points, Workspace &ws, Index &ix) {
    const bool f64 = ix.arith == Arith::F64;
    switch (ix.d) {
#define DPC_KD_CASE(DD) \
    case DD:            \
        return f64 ? build_kd<double, DD>(points, ws, ix) : build_kd<int64_t, DD>(points, ws, ix);
        DPC_KD_CASE(1)
        DPC_KD_CASE(2)
        DPC_KD_CASE(3)
        DPC_KD_CASE(4)
        DPC_KD_CASE(5)
        DPC_KD_CASE(6)
        DPC_KD_CASE(7)
        DPC_KD_CASE(8)
#undef DPC_KD_CASE
    default:
        return DPC_ERR_INVALID_ARG;
    }
}

}  // namespace dpc
