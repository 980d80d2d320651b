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
// so far (11-bit digits while a level has few nodes, 10-bit and then 8-bit
// below), and the workgroup whose tiles complete a node's histogram picks the
// node's digit.
// The node is then partitioned stably: "less than the median" and "equal to
// the median" flags are counted per tile and scanned, and the first equal
// points in array order fill the left half.  The same pass reduces the
// children's boxes.
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
// node sizes there are multiples of the tile, and inside a single instance of
// the group; each kernel finds its instance from its tile.
#include "dpc_internal.hpp"

#include <algorithm>
#include <limits>

namespace dpc {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
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
    static constexpr int kNodes = kSize >> kMinLeafLog2;  // most nodes on one level
};

__device__ inline uint64_t lanes_below() { return (1ull << __lane_id()) - 1ull; }

// Inclusive prefix sum across the wave with DPP lane moves: a doubling scan
// within each 16-lane row (lanes before the row's start bring in 0), then
// each row adds the total of the rows before it by row broadcasts.
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    v += dpp_move<0x111, 0xF>(v, 0u);  // row_shr:1
    v += dpp_move<0x112, 0xF>(v, 0u);  // row_shr:2
    v += dpp_move<0x114, 0xF>(v, 0u);  // row_shr:4
    v += dpp_move<0x118, 0xF>(v, 0u);  // row_shr:8
    v += dpp_move<0x142, 0xA>(v, 0u);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xC>(v, 0u);  // row_bcast:31 into rows 2 and 3
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

// The kItems values of one wave's items (positions base + r * 64 + lane),
// loaded without branches so that all loads are in flight together; items
// past the end read the last element instead and must be ignored.
__device__ inline void load_items(const uint32_t *__restrict__ a, int64_t n, int64_t base, uint32_t (&out)[kItems]) {
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t e = base + (int64_t)r * kWave + __lane_id();
        out[r] = a[e < n ? e : n - 1];
    }
}

// Orders the LDS accesses of the lanes of one wavefront: everything a lane
// did before is visible to every lane of the wave after.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

__host__ __device__ inline int level_bits(int j) { return top_level_bits(j); }

// Words of an instance's histograms of levels [0, j): passes x nodes x bins.
__host__ __device__ inline int64_t hist_words_below(int j, int wbits) {
    int64_t w = 0;
    for (int l = 0; l < j; ++l) {
        const int bits = level_bits(l);
        w += (int64_t)((wbits + bits - 1) / bits) * (1ll << l) * (1ll << bits);
    }
    return w;
}

// A tile of the top-level passes at level j: its instance and the
// instance-local geometry of the tile and of its node.
struct TopTile {
    const Inst *I;
    int64_t e0;     // instance-local first position
    int64_t t;      // the node's index within level j
    int64_t tile0;  // group tile of the node's first position
    NodeGeom g;
};

// False when the tile has no work at level j (padding, or an instance whose
// level j is built in LDS or split one workgroup per node).
__device__ inline bool top_tile(const Inst *__restrict__ inst, const uint32_t *__restrict__ tile_inst, int64_t tile,
                                int j, TopTile &tt) {
    const Inst &I = inst_of_tile(inst, tile_inst, tile);
    if (j >= top_owned_from(I.height, I.lsh, I.jb))
        return false;
    const int64_t first = I.P / kTile;
    tt.e0 = (tile - first) * kTile;
    if (tt.e0 >= I.n)
        return false;
    tt.I = &I;
    const int64_t S = 1ll << (I.height - j + I.lsh);
    tt.t = tt.e0 / S;
    tt.g = node_geom(tt.t, S, I.n);
    tt.tile0 = first + tt.g.start / kTile;
    return true;
}

// A node of level j, for the kernels with one workgroup per node: from the
// group's node table, or node blockIdx.x of the single instance.
__device__ inline bool top_node(const Inst *__restrict__ inst, const uint2 *__restrict__ node_tab, int j,
                                TopTile &tt) {
    const uint2 e = node_tab ? node_tab[blockIdx.x] : make_uint2(0u, blockIdx.x);
    const Inst &I = inst[e.x];
    if (j >= top_owned_from(I.height, I.lsh, I.jb))
        return false;
    const int64_t S = 1ll << (I.height - j + I.lsh);
    tt.t = e.y;
    if (tt.t * S >= I.n)
        return false;
    tt.I = &I;
    tt.g = node_geom(tt.t, S, I.n);
    tt.e0 = tt.g.start;
    tt.tile0 = I.P / kTile + tt.g.start / kTile;
    return true;
}

// Per-instance pieces of the group's top-level work arrays.
struct TopArrays {
    uint32_t *X;          // [d][positions] coordinates relative to lo (this pass's input)
    int64_t positions;
    uint32_t *nboxes;     // relative node boxes of the top levels
    uint32_t *hist;
    void *state;          // SelectState records
    void *split;          // NodeSplit records
};

struct NodeSelect {
    int axis;
    uint32_t base;  // the box minimum along the axis; select works on x - base
    int bits;       // bits of the axis extent
    int passes;     // digits of the axis extent
};

template <int D, int BITS>
__device__ inline NodeSelect node_select(const uint32_t *__restrict__ nbox) {
    NodeSelect s;
    s.axis = longest_axis<D>(nbox);
    s.base = nbox[2 * s.axis];
    s.bits = (int)bit_length(nbox[2 * s.axis + 1] - s.base);
    s.passes = (s.bits + BITS - 1) / BITS;
    return s;
}

// Bits [lo, hi) of x - base form the digit of a select pass: the passes take
// BITS bits each from the top, and the last one the few that remain.  (The
// first passes, which see every point, thus spread them over all bins; a
// short digit, whose few bins would collect every point, is left for the
// last pass, which only sees the points that matched the prefix.)
__host__ __device__ inline void digit_bits(int bits, int pass, int width, int &lo, int &hi) {
    hi = bits - pass * width;
    lo = hi > width ? hi - width : 0;
}

// State of a node's radix select after some passes: the digits of the
// median found so far (prefix), how many of the node's points lie below the
// prefix range (less), the median's rank among the points matching the
// prefix (rank) and how many points match it (match); and the count of the
// node's tiles whose histogram additions of the current pass are issued
// (arrive, cleared by the pick).
struct SelectState {
    uint32_t prefix, less, rank, match;
    uint32_t arrive;
};

// Bound on the polls of a wait for other workgroups' atomics (each poll
// sleeps briefly): far beyond any real wait, it only keeps a wait from
// running forever.
constexpr uint32_t kMaxPolls = 1u << 16;

__device__ inline uint32_t load_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Chooses the digit of one pass from the node's finished histogram (all
// threads of the block take part).  Other workgroups completed the
// histogram with relaxed device-scope atomics, which this reads with
// relaxed device-scope loads (they reach the point where those atomics are
// performed, without flushing any cache): the counts are read again until
// they add up to the node's matching points, so every addition is in.
template <int BITS>
__device__ inline void pick_digit(const uint32_t *__restrict__ hp, int width, SelectState &st, uint32_t *s_w,
                                  uint32_t *s_pick) {
    using Dg = Digit<BITS>;
    uint32_t c[Dg::kPerThread];
    uint32_t mine = 0, cum = 0;
    for (uint32_t polls = 0;; ++polls) {
        mine = 0;
#pragma unroll
        for (int b = 0; b < Dg::kPerThread; ++b) {
            c[b] = load_agent(hp + threadIdx.x * Dg::kPerThread + b);
            mine += c[b];
        }
        cum = block_incl_scan(mine, s_w);
        if (threadIdx.x == kThreads - 1)
            s_pick[0] = cum;
        __syncthreads();
        const uint32_t total = s_pick[0];
        __syncthreads();
        if (total == st.match || polls >= kMaxPolls)
            break;
        __builtin_amdgcn_s_sleep(2);
    }
    cum -= mine;
#pragma unroll
    for (int b = 0; b < Dg::kPerThread; ++b) {
        if (cum <= st.rank && st.rank < cum + c[b]) {
            s_pick[0] = threadIdx.x * Dg::kPerThread + b;
            s_pick[1] = cum;
            s_pick[2] = c[b];
        }
        cum += c[b];
    }
    __syncthreads();
    const uint32_t dg = s_pick[0], below = s_pick[1], count = s_pick[2];
    __syncthreads();
    st.prefix = (st.prefix << width) | dg;
    st.less += below;
    st.rank -= below;
    st.match = count;
}

// One pass of the radix select of every node of level j: each workgroup
// histograms the digit of the points of `tiles` consecutive tiles (all in one
// node) that still match the node's prefix, then adds its histogram to the
// node's; the workgroup whose tiles complete the node's histogram chooses the
// digit and stores the node's state for the next pass.  Several tiles per
// workgroup keep the number of global additions to one bin low on the first
// levels, where every workgroup works on one of very few nodes.
template <int D, int BITS>
__global__ __launch_bounds__(kThreads) void k_sel_hist(const Inst *__restrict__ inst,
                                                       const uint32_t *__restrict__ tile_inst,
                                                       const uint32_t *__restrict__ blocks, int per, TopArrays A,
                                                       int j, int pass) {
    using Dg = Digit<BITS>;
    __shared__ uint32_t s_h[Dg::kBins];
    __shared__ uint32_t s_w[kWaves];
    __shared__ uint32_t s_pick[3];
    __shared__ uint32_t s_last;
    // this workgroup's tiles: from the table (a group), or `per` at a time
    int64_t tile;
    int tiles;
    if (blocks) {
        tile = blocks[blockIdx.x] >> 4;
        tiles = (int)(blocks[blockIdx.x] & 15u) + 1;
    } else {
        tile = (int64_t)blockIdx.x * per;
        tiles = per;
    }
    TopTile tt;
    if (!top_tile(inst, tile_inst, tile, j, tt))
        return;
    const Inst &I = *tt.I;
    const int64_t n = I.n;
    const uint32_t *nbox = A.nboxes + I.B + tt.t * 2 * D + (1ll << j) * 2 * D;
    const NodeSelect ns = node_select<D, BITS>(nbox);
    if (pass >= ns.passes || tt.g.half == tt.g.count)
        return;  // this node's median is already known (or it has no right half)
    SelectState *state = static_cast<SelectState *>(A.state) + I.S;
    SelectState st = {0u, 0u, (uint32_t)tt.g.half, (uint32_t)tt.g.count, 0u};
    if (pass > 0) {
        st.prefix = load_agent(&state[tt.t].prefix);
        st.less = load_agent(&state[tt.t].less);
        st.rank = load_agent(&state[tt.t].rank);
        st.match = load_agent(&state[tt.t].match);
    }
    int lo, hi;
    digit_bits(ns.bits, pass, BITS, lo, hi);
    const uint32_t dmask = (1u << (hi - lo)) - 1u;
    for (int b = threadIdx.x; b < Dg::kBins; b += kThreads)
        s_h[b] = 0;
    __syncthreads();
    const uint32_t *x = A.X + (int64_t)ns.axis * A.positions + I.P;
    const int w = threadIdx.x / kWave;
    uint32_t done_tiles = 0;
    // the next tile's values are loaded before this tile's are counted, so
    // two tiles' loads are in flight at once
    uint32_t xn[kItems];
    load_items(x, n, tt.e0 + (int64_t)w * kWaveItems, xn);
    for (int q = 0; q < tiles; ++q) {
        const int64_t e0 = tt.e0 + (int64_t)q * kTile;
        if (e0 >= n)
            break;
        ++done_tiles;
        uint32_t xv[kItems];
#pragma unroll
        for (int r = 0; r < kItems; ++r)
            xv[r] = xn[r];
        if (q + 1 < tiles && e0 + kTile < n)
            load_items(x, n, e0 + kTile + (int64_t)w * kWaveItems, xn);
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const int64_t e = e0 + (int64_t)w * kWaveItems + (int64_t)r * kWave + __lane_id();
            const uint64_t v = (uint64_t)(xv[r] - ns.base);
            const bool match = e < n && (v >> hi) == (uint64_t)st.prefix;
            const uint32_t dg = (uint32_t)(v >> lo) & dmask;
            // clustered points often share one digit across the wave: one
            // addition then serves them all
            const uint64_t mm = __ballot(match);
            const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)dg);
            if (__ballot(match && dg != d0) == 0) {
                if (mm != 0 && __lane_id() == 0)
                    atomicAdd(&s_h[d0], (uint32_t)__popcll(mm));
            } else if (match) {
                atomicAdd(&s_h[dg], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t *hp = A.hist + I.H + hist_words_below(j, I.wbits) + (int64_t)pass * (1ll << j) * Dg::kBins +
                   tt.t * Dg::kBins;
    for (int b = threadIdx.x; b < Dg::kBins; b += kThreads) {
        const uint32_t c = s_h[b];
        if (c)
            atomicAdd(&hp[b], c);
    }
    // every tile of the node is counted once; the workgroup whose tiles
    // complete the count picks the digit
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t node_tiles = (uint32_t)((tt.g.count + kTile - 1) / kTile);
        const uint32_t before = __hip_atomic_fetch_add(&state[tt.t].arrive, done_tiles, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
        s_last = before + done_tiles == node_tiles ? 1u : 0u;
    }
    __syncthreads();
    if (s_last == 0)
        return;
    pick_digit<BITS>(hp, hi - lo, st, s_w, s_pick);
    if (threadIdx.x == 0) {
        __hip_atomic_store(&state[tt.t].prefix, st.prefix, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&state[tt.t].less, st.less, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&state[tt.t].rank, st.rank, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&state[tt.t].match, st.match, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&state[tt.t].arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

struct NodeSplit {
    uint32_t base;     // box minimum along the axis
    uint32_t median;   // relative to base
    uint32_t need_eq;  // points equal to the median that go left (the first ones in array order)
    int32_t axis;
    int32_t all_left;  // the node has no right half
};

// Per-tile counts of points below and equal to their node's median (the
// workgroup of a node's first tile also records the node's split and box).
template <typename C, int D, int BITS>
__global__ __launch_bounds__(kThreads) void k_part_count(const Inst *__restrict__ inst,
                                                         const uint32_t *__restrict__ tile_inst, TopArrays A, int j,
                                                         uint32_t *__restrict__ cnt_less, uint32_t *__restrict__ cnt_eq,
                                                         C *__restrict__ tree_box, uint32_t *__restrict__ rel_box,
                                                         uint64_t *__restrict__ split_hint) {
    __shared__ uint32_t s_c[2][kWaves];
    TopTile tt;
    if (!top_tile(inst, tile_inst, blockIdx.x, j, tt))
        return;
    const Inst &I = *tt.I;
    const int64_t n = I.n;
    const NodeGeom g = tt.g;
    const uint32_t *nb = A.nboxes + I.B + ((1ll << j) + tt.t) * 2 * D;
    const NodeSelect ns = node_select<D, BITS>(nb);
    const bool all_left = g.half == g.count;
    SelectState st = {0u, 0u, (uint32_t)g.half, 0u, 0u};
    if (!all_left && ns.passes > 0) {
        const SelectState *state = static_cast<const SelectState *>(A.state) + I.S;
        st.prefix = load_agent(&state[tt.t].prefix);
        st.rank = load_agent(&state[tt.t].rank);
    }
    // with every digit chosen, prefix is the exact median and rank its rank
    // among the points equal to it
    if (tt.e0 == g.start && threadIdx.x == 0) {
        NodeSplit sp;
        sp.base = ns.base;
        sp.median = st.prefix;
        sp.need_eq = st.rank;
        sp.axis = ns.axis;
        sp.all_left = all_left ? 1 : 0;
        (static_cast<NodeSplit *>(A.split) + I.S)[tt.t] = sp;
        const int64_t v = (1ll << j) + tt.t;
        split_hint[I.N + v] = ((uint64_t)(uint32_t)sp.axis << 32) | (uint64_t)(sp.base + sp.median);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            tree_box[((I.N + v) * D + k) * 2 + 0] = (C)((int64_t)I.lo[k] + (int64_t)nb[2 * k]);
            tree_box[((I.N + v) * D + k) * 2 + 1] = (C)((int64_t)I.lo[k] + (int64_t)nb[2 * k + 1]);
            rel_box[((I.N + v) * D + k) * 2 + 0] = nb[2 * k];
            rel_box[((I.N + v) * D + k) * 2 + 1] = nb[2 * k + 1];
        }
    }
    const uint32_t *x = A.X + (int64_t)ns.axis * A.positions + I.P;
    const int w = threadIdx.x / kWave;
    uint32_t xv[kItems];
    load_items(x, n, tt.e0 + (int64_t)w * kWaveItems, xv);
    uint32_t nl = 0, ne = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t e = tt.e0 + (int64_t)w * kWaveItems + (int64_t)r * kWave + __lane_id();
        const uint32_t v = xv[r] - ns.base;
        const bool less = e < n && (all_left || v < st.prefix);
        const bool eq = e < n && !all_left && v == st.prefix;
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

// Exclusive scans of the per-tile counts (block 0: less, block 1: equal):
// each thread sums a contiguous run of tiles, one block scan, then each
// thread writes its run's prefixes.  Tiles without work at this level hold
// stale counts; they cancel, because a tile only ever subtracts the prefix at
// its own node's first tile.
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void k_part_scan(uint32_t *__restrict__ cnt_less,
                                                            uint32_t *__restrict__ cnt_eq, int m) {
    __shared__ uint32_t s_w[kScanThreads / kWave];
    uint32_t *a = blockIdx.x == 0 ? cnt_less : cnt_eq;
    const int per = (m + kScanThreads - 1) / kScanThreads;
    const int b = threadIdx.x * per;
    const int e = b + per < m ? b + per : m;
    uint32_t sum = 0;
    for (int i = b; i < e; ++i)
        sum += a[i];
    uint32_t run = block_incl_scan(sum, s_w) - sum;
    for (int i = b; i < e; ++i) {
        const uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
}

template <int D>
__global__ __launch_bounds__(kThreads) void k_part_scatter(const Inst *__restrict__ inst,
                                                           const uint32_t *__restrict__ tile_inst, TopArrays A,
                                                           const uint32_t *__restrict__ Iin_all,
                                                           uint32_t *__restrict__ Xout_all,
                                                           uint32_t *__restrict__ Iout_all, int j,
                                                           const uint32_t *__restrict__ scan_less,
                                                           const uint32_t *__restrict__ scan_eq,
                                                           uint32_t *__restrict__ tile_box) {
    __shared__ uint32_t s_w[2][kWaves];
    __shared__ uint32_t s_box[2][D][2];
    TopTile tt;
    if (!top_tile(inst, tile_inst, blockIdx.x, j, tt))
        return;
    const Inst &I = *tt.I;
    const int64_t n = I.n, e0 = tt.e0, tile0 = tt.tile0;
    const NodeGeom g = tt.g;
    const NodeSplit sp = (static_cast<const NodeSplit *>(A.split) + I.S)[tt.t];
    // instance-local views of the group arrays
    const int64_t np = A.positions;
    const uint32_t *Xin = A.X + I.P;
    const uint32_t *Iin = Iin_all + I.P;
    uint32_t *Xout = Xout_all + I.P;
    uint32_t *Iout = Iout_all + I.P;
    // points of this node before this tile that are below / equal to the median
    const uint32_t less_base = scan_less[blockIdx.x] - scan_less[tile0];
    const uint32_t eq_base = scan_eq[blockIdx.x] - scan_eq[tile0];
    if (threadIdx.x < 2 * D) {
        const int c = threadIdx.x / D, k = threadIdx.x % D;
        s_box[c][k][0] = 0xFFFFFFFFu;
        s_box[c][k][1] = 0u;
    }
    const int w = threadIdx.x / kWave;
    const int64_t ew = e0 + (int64_t)w * kWaveItems;
    // every value this thread moves, loaded up front
    uint32_t xv[D][kItems], iv[kItems];
#pragma unroll
    for (int k = 0; k < D; ++k)
        load_items(Xin + (int64_t)k * np, n, ew, xv[k]);
    load_items(Iin, n, ew, iv);
    uint32_t lb[kItems], eb[kItems];
    uint32_t less_bits = 0, eq_bits = 0;
    uint32_t run_l = 0, run_e = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t e = ew + (int64_t)r * kWave + __lane_id();
        uint32_t va = xv[0][r];
#pragma unroll
        for (int k = 1; k < D; ++k)
            va = sp.axis == k ? xv[k][r] : va;
        const uint32_t v = va - sp.base;
        const bool less = e < n && (sp.all_left || v < sp.median);
        const bool eq = e < n && !sp.all_left && v == sp.median;
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
        const int64_t e = ew + (int64_t)r * kWave + __lane_id();
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
            const uint32_t v = xv[k][r];
            Xout[(int64_t)k * np + dst] = v;
            if (left) {
                lmin[k] = v < lmin[k] ? v : lmin[k];
                lmax[k] = v > lmax[k] ? v : lmax[k];
            } else {
                rmin[k] = v < rmin[k] ? v : rmin[k];
                rmax[k] = v > rmax[k] ? v : rmax[k];
            }
        }
        Iout[dst] = iv[r];
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
    // this tile's share of the two children's boxes (an empty share has
    // min > max); k_box_reduce combines the shares of a node's tiles
    if (threadIdx.x < 4 * D)
        tile_box[(int64_t)blockIdx.x * 4 * D + threadIdx.x] = (&s_box[0][0][0])[threadIdx.x];
}

// The children's boxes of every node of level j from the per-tile shares
// (one workgroup per node).
template <int D>
__global__ __launch_bounds__(kThreads) void k_box_reduce(const Inst *__restrict__ inst,
                                                         const uint2 *__restrict__ node_tab, TopArrays A, int j,
                                                         const uint32_t *__restrict__ tile_box) {
    __shared__ uint32_t s_r[kWaves][4 * D];
    TopTile tt;
    if (!top_node(inst, node_tab, j, tt))
        return;
    const Inst &I = *tt.I;
    const int64_t t = tt.t;
    const NodeGeom g = tt.g;
    uint32_t *child_boxes = A.nboxes + I.B + (2ll << j) * 2 * D;
    const int64_t t0 = tt.tile0, t1 = tt.tile0 + (g.count + kTile - 1) / kTile;
    uint32_t acc[4 * D];
#pragma unroll
    for (int i = 0; i < 4 * D; ++i)
        acc[i] = (i & 1) ? 0u : 0xFFFFFFFFu;  // [c][k][min, max]
    for (int64_t q = t0 + threadIdx.x; q < t1; q += kThreads) {
#pragma unroll
        for (int i = 0; i < 4 * D; ++i) {
            const uint32_t v = tile_box[q * 4 * D + i];
            acc[i] = (i & 1) ? (v > acc[i] ? v : acc[i]) : (v < acc[i] ? v : acc[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4 * D; ++i)
        acc[i] = (i & 1) ? wave_max_u32(acc[i]) : wave_min_u32(acc[i]);
    const int w = threadIdx.x / kWave;
    if (__lane_id() == 0) {
#pragma unroll
        for (int i = 0; i < 4 * D; ++i)
            s_r[w][i] = acc[i];
    }
    __syncthreads();
    if (threadIdx.x < 4 * D) {
        const int i = threadIdx.x;
        uint32_t v = s_r[0][i];
        for (int q = 1; q < kWaves; ++q)
            v = (i & 1) ? (s_r[q][i] > v ? s_r[q][i] : v) : (s_r[q][i] < v ? s_r[q][i] : v);
        child_boxes[2 * t * 2 * D + i] = v;
    }
}

// ---------------------------------------------------------------------------
// top levels with small nodes: one workgroup per node

// Splits every node of level j that holds at most 2^kOwnLog2 points with one
// workgroup of NT threads: the node's median along its split axis by radix
// select over an LDS histogram (11-bit digits, each pass reading the node's
// axis values again), then the same stable partition as the shared passes
// (points below the median, then the first need_eq points equal to it, go
// left) in runs of NT * kItems points in array order, with the children's
// boxes reduced on the way.  It writes the same records as those passes.
template <typename C, int D, int NT>
__global__ __launch_bounds__(NT) void k_node_split(const Inst *__restrict__ inst, const uint2 *__restrict__ node_tab,
                                                   TopArrays A, const uint32_t *__restrict__ Iin_all,
                                                   uint32_t *__restrict__ Xout_all, uint32_t *__restrict__ Iout_all,
                                                   int j, C *__restrict__ tree_box, uint32_t *__restrict__ rel_box,
                                                   uint64_t *__restrict__ split_hint) {
    constexpr int kB = 11;
    constexpr int kBins = 1 << kB;
    constexpr int kPer = kBins / NT;  // bins per thread in the pick
    constexpr int NW = NT / kWave;
    constexpr int kRun = NT * kItems;  // positions per run
    static_assert(kPer >= 1 && kBins % NT == 0, "whole bins per thread");
    __shared__ uint32_t s_h[kBins];
    __shared__ uint32_t s_w[2][2][NW];  // [run parity][below, equal][wave]
    __shared__ uint32_t s_scan[NW];
    __shared__ uint32_t s_pick[2];
    __shared__ uint32_t s_box[NW][4 * D];

    const uint2 job = node_tab ? node_tab[blockIdx.x] : make_uint2(0u, blockIdx.x);
    const Inst &I = inst[job.x];
    if (j < top_owned_from(I.height, I.lsh, I.jb) || j >= I.jb)
        return;
    const int64_t n = I.n;
    const int64_t S = 1ll << (I.height - j + I.lsh);
    const int64_t t = job.y;
    if (t * S >= n)
        return;
    const NodeGeom g = node_geom(t, S, n);
    const int64_t end = g.start + g.count;
    const uint32_t *nb = A.nboxes + I.B + ((1ll << j) + t) * 2 * D;
    const NodeSelect ns = node_select<D, kB>(nb);
    const bool all_left = g.half == g.count;
    const int64_t np = A.positions;
    const uint32_t *Xin = A.X + I.P;
    const uint32_t *x = Xin + (int64_t)ns.axis * np;
    const int w = threadIdx.x / kWave;
    const int lane = __lane_id();

    // the median: the point of rank `half` along the axis, digit by digit
    // (with no right half every point goes left and none is needed)
    uint32_t prefix = 0u, rank = (uint32_t)g.half;
    for (int pass = 0; !all_left && pass < ns.passes; ++pass) {
        int lo, hi;
        digit_bits(ns.bits, pass, kB, lo, hi);
        const uint32_t dmask = (1u << (hi - lo)) - 1u;
        for (int b = threadIdx.x; b < kBins; b += NT)
            s_h[b] = 0u;
        __syncthreads();
        uint32_t xn[kItems];
        load_items(x, end, g.start + (int64_t)w * kWaveItems, xn);
        for (int64_t c = g.start; c < end; c += kRun) {
            uint32_t xv[kItems];
#pragma unroll
            for (int r = 0; r < kItems; ++r)
                xv[r] = xn[r];
            if (c + kRun < end)
                load_items(x, end, c + kRun + (int64_t)w * kWaveItems, xn);
#pragma unroll
            for (int r = 0; r < kItems; ++r) {
                const int64_t e = c + (int64_t)w * kWaveItems + (int64_t)r * kWave + lane;
                const uint64_t v = (uint64_t)(xv[r] - ns.base);
                const bool match = e < end && (v >> hi) == (uint64_t)prefix;
                const uint32_t dg = (uint32_t)(v >> lo) & dmask;
                const uint64_t mm = __ballot(match);
                const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)dg);
                if (__ballot(match && dg != d0) == 0) {
                    if (mm != 0 && lane == 0)
                        atomicAdd(&s_h[d0], (uint32_t)__popcll(mm));
                } else if (match) {
                    atomicAdd(&s_h[dg], 1u);
                }
            }
        }
        __syncthreads();
        uint32_t cnt[kPer], mine = 0u;
#pragma unroll
        for (int b = 0; b < kPer; ++b) {
            cnt[b] = s_h[threadIdx.x * kPer + b];
            mine += cnt[b];
        }
        uint32_t cum = block_incl_scan(mine, s_scan) - mine;
#pragma unroll
        for (int b = 0; b < kPer; ++b) {
            if (cum <= rank && rank < cum + cnt[b]) {
                s_pick[0] = threadIdx.x * kPer + b;
                s_pick[1] = cum;
            }
            cum += cnt[b];
        }
        __syncthreads();
        prefix = (prefix << (hi - lo)) | s_pick[0];
        rank -= s_pick[1];
        __syncthreads();  // s_pick and s_h are used again
    }
    const uint32_t median = prefix, need_eq = rank;
    if (threadIdx.x == 0) {
        const int64_t v = (1ll << j) + t;
        split_hint[I.N + v] = ((uint64_t)(uint32_t)ns.axis << 32) | (uint64_t)(ns.base + median);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            tree_box[((I.N + v) * D + k) * 2 + 0] = (C)((int64_t)I.lo[k] + (int64_t)nb[2 * k]);
            tree_box[((I.N + v) * D + k) * 2 + 1] = (C)((int64_t)I.lo[k] + (int64_t)nb[2 * k + 1]);
            rel_box[((I.N + v) * D + k) * 2 + 0] = nb[2 * k];
            rel_box[((I.N + v) * D + k) * 2 + 1] = nb[2 * k + 1];
        }
    }

    // the stable partition, run by run
    const uint32_t *Iin = Iin_all + I.P;
    uint32_t *Xout = Xout_all + I.P;
    uint32_t *Iout = Iout_all + I.P;
    uint32_t lmin[D], lmax[D], rmin[D], rmax[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lmin[k] = rmin[k] = 0xFFFFFFFFu;
        lmax[k] = rmax[k] = 0u;
    }
    uint32_t below_run = 0u, equal_run = 0u;  // the node's points before this run below / equal to the median
    int par = 0;
    for (int64_t c = g.start; c < end; c += kRun, par ^= 1) {
        const int64_t ew = c + (int64_t)w * kWaveItems;
        uint32_t xv[D][kItems], iv[kItems];
#pragma unroll
        for (int k = 0; k < D; ++k)
            load_items(Xin + (int64_t)k * np, end, ew, xv[k]);
        load_items(Iin, end, ew, iv);
        uint32_t lb[kItems], eb[kItems];
        uint32_t less_bits = 0u, eq_bits = 0u, run_l = 0u, run_e = 0u;
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const int64_t e = ew + (int64_t)r * kWave + lane;
            uint32_t va = xv[0][r];
#pragma unroll
            for (int k = 1; k < D; ++k)
                va = ns.axis == k ? xv[k][r] : va;
            const uint32_t v = va - ns.base;
            const bool less = e < end && (all_left || v < median);
            const bool eq = e < end && !all_left && v == median;
            const uint64_t ml = __ballot(less), me = __ballot(eq);
            lb[r] = run_l + (uint32_t)__popcll(ml & lanes_below());
            eb[r] = run_e + (uint32_t)__popcll(me & lanes_below());
            run_l += (uint32_t)__popcll(ml);
            run_e += (uint32_t)__popcll(me);
            less_bits |= (less ? 1u : 0u) << r;
            eq_bits |= (eq ? 1u : 0u) << r;
        }
        if (lane == 0) {
            s_w[par][0][w] = run_l;
            s_w[par][1][w] = run_e;
        }
        __syncthreads();
        uint32_t off_l = below_run, off_e = equal_run;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const uint32_t a = s_w[par][0][q], b = s_w[par][1][q];
            off_l += q < w ? a : 0u;
            off_e += q < w ? b : 0u;
            below_run += a;
            equal_run += b;
        }
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const int64_t e = ew + (int64_t)r * kWave + lane;
            if (e >= end)
                continue;
            const bool less = (less_bits >> r) & 1u, eq = (eq_bits >> r) & 1u;
            const uint32_t lbefore = off_l + lb[r];
            const uint32_t ebefore = off_e + eb[r];
            const bool left = less || (eq && ebefore < need_eq);
            const uint32_t eq_left_before = ebefore < need_eq ? ebefore : need_eq;
            const int64_t left_before = (int64_t)lbefore + (int64_t)eq_left_before;
            const int64_t pos = e - g.start;
            const int64_t dst = left ? g.start + left_before : g.start + g.half + (pos - left_before);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const uint32_t v = xv[k][r];
                Xout[(int64_t)k * np + dst] = v;
                if (left) {
                    lmin[k] = v < lmin[k] ? v : lmin[k];
                    lmax[k] = v > lmax[k] ? v : lmax[k];
                } else {
                    rmin[k] = v < rmin[k] ? v : rmin[k];
                    rmax[k] = v > rmax[k] ? v : rmax[k];
                }
            }
            Iout[dst] = iv[r];
        }
    }
    // the children's boxes ([child][axis][min, max]; an empty child keeps min > max)
#pragma unroll
    for (int k = 0; k < D; ++k) {
        group_min_max<6>(lmin[k], lmax[k]);
        group_min_max<6>(rmin[k], rmax[k]);
        if (lane == kWave - 1) {
            s_box[w][2 * k] = lmin[k];
            s_box[w][2 * k + 1] = lmax[k];
            s_box[w][2 * D + 2 * k] = rmin[k];
            s_box[w][2 * D + 2 * k + 1] = rmax[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 4 * D) {
        const int i = threadIdx.x;
        uint32_t v = s_box[0][i];
        for (int q = 1; q < NW; ++q)
            v = (i & 1) ? (s_box[q][i] > v ? s_box[q][i] : v) : (s_box[q][i] < v ? s_box[q][i] : v);
        uint32_t *child_boxes = A.nboxes + I.B + (2ll << j) * 2 * D;
        child_boxes[2 * t * 2 * D + i] = v;
    }
}

__global__ void k_fill_u32(uint32_t *__restrict__ a, int64_t m, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m)
        a[i] = v;
}

// each instance's root box in relative coordinates: [0, span] on every axis
// (instances built entirely in LDS have none)
template <int D>
__global__ void k_root_box(const Inst *__restrict__ inst, int count, uint32_t *__restrict__ nboxes) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count)
        return;
    const Inst &I = inst[i];
    if (I.jb == 0)
        return;
    uint32_t *nb = nboxes + I.B + 2 * D;  // node 1
#pragma unroll
    for (int k = 0; k < D; ++k) {
        nb[2 * k] = 0u;
        nb[2 * k + 1] = I.span[k];
    }
}

// Coordinates relative to lo in structure-of-arrays form, and the identity
// permutation, at every instance's positions.  Each is clamped to [0, span]:
// a no-op for bounds just measured, and on a plan's replay over points that
// left the planned bounds (reported through the plan's status word) it keeps
// every later extent, digit count and histogram inside what was planned.
template <int D>
__global__ __launch_bounds__(kThreads) void k_soa_init(const Inst *__restrict__ inst,
                                                       const uint32_t *__restrict__ tile_inst, int64_t positions,
                                                       uint32_t *__restrict__ X, uint32_t *__restrict__ Ids) {
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const Inst &I = inst_of_tile(inst, tile_inst, ((int64_t)blockIdx.x * blockDim.x) / kTile);
    const int64_t i = pos - I.P;
    if (i >= I.n)
        return;
    const int32_t *P = I.points;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        int64_t v = (int64_t)P[i * D + k] - (int64_t)I.lo[k];
        v = v < 0 ? 0 : v;
        v = v > (int64_t)I.span[k] ? (int64_t)I.span[k] : v;
        X[(int64_t)k * positions + pos] = (uint32_t)v;
    }
    Ids[pos] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// bottom levels: one workgroup per subtree, in LDS

template <typename C, int D, int LSH>
__global__ __launch_bounds__(kThreads) void k_bottom(const Inst *__restrict__ inst, const uint2 *__restrict__ sub,
                                                     const uint32_t *__restrict__ XA, const uint32_t *__restrict__ XB,
                                                     const uint32_t *__restrict__ IA, const uint32_t *__restrict__ IB,
                                                     int64_t np,
                                                     C *__restrict__ tree_box_all, uint32_t *__restrict__ rel_box_all,
                                                     C *__restrict__ coords_all, int32_t *__restrict__ sidx_all,
                                                     uint32_t *__restrict__ leaf_org_all,
                                                     uint32_t *__restrict__ leaf_ext_all,
                                                     uint32_t *__restrict__ leaf_pack_all,
                                                     uint64_t *__restrict__ split_hint_all) {
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
    __shared__ uint32_t s_pick[kWaves][2];
    __shared__ uint32_t s_cnt[kWaves][2];

    // this workgroup's instance and subtree (a group of one: blockIdx)
    const uint2 job = sub ? sub[blockIdx.x] : make_uint2(0u, blockIdx.x);
    const Inst &In = inst[job.x];
    const int64_t n = In.n;
    const int jb = In.jb, h = In.height;
    constexpr int lsh = LSH;  // log2 of the points per leaf (the group's In.lsh)
    constexpr int W = (D + 1) / 2;
    // after jb top-level passes (each moves the points to the other buffer)
    // the instance's points are in buffer jb mod 2
    const uint32_t *X = ((jb & 1) ? XB : XA) + In.P;
    const uint32_t *ids = ((jb & 1) ? IB : IA) + In.P;
    C *tree_box = tree_box_all + In.N * 2 * D;
    uint32_t *rel_box = rel_box_all + In.N * 2 * D;
    C *coords = coords_all + In.P * D;
    int32_t *sidx = sidx_all + In.P;
    uint32_t *leaf_org = leaf_org_all + In.L * D;
    uint32_t *leaf_ext = leaf_ext_all + In.L;
    uint32_t *leaf_pack = leaf_pack_all + In.P * W;
    uint64_t *split_hint = split_hint_all + In.N;
    const int64_t S0 = 1ll << (h - jb + lsh);  // at most M
    const int64_t s0 = (int64_t)job.y * S0;
    if (s0 >= n)
        return;
    const int cnt0 = (int)(n - s0 < S0 ? n - s0 : S0);
    for (int i = threadIdx.x; i < cnt0; i += kThreads) {
#pragma unroll
        for (int k = 0; k < D; ++k)
            s_x[k][i] = X[(int64_t)k * np + s0 + i];
        s_id[i] = ids[s0 + i];
    }
    const int w = threadIdx.x / kWave;
    const int lane = __lane_id();
    for (int l = jb; l <= h; ++l) {
        const int S = 1 << (h - l + lsh);  // node size on this level
        const int nsub = (cnt0 + S - 1) / S;
        for (int u = threadIdx.x; u < nsub; u += kThreads)
#pragma unroll
            for (int k = 0; k < D; ++k) {
                s_box[u][k][0] = 0xFFFFFFFFu;
                s_box[u][k][1] = 0u;
            }
        __syncthreads();
        // boxes: each wave takes a contiguous share of the points and
        // reduces each node's part of it once (nodes are aligned runs of S
        // points, so a share holds whole nodes or lies inside one)
        {
            constexpr int PW = M / kWaves;  // points per wave
            const int i0 = w * PW;
            if (S >= kWave) {
                // one node per run of min(S, PW) points: lanes gather its
                // 64-point chunks, then one reduction across the wave
                const int run = S < PW ? S : PW;
                for (int r0 = i0; r0 < i0 + PW && r0 < cnt0; r0 += run) {
                    uint32_t mn[D], mx[D];
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        mn[k] = 0xFFFFFFFFu;
                        mx[k] = 0u;
                    }
                    for (int c = r0; c < r0 + run; c += kWave) {
                        const int i = c + lane;
                        if (i < cnt0) {
#pragma unroll
                            for (int k = 0; k < D; ++k) {
                                const uint32_t x = s_x[k][i];
                                mn[k] = x < mn[k] ? x : mn[k];
                                mx[k] = x > mx[k] ? x : mx[k];
                            }
                        }
                    }
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        group_min_max<6>(mn[k], mx[k]);
                        const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)mn[k], kWave - 1);
                        const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)mx[k], kWave - 1);
                        if (lane == 0) {
                            atomicMin(&s_box[r0 / S][k][0], a);
                            atomicMax(&s_box[r0 / S][k][1], b);
                        }
                    }
                }
            } else {
                // leaf level: every 64-point chunk holds 64 / S leaves, one
                // reduction per group of S lanes (its last lane holds it)
                for (int c = i0; c < i0 + PW && c < cnt0; c += kWave) {
                    const int i = c + lane;
                    const bool have = i < cnt0;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        uint32_t a = have ? s_x[k][i] : 0xFFFFFFFFu;
                        uint32_t b = have ? s_x[k][i] : 0u;
                        if (S == 16)
                            group_min_max<4>(a, b);
                        else
                            group_min_max<5>(a, b);
                        if ((i & (S - 1)) == S - 1 && i - (S - 1) < cnt0) {
                            atomicMin(&s_box[i / S][k][0], a);
                            atomicMax(&s_box[i / S][k][1], b);
                        }
                    }
                }
            }
        }
        __syncthreads();
        for (int u = threadIdx.x; u < nsub; u += kThreads) {
            const int64_t v = (1ll << l) + s0 / S + u;
            uint32_t ext = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                tree_box[(v * D + k) * 2 + 0] = (C)((int64_t)In.lo[k] + (int64_t)s_box[u][k][0]);
                tree_box[(v * D + k) * 2 + 1] = (C)((int64_t)In.lo[k] + (int64_t)s_box[u][k][1]);
                rel_box[(v * D + k) * 2 + 0] = s_box[u][k][0];
                rel_box[(v * D + k) * 2 + 1] = s_box[u][k][1];
                const uint32_t e = s_box[u][k][1] - s_box[u][k][0];
                ext = e > ext ? e : ext;
            }
            if (l == h) {
                // leaf record: corner (relative to the global minimum) and widest extent
                const int64_t c = (s0 >> lsh) + u;
#pragma unroll
                for (int k = 0; k < D; ++k)
                    leaf_org[c * D + k] = s_box[u][k][0];
                leaf_ext[c] = ext;
            }
        }
        if (l == h)
            break;
        if (2 * nsub <= kWaves) {
            // Few nodes: G = kWaves / nsub waves split each node together.
            // Every wave runs the same number of passes (the most any node
            // needs) so that the block barriers line up.
            const int G = kWaves / nsub;
            const int u = w / G, sw = w % G;
            const int base = u * S;
            const int cnt = cnt0 - base < S ? cnt0 - base : S;
            const int half = cnt < S / 2 ? cnt : S / 2;
            const int a = longest_axis<D>(&s_box[u][0][0]);
            const uint32_t lo = s_box[u][a][0];
            const int bits = (int)bit_length(s_box[u][a][1] - lo);
            int passes_max = 0, passes = 0;
            for (int uu = 0; uu < nsub; ++uu) {
                const int b_u = uu * S;
                const int c_u = cnt0 - b_u < S ? cnt0 - b_u : S;
                const int h_u = c_u < S / 2 ? c_u : S / 2;
                const int a_u = longest_axis<D>(&s_box[uu][0][0]);
                const int p_u =
                    h_u == c_u ? 0 : (int)((bit_length(s_box[uu][a_u][1] - s_box[uu][a_u][0]) + kB - 1) / kB);
                passes_max = p_u > passes_max ? p_u : passes_max;
                if (uu == u)
                    passes = p_u;
            }
            // this wave's contiguous share of the node's points
            const int chunk = ((cnt + G * kWave - 1) / (G * kWave)) * kWave;
            const int c_begin = sw * chunk < cnt ? sw * chunk : cnt;
            const int c_end = c_begin + chunk < cnt ? c_begin + chunk : cnt;
            uint32_t prefix = 0, rank = (uint32_t)half;
            for (int p = 0; p < passes_max; ++p) {
                const bool act = p < passes;
                int dlo, dhi;
                digit_bits(bits, p, kB, dlo, dhi);
                const uint32_t dmask = (1u << (dhi - dlo)) - 1u;
                for (int b = sw * kWave + lane; b < kNB; b += G * kWave)
                    s_hist[u][b] = 0u;
                __syncthreads();
                if (act) {
                    for (int i = c_begin + lane; i < c_end; i += kWave) {
                        const uint64_t v = (uint64_t)(s_x[a][base + i] - lo);
                        if ((v >> dhi) == (uint64_t)prefix)
                            atomicAdd(&s_hist[u][(uint32_t)(v >> dlo) & dmask], 1u);
                    }
                }
                __syncthreads();
                if (act && sw == 0) {
                    uint32_t c[kLaneBins];
                    uint32_t mine = 0;
#pragma unroll
                    for (int b = 0; b < kLaneBins; ++b) {
                        c[b] = s_hist[u][lane * kLaneBins + b];
                        mine += c[b];
                    }
                    uint32_t cum = wave_incl_scan(mine) - mine;
#pragma unroll
                    for (int b = 0; b < kLaneBins; ++b) {
                        if (cum <= rank && rank < cum + c[b]) {
                            s_pick[u][0] = (uint32_t)(lane * kLaneBins + b);
                            s_pick[u][1] = cum;
                        }
                        cum += c[b];
                    }
                }
                __syncthreads();
                if (act) {
                    prefix = (prefix << (dhi - dlo)) | s_pick[u][0];
                    rank -= s_pick[u][1];
                }
            }
            const uint32_t median = prefix, need_eq = rank;
            const bool split_node = half != cnt;
            if (split_node && sw == 0 && lane == 0)
                split_hint[(1ll << l) + s0 / S + u] = ((uint64_t)(uint32_t)a << 32) | (uint64_t)(lo + median);
            // counts of this wave's share, then stable destinations
            uint32_t nl = 0, ne = 0;
            if (split_node) {
                for (int i0 = c_begin; i0 < c_end; i0 += kWave) {
                    const int i = i0 + lane;
                    const bool valid = i < c_end;
                    const uint32_t v = valid ? s_x[a][base + i] - lo : 0u;
                    nl += (uint32_t)__popcll(__ballot(valid && v < median));
                    ne += (uint32_t)__popcll(__ballot(valid && v == median));
                }
            }
            if (lane == 0) {
                s_cnt[w][0] = nl;
                s_cnt[w][1] = ne;
            }
            __syncthreads();
            uint32_t run_l = 0, run_e = 0;
            for (int q = u * G; q < w; ++q) {
                run_l += s_cnt[q][0];
                run_e += s_cnt[q][1];
            }
            for (int i0 = c_begin; i0 < c_end; i0 += kWave) {
                const int i = i0 + lane;
                const bool valid = i < c_end;
                if (!split_node) {
                    if (valid)
                        s_dst[base + i] = (uint16_t)(base + i);
                    continue;
                }
                const uint32_t v = valid ? s_x[a][base + i] - lo : 0u;
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
        } else {
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
            const int bits = (int)bit_length(s_box[u][a][1] - lo);
            const int passes = (bits + kB - 1) / kB;
            uint32_t prefix = 0, rank = (uint32_t)half;
            for (int p = 0; p < passes; ++p) {
                int dlo, dhi;
                digit_bits(bits, p, kB, dlo, dhi);
                const uint32_t dmask = (1u << (dhi - dlo)) - 1u;
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
                    if ((v >> dhi) == (uint64_t)prefix)
                        __hip_atomic_fetch_add(&s_hist[w][(uint32_t)(v >> dlo) & dmask], 1u, __ATOMIC_RELAXED,
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
                prefix = (prefix << (dhi - dlo)) | pick;
                rank -= below;
            }
            const uint32_t median = prefix, need_eq = rank;
            if (lane == 0)
                split_hint[(1ll << l) + s0 / S + u] = ((uint64_t)(uint32_t)a << 32) | (uint64_t)(lo + median);
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
    for (int i = threadIdx.x; i < cnt0; i += kThreads) {
#pragma unroll
        for (int k = 0; k < D; ++k)
            coords[(s0 + i) * D + k] = (C)((int64_t)In.lo[k] + (int64_t)s_x[k][i]);
        sidx[s0 + i] = (int32_t)s_id[i];
        // offsets from the leaf corner, two 16-bit halves per word (read only
        // for leaves narrow enough that every offset fits)
        const int u = i >> lsh;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint32_t a = s_x[2 * w][i] - s_box[u][2 * w][0];
            const uint32_t b = 2 * w + 1 < D ? s_x[2 * w + 1][i] - s_box[u][2 * w + 1][0] : 0u;
            leaf_pack[(s0 + i) * W + w] = (a & 0xFFFFu) | (b << 16);
        }
    }
}

template <typename C, int D>
dpc_status build_kd(Workspace &ws, Index &ix) {
    hipStream_t s = ws.stream;
    const int64_t np = ix.positions;
    const int64_t tiles = np / kTile;
    constexpr int W = (D + 1) / 2;
    const bool single = ix.count == 1;
    C *coords, *box;
    DPC_TRY(ws.alloc(&coords, (size_t)np * D));
    DPC_TRY(ws.alloc(&box, (size_t)ix.nodes * 2 * D));
    DPC_TRY(ws.alloc(&ix.rbox, (size_t)ix.nodes * 2 * D));
    DPC_TRY(ws.alloc(&ix.split, (size_t)ix.nodes));
    DPC_TRY(ws.alloc(&ix.sidx, (size_t)np));
    DPC_TRY(ws.alloc(&ix.leaf_org, (size_t)ix.leaves * D));
    DPC_TRY(ws.alloc(&ix.leaf_ext, (size_t)ix.leaves));
    DPC_TRY(ws.alloc(&ix.leaf_pack, (size_t)np * W));
    ix.coords = coords;
    ix.box = box;

    uint32_t *XA, *XB = nullptr, *IA, *IB = nullptr;
    DPC_TRY(ws.alloc(&XA, (size_t)D * np));
    DPC_TRY(ws.alloc(&IA, (size_t)np));
    DPC_TRY(upload_group(ws, ix));
    launch((k_soa_init<D>), dim3(blocks_for(np, kThreads)), dim3(kThreads), 0, s, ix.inst, ix.tile_inst,
                       np, XA, IA);
    DPC_HIP(hipGetLastError());

    // host tables: histogram workgroups and nodes of every top level (groups
    // only; the nodes split with shared passes and those split one workgroup
    // each apart), the largest node of the latter per level, and the LDS
    // subtrees
    std::vector<uint32_t> hist_blocks;
    std::vector<int64_t> hist_first(ix.max_jb + 1, 0), node_first(ix.max_jb + 1, 0), own_first(ix.max_jb + 1, 0),
        own_size(ix.max_jb, 0);
    std::vector<uint2> subs, nodes, own_nodes;
    for (int j = 0; j < ix.max_jb; ++j) {
        hist_first[j] = (int64_t)hist_blocks.size();
        node_first[j] = (int64_t)nodes.size();
        own_first[j] = (int64_t)own_nodes.size();
        for (const Inst &I : ix.host)
            if (j >= top_owned_from(I.height, I.lsh, I.jb) && j < I.jb)
                own_size[j] = std::max<int64_t>(own_size[j], (int64_t)1 << (I.height - j + I.lsh));
        if (single)
            continue;
        for (int i = 0; i < ix.count; ++i) {
            const Inst &I = ix.host[i];
            if (j >= I.jb)
                continue;
            const int64_t S = 1ll << (I.height - j + I.lsh);
            std::vector<uint2> &tab = j < top_owned_from(I.height, I.lsh, I.jb) ? nodes : own_nodes;
            for (int64_t t = 0; t * S < I.n; ++t)
                tab.push_back(make_uint2((uint32_t)i, (uint32_t)t));
        }
        for (const Inst &I : ix.host) {
            if (j >= top_owned_from(I.height, I.lsh, I.jb))
                continue;
            const int64_t node_tiles = (1ll << (I.height - j + I.lsh)) / kTile;
            const int64_t per = node_tiles < 8 ? node_tiles : 8;
            const int64_t t_i = (I.n + kTile - 1) / kTile;
            for (int64_t q = 0; q < t_i; q += per) {
                const int64_t c = t_i - q < per ? t_i - q : per;
                hist_blocks.push_back((uint32_t)(((I.P / kTile + q) << 4) | (c - 1)));
            }
        }
    }
    hist_first[ix.max_jb] = (int64_t)hist_blocks.size();
    node_first[ix.max_jb] = (int64_t)nodes.size();
    own_first[ix.max_jb] = (int64_t)own_nodes.size();
    if (!single) {
        for (int i = 0; i < ix.count; ++i) {
            const Inst &I = ix.host[i];
            const int64_t S0 = 1ll << (I.height - I.jb + I.lsh);
            for (int64_t q = 0; q * S0 < I.n; ++q)
                subs.push_back(make_uint2((uint32_t)i, (uint32_t)q));
        }
    }
    uint32_t *d_hist_blocks = nullptr;
    uint2 *d_subs = nullptr, *d_nodes = nullptr, *d_own = nullptr;
    if (!single) {
        DPC_TRY(ws.alloc(&d_hist_blocks, hist_blocks.size() + 1));
        DPC_TRY(ws.alloc(&d_subs, subs.size() + 1));
        DPC_TRY(ws.alloc(&d_nodes, nodes.size() + 1));
        DPC_TRY(ws.alloc(&d_own, own_nodes.size() + 1));
        if (!hist_blocks.empty())
            DPC_HIP(hipMemcpyAsync(d_hist_blocks, hist_blocks.data(), hist_blocks.size() * sizeof(uint32_t),
                                   hipMemcpyHostToDevice, s));
        if (!subs.empty())
            DPC_HIP(hipMemcpyAsync(d_subs, subs.data(), subs.size() * sizeof(uint2), hipMemcpyHostToDevice, s));
        if (!nodes.empty())
            DPC_HIP(hipMemcpyAsync(d_nodes, nodes.data(), nodes.size() * sizeof(uint2), hipMemcpyHostToDevice, s));
        if (!own_nodes.empty())
            DPC_HIP(hipMemcpyAsync(d_own, own_nodes.data(), own_nodes.size() * sizeof(uint2), hipMemcpyHostToDevice,
                                   s));
        DPC_HIP(hipStreamSynchronize(s));  // the host tables go out of scope
    }

    if (ix.max_jb > 0) {
        DPC_TRY(ws.alloc(&XB, (size_t)D * np));
        DPC_TRY(ws.alloc(&IB, (size_t)np));
        int64_t nb_words = 0, hist_words = 0, sel = 0;
        for (const Inst &I : ix.host) {
            nb_words += I.jb > 0 ? (2ll << I.jb) * 2 * D : 0;
            hist_words += hist_words_below(top_owned_from(I.height, I.lsh, I.jb), I.wbits);
            sel += I.jb > 0 ? 1ll << (I.jb - 1) : 0;
        }
        uint32_t *nboxes, *hist, *cnt_less, *cnt_eq, *tile_box;
        NodeSplit *splits;
        SelectState *state;
        DPC_TRY(ws.alloc(&nboxes, (size_t)nb_words));
        DPC_TRY(ws.alloc(&hist, (size_t)(hist_words > 0 ? hist_words : 1)));
        DPC_TRY(ws.alloc(&splits, (size_t)sel));
        DPC_TRY(ws.alloc(&state, (size_t)sel));
        DPC_TRY(ws.alloc(&cnt_less, (size_t)tiles));
        DPC_TRY(ws.alloc(&cnt_eq, (size_t)tiles));
        DPC_TRY(ws.alloc(&tile_box, (size_t)tiles * 4 * D));
        // histograms and select records (their arrival counters) start at zero
        if (hist_words > 0)
            launch(k_fill_u32, dim3(blocks_for(hist_words, kThreads)), dim3(kThreads), 0, s, hist, hist_words, 0u);
        const int64_t state_words = sel * (int64_t)(sizeof(SelectState) / sizeof(uint32_t));
        launch(k_fill_u32, dim3(blocks_for(state_words, kThreads)), dim3(kThreads), 0, s, (uint32_t *)state,
               state_words, 0u);
        launch((k_root_box<D>), dim3(blocks_for(ix.count, kThreads)), dim3(kThreads), 0, s, ix.inst, ix.count,
               nboxes);
        TopArrays A{XA, np, nboxes, hist, state, splits};
        uint32_t *Iin = IA, *Xout = XB, *Iout = IB;  // level j reads buffer j mod 2
        const unsigned grid = (unsigned)tiles;
        for (int j = 0; j < ix.max_jb; ++j) {
            const int bits = level_bits(j);
            const int passes = (ix.max_wbits + bits - 1) / bits;
            // nodes split one workgroup each (instances whose level j is that small)
            const unsigned ogrid =
                single ? (own_size[j] > 0 ? 1u << j : 0u) : (unsigned)(own_first[j + 1] - own_first[j]);
            if (ogrid > 0) {
                const uint2 *ot = single ? nullptr : d_own + own_first[j];
                if (own_size[j] > 8192)
                    launch((k_node_split<C, D, 512>), dim3(ogrid), dim3(512), 0, s, ix.inst, ot, A,
                           (const uint32_t *)Iin, Xout, Iout, j, box, ix.rbox, ix.split);
                else
                    launch((k_node_split<C, D, 256>), dim3(ogrid), dim3(256), 0, s, ix.inst, ot, A,
                           (const uint32_t *)Iin, Xout, Iout, j, box, ix.rbox, ix.split);
                DPC_HIP(hipGetLastError());
            }
            // nodes split by the shared passes
            const bool shared = single ? own_size[j] == 0 : node_first[j + 1] > node_first[j];
            if (!shared) {
                std::swap(A.X, Xout);
                std::swap(Iin, Iout);
                continue;
            }
            // histogram workgroups: a table for groups; a fixed number of
            // tiles each (up to 8, never more than a node holds) for one instance
            const uint32_t *hb = nullptr;
            const uint2 *nt = nullptr;
            int per = 1;
            unsigned hgrid, ngrid;
            if (single) {
                const int64_t node_tiles = (1ll << (ix.host[0].height - j + ix.lsh)) / kTile;
                per = node_tiles < 8 ? (int)node_tiles : 8;
                hgrid = (unsigned)((tiles + per - 1) / per);
                ngrid = 1u << j;
            } else {
                hb = d_hist_blocks + hist_first[j];
                hgrid = (unsigned)(hist_first[j + 1] - hist_first[j]);
                nt = d_nodes + node_first[j];
                ngrid = (unsigned)(node_first[j + 1] - node_first[j]);
            }
            for (int p = 0; p < passes && hgrid > 0; ++p) {
                if (bits == 11)
                    launch((k_sel_hist<D, 11>), dim3(hgrid), dim3(kThreads), 0, s, ix.inst, ix.tile_inst, hb, per,
                           A, j, p);
                else if (bits == 10)
                    launch((k_sel_hist<D, 10>), dim3(hgrid), dim3(kThreads), 0, s, ix.inst, ix.tile_inst, hb, per,
                           A, j, p);
                else
                    launch((k_sel_hist<D, 8>), dim3(hgrid), dim3(kThreads), 0, s, ix.inst, ix.tile_inst, hb, per,
                           A, j, p);
            }
            if (bits == 11)
                launch((k_part_count<C, D, 11>), dim3(grid), dim3(kThreads), 0, s, ix.inst, ix.tile_inst, A, j,
                       cnt_less, cnt_eq, box, ix.rbox, ix.split);
            else if (bits == 10)
                launch((k_part_count<C, D, 10>), dim3(grid), dim3(kThreads), 0, s, ix.inst, ix.tile_inst, A, j,
                       cnt_less, cnt_eq, box, ix.rbox, ix.split);
            else
                launch((k_part_count<C, D, 8>), dim3(grid), dim3(kThreads), 0, s, ix.inst, ix.tile_inst, A, j,
                       cnt_less, cnt_eq, box, ix.rbox, ix.split);
            launch(k_part_scan, dim3(2), dim3(kScanThreads), 0, s, cnt_less, cnt_eq, (int)tiles);
            launch((k_part_scatter<D>), dim3(grid), dim3(kThreads), 0, s, ix.inst, ix.tile_inst, A,
                   (const uint32_t *)Iin, Xout, Iout, j, (const uint32_t *)cnt_less, (const uint32_t *)cnt_eq,
                   tile_box);
            launch((k_box_reduce<D>), dim3(ngrid), dim3(kThreads), 0, s, ix.inst, nt, A, j,
                   (const uint32_t *)tile_box);
            DPC_HIP(hipGetLastError());
            std::swap(A.X, Xout);
            std::swap(Iin, Iout);
        }
    }
    const unsigned bgrid = single ? (unsigned)(1ll << ix.host[0].jb) : (unsigned)subs.size();
    if (ix.lsh == 4)
        launch((k_bottom<C, D, 4>), dim3(bgrid), dim3(kThreads), 0, s, ix.inst,
                           single ? nullptr : d_subs, XA, XB, IA, IB, np, box, ix.rbox, coords, ix.sidx, ix.leaf_org,
                           ix.leaf_ext, ix.leaf_pack, ix.split);
    else if (ix.lsh == 5)
        launch((k_bottom<C, D, 5>), dim3(bgrid), dim3(kThreads), 0, s, ix.inst,
                           single ? nullptr : d_subs, XA, XB, IA, IB, np, box, ix.rbox, coords, ix.sidx, ix.leaf_org,
                           ix.leaf_ext, ix.leaf_pack, ix.split);
    else
        launch((k_bottom<C, D, 6>), dim3(bgrid), dim3(kThreads), 0, s, ix.inst,
                           single ? nullptr : d_subs, XA, XB, IA, IB, np, box, ix.rbox, coords, ix.sidx, ix.leaf_org,
                           ix.leaf_ext, ix.leaf_pack, ix.split);
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

}  // namespace

dpc_status build_kdtree(Workspace &ws, Index &ix) {
    const bool f64 = ix.arith == Arith::F64;
    switch (ix.d) {
#define DPC_KD_CASE(DD) \
    case DD:            \
        return f64 ? build_kd<double, DD>(ws, ix) : build_kd<int64_t, DD>(ws, ix);
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
