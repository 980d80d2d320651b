// Density (Section 3, Definition 1): rho_i = #{ j : D^2(i, j) <= T }.
//
// Each wavefront takes 64 consecutive sorted points (one leaf of 64 points,
// or the two or four leaves below one node: its "home" node) and walks the
// tree.  For every node a lane classifies
// the node's box against its own ball:
//   outside  (nearest corner beyond the radius)   -> nothing to count;
//   inside   (farthest corner within the radius)  -> add the node's point
//            count without visiting its points (Section 6.1);
//   partial  -> the wave descends (a leaf's points are tested one by one).
// A lane that settled a node skips that node's subtree; it remembers the
// depth at which it settled, which stays valid while the walk is below it.
//
// The walk does not start at the root.  Every point lies in the home node or
// in the sibling of one of the home node's ancestors; a sibling whose box is
// more than r = floor(sqrt(T)) away from the home box along some axis holds
// no point within the radius of any query.  Lane l tests the sibling at depth
// l, and the walk starts at the parent of the shallowest sibling that may
// hold such a point (all shallower siblings are known to hold none).
//
// Leaf points are compared exactly in one of two ways.  In general the
// squared distance is formed in the coordinate type.  When the leaf is
// narrow (widest side at most R - M, where M = r + 1 and d * R^2 < 2^31),
// the query's offsets from the leaf corner are clamped to [-M, R] and every
// point's stored 16-bit offsets are subtracted in packed 16-bit lanes and
// squared and summed by 2-way dot products.  Unclamped offsets give the
// exact squared distance; a clamped one gives at least M^2 > T, and so does
// the true distance, since the clamped axis alone differs by at least M.
#include "traverse.hpp"

#include <climits>
#include <type_traits>

namespace dpc {
namespace {

constexpr int kThreads = 256;

typedef short short2_t __attribute__((ext_vector_type(2)));

// Parameters of the packed comparison of narrow leaves.
struct Narrow {
    const uint32_t *org;   // leaf corner relative to lo, [n_leaves][D]
    const uint32_t *ext;   // widest side of each leaf
    const uint32_t *pack;  // 16-bit offsets from the corner, [n][(D+1)/2]
    int32_t lo[kMaxDim];   // global minimum per axis
    int32_t M;             // floor(sqrt(T)) + 1 (at most R + 1)
    int32_t R;             // largest offset: D * R^2 < 2^31
    int32_t limit;         // largest widest side of a narrow leaf (R - M; negative: none)
    int32_t T;             // the threshold (used when limit >= 0, then T < M^2 <= 2^30)
};

// Points of one leaf within distance^2 T of x.  The leaf's coordinates are
// wave-uniform: scalar loads from global memory, or (kStaged) the wave's copy
// in LDS, which every lane reads at the same address.  A batch of kBatch
// points is read before any is used so that the reads overlap; the staged
// loop is not unrolled further (its values live in vector registers).
template <typename C, int D, int kBatch, bool kStaged>
__device__ inline int32_t count_within(const C (&x)[D], const C *__restrict__ p, int count, C T) {
    auto batch = [&](int t) {
        C q[kBatch][D];
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
#pragma unroll
            for (int k = 0; k < D; ++k)
                q[b][k] = p[(t + b) * D + k];
        int32_t c = 0;
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
            c += dist2<C, D>(x, q[b]) <= T ? 1 : 0;
        return c;
    };
    int32_t c = 0;
    int t = 0;
    if constexpr (kStaged) {
#pragma unroll 1
        for (; t + kBatch <= count; t += kBatch)
            c += batch(t);
    } else {
        for (; t + kBatch <= count; t += kBatch)
            c += batch(t);
    }
    for (; t < count; ++t)
        c += point_dist2<C, D>(x, p + t * D) <= T ? 1 : 0;
    return c;
}

// The same count on a narrow leaf: q holds the query's clamped offsets from
// the leaf corner, packed like the leaf's points.  Each dot product starts
// from -(T + 1), so a point is within the radius exactly when the result is
// negative (T < 2^30 and every clamped squared distance is below 2^31, so
// nothing wraps).  A batch shifts its points' sign bits into one word, one
// funnel shift per point, and counts them with one population count.
template <int W, int kBatch, bool kStaged>
__device__ inline int32_t count_within_packed(const uint32_t (&q)[W], const uint32_t *__restrict__ p, int count,
                                              int32_t T) {
    static_assert(kBatch >= 1 && kBatch <= 32, "a batch's sign bits fit one word");
    short2_t qv[W];
#pragma unroll
    for (int w = 0; w < W; ++w)
        qv[w] = __builtin_bit_cast(short2_t, q[w]);
    const int32_t base = -(T + 1);
    auto point = [&](const uint32_t *pp) {
        // (saturation never applies; asking for it selects the encoding
        // that reads the start value from a scalar register)
        int32_t acc = base;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const short2_t dv = qv[w] - __builtin_bit_cast(short2_t, pp[w]);
            acc = __builtin_amdgcn_sdot2(dv, dv, acc, true);
        }
        return (uint32_t)acc;
    };
    auto batch = [&](int t) {
        uint32_t pb[kBatch][W];
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
#pragma unroll
            for (int w = 0; w < W; ++w)
                pb[b][w] = p[(t + b) * W + w];
        uint32_t bits = point(pb[0]) >> 31;
#pragma unroll
        for (int b = 1; b < kBatch; ++b)
            bits = __builtin_amdgcn_alignbit(bits, point(pb[b]), 31u);  // (bits << 1) | sign
        return (int32_t)__builtin_popcount(bits);
    };
    int32_t c = 0;
    int t = 0;
    if constexpr (kStaged) {
#pragma unroll 1
        for (; t + kBatch <= count; t += kBatch)
            c += batch(t);
    } else {
        for (; t + kBatch <= count; t += kBatch)
            c += batch(t);
    }
    for (; t < count; ++t)
        c += (int32_t)(point(p + t * W) >> 31);
    return c;
}

__device__ inline int32_t clamp_i32(int32_t v, int32_t lo, int32_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Leaves partial to at most this many lanes of a wave are counted the
// cooperative way (measured best: 32 lanes up to 2-D; every leaf from 3-D
// on).
template <int D>
constexpr int den_coop_max() {
    return D <= 2 ? 32 : 64;
}
constexpr int kDenCoopMax = den_coop_max<kMaxDim>();  // the most any dimension uses
static_assert(den_coop_max<1>() <= kDenCoopMax && den_coop_max<3>() <= kDenCoopMax &&
                  den_coop_max<5>() <= kDenCoopMax && kDenCoopMax <= kWave,
              "the query slots hold every cooperative query");

// Count of one leaf for the lanes in pm (the leaf is partial to them), the
// cooperative way: each group of leaf-size lanes holds the leaf's points
// (one per lane), the lanes in pm publish their query in an LDS slot each,
// and every step tests one query per group against all points; the group's
// hits are one population count, added by the query's own lane.  P holds the
// point (a packed word set or coordinates), Q a query, and within(P, Q) is
// the exact test.
template <int LSH, typename P, typename Q, typename F>
__device__ inline int32_t coop_count(uint64_t pm, bool partial, const P &pt, bool has, const Q &mine_q,
                                     Q *__restrict__ slots, F within) {
    constexpr int kL = 1 << LSH, kG = kWave / kL;
    const int lane = __lane_id();
    const int grp = kG == 1 ? 0 : lane >> LSH;  // (a constant with one group per wave)
    const int mine = __popcll(pm & ((1ull << lane) - 1ull));
    const uint64_t hasm = __builtin_amdgcn_ballot_w64(has);
    if (partial)
        slots[mine] = mine_q;
    wave_lds_sync();
    const int nq = __popcll(pm);
    int32_t c = 0;
    if constexpr (kG == 1) {
        // one query a step: its hits go straight to the lane of that rank
        // (other lanes may hold one too; they are cleared at the end), two
        // queries at a time so that their tests interleave
        int r0 = 0;
        for (; r0 + 2 <= nq; r0 += 2) {
            const Q qa = slots[r0], qb = slots[r0 + 1];
            const uint64_t ma = hasm & __builtin_amdgcn_ballot_w64(within(pt, qa));
            const uint64_t mb = hasm & __builtin_amdgcn_ballot_w64(within(pt, qb));
            c = mine == r0 ? __popcll(ma) : c;
            c = mine == r0 + 1 ? __popcll(mb) : c;
        }
        if (r0 < nq) {
            const Q q = slots[r0];
            const uint64_t m = hasm & __builtin_amdgcn_ballot_w64(within(pt, q));
            c = mine == r0 ? __popcll(m) : c;
        }
        c = partial ? c : 0;
    } else {
        for (int r0 = 0; r0 < nq; r0 += kG) {
            const int r = r0 + grp;
            const bool live = r < nq;
            const Q q = slots[live ? r : r0];
            // (one ballot per condition: the test's is its comparison's lane mask)
            const uint64_t m = hasm & __builtin_amdgcn_ballot_w64(live) & __builtin_amdgcn_ballot_w64(within(pt, q));
#pragma unroll
            for (int g = 0; g < kG; ++g) {
                const int hits = __popcll((m >> (g * kL)) & ((1ull << kL) - 1ull));
                c += (partial && mine == r0 + g) ? hits : 0;
            }
        }
    }
    wave_lds_sync();  // the slots are written again at the next leaf
    return c;
}

// Nearest and farthest squared distance from x to a box (both relative to
// lo), with every per-axis gap clamped to M: a gap of M or more already puts
// the distance above T, and a clamped sum is then still at least M^2 > T, so
// both comparisons with T come out as with the exact values.  24-bit
// products suffice (M <= R < 2^15 and d * R^2 < 2^31).
template <int D>
__device__ inline void box_dist2_clamped(const int32_t (&xi)[D], const uint32_t *__restrict__ b, int32_t M,
                                         int32_t &dmin2, int32_t &dmax2) {
    int32_t mn = 0, mx = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int32_t a = (int32_t)b[2 * k] - xi[k];      // lo - x
        const int32_t c = xi[k] - (int32_t)b[2 * k + 1];  // x - hi
        int32_t near = a > c ? a : c;
        near = near > 0 ? near : 0;
        near = near < M ? near : M;
        int32_t farn = a < c ? a : c;  // minus the far gap
        farn = farn > -M ? farn : -M;
        mn += __mul24(near, near);
        mx += __mul24(farn, farn);
    }
    dmin2 = mn;
    dmax2 = mx;
}

// The group's arrays (position-, node- or leaf-indexed).
template <typename C>
struct DensityArrays {
    const C *coords;
    const C *box;
    const uint32_t *rbox;
    const uint32_t *org;
    const uint32_t *ext;
    const uint32_t *pack;
    int32_t *srho;
    const int32_t *sidx;
};

template <typename C, int D, bool STATS, bool INTBOX, int LSH>
__global__ __launch_bounds__(kThreads) void k_density(const Inst *__restrict__ inst,
                                                      const uint32_t *__restrict__ tile_inst, DensityArrays<C> G,
                                                      int64_t *counters) {
    constexpr bool kPacked = std::is_same<C, double>::value;
    constexpr int W = (D + 1) / 2;
    // one staged leaf per wave: D 8-byte coordinates or W packed words per point
    // (also the query slots of the cooperative count: at most kDenCoopMax)
    __shared__ uint64_t s_leaf[kThreads / kWave]
                              [D >= 3 ? ((1 << LSH) > kDenCoopMax ? (1 << LSH) : kDenCoopMax) * D
                                      : (den_coop_max<D>() > 0 ? den_coop_max<D>() * D : 1)];
    uint64_t n_pairs = 0, n_nodes = 0, n_contained = 0, w_nodes = 0, w_points = 0;
    const int lane = __lane_id();
    // this wave's instance; positions, nodes and leaves below are its own
    // XCD runs measured best: 16 workgroups in 2-D, 128 from 3-D on
    const int64_t g0 = wave_base<(D <= 2 ? 16u : 128u)>(kThreads);
    const Inst &I = inst_of_tile(inst, tile_inst, g0 / kTile);
    const int64_t n = I.n;
    const int height = I.height;
    constexpr int lsh = LSH;  // log2 of the points per leaf (the group's I.lsh)
    const int64_t q0 = g0 - I.P;
    const int64_t q = q0 + lane;
    if (q0 >= n)
        return;  // the whole wave lies past the end
    const C *coords = G.coords + I.P * D;
    const C *box = G.box + I.N * 2 * D;
    const uint32_t *rbox = G.rbox + I.N * 2 * D;
    int32_t *srho = G.srho + I.P;
    const int32_t *sidx = G.sidx + I.P;
    int32_t *rho_out = I.rho;
    // every squared distance is below 2^53 on the double path, so a larger
    // threshold acts like 2^53
    const C T = kPacked ? (C)(I.T >= (1ll << 53) ? (1ll << 53) : I.T) : (C)I.T;
    const C r = (C)I.r;
    Narrow nw;
    nw.org = G.org + I.L * D;
    nw.ext = G.ext + I.L;
    nw.pack = G.pack + I.P * W;
#pragma unroll
    for (int k = 0; k < kMaxDim; ++k)
        nw.lo[k] = I.lo[k];
    nw.M = I.M;
    nw.R = I.R;
    nw.limit = I.limit;
    nw.T = I.Tn;
    const bool valid = q < n;
    const int64_t qq = valid ? q : q0;
    C x[D];
#pragma unroll
    for (int k = 0; k < D; ++k)
        x[k] = coords[qq * D + k];
    int32_t xi[D] = {};  // offsets from the global minimum (narrow-leaf path)
    if constexpr (kPacked) {
#pragma unroll
        for (int k = 0; k < D; ++k)
            xi[k] = (int32_t)x[k] - nw.lo[k];
    }

    // home node (depth hd: the node of this wave's 64 positions) and the
    // start of the walk
    const int hd = height > 6 - lsh ? height - (6 - lsh) : 0;
    const uint32_t home = (1u << hd) + (uint32_t)((q0 >> lsh) >> (height - hd));
    int sd = hd;
    if (hd > 0) {
        const C *hb = box + (size_t)home * 2 * D;
        bool near = false;
        if (lane >= 1 && lane <= hd) {
            const uint32_t s = (home >> (hd - lane)) ^ 1u;
            int64_t st, cnt;
            node_range(s, lane, height, lsh, n, st, cnt);
            if (cnt > 0) {
                const C *sb = box + (size_t)s * 2 * D;
                bool far = false;
#pragma unroll
                for (int k = 0; k < D; ++k)
                    far |= (sb[2 * k] > hb[2 * k + 1] + r) || (sb[2 * k + 1] < hb[2 * k] - r);
                near = !far;
            }
        }
        const uint64_t m = __ballot(near);
        if (m)
            sd = __ffsll((unsigned long long)m) - 2;  // the parent of the first sibling that may count
    }

    int32_t cnt = 0;
    int settled = valid ? INT_MAX : -1;  // depth at which this lane settled the current path
    const uint32_t first_leaf = 1u << height;
    uint32_t v = home >> (hd - sd);
    int depth = sd;

    // Points of leaf v (positions [start, start + count)) within the radius,
    // for the lanes to which the leaf is partial.  From three dimensions on,
    // the wave first stages the leaf in its LDS slot with coalesced loads (the
    // packed offsets while the leaf's width is read; the coordinates when the
    // leaf is wide) and the lanes read each point from there; below that the
    // leaf is small enough for a few scalar loads.
    constexpr bool kStage = D >= 3;
    constexpr int kPackBatch = kStage ? 2 : (W == 1 ? 16 : 8 / W);
    constexpr int kWideBatch = kStage ? 1 : (INTBOX ? 2 : 8);
    auto leaf_count = [&](uint32_t leaf, int64_t start, int64_t count, bool partial) {
        const bool any = __ballot(partial) != 0;
        if (STATS && any)
            w_points += (uint64_t)count;
        if (!any)
            return;
        if (STATS && partial)
            n_pairs += (uint64_t)count;
        const uint32_t c = leaf - first_leaf;
        const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
        if constexpr (den_coop_max<D>() > 0) {
            const uint64_t pm = __builtin_amdgcn_ballot_w64(partial);
            if (__popcll(pm) <= den_coop_max<D>()) {
                constexpr int kL = 1 << lsh;
                const int pl = lane & (kL - 1);
                const bool has = pl < count;
                const int64_t pp = start + (has ? pl : 0);
                if constexpr (kPacked) {
                    if ((int32_t)nw.ext[c] <= nw.limit) {
                        struct PW {
                            uint32_t v[W];
                        };
                        PW pt, qw;
#pragma unroll
                        for (int k = 0; k < W; ++k)
                            pt.v[k] = nw.pack[pp * W + k];
#pragma unroll
                        for (int k = 0; k < W; ++k) {
                            const int32_t a =
                                clamp_i32(xi[2 * k] - (int32_t)nw.org[(size_t)c * D + 2 * k], -nw.M, nw.R);
                            const int32_t b =
                                2 * k + 1 < D
                                    ? clamp_i32(xi[2 * k + 1] - (int32_t)nw.org[(size_t)c * D + 2 * k + 1], -nw.M,
                                                nw.R)
                                    : 0;
                            qw.v[k] = ((uint32_t)a & 0xFFFFu) | ((uint32_t)b << 16);
                        }
                        const int32_t base = -(nw.T + 1);
                        cnt += coop_count<lsh>(pm, partial, pt, has, qw, reinterpret_cast<PW *>(s_leaf[w]),
                                               [&](const PW &a, const PW &b) {
                                                   int32_t acc = base;
#pragma unroll
                                                   for (int k = 0; k < W; ++k) {
                                                       const short2_t dv = __builtin_bit_cast(short2_t, b.v[k]) -
                                                                           __builtin_bit_cast(short2_t, a.v[k]);
                                                       acc = __builtin_amdgcn_sdot2(dv, dv, acc, true);
                                                   }
                                                   return acc < 0;
                                               });
                        return;
                    }
                }
                struct PC {
                    C v[D];
                };
                PC pt, qx;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    pt.v[k] = coords[pp * D + k];
                    qx.v[k] = x[k];
                }
                cnt += coop_count<lsh>(pm, partial, pt, has, qx, reinterpret_cast<PC *>(s_leaf[w]),
                                       [&](const PC &a, const PC &b) { return dist2<C, D>(a.v, b.v) <= T; });
                return;
            }
        }
        if constexpr (kPacked) {
            const uint32_t *pk = nw.pack + start * W;
            if constexpr (kStage) {
                uint32_t *sp = reinterpret_cast<uint32_t *>(s_leaf[w]);
                if constexpr (lsh <= 5) {
                    // at most 32 points of at most 4 words: two loads per lane
                    if (lane < (int)count * W)
                        sp[lane] = pk[lane];
                    if (W > 2 && lane + kWave < (int)count * W)
                        sp[lane + kWave] = pk[lane + kWave];
                } else {
                    for (int j = lane; j < (int)count * W; j += kWave)
                        sp[j] = pk[j];
                }
                pk = sp;
            }
            if ((int32_t)nw.ext[c] <= nw.limit) {
                uint32_t qw[W];
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const int32_t a = clamp_i32(xi[2 * k] - (int32_t)nw.org[(size_t)c * D + 2 * k], -nw.M, nw.R);
                    const int32_t b = 2 * k + 1 < D
                                          ? clamp_i32(xi[2 * k + 1] - (int32_t)nw.org[(size_t)c * D + 2 * k + 1],
                                                      -nw.M, nw.R)
                                          : 0;
                    qw[k] = ((uint32_t)a & 0xFFFFu) | ((uint32_t)b << 16);
                }
                if (kStage)
                    wave_lds_sync();
                if (partial)
                    cnt += count_within_packed<W, kPackBatch, kStage>(qw, pk, (int)count, nw.T);
                if (kStage)
                    wave_lds_sync();
                return;
            }
        }
        const C *pc = coords + start * D;
        if constexpr (kStage) {
            C *sc = reinterpret_cast<C *>(s_leaf[w]);
            if (lane < count) {
#pragma unroll
                for (int k = 0; k < D; ++k)
                    sc[lane * D + k] = pc[lane * D + k];
            }
            wave_lds_sync();
            pc = sc;
        }
        if (partial)
            cnt += count_within<C, D, kWideBatch, kStage>(x, pc, (int)count, T);
        if (kStage)
            wave_lds_sync();
    };
    // Classifies the current node for this lane (unless it settled above);
    // returns whether the node is partial to it.
    auto classify = [&](bool outside, bool inside, int64_t count) {
        if (outside) {
            settled = depth;
        } else if (inside) {
            cnt += (int32_t)count;
            settled = depth;
            if (STATS)
                n_contained += (uint64_t)count;
        } else {
            return true;
        }
        return false;
    };

    if constexpr (INTBOX) {
        // Integer boxes (relative to the instance's minimum corner), read
        // with scalar loads at each node: a node's box shares a cache line
        // with its sibling's.
        constexpr int B = 2 * D;
        for (;;) {
            int64_t start, count;
            node_range(v, depth, height, lsh, n, start, count);
            const bool internal = v < first_leaf;
            bool descend = false;
            if (count > 0) {
                if (STATS)
                    ++w_nodes;
                uint32_t cur[B];
#pragma unroll
                for (int i = 0; i < B; ++i)
                    cur[i] = rbox[(size_t)v * B + i];
                bool partial = false;
                if (settled >= depth) {
                    settled = INT_MAX;
                    if (STATS)
                        ++n_nodes;
                    int32_t dmin2, dmax2;
                    box_dist2_clamped<D>(xi, cur, nw.M, dmin2, dmax2);
                    partial = classify(dmin2 > nw.T, dmax2 <= nw.T, count);
                }
                if (!internal)
                    leaf_count(v, start, count, partial);
                else
                    descend = __ballot(partial) != 0;
            }
            if (descend) {
                v <<= 1;
                ++depth;
                continue;
            }
            while (depth > sd && (v & 1u)) {
                v >>= 1;
                --depth;
            }
            if (depth == sd)
                break;
            v += 1;
        }
    } else {
        for (;;) {
            int64_t start, count;
            node_range(v, depth, height, lsh, n, start, count);
            bool descend = false;
            if (count > 0) {
                if (STATS)
                    ++w_nodes;
                bool partial = false;
                if (settled >= depth) {
                    settled = INT_MAX;
                    if (STATS)
                        ++n_nodes;
                    C dmin2, dmax2;
                    box_dist2<C, D>(x, box + (size_t)v * 2 * D, dmin2, dmax2);
                    partial = classify(dmin2 > T, dmax2 <= T, count);
                }
                if (v >= first_leaf)
                    leaf_count(v, start, count, partial);
                else
                    descend = __ballot(partial) != 0;
            }
            if (descend) {
                v <<= 1;
                ++depth;
                continue;
            }
            // next node of the walk below the start node
            while (depth > sd && (v & 1u)) {
                v >>= 1;
                --depth;
            }
            if (depth == sd)
                break;
            v += 1;
        }
    }
    if (valid) {
        srho[q] = cnt;
        rho_out[sidx[q]] = cnt;
    }
    if (STATS) {
        add_wave_count(counters, kDensityPairs, n_pairs);
        add_wave_count(counters, kDensityNodes, n_nodes);
        add_wave_count(counters, kDensityContained, n_contained);
        add_wave_count(counters, kDensityWaveNodes, lane == 0 ? w_nodes : 0);
        add_wave_count(counters, kDensityWavePoints, lane == 0 ? w_points : 0);
    }
}

template <typename C, bool STATS, bool INTBOX, int LSH>
dpc_status launch_typed(const Index &ix, int32_t *srho, int64_t *counters, hipStream_t s) {
    DensityArrays<C> G{static_cast<const C *>(ix.coords), static_cast<const C *>(ix.box), ix.rbox, ix.leaf_org,
                       ix.leaf_ext, ix.leaf_pack, srho, ix.sidx};
    const dim3 grid(blocks_for(ix.positions, kThreads)), block(kThreads);
    switch (ix.d) {
#define DPC_DENSITY_CASE(DD)                                                                                    \
    case DD:                                                                                                    \
        launch((k_density<C, DD, STATS, INTBOX, LSH>), grid, block, 0, s, ix.inst, ix.tile_inst, \
                           G, counters);                                                                        \
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

template <int LSH>
dpc_status launch_leaf(const Index &ix, int32_t *srho, int64_t *counters, hipStream_t s) {
    if (ix.arith == Arith::F64) {
        // integer boxes when every instance's clamped gaps fit (then T < M^2 <= R^2)
        if (ix.intbox)
            return counters ? launch_typed<double, true, true, LSH>(ix, srho, counters, s)
                            : launch_typed<double, false, true, LSH>(ix, srho, nullptr, s);
        return counters ? launch_typed<double, true, false, LSH>(ix, srho, counters, s)
                        : launch_typed<double, false, false, LSH>(ix, srho, nullptr, s);
    }
    return counters ? launch_typed<int64_t, true, false, LSH>(ix, srho, counters, s)
                    : launch_typed<int64_t, false, false, LSH>(ix, srho, nullptr, s);
}

}  // namespace

dpc_status launch_density(const Index &ix, int32_t *srho, int64_t *counters, hipStream_t s) {
    return ix.lsh == 4 ? launch_leaf<4>(ix, srho, counters, s)
                       : (ix.lsh == 5 ? launch_leaf<5>(ix, srho, counters, s) : launch_leaf<6>(ix, srho, counters, s));
}

}  // namespace dpc
