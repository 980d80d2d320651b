// Dependent points (Section 3, Definitions 2-3): for each query i, the
// lexicographic minimum of (D^2(i, j), j) over the points j of strictly
// higher priority (rho_j, -j).
//
// This is the priority nearest-neighbour query of Section 4.2.2: a node whose
// highest key is not above the query's key holds no candidate and is pruned,
// like any node whose box is farther than the best distance found so far.
// A node at exactly the best distance is still visited, since it may hold an
// equally near point of smaller index.  Each wavefront walks the tree with 64
// consecutive sorted queries, the points of its "home" node (one, two or
// four leaves by leaf size).
// The walk goes bottom-up: first the home node, then the sibling subtree of
// each ancestor of the home node from the deepest up, which together hold
// every point once; near candidates are met first, so the distance bounds
// are tight by the time the large subtrees near the root are tested, and the
// walk stops early once every lane's best is nearer than the boundary of the
// finished ancestor's box.  Inside a subtree the child on the side of the
// wave's first query is visited first (measured better than the side of the
// first lane that still needs the node, or of the home node's centre).  A
// leaf that few lanes need is searched cooperatively (leaf_coop), one that
// many need by each of those lanes in turn.
#include "traverse.hpp"

#include <limits>

namespace dpc {
namespace {

constexpr int kThreads = 256;
constexpr uint32_t kDepXcdRun = 128;  // XCD run length (workgroups), measured best in 2-D to 8-D

struct Lo {
    int32_t v[kMaxDim];  // global minimum per axis
};

// One candidate: keep the lexicographic minimum of (D^2, index) over points
// of higher priority; a larger low key word means a smaller index.
template <typename C>
__device__ inline void update_best(C s, uint64_t kj, uint64_t kq, C &best, uint32_t &best_low) {
    const uint32_t low = (uint32_t)kj;
    const bool better = (kj > kq) & ((s < best) | ((s == best) & (low > best_low)));
    best = better ? s : best;
    best_low = better ? low : best_low;
}

// kB candidates q[0..kB): most are no nearer than the best so far, so the
// distances and that test come first for the whole batch, and the wave takes
// the lexicographic update only when some lane has a candidate at most as
// near (the best only shrinks, so testing against the best from before the
// batch misses nothing).
template <typename C, int D, bool STATS, int kB>
__device__ inline void consider_batch(const C (&x)[D], const C (&q)[kB][D], const uint64_t (&kj)[kB], uint64_t kq,
                                      C &best, uint32_t &best_low, uint64_t &n_pairs) {
    C s[kB];
    uint64_t any = 0;  // lanes with a candidate (wave masks, combined in scalar registers)
#pragma unroll
    for (int b = 0; b < kB; ++b) {
        if (STATS)
            n_pairs += kj[b] > kq ? 1u : 0u;
        s[b] = dist2<C, D>(x, q[b]);
        any |= __builtin_amdgcn_ballot_w64(kj[b] > kq) & __builtin_amdgcn_ballot_w64(s[b] <= best);
    }
    if (__builtin_expect(any != 0, 0)) {
#pragma unroll
        for (int b = 0; b < kB; ++b)
            update_best<C>(s[b], kj[b], kq, best, best_low);
    }
}

// Leaves wanted by at most this many lanes of a wave go the cooperative way
// (measured: up to 32 of 64 lanes in 1-D to 4-D, every leaf from 5-D on).
template <int D>
constexpr int coop_max() {
    return D <= 4 ? 32 : kWave;
}

// One step of group_lex_min: (s, l) against the pair DPP move CTRL brings in
// (rows outside ROWS compare against the identity and keep theirs).
template <int CTRL, int ROWS, typename C>
__device__ inline void lex_min_step(C &s, uint32_t &l) {
    static_assert(sizeof(C) == 8, "64-bit distances");
    const uint64_t b = __builtin_bit_cast(uint64_t, s);
    const uint64_t id = __builtin_bit_cast(uint64_t, std::numeric_limits<C>::max());
    const uint32_t lo = dpp_move<CTRL, ROWS>((uint32_t)b, (uint32_t)id);
    const uint32_t hi = dpp_move<CTRL, ROWS>((uint32_t)(b >> 32), (uint32_t)(id >> 32));
    const uint32_t ol = dpp_move<CTRL, ROWS>(l, 0u);
    const C os = __builtin_bit_cast(C, ((uint64_t)hi << 32) | lo);
    const bool take = (os < s) | ((os == s) & (ol > l));
    s = take ? os : s;
    l = take ? ol : l;
}

// Lexicographic minimum of (D^2, index) over groups of 2^G lanes (a larger
// low key word is a smaller index), by DPP lane moves: within quads, the
// mirrored halves of 8- and 16-lane rows, then (G >= 5) row 1 from row 0's
// and row 3 from row 2's last lane, and (G = 6) rows 2 and 3 from lane 31.
// The result is in every lane of a 16-lane group and in the last lane of a
// 32- or 64-lane one.
template <int G, typename C>
__device__ inline void group_lex_min(C &s, uint32_t &l) {
    static_assert(G >= 4 && G <= 6, "groups of 16, 32 or 64 lanes");
    lex_min_step<0xB1, 0xF>(s, l);   // quad_perm [1,0,3,2]
    lex_min_step<0x4E, 0xF>(s, l);   // quad_perm [2,3,0,1]
    lex_min_step<0x141, 0xF>(s, l);  // row_half_mirror
    lex_min_step<0x140, 0xF>(s, l);  // row_mirror
    if constexpr (G >= 5)
        lex_min_step<0x142, 0xA>(s, l);  // row_bcast:15 into rows 1 and 3
    if constexpr (G >= 6)
        lex_min_step<0x143, 0xC>(s, l);  // row_bcast:31 into rows 2 and 3
}

// A leaf that few lanes of the wave want.  Looping each of those lanes over
// the leaf's points would leave most lanes idle, so the work is turned
// around: every group of leaf-size lanes holds the leaf's points (one per
// lane), the wanting lanes publish their query, current best and key in an
// LDS slot each, and every step tests one query per group against all
// points at once.  Only when some point is a candidate at most as near as a
// query's best does the group reduce to the lexicographic minimum of
// (D^2, index) and update that query's slot (with one group per wave, a
// single such point is read from its lane instead).  Same result as the
// per-lane loop.
template <typename C, int D, bool STATS, int LSH>
__device__ inline void leaf_coop(const C *__restrict__ coords, const uint64_t *__restrict__ skey, int64_t start,
                                 int count, uint64_t wm, bool want, const C (&x)[D], uint64_t kq, C &best,
                                 uint32_t &best_low, C *__restrict__ sq, uint64_t *__restrict__ sqk,
                                 C *__restrict__ sqb, uint32_t *__restrict__ sql, uint64_t &n_pairs) {
    // kG groups of 2^LSH lanes, each holding the leaf's points, take kG
    // queries per step
    constexpr int kL = 1 << LSH, kG = kWave / kL;
    const int lane = __lane_id();
    const int grp = kG == 1 ? 0 : lane >> LSH;  // (a constant with one group per wave)
    const int pl = lane & (kL - 1);
    const bool has = pl < count;
    const int64_t pp = start + (has ? pl : 0);
    C px[D];
#pragma unroll
    for (int k = 0; k < D; ++k)
        px[k] = coords[pp * D + k];
    const uint64_t pk = has ? skey[pp] : 0ull;  // 0: above no query's key
    const int mine = __popcll(wm & ((1ull << lane) - 1ull));
    if (want) {
#pragma unroll
        for (int k = 0; k < D; ++k)
            sq[mine * D + k] = x[k];
        sqk[mine] = kq;
        sqb[mine] = best;
        sql[mine] = best_low;
    }
    wave_lds_sync();
    const int nq = __popcll(wm);
    for (int r0 = 0; r0 < nq; r0 += kG) {
        const int r = r0 + grp;
        const bool live = r < nq;
        const int rr = live ? r : r0;
        C qx[D];
#pragma unroll
        for (int k = 0; k < D; ++k)
            qx[k] = sq[rr * D + k];
        const uint64_t qk = sqk[rr];
        const C qb = sqb[rr];
        const C s = dist2<C, D>(px, qx);
        const bool cand = live && has && pk > qk;
        if (STATS)
            n_pairs += cand ? 1u : 0u;
        const bool hit = cand && s <= qb;
        const uint64_t hm = __builtin_amdgcn_ballot_w64(hit);
        if (hm != 0) {
            C hs;
            uint32_t hl;
            bool any;
            if (kL == kWave && __popcll(hm) == 1) {
                // a single hit is the minimum: read it from its lane
                const int src = __ffsll((unsigned long long)hm) - 1;
                const uint64_t sb = __builtin_bit_cast(uint64_t, s);
                const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)sb, src);
                const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(sb >> 32), src);
                hs = __builtin_bit_cast(C, ((uint64_t)hi << 32) | lo);
                hl = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)pk, src);
                any = true;
            } else {
                hs = hit ? s : std::numeric_limits<C>::max();
                hl = hit ? (uint32_t)pk : 0u;
                group_lex_min<LSH, C>(hs, hl);
                const uint64_t gm = kL == kWave ? ~0ull : ((1ull << (kL % kWave)) - 1ull) << (kL * grp);
                any = (hm & gm) != 0;
            }
            if (pl == kL - 1 && live && any) {
                const uint32_t ql = sql[rr];
                if ((hs < qb) | ((hs == qb) & (hl > ql))) {
                    sqb[rr] = hs;
                    sql[rr] = hl;
                }
            }
        }
    }
    wave_lds_sync();
    if (want) {
        best = sqb[mine];
        best_low = sql[mine];
    }
    wave_lds_sync();  // the slots are written again at the next leaf
}

// GROUP = false: one instance, whose arrays and parameters are the kernel's
// arguments.  GROUP = true: each wave finds its instance from its tile; the
// arguments are the group's arrays and the rest is read from the
// instance's descriptor.  (Separate instantiations, so that the single
// instance keeps every parameter in kernel arguments.)
template <typename C, int D, bool STATS, bool GROUP, int LSH>
__global__ __launch_bounds__(kThreads) void k_dependent(const C *__restrict__ coords, const C *__restrict__ box,
                                                        const uint64_t *__restrict__ skey,
                                                        const uint64_t *__restrict__ maxkey,
                                                        const uint64_t *__restrict__ split, Lo lo, int64_t n,
                                                        int height, int32_t rho_min, int32_t rho_max,
                                                        const int32_t *__restrict__ sidx,
                                                        int32_t *__restrict__ dep_out,
                                                        int64_t *__restrict__ delta2_out, int64_t *counters,
                                                        const Inst *__restrict__ inst,
                                                        const uint32_t *__restrict__ tile_inst) {
    __shared__ C s_pts[kThreads / kWave][(1 << LSH) * D];
    __shared__ uint64_t s_key[kThreads / kWave][1 << LSH];
    // query slots of the cooperative leaf path
    constexpr int kCoopMax = coop_max<D>();
    __shared__ C s_qx[kThreads / kWave][kCoopMax * D];
    __shared__ uint64_t s_qk[kThreads / kWave][kCoopMax];
    __shared__ C s_qb[kThreads / kWave][kCoopMax];
    __shared__ uint32_t s_ql[kThreads / kWave][kCoopMax];
    uint64_t n_pairs = 0, n_nodes = 0, w_nodes = 0, w_points = 0;
    const int lane = __lane_id();
    int64_t q0 = wave_base<kDepXcdRun>(kThreads);
    if (GROUP) {
        const Inst &I = inst_of_tile(inst, tile_inst, q0 / kTile);
        q0 -= I.P;
        n = I.n;
        height = I.height;
        rho_min = I.dep_rho_min;
        rho_max = I.dep_rho_max;
        coords += I.P * D;
        box += I.N * 2 * D;
        skey += I.P;
        maxkey += I.N;
        split += I.N;
        sidx += I.P;
#pragma unroll
        for (int k = 0; k < D; ++k)
            lo.v[k] = I.lo[k];
    }
    const int64_t q = q0 + lane;
    if (q0 >= n)
        return;
    const bool valid = q < n;
    const int64_t qq = valid ? q : q0;
    C x[D];
#pragma unroll
    for (int k = 0; k < D; ++k)
        x[k] = coords[qq * D + k];
    const uint64_t kq = skey[qq];
    const int32_t rho_q = (int32_t)((uint32_t)(kq >> 32) ^ 0x80000000u);
    const bool active = valid && rho_q >= rho_min && rho_q <= rho_max;
    // the wave's first query, relative to lo: the reference point that
    // decides which child of a node is searched first
    uint32_t ref[D];
#pragma unroll
    for (int k = 0; k < D; ++k)
        ref[k] = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((int64_t)x[k] - lo.v[k]));

    C best = std::numeric_limits<C>::max();
    uint32_t best_low = 0;  // low key word of the best point; 0 = none yet
    const uint32_t first_leaf = 1u << height;
    // home node; a: the ancestor whose sibling subtree is walked next
    constexpr int lsh = LSH;  // log2 of the points per leaf (the group's I.lsh)
    const int hd = height > 6 - lsh ? height - (6 - lsh) : 0;  // the node of the wave's 64 positions
    const uint32_t home = (1u << hd) + (uint32_t)((q0 >> lsh) >> (height - hd));
    uint32_t a = home;
    int da = hd;
    uint32_t u = 1, v = home;  // virtual (visit order, relative to the subtree) and real node index
    int depth = hd;
    for (;;) {
        int64_t start, count;
        node_range(v, depth, height, lsh, n, start, count);
        bool descend = false;
        uint32_t first_child = 0;
        if (count > 0) {
            if (STATS)
                ++w_nodes;
            // key and box are loaded together and tested without branches
            const uint64_t mk = maxkey[v];
            const C bd = box_min_dist2<C, D>(x, box + (size_t)v * 2 * D);
            const bool higher = active && mk > kq;
            const bool want = higher && bd <= best;
            if (STATS)
                n_nodes += higher ? 1u : 0u;
            if (v >= first_leaf) {
                const uint64_t wm = __builtin_amdgcn_ballot_w64(want);
                if (STATS && wm != 0)
                    w_points += (uint64_t)count;
                if (wm != 0 && (kCoopMax == kWave || __popcll(wm) <= kCoopMax)) {
                    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
                    leaf_coop<C, D, STATS, LSH>(coords, skey, start, (int)count, wm, want, x, kq, best, best_low,
                                                s_qx[w], s_qk[w], s_qb[w], s_ql[w], n_pairs);
                } else if (kCoopMax < kWave && wm != 0) {
                    // the wave stages the leaf in its LDS slot (one coalesced
                    // load), then the lanes that want it read every point
                    // from there (same address for all lanes: a broadcast)
                    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
                    C *sp = s_pts[w];
                    uint64_t *sk = s_key[w];
                    if (lane < count) {
#pragma unroll
                        for (int k = 0; k < D; ++k)
                            sp[lane * D + k] = coords[(start + lane) * D + k];
                        sk[lane] = skey[start + lane];
                    }
                    wave_lds_sync();
                    if (want) {
                        constexpr int kB = D <= 2 ? 4 : (D <= 4 ? 2 : 1);
                        int t = 0;
                        for (; t + kB <= (int)count; t += kB) {
                            C qv[kB][D];
                            uint64_t kv[kB];
#pragma unroll
                            for (int b = 0; b < kB; ++b) {
                                kv[b] = sk[t + b];
#pragma unroll
                                for (int k = 0; k < D; ++k)
                                    qv[b][k] = sp[(t + b) * D + k];
                            }
                            consider_batch<C, D, STATS, kB>(x, qv, kv, kq, best, best_low, n_pairs);
                        }
                        for (; t < (int)count; ++t) {
                            C qv[1][D];
                            const uint64_t kv[1] = {sk[t]};
#pragma unroll
                            for (int k = 0; k < D; ++k)
                                qv[0][k] = sp[t * D + k];
                            consider_batch<C, D, STATS, 1>(x, qv, kv, kq, best, best_low, n_pairs);
                        }
                    }
                    wave_lds_sync();
                }
            } else {
                const uint64_t m = __ballot(want);
                if (m) {
                    descend = true;
                    // the left child is never empty; the right one may be.
                    // The child on the reference point's side goes first.
                    if (count > ((int64_t)1 << (height - depth - 1 + lsh))) {
                        const uint64_t sp = split[v];
                        const uint32_t axis = (uint32_t)(sp >> 32);
                        uint32_t r = ref[0];
#pragma unroll
                        for (int k = 1; k < D; ++k)
                            r = axis == (uint32_t)k ? ref[k] : r;
                        first_child = r < (uint32_t)sp ? 0u : 1u;
                    }
                }
            }
        }
        if (descend) {
            u <<= 1;
            v = (v << 1) | first_child;
            ++depth;
            continue;
        }
        while (u & 1u) {
            u >>= 1;
            v >>= 1;
            --depth;
        }
        if (u != 0) {
            u += 1;
            v ^= 1u;
            continue;
        }
        // this subtree is done: the next one is the sibling of the next ancestor
        if (a <= 1)
            break;
        {
            // Every point not yet searched lies outside subtree a, beyond one
            // of the split planes that bound it, and a's box lies on this
            // side of each of them: such a point is at least the query's gap
            // to the box's boundary away.  A lane whose best is below the
            // square of that gap is settled (an equal distance could still
            // meet a smaller index), and when every lane is, the walk ends.
            const C *ab = box + (size_t)a * 2 * D;
            C g = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const C lo_gap = x[k] - ab[2 * k], hi_gap = ab[2 * k + 1] - x[k];
                const C m = lo_gap < hi_gap ? lo_gap : hi_gap;
                g = k == 0 ? m : (m < g ? m : g);
            }
            const bool settled = !active || (best_low != 0 && best < g * g);
            if (__builtin_amdgcn_ballot_w64(!settled) == 0)
                break;
        }
        v = a ^ 1u;
        depth = da;
        u = 1;
        a >>= 1;
        --da;
    }
    if (valid) {
        if (GROUP) {
            // the output arrays are looked up only now, so that their
            // addresses do not hold scalar registers during the walk
            const Inst &J = inst_of_tile(inst, tile_inst, wave_base<kDepXcdRun>(kThreads) / kTile);
            dep_out = J.dep;
            delta2_out = J.delta2;
        }
        const int32_t o = sidx[q];
        dep_out[o] = best_low != 0 ? (int32_t)(0xFFFFFFFFu - best_low) : -1;
        delta2_out[o] = best_low != 0 ? (int64_t)best : std::numeric_limits<int64_t>::max();
    }
    if (STATS) {
        add_wave_count(counters, kDependentPairs, n_pairs);
        add_wave_count(counters, kDependentNodes, n_nodes);
        add_wave_count(counters, kDependentWaveNodes, lane == 0 ? w_nodes : 0);
        add_wave_count(counters, kDependentWavePoints, lane == 0 ? w_points : 0);
    }
}

template <typename C, bool STATS, bool GROUP, int LSH>
dpc_status launch_typed(const Index &ix, int64_t *counters, hipStream_t s) {
    const C *coords = static_cast<const C *>(ix.coords);
    const C *box = static_cast<const C *>(ix.box);
    const dim3 grid(blocks_for(ix.positions, kThreads)), block(kThreads);
    // a single instance's parameters (ignored by the group kernel)
    const Inst &I = ix.host[0];
    Lo lo{};
    for (int k = 0; k < kMaxDim; ++k)
        lo.v[k] = I.lo[k];
    switch (ix.d) {
#define DPC_DEP_CASE(DD)                                                                                          \
    case DD:                                                                                                      \
        launch((k_dependent<C, DD, STATS, GROUP, LSH>), grid, block, 0, s, coords, box, ix.skey,     \
                           ix.maxkey, ix.split, lo, I.n, I.height, I.dep_rho_min, I.dep_rho_max, ix.sidx, I.dep, I.delta2, counters, \
                           ix.inst, ix.tile_inst);                                                                 \
        break;
        DPC_DEP_CASE(1)
        DPC_DEP_CASE(2)
        DPC_DEP_CASE(3)
        DPC_DEP_CASE(4)
        DPC_DEP_CASE(5)
        DPC_DEP_CASE(6)
        DPC_DEP_CASE(7)
        DPC_DEP_CASE(8)
#undef DPC_DEP_CASE
    default:
        return DPC_ERR_INVALID_ARG;
    }
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

template <typename C, bool STATS>
dpc_status launch_arith(const Index &ix, int64_t *counters, hipStream_t s) {
    if (ix.lsh == 4)
        return ix.count == 1 ? launch_typed<C, STATS, false, 4>(ix, counters, s)
                             : launch_typed<C, STATS, true, 4>(ix, counters, s);
    if (ix.lsh == 5)
        return ix.count == 1 ? launch_typed<C, STATS, false, 5>(ix, counters, s)
                             : launch_typed<C, STATS, true, 5>(ix, counters, s);
    return ix.count == 1 ? launch_typed<C, STATS, false, 6>(ix, counters, s)
                         : launch_typed<C, STATS, true, 6>(ix, counters, s);
}

}  // namespace

dpc_status launch_dependent(const Index &ix, int64_t *counters, hipStream_t s) {
    if (ix.arith == Arith::F64)
        return counters ? launch_arith<double, true>(ix, counters, s) : launch_arith<double, false>(ix, nullptr, s);
    return counters ? launch_arith<int64_t, true>(ix, counters, s) : launch_arith<int64_t, false>(ix, nullptr, s);
}

}  // namespace dpc
