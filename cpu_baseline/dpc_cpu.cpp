// Multithreaded CPU exact Density Peaks Clustering: the speed baseline the
// GPU library is measured beside.  Not the oracle (that is the plain O(n^2)
// definition) and not part of the GPU path; it shares no code with either.
//
// The method follows the paper's CPU design in outline: a k-d tree whose
// nodes carry the highest priority below them (Section 4.2.1), density by
// range counting with whole contained nodes counted at once (Section 6.1),
// the dependent point as a priority nearest-neighbour query that skips nodes
// holding no higher priority (Section 4.2.2, Algorithm 1), and labels by
// following dependent points (Section 6.2).  Work is spread over threads with
// a shared atomic chunk counter.  All distances are exact 64-bit integers;
// priorities are (rho, -index) and equal distances go to the smaller index,
// as in the library.
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <limits>
#include <thread>
#include <vector>

namespace {

constexpr int kLeaf = 16;
constexpr int kMaxD = 8;
constexpr int64_t kInf = std::numeric_limits<int64_t>::max();

// floor(r^2) (or ceil) of a double r >= 0, exactly: r = m * 2^e with an
// integer mantissa m, so r^2 = m^2 * 2^(2e) with m^2 below 2^106.
int64_t square_threshold(double r, bool up) {
    if (std::isinf(r))
        return kInf;
    if (r == 0.0)
        return 0;
    int e = 0;
    const double f = std::frexp(r, &e);  // r = f * 2^e, f in [0.5, 1)
    const unsigned __int128 m = (unsigned __int128)(uint64_t)std::ldexp(f, 53);
    const int sh = 2 * (e - 53);
    const unsigned __int128 sq = m * m;
    unsigned __int128 v;
    if (sh >= 0) {
        if (sh >= 64 || (sq >> (127 - sh)) != 0)
            return kInf;
        v = sq << sh;
    } else {
        const int s = -sh;
        if (s >= 127) {
            v = up ? 1 : 0;
        } else {
            v = sq >> s;
            if (up && (v << s) != sq)
                v += 1;
        }
    }
    return v > (unsigned __int128)kInf ? kInf : (int64_t)v;
}

struct Tree {
    int d = 0;
    int64_t n = 0;
    std::vector<int32_t> idx;     // point order: leaves are contiguous ranges
    std::vector<int64_t> x;       // coordinates in tree order [n][d]
    struct Node {
        int64_t lo, hi;           // range of positions
        int32_t left, right;      // children (-1 for a leaf)
        int64_t bmin[kMaxD], bmax[kMaxD];
    };
    std::vector<Node> nodes;
};

template <class F>
void parallel_for(int64_t count, int64_t chunk, int threads, F f) {
    std::atomic<int64_t> next(0);
    auto work = [&]() {
        for (;;) {
            const int64_t s = next.fetch_add(chunk);
            if (s >= count)
                return;
            const int64_t e = std::min(count, s + chunk);
            for (int64_t i = s; i < e; ++i)
                f(i);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < threads; ++t)
        th.emplace_back(work);
    work();
    for (auto &t : th)
        t.join();
}

// Builds the subtree over positions [lo, hi) of idx; returns its node id.
int32_t build(Tree &T, const int32_t *pts, int64_t lo, int64_t hi, std::vector<Tree::Node> &out) {
    Tree::Node nd;
    nd.lo = lo;
    nd.hi = hi;
    nd.left = nd.right = -1;
    const int d = T.d;
    for (int k = 0; k < d; ++k) {
        nd.bmin[k] = std::numeric_limits<int64_t>::max();
        nd.bmax[k] = std::numeric_limits<int64_t>::min();
    }
    for (int64_t i = lo; i < hi; ++i)
        for (int k = 0; k < d; ++k) {
            const int64_t v = pts[(int64_t)T.idx[i] * d + k];
            nd.bmin[k] = std::min(nd.bmin[k], v);
            nd.bmax[k] = std::max(nd.bmax[k], v);
        }
    const int32_t id = (int32_t)out.size();
    out.push_back(nd);
    if (hi - lo <= kLeaf)
        return id;
    int ax = 0;
    for (int k = 1; k < d; ++k)
        if (nd.bmax[k] - nd.bmin[k] > nd.bmax[ax] - nd.bmin[ax])
            ax = k;
    const int64_t mid = lo + (hi - lo) / 2;
    std::nth_element(T.idx.begin() + lo, T.idx.begin() + mid, T.idx.begin() + hi, [&](int32_t a, int32_t b) {
        const int32_t va = pts[(int64_t)a * d + ax], vb = pts[(int64_t)b * d + ax];
        return va < vb || (va == vb && a < b);
    });
    const int32_t l = build(T, pts, lo, mid, out);
    const int32_t r = build(T, pts, mid, hi, out);
    out[id].left = l;
    out[id].right = r;
    return id;
}

// The top of the tree is split serially into 4 * threads subtrees, which are
// built in parallel and then linked under the top nodes.
void build_tree(Tree &T, const int32_t *pts, int threads) {
    const int64_t n = T.n;
    T.idx.resize(n);
    for (int64_t i = 0; i < n; ++i)
        T.idx[i] = (int32_t)i;
    std::vector<Tree::Node> top;
    std::vector<std::pair<int64_t, int64_t>> parts;
    std::vector<int32_t> part_parent;
    std::vector<int> part_side;
    const int64_t target = std::max<int64_t>(kLeaf, n / (4 * (int64_t)threads) + 1);
    // breadth of the serial top: split ranges larger than target
    struct Item {
        int64_t lo, hi;
        int32_t parent;
        int side;
    };
    std::vector<Item> stack{{0, n, -1, 0}};
    while (!stack.empty()) {
        Item it = stack.back();
        stack.pop_back();
        if (it.hi - it.lo <= target) {
            parts.push_back({it.lo, it.hi});
            part_parent.push_back(it.parent);
            part_side.push_back(it.side);
            continue;
        }
        // a top node: box and split as in build(), without recursing
        Tree::Node nd;
        nd.lo = it.lo;
        nd.hi = it.hi;
        nd.left = nd.right = -1;
        const int d = T.d;
        for (int k = 0; k < d; ++k) {
            nd.bmin[k] = std::numeric_limits<int64_t>::max();
            nd.bmax[k] = std::numeric_limits<int64_t>::min();
        }
        for (int64_t i = it.lo; i < it.hi; ++i)
            for (int k = 0; k < d; ++k) {
                const int64_t v = pts[(int64_t)T.idx[i] * d + k];
                nd.bmin[k] = std::min(nd.bmin[k], v);
                nd.bmax[k] = std::max(nd.bmax[k], v);
            }
        int ax = 0;
        for (int k = 1; k < d; ++k)
            if (nd.bmax[k] - nd.bmin[k] > nd.bmax[ax] - nd.bmin[ax])
                ax = k;
        const int64_t mid = it.lo + (it.hi - it.lo) / 2;
        std::nth_element(T.idx.begin() + it.lo, T.idx.begin() + mid, T.idx.begin() + it.hi,
                         [&](int32_t a, int32_t b) {
                             const int32_t va = pts[(int64_t)a * d + ax], vb = pts[(int64_t)b * d + ax];
                             return va < vb || (va == vb && a < b);
                         });
        const int32_t id = (int32_t)top.size();
        top.push_back(nd);
        if (it.parent >= 0)
            (it.side == 0 ? top[it.parent].left : top[it.parent].right) = id;
        stack.push_back({mid, it.hi, id, 1});
        stack.push_back({it.lo, mid, id, 0});
    }
    std::vector<std::vector<Tree::Node>> sub(parts.size());
    std::vector<int32_t> sub_root(parts.size());
    parallel_for((int64_t)parts.size(), 1, threads, [&](int64_t p) {
        sub_root[p] = build(T, pts, parts[p].first, parts[p].second, sub[p]);
    });
    // concatenate: top nodes first, then each subtree with shifted ids
    T.nodes = top;
    for (size_t p = 0; p < parts.size(); ++p) {
        const int32_t base = (int32_t)T.nodes.size();
        for (Tree::Node nd : sub[p]) {
            if (nd.left >= 0) {
                nd.left += base;
                nd.right += base;
            }
            T.nodes.push_back(nd);
        }
        const int32_t root = base + sub_root[p];
        if (part_parent[p] >= 0)
            (part_side[p] == 0 ? T.nodes[part_parent[p]].left : T.nodes[part_parent[p]].right) = root;
    }
    // the root is node 0 (the first top node, or the single subtree)
    T.x.resize((size_t)n * T.d);
    parallel_for(n, 4096, threads, [&](int64_t i) {
        for (int k = 0; k < T.d; ++k)
            T.x[(size_t)i * T.d + k] = pts[(int64_t)T.idx[i] * T.d + k];
    });
}

inline int64_t box_min_dist2(const Tree::Node &nd, const int64_t *q, int d) {
    int64_t s = 0;
    for (int k = 0; k < d; ++k) {
        const int64_t t = q[k] < nd.bmin[k] ? nd.bmin[k] - q[k] : (q[k] > nd.bmax[k] ? q[k] - nd.bmax[k] : 0);
        s += t * t;
    }
    return s;
}

inline int64_t box_max_dist2(const Tree::Node &nd, const int64_t *q, int d) {
    int64_t s = 0;
    for (int k = 0; k < d; ++k) {
        const int64_t t = std::max(q[k] - nd.bmin[k], nd.bmax[k] - q[k]);
        s += t * t;
    }
    return s;
}

inline int64_t dist2(const int64_t *a, const int64_t *b, int d) {
    int64_t s = 0;
    for (int k = 0; k < d; ++k) {
        const int64_t t = a[k] - b[k];
        s += t * t;
    }
    return s;
}

}  // namespace

extern "C" {

// Returns 0 on success, 1 for invalid arguments, 2 when squared distances
// could exceed int64 (the library's status codes).  threads <= 0: one per
// hardware thread.
int dpc_cpu_run(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min, double delta_min,
                int32_t threads, int32_t *rho, int32_t *dep, int64_t *delta2, int32_t *label) {
    if (n < 0 || d < 1 || d > kMaxD || std::isnan(d_cut) || d_cut < 0 || std::isnan(delta_min) || rho_min < 0)
        return 1;
    if (n == 0)
        return 0;
    if (!points || !rho || !dep || !delta2 || !label)
        return 1;
    if (threads <= 0)
        threads = (int)std::max(1u, std::thread::hardware_concurrency());
    // range check: the widest squared distance must fit
    {
        unsigned __int128 s = 0;
        for (int k = 0; k < d; ++k) {
            int64_t lo = points[k], hi = points[k];
            for (int64_t i = 1; i < n; ++i) {
                lo = std::min<int64_t>(lo, points[i * d + k]);
                hi = std::max<int64_t>(hi, points[i * d + k]);
            }
            s += (unsigned __int128)(hi - lo) * (unsigned __int128)(hi - lo);
        }
        if (s > (unsigned __int128)kInf)
            return 2;
    }
    const int64_t T = square_threshold(d_cut, false);
    const int64_t Td = delta_min <= 0 ? 0 : square_threshold(delta_min, true);

    Tree tr;
    tr.d = d;
    tr.n = n;
    build_tree(tr, points, threads);
    const std::vector<Tree::Node> &nodes = tr.nodes;

    // density: range count; a node inside the ball counts whole
    std::vector<int32_t> srho(n);
    parallel_for(n, 256, threads, [&](int64_t qi) {
        const int64_t *q = &tr.x[(size_t)qi * d];
        int64_t cnt = 0;
        int32_t stack[128];
        int sp = 0;
        stack[sp++] = 0;
        while (sp) {
            const Tree::Node &nd = nodes[stack[--sp]];
            if (box_min_dist2(nd, q, d) > T)
                continue;
            if (box_max_dist2(nd, q, d) <= T) {
                cnt += nd.hi - nd.lo;
                continue;
            }
            if (nd.left < 0) {
                for (int64_t i = nd.lo; i < nd.hi; ++i)
                    cnt += dist2(q, &tr.x[(size_t)i * d], d) <= T;
                continue;
            }
            stack[sp++] = nd.left;
            stack[sp++] = nd.right;
        }
        srho[qi] = (int32_t)cnt;
        rho[tr.idx[qi]] = (int32_t)cnt;
    });

    // priorities: (rho, -index); per-node maximum.  Every node's children
    // have larger ids (top nodes precede the subtrees, and a subtree lists a
    // parent before its children), so a reverse sweep sees children first.
    std::vector<uint64_t> key(n);
    for (int64_t i = 0; i < n; ++i)
        key[i] = ((uint64_t)(uint32_t)((uint32_t)srho[i] ^ 0x80000000u) << 32) |
                 (uint64_t)(0xFFFFFFFFu - (uint32_t)tr.idx[i]);
    std::vector<uint64_t> mk(nodes.size(), 0);
    for (int64_t v = (int64_t)nodes.size() - 1; v >= 0; --v) {
        const Tree::Node &nd = nodes[v];
        uint64_t m = 0;
        if (nd.left < 0) {
            for (int64_t i = nd.lo; i < nd.hi; ++i)
                m = std::max(m, key[i]);
        } else {
            m = std::max(mk[nd.left], mk[nd.right]);
        }
        mk[v] = m;
    }

    // dependent points: priority nearest neighbour, the nearer child first
    parallel_for(n, 256, threads, [&](int64_t qi) {
        const int64_t *q = &tr.x[(size_t)qi * d];
        const uint64_t kq = key[qi];
        int64_t best = kInf;
        uint32_t best_low = 0;
        int32_t stack[128];
        int sp = 0;
        stack[sp++] = 0;
        while (sp) {
            const int32_t v = stack[--sp];
            const Tree::Node &nd = nodes[v];
            if (mk[v] <= kq || box_min_dist2(nd, q, d) > best)
                continue;
            if (nd.left < 0) {
                for (int64_t i = nd.lo; i < nd.hi; ++i) {
                    if (key[i] <= kq)
                        continue;
                    const int64_t s = dist2(q, &tr.x[(size_t)i * d], d);
                    const uint32_t low = (uint32_t)key[i];
                    if (s < best || (s == best && low > best_low)) {
                        best = s;
                        best_low = low;
                    }
                }
                continue;
            }
            const int64_t dl = box_min_dist2(nodes[nd.left], q, d), dr = box_min_dist2(nodes[nd.right], q, d);
            // push the farther child first so the nearer one is searched first
            if (dl <= dr) {
                stack[sp++] = nd.right;
                stack[sp++] = nd.left;
            } else {
                stack[sp++] = nd.left;
                stack[sp++] = nd.right;
            }
        }
        const int32_t o = tr.idx[qi];
        dep[o] = best_low ? (int32_t)(0xFFFFFFFFu - best_low) : -1;
        delta2[o] = best_low ? best : kInf;
    });

    // labels: follow dependents up to the centre, memoised (sequential, O(n))
    std::vector<int32_t> memo(n, -2);
    std::vector<int32_t> chain;
    for (int64_t i = 0; i < n; ++i) {
        if (rho[i] < rho_min) {
            label[i] = -1;
            continue;
        }
        int32_t c = (int32_t)i;
        chain.clear();
        while (memo[c] == -2 && delta2[c] < Td) {
            chain.push_back(c);
            c = dep[c];
        }
        const int32_t root = memo[c] != -2 ? memo[c] : c;
        memo[c] = root;
        for (int32_t x : chain)
            memo[x] = root;
        label[i] = root;
    }
    return 0;
}

}  // extern "C"
