// Cluster labels (Section 3, Definitions 4-5; Section 6.2, Algorithm 3).
//
// Cutting every dependent edge with delta >= delta_min leaves a forest whose
// trees are the clusters; the paper joins the kept edges with a concurrent
// union-find.  Here every kept edge already points to a point of strictly
// higher priority, so each tree's root is its centre and a label is found by
// walking parent pointers up to the root.  Walks halve their path as they go
// (a node's parent is replaced by its grandparent), and a finished walk points
// its whole path at the root, so later walks are short.  Those writes race
// with other walks' reads, but every value ever stored in parent[x] is an
// ancestor of x in the same tree, so any value read is a valid step and every
// walk ends at the same root.
#include "dpc_internal.hpp"

namespace dpc {
namespace {

constexpr int kThreads = 256;

// Points the path from x0 at its root: every node on it gets the root as its
// parent, so that later walks through the path stop there (full path
// compression; each store is again an ancestor of its node).
__device__ inline void compress_path(int32_t *par, int32_t x0, int32_t root, int64_t n) {
    int32_t y = x0;
    for (int64_t steps = 0; y != root && steps <= n; ++steps) {
        const int32_t p = __hip_atomic_load(&par[y], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (p == root)
            break;
        __hip_atomic_store(&par[y], root, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        y = p;
    }
}

__global__ void k_flag_init(int32_t *flag) {
    if (threadIdx.x == 0)
        flag[0] = 0;
}

__global__ __launch_bounds__(kThreads) void k_parent(int64_t n, const int32_t *__restrict__ rho,
                                                     const int32_t *__restrict__ dep,
                                                     const int64_t *__restrict__ delta2, int32_t rho_min, int64_t Td,
                                                     int validate, int32_t *__restrict__ par, int32_t *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int32_t r = rho[i];
    int32_t p = (int32_t)i;
    if (r >= rho_min && delta2[i] < Td) {
        const int32_t j = dep[i];
        bool ok = true;
        if (validate) {
            ok = j >= 0 && (int64_t)j < n;
            if (ok) {
                const int32_t rj = rho[j];
                ok = rj > r || (rj == r && (int64_t)j < i);
            }
            if (!ok)
                __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (ok)
            p = j;
    }
    par[i] = p;
}

__global__ __launch_bounds__(kThreads) void k_roots(int64_t n, const int32_t *__restrict__ rho, int32_t rho_min,
                                                    int32_t *par, int32_t *__restrict__ label) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    if (rho[i] < rho_min) {
        label[i] = -1;
        return;
    }
    int32_t x = (int32_t)i;
    // every followed edge rises (checked, or produced by the library's own
    // dependent step), so a chain has fewer than n edges; the bound only
    // keeps a walk finite
    for (int64_t steps = 0; steps <= n; ++steps) {
        const int32_t p = __hip_atomic_load(&par[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (p == x)
            break;
        const int32_t g = __hip_atomic_load(&par[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (g == p) {
            x = p;
            break;
        }
        __hip_atomic_store(&par[x], g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = g;
    }
    label[i] = x;
    compress_path(par, (int32_t)i, x, n);
}

// The same two steps for every instance of a group, on the instances' own
// arrays (input order; the group's parent array holds instance i's parents
// at positions [P_i, P_i + n_i)).  The edges come from the library's own
// dependent step, so they form a forest by construction.
__global__ __launch_bounds__(kThreads) void k_parent_group(const Inst *__restrict__ inst,
                                                           const uint32_t *__restrict__ tile_inst,
                                                           int32_t *__restrict__ par) {
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const Inst &I = inst_of_tile(inst, tile_inst, ((int64_t)blockIdx.x * blockDim.x) / kTile);
    const int64_t i = pos - I.P;
    if (i >= I.n)
        return;
    int32_t p = (int32_t)i;
    if (global_ptr(I.rho)[i] >= I.rho_min && global_ptr(I.delta2)[i] < I.Td)
        p = global_ptr(I.dep)[i];
    par[pos] = p;
}

__global__ __launch_bounds__(kThreads) void k_roots_group(const Inst *__restrict__ inst,
                                                          const uint32_t *__restrict__ tile_inst, int32_t *par_all) {
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const Inst &I = inst_of_tile(inst, tile_inst, ((int64_t)blockIdx.x * blockDim.x) / kTile);
    const int64_t i = pos - I.P;
    if (i >= I.n)
        return;
    __attribute__((address_space(1))) int32_t *label = global_ptr(I.label);
    if (global_ptr(I.rho)[i] < I.rho_min) {
        label[i] = -1;
        return;
    }
    int32_t *par = par_all + I.P;
    int32_t x = (int32_t)i;
    // a chain of strictly rising priorities has fewer than n edges
    for (int64_t steps = 0; steps <= I.n; ++steps) {
        const int32_t p = __hip_atomic_load(&par[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (p == x)
            break;
        const int32_t g = __hip_atomic_load(&par[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (g == p) {
            x = p;
            break;
        }
        __hip_atomic_store(&par[x], g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = g;
    }
    label[i] = x;
    compress_path(par, (int32_t)i, x, I.n);
}

// One parent array per parameter pair (blockIdx.y), with the checks of
// k_parent; flag[k] is set when pair k follows an edge that does not rise.
__global__ __launch_bounds__(kThreads) void k_parent_sweep(int64_t n, const int32_t *__restrict__ rho,
                                                           const int32_t *__restrict__ dep,
                                                           const int64_t *__restrict__ delta2,
                                                           const int32_t *__restrict__ rho_mins,
                                                           const int64_t *__restrict__ Tds, int32_t *__restrict__ par,
                                                           int32_t *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= n)
        return;
    const int32_t r = rho[i];
    int32_t p = (int32_t)i;
    if (r >= rho_mins[k] && delta2[i] < Tds[k]) {
        const int32_t j = dep[i];
        bool ok = j >= 0 && (int64_t)j < n;
        if (ok) {
            const int32_t rj = rho[j];
            ok = rj > r || (rj == r && (int64_t)j < i);
        }
        if (ok)
            p = j;
        else
            __hip_atomic_store(flag + k, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    par[(int64_t)k * n + i] = p;
}

__global__ __launch_bounds__(kThreads) void k_roots_sweep(int64_t n, const int32_t *__restrict__ rho,
                                                          const int32_t *__restrict__ rho_mins, int32_t *par_all,
                                                          int32_t *__restrict__ label_all) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= n)
        return;
    int32_t *label = label_all + (int64_t)k * n;
    if (rho[i] < rho_mins[k]) {
        label[i] = -1;
        return;
    }
    int32_t *par = par_all + (int64_t)k * n;
    int32_t x = (int32_t)i;
    // every followed edge rises (checked), so a chain has fewer than n edges
    for (int64_t steps = 0; steps <= n; ++steps) {
        const int32_t p = __hip_atomic_load(&par[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (p == x)
            break;
        const int32_t g = __hip_atomic_load(&par[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (g == p) {
            x = p;
            break;
        }
        __hip_atomic_store(&par[x], g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = g;
    }
    label[i] = x;
    compress_path(par, (int32_t)i, x, n);
}

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = v;
}

}  // namespace

dpc_status launch_group_labels(const Index &ix, Workspace &ws) {
    hipStream_t s = ws.stream;
    int32_t *par;
    DPC_TRY(ws.alloc(&par, (size_t)ix.positions));
    const dim3 grid(blocks_for(ix.positions, kThreads)), block(kThreads);
    launch(k_parent_group, grid, block, 0, s, ix.inst, ix.tile_inst, par);
    launch(k_roots_group, grid, block, 0, s, ix.inst, ix.tile_inst, par);
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

dpc_status launch_cluster(int64_t n, const int32_t *rho, const int32_t *dep, const int64_t *delta2, int32_t rho_min,
                          int64_t Td, bool validate, int32_t *label, Workspace &ws) {
    hipStream_t s = ws.stream;
    int32_t *par, *flag;
    DPC_TRY(ws.alloc(&par, n));
    DPC_TRY(ws.alloc(&flag, 1));
    const dim3 grid(blocks_for(n, kThreads)), block(kThreads);
    launch(k_flag_init, dim3(1), dim3(kWave), 0, s, flag);
    launch(k_parent, grid, block, 0, s, n, rho, dep, delta2, rho_min, Td, validate ? 1 : 0, par, flag);
    DPC_HIP(hipGetLastError());
    if (validate) {
        // an unchecked cycle would never let the walks end: check first
        int32_t h = 0;
        DPC_HIP(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s));
        DPC_HIP(hipStreamSynchronize(s));
        if (h != 0)
            return DPC_ERR_NOT_FOREST;
    }
    launch(k_roots, grid, block, 0, s, n, rho, rho_min, par, label);
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

dpc_status launch_cluster_sweep(int64_t n, const int32_t *rho, const int32_t *dep, const int64_t *delta2, int count,
                                const int32_t *rho_mins, const int64_t *Tds, int32_t *label, Workspace &ws) {
    hipStream_t s = ws.stream;
    int32_t *par, *flag, *d_rmin;
    int64_t *d_Td;
    DPC_TRY(ws.alloc(&par, (size_t)n * count));
    DPC_TRY(ws.alloc(&flag, (size_t)count));
    DPC_TRY(ws.alloc(&d_rmin, (size_t)count));
    DPC_TRY(ws.alloc(&d_Td, (size_t)count));
    DPC_HIP(hipMemcpyAsync(d_rmin, rho_mins, count * sizeof(int32_t), hipMemcpyHostToDevice, s));
    DPC_HIP(hipMemcpyAsync(d_Td, Tds, count * sizeof(int64_t), hipMemcpyHostToDevice, s));
    launch(k_fill_i32, dim3(blocks_for(count, kThreads)), dim3(kThreads), 0, s, flag, (int64_t)count, 0);
    const dim3 grid(blocks_for(n, kThreads), (unsigned)count), block(kThreads);
    launch(k_parent_sweep, grid, block, 0, s, n, rho, dep, delta2, d_rmin, d_Td, par, flag);
    DPC_HIP(hipGetLastError());
    // an unchecked cycle would never let the walks end: check first (this
    // also keeps the host parameter arrays alive until they are copied)
    std::vector<int32_t> h((size_t)count, 0);
    DPC_HIP(hipMemcpyAsync(h.data(), flag, count * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DPC_HIP(hipStreamSynchronize(s));
    for (int32_t f : h)
        if (f != 0)
            return DPC_ERR_NOT_FOREST;
    launch(k_roots_sweep, grid, block, 0, s, n, rho, d_rmin, par, label);
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

}  // namespace dpc
