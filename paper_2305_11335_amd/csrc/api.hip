// The C interface declared in include/libdpc.h: argument checks, exact
// thresholds, workspace lifetime and the order of the steps.
#include "dpc_internal.hpp"

#include <algorithm>
#include <atomic>

#include <cmath>
#include <limits>
#include <mutex>
#include <thread>

// The scratch of dpc_run_noalloc: device memory beyond its inputs and
// outputs that the library holds on every device it runs on (as a static
// array of its code object) instead of allocating per call.  In host code
// this name stands for a host-side shadow, not a device address: the device
// address of each device's copy comes from hipGetSymbolAddress
// (dpc::scratch_on_current_device) and only that address is ever used.
static __device__ __align__(256) unsigned char scratch[DPC_NOALLOC_SCRATCH_BYTES];

namespace dpc {

// floor(r^2) or ceil(r^2) of the exact value of the double r, saturating at
// INT64_MAX.  For r >= 1 the product splits exactly into hi + lo with
// hi = fl(r*r) and lo = fma(r, r, -hi) (an error-free transformation), and
// the rounding of hi + lo to an integer is decided from the two parts.
dpc_status square_threshold(double r, bool round_up, int64_t *out) {
    constexpr int64_t kMax = std::numeric_limits<int64_t>::max();
    if (out == nullptr || std::isnan(r) || r < 0.0)
        return DPC_ERR_INVALID_ARG;
    if (std::isinf(r)) {
        *out = kMax;
        return DPC_OK;
    }
    if (r < 1.0) {  // 0 <= r^2 < 1
        *out = (round_up && r > 0.0) ? 1 : 0;
        return DPC_OK;
    }
    const double hi = r * r;
    const double lo = std::fma(r, r, -hi);
    const double two63 = 9223372036854775808.0;
    const double two53 = 9007199254740992.0;
    if (hi > two63) {
        *out = kMax;
        return DPC_OK;
    }
    if (hi == two63) {
        // r^2 = 2^63 + lo with |lo| <= 512
        const double f = round_up ? std::ceil(lo) : std::floor(lo);
        *out = f >= 0.0 ? kMax : kMax + (int64_t)(f + 1.0);
        return DPC_OK;
    }
    if (hi >= two53) {
        // hi is an integer below 2^63; lo is the exact remainder
        const double f = round_up ? std::ceil(lo) : std::floor(lo);
        *out = (int64_t)hi + (int64_t)f;
        return DPC_OK;
    }
    const double fh = std::floor(hi);
    if (fh != hi) {
        // hi is at least one ulp from an integer and |lo| is at most half an ulp
        *out = (int64_t)fh + (round_up ? 1 : 0);
    } else {
        int64_t v = (int64_t)hi;
        if (round_up && lo > 0.0)
            v += 1;
        if (!round_up && lo < 0.0)
            v -= 1;
        *out = v;
    }
    return DPC_OK;
}

thread_local LaunchRecord *t_record = nullptr;
thread_local int32_t *t_plan_status = nullptr;

hipMemPool_t workspace_pool() {
    static std::mutex mu;
    static hipMemPool_t pools[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (pools[dev] == nullptr) {
        hipMemPoolProps props = {};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t p = nullptr;
        if (hipMemPoolCreate(&p, &props) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep);
        pools[dev] = p;
    }
    return pools[dev];
}

// The device address of the scratch on the current device, looked up once
// per device (with that device current) and kept; nullptr if the lookup fails.
void *scratch_on_current_device() {
    static std::mutex mu;
    static void *addr[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        addr[dev] = p;
    }
    return addr[dev];
}

namespace {

__global__ void k_zero_counters(int64_t *c) {
    if (threadIdx.x < kCounters)
        c[threadIdx.x] = 0;
}

// Measurements of dpc_run calls made with DPC_TIME_STAGES / DPC_COUNT_WORK,
// kept per host thread.  Events are created once per thread and device.
struct ThreadStats {
    bool valid = false;
    uint32_t flags = 0;
    int device = -1;
    hipEvent_t ev[DPC_STAGES + 1] = {};
    int64_t counters[kCounters] = {};
    uint64_t workspace_bytes = 0;
};

thread_local ThreadStats t_stats;

class RunRecorder {
  public:
    RunRecorder(uint32_t flags, hipStream_t s)
        : flags_(flags & (DPC_TIME_STAGES | DPC_COUNT_WORK)), stream_(s) {}

    dpc_status begin() {
        if (flags_ == 0)
            return DPC_OK;
        t_stats.valid = false;
        if (flags_ & DPC_TIME_STAGES) {
            int dev = 0;
            DPC_HIP(hipGetDevice(&dev));
            if (t_stats.device != dev) {
                for (auto &e : t_stats.ev) {
                    if (e)
                        (void)hipEventDestroy(e);
                    e = nullptr;
                }
                for (auto &e : t_stats.ev)
                    DPC_HIP(hipEventCreate(&e));
                t_stats.device = dev;
            }
            DPC_HIP(hipEventRecord(t_stats.ev[0], stream_));
        }
        return DPC_OK;
    }
    dpc_status mark(int stage) {
        if (flags_ & DPC_TIME_STAGES)
            DPC_HIP(hipEventRecord(t_stats.ev[stage + 1], stream_));
        return DPC_OK;
    }
    dpc_status read_counters(const int64_t *dev) {
        DPC_HIP(hipMemcpyAsync(t_stats.counters, dev, sizeof(t_stats.counters), hipMemcpyDeviceToHost, stream_));
        DPC_HIP(hipStreamSynchronize(stream_));
        return DPC_OK;
    }
    void commit(size_t workspace_bytes) {
        if (flags_ == 0)
            return;
        t_stats.workspace_bytes = workspace_bytes;
        if (!(flags_ & DPC_COUNT_WORK))
            for (auto &c : t_stats.counters)
                c = 0;
        t_stats.flags = flags_;
        t_stats.valid = true;
    }
    static int last(dpc_stats *out) {
        if (!t_stats.valid)
            return DPC_ERR_INVALID_ARG;
        *out = dpc_stats{};
        out->flags = t_stats.flags;
        if (t_stats.flags & DPC_TIME_STAGES) {
            DPC_HIP(hipEventSynchronize(t_stats.ev[DPC_STAGES]));
            for (int s = 0; s < DPC_STAGES; ++s) {
                float ms = 0.0f;
                DPC_HIP(hipEventElapsedTime(&ms, t_stats.ev[s], t_stats.ev[s + 1]));
                out->stage_ms[s] = ms;
            }
        }
        out->density_pairs = t_stats.counters[kDensityPairs];
        out->density_nodes = t_stats.counters[kDensityNodes];
        out->density_contained = t_stats.counters[kDensityContained];
        out->dependent_pairs = t_stats.counters[kDependentPairs];
        out->dependent_nodes = t_stats.counters[kDependentNodes];
        out->density_wave_nodes = t_stats.counters[kDensityWaveNodes];
        out->density_wave_points = t_stats.counters[kDensityWavePoints];
        out->dependent_wave_nodes = t_stats.counters[kDependentWaveNodes];
        out->dependent_wave_points = t_stats.counters[kDependentWavePoints];
        out->workspace_bytes = t_stats.workspace_bytes;
        return DPC_OK;
    }

  private:
    uint32_t flags_;
    hipStream_t stream_;
};

bool bad_shape(int64_t n, int32_t d) {
    return n < 0 || n > (int64_t)std::numeric_limits<int32_t>::max() - 1 || d < 1 || d > kMaxDim;
}

dpc_status delta_threshold(double delta_min, int64_t *Td) {
    if (std::isnan(delta_min))
        return DPC_ERR_INVALID_ARG;
    if (delta_min <= 0.0) {
        *Td = 0;
        return DPC_OK;
    }
    return square_threshold(delta_min, true, Td);
}

// Checks one instance's arguments and fills its job (flags as for dpc_run).
dpc_status make_job(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min, double delta_min,
                    uint32_t flags, int32_t *rho, int32_t *dep, int64_t *delta2, int32_t *label, Job &J) {
    if (bad_shape(n, d) || std::isnan(d_cut) || d_cut < 0.0 || rho_min < 0)
        return DPC_ERR_INVALID_ARG;
    int64_t Td;
    if (delta_threshold(delta_min, &Td) != DPC_OK)
        return DPC_ERR_INVALID_ARG;
    if (n > 0 && (points == nullptr || rho == nullptr || dep == nullptr || delta2 == nullptr || label == nullptr))
        return DPC_ERR_INVALID_ARG;
    J.points = points;
    J.n = n;
    DPC_TRY(square_threshold(d_cut, false, &J.T));
    J.rho_min = rho_min;
    J.Td = Td;
    J.dep_rho_min = (flags & DPC_SKIP_NOISE_DEPENDENTS) ? rho_min : std::numeric_limits<int32_t>::min();
    J.rho = rho;
    J.dep = dep;
    J.delta2 = delta2;
    J.label = label;
    return DPC_OK;
}

// The whole method on one group (instances of one dimension and one
// arithmetic), every step once for all of them.
// backend: DPC_BACKEND_* (the Fenwick tree and the priority-search tree
// serve single instances; groups always use the k-d tree).
dpc_status run_group(const std::vector<Job> &jobs, int d, Arith arith, RunRecorder *rec, int64_t *counters,
                     Workspace &ws, int backend = DPC_BACKEND_PRIORITY_TREE) {
    hipStream_t stream = ws.stream;
    Index ix;
    DPC_TRY(build_group(jobs, d, arith, leaf_log2(d), ws, ix));
    if (rec)
        DPC_TRY(rec->mark(DPC_STAGE_INDEX));
    int32_t *srho;
    DPC_TRY(ws.alloc(&srho, (size_t)ix.positions));
    DPC_TRY(launch_density(ix, srho, counters, stream));
    if (rec)
        DPC_TRY(rec->mark(DPC_STAGE_DENSITY));
    if (backend == DPC_BACKEND_FENWICK && ix.count == 1) {
        // the Fenwick tree of Algorithm 2 orders the points by priority itself
        if (rec)
            DPC_TRY(rec->mark(DPC_STAGE_PRIORITY));
        DPC_TRY(fenwick_dependent(jobs[0], d, arith, ix.lsh, ws));
    } else if (backend == DPC_BACKEND_PRIORITY_SEARCH_TREE && ix.count == 1) {
        // the priority-search tree of Section 4.2 is built from the priorities
        if (rec)
            DPC_TRY(rec->mark(DPC_STAGE_PRIORITY));
        DPC_TRY(pst_dependent(jobs[0], d, ws));
    } else {
        DPC_TRY(build_priority(srho, false, ws, ix));
        if (rec)
            DPC_TRY(rec->mark(DPC_STAGE_PRIORITY));
        DPC_TRY(launch_dependent(ix, counters, stream));
    }
    if (rec)
        DPC_TRY(rec->mark(DPC_STAGE_DEPENDENT));
    DPC_TRY(launch_group_labels(ix, ws));
    if (rec)
        DPC_TRY(rec->mark(DPC_STAGE_LABELS));
    return DPC_OK;
}

}  // namespace

dpc_status check_instance(const dpc_instance &q, uint32_t flags) {
    Job J;
    return make_job(q.points, q.n, q.d, q.d_cut, q.rho_min, q.delta_min, flags, q.rho, q.dep, q.delta2, q.label, J);
}

// Every step for a list of instances (each with its own flags: 0 or
// DPC_SKIP_NOISE_DEPENDENTS), grouped by dimension and arithmetic; sets each
// record's status.  peak_bytes (optional): the largest workspace held at
// once.
namespace {

// One dimension's instances of a batch: bounds, then one group per
// arithmetic.  Sets the range errors of its instances; *range_error tells
// whether there was one.
dpc_status run_dimension(int d, const std::vector<int> &ids, const std::vector<Job> &all, dpc_instance *instances,
                         hipStream_t stream, size_t *peak, bool *range_error, Workspace *persist) {
    *peak = 0;
    *range_error = false;
    std::vector<Job> jobs;
    for (int i : ids)
        jobs.push_back(all[i]);
    std::vector<int> bad;
    {
        // (persist: a plan records the call and keeps every allocation)
        Workspace local(stream);
        Workspace &ws = persist ? *persist : local;
        const dpc_status st = job_bounds(jobs, d, ws, &bad);
        *peak = ws.bytes > *peak ? ws.bytes : *peak;
        if (st != DPC_OK && st != DPC_ERR_RANGE)
            return st;
    }
    for (int b : bad) {
        instances[ids[b]].status = DPC_ERR_RANGE;
        *range_error = true;
    }
    // one group per arithmetic
    for (int a = 0; a < 2; ++a) {
        const Arith arith = a == 0 ? Arith::F64 : Arith::I64;
        std::vector<Job> group;
        for (size_t k = 0; k < jobs.size(); ++k) {
            if (instances[ids[k]].status != DPC_OK || job_arith(jobs[k], d) != arith)
                continue;
            group.push_back(jobs[k]);
        }
        // largest instances first: the dispatcher starts their waves
        // first, so the group does not end on one large instance's tail
        std::stable_sort(group.begin(), group.end(), [](const Job &x, const Job &y) { return x.n > y.n; });
        if (!group.empty()) {
            uint64_t bound = 0;  // a group takes at most the sum of its instances' bounds
            for (const Job &J : group)
                bound += workspace_bound(J.n, d);
            Workspace local(stream, bound);
            Workspace &ws = persist ? *persist : local;
            const dpc_status st = run_group(group, d, arith, nullptr, nullptr, ws);
            *peak = ws.bytes > *peak ? ws.bytes : *peak;
            if (st != DPC_OK)
                return st;
        }
    }
    return DPC_OK;
}

}  // namespace

dpc_status run_instances(dpc_instance *instances, const uint32_t *flags, int count, hipStream_t stream,
                         size_t *peak_bytes, Workspace *persist) {
    // checks, then groups by dimension
    std::vector<std::vector<int>> by_d(kMaxDim + 1);
    std::vector<Job> all(count);
    int first_error = DPC_OK;
    for (int i = 0; i < count; ++i) {
        dpc_instance &q = instances[i];
        q.status = make_job(q.points, q.n, q.d, q.d_cut, q.rho_min, q.delta_min, flags[i], q.rho, q.dep,
                            q.delta2, q.label, all[i]);
        if (q.status == DPC_OK && q.n > 0)
            by_d[q.d].push_back(i);
        if (q.status != DPC_OK && first_error == DPC_OK)
            first_error = q.status;
    }
    std::vector<int> dims;
    for (int d = 1; d <= kMaxDim; ++d)
        if (!by_d[d].empty())
            dims.push_back(d);
    std::vector<dpc_status> st(dims.size(), DPC_OK);
    std::vector<size_t> peak(dims.size(), 0);
    std::vector<char> range(dims.size(), 0);
    if (dims.size() <= 1 || persist) {
        // (a plan records on this thread and stream only)
        for (size_t k = 0; k < dims.size(); ++k) {
            bool r = false;
            st[k] = run_dimension(dims[k], by_d[dims[k]], all, instances, stream, &peak[k], &r, persist);
            range[k] = r;
        }
    } else {
        // several dimensions: each on a stream and host thread of its own,
        // so that one group's host waits and short launches overlap another
        // group's kernels.  The streams start after the caller's prior work
        // and the caller's stream waits for all of them.
        int dev = 0;
        DPC_HIP(hipGetDevice(&dev));
        hipEvent_t start_ev;
        DPC_HIP(hipEventCreateWithFlags(&start_ev, hipEventDisableTiming));
        std::vector<hipStream_t> streams(dims.size(), nullptr);
        std::vector<hipEvent_t> done(dims.size(), nullptr);
        dpc_status setup = hipEventRecord(start_ev, stream) == hipSuccess ? DPC_OK : DPC_ERR_HIP;
        for (size_t k = 0; k < dims.size() && setup == DPC_OK; ++k) {
            if (hipStreamCreateWithFlags(&streams[k], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&done[k], hipEventDisableTiming) != hipSuccess ||
                hipStreamWaitEvent(streams[k], start_ev, 0) != hipSuccess)
                setup = DPC_ERR_HIP;
        }
        if (setup == DPC_OK) {
            std::vector<std::thread> workers;
            for (size_t k = 0; k < dims.size(); ++k) {
                workers.emplace_back([&, k]() {
                    if (hipSetDevice(dev) != hipSuccess) {
                        st[k] = DPC_ERR_HIP;
                        return;
                    }
                    bool r = false;
                    st[k] = run_dimension(dims[k], by_d[dims[k]], all, instances, streams[k], &peak[k], &r,
                                          nullptr);
                    range[k] = r;
                    if (hipEventRecord(done[k], streams[k]) != hipSuccess && st[k] == DPC_OK)
                        st[k] = DPC_ERR_HIP;
                });
            }
            for (auto &t : workers)
                t.join();
            for (size_t k = 0; k < dims.size(); ++k)
                if (hipStreamWaitEvent(stream, done[k], 0) != hipSuccess && st[k] == DPC_OK)
                    st[k] = DPC_ERR_HIP;
        } else {
            (void)hipGetLastError();
        }
        for (size_t k = 0; k < dims.size(); ++k) {
            if (done[k])
                (void)hipEventDestroy(done[k]);
            if (streams[k])
                (void)hipStreamDestroy(streams[k]);  // released once its work is done
        }
        (void)hipEventDestroy(start_ev);
        if (setup != DPC_OK)
            return setup;
    }
    size_t total = 0;
    for (size_t k = 0; k < dims.size(); ++k) {
        if (st[k] != DPC_OK)
            return st[k];
        if (range[k] && first_error == DPC_OK)
            first_error = DPC_ERR_RANGE;
        // concurrent dimensions hold their workspaces at the same time
        const bool concurrent = dims.size() > 1 && !persist;
        total = concurrent ? total + peak[k] : (peak[k] > total ? peak[k] : total);
    }
    if (peak_bytes)
        *peak_bytes = total;
    return (dpc_status)first_error;
}


namespace {

// Dependent-point backend per dimension (DPC_BACKEND_*), read by dpc_run.
std::atomic<int> g_backend[kMaxDim + 1] = {};

// The whole method on one instance with the current settings: one warm-up
// run, then the faster of two, timed with HIP events on the stream; the
// outputs go to workspace.
dpc_status time_choice(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min, double delta_min,
                       int backend, hipStream_t stream, float *best_ms) {
    Job J;
    int32_t *rho, *dep, *label;
    int64_t *delta2;
    Workspace ws(stream);
    DPC_TRY(ws.alloc(&rho, (size_t)n));
    DPC_TRY(ws.alloc(&dep, (size_t)n));
    DPC_TRY(ws.alloc(&label, (size_t)n));
    DPC_TRY(ws.alloc(&delta2, (size_t)n));
    DPC_TRY(make_job(points, n, d, d_cut, rho_min, delta_min, 0, rho, dep, delta2, label, J));
    hipEvent_t e0, e1;
    DPC_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipGetLastError();
        return DPC_ERR_HIP;
    }
    dpc_status st = DPC_OK;
    for (int r = 0; r < 3 && st == DPC_OK; ++r) {
        std::vector<Job> jobs{J};
        Workspace run_ws(stream, workspace_bound(n, d));
        if (hipEventRecord(e0, stream) != hipSuccess)
            st = DPC_ERR_HIP;
        if (st == DPC_OK)
            st = job_bounds(jobs, d, run_ws, nullptr);
        if (st == DPC_OK)
            st = run_group(jobs, d, job_arith(jobs[0], d), nullptr, nullptr, run_ws, backend);
        if (st == DPC_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
            st = DPC_ERR_HIP;
        float ms = 0.0f;
        if (st == DPC_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            st = DPC_ERR_HIP;
        if (st == DPC_OK && r > 0 && (r == 1 || ms < *best_ms))
            *best_ms = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != DPC_OK)
        (void)hipGetLastError();
    return st;
}

}  // namespace

}  // namespace dpc

namespace dpc {
namespace {
// First launch of every replay: the status word starts clear, and the
// recorded bound checks set it to the range error.
__global__ void k_plan_clear(int32_t *status) {
    if (threadIdx.x == 0)
        status[0] = 0;
}
}  // namespace
}  // namespace dpc

// A recorded dpc_run (or dpc_batch_run): its workspace stays allocated and
// its kernel launches (with their argument values) are kept for replay.
struct dpc_plan {
    dpc::Workspace *ws = nullptr;
    dpc::LaunchRecord ops;
    int32_t *status = nullptr;  // device word set by every replay's bounds check
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace dpc;

extern "C" {

const char *dpc_status_str(int status) {
    switch (status) {
    case DPC_OK: return "ok";
    case DPC_ERR_INVALID_ARG: return "invalid argument";
    case DPC_ERR_RANGE: return "coordinate range too wide: squared distances could exceed int64";
    case DPC_ERR_NOT_FOREST: return "dependent edges do not form a forest of rising priority";
    case DPC_ERR_OOM: return "device workspace allocation failed";
    case DPC_ERR_HIP: return "HIP runtime error";
    case DPC_ERR_SCRATCH: return "instance too large for the fixed scratch of dpc_run_noalloc";
    default: return "unknown status";
    }
}

int dpc_square_threshold(double r, int32_t round_up, int64_t *out) {
    return square_threshold(r, round_up != 0, out);
}

int dpc_density(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t *rho, hipStream_t stream) {
    if (bad_shape(n, d) || std::isnan(d_cut) || d_cut < 0.0)
        return DPC_ERR_INVALID_ARG;
    if (n > 0 && (points == nullptr || rho == nullptr))
        return DPC_ERR_INVALID_ARG;
    if (n == 0)
        return DPC_OK;
    Job J;
    J.points = points;
    J.n = n;
    J.rho = rho;
    DPC_TRY(square_threshold(d_cut, false, &J.T));
    Workspace ws(stream);
    std::vector<Job> jobs{J};
    DPC_TRY(job_bounds(jobs, d, ws, nullptr));
    Index ix;
    DPC_TRY(build_group(jobs, d, job_arith(jobs[0], d), leaf_log2(d), ws, ix));
    int32_t *srho;
    DPC_TRY(ws.alloc(&srho, (size_t)ix.positions));
    return launch_density(ix, srho, nullptr, stream);
}

int dpc_dependent(const int32_t *points, int64_t n, int32_t d, const int32_t *rho, int32_t rho_min, int32_t *dep,
                  int64_t *delta2, hipStream_t stream) {
    if (bad_shape(n, d) || rho_min < 0)
        return DPC_ERR_INVALID_ARG;
    if (n > 0 && (points == nullptr || rho == nullptr || dep == nullptr || delta2 == nullptr))
        return DPC_ERR_INVALID_ARG;
    if (n == 0)
        return DPC_OK;
    Job J;
    J.points = points;
    J.n = n;
    J.rho = const_cast<int32_t *>(rho);  // read only here
    J.dep = dep;
    J.delta2 = delta2;
    J.dep_rho_min = rho_min > 0 ? rho_min : std::numeric_limits<int32_t>::min();
    Workspace ws(stream);
    std::vector<Job> jobs{J};
    DPC_TRY(job_bounds(jobs, d, ws, nullptr));
    Index ix;
    DPC_TRY(build_group(jobs, d, job_arith(jobs[0], d), leaf_log2(d), ws, ix));
    DPC_TRY(build_priority(nullptr, true, ws, ix));
    return launch_dependent(ix, nullptr, stream);
}

int dpc_cluster(int64_t n, const int32_t *rho, const int32_t *dep, const int64_t *delta2, int32_t rho_min,
                double delta_min, int32_t *label, hipStream_t stream) {
    if (n < 0 || n > (int64_t)std::numeric_limits<int32_t>::max() - 1 || rho_min < 0)
        return DPC_ERR_INVALID_ARG;
    int64_t Td;
    if (delta_threshold(delta_min, &Td) != DPC_OK)
        return DPC_ERR_INVALID_ARG;
    if (n > 0 && (rho == nullptr || dep == nullptr || delta2 == nullptr || label == nullptr))
        return DPC_ERR_INVALID_ARG;
    if (n == 0)
        return DPC_OK;
    Workspace ws(stream);
    return launch_cluster(n, rho, dep, delta2, rho_min, Td, true, label, ws);
}

int dpc_density_sweep(const int32_t *points, int64_t n, int32_t d, const double *d_cuts, int32_t count, int32_t *rho,
                      hipStream_t stream) {
    if (bad_shape(n, d) || count < 0 || (count > 0 && d_cuts == nullptr))
        return DPC_ERR_INVALID_ARG;
    std::vector<int64_t> T((size_t)count);
    for (int k = 0; k < count; ++k)
        if (std::isnan(d_cuts[k]) || d_cuts[k] < 0.0 || square_threshold(d_cuts[k], false, &T[k]) != DPC_OK)
            return DPC_ERR_INVALID_ARG;
    if (n > 0 && count > 0 && (points == nullptr || rho == nullptr))
        return DPC_ERR_INVALID_ARG;
    if (n == 0 || count == 0)
        return DPC_OK;
    // one index for every radius: the tree does not depend on d_cut
    Job J;
    J.points = points;
    J.n = n;
    J.rho = rho;
    J.T = T[0];
    Workspace ws(stream);
    std::vector<Job> jobs{J};
    DPC_TRY(job_bounds(jobs, d, ws, nullptr));
    Index ix;
    DPC_TRY(build_group(jobs, d, job_arith(jobs[0], d), leaf_log2(d), ws, ix));
    int32_t *srho;
    DPC_TRY(ws.alloc(&srho, (size_t)ix.positions));
    // one descriptor per radius, each writing its own row of rho
    std::vector<Inst> desc((size_t)count, ix.host[0]);
    for (int k = 0; k < count; ++k) {
        density_params(desc[k], T[k], d);
        desc[k].rho = rho + (int64_t)k * n;
    }
    Inst *d_desc;
    DPC_TRY(ws.alloc(&d_desc, (size_t)count));
    DPC_HIP(hipMemcpyAsync(d_desc, desc.data(), count * sizeof(Inst), hipMemcpyHostToDevice, stream));
    for (int k = 0; k < count; ++k) {
        Index one = ix;
        one.inst = d_desc + k;
        one.host.assign(1, desc[k]);
        one.intbox = ix.arith == Arith::F64 && desc[k].limit >= 0;
        DPC_TRY(launch_density(one, srho, nullptr, stream));
    }
    DPC_HIP(hipStreamSynchronize(stream));  // the host descriptors go out of scope
    return DPC_OK;
}

int dpc_cluster_sweep(int64_t n, const int32_t *rho, const int32_t *dep, const int64_t *delta2,
                      const int32_t *rho_mins, const double *delta_mins, int32_t count, int32_t *label,
                      hipStream_t stream) {
    if (n < 0 || n > (int64_t)std::numeric_limits<int32_t>::max() - 1 || count < 0 || count > 65535)
        return DPC_ERR_INVALID_ARG;
    if (count > 0 && (rho_mins == nullptr || delta_mins == nullptr))
        return DPC_ERR_INVALID_ARG;
    std::vector<int64_t> Td((size_t)count);
    for (int k = 0; k < count; ++k)
        if (rho_mins[k] < 0 || delta_threshold(delta_mins[k], &Td[k]) != DPC_OK)
            return DPC_ERR_INVALID_ARG;
    if (n > 0 && count > 0 && (rho == nullptr || dep == nullptr || delta2 == nullptr || label == nullptr))
        return DPC_ERR_INVALID_ARG;
    if (n == 0 || count == 0)
        return DPC_OK;
    Workspace ws(stream);
    return launch_cluster_sweep(n, rho, dep, delta2, count, rho_mins, Td.data(), label, ws);
}

int dpc_run(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min, double delta_min,
            uint32_t flags, int32_t *rho, int32_t *dep, int64_t *delta2, int32_t *label, hipStream_t stream) {
    const uint32_t known =
        DPC_SKIP_NOISE_DEPENDENTS | DPC_TIME_STAGES | DPC_COUNT_WORK | DPC_FENWICK_DEPENDENTS | DPC_PST_DEPENDENTS;
    if ((flags & ~known) || ((flags & DPC_FENWICK_DEPENDENTS) && (flags & DPC_PST_DEPENDENTS)))
        return DPC_ERR_INVALID_ARG;
    Job J;
    DPC_TRY(make_job(points, n, d, d_cut, rho_min, delta_min, flags, rho, dep, delta2, label, J));
    if (n == 0)
        return DPC_OK;
    RunRecorder rec(flags, stream);
    DPC_TRY(rec.begin());
    Workspace ws(stream, workspace_bound(n, d));
    int64_t *counters = nullptr;
    if (flags & DPC_COUNT_WORK) {
        DPC_TRY(ws.alloc(&counters, kCounters));
        launch(k_zero_counters, dim3(1), dim3(kWave), 0, stream, counters);
        DPC_HIP(hipGetLastError());
    }
    std::vector<Job> jobs{J};
    DPC_TRY(job_bounds(jobs, d, ws, nullptr));
    const int backend = (flags & DPC_FENWICK_DEPENDENTS)   ? DPC_BACKEND_FENWICK
                        : (flags & DPC_PST_DEPENDENTS)     ? DPC_BACKEND_PRIORITY_SEARCH_TREE
                                                           : g_backend[d].load(std::memory_order_relaxed);
    DPC_TRY(run_group(jobs, d, job_arith(jobs[0], d), &rec, counters, ws, backend));
    if (counters)
        DPC_TRY(rec.read_counters(counters));
    rec.commit(ws.bytes);
    return DPC_OK;
}

int dpc_run_noalloc(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min, double delta_min,
                    uint32_t flags, int32_t *rho, int32_t *dep, int64_t *delta2, int32_t *label,
                    hipStream_t stream) {
    if (flags & ~(uint32_t)DPC_SKIP_NOISE_DEPENDENTS)
        return DPC_ERR_INVALID_ARG;
    Job J;
    DPC_TRY(make_job(points, n, d, d_cut, rho_min, delta_min, flags, rho, dep, delta2, label, J));
    if (n == 0)
        return DPC_OK;
    // the bound covers every array the call carves (checked on the host,
    // before any GPU work)
    if (workspace_bound(n, d) > DPC_NOALLOC_SCRATCH_BYTES)
        return DPC_ERR_SCRATCH;
    void *buf = scratch_on_current_device();
    if (buf == nullptr)
        return DPC_ERR_HIP;
    Workspace ws(stream, buf, DPC_NOALLOC_SCRATCH_BYTES);
    ws.cap = std::numeric_limits<int>::max();
    std::vector<Job> jobs{J};
    DPC_TRY(job_bounds(jobs, d, ws, nullptr));
    const dpc_status st = run_group(jobs, d, job_arith(jobs[0], d), nullptr, nullptr, ws, false);
    return st == DPC_ERR_OOM ? DPC_ERR_SCRATCH : st;
}

int dpc_batch_run(dpc_instance *instances, int32_t count, uint32_t flags, hipStream_t stream) {
    if (count < 0 || (count > 0 && instances == nullptr) || (flags & ~(uint32_t)DPC_SKIP_NOISE_DEPENDENTS))
        return DPC_ERR_INVALID_ARG;
    std::vector<uint32_t> fl((size_t)count, flags);
    return run_instances(instances, fl.data(), count, stream, nullptr);
}

uint64_t dpc_workspace_bytes(int64_t n, int32_t d) {
    if (bad_shape(n, d))
        return 0;
    return workspace_bound(n, d);
}

int dpc_set_leaf_size(int32_t d, int32_t leaf_points) {
    if (d < 1 || d > kMaxDim || (leaf_points != 16 && leaf_points != 32 && leaf_points != 64))
        return DPC_ERR_INVALID_ARG;
    set_leaf_log2(d, leaf_points == 16 ? 4 : (leaf_points == 32 ? 5 : 6));
    return DPC_OK;
}

int32_t dpc_leaf_size(int32_t d) {
    if (d < 1 || d > kMaxDim)
        return 0;
    return 1 << leaf_log2(d);
}

int dpc_autotune(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min, double delta_min,
                 hipStream_t stream, double *ms_out, int32_t *chosen) {
    if (bad_shape(n, d) || n == 0 || points == nullptr)
        return DPC_ERR_INVALID_ARG;
    const int before = leaf_log2(d);
    float best_ms[DPC_LEAF_SIZES] = {};
    dpc_status st = DPC_OK;
    for (int c = 0; c < DPC_LEAF_SIZES && st == DPC_OK; ++c) {
        set_leaf_log2(d, kMinLeafLog2 + c);
        st = time_choice(points, n, d, d_cut, rho_min, delta_min, DPC_BACKEND_PRIORITY_TREE, stream, &best_ms[c]);
    }
    if (st != DPC_OK) {
        set_leaf_log2(d, before);
        return st;
    }
    int pick = 0;
    for (int c = 1; c < DPC_LEAF_SIZES; ++c)
        pick = best_ms[c] < best_ms[pick] ? c : pick;
    pick += kMinLeafLog2;
    set_leaf_log2(d, pick);
    if (ms_out) {
        for (int c = 0; c < DPC_LEAF_SIZES; ++c)
            ms_out[c] = best_ms[c];
    }
    if (chosen)
        *chosen = 1 << pick;
    return DPC_OK;
}

int dpc_set_dependent_backend(int32_t d, int32_t backend) {
    if (d < 1 || d > kMaxDim || backend < DPC_BACKEND_PRIORITY_TREE || backend >= DPC_BACKENDS)
        return DPC_ERR_INVALID_ARG;
    g_backend[d].store(backend, std::memory_order_relaxed);
    return DPC_OK;
}

int32_t dpc_dependent_backend(int32_t d) {
    if (d < 1 || d > kMaxDim)
        return -1;
    return g_backend[d].load(std::memory_order_relaxed);
}

int dpc_autotune_dependent(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min,
                           double delta_min, hipStream_t stream, double *ms_out, int32_t *chosen) {
    if (bad_shape(n, d) || n == 0 || points == nullptr)
        return DPC_ERR_INVALID_ARG;
    float best_ms[DPC_BACKENDS] = {};
    int pick = DPC_BACKEND_PRIORITY_TREE;
    for (int c = 0; c < DPC_BACKENDS; ++c) {
        DPC_TRY(time_choice(points, n, d, d_cut, rho_min, delta_min, c, stream, &best_ms[c]));
        if (best_ms[c] < best_ms[pick])
            pick = c;
    }
    g_backend[d].store(pick, std::memory_order_relaxed);
    if (ms_out)
        for (int c = 0; c < DPC_BACKENDS; ++c)
            ms_out[c] = best_ms[c];
    if (chosen)
        *chosen = pick;
    return DPC_OK;
}

int dpc_plan_create(const int32_t *points, int64_t n, int32_t d, double d_cut, int32_t rho_min, double delta_min,
                    uint32_t flags, int32_t *rho, int32_t *dep, int64_t *delta2, int32_t *label, hipStream_t stream,
                    dpc_plan **out) {
    if (out == nullptr)
        return DPC_ERR_INVALID_ARG;
    *out = nullptr;
    if (flags & ~(uint32_t)DPC_SKIP_NOISE_DEPENDENTS)
        return DPC_ERR_INVALID_ARG;
    Job J;
    DPC_TRY(make_job(points, n, d, d_cut, rho_min, delta_min, flags, rho, dep, delta2, label, J));
    dpc_plan *pl = new (std::nothrow) dpc_plan;
    if (pl == nullptr)
        return DPC_ERR_OOM;
    pl->ws = new (std::nothrow) Workspace(stream);
    if (pl->ws == nullptr) {
        delete pl;
        return DPC_ERR_OOM;
    }
    pl->ws->cap = std::numeric_limits<int>::max();
    dpc_status st = DPC_OK;
    if (n > 0) {
        st = pl->ws->alloc(&pl->status, 1);
        if (st == DPC_OK) {
            t_record = &pl->ops;
            t_plan_status = pl->status;
            launch(k_plan_clear, dim3(1), dim3(kWave), 0, stream, pl->status);
            std::vector<Job> jobs{J};
            st = job_bounds(jobs, d, *pl->ws, nullptr);
            if (st == DPC_OK)
                st = run_group(jobs, d, job_arith(jobs[0], d), nullptr, nullptr, *pl->ws);
            t_record = nullptr;
            t_plan_status = nullptr;
        }
        if (st == DPC_OK && hipStreamSynchronize(stream) != hipSuccess)
            st = DPC_ERR_HIP;
    }
    if (st != DPC_OK) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(stream);
        delete pl->ws;
        delete pl;
        return st;
    }
    *out = pl;
    return DPC_OK;
}

int dpc_plan_create_batch(dpc_instance *instances, int32_t count, uint32_t flags, hipStream_t stream,
                          dpc_plan **out) {
    if (out == nullptr)
        return DPC_ERR_INVALID_ARG;
    *out = nullptr;
    if (count < 0 || (count > 0 && instances == nullptr) || (flags & ~(uint32_t)DPC_SKIP_NOISE_DEPENDENTS))
        return DPC_ERR_INVALID_ARG;
    // every instance must be valid: the plan replays all of them
    int first = DPC_OK;
    for (int i = 0; i < count; ++i) {
        instances[i].status = check_instance(instances[i], flags);
        if (instances[i].status != DPC_OK && first == DPC_OK)
            first = instances[i].status;
    }
    if (first != DPC_OK)
        return first;
    dpc_plan *pl = new (std::nothrow) dpc_plan;
    if (pl == nullptr)
        return DPC_ERR_OOM;
    pl->ws = new (std::nothrow) Workspace(stream);
    if (pl->ws == nullptr) {
        delete pl;
        return DPC_ERR_OOM;
    }
    pl->ws->cap = std::numeric_limits<int>::max();
    dpc_status st = pl->ws->alloc(&pl->status, 1);
    if (st == DPC_OK) {
        t_record = &pl->ops;
        t_plan_status = pl->status;
        launch(k_plan_clear, dim3(1), dim3(kWave), 0, stream, pl->status);
        std::vector<uint32_t> fl((size_t)count, flags);
        st = run_instances(instances, fl.data(), count, stream, nullptr, pl->ws);
        t_record = nullptr;
        t_plan_status = nullptr;
    }
    if (st == DPC_OK && hipStreamSynchronize(stream) != hipSuccess)
        st = DPC_ERR_HIP;
    if (st != DPC_OK) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(stream);
        delete pl->ws;
        delete pl;
        return st;
    }
    *out = pl;
    return DPC_OK;
}

int dpc_plan_launch(dpc_plan *plan, hipStream_t stream) {
    if (plan == nullptr)
        return DPC_ERR_INVALID_ARG;
    if (plan->exec) {
        DPC_HIP(hipGraphLaunch(plan->exec, stream));
        return DPC_OK;
    }
    for (auto &op : plan->ops)
        op(stream);
    DPC_HIP(hipGetLastError());
    return DPC_OK;
}

int dpc_plan_capture(dpc_plan *plan, hipStream_t stream) {
    if (plan == nullptr || stream == nullptr || plan->exec != nullptr)
        return DPC_ERR_INVALID_ARG;
    DPC_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    for (auto &op : plan->ops)
        op(stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(stream, &g);
    if (e != hipSuccess || g == nullptr) {
        (void)hipGetLastError();
        return DPC_ERR_HIP;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(g);
        return DPC_ERR_HIP;
    }
    plan->graph = g;
    plan->exec = x;
    return DPC_OK;
}

int dpc_plan_status(dpc_plan *plan, hipStream_t stream, int32_t *status) {
    if (plan == nullptr || status == nullptr)
        return DPC_ERR_INVALID_ARG;
    *status = DPC_OK;
    if (plan->status == nullptr)
        return DPC_OK;
    int32_t h = 0;
    DPC_HIP(hipMemcpyAsync(&h, plan->status, sizeof(h), hipMemcpyDeviceToHost, stream));
    DPC_HIP(hipStreamSynchronize(stream));
    *status = h;
    return DPC_OK;
}

int dpc_plan_destroy(dpc_plan *plan) {
    if (plan == nullptr)
        return DPC_ERR_INVALID_ARG;
    // replays may have run on any stream: let them finish before the
    // workspace goes back to the pool
    (void)hipDeviceSynchronize();
    if (plan->exec)
        (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph)
        (void)hipGraphDestroy(plan->graph);
    // the creating stream may be gone by now; the device is idle
    plan->ws->stream = nullptr;
    delete plan->ws;
    (void)hipStreamSynchronize(nullptr);
    delete plan;
    return DPC_OK;
}

int dpc_last_stats(dpc_stats *out) {
    if (out == nullptr)
        return DPC_ERR_INVALID_ARG;
    return RunRecorder::last(out);
}

}  // extern "C"
