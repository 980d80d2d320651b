// Served clustering: requests (independent instances) arrive one by one and
// are run in batches as device memory and batch slots free up (continuous
// batching).  Each slot is a host thread with a HIP stream of its own, so
// several batches are in flight on the device at once; a request that
// arrives while they run joins the next batch that any slot forms.
// Admission is first come, first served, bounded by the summed footprint of
// the admitted requests: each one's workspace bound (workspace_bound, which
// the batch workspaces never exceed) plus its own input and output arrays
// (4d + 20 bytes per point), all of which are resident while it runs.  A batch is one run_instances call (the batched
// path of dpc_batch_run), so every request's outputs are those of dpc_run
// with the same arguments, whatever it was batched with.
#include "dpc_internal.hpp"

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace dpc {
namespace {

int64_t now_ns() {
    return (int64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    dpc_instance inst;
    uint32_t flags;
    dpc_request_info info;
};

}  // namespace
}  // namespace dpc

struct dpc_server {
    int device = 0;
    uint64_t budget = 0;
    int max_batch = 1;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;

    std::mutex mu;
    std::condition_variable cv_work;  // a request arrived, memory freed, or stop
    std::condition_variable cv_done;  // a batch completed
    bool stop = false;
    uint64_t next_ticket = 1;
    uint64_t admitted = 0;  // summed footprint of the requests in flight
    int busy = 0;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, dpc::Request> reqs;
    dpc_server_stats stats = {};

    bool can_admit() const {
        return !pending.empty() && admitted + reqs.at(pending.front()).info.footprint <= budget;
    }

    void worker(int slot) {
        (void)hipSetDevice(device);
        hipStream_t stream = streams[slot];
        std::vector<uint64_t> batch;
        std::vector<dpc_instance> recs;
        std::vector<uint32_t> flags;
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_work.wait(lk, [&] { return can_admit() || (stop && pending.empty()); });
            if (!can_admit())
                break;  // stopping and nothing left
            // the longest prefix of the queue that fits
            batch.clear();
            recs.clear();
            flags.clear();
            uint64_t fp = 0;
            const int64_t t_admit = dpc::now_ns();
            while (!pending.empty() && (int)batch.size() < max_batch) {
                dpc::Request &r = reqs.at(pending.front());
                if (admitted + fp + r.info.footprint > budget)
                    break;
                fp += r.info.footprint;
                r.info.admit_ns = t_admit;
                batch.push_back(pending.front());
                recs.push_back(r.inst);
                flags.push_back(r.flags);
                pending.pop_front();
            }
            admitted += fp;
            ++busy;
            stats.batches += 1;
            stats.max_batch_seen = (int64_t)batch.size() > stats.max_batch_seen ? (int64_t)batch.size()
                                                                                 : stats.max_batch_seen;
            stats.max_slots_busy = busy > stats.max_slots_busy ? busy : stats.max_slots_busy;
            stats.max_admitted_bytes = admitted > stats.max_admitted_bytes ? admitted : stats.max_admitted_bytes;
            if (can_admit())
                cv_work.notify_one();  // another slot can start on the rest
            lk.unlock();

            size_t peak = 0;
            dpc_status st = dpc::run_instances(recs.data(), flags.data(), (int)recs.size(), stream, &peak);
            if (hipStreamSynchronize(stream) != hipSuccess) {
                (void)hipGetLastError();
                st = DPC_ERR_HIP;
            }
            const int64_t t_done = dpc::now_ns();

            lk.lock();
            admitted -= fp;
            --busy;
            stats.max_workspace_bytes = peak > stats.max_workspace_bytes ? peak : stats.max_workspace_bytes;
            if (peak > fp)
                stats.over_footprint += 1;
            const bool runtime_error = st == DPC_ERR_HIP || st == DPC_ERR_OOM;
            for (size_t k = 0; k < batch.size(); ++k) {
                dpc_request_info &info = reqs.at(batch[k]).info;
                info.status = recs[k].status;
                if (runtime_error && info.status == DPC_OK)
                    info.status = st;  // the batch failed before this request's outputs were written
                info.done = 1;
                info.done_ns = t_done;
                info.batch_size = (int32_t)batch.size();
                info.slot = slot;
            }
            stats.completed += (int64_t)batch.size();
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
};

using namespace dpc;

extern "C" {

int dpc_server_create(const dpc_server_config *cfg, dpc_server **out) {
    if (out == nullptr)
        return DPC_ERR_INVALID_ARG;
    *out = nullptr;
    if (cfg == nullptr || cfg->slots < 1 || cfg->slots > 16 || cfg->max_batch < 1 || cfg->hbm_budget_bytes == 0)
        return DPC_ERR_INVALID_ARG;
    int device = 0;
    DPC_HIP(hipGetDevice(&device));
    dpc_server *s = new (std::nothrow) dpc_server;
    if (s == nullptr)
        return DPC_ERR_OOM;
    try {
        s->streams.reserve(cfg->slots);
        s->workers.reserve(cfg->slots);
    } catch (...) {
        delete s;
        return DPC_ERR_OOM;
    }
    s->device = device;
    s->budget = cfg->hbm_budget_bytes;
    s->max_batch = cfg->max_batch;
    for (int k = 0; k < cfg->slots; ++k) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            for (hipStream_t t : s->streams)
                (void)hipStreamDestroy(t);
            delete s;
            return DPC_ERR_HIP;
        }
        s->streams.push_back(st);
    }
    try {
        for (int k = 0; k < cfg->slots; ++k)
            s->workers.emplace_back([s, k] { s->worker(k); });
    } catch (...) {
        (void)dpc_server_destroy(s);  // stops the workers already started
        return DPC_ERR_HIP;
    }
    *out = s;
    return DPC_OK;
}

int dpc_server_submit(dpc_server *s, const dpc_instance *req, uint32_t flags, uint64_t *ticket) {
    if (s == nullptr || req == nullptr || ticket == nullptr || (flags & ~(uint32_t)DPC_SKIP_NOISE_DEPENDENTS))
        return DPC_ERR_INVALID_ARG;
    *ticket = 0;
    dpc_instance probe = *req;
    DPC_TRY(check_instance(probe, flags));
    Request r;
    r.inst = *req;
    r.inst.status = -1;
    r.flags = flags;
    r.info = dpc_request_info{};
    // workspace, plus the caller's points (4d bytes per point) and the four
    // outputs (rho, dep, label 4 bytes each, delta2 8)
    r.info.footprint = workspace_bound(req->n, req->d) + (uint64_t)req->n * (4ull * (uint64_t)req->d + 20ull);
    r.info.submit_ns = now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    if (r.info.footprint > s->budget) {
        s->stats.rejected += 1;
        return DPC_ERR_OOM;
    }
    const uint64_t t = s->next_ticket++;
    try {
        s->reqs.emplace(t, r);
        s->pending.push_back(t);
    } catch (...) {
        s->reqs.erase(t);
        return DPC_ERR_OOM;
    }
    s->stats.submitted += 1;
    *ticket = t;
    s->cv_work.notify_one();
    return DPC_OK;
}

int dpc_server_poll(dpc_server *s, uint64_t ticket, dpc_request_info *info) {
    if (s == nullptr || info == nullptr)
        return DPC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return DPC_ERR_INVALID_ARG;
    *info = it->second.info;
    if (info->done)
        s->reqs.erase(it);
    return DPC_OK;
}

int dpc_server_wait(dpc_server *s, uint64_t ticket, dpc_request_info *info) {
    if (s == nullptr || info == nullptr)
        return DPC_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return DPC_ERR_INVALID_ARG;
    s->cv_done.wait(lk, [&] {
        auto f = s->reqs.find(ticket);
        return f == s->reqs.end() || f->second.info.done != 0;
    });
    it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return DPC_ERR_INVALID_ARG;  // another waiter took the result
    *info = it->second.info;
    s->reqs.erase(it);
    return DPC_OK;
}

int dpc_server_get_stats(dpc_server *s, dpc_server_stats *out) {
    if (s == nullptr || out == nullptr)
        return DPC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->in_flight_bytes = s->admitted;
    out->queued = (int64_t)s->pending.size();
    return DPC_OK;
}

int dpc_server_destroy(dpc_server *s) {
    if (s == nullptr)
        return DPC_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (std::thread &t : s->workers)
        t.join();
    for (hipStream_t t : s->streams)
        (void)hipStreamDestroy(t);
    delete s;
    return DPC_OK;
}

}  // extern "C"
