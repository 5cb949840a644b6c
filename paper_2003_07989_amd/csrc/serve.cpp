// serve.cpp -- a serving loop for barcode requests with continuous admission.
//
// S slots run requests concurrently, each on its own HIP stream with its own
// device workspace, so the GPU stages of different requests overlap on the
// device and their filtrations and clearing state stay resident in the
// slot's HBM buffers until they finish.  A request is admitted as soon as a
// slot is free and its footprint fits the HBM budget -- requests that
// arrive while others run join immediately, without waiting for a batch to
// drain.  The queue is scanned in arrival order and the first request that
// fits is admitted.
//
// Memory accounting.  A running slot holds a reservation: the device bytes
// its workspace and input buffer may reach during the request, enforced by
// the workspace's own limit.  An idle slot holds what its buffers retain from
// earlier requests (grow-only buffers are what lets a warm server allocate
// nothing).  A request fits when the reservations of the running slots, the
// retained bytes of the idle ones and its own reservation stay within the
// budget.  Its reservation is its footprint bound (rpp_workspace_bytes +
// input) on top of what the slot already retains, or, if that does not fit,
// the bound alone once the slot's buffers are freed; if even that does not
// fit, the buffers of the other idle slots are freed too.  So the device
// memory held by the slots never passes the budget, except for a request
// whose bound alone exceeds it, which runs by itself, without a limit, when
// nothing else is in flight.  Per request the server records the time spent
// queued and the latency from submission to completion.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/rpp.h"
#include "host_common.h"
#include "pipeline.h"

namespace rpp {
int build_result_public(const RunOut &ro, int n, int maxdim, uint32_t flags, rpp_result **out);
void set_last_error(const std::string &msg);
}

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    std::vector<float> dist;  // host copy
    int n = 0, maxdim = 0;
    float threshold = 0.0f;
    uint32_t flags = 0;
    size_t need = 0;  // footprint bound
    Clock::time_point submitted, started, finished;
    bool done = false;
    int rc = RPP_OK;
    std::string err;
    rpp_result *result = nullptr;
    int slot = -1;
    std::atomic<bool> cancel{false};
};

}  // namespace

struct rpp_server {
    std::mutex mu;
    std::condition_variable work_cv, done_cv;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<uint64_t, std::shared_ptr<Request>> tickets;
    uint64_t next_ticket = 1;
    size_t budget = 0, in_flight = 0, peak_in_flight = 0;
    int running = 0, peak_running = 0;
    int64_t admitted = 0, completed = 0;
    bool stop = false;
    int device = 0;
    std::vector<std::thread> slots;
    std::vector<void *> workspaces;
    std::vector<hipStream_t> streams;
    std::vector<float *> dev_in;
    std::vector<size_t> dev_in_cap;
    std::vector<size_t> reserve;  // running slot: its reservation; idle: 0
    size_t peak_allocated = 0;

    // Device bytes slot k retains (its workspace buffers and input buffer).
    size_t retained(int k) { return rpp::workspace_allocated(workspaces[k]) + dev_in_cap[k]; }

    // Bytes counted against the budget by every slot except k.
    size_t committed_except(int k)
    {
        size_t t = 0;
        for (int j = 0; j < (int)workspaces.size(); ++j)
            if (j != k)
                t += reserve[j] ? reserve[j] : retained(j);
        return t;
    }

    void free_slot(int j)
    {
        rpp::workspace_trim(workspaces[j]);
        if (dev_in[j]) {
            (void)hipStreamSynchronize(streams[j]);
            (void)hipFree(dev_in[j]);
        }
        dev_in[j] = nullptr;
        dev_in_cap[j] = 0;
    }

    // Admission of r on idle slot k: 0 = does not fit now; otherwise the
    // reservation (the slot's buffers trimmed first when `trim` comes back
    // true, the other idle slots' when `trim_others` does).
    size_t plan(const Request &r, int k, bool *trim, bool *trim_others)
    {
        *trim = *trim_others = false;
        const size_t in_bytes = rpp::grow_capacity(0, r.dist.size() * sizeof(float));
        const size_t others = committed_except(k);
        const size_t keep = retained(k) + r.need;
        if (others + keep <= budget)
            return keep;
        const size_t fresh = in_bytes + (r.need - r.dist.size() * sizeof(float));
        *trim = true;
        if (others + fresh <= budget)
            return fresh;
        size_t busy = 0;
        for (int j = 0; j < (int)workspaces.size(); ++j)
            if (j != k && reserve[j])
                busy += reserve[j];
        *trim_others = true;
        if (busy + fresh <= budget || running == 0)
            return fresh;
        return 0;
    }

    void slot_loop(int k)
    {
        (void)hipSetDevice(device);
        while (true) {
            std::shared_ptr<Request> r;
            {
                std::unique_lock<std::mutex> lk(mu);
                bool trim = false, trim_others = false;
                size_t res = 0;
                auto pick = [&]() {
                    for (auto it = queue.begin(); it != queue.end(); ++it)
                        if ((res = plan(**it, k, &trim, &trim_others)) != 0)
                            return it;
                    return queue.end();
                };
                auto it = queue.end();
                work_cv.wait(lk, [&] { return stop || (it = pick()) != queue.end(); });
                if (it == queue.end()) {
                    if (stop && queue.empty())
                        return;
                    continue;
                }
                r = *it;
                queue.erase(it);
                if (trim_others)
                    for (int j = 0; j < (int)workspaces.size(); ++j)
                        if (j != k && !reserve[j])
                            free_slot(j);
                if (trim)
                    free_slot(k);
                const bool oversize = r->need > budget;
                reserve[k] = res;
                // the workspace's share: the reservation less the input buffer
                const size_t in_bytes =
                    std::max(dev_in_cap[k], rpp::grow_capacity(0, r->dist.size() * sizeof(float)));
                rpp::workspace_set_limit(workspaces[k],
                                         oversize ? SIZE_MAX : res - std::min(res, in_bytes));
                in_flight += res;
                peak_in_flight = std::max(peak_in_flight, in_flight);
                ++running;
                peak_running = std::max(peak_running, running);
                ++admitted;
                r->slot = k;
                r->started = Clock::now();
            }
            execute(k, *r);
            {
                std::lock_guard<std::mutex> lk(mu);
                peak_allocated = std::max(peak_allocated, allocated_locked());
                in_flight -= reserve[k];
                reserve[k] = 0;
                --running;
                ++completed;
                r->finished = Clock::now();
                r->done = true;
            }
            done_cv.notify_all();
            work_cv.notify_all();
        }
    }

    size_t allocated_locked()
    {
        size_t t = 0;
        for (size_t k = 0; k < workspaces.size(); ++k)
            t += retained((int)k);
        return t;
    }

    void execute(int k, Request &r)
    {
        if (r.cancel.load()) {
            r.rc = RPP_E_CANCELLED;
            r.err = "request cancelled";
            return;
        }
        const size_t m = r.dist.size();
        hipStream_t s = streams[k];
        if (m * sizeof(float) > dev_in_cap[k]) {  // capacity is in bytes
            if (dev_in[k]) {
                (void)hipStreamSynchronize(s);
                (void)hipFree(dev_in[k]);
            }
            dev_in[k] = nullptr;
            dev_in_cap[k] = 0;
            const size_t b = rpp::grow_capacity(0, m * sizeof(float));
            if (hipMalloc(&dev_in[k], b) != hipSuccess) {
                dev_in[k] = nullptr;
                r.rc = RPP_E_NOMEM;
                r.err = "hipMalloc of the request input failed";
                return;
            }
            dev_in_cap[k] = b;
        }
        if (m && hipMemcpyAsync(dev_in[k], r.dist.data(), m * sizeof(float),
                                hipMemcpyHostToDevice, s) != hipSuccess) {
            r.rc = RPP_E_DEVICE;
            r.err = "hipMemcpyAsync of the request input failed";
            return;
        }
        rpp::RunArgs a;
        a.dcond_dev = dev_in[k];
        a.n = r.n;
        a.maxdim = r.maxdim;
        a.threshold = r.threshold;
        a.flags = r.flags;
        a.stream = s;
        a.workspace = workspaces[k];
        a.cancel = &r.cancel;
        rpp::RunOut ro;
        r.rc = rpp::run_pipeline(a, ro, r.err);
        if (r.rc == RPP_OK)
            r.rc = rpp::build_result_public(ro, r.n, r.maxdim, r.flags, &r.result);
    }
};

extern "C" {

int rpp_server_create(int32_t slots, size_t hbm_budget_bytes, rpp_server **out)
{
    if (!out || slots < 1 || slots > 64)
        return RPP_E_INVAL;
    *out = nullptr;
    auto *sv = new (std::nothrow) rpp_server();
    if (!sv)
        return RPP_E_NOMEM;
    (void)hipGetDevice(&sv->device);
    if (hbm_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete sv;
            return RPP_E_DEVICE;
        }
        hbm_budget_bytes = fr / 4 * 3;
    }
    sv->budget = hbm_budget_bytes;
    for (int k = 0; k < slots; ++k) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            rpp_server_destroy(sv);
            return RPP_E_DEVICE;
        }
        sv->streams.push_back(s);
        sv->workspaces.push_back(rpp::workspace_new());
        sv->dev_in.push_back(nullptr);
        sv->dev_in_cap.push_back(0);
        sv->reserve.push_back(0);
    }
    for (int k = 0; k < slots; ++k)
        sv->slots.emplace_back([sv, k] { sv->slot_loop(k); });
    *out = sv;
    return RPP_OK;
}

int rpp_server_submit(rpp_server *sv, const float *dist, int32_t n, int32_t maxdim,
                      float threshold, uint32_t flags, uint64_t *ticket)
{
    if (!sv || !ticket || n < 1 || maxdim < 0 || maxdim > RPP_MAX_DIM || (n > 1 && !dist))
        return RPP_E_INVAL;
    if (threshold != threshold || threshold < 0.0f)
        return RPP_E_INVAL;
    auto r = std::make_shared<Request>();
    const size_t m = (size_t)n * (n - 1) / 2;
    try {
        r->dist.assign(dist, dist + m);
    } catch (const std::bad_alloc &) {
        return RPP_E_NOMEM;
    }
    for (size_t i = 0; i < m; ++i)
        if (!(r->dist[i] >= 0.0f) || r->dist[i] == INFINITY)
            return RPP_E_DATA;
    r->n = n;
    r->maxdim = maxdim;
    r->threshold = threshold;
    r->flags = flags & ~(uint32_t)RPP_WANT_PAIRS;
    r->need = rpp_workspace_bytes(n, maxdim, threshold) + m * sizeof(float);
    r->submitted = Clock::now();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        r->ticket = sv->next_ticket++;
        sv->tickets[r->ticket] = r;
        sv->queue.push_back(r);
        *ticket = r->ticket;
    }
    sv->work_cv.notify_all();
    return RPP_OK;
}

int rpp_server_wait(rpp_server *sv, uint64_t ticket, rpp_result **out, double *latency_ms,
                    double *queue_ms)
{
    if (!sv || !out)
        return RPP_E_INVAL;
    *out = nullptr;
    std::shared_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        auto it = sv->tickets.find(ticket);
        if (it == sv->tickets.end())
            return RPP_E_INVAL;
        r = it->second;
        sv->done_cv.wait(lk, [&] { return r->done; });
        sv->tickets.erase(ticket);
    }
    if (latency_ms)
        *latency_ms = std::chrono::duration<double, std::milli>(r->finished - r->submitted).count();
    if (queue_ms)
        *queue_ms = std::chrono::duration<double, std::milli>(r->started - r->submitted).count();
    if (r->rc != RPP_OK) {
        rpp::set_last_error("request " + std::to_string(ticket) + ": " + r->err);
        return r->rc;
    }
    *out = r->result;
    r->result = nullptr;
    return RPP_OK;
}

int rpp_server_cancel(rpp_server *sv, uint64_t ticket)
{
    if (!sv)
        return RPP_E_INVAL;
    std::shared_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->tickets.find(ticket);
        if (it == sv->tickets.end() || it->second->done)
            return RPP_E_INVAL;
        r = it->second;
        r->cancel.store(true);
        auto q = std::find(sv->queue.begin(), sv->queue.end(), r);
        if (q != sv->queue.end()) {
            // never admitted: finished here
            sv->queue.erase(q);
            r->rc = RPP_E_CANCELLED;
            r->err = "request cancelled";
            r->started = r->finished = Clock::now();
            r->done = true;
        }
    }
    sv->done_cv.notify_all();
    sv->work_cv.notify_all();
    return RPP_OK;
}

int rpp_server_stats(rpp_server *sv, rpp_server_info *st)
{
    if (!sv || !st)
        return RPP_E_INVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    st->slots = (int32_t)sv->slots.size();
    st->budget_bytes = sv->budget;
    st->in_flight_bytes = sv->in_flight;
    st->peak_in_flight_bytes = sv->peak_in_flight;
    st->peak_allocated_bytes = std::max(sv->peak_allocated, sv->allocated_locked());
    st->peak_concurrency = sv->peak_running;
    st->admitted = sv->admitted;
    st->completed = sv->completed;
    st->queued = (int64_t)sv->queue.size();
    return RPP_OK;
}

void rpp_server_destroy(rpp_server *sv)
{
    if (!sv)
        return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->work_cv.notify_all();
    for (auto &t : sv->slots)
        t.join();
    for (auto &kv : sv->tickets)
        if (kv.second->result)
            rpp_result_free(kv.second->result);
    for (size_t k = 0; k < sv->streams.size(); ++k) {
        (void)hipStreamSynchronize(sv->streams[k]);
        if (sv->dev_in[k])
            (void)hipFree(sv->dev_in[k]);
        rpp::workspace_delete(sv->workspaces[k]);
        (void)hipStreamDestroy(sv->streams[k]);
    }
    delete sv;
}

}  // extern "C"
