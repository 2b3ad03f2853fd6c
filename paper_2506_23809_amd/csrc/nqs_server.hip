// Serving runtime: a request loop with continuous batching over resident
// Pauli tables.
//
// One dispatcher thread owns the device work.  The device is divided into
// lanes: each lane is a stream with its own evaluation scratch (sample
// hash, partial sums, filters, enumeration areas, pair-join buckets) and its
// own counters and error latch, all allocated when handles are registered.
// Pending requests wait in arrival order; whenever a lane is free the
// dispatcher admits the oldest request whose footprint fits the HBM budget
// and launches it on that lane, with the plan nqs_eloc_eval would take (so
// the device picks the pair join, the enumeration or streaming per
// request).  Lanes run concurrently, so requests that arrive while others
// run join the device's work as soon as a lane frees up, whatever
// Hamiltonian they use (two requests for one handle overlap on two lanes).
// Each request completes on its own lane event, seen with hipEventQuery; a
// small request never waits for a large one that started with it.  Nothing
// in the loop allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/nqs.h"
#include "nqs_device.hpp"
#include "nqs_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;
constexpr int64_t kBytesPerSample = 16 + 8 + 8 + 8 + 16;  // samples, a, phi, count, E_loc

struct SrvRequest {
    int64_t ticket;
    nqs_batch_item item;
    int64_t bytes;
    Clock::time_point t_submit;
};

struct Lane {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    SrvRequest req{};
    char *ctx = nullptr;  // evaluation scratch
    size_t ctx_bytes = 0;
    void *small = nullptr;  // counters, error latch, sector flag
    int *h_err = nullptr;   // pinned copy of the lane's error latch after a request
};

struct Registered {
    int64_t table_bytes;
    int64_t max_samples;
};

}  // namespace

struct nqs_server_s {
    nqs_server_config cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;       // wakes the dispatcher
    std::condition_variable done_cv;  // wakes drain()
    std::deque<SrvRequest> pending;
    std::vector<std::pair<int64_t, double>> finished;
    std::unordered_map<nqs_ham, Registered> resident;
    int64_t resident_bytes = 0;  // tables plus the lanes' scratch
    int64_t lane_bytes = 0;      // scratch of all lanes
    int64_t inflight_bytes = 0;
    std::vector<Lane> lanes;
    std::thread worker;
    bool stop = false;
    int error = 0;
    std::string error_msg;
    int64_t next_ticket = 1;
    // statistics
    int64_t submitted = 0, completed = 0, rejected = 0, launches = 0;
    int64_t max_reqs_inflight = 0, max_launches_inflight = 0, peak_bytes = 0;
    int64_t reqs_inflight = 0;
};

namespace {

int fail(int code, const std::string &msg) { return nqs::detail::fail(code, msg); }

void free_lane(Lane &l) {
    if (l.done) (void)hipEventDestroy(l.done);
    if (l.st) (void)hipStreamDestroy(l.st);
    if (l.ctx) (void)hipFree(l.ctx);
    if (l.small) (void)hipFree(l.small);
    if (l.h_err) (void)hipHostFree(l.h_err);
    l = Lane{};
}

// Launch the lane's request (called without the server lock).  After the
// evaluation the lane's error word is copied to pinned memory, then the
// lane's event is recorded: the request is done when the event is.
int launch_lane(nqs_server s, Lane &l) {
    const nqs_batch_item &it = l.req.item;
    int rc = nqs::detail::eval_in(it.ham, it, s->cfg.precision, l.ctx, l.ctx_bytes, l.small, l.st);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(l.h_err, static_cast<char *>(l.small) + nqs::detail::small_err_offset(),
                                  sizeof(int), hipMemcpyDeviceToHost, l.st);
    if (e == hipSuccess) e = hipEventRecord(l.done, l.st);
    if (e != hipSuccess) return fail(NQS_E_DEVICE, std::string("serving launch: ") + hipGetErrorString(e));
    nqs::detail::mark_evaluated(it.ham, it.n);
    return NQS_OK;
}

// Called with the lock held once a lane's request has completed.
void retire_lane(nqs_server s, Lane &l, const Clock::time_point now, bool ok) {
    const double us =
        ok ? std::chrono::duration<double, std::micro>(now - l.req.t_submit).count() : -1.0;
    if (ok && *l.h_err != 0) {
        // a device-detected error of this request (duplicate samples, bits
        // out of range): latched on its handle for nqs_sync; the lane's latch
        // is cleared on its stream before the lane's next request
        nqs::detail::latch_host_error(l.req.item.ham, *l.h_err);
        *l.h_err = 0;
        (void)hipMemsetAsync(static_cast<char *>(l.small) + nqs::detail::small_err_offset(), 0,
                             sizeof(int), l.st);
    }
    s->finished.emplace_back(l.req.ticket, us);
    s->completed += 1;
    s->reqs_inflight -= 1;
    s->inflight_bytes -= l.req.bytes;
    l.busy = false;
}

void dispatcher(nqs_server s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // 1. retire finished requests
        const Clock::time_point now = Clock::now();
        bool retired = false;
        for (Lane &l : s->lanes) {
            if (!l.busy) continue;
            const hipError_t q = hipEventQuery(l.done);
            if (q == hipSuccess) {
                retire_lane(s, l, now, true);
                retired = true;
            } else if (q != hipErrorNotReady) {
                s->error = NQS_E_DEVICE;
                s->error_msg = std::string("serving launch failed: ") + hipGetErrorString(q);
                retire_lane(s, l, now, false);
                retired = true;
            }
        }
        if (retired) s->done_cv.notify_all();
        bool any_busy = false;
        for (const Lane &l : s->lanes) any_busy = any_busy || l.busy;
        if (s->error && !s->pending.empty()) {
            // after a failed launch nothing more is admitted: fail the queue
            for (const SrvRequest &r : s->pending) s->finished.emplace_back(r.ticket, -1.0);
            s->completed += static_cast<int64_t>(s->pending.size());
            s->pending.clear();
            s->done_cv.notify_all();
        }
        if (s->stop && s->pending.empty() && !any_busy) break;

        // 2. admit the oldest request that fits into each free lane
        bool launched = false;
        for (Lane &l : s->lanes) {
            if (l.busy || s->pending.empty() || s->error) continue;
            auto it = s->pending.begin();
            while (it != s->pending.end() &&
                   s->resident_bytes + s->inflight_bytes + it->bytes > s->cfg.hbm_budget_bytes)
                ++it;
            if (it == s->pending.end()) break;
            l.req = *it;
            s->pending.erase(it);
            l.busy = true;
            s->inflight_bytes += l.req.bytes;
            s->reqs_inflight += 1;
            s->launches += 1;
            s->max_reqs_inflight = std::max(s->max_reqs_inflight, s->reqs_inflight);
            s->max_launches_inflight = s->max_reqs_inflight;
            s->peak_bytes = std::max(s->peak_bytes, s->resident_bytes + s->inflight_bytes);
            lk.unlock();
            const int rc = launch_lane(s, l);
            lk.lock();
            if (rc) {
                s->error = rc;
                s->error_msg = "serving launch could not be planned or enqueued";
                retire_lane(s, l, Clock::now(), false);
                s->done_cv.notify_all();
            }
            launched = true;
        }
        if (launched) continue;
        // 3. wait: poll completions while requests run, sleep when idle
        if (any_busy)
            s->cv.wait_for(lk, std::chrono::microseconds(20));
        else
            s->cv.wait(lk, [s] { return s->stop || (!s->pending.empty() && !s->error); });
    }
}

}  // namespace

extern "C" {

int nqs_server_create(nqs_server *out, const nqs_server_config *cfg) {
    if (!out || !cfg) return fail(NQS_E_ARG, "null argument");
    *out = nullptr;
    nqs_server_config c = *cfg;
    if (c.streams == 0) c.streams = 4;
    if (c.hbm_budget_bytes <= 0 || c.streams < 1 || c.streams > 8 ||
        (c.precision != NQS_FP64 && c.precision != NQS_FP32_KAHAN))
        return fail(NQS_E_ARG, "server configuration out of range");
    nqs_server s = new (std::nothrow) nqs_server_s();
    if (!s) return fail(NQS_E_NOMEM, "host allocation failed");
    s->cfg = c;
    hipError_t e = hipGetDevice(&s->device);
    s->lanes.resize(c.streams);
    for (Lane &l : s->lanes) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&l.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&l.small, nqs::detail::small_bytes());
        if (e == hipSuccess) e = hipMemset(l.small, 0, nqs::detail::small_bytes());
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&l.h_err), sizeof(int), hipHostMallocDefault);
        if (e == hipSuccess) *l.h_err = 0;
    }
    if (e != hipSuccess) {
        for (Lane &l : s->lanes) free_lane(l);
        delete s;
        return fail(NQS_E_DEVICE, std::string("creating the server: ") + hipGetErrorString(e));
    }
    s->lane_bytes = static_cast<int64_t>(nqs::detail::small_bytes()) * c.streams;
    s->resident_bytes = s->lane_bytes;
    s->worker = std::thread(dispatcher, s);
    *out = s;
    return NQS_OK;
}

int nqs_server_add_ham(nqs_server s, nqs_ham h, int64_t max_samples) {
    if (!s) return fail(NQS_E_STATE, "invalid server");
    if (!nqs::detail::valid_handle(h)) return fail(NQS_E_ARG, "invalid handle");
    if (max_samples < 1) return fail(NQS_E_ARG, "max_samples must be positive");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->resident.count(h)) return fail(NQS_E_ARG, "handle already registered");
    const int64_t table = nqs::detail::table_bytes(h);
    const int64_t small = static_cast<int64_t>(nqs::detail::small_bytes()) * s->cfg.streams;
    // every lane must hold this handle's largest request
    const size_t need = nqs::detail::request_scratch_bytes(h, max_samples);
    const size_t have = s->lanes[0].ctx_bytes;
    const int64_t lanes_after =
        small + static_cast<int64_t>(std::max(need, have)) * s->cfg.streams;
    if (s->resident_bytes - s->lane_bytes + lanes_after + table > s->cfg.hbm_budget_bytes)
        return fail(NQS_E_NOMEM, "resident tables and lane scratch would exceed the HBM budget");
    if (need > have) {
        for (const Lane &l : s->lanes)
            if (l.busy) return fail(NQS_E_STATE, "lanes are running: register handles first");
        bool ok = true;
        for (Lane &l : s->lanes) {
            if (l.ctx) (void)hipFree(l.ctx);
            l.ctx = nullptr;
            l.ctx_bytes = 0;
            if (ok && hipMalloc(reinterpret_cast<void **>(&l.ctx), need) == hipSuccess)
                l.ctx_bytes = need;
            else
                ok = false;
        }
        if (!ok) {
            // no lane keeps scratch it cannot use: all empty, nothing admitted
            // until a registration succeeds
            for (Lane &l : s->lanes) {
                if (l.ctx) (void)hipFree(l.ctx);
                l.ctx = nullptr;
                l.ctx_bytes = 0;
            }
            s->resident_bytes += small - s->lane_bytes;
            s->lane_bytes = small;
            for (auto &kv : s->resident) kv.second.max_samples = 0;
            return fail(NQS_E_NOMEM, "allocating the lanes' scratch");
        }
        s->resident_bytes += lanes_after - s->lane_bytes;
        s->lane_bytes = lanes_after;
    }
    s->resident[h] = Registered{table, max_samples};
    s->resident_bytes += table;
    return NQS_OK;
}

int nqs_server_submit(nqs_server s, const nqs_batch_item *req, int64_t *ticket) {
    if (!s) return fail(NQS_E_STATE, "invalid server");
    if (!req || !ticket) return fail(NQS_E_ARG, "null argument");
    if (req->n < 0 || req->n > (int64_t(1) << 30)) return fail(NQS_E_ARG, "bad batch size");
    if (req->n > 0 && (!req->samples || !req->log_amp || !req->phase || !req->eloc))
        return fail(NQS_E_ARG, "null pointer in request");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(NQS_E_STATE, "server is stopping");
    if (s->error) return fail(NQS_E_STATE, "server failed: " + s->error_msg);
    const auto reg = s->resident.find(req->ham);
    if (reg == s->resident.end()) return fail(NQS_E_ARG, "handle not registered with the server");
    if (req->n > reg->second.max_samples)
        return fail(NQS_E_ARG, "request larger than the handle's registered max_samples");
    SrvRequest r;
    r.ticket = s->next_ticket++;
    r.item = *req;
    r.bytes = kBytesPerSample * req->n;
    r.t_submit = Clock::now();
    if (s->resident_bytes + r.bytes > s->cfg.hbm_budget_bytes) {
        s->rejected += 1;
        return fail(NQS_E_NOMEM, "request can never fit the HBM budget");
    }
    s->pending.push_back(r);
    s->submitted += 1;
    *ticket = r.ticket;
    s->cv.notify_one();
    return NQS_OK;
}

int nqs_server_poll(nqs_server s, int64_t *tickets, double *latency_us, int capacity,
                    int *n_out) {
    if (!s) return fail(NQS_E_STATE, "invalid server");
    if (!n_out || capacity < 0 || (capacity > 0 && (!tickets || !latency_us)))
        return fail(NQS_E_ARG, "bad output buffers");
    std::lock_guard<std::mutex> lk(s->mu);
    const int m = std::min<int>(capacity, static_cast<int>(s->finished.size()));
    for (int k = 0; k < m; ++k) {
        tickets[k] = s->finished[k].first;
        latency_us[k] = s->finished[k].second;
    }
    s->finished.erase(s->finished.begin(), s->finished.begin() + m);
    *n_out = m;
    if (s->error) return fail(s->error, "server: " + s->error_msg);
    return NQS_OK;
}

int nqs_server_drain(nqs_server s, double timeout_s) {
    if (!s) return fail(NQS_E_STATE, "invalid server");
    std::unique_lock<std::mutex> lk(s->mu);
    const auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                             std::chrono::duration<double>(timeout_s));
    while (s->completed < s->submitted && !s->error) {
        if (s->done_cv.wait_until(lk, deadline) == std::cv_status::timeout &&
            s->completed < s->submitted)
            return fail(NQS_E_STATE, "timed out waiting for requests");
    }
    if (s->error) return fail(s->error, "server: " + s->error_msg);
    return NQS_OK;
}

int nqs_server_stats(nqs_server s, int64_t out[8]) {
    if (!s) return fail(NQS_E_STATE, "invalid server");
    if (!out) return fail(NQS_E_ARG, "null output");
    std::lock_guard<std::mutex> lk(s->mu);
    out[0] = s->submitted;
    out[1] = s->completed;
    out[2] = s->rejected;
    out[3] = s->launches;
    out[4] = s->max_reqs_inflight;
    out[5] = s->max_launches_inflight;
    out[6] = s->peak_bytes;
    out[7] = s->resident_bytes;
    return NQS_OK;
}

int nqs_server_destroy(nqs_server s) {
    if (!s) return NQS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (Lane &l : s->lanes) {
        if (l.st) (void)hipStreamSynchronize(l.st);
        free_lane(l);
    }
    const int err = s->error;
    delete s;
    return err ? fail(err, "server stopped after an error") : NQS_OK;
}

}  // extern "C"
