// Serving runtime: a request loop with continuous batching over resident
// Pauli tables.
//
// One dispatcher thread owns the device work.  Pending requests wait in
// arrival order; whenever a stream slot is free the dispatcher admits every
// request it can (handle not already running, footprint within the HBM
// budget, at most max_batch), plans them as one batched launch into the
// slot's preallocated descriptor buffers, uploads the plan from pinned
// staging and launches on the slot's stream.  Completion is seen with
// hipEventQuery, so slots refill as soon as their launch ends while other
// slots keep running.  Nothing in the loop allocates device memory once a
// slot's buffers have reached their working size.
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
#include <unordered_set>
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

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<SrvRequest> reqs;
    int64_t bytes = 0;
    // device plan buffers and their pinned staging
    nqs::JobDesc *d_jobs = nullptr;
    nqs::WorkItem *d_items = nullptr;
    unsigned *d_next = nullptr;
    nqs::JobDesc *h_jobs = nullptr;
    nqs::WorkItem *h_items = nullptr;
    size_t jobs_cap = 0;
    size_t items_cap = 0;
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
    std::unordered_map<nqs_ham, int64_t> resident;  // handle -> bytes counted as resident
    std::unordered_set<nqs_ham> running;
    int64_t resident_bytes = 0;
    int64_t inflight_bytes = 0;
    std::vector<Slot> slots;
    std::thread worker;
    bool stop = false;
    int error = 0;
    std::string error_msg;
    int64_t next_ticket = 1;
    // statistics
    int64_t submitted = 0, completed = 0, rejected = 0, launches = 0;
    int64_t max_reqs_inflight = 0, max_launches_inflight = 0, peak_bytes = 0;
    int64_t reqs_inflight = 0, launches_inflight = 0;
};

namespace {

int fail(int code, const std::string &msg) { return nqs::detail::fail(code, msg); }

void free_slot(Slot &f) {
    if (f.done) (void)hipEventDestroy(f.done);
    if (f.st) (void)hipStreamDestroy(f.st);
    if (f.d_jobs) (void)hipFree(f.d_jobs);
    if (f.d_items) (void)hipFree(f.d_items);
    if (f.d_next) (void)hipFree(f.d_next);
    if (f.h_jobs) (void)hipHostFree(f.h_jobs);
    if (f.h_items) (void)hipHostFree(f.h_items);
    f = Slot{};
}

// Grow a slot's plan buffers (rare: only past the largest plan seen so far).
hipError_t ensure_slot(Slot &f, size_t jobs, size_t items) {
    hipError_t e = hipSuccess;
    if (jobs > f.jobs_cap) {
        if (f.d_jobs) (void)hipFree(f.d_jobs);
        if (f.h_jobs) (void)hipHostFree(f.h_jobs);
        f.d_jobs = nullptr;
        f.h_jobs = nullptr;
        const size_t cap = std::max<size_t>(jobs, 64);
        e = hipMalloc(&f.d_jobs, cap * sizeof(nqs::JobDesc));
        if (e == hipSuccess) e = hipHostMalloc(&f.h_jobs, cap * sizeof(nqs::JobDesc), hipHostMallocDefault);
        if (e != hipSuccess) return e;
        f.jobs_cap = cap;
    }
    if (items > f.items_cap) {
        if (f.d_items) (void)hipFree(f.d_items);
        if (f.h_items) (void)hipHostFree(f.h_items);
        f.d_items = nullptr;
        f.h_items = nullptr;
        const size_t cap = std::max<size_t>(items, size_t(1) << 16);
        e = hipMalloc(&f.d_items, cap * sizeof(nqs::WorkItem));
        if (e == hipSuccess) e = hipHostMalloc(&f.h_items, cap * sizeof(nqs::WorkItem), hipHostMallocDefault);
        if (e != hipSuccess) return e;
        f.items_cap = cap;
    }
    return e;
}

// Plan and launch the slot's requests (called without the server lock).
int launch_slot(nqs_server s, Slot &f) {
    std::vector<nqs_batch_item> items;
    items.reserve(f.reqs.size());
    for (const SrvRequest &r : f.reqs) items.push_back(r.item);
    std::vector<nqs::JobDesc> jobs;
    std::vector<nqs::WorkItem> work;
    nqs::BatchShape shape{};
    int rc = nqs::detail::plan_batch(items.data(), static_cast<int>(items.size()), s->cfg.threads,
                                     f.st, &jobs, &work, &shape);
    if (rc) return rc;
    hipError_t e = ensure_slot(f, jobs.size(), std::max<size_t>(work.size(), 1));
    if (e != hipSuccess) return fail(NQS_E_NOMEM, "allocating a serving slot's plan buffers");
    std::memcpy(f.h_jobs, jobs.data(), jobs.size() * sizeof(nqs::JobDesc));
    if (!work.empty()) std::memcpy(f.h_items, work.data(), work.size() * sizeof(nqs::WorkItem));
    e = hipMemcpyAsync(f.d_jobs, f.h_jobs, jobs.size() * sizeof(nqs::JobDesc), hipMemcpyHostToDevice, f.st);
    if (e == hipSuccess && !work.empty())
        e = hipMemcpyAsync(f.d_items, f.h_items, work.size() * sizeof(nqs::WorkItem),
                           hipMemcpyHostToDevice, f.st);
    if (e == hipSuccess)
        e = nqs::launch_batch(f.d_jobs, static_cast<int>(jobs.size()), f.d_items,
                              static_cast<int>(work.size()), f.d_next, shape, s->cfg.precision, f.st);
    if (e == hipSuccess) e = hipEventRecord(f.done, f.st);
    if (e != hipSuccess) return fail(NQS_E_DEVICE, std::string("serving launch: ") + hipGetErrorString(e));
    for (const SrvRequest &r : f.reqs) nqs::detail::mark_evaluated(r.item.ham, r.item.n);
    return NQS_OK;
}

// Called with the lock held once a slot's launch has completed.
void retire_slot(nqs_server s, Slot &f, const Clock::time_point now, bool ok) {
    for (const SrvRequest &r : f.reqs) {
        const double us =
            ok ? std::chrono::duration<double, std::micro>(now - r.t_submit).count() : -1.0;
        s->finished.emplace_back(r.ticket, us);
        s->running.erase(r.item.ham);
    }
    s->completed += static_cast<int64_t>(f.reqs.size());
    s->reqs_inflight -= static_cast<int64_t>(f.reqs.size());
    s->launches_inflight -= 1;
    s->inflight_bytes -= f.bytes;
    f.reqs.clear();
    f.bytes = 0;
    f.busy = false;
}

void dispatcher(nqs_server s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // 1. retire finished launches
        const Clock::time_point now = Clock::now();
        bool retired = false;
        for (Slot &f : s->slots) {
            if (!f.busy) continue;
            const hipError_t q = hipEventQuery(f.done);
            if (q == hipSuccess) {
                retire_slot(s, f, now, true);
                retired = true;
            } else if (q != hipErrorNotReady) {
                s->error = NQS_E_DEVICE;
                s->error_msg = std::string("serving launch failed: ") + hipGetErrorString(q);
                retire_slot(s, f, now, false);
                retired = true;
            }
        }
        if (retired) s->done_cv.notify_all();
        bool any_busy = false;
        for (const Slot &f : s->slots) any_busy = any_busy || f.busy;
        if (s->error && !s->pending.empty()) {
            // after a failed launch nothing more is admitted: fail the queue
            for (const SrvRequest &r : s->pending) s->finished.emplace_back(r.ticket, -1.0);
            s->completed += static_cast<int64_t>(s->pending.size());
            s->pending.clear();
            s->done_cv.notify_all();
        }
        if (s->stop && s->pending.empty() && !any_busy) break;

        // 2. admit pending requests into free slots
        bool launched = false;
        for (Slot &f : s->slots) {
            if (f.busy || s->pending.empty() || s->error) continue;
            std::vector<SrvRequest> pick;
            std::unordered_set<nqs_ham> in_pick;
            int64_t bytes = 0;
            for (auto it = s->pending.begin();
                 it != s->pending.end() && static_cast<int>(pick.size()) < s->cfg.max_batch;) {
                const nqs_ham h = it->item.ham;
                const bool free_handle = !s->running.count(h) && !in_pick.count(h);
                const bool fits = s->resident_bytes + s->inflight_bytes + bytes + it->bytes <=
                                  s->cfg.hbm_budget_bytes;
                if (free_handle && fits) {
                    bytes += it->bytes;
                    in_pick.insert(h);
                    pick.push_back(*it);
                    it = s->pending.erase(it);
                } else {
                    ++it;
                }
            }
            if (pick.empty()) break;
            for (const SrvRequest &r : pick) s->running.insert(r.item.ham);
            f.reqs = std::move(pick);
            f.bytes = bytes;
            f.busy = true;
            s->inflight_bytes += bytes;
            s->reqs_inflight += static_cast<int64_t>(f.reqs.size());
            s->launches_inflight += 1;
            s->launches += 1;
            s->max_reqs_inflight = std::max(s->max_reqs_inflight, s->reqs_inflight);
            s->max_launches_inflight = std::max(s->max_launches_inflight, s->launches_inflight);
            s->peak_bytes = std::max(s->peak_bytes, s->resident_bytes + s->inflight_bytes);
            lk.unlock();
            const int rc = launch_slot(s, f);
            lk.lock();
            if (rc) {
                s->error = rc;
                s->error_msg = "serving launch could not be planned or enqueued";
                retire_slot(s, f, Clock::now(), false);
                s->done_cv.notify_all();
            }
            launched = true;
        }
        if (launched) continue;
        // 3. wait: poll completions while launches run, sleep when idle
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
    if (c.max_batch == 0) c.max_batch = 64;
    if (c.hbm_budget_bytes <= 0 || c.streams < 1 || c.streams > 8 || c.max_batch < 1 ||
        c.max_batch > 256 || (c.precision != NQS_FP64 && c.precision != NQS_FP32_KAHAN) ||
        !(c.threads == 0 || c.threads == 256 || c.threads == 512 || c.threads == 1024))
        return fail(NQS_E_ARG, "server configuration out of range");
    nqs_server s = new (std::nothrow) nqs_server_s();
    if (!s) return fail(NQS_E_NOMEM, "host allocation failed");
    s->cfg = c;
    hipError_t e = hipGetDevice(&s->device);
    s->slots.resize(c.streams);
    for (Slot &f : s->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&f.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&f.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&f.d_next, nqs::kBatchCounters * sizeof(unsigned));
        if (e == hipSuccess) e = ensure_slot(f, 64, size_t(1) << 16);
    }
    if (e == hipSuccess) e = nqs::prepare_batch_kernels();
    if (e != hipSuccess) {
        for (Slot &f : s->slots) free_slot(f);
        delete s;
        return fail(NQS_E_DEVICE, std::string("creating the server: ") + hipGetErrorString(e));
    }
    s->worker = std::thread(dispatcher, s);
    *out = s;
    return NQS_OK;
}

int nqs_server_add_ham(nqs_server s, nqs_ham h, int64_t max_samples) {
    if (!s) return fail(NQS_E_STATE, "invalid server");
    if (!nqs::detail::valid_handle(h)) return fail(NQS_E_ARG, "invalid handle");
    if (max_samples < 1) return fail(NQS_E_ARG, "max_samples must be positive");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->resident.count(h)) return fail(NQS_E_ARG, "handle already registered");
        if (s->running.count(h)) return fail(NQS_E_STATE, "handle is running");
    }
    // scratch is sized now so that the serving loop does not allocate
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(NQS_E_DEVICE, "creating a stream");
    int rc = nqs::detail::reserve(h, max_samples, s->cfg.threads, st);
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    if (rc) return rc;
    const int64_t bytes = nqs::detail::table_bytes(h);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->resident_bytes + bytes > s->cfg.hbm_budget_bytes)
        return fail(NQS_E_NOMEM, "resident tables would exceed the HBM budget");
    s->resident[h] = bytes;
    s->resident_bytes += bytes;
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
    if (!s->resident.count(req->ham)) return fail(NQS_E_ARG, "handle not registered with the server");
    SrvRequest r;
    r.ticket = s->next_ticket++;
    r.item = *req;
    r.bytes = kBytesPerSample * req->n + nqs::detail::scratch_bytes(req->ham);
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
    for (Slot &f : s->slots) {
        if (f.st) (void)hipStreamSynchronize(f.st);
        free_slot(f);
    }
    const int err = s->error;
    delete s;
    return err ? fail(err, "server stopped after an error") : NQS_OK;
}

}  // extern "C"
