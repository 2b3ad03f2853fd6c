// Library internals shared between the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nqs.h"
#include "nqs_device.hpp"

namespace nqs {
namespace detail {

// Record msg as the calling thread's last error and return code.
int fail(int code, const std::string &msg);
bool valid_handle(nqs_ham h);
// Device bytes of the resident table, and of the handle's current scratch.
int64_t table_bytes(nqs_ham h);
int64_t scratch_bytes(nqs_ham h);
// Grow the handle's scratch for batches of n samples (may allocate).
int reserve(nqs_ham h, int64_t n, int threads, hipStream_t st);
// Bookkeeping of nqs_eval_stats after a launch that evaluated n samples.
void mark_evaluated(nqs_ham h, int64_t n);
// Server lanes: the evaluation scratch a request of n samples needs (the
// plan nqs_eloc_eval would take), and one evaluation of a request with its
// scratch carved from ctx (ctx_bytes) and its counters, error latch and
// sector flag in small (small_bytes(), the error word at
// small_err_offset()), on st, without allocating.
size_t request_scratch_bytes(nqs_ham h, int64_t n);
size_t small_bytes();
size_t small_err_offset();
int eval_in(nqs_ham h, const nqs_batch_item &it, int precision, char *ctx, size_t ctx_bytes,
            void *small, hipStream_t st);
// Latch an error seen for one of h's requests (the next nqs_sync reports it).
void latch_host_error(nqs_ham h, int code);
// Validate batch items, grow scratch, and build the job descriptors, the
// work list and the launch shape (host side only; no upload).
int plan_batch(const nqs_batch_item *items, int n_items, int threads, hipStream_t st,
               std::vector<JobDesc> *jobs, std::vector<WorkItem> *work, BatchShape *shape);

}  // namespace detail
}  // namespace nqs
