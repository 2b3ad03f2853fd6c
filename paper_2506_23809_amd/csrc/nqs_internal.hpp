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
// Validate batch items, grow scratch, and build the job descriptors, the
// work list and the launch shape (host side only; no upload).
int plan_batch(const nqs_batch_item *items, int n_items, int threads, hipStream_t st,
               std::vector<JobDesc> *jobs, std::vector<WorkItem> *work, BatchShape *shape);

}  // namespace detail
}  // namespace nqs
