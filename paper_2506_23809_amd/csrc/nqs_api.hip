// C ABI of libnqs.so: handles, argument checks, scratch management, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>

#include "../../include/nqs.h"
#include "nqs_device.hpp"
#include "nqs_internal.hpp"
#include "nqs_table.hpp"

// Scratch of nqs_eloc_eval_noalloc (one copy per device, in the library's
// code object).  Its name is a host-side stand-in: host code takes the
// device address with hipGetSymbolAddress and uses only that.
static __device__ __align__(256) unsigned char scratch[NQS_NOALLOC_SCRATCH_BYTES];

namespace {

int fail(int code, const std::string &msg) { return nqs::detail::fail(code, msg); }

int fail_hip(hipError_t e, const char *what) {
    return fail(NQS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define NQS_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return fail_hip(e_, #call); \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// counters (kCounterSlots copies), error latch, sector flag
constexpr size_t kErrOffset = 8 * nqs::kCounters * nqs::kCounterSlots;
constexpr size_t kSmallBytes = kErrOffset + 64;
// nqs_eloc_energy's pinned host buffer: the error word, then out[4]
constexpr size_t kEnergyHostSeq = 4;     // sequence number the host polls
constexpr size_t kEnergyHostChosen = 8;  // the join's decision (2: no join launched)
constexpr size_t kEnergyHostOut = 16;
constexpr size_t kSeqOffset = kErrOffset + 8;  // the device's copy of it (in small)
constexpr size_t kEnergyHostBytes = kEnergyHostOut + 4 * sizeof(double);
constexpr size_t kMaxFilterWords = size_t(1) << 15;  // 128 KB Bloom bitmap
constexpr size_t kMaxEFilterWords = kMaxFilterWords * nqs::kEnumMaxParts;
constexpr int64_t kMaxGroups = int64_t(1) << 26;     // queue entries pack the group in 26 bits

}  // namespace

struct nqs_ham_s {
    int device = 0;
    int words = 1;
    nqs::DevTable dt{};
    void *table_mem = nullptr;
    int64_t table_bytes = 0;
    // scratch, grown on demand and reused
    void *slots = nullptr;
    uint32_t slot_cap = 0;
    size_t slot_bytes = 0;
    uint32_t *shx = nullptr;
    int64_t shx_cap = 0;
    double *part = nullptr;
    int64_t part_cap = 0;  // doubles
    uint32_t *filter = nullptr;  // Bloom bitmap, kMaxFilterWords words
    uint32_t *efilter = nullptr; // enumeration filter partitions (allocated when first needed)
    // the enumeration blocks' areas of device scratch (one per CU)
    char *eblk = nullptr;
    int64_t eblk_stride = 0;
    uint32_t eblk_blocks = 0;
    void *jmem = nullptr;  // the pair join's buckets and entries
    size_t jmem_bytes = 0;
    void *small = nullptr; // counters[8] u64, err, mixed
    // nqs_eloc_energy: per-finish-block partials of Eq. 1 (device) and the
    // pinned host buffer its last kernel writes {err, pad, out[4]} to
    double *epart = nullptr;
    int64_t epart_cap = 0;  // doubles
    char *ehost = nullptr;
    // the previous nqs_eloc_energy ran the pair join: the next one launches
    // only the join's kernels (checked against the device's decision)
    bool join_likely = false;
    // an error a server lane saw for one of this handle's requests, reported
    // by the next nqs_sync like a latched device error
    std::atomic<int> host_err{0};
    int64_t last_pairs = 0;
    bool ever_evaluated = false;
    nqs::EvalLaunch last_plan{};  // launch plan of the last evaluation
    unsigned long long *last_jctl = nullptr;  // its pair-join control words (device)
    // optional per-stage events: hash start, hash end / lookup start,
    // lookup end / finish start, finish end
    bool profiling = false;
    bool profiled = false;
    // profiling events: start, after the hash stage, after the lookup
    // stage, after the finish, after the join grouping, after the join pairs
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // launch tuning (all-zero = built-in plan)
    nqs::Tuning tune{0, 0, 0, 0};
    // replay of a repeated evaluation: the launch sequence of the last call,
    // captured on a private stream once the same arguments come twice in a
    // row, and launched as one graph while they keep coming
    bool graphs = true;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t eval_exec = nullptr;
    bool have_key = false;
    unsigned char eval_key[256] = {};
};

namespace {

// Slot arrays of a sample hash of cap slots (a power of two) at base: keys
// first, then the slot indices, then the slot fingerprints.
void set_slots(nqs::DevScratch *s, void *base, uint32_t cap, int words) {
    s->skey = static_cast<uint64_t *>(base);
    s->sidx = base ? reinterpret_cast<int32_t *>(static_cast<char *>(base) +
                                                 sizeof(uint64_t) * words * cap)
                   : nullptr;
    s->sfp = base ? reinterpret_cast<uint32_t *>(s->sidx + cap) : nullptr;
    s->slot_mask = cap - 1;
    int lg = 0;
    while ((1u << lg) < cap) ++lg;
    s->slot_shift = 32 - (lg - nqs::bucket_log2(words));
}

// Bytes of a sample hash of cap slots.
size_t slot_array_bytes(uint32_t cap, int words) {
    return static_cast<size_t>(cap) * (sizeof(uint64_t) * words + sizeof(int32_t) + sizeof(uint32_t));
}

nqs::DevScratch scratch_of(nqs_ham h) {
    nqs::DevScratch s{};
    set_slots(&s, h->slots, h->slot_cap, h->words);
    s.shx = h->shx;
    s.part = h->part;
    s.filter = h->filter;
    s.eblk = h->eblk;
    s.eblk_stride = h->eblk_stride;
    s.eblk_blocks = h->eblk_blocks;
    s.counters = static_cast<unsigned long long *>(h->small);
    s.err = reinterpret_cast<int *>(static_cast<char *>(h->small) + kErrOffset);
    s.mixed = reinterpret_cast<int *>(static_cast<char *>(h->small) + kErrOffset + 4);
    return s;
}

// Filter sizes of one evaluation plan.
void set_filters(nqs::DevScratch *s, nqs_ham h, const nqs::EvalLaunch &L) {
    s->filter_log2 = L.filter_log2;
    s->eparts_log2 = L.eparts_log2;
    s->efilter_log2 = L.efilter_log2;
    s->efilter = L.eparts_log2 > 0 ? h->efilter : h->filter;
    if (L.join && h->jmem) {
        nqs::join_scratch_layout(h->dt, L.n, L.join_log2m, static_cast<char *>(h->jmem), s);
        s->join_force = L.join_force;
    }
}

// Partial-sum slots per sample a plan needs: its group chunks, or one per
// join block when the pair join may run.
int64_t plan_chunks(const nqs_ham h, const nqs::EvalLaunch &L) {
    const int64_t c = L.n_chunks > 0 ? L.n_chunks : 1;
    return L.join ? std::max<int64_t>(c, h->dt.join_blocks) : c;
}

// Bytes of the pair join's scratch for a plan (0: none planned).
size_t plan_join_bytes(const nqs_ham h, const nqs::EvalLaunch &L) {
    return L.join ? nqs::join_scratch_bytes(h->dt, L.n, L.join_log2m) : 0;
}

// Grow the per-handle scratch to hold a batch of n samples (and the
// partitioned enumeration filter when the plan uses it).
// Bytes of one enumeration block's area for this table: the most any
// occupation of its spin orbitals needs.
int64_t enum_blk_stride(const nqs::DevTable &t) {
    if (!t.enum_ok) return 0;
    int64_t m = 0;
    for (int na = 0; na <= t.k_alpha; ++na)
        for (int nb = 0; nb <= t.k_beta; ++nb)
            m = std::max(m, nqs::enum_blk_bytes(t.k_alpha, t.k_beta, na, nb));
    return (m + 255) & ~static_cast<int64_t>(255);
}

// Test hook (nqs_debug_fail_allocs): the g_fail_at-th scratch allocation
// from the time it was set reports out-of-memory without allocating (once).
std::atomic<int> g_fail_at{0};

hipError_t scratch_malloc(void **p, size_t bytes) {
    int left = g_fail_at.load();
    while (left > 0) {
        if (g_fail_at.compare_exchange_weak(left, left - 1)) {
            if (left == 1) {
                *p = nullptr;
                return hipErrorOutOfMemory;
            }
            break;
        }
    }
    return hipMalloc(p, bytes);
}

// Replace a scratch buffer by one of `bytes`: the old one is released and
// its recorded capacity zeroed first, so a failed allocation leaves an empty
// buffer (capacity 0) that the next call grows again, never a stale
// capacity over a null pointer.
template <typename T, typename C>
int regrow(T **buf, C *cap, C new_cap, size_t bytes, const char *what) {
    if (*buf) {
        const hipError_t e = hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
        if (e != hipSuccess) return fail_hip(e, "hipFree of scratch");
    }
    *cap = 0;
    void *p = nullptr;
    if (scratch_malloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(NQS_E_NOMEM, std::string("device allocation of ") + what + " failed");
    }
    *buf = static_cast<T *>(p);
    *cap = new_cap;
    return NQS_OK;
}

int ensure_scratch(nqs_ham h, int64_t n, int64_t n_chunks, hipStream_t st,
                   bool efilter = false, size_t join_bytes = 0) {
    uint64_t want = 64;
    while (want < nqs::kSlotsPerSample * static_cast<uint64_t>(n)) want <<= 1;
    if (want > (1ull << 31)) return fail(NQS_E_ARG, "batch too large for the sample hash");
    // key + index + fingerprint
    const size_t slot_size = sizeof(uint64_t) * h->words + sizeof(int32_t) + sizeof(uint32_t);
    const int64_t part_need = 2 * n * (n_chunks > 0 ? n_chunks : 1);
    // the block areas: allocated once, one per CU of the handle's device
    int n_cu = 0;
    int64_t blk_stride = 0;
    if (!h->eblk && h->dt.enum_ok) {
        NQS_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device));
        blk_stride = enum_blk_stride(h->dt);
    }
    const bool blk_grow = blk_stride > 0 && n_cu > 0;
    const bool grow = want > h->slot_cap || n > h->shx_cap || part_need > h->part_cap ||
                      (efilter && !h->efilter) || blk_grow || join_bytes > h->jmem_bytes;
    if (!grow) return NQS_OK;
    NQS_HIP(hipStreamSynchronize(st));
    int rc = NQS_OK;
    if (blk_grow) {
        uint32_t blocks = 0;
        rc = regrow(&h->eblk, &blocks, static_cast<uint32_t>(n_cu),
                    static_cast<size_t>(blk_stride) * n_cu, "the enumeration block areas");
        h->eblk_blocks = blocks;
        h->eblk_stride = h->eblk ? blk_stride : 0;
        if (rc) return rc;
    }
    if (efilter && !h->efilter) {
        int have = 0;
        rc = regrow(&h->efilter, &have, 1, kMaxEFilterWords * 4, "the filter partitions");
        if (rc) return rc;
    }
    if (want > h->slot_cap) {
        uint32_t cap = h->slot_cap;
        h->slot_bytes = 0;
        rc = regrow(&h->slots, &cap, static_cast<uint32_t>(want),
                    want * slot_size, "the sample hash");
        h->slot_cap = cap;
        if (rc) return rc;
        h->slot_bytes = want * slot_size;
    }
    if (n > h->shx_cap) {
        rc = regrow(&h->shx, &h->shx_cap, n, sizeof(uint32_t) * n, "sample hashes");
        if (rc) return rc;
    }
    if (part_need > h->part_cap) {
        rc = regrow(&h->part, &h->part_cap, part_need, sizeof(double) * part_need,
                    "partial sums");
        if (rc) return rc;
    }
    if (join_bytes > h->jmem_bytes) {
        rc = regrow(&h->jmem, &h->jmem_bytes, join_bytes, join_bytes, "the pair join's buckets");
        if (rc) return rc;
    }
    return NQS_OK;
}

// Whether the scratch a plan needs is all present (a failed growth leaves
// a buffer empty; nothing may be launched over it).
int scratch_ready(nqs_ham h, const nqs::EvalLaunch &L) {
    const bool ok = h->slots && h->slot_cap >= 64 && h->shx && h->part && h->filter && h->small &&
                    (L.eparts_log2 == 0 || h->efilter) &&
                    (L.strategy != nqs::kStrategyEnum || !h->dt.enum_ok || h->eblk) &&
                    (!L.join || (h->jmem && h->jmem_bytes >= plan_join_bytes(h, L))) &&
                    h->part_cap >= 2 * L.n * plan_chunks(h, L);
    return ok ? NQS_OK : fail(NQS_E_STATE, "scratch buffers missing after a failed allocation");
}

bool valid_handle(nqs_ham h) { return h && h->table_mem && h->small; }

// Everything the launches of one evaluation depend on besides the table.
struct EvalKey {
    int64_t n;
    const void *samples, *weights, *log_amp, *phase, *eloc;
    int precision;
    int strategy;
    unsigned enum_blocks;
    int64_t n_chunks, chunk_len, g_first;
    int threads, filter_log2;
    size_t lds_bytes;
    int eparts_log2, efilter_log2;
    int join, join_force, join_log2m;
    const void *slots, *shx, *part, *filter, *efilter, *small, *eblk, *jmem;
    uint32_t slot_cap;
    int energy, join_only;
    const void *epart, *ehost;
};
static_assert(sizeof(EvalKey) <= sizeof(nqs_ham_s::eval_key), "key fits");

// The launches of one evaluation on stream s.
hipError_t issue_eval(nqs_ham h, const nqs::DevScratch &sc, const nqs::EvalLaunch &L, int64_t n,
                      const uint64_t *samples, const int64_t *weights, const double *log_amp,
                      const double *phase, double *eloc, int precision, int32_t *hit_idx,
                      uint32_t *sign_bits, hipStream_t s, bool may_profile = true,
                      bool energy = false) {
    hipError_t e;
    const bool prof = h->profiling && may_profile;
    if (prof && (e = hipEventRecord(h->ev[0], s)) != hipSuccess) return e;
    if ((e = nqs::launch_hash(h->dt, sc, sc.slot_mask + 1u, samples, weights, n, s,
                              prof ? h->ev[4] : nullptr, L.join_only != 0)) != hipSuccess)
        return e;
    if (prof && (e = hipEventRecord(h->ev[1], s)) != hipSuccess) return e;
    const int64_t sign_words = (h->dt.n_terms + 31) / 32;
    nqs::EvalStageEvents stages{prof ? h->ev[2] : nullptr, prof ? h->ev[5] : nullptr, nullptr,
                                prof ? h->ev[3] : nullptr};
    // with the energy, its combining kernel writes the result and the error
    // word straight to the handle's pinned host buffer (no copy to wait for)
    const nqs::EnergyFused ef =
        energy ? nqs::EnergyFused{weights, h->epart,
                                  reinterpret_cast<double *>(h->ehost + kEnergyHostOut),
                                  reinterpret_cast<int *>(h->ehost),
                                  reinterpret_cast<unsigned *>(static_cast<char *>(h->small) +
                                                               kSeqOffset),
                                  reinterpret_cast<unsigned *>(h->ehost + kEnergyHostSeq),
                                  reinterpret_cast<unsigned *>(h->ehost + kEnergyHostChosen)}
               : nqs::EnergyFused{weights, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    if ((e = nqs::launch_eloc(h->dt, sc, L, samples, weights, log_amp, phase, eloc, precision,
                              hit_idx, sign_bits, sign_words, stages, ef, s)) != hipSuccess)
        return e;
    // (ev[3], after the finish kernel, is recorded inside the launch: an
    // energy's combining kernel follows it)
    return hipSuccess;
}

// Capture the launches of one evaluation into a graph (on the handle's own
// stream: the caller's may be the null stream, which cannot be captured).
// Never with profiling on (its events are recorded eagerly).
hipError_t capture_eval(nqs_ham h, const nqs::DevScratch &sc, const nqs::EvalLaunch &L, int64_t n,
                        const uint64_t *samples, const int64_t *weights, const double *log_amp,
                        const double *phase, double *eloc, int precision, bool energy,
                        hipGraphExec_t *out) {
    hipError_t e = hipSuccess;
    if (!h->cap_stream) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t e1 = issue_eval(h, sc, L, n, samples, weights, log_amp, phase, eloc,
                                     precision, nullptr, nullptr, h->cap_stream, true, energy);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
    e = e1 != hipSuccess ? e1 : e2;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

// The device's error word back to zero (after the host has read it).
hipError_t clear_device_error(nqs_ham h) {
    const int zero = 0;
    return hipMemcpy(static_cast<char *>(h->small) + kErrOffset, &zero, sizeof(int),
                     hipMemcpyHostToDevice);
}

int report_device_error(int err) {
    switch (err) {
        case 0: return NQS_OK;
        case NQS_E_DUPLICATE: return fail(err, "a sample occurs more than once in the batch");
        case NQS_E_RANGE:
            return fail(err, "a sample has bits at or above n_qubits, or a count is negative");
        default: return fail(err, "device-detected error");
    }
}

int eval_impl(nqs_ham h, int64_t n, const uint64_t *samples, const int64_t *weights,
              const double *log_amp, const double *phase, double *eloc, int precision,
              int32_t *hit_idx, uint32_t *sign_bits, void *stream, bool energy = false,
              bool join_only = false) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (n < 0) return fail(NQS_E_ARG, "n < 0");
    if (precision != NQS_FP64 && precision != NQS_FP32_KAHAN)
        return fail(NQS_E_ARG, "unknown precision");
    if (h->dt.sc && precision != NQS_FP64)
        return fail(NQS_E_ARG, "the integral form evaluates in FP64 only");
    if (n == 0) return NQS_OK;
    if (!samples || !log_amp || !phase || !eloc)
        return fail(NQS_E_ARG, "null sample, amplitude, phase or output pointer");
    if (n > (int64_t(1) << 30)) return fail(NQS_E_ARG, "batch larger than 2^30 samples");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool dump = hit_idx || sign_bits;
    nqs::EvalLaunch L = nqs::plan_eval(h->dt, n, dump, &h->tune);
    // (only where a join is launched and may be chosen)
    L.join_only = join_only && L.join && !dump ? 1 : 0;
    int rc = ensure_scratch(h, n, plan_chunks(h, L), st, L.eparts_log2 > 0, plan_join_bytes(h, L));
    if (!rc) rc = scratch_ready(h, L);
    if (rc) return rc;
    nqs::DevScratch sc = scratch_of(h);
    set_filters(&sc, h, L);
    bool done = false;
    // profiling stays eager: its events time each kernel of every call
    if (h->graphs && !dump && !h->profiling) {
        EvalKey key;
        std::memset(&key, 0, sizeof key);
        key.n = n;
        key.samples = samples;
        key.weights = weights;
        key.log_amp = log_amp;
        key.phase = phase;
        key.eloc = eloc;
        key.precision = precision;
        key.strategy = L.strategy;
        key.enum_blocks = L.enum_blocks;
        key.n_chunks = L.n_chunks;
        key.chunk_len = L.chunk_len;
        key.g_first = L.g_first;
        key.threads = L.threads;
        key.filter_log2 = L.filter_log2;
        key.lds_bytes = L.lds_bytes;
        key.eparts_log2 = L.eparts_log2;
        key.efilter_log2 = L.efilter_log2;
        key.join = L.join;
        key.join_force = L.join_force;
        key.join_log2m = L.join_log2m;
        key.jmem = h->jmem;
        key.slots = h->slots;
        key.shx = h->shx;
        key.part = h->part;
        key.filter = h->filter;
        key.efilter = h->efilter;
        key.small = h->small;
        key.eblk = h->eblk;
        key.slot_cap = h->slot_cap;
        key.energy = energy ? 1 : 0;
        key.join_only = L.join_only;
        key.epart = energy ? h->epart : nullptr;
        key.ehost = energy ? h->ehost : nullptr;
        const bool same = h->have_key && std::memcmp(h->eval_key, &key, sizeof key) == 0;
        if (!same) {
            // a new argument set: run it eagerly, remember it
            if (h->eval_exec) {
                (void)hipGraphExecDestroy(h->eval_exec);
                h->eval_exec = nullptr;
            }
            std::memcpy(h->eval_key, &key, sizeof key);
            h->have_key = true;
        } else {
            if (!h->eval_exec) {
                hipGraphExec_t ex = nullptr;
                if (capture_eval(h, sc, L, n, samples, weights, log_amp, phase, eloc, precision,
                                 energy, &ex) == hipSuccess) {
                    h->eval_exec = ex;
                } else {
                    // graphs unavailable: stay eager from now on
                    (void)hipGetLastError();
                    if (ex) (void)hipGraphExecDestroy(ex);
                    h->graphs = false;
                }
            }
            if (h->eval_exec) {
                NQS_HIP(hipGraphLaunch(h->eval_exec, st));
                done = true;
            }
        }
    }
    if (!done)
        NQS_HIP(issue_eval(h, sc, L, n, samples, weights, log_amp, phase, eloc, precision, hit_idx,
                           sign_bits, st, true, energy));
    if (h->profiling) h->profiled = true;
    h->last_pairs = n * h->dt.n_groups;
    h->last_plan = L;
    h->last_jctl = sc.jctl;
    h->ever_evaluated = true;
    return NQS_OK;
}

// ---- the entry point that allocates nothing (nqs_eloc_eval_noalloc)
//
// Its evaluation scratch (sample hash, sample hashes, partial sums, filters,
// the enumeration's block areas) is carved out of one file-scope device
// array, resident on every device the library runs on for the life of the
// process.  Host code never uses the array's name as an address: the
// device address is taken once per device with hipGetSymbolAddress and kept.
constexpr size_t kNoAllocBytes = static_cast<size_t>(NQS_NOALLOC_SCRATCH_BYTES);

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mutex;
void *g_noalloc_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use,
// with the device current).
int noalloc_base(int dev, char **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(NQS_E_DEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail_hip(e, "hipGetSymbolAddress of the scratch array");
        g_noalloc_ptr[dev] = p;
    }
    *out = static_cast<char *>(g_noalloc_ptr[dev]);
    return NQS_OK;
}

// Lay the scratch of one evaluation out from base (256-byte aligned pieces):
// slots, sample hashes, partial sums, filter, filter partitions, block
// areas.  Returns the bytes it needs; fills *sc only when they fit in cap.
size_t layout_scratch(nqs_ham h, const nqs::EvalLaunch &L, int64_t n, int n_cu, char *base,
                      size_t cap, nqs::DevScratch *sc, void *small = nullptr) {
    if (!small) small = h->small;
    uint64_t slots = 64;
    while (slots < nqs::kSlotsPerSample * static_cast<uint64_t>(n)) slots <<= 1;
    const int64_t chunks = plan_chunks(h, L);
    const size_t sizes[7] = {
        slot_array_bytes(static_cast<uint32_t>(slots), h->words),
        sizeof(uint32_t) * static_cast<size_t>(n),
        sizeof(double) * 2 * static_cast<size_t>(n) * chunks,
        kMaxFilterWords * 4,
        L.eparts_log2 > 0 ? kMaxEFilterWords * 4 : 0,
        h->dt.enum_ok ? static_cast<size_t>(enum_blk_stride(h->dt)) * n_cu : 0,
        plan_join_bytes(h, L),
    };
    size_t off[7];
    size_t total = 0;
    for (int k = 0; k < 7; ++k) {
        off[k] = total;
        total = align_up(total + sizes[k], 256);
    }
    if (slots > (1ull << 31) || total > cap) return total;
    set_slots(sc, base + off[0], static_cast<uint32_t>(slots), h->words);
    sc->shx = reinterpret_cast<uint32_t *>(base + off[1]);
    sc->part = reinterpret_cast<double *>(base + off[2]);
    sc->filter = reinterpret_cast<uint32_t *>(base + off[3]);
    sc->efilter = L.eparts_log2 > 0 ? reinterpret_cast<uint32_t *>(base + off[4]) : sc->filter;
    sc->eblk = h->dt.enum_ok ? base + off[5] : nullptr;
    sc->eblk_stride = h->dt.enum_ok ? enum_blk_stride(h->dt) : 0;
    sc->eblk_blocks = h->dt.enum_ok ? static_cast<uint32_t>(n_cu) : 0;
    sc->counters = static_cast<unsigned long long *>(small);
    sc->err = reinterpret_cast<int *>(static_cast<char *>(small) + kErrOffset);
    sc->mixed = reinterpret_cast<int *>(static_cast<char *>(small) + kErrOffset + 4);
    sc->filter_log2 = L.filter_log2;
    sc->eparts_log2 = L.eparts_log2;
    sc->efilter_log2 = L.efilter_log2;
    if (L.join) {
        nqs::join_scratch_layout(h->dt, n, L.join_log2m, base + off[6], sc);
        sc->join_force = L.join_force;
    }
    return total;
}

int eval_noalloc(nqs_ham h, int64_t n, const uint64_t *samples, const int64_t *weights,
                 const double *log_amp, const double *phase, double *eloc, int precision,
                 void *stream) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (n < 0) return fail(NQS_E_ARG, "n < 0");
    if (precision != NQS_FP64 && precision != NQS_FP32_KAHAN)
        return fail(NQS_E_ARG, "unknown precision");
    if (h->dt.sc && precision != NQS_FP64)
        return fail(NQS_E_ARG, "the integral form evaluates in FP64 only");
    if (n == 0) return NQS_OK;
    if (!samples || !log_amp || !phase || !eloc)
        return fail(NQS_E_ARG, "null sample, amplitude, phase or output pointer");
    if (n > (int64_t(1) << 30)) return fail(NQS_E_ARG, "batch larger than 2^30 samples");
    int dev = -1;
    NQS_HIP(hipGetDevice(&dev));
    if (dev != h->device) return fail(NQS_E_STATE, "the handle's device is not current");
    int n_cu = 0;
    NQS_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const nqs::EvalLaunch L = nqs::plan_eval(h->dt, n, false, &h->tune);
    nqs::DevScratch sc{};
    const size_t need = layout_scratch(h, L, n, n_cu, nullptr, 0, &sc);
    if (need > kNoAllocBytes)
        return fail(NQS_E_ARG, "batch needs " + std::to_string(need) +
                                   " bytes of scratch, more than the " +
                                   std::to_string(kNoAllocBytes) +
                                   " the allocation-free entry point holds");
    char *base = nullptr;
    int rc = noalloc_base(dev, &base);
    if (rc) return rc;
    layout_scratch(h, L, n, n_cu, base, kNoAllocBytes, &sc);
    NQS_HIP(issue_eval(h, sc, L, n, samples, weights, log_amp, phase, eloc, precision, nullptr,
                       nullptr, static_cast<hipStream_t>(stream)));
    if (h->profiling) h->profiled = true;
    h->last_pairs = n * h->dt.n_groups;
    h->last_plan = L;
    h->last_jctl = sc.jctl;
    h->ever_evaluated = true;
    return NQS_OK;
}

// Process-wide scratch of nqs_energy, one per device, used under a lock.
struct EnergyScratch {
    double *dev = nullptr;   // block partials | out[4]
    double *host = nullptr;  // pinned out[4]
};
std::mutex g_energy_mutex;
std::unordered_map<int, EnergyScratch> g_energy;

}  // namespace

namespace {

// Upload a host table (and, for the integral form, h_pq and packed (pq|rs))
// into one device allocation and make a handle of it.
int create_handle(nqs_ham *out, const nqs::HostTable &T, const std::vector<double> *h1,
                  const std::vector<double> *eri, int sc_k, hipStream_t st) {
    if (T.n_groups >= kMaxGroups) return fail(NQS_E_ARG, "more than 2^26 X groups");
    const int64_t G = T.n_groups, Tn = T.n_terms;
    // one allocation holding every table array, each 256-byte aligned
    std::vector<float> tc32(2 * static_cast<size_t>(Tn));
    for (int64_t t = 0; t < Tn; ++t) {
        const float hi = static_cast<float>(T.tc[t]);
        tc32[2 * t] = hi;
        tc32[2 * t + 1] = static_cast<float>(T.tc[t] - static_cast<double>(hi));
    }
    std::vector<float> diag32(2 * T.diag.size());
    for (size_t k = 0; k < T.diag.size(); ++k) {
        const float hi = static_cast<float>(T.diag[k]);
        diag32[2 * k] = hi;
        diag32[2 * k + 1] = static_cast<float>(T.diag[k] - static_cast<double>(hi));
    }
    // the occupation form as int8 digit tiles for the matrix cores
    std::vector<int8_t> diag_q8;
    double diag_scale = 1.0;
    const int diag_jtiles = T.diag_occ ? (T.n_qubits + 15) / 16 : 0;
    if (T.diag_occ) nqs::build_diag_tiles(T, &diag_q8, &diag_scale);
    std::vector<uint32_t> goff32(T.goff.size());
    for (size_t k = 0; k < T.goff.size(); ++k) goff32[k] = static_cast<uint32_t>(T.goff[k]);
    const nqs::LinearHash lh;
    struct Piece {
        const void *src;
        size_t bytes;
        size_t off;
    };
    Piece pieces[] = {
        {T.gx.data(), sizeof(uint64_t) * T.gx.size(), 0},
        {T.gsec.data(), sizeof(uint64_t) * T.gsec.size(), 0},
        {T.ghm.data(), sizeof(uint32_t) * T.ghm.size(), 0},
        {goff32.data(), sizeof(uint32_t) * goff32.size(), 0},
        {T.tz.data(), sizeof(uint64_t) * T.tz.size(), 0},
        {T.tc.data(), sizeof(double) * T.tc.size(), 0},
        {tc32.data(), sizeof(float) * tc32.size(), 0},
        {lh.r, sizeof(lh.r), 0},
        {h1 ? h1->data() : nullptr, h1 ? sizeof(double) * h1->size() : 0, 0},
        {eri ? eri->data() : nullptr, eri ? sizeof(double) * eri->size() : 0, 0},
        {T.spin_q, sizeof(T.spin_q), 0},
        {T.gh.data(), sizeof(uint32_t) * T.gh.size(), 0},
        {T.qcls, sizeof(T.qcls), 0},
        {T.diag.data(), sizeof(double) * T.diag.size(), 0},
        {diag32.data(), sizeof(float) * diag32.size(), 0},
        {diag_q8.data(), diag_q8.size(), 0},
    };
    size_t total = 0;
    for (Piece &p : pieces) {
        p.off = total;
        total = align_up(total + (p.bytes ? p.bytes : 1), 256);
    }
    nqs_ham h = new (std::nothrow) nqs_ham_s();
    if (!h) return fail(NQS_E_NOMEM, "host allocation failed");
    // NQS_EVAL_GRAPHS=0 keeps every evaluation eager
    if (const char *g = std::getenv("NQS_EVAL_GRAPHS")) h->graphs = std::strcmp(g, "0") != 0;
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return fail_hip(e, "hipGetDevice");
    }
    if (hipMalloc(&h->table_mem, total) != hipSuccess) {
        delete h;
        return fail(NQS_E_NOMEM, "device allocation of the Hamiltonian table failed");
    }
    if (hipMalloc(&h->small, kSmallBytes) != hipSuccess ||
        hipMalloc(&h->filter, kMaxFilterWords * 4) != hipSuccess) {
        (void)hipFree(h->table_mem);
        if (h->small) (void)hipFree(h->small);
        delete h;
        return fail(NQS_E_NOMEM, "device allocation failed");
    }
    char *base = static_cast<char *>(h->table_mem);
    for (const Piece &p : pieces) {
        if (!p.bytes) continue;
        e = hipMemcpyAsync(base + p.off, p.src, p.bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess) e = hipMemsetAsync(h->small, 0, kSmallBytes, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(h->table_mem);
        (void)hipFree(h->small);
        (void)hipFree(h->filter);
        delete h;
        return fail_hip(e, "uploading the Hamiltonian table");
    }
    h->table_bytes = static_cast<int64_t>(total);
    h->words = T.words;
    nqs::DevTable &d = h->dt;
    d.gx = reinterpret_cast<const uint64_t *>(base + pieces[0].off);
    d.gsec = reinterpret_cast<const uint64_t *>(base + pieces[1].off);
    d.ghm = reinterpret_cast<const uint32_t *>(base + pieces[2].off);
    d.goff = reinterpret_cast<const uint32_t *>(base + pieces[3].off);
    d.tz = reinterpret_cast<const uint64_t *>(base + pieces[4].off);
    d.tc = reinterpret_cast<const double *>(base + pieces[5].off);
    d.tc32 = reinterpret_cast<const float *>(base + pieces[6].off);
    d.hr = reinterpret_cast<const uint32_t *>(base + pieces[7].off);
    d.sc_h1 = h1 ? reinterpret_cast<const double *>(base + pieces[8].off) : nullptr;
    d.sc_eri = eri ? reinterpret_cast<const double *>(base + pieces[9].off) : nullptr;
    d.sc = h1 ? 1 : 0;
    d.sc_k = sc_k;
    d.n_groups = G;
    d.n_terms = Tn;
    d.n_qubits = T.n_qubits;
    d.has_diagonal = T.has_diagonal ? 1 : 0;
    d.sector_filter = T.sector_filter ? 1 : 0;
    d.sector32 = T.sector32 ? 1 : 0;
    d.spin_a0 = T.spin[0][0];
    d.spin_a1 = T.spin[0][1];
    d.spin_b0 = T.spin[1][0];
    d.spin_b1 = T.spin[1][1];
    d.enum_ok = T.enum_ok ? 1 : 0;
    d.k_alpha = T.k_alpha;
    d.k_beta = T.k_beta;
    d.spin_q = reinterpret_cast<const uint8_t *>(base + pieces[10].off);
    d.gh = reinterpret_cast<const uint32_t *>(base + pieces[11].off);
    d.gh_shift = T.gh_shift;
    d.qcls = reinterpret_cast<const uint8_t *>(base + pieces[12].off);
    d.max_flip = T.max_flip;
    d.join_blocks = T.max_flip + 1 <= nqs::kJoinMaxBlocks ? T.max_flip + 1 : 0;
    for (int b = 0; b < nqs::kJoinMaxBlocks; ++b) {
        d.jmask[b][0] = d.jmask[b][1] = 0;
        if (b >= d.join_blocks) continue;
        // block b: qubits [b nq / B, (b + 1) nq / B)
        const int q0 = b * T.n_qubits / d.join_blocks, q1 = (b + 1) * T.n_qubits / d.join_blocks;
        for (int q = q0; q < q1; ++q) d.jmask[b][q >> 6] |= 1ull << (q & 63);
    }
    d.diag_occ = T.diag_occ ? 1 : 0;
    d.diag = T.diag_occ ? reinterpret_cast<const double *>(base + pieces[13].off) : nullptr;
    d.diag32 = T.diag_occ ? reinterpret_cast<const float *>(base + pieces[14].off) : nullptr;
    d.diag_q8 = T.diag_occ ? reinterpret_cast<const int8_t *>(base + pieces[15].off) : nullptr;
    d.diag_scale = diag_scale;
    d.diag_jtiles = diag_jtiles;
    *out = h;
    return NQS_OK;
}

}  // namespace

extern "C" {

int nqs_ham_create(nqs_ham *out, int n_qubits, int64_t n_terms, const uint64_t *x_masks,
                   const uint64_t *z_masks, const double *coeffs, const uint64_t *spin_masks,
                   void *hip_stream) {
    if (!out) return fail(NQS_E_ARG, "null handle output");
    *out = nullptr;
    nqs::HostTable T;
    std::string err;
    int rc;
    try {
        rc = nqs::build_table(n_qubits, n_terms, x_masks, z_masks, coeffs, spin_masks, &T, &err);
        if (rc) return fail(rc, err);
        return create_handle(out, T, nullptr, nullptr, 0, static_cast<hipStream_t>(hip_stream));
    } catch (const std::bad_alloc &) {
        return fail(NQS_E_NOMEM, "host allocation failed");
    }
}

int nqs_ham_create_integrals(nqs_ham *out, int n_orbitals, const double *h1e, const double *eri,
                             void *hip_stream) {
    if (!out) return fail(NQS_E_ARG, "null handle output");
    *out = nullptr;
    if (!h1e || !eri) return fail(NQS_E_ARG, "null integral arrays");
    const int K = n_orbitals;
    if (K < 1 || 2 * K > nqs::kMaxQubits) return fail(NQS_E_RANGE, "n_orbitals must be in [1, 63]");
    try {
        const size_t K2 = size_t(K) * K;
        double scale = 0.0;
        for (size_t k = 0; k < K2; ++k) {
            if (!std::isfinite(h1e[k])) return fail(NQS_E_ARG, "non-finite h1e");
            scale = std::max(scale, std::fabs(h1e[k]));
        }
        for (size_t k = 0; k < K2 * K2; ++k) {
            if (!std::isfinite(eri[k])) return fail(NQS_E_ARG, "non-finite eri");
            scale = std::max(scale, std::fabs(eri[k]));
        }
        const double tol = 1e-12 * std::max(scale, 1e-300);
        auto E = [&](int p, int q, int r, int s) { return eri[((size_t(p) * K + q) * K + r) * K + s]; };
        for (int p = 0; p < K; ++p)
            for (int q = 0; q < K; ++q)
                if (std::fabs(h1e[size_t(p) * K + q] - h1e[size_t(q) * K + p]) > tol)
                    return fail(NQS_E_ARG, "h1e is not symmetric");
        const int npair = K * (K + 1) / 2;
        std::vector<double> packed(size_t(npair) * (npair + 1) / 2);
        for (int p = 0; p < K; ++p)
            for (int q = 0; q < K; ++q)
                for (int r = 0; r < K; ++r)
                    for (int s = 0; s < K; ++s) {
                        const double v = E(p, q, r, s);
                        // the 8-fold permutational symmetry of real orbitals
                        if (std::fabs(v - E(q, p, r, s)) > tol || std::fabs(v - E(p, q, s, r)) > tol ||
                            std::fabs(v - E(r, s, p, q)) > tol)
                            return fail(NQS_E_ARG, "eri lacks the 8-fold symmetry of real orbitals");
                        if (p >= q && r >= s) {
                            const size_t pq = size_t(p) * (p + 1) / 2 + q, rs = size_t(r) * (r + 1) / 2 + s;
                            if (pq >= rs) packed[pq * (pq + 1) / 2 + rs] = v;
                        }
                    }
        std::vector<double> h1(h1e, h1e + K2);
        nqs::HostTable T;
        std::string err;
        const int rc = nqs::build_flip_table(K, &T, &err);
        if (rc) return fail(rc, err);
        return create_handle(out, T, &h1, &packed, K, static_cast<hipStream_t>(hip_stream));
    } catch (const std::bad_alloc &) {
        return fail(NQS_E_NOMEM, "host allocation failed");
    }
}

int nqs_ham_info(nqs_ham h, int64_t *n_groups, int64_t *n_terms, int64_t *device_bytes) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (n_groups) *n_groups = h->dt.n_groups;
    if (n_terms) *n_terms = h->dt.n_terms;
    if (device_bytes)
        *device_bytes = h->table_bytes + static_cast<int64_t>(h->slot_bytes) +
                        h->shx_cap * 4 + h->part_cap * 8 + kSmallBytes +
                        static_cast<int64_t>(kMaxFilterWords * 4) +
                        (h->efilter ? static_cast<int64_t>(kMaxEFilterWords * 4) : 0) +
                        h->eblk_stride * h->eblk_blocks + static_cast<int64_t>(h->jmem_bytes);
    return NQS_OK;
}

int nqs_ham_destroy(nqs_ham h) {
    if (!h) return NQS_OK;
    int rc = NQS_OK;
    if (hipDeviceSynchronize() != hipSuccess) rc = fail(NQS_E_DEVICE, "synchronising before destroy");
    if (h->table_mem) (void)hipFree(h->table_mem);
    if (h->small) (void)hipFree(h->small);
    if (h->filter) (void)hipFree(h->filter);
    if (h->efilter) (void)hipFree(h->efilter);
    if (h->eblk) (void)hipFree(h->eblk);
    if (h->slots) (void)hipFree(h->slots);
    if (h->shx) (void)hipFree(h->shx);
    if (h->part) (void)hipFree(h->part);
    if (h->jmem) (void)hipFree(h->jmem);
    if (h->epart) (void)hipFree(h->epart);
    if (h->ehost) (void)hipHostFree(h->ehost);
    for (hipEvent_t e : h->ev)
        if (e) (void)hipEventDestroy(e);
    if (h->eval_exec) (void)hipGraphExecDestroy(h->eval_exec);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
    return rc;
}

int nqs_eloc_eval(nqs_ham h, int64_t n, const uint64_t *samples, const int64_t *weights,
                  const double *log_amp, const double *phase, double *eloc, int precision,
                  void *hip_stream) {
    return eval_impl(h, n, samples, weights, log_amp, phase, eloc, precision, nullptr, nullptr,
                     hip_stream);
}

int nqs_eloc_eval_noalloc(nqs_ham h, int64_t n, const uint64_t *samples, const int64_t *weights,
                          const double *log_amp, const double *phase, double *eloc, int precision,
                          void *hip_stream) {
    return eval_noalloc(h, n, samples, weights, log_amp, phase, eloc, precision, hip_stream);
}

int nqs_profile(nqs_ham h, int enable) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (enable && !h->ev[0]) {
        for (hipEvent_t &e : h->ev) NQS_HIP(hipEventCreate(&e));
    }
    h->profiling = enable != 0;
    h->profiled = false;
    return NQS_OK;
}

int nqs_last_kernel_ms(nqs_ham h, float out[3]) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (!out) return fail(NQS_E_ARG, "null output");
    if (!h->profiling || !h->profiled) return fail(NQS_E_STATE, "no profiled evaluation");
    NQS_HIP(hipEventSynchronize(h->ev[3]));
    NQS_HIP(hipEventElapsedTime(&out[0], h->ev[0], h->ev[1]));
    NQS_HIP(hipEventElapsedTime(&out[1], h->ev[1], h->ev[2]));
    NQS_HIP(hipEventElapsedTime(&out[2], h->ev[2], h->ev[3]));
    return NQS_OK;
}

int nqs_last_stage_ms(nqs_ham h, float out[6]) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (!out) return fail(NQS_E_ARG, "null output");
    if (!h->profiling || !h->profiled) return fail(NQS_E_STATE, "no profiled evaluation");
    NQS_HIP(hipEventSynchronize(h->ev[3]));
    // the events of the last evaluation: start, grouping done, hash done,
    // pairs done, lookup done, finish done (the grouping and pair events are
    // recorded on every profiled call, so they always belong to it)
    NQS_HIP(hipEventElapsedTime(&out[0], h->ev[0], h->ev[4]));
    NQS_HIP(hipEventElapsedTime(&out[1], h->ev[4], h->ev[1]));
    NQS_HIP(hipEventElapsedTime(&out[2], h->ev[1], h->ev[5]));
    NQS_HIP(hipEventElapsedTime(&out[3], h->ev[5], h->ev[2]));
    NQS_HIP(hipEventElapsedTime(&out[4], h->ev[2], h->ev[3]));
    NQS_HIP(hipEventElapsedTime(&out[5], h->ev[0], h->ev[3]));
    return NQS_OK;
}

int nqs_debug_dump(nqs_ham h, int64_t n, const uint64_t *samples, const double *log_amp,
                   const double *phase, double *eloc, int32_t *hit_idx, uint32_t *sign_bits,
                   void *hip_stream) {
    if (!hit_idx && !sign_bits) return fail(NQS_E_ARG, "no dump buffer given");
    return eval_impl(h, n, samples, nullptr, log_amp, phase, eloc, NQS_FP64, hit_idx, sign_bits,
                     hip_stream);
}

int nqs_sync(nqs_ham h, void *hip_stream) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    NQS_HIP(hipStreamSynchronize(st));
    int err = h->host_err.exchange(0);
    if (err == 0) {
        NQS_HIP(hipMemcpy(&err, static_cast<char *>(h->small) + kErrOffset, sizeof(int),
                          hipMemcpyDeviceToHost));
        if (err != 0) NQS_HIP(clear_device_error(h));
    }
    return report_device_error(err);
}

int nqs_eloc_energy(nqs_ham h, int64_t n, const uint64_t *samples, const int64_t *weights,
                    const double *log_amp, const double *phase, double *eloc, int precision,
                    double out[4], void *hip_stream) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (n <= 0) return fail(NQS_E_ARG, "n must be positive");
    if (!weights || !out) return fail(NQS_E_ARG, "null weights or output");
    if (n > (int64_t(1) << 30)) return fail(NQS_E_ARG, "batch larger than 2^30 samples");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // one partial set per block of the finish kernel (256 samples or more)
    const int64_t need = 4 * ((n + 255) / 256);
    if (need > h->epart_cap) {
        NQS_HIP(hipStreamSynchronize(st));
        const int rc = regrow(&h->epart, &h->epart_cap, need, sizeof(double) * need,
                              "the energy partials");
        if (rc) return rc;
    }
    if (!h->ehost) {
        void *p = nullptr;
        // fine-grained: the device's writes reach the host without a cache flush
        if (hipHostMalloc(&p, kEnergyHostBytes, hipHostMallocCoherent) != hipSuccess) {
            (void)hipGetLastError();
            return fail(NQS_E_NOMEM, "pinned host allocation failed");
        }
        std::memset(p, 0, kEnergyHostBytes);
        h->ehost = static_cast<char *>(p);
    }
    // the last kernel publishes a new sequence number after the results:
    // wait for it rather than for the stream (the stream's completion is
    // seen later); the stream's state ends the wait if the kernel never runs
    volatile unsigned *hseq = reinterpret_cast<volatile unsigned *>(h->ehost + kEnergyHostSeq);
    const volatile unsigned *hchosen =
        reinterpret_cast<const volatile unsigned *>(h->ehost + kEnergyHostChosen);
    // after a call that chose the join, launch only the join's kernels (the
    // enumeration and streaming launches would return at once); if the
    // device decides otherwise this time, evaluate again with every launch
    for (bool join_only = h->join_likely;; join_only = false) {
        const unsigned before = *hseq;
        const int rc = eval_impl(h, n, samples, weights, log_amp, phase, eloc, precision, nullptr,
                                 nullptr, hip_stream, true, join_only);
        if (rc) return rc;
        for (uint64_t k = 1; *hseq == before; ++k) {
            if ((k & 1023u) == 0) {
                const hipError_t q = hipStreamQuery(st);
                if (q == hipErrorNotReady) continue;
                if (q != hipSuccess) return fail_hip(q, "hipStreamQuery");
                if (*hseq == before) return fail(NQS_E_DEVICE, "the energy kernel did not report");
            }
        }
        std::atomic_thread_fence(std::memory_order_acquire);
        const unsigned chosen = *hchosen;
        h->join_likely = chosen == 1u;
        if (!join_only || chosen == 1u) break;
    }
    int err = h->host_err.exchange(0);
    if (err == 0) {
        std::memcpy(&err, h->ehost, sizeof(int));
        if (err != 0) NQS_HIP(clear_device_error(h));
    }
    if (err != 0) return report_device_error(err);
    std::memcpy(out, h->ehost + kEnergyHostOut, 4 * sizeof(double));
    if (out[3] == 0.0) return fail(NQS_E_ARG, "sum of weights is zero");
    return NQS_OK;
}

int nqs_eval_stats(nqs_ham h, int64_t out[6]) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (!out) return fail(NQS_E_ARG, "null output");
    if (!h->ever_evaluated) return fail(NQS_E_STATE, "no evaluation on this handle yet");
    unsigned long long slots[nqs::kCounters * nqs::kCounterSlots];
    NQS_HIP(hipMemcpy(slots, h->small, sizeof(slots), hipMemcpyDeviceToHost));
    unsigned long long c[nqs::kCounters] = {};
    for (int s = 0; s < nqs::kCounterSlots; ++s)
        for (int k = 0; k < nqs::kCounters; ++k) c[k] += slots[s * nqs::kCounters + k];
    out[0] = h->last_pairs;
    for (int k = 1; k < 5; ++k) out[k] = static_cast<int64_t>(c[k]);
    out[5] = static_cast<int64_t>(c[6]);
    return NQS_OK;
}

int nqs_eval_plan(nqs_ham h, int64_t out[8]) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (!out) return fail(NQS_E_ARG, "null output");
    if (!h->ever_evaluated) return fail(NQS_E_STATE, "no evaluation on this handle yet");
    const nqs::EvalLaunch &L = h->last_plan;
    out[0] = L.strategy;
    out[1] = L.strategy == nqs::kStrategyEnum ? (int64_t(1) << L.eparts_log2) : 0;
    out[2] = int64_t(1) << (L.eparts_log2 > 0 ? L.efilter_log2 : L.filter_log2);
    out[3] = L.chunk_len > 0 ? L.n_chunks : 0;
    out[4] = L.n;
    out[5] = int64_t(1) << L.filter_log2;
    out[6] = L.join ? h->dt.join_blocks : 0;
    out[7] = -1;
    if (L.join && h->last_jctl) {
        // the device's decision, in the control words of the join scratch
        unsigned long long chosen = 0;
        NQS_HIP(hipMemcpy(&chosen, h->last_jctl + nqs::kJoinCtlChosen, sizeof(chosen),
                          hipMemcpyDeviceToHost));
        out[7] = chosen ? 1 : 0;
    }
    return NQS_OK;
}

int nqs_debug_fail_allocs(int k) {
    if (k < 0) return fail(NQS_E_ARG, "k < 0");
    g_fail_at.store(k);
    return NQS_OK;
}

int nqs_energy(int64_t n, const int64_t *weights, const double *eloc, double out[4],
               void *hip_stream) {
    if (n <= 0) return fail(NQS_E_ARG, "n must be positive");
    if (!weights || !eloc || !out) return fail(NQS_E_ARG, "null pointer");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    int dev = 0;
    NQS_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_energy_mutex);
    EnergyScratch &es = g_energy[dev];
    if (!es.dev) {
        if (hipMalloc(&es.dev, sizeof(double) * (nqs::kEnergyPartDoubles + 8)) != hipSuccess) {
            es.dev = nullptr;
            return fail(NQS_E_NOMEM, "device allocation failed");
        }
        if (hipHostMalloc(&es.host, sizeof(double) * 4, hipHostMallocDefault) != hipSuccess) {
            (void)hipFree(es.dev);
            es.dev = nullptr;
            es.host = nullptr;
            return fail(NQS_E_NOMEM, "pinned host allocation failed");
        }
    }
    double *part = es.dev;
    double *dout = es.dev + nqs::kEnergyPartDoubles;
    NQS_HIP(nqs::launch_energy(weights, eloc, n, part, dout, st));
    NQS_HIP(hipMemcpyAsync(es.host, dout, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
    NQS_HIP(hipStreamSynchronize(st));
    std::memcpy(out, es.host, sizeof(double) * 4);
    if (out[3] == 0.0) return fail(NQS_E_ARG, "sum of weights is zero");
    return NQS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ tuning

namespace {

bool tuning_valid(const nqs_tuning &t) {
    const bool th = t.threads == 0 || t.threads == 256 || t.threads == 512 || t.threads == 1024;
    const bool fb = t.filter_bits == 0 || (t.filter_bits >= 4 && t.filter_bits <= 64);
    const bool bc = t.blocks_per_cu == 0 || (t.blocks_per_cu >= 1 && t.blocks_per_cu <= 64);
    const bool sg = t.strategy >= nqs::kStrategyAuto && t.strategy <= nqs::kStrategyJoin;
    return th && fb && bc && sg;
}

nqs_tuning filled(const nqs::Tuning &t) {
    nqs_tuning o{};
    o.threads = t.threads ? t.threads : 1024;
    o.filter_bits = t.filter_bits ? t.filter_bits : 16;
    o.blocks_per_cu = t.blocks_per_cu ? t.blocks_per_cu : 4;
    o.strategy = t.strategy;
    return o;
}

std::string shape_key(nqs_ham h, int64_t n, int precision) {
    const int lgn = n > 0 ? static_cast<int>(std::lround(std::log2(static_cast<double>(n)))) : 0;
    const int lgg = h->dt.n_groups > 0
                        ? static_cast<int>(std::lround(std::log2(static_cast<double>(h->dt.n_groups))))
                        : 0;
    char buf[96];
    // (jb: the pair join's blocks; shapes tuned before the join had none)
    std::snprintf(buf, sizeof(buf), "w%d_sec%d_s32_%d_en%d_jb%d_lgn%d_lgg%d_p%d", h->words,
                  h->dt.sector_filter, h->dt.sector32, h->dt.enum_ok, h->dt.join_blocks, lgn,
                  lgg, precision);
    return buf;
}

struct CacheEntry {
    nqs_tuning t;
    double ms;
};

// The cache file is a JSON object with one entry per line:
//   "key": {"threads": T, "filter_bits": F, "blocks_per_cu": B, "strategy": S, "ms": X},
std::map<std::string, CacheEntry> read_cache(const char *path) {
    std::map<std::string, CacheEntry> m;
    if (!path) return m;
    FILE *f = std::fopen(path, "r");
    if (!f) return m;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        char key[128];
        CacheEntry e{};
        if (std::sscanf(line, " \"%127[^\"]\": {\"threads\": %d, \"filter_bits\": %d, "
                              "\"blocks_per_cu\": %d, \"strategy\": %d, \"ms\": %lf",
                        key, &e.t.threads, &e.t.filter_bits, &e.t.blocks_per_cu, &e.t.strategy,
                        &e.ms) == 6 &&
            tuning_valid(e.t))
            m[key] = e;
    }
    std::fclose(f);
    return m;
}

bool write_cache(const char *path, const std::map<std::string, CacheEntry> &m) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\n");
    size_t k = 0;
    for (const auto &kv : m) {
        std::fprintf(f, "  \"%s\": {\"threads\": %d, \"filter_bits\": %d, \"blocks_per_cu\": %d, "
                        "\"strategy\": %d, \"ms\": %.6f}%s\n",
                     kv.first.c_str(), kv.second.t.threads, kv.second.t.filter_bits,
                     kv.second.t.blocks_per_cu, kv.second.t.strategy, kv.second.ms,
                     ++k < m.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

std::mutex g_cache_mutex;

}  // namespace

extern "C" {

int nqs_set_tuning(nqs_ham h, const nqs_tuning *t) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (!t) {
        h->tune = nqs::Tuning{0, 0, 0, 0};
        return NQS_OK;
    }
    if (!tuning_valid(*t)) return fail(NQS_E_ARG, "tuning value out of range");
    h->tune = nqs::Tuning{t->threads, t->filter_bits, t->blocks_per_cu, t->strategy};
    return NQS_OK;
}

int nqs_get_tuning(nqs_ham h, nqs_tuning *out) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (!out) return fail(NQS_E_ARG, "null output");
    *out = filled(h->tune);
    return NQS_OK;
}

int nqs_autotune(nqs_ham h, int64_t n, const uint64_t *samples, const double *log_amp,
                 const double *phase, double *eloc, int precision, const char *cache_path,
                 nqs_tuning *best, double *best_ms, void *hip_stream) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (n <= 0) return fail(NQS_E_ARG, "autotuning needs a non-empty batch");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const std::string key = shape_key(h, n, precision);
    {
        std::lock_guard<std::mutex> lock(g_cache_mutex);
        const auto cache = read_cache(cache_path);
        const auto it = cache.find(key);
        if (it != cache.end()) {
            h->tune = nqs::Tuning{it->second.t.threads, it->second.t.filter_bits,
                                  it->second.t.blocks_per_cu, it->second.t.strategy};
            if (best) *best = filled(h->tune);
            if (best_ms) *best_ms = -1.0;
            return NQS_OK;
        }
    }
    hipEvent_t e0, e1;
    NQS_HIP(hipEventCreate(&e0));
    NQS_HIP(hipEventCreate(&e1));
    const nqs::Tuning saved = h->tune;
    nqs::Tuning win{0, 0, 0, 0};
    double win_ms = 1e300;
    int rc = NQS_OK;
    // candidates: the streaming kernel's (threads, filter bits, items per
    // CU) grid, and for tables that allow it the enumeration's filter sizes
    std::vector<nqs::Tuning> cands;
    // first the built-in plan (the device picks the join or the other
    // strategy per batch): a forced strategy must beat it to be kept
    cands.push_back(nqs::Tuning{0, 0, 0, nqs::kStrategyAuto});
    for (int th : {256, 512, 1024})
        for (int fb : {8, 16, 32})
            for (int bc : {2, 4, 8}) cands.push_back(nqs::Tuning{th, fb, bc, nqs::kStrategyStream});
    if (h->dt.enum_ok)
        for (int fb : {8, 16, 32}) cands.push_back(nqs::Tuning{1024, fb, 4, nqs::kStrategyEnum});
    if (h->dt.join_blocks > 0) cands.push_back(nqs::Tuning{1024, 16, 4, nqs::kStrategyJoin});
    for (const nqs::Tuning &cand : cands) {
        h->tune = cand;
        float best_run = 1e30f;
        for (int rep = 0; rep < 4 && rc == NQS_OK; ++rep) {
            hipError_t e = hipEventRecord(e0, st);
            if (e == hipSuccess) {
                rc = eval_impl(h, n, samples, nullptr, log_amp, phase, eloc, precision, nullptr,
                               nullptr, st);
                if (rc) break;
                e = hipEventRecord(e1, st);
            }
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = fail_hip(e, "timing a candidate tuning");
                break;
            }
            if (rep > 0) best_run = std::min(best_run, ms);  // first run warms up
        }
        if (rc) break;
        if (best_run < win_ms) {
            win_ms = best_run;
            win = h->tune;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        h->tune = saved;
        return rc;
    }
    h->tune = win;
    if (best) *best = filled(win);
    if (best_ms) *best_ms = win_ms;
    if (cache_path) {
        std::lock_guard<std::mutex> lock(g_cache_mutex);
        auto cache = read_cache(cache_path);
        cache[key] = CacheEntry{filled(win), win_ms};
        if (!write_cache(cache_path, cache))
            return fail(NQS_E_STATE, std::string("cannot write tuning cache ") + cache_path);
    }
    // leave eloc holding the result of the chosen tuning
    return eval_impl(h, n, samples, nullptr, log_amp, phase, eloc, precision, nullptr, nullptr, st);
}

}  // extern "C"

// ------------------------------------------------------------------ batched form

struct nqs_batch_s {
    int precision = NQS_FP64;
    std::vector<nqs_ham> hams;
    std::vector<nqs::JobDesc> jobs;  // host copy of d_jobs (the join's per-job launches)
    std::vector<int64_t> ns;
    nqs::JobDesc *d_jobs = nullptr;
    nqs::WorkItem *d_items = nullptr;
    unsigned *d_next = nullptr;
    int n_jobs = 0;
    int n_items = 0;
    nqs::BatchShape shape{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void batch_free(nqs_batch b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_jobs) (void)hipFree(b->d_jobs);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_next) (void)hipFree(b->d_next);
    delete b;
}

void batch_mark(nqs_batch b) {
    for (size_t k = 0; k < b->hams.size(); ++k) {
        b->hams[k]->last_pairs = b->ns[k] * b->hams[k]->dt.n_groups;
        b->hams[k]->ever_evaluated = true;
        b->hams[k]->profiled = false;
    }
}

}  // namespace

extern "C" {

int nqs_batch_create(nqs_batch *out, int n_items, const nqs_batch_item *items, int precision,
                     int threads, void *hip_stream) {
    if (!out) return fail(NQS_E_ARG, "null batch output");
    *out = nullptr;
    if (precision != NQS_FP64 && precision != NQS_FP32_KAHAN)
        return fail(NQS_E_ARG, "unknown precision");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    std::vector<nqs::JobDesc> jobs;
    std::vector<nqs::WorkItem> work;
    nqs::BatchShape shape{};
    int rc = nqs::detail::plan_batch(items, n_items, threads, st, &jobs, &work, &shape);
    if (rc) return rc;
    nqs_batch b = new (std::nothrow) nqs_batch_s();
    if (!b) return fail(NQS_E_NOMEM, "host allocation failed");
    b->precision = precision;
    b->jobs = jobs;
    b->n_jobs = n_items;
    b->n_items = static_cast<int>(work.size());
    b->shape = shape;
    for (int k = 0; k < n_items; ++k) {
        b->hams.push_back(items[k].ham);
        b->ns.push_back(items[k].n);
    }
    hipError_t e = hipMalloc(&b->d_jobs, sizeof(nqs::JobDesc) * n_items);
    if (e == hipSuccess) e = hipMalloc(&b->d_items, sizeof(nqs::WorkItem) * std::max<size_t>(work.size(), 1));
    if (e == hipSuccess) e = hipMalloc(&b->d_next, nqs::kBatchCounters * sizeof(unsigned));
    if (e != hipSuccess) {
        batch_free(b);
        return fail(NQS_E_NOMEM, "device allocation of the batch plan failed");
    }
    e = hipMemcpyAsync(b->d_jobs, jobs.data(), sizeof(nqs::JobDesc) * n_items, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !work.empty())
        e = hipMemcpyAsync(b->d_items, work.data(), sizeof(nqs::WorkItem) * work.size(),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        batch_free(b);
        return fail_hip(e, "uploading the batch plan");
    }
    *out = b;
    return NQS_OK;
}

int nqs_batch_launch(nqs_batch b, void *hip_stream) {
    if (!b || !b->d_jobs) return fail(NQS_E_STATE, "invalid batch");
    NQS_HIP(nqs::launch_batch(b->d_jobs, b->n_jobs, b->d_items, b->n_items, b->d_next, b->shape,
                              b->precision, static_cast<hipStream_t>(hip_stream), b->jobs.data()));
    batch_mark(b);
    return NQS_OK;
}

int nqs_batch_capture(nqs_batch b, void *hip_stream) {
    if (!b || !b->d_jobs) return fail(NQS_E_STATE, "invalid batch");
    if (!hip_stream) return fail(NQS_E_ARG, "graph capture needs a non-default stream");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    // kernel attributes are set by one eager launch-free call before capture
    NQS_HIP(nqs::prepare_batch_kernels());
    NQS_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const hipError_t le = nqs::launch_batch(b->d_jobs, b->n_jobs, b->d_items, b->n_items,
                                            b->d_next, b->shape, b->precision, st,
                                            b->jobs.data());
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(st, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail_hip(le, "launching the batch under capture");
    }
    if (ce != hipSuccess) return fail_hip(ce, "hipStreamEndCapture");
    b->graph = g;
    NQS_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return NQS_OK;
}

int nqs_batch_replay(nqs_batch b, void *hip_stream) {
    if (!b || !b->exec) return fail(NQS_E_STATE, "no captured graph in this batch");
    NQS_HIP(hipGraphLaunch(b->exec, static_cast<hipStream_t>(hip_stream)));
    batch_mark(b);
    return NQS_OK;
}

int nqs_batch_destroy(nqs_batch b) {
    if (!b) return NQS_OK;
    const hipError_t e = hipDeviceSynchronize();
    batch_free(b);
    if (e != hipSuccess) return fail_hip(e, "synchronising before batch destroy");
    return NQS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ internals shared with the server

namespace nqs {
namespace detail {

bool valid_handle(nqs_ham h) { return ::valid_handle(h); }

int64_t table_bytes(nqs_ham h) { return h->table_bytes; }

int64_t scratch_bytes(nqs_ham h) {
    return static_cast<int64_t>(h->slot_bytes) + h->shx_cap * 4 + h->part_cap * 8 +
           static_cast<int64_t>(kSmallBytes + kMaxFilterWords * 4) +
           (h->efilter ? static_cast<int64_t>(kMaxEFilterWords * 4) : 0) +
           h->eblk_stride * h->eblk_blocks + static_cast<int64_t>(h->jmem_bytes);
}

int reserve(nqs_ham h, int64_t n, int threads, hipStream_t st) {
    nqs::Tuning t = h->tune;
    if (threads) t.threads = threads;
    n = std::max<int64_t>(n, 1);
    nqs::EvalLaunch L = nqs::plan_eval(h->dt, n, false, &t);
    L.join = 0;  // batches (and so the server) do not run the pair join
    // A batch of m <= n samples plans about (items per GPU) / tiles(m) chunks,
    // so m * chunks(m) <= items * threads + m: size the partials for that.
    const int64_t items = int64_t(t.blocks_per_cu ? t.blocks_per_cu : 4) * 256 * 1024 / L.threads;
    const int64_t bound = (items * L.threads + n + n - 1) / n;
    return ensure_scratch(h, n, std::max<int64_t>(L.n_chunks, bound), st, L.eparts_log2 > 0);
}

size_t request_scratch_bytes(nqs_ham h, int64_t n) {
    n = std::max<int64_t>(n, 1);
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess)
        n_cu = 256;
    const nqs::EvalLaunch L = nqs::plan_eval(h->dt, n, false, &h->tune);
    nqs::DevScratch sc{};
    return layout_scratch(h, L, n, n_cu, nullptr, 0, &sc);
}

size_t small_bytes() { return kSmallBytes; }
size_t small_err_offset() { return kErrOffset; }

int eval_in(nqs_ham h, const nqs_batch_item &it, int precision, char *ctx, size_t ctx_bytes,
            void *small, hipStream_t st) {
    if (!::valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (it.n <= 0) return NQS_OK;
    if (h->dt.sc) precision = NQS_FP64;  // the integral form evaluates in FP64 only
    int n_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device);
    if (e != hipSuccess) return fail_hip(e, "querying the device");
    const nqs::EvalLaunch L = nqs::plan_eval(h->dt, it.n, false, &h->tune);
    nqs::DevScratch sc{};
    const size_t need = layout_scratch(h, L, it.n, n_cu, nullptr, 0, &sc);
    if (need > ctx_bytes) return fail(NQS_E_ARG, "request larger than its lane's scratch");
    layout_scratch(h, L, it.n, n_cu, ctx, ctx_bytes, &sc, small);
    e = issue_eval(h, sc, L, it.n, it.samples, it.weights, it.log_amp, it.phase, it.eloc,
                   precision, nullptr, nullptr, st, false);
    if (e != hipSuccess) return fail_hip(e, "launching a served request");
    return NQS_OK;
}

void latch_host_error(nqs_ham h, int code) {
    int expected = 0;
    h->host_err.compare_exchange_strong(expected, code);
}

void mark_evaluated(nqs_ham h, int64_t n) {
    h->last_pairs = n * h->dt.n_groups;
    h->ever_evaluated = true;
    h->profiled = false;
}

int plan_batch(const nqs_batch_item *items, int n_items, int threads, hipStream_t st,
               std::vector<JobDesc> *jobs_out, std::vector<WorkItem> *work_out,
               BatchShape *shape_out) {
    if (n_items <= 0 || !items) return fail(NQS_E_ARG, "a batch needs at least one item");
    if (!(threads == 0 || threads == 256 || threads == 512 || threads == 1024))
        return fail(NQS_E_ARG, "threads must be 0, 256, 512 or 1024");
    const int th = threads ? threads : 1024;
    for (int k = 0; k < n_items; ++k) {
        const nqs_batch_item &it = items[k];
        if (!::valid_handle(it.ham)) return fail(NQS_E_ARG, "invalid handle in batch item");
        if (it.n < 0 || it.n > (int64_t(1) << 30)) return fail(NQS_E_ARG, "bad batch size");
        if (it.n > 0 && (!it.samples || !it.log_amp || !it.phase || !it.eloc))
            return fail(NQS_E_ARG, "null pointer in batch item");
        for (int m = 0; m < k; ++m)
            if (items[m].ham == it.ham) return fail(NQS_E_ARG, "a handle appears twice in a batch");
    }
    int dev = 0, n_cu = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he == hipSuccess) he = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (he != hipSuccess) return fail_hip(he, "querying the device");

    std::vector<JobDesc> &jobs = *jobs_out;
    std::vector<WorkItem> &work = *work_out;
    jobs.assign(n_items, JobDesc{});
    work.clear();
    std::vector<int64_t> cost(n_items);
    BatchShape shape{};
    shape.threads = th;
    shape.max_filter_log2 = 7;
    for (int k = 0; k < n_items; ++k) {
        const nqs_batch_item &it = items[k];
        nqs_ham h = it.ham;
        nqs::Tuning t = h->tune;
        t.threads = th;
        // enumeration rounds assume 1024-thread blocks
        if (th != kEnumThreads) t.strategy = kStrategyStream;
        EvalLaunch L = plan_eval(h->dt, std::max<int64_t>(it.n, 1), false, &t);
        if (it.n == 0) L.join = 0;
        if (L.strategy == kStrategyEnum && L.chunk_len > 0) {
            // the streaming items are only a fallback here (mixed sectors):
            // one group chunk keeps their number small
            L.n_chunks = 1;
            L.chunk_len = h->dt.n_groups - L.g_first;
        }
        int rc = ensure_scratch(h, std::max<int64_t>(it.n, 1), plan_chunks(h, L), st,
                                L.eparts_log2 > 0, plan_join_bytes(h, L));
        if (!rc) rc = scratch_ready(h, L);
        if (rc) return rc;
        JobDesc &J = jobs[k];
        J.tab = h->dt;
        J.sc = scratch_of(h);
        set_filters(&J.sc, h, L);
        J.samples = it.samples;
        J.weights = it.weights;
        J.log_amp = it.log_amp;
        J.phase = it.phase;
        J.eloc = it.eloc;
        J.n = it.n;
        J.g_first = L.g_first;
        J.chunk_len = L.chunk_len;
        J.n_chunks = L.n_chunks;
        const int w2 = h->words == 2 ? 1 : 0;
        J.kind = !h->dt.sector_filter ? (w2 ? kJobW2Nosec : kJobW1Nosec)
                 : h->dt.sector32     ? (w2 ? kJobW2S32 : kJobW1S32)
                                      : (w2 ? kJobW2S64 : kJobW1S64);
        if (h->dt.sc) J.kind += kJobIntegrals;
        J.capacity = h->slot_cap;
        J.strategy = L.strategy;
        shape.max_filter_log2 = std::max(shape.max_filter_log2, L.filter_log2);
        shape.max_n = std::max(shape.max_n, it.n);
        shape.max_clear = std::max<int64_t>(shape.max_clear,
                                            std::max<int64_t>(h->slot_cap, int64_t(1) << L.filter_log2));
        if (L.eparts_log2 > 0)
            shape.max_clear = std::max<int64_t>(shape.max_clear,
                                                int64_t(1) << (L.eparts_log2 + L.efilter_log2));
        if (J.sc.jctl)
            shape.max_clear = std::max<int64_t>(
                shape.max_clear, std::max<int64_t>(std::max<int64_t>(J.sc.join_parts, nqs::kJoinCtl),
                                                   (J.tab.join_blocks * J.n + 31) / 32));
        cost[k] = it.n * (h->dt.n_groups - L.g_first);
    }
    // work list: largest jobs first (the persistent kernel drains it in order),
    // chunk-major within a job so consecutive items share group records
    std::vector<int> order(n_items);
    for (int k = 0; k < n_items; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
    // enumeration items first, grouped by variant (rounds q, q + S,
    // q + 2 S, ... of a job; the round size is known on the device only),
    // then the streaming items
    for (int v = 0; v < kEnumVariants; ++v) {
        shape.enum_begin[v] = static_cast<int>(work.size());
        for (int k : order) {
            const JobDesc &J = jobs[k];
            if (J.n == 0 || J.strategy != kStrategyEnum) continue;
            const int jv = (J.kind & 1) + ((J.kind & kJobIntegrals) ? 2 : 0);
            if (jv != v) continue;
            const int64_t S = std::min<int64_t>((J.n + 63) / 64, int64_t(1) << 20);
            for (int64_t q = 0; q < S; ++q)
                work.push_back(WorkItem{k, -1, static_cast<int32_t>(q), static_cast<int32_t>(S)});
        }
    }
    shape.enum_begin[kEnumVariants] = static_cast<int>(work.size());
    for (int k : order) {
        const JobDesc &J = jobs[k];
        if (J.n == 0 || J.chunk_len == 0) continue;
        const int64_t tiles = (J.n + th - 1) / th;
        for (int64_t c = 0; c < J.n_chunks; ++c)
            for (int64_t t = 0; t < tiles; ++t)
                work.push_back(WorkItem{k, static_cast<int32_t>(c), static_cast<int32_t>(t), 0});
    }
    if (work.size() >= (size_t(1) << 31)) return fail(NQS_E_ARG, "work list too long");
    const size_t lds = batch_lds_bytes(th, shape.max_filter_log2);
    const int per_cu_lds = static_cast<int>((160 * 1024) / lds);
    const int per_cu_waves = (32 * 64) / th;
    shape.lookup_blocks = static_cast<unsigned>(n_cu * std::max(1, std::min(per_cu_lds, per_cu_waves)));
    shape.enum_blocks = static_cast<unsigned>(n_cu);
    *shape_out = shape;
    return NQS_OK;
}

}  // namespace detail
}  // namespace nqs
