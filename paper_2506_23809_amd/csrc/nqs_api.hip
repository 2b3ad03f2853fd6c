// C ABI of libnqs.so: handles, argument checks, scratch management, launches.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>

#include "../../include/nqs.h"
#include "nqs_device.hpp"
#include "nqs_table.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

int fail_hip(hipError_t e, const char *what) {
    return fail(NQS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define NQS_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return fail_hip(e_, #call); \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

constexpr size_t kSmallBytes = 128;                  // counters, error latch, sector flag
constexpr size_t kErrOffset = 8 * nqs::kCounters;    // after the counters
constexpr size_t kMaxFilterWords = size_t(1) << 15;  // 128 KB Bloom bitmap
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
    void *small = nullptr; // counters[8] u64, err, mixed
    int64_t last_pairs = 0;
    bool ever_evaluated = false;
    // optional per-stage events: hash start, hash end / lookup start,
    // lookup end / finish start, finish end
    bool profiling = false;
    bool profiled = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace {

nqs::DevScratch scratch_of(nqs_ham h) {
    nqs::DevScratch s{};
    s.slots = h->slots;
    s.shx = h->shx;
    s.part = h->part;
    s.filter = h->filter;
    s.counters = static_cast<unsigned long long *>(h->small);
    s.err = reinterpret_cast<int *>(static_cast<char *>(h->small) + kErrOffset);
    s.mixed = reinterpret_cast<int *>(static_cast<char *>(h->small) + kErrOffset + 4);
    uint32_t cap = h->slot_cap;
    s.slot_mask = cap - 1;
    int lg = 0;
    while ((1u << lg) < cap) ++lg;
    s.slot_shift = 32 - lg;
    return s;
}

// Grow the per-handle scratch to hold a batch of n samples.
int ensure_scratch(nqs_ham h, int64_t n, int64_t n_chunks, hipStream_t st) {
    uint64_t want = 64;
    while (want < 2 * static_cast<uint64_t>(n)) want <<= 1;
    if (want > (1ull << 31)) return fail(NQS_E_ARG, "batch too large for the sample hash");
    const size_t slot_size = h->words == 1 ? sizeof(nqs::Slot1) : sizeof(nqs::Slot2);
    const int64_t part_need = 2 * n * (n_chunks > 0 ? n_chunks : 1);
    const bool grow = want > h->slot_cap || n > h->shx_cap || part_need > h->part_cap;
    if (grow) {
        NQS_HIP(hipStreamSynchronize(st));
        if (want > h->slot_cap) {
            if (h->slots) NQS_HIP(hipFree(h->slots));
            h->slots = nullptr;
            if (hipMalloc(&h->slots, want * slot_size) != hipSuccess)
                return fail(NQS_E_NOMEM, "device allocation of the sample hash failed");
            h->slot_cap = static_cast<uint32_t>(want);
            h->slot_bytes = want * slot_size;
        }
        if (n > h->shx_cap) {
            if (h->shx) NQS_HIP(hipFree(h->shx));
            h->shx = nullptr;
            if (hipMalloc(&h->shx, sizeof(uint32_t) * n) != hipSuccess)
                return fail(NQS_E_NOMEM, "device allocation of sample hashes failed");
            h->shx_cap = n;
        }
        if (part_need > h->part_cap) {
            if (h->part) NQS_HIP(hipFree(h->part));
            h->part = nullptr;
            if (hipMalloc(&h->part, sizeof(double) * part_need) != hipSuccess)
                return fail(NQS_E_NOMEM, "device allocation of partial sums failed");
            h->part_cap = part_need;
        }
    }
    return NQS_OK;
}

bool valid_handle(nqs_ham h) { return h && h->table_mem && h->small; }

int eval_impl(nqs_ham h, int64_t n, const uint64_t *samples, const int64_t *weights,
              const double *log_amp, const double *phase, double *eloc, int precision,
              int32_t *hit_idx, uint32_t *sign_bits, void *stream) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (n < 0) return fail(NQS_E_ARG, "n < 0");
    if (precision != NQS_FP64 && precision != NQS_FP32_KAHAN)
        return fail(NQS_E_ARG, "unknown precision");
    if (n == 0) return NQS_OK;
    if (!samples || !log_amp || !phase || !eloc)
        return fail(NQS_E_ARG, "null sample, amplitude, phase or output pointer");
    if (n > (int64_t(1) << 30)) return fail(NQS_E_ARG, "batch larger than 2^30 samples");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool dump = hit_idx || sign_bits;
    const nqs::EvalLaunch L = nqs::plan_eval(h->dt, n, dump);
    int rc = ensure_scratch(h, n, L.n_chunks, st);
    if (rc) return rc;
    nqs::DevScratch sc = scratch_of(h);
    sc.filter_log2 = L.filter_log2;
    NQS_HIP(nqs::launch_reset(sc, st));
    if (h->profiling) NQS_HIP(hipEventRecord(h->ev[0], st));
    NQS_HIP(nqs::launch_hash(h->dt, sc, h->slot_cap, samples, weights, n, st));
    if (h->profiling) NQS_HIP(hipEventRecord(h->ev[1], st));
    const int64_t sign_words = (h->dt.n_terms + 31) / 32;
    nqs::EvalStageEvents stages{h->profiling ? h->ev[2] : nullptr};
    NQS_HIP(nqs::launch_eloc(h->dt, sc, L, samples, log_amp, phase, eloc, precision, hit_idx,
                             sign_bits, sign_words, stages, st));
    if (h->profiling) {
        NQS_HIP(hipEventRecord(h->ev[3], st));
        h->profiled = true;
    }
    h->last_pairs = n * h->dt.n_groups;
    h->ever_evaluated = true;
    return NQS_OK;
}

// Process-wide scratch of nqs_energy, one per device, used under a lock.
struct EnergyScratch {
    double *dev = nullptr;   // part[3*256] | result[3] | out[4]
    double *host = nullptr;  // pinned out[4]
};
std::mutex g_energy_mutex;
std::unordered_map<int, EnergyScratch> g_energy;

}  // namespace

extern "C" {

const char *nqs_last_error(void) { return g_last_error.c_str(); }

int nqs_version(void) { return 100; }

int nqs_table_host(int n_qubits, int64_t n_terms, const uint64_t *x_masks,
                   const uint64_t *z_masks, const double *coeffs, int64_t *n_groups,
                   int64_t *n_merged, uint64_t *group_x, int64_t *group_off, uint64_t *term_z,
                   double *term_c) {
    if (!n_groups || !n_merged) return fail(NQS_E_ARG, "null count outputs");
    nqs::HostTable T;
    std::string err;
    int rc;
    try {
        rc = nqs::build_table(n_qubits, n_terms, x_masks, z_masks, coeffs, nullptr, &T, &err);
    } catch (const std::bad_alloc &) {
        return fail(NQS_E_NOMEM, "host allocation failed");
    }
    if (rc) return fail(rc, err);
    *n_groups = T.n_groups;
    *n_merged = T.n_terms;
    if (group_x) std::memcpy(group_x, T.gx.data(), sizeof(uint64_t) * T.gx.size());
    if (group_off) std::memcpy(group_off, T.goff.data(), sizeof(int64_t) * T.goff.size());
    if (term_z) std::memcpy(term_z, T.tz.data(), sizeof(uint64_t) * T.tz.size());
    if (term_c) std::memcpy(term_c, T.tc.data(), sizeof(double) * T.tc.size());
    return NQS_OK;
}

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
    } catch (const std::bad_alloc &) {
        return fail(NQS_E_NOMEM, "host allocation failed");
    }
    if (rc) return fail(rc, err);
    if (T.n_groups >= kMaxGroups) return fail(NQS_E_ARG, "more than 2^26 X groups");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);

    const int64_t G = T.n_groups, Tn = T.n_terms;
    // one allocation holding every table array, each 256-byte aligned
    std::vector<float> tc32(2 * static_cast<size_t>(Tn));
    for (int64_t t = 0; t < Tn; ++t) {
        const float hi = static_cast<float>(T.tc[t]);
        tc32[2 * t] = hi;
        tc32[2 * t + 1] = static_cast<float>(T.tc[t] - static_cast<double>(hi));
    }
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
    };
    size_t total = 0;
    for (Piece &p : pieces) {
        p.off = total;
        total = align_up(total + (p.bytes ? p.bytes : 1), 256);
    }
    nqs_ham h = new (std::nothrow) nqs_ham_s();
    if (!h) return fail(NQS_E_NOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return fail_hip(e, "hipGetDevice");
    }
    if (hipMalloc(&h->table_mem, total) != hipSuccess) {
        delete h;
        return fail(NQS_E_NOMEM, "device allocation of the Pauli table failed");
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
        return fail_hip(e, "uploading the Pauli table");
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
    d.n_groups = G;
    d.n_terms = Tn;
    d.n_qubits = n_qubits;
    d.has_diagonal = T.has_diagonal ? 1 : 0;
    d.sector_filter = T.sector_filter ? 1 : 0;
    d.sector32 = T.sector32 ? 1 : 0;
    d.spin_a0 = T.spin[0][0];
    d.spin_a1 = T.spin[0][1];
    d.spin_b0 = T.spin[1][0];
    d.spin_b1 = T.spin[1][1];
    *out = h;
    return NQS_OK;
}

int nqs_ham_info(nqs_ham h, int64_t *n_groups, int64_t *n_terms, int64_t *device_bytes) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (n_groups) *n_groups = h->dt.n_groups;
    if (n_terms) *n_terms = h->dt.n_terms;
    if (device_bytes)
        *device_bytes = h->table_bytes + static_cast<int64_t>(h->slot_bytes) +
                        h->shx_cap * 4 + h->part_cap * 8 + kSmallBytes +
                        static_cast<int64_t>(kMaxFilterWords * 4);
    return NQS_OK;
}

int nqs_ham_destroy(nqs_ham h) {
    if (!h) return NQS_OK;
    int rc = NQS_OK;
    if (hipDeviceSynchronize() != hipSuccess) rc = fail(NQS_E_DEVICE, "synchronising before destroy");
    if (h->table_mem) (void)hipFree(h->table_mem);
    if (h->small) (void)hipFree(h->small);
    if (h->filter) (void)hipFree(h->filter);
    if (h->slots) (void)hipFree(h->slots);
    if (h->shx) (void)hipFree(h->shx);
    if (h->part) (void)hipFree(h->part);
    for (hipEvent_t e : h->ev)
        if (e) (void)hipEventDestroy(e);
    delete h;
    return rc;
}

int nqs_eloc_eval(nqs_ham h, int64_t n, const uint64_t *samples, const int64_t *weights,
                  const double *log_amp, const double *phase, double *eloc, int precision,
                  void *hip_stream) {
    return eval_impl(h, n, samples, weights, log_amp, phase, eloc, precision, nullptr, nullptr,
                     hip_stream);
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
    int err = 0;
    NQS_HIP(hipMemcpy(&err, static_cast<char *>(h->small) + kErrOffset, sizeof(int),
                      hipMemcpyDeviceToHost));
    if (err != 0) {
        const int zero = 0;
        NQS_HIP(hipMemcpy(static_cast<char *>(h->small) + kErrOffset, &zero, sizeof(int),
                          hipMemcpyHostToDevice));
        switch (err) {
            case NQS_E_DUPLICATE: return fail(err, "a sample occurs more than once in the batch");
            case NQS_E_RANGE: return fail(err, "a sample has bits at or above n_qubits, or a count is negative");
            default: return fail(err, "device-detected error");
        }
    }
    return NQS_OK;
}

int nqs_eval_stats(nqs_ham h, int64_t out[5]) {
    if (!valid_handle(h)) return fail(NQS_E_STATE, "invalid handle");
    if (!out) return fail(NQS_E_ARG, "null output");
    if (!h->ever_evaluated) return fail(NQS_E_STATE, "no evaluation on this handle yet");
    unsigned long long c[nqs::kCounters];
    NQS_HIP(hipMemcpy(c, h->small, sizeof(c), hipMemcpyDeviceToHost));
    out[0] = h->last_pairs;
    for (int k = 1; k < 5; ++k) out[k] = static_cast<int64_t>(c[k]);
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
    double *result = es.dev + nqs::kEnergyPartDoubles;
    double *dout = result + 4;
    NQS_HIP(nqs::launch_energy(weights, eloc, n, part, result, dout, st));
    NQS_HIP(hipMemcpyAsync(es.host, dout, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
    NQS_HIP(hipStreamSynchronize(st));
    std::memcpy(out, es.host, sizeof(double) * 4);
    if (out[3] == 0.0) return fail(NQS_E_ARG, "sum of weights is zero");
    return NQS_OK;
}

}  // extern "C"
