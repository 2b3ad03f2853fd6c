// Device-side data structures shared by the kernels and the host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nqs {

// Resident Pauli table (structure of arrays, all device pointers).
struct DevTable {
    const uint64_t *gx;    // [G][2] flip masks
    const uint64_t *gsec;  // [G][2] flip mask compressed to (alpha bits, beta bits)
    const uint32_t *ghm;   // [G][2] (linear hash of X, sector key)
    const uint32_t *goff;  // [G + 1] term offsets
    const uint64_t *tz;    // [T][2] Z masks
    const double *tc;      // [T] folded coefficients
    const float *tc32;     // [T][2] coefficients as FP32 (hi, lo) pairs
    const uint32_t *hr;    // [128] linear-hash words
    const double *sc_h1;   // integral form: h_pq [K][K]
    const double *sc_eri;  // integral form: (pq|rs), 8-fold packed by compound index
    int sc;                // 1: matrix elements from the integrals (no Pauli terms)
    int sc_k;              // spatial orbitals of the integral form
    int64_t n_groups;
    int64_t n_terms;
    int n_qubits;
    int has_diagonal;
    int sector_filter;     // compressed sector test available
    int sector32;          // both compressed widths fit in 32 bits
    uint64_t spin_a0, spin_a1, spin_b0, spin_b1;
};

// Sector key of a group: (half popcount of its alpha flips) | (half popcount
// of its beta flips) << 8.  A flip x -> x ^ X keeps (N_alpha, N_beta) iff
// popc(x & X_alpha) | popc(x & X_beta) << 8 equals the key.  Flips with an
// odd alpha or beta popcount always leave the sector and get a key no sample
// can produce.
constexpr uint32_t kSectorNever = 0xFFFFu;

// Per-handle scratch for one batch.
struct DevScratch {
    void *slots;            // hash slots (layout depends on the word count)
    uint32_t *shx;          // [n] linear hash of each sample
    uint32_t *filter;       // [1 << filter_log2 words] Bloom bitmap of sample hashes
    double *part;           // [n_chunks][n][2] partial E_loc per group chunk
    unsigned long long *counters;  // [8] pairs, probes, hits, terms, candidates
    int *err;               // first device-detected error (0 = none)
    int *mixed;             // set when samples span more than one sector
    uint32_t slot_mask;     // capacity - 1 (capacity is a power of two)
    uint32_t slot_shift;    // 32 - log2(capacity)
    int filter_log2;        // log2 of the filter size in 32-bit words
};

constexpr uint32_t kGoldenMul = 0x9E3779B1u;

// Hash slots.  The claim protocol CASes idx from -1 to the sample index and
// then stores the key; lookups run in a later kernel, so keys are visible.
struct alignas(16) Slot1 {
    uint64_t k0;
    int32_t idx;
    int32_t pad;
};
struct alignas(32) Slot2 {
    uint64_t k0, k1;
    int32_t idx;
    int32_t pad[3];
};

// Launch plan of one evaluation: sample tiles x group chunks.
struct EvalLaunch {
    int64_t n;
    int64_t n_chunks;
    int64_t chunk_len;
    int64_t g_first;
    int threads;        // lookup kernel block size
    int filter_log2;    // filter words = 1 << filter_log2
    size_t lds_bytes;   // dynamic LDS of the lookup kernel
};

// Optional event recorded between the lookup and the finish kernels.
struct EvalStageEvents {
    hipEvent_t after_lookup;
};

// Launch parameters chosen by the autotuner; 0 means the built-in default
// (1024 threads, 16 filter bits per sample, about 4 lookup blocks per CU's
// worth of 1024-thread blocks).
struct Tuning {
    int threads;        // lookup block size: 256, 512 or 1024
    int filter_bits;    // Bloom bits per sample (the bitmap is capped at 128 KB)
    int blocks_per_cu;  // target (tile, chunk) items per CU
};

EvalLaunch plan_eval(const DevTable &tab, int64_t n, bool dump, const Tuning *tune);
hipError_t launch_reset(const DevScratch &sc, hipStream_t st);
hipError_t launch_hash(const DevTable &tab, const DevScratch &sc, uint32_t capacity,
                       const uint64_t *samples, const int64_t *weights, int64_t n,
                       hipStream_t st);
hipError_t launch_eloc(const DevTable &tab, const DevScratch &sc, const EvalLaunch &L,
                       const uint64_t *samples, const double *log_amp, const double *phase,
                       double *eloc, int precision, int32_t *hit_idx, uint32_t *sign_bits,
                       int64_t sign_words, EvalStageEvents ev, hipStream_t st);
hipError_t launch_energy(const int64_t *w, const double *e, int64_t n, double *part,
                         double *result, double *out, hipStream_t st);
constexpr int kEnergyPartDoubles = 3 * 256;
constexpr int kCounters = 8;

// ---- batched form

// Lookup variant of a job: bit 0 = two mask words, then the sector test.
enum JobKind : int {
    kJobW1Nosec = 0, kJobW2Nosec = 1,
    kJobW1S32 = 2, kJobW2S32 = 3,
    kJobW1S64 = 4, kJobW2S64 = 5,
    kJobIntegrals = 8,  // added to a sector kind: Slater-Condon elements
};

struct JobDesc {
    DevTable tab;
    DevScratch sc;
    const uint64_t *samples;
    const int64_t *weights;
    const double *log_amp;
    const double *phase;
    double *eloc;
    int64_t n;
    int64_t g_first;
    int64_t chunk_len;
    int64_t n_chunks;
    int kind;
    uint32_t capacity;  // hash slots
};

struct WorkItem {
    int32_t job;
    int32_t chunk;
    int32_t tile;
    int32_t pad;
};

struct BatchShape {
    int threads;          // lookup block size, shared by all jobs
    int max_filter_log2;  // largest Bloom bitmap (sets the dynamic LDS)
    int64_t max_n;        // largest batch
    int64_t max_clear;    // largest of slot capacity and filter words
    unsigned lookup_blocks;
};

hipError_t launch_batch(const JobDesc *d_jobs, int n_jobs, const WorkItem *d_items, int n_items,
                        unsigned *d_next, const BatchShape &shape, int precision, hipStream_t st);
size_t batch_lds_bytes(int threads, int max_filter_log2);
// Set the dynamic-LDS limit of the batch kernels (outside any graph capture).
hipError_t prepare_batch_kernels();

}  // namespace nqs
