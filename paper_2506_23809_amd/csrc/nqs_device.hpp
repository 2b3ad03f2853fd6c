// Device-side data structures shared by the kernels and the host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nqs {

// Resident Pauli table (structure of arrays, all device pointers).
struct DevTable {
    const uint64_t *gx;    // [G][2] flip masks
    const uint64_t *gxa;   // [G][2] alpha part of the flip mask
    const uint64_t *gxb;   // [G][2] beta part of the flip mask
    const uint32_t *gmeta; // [G] half counts | infeasible bit 16
    const uint32_t *ghx;   // [G] linear hash of the flip mask
    const uint32_t *goff;  // [G + 1] term offsets
    const uint64_t *tz;    // [T][2] Z masks
    const double *tc;      // [T] folded coefficients
    const float *tc32;     // [T][2] coefficients as FP32 (hi, lo) pairs
    const uint32_t *hr;    // [128] linear-hash words
    int64_t n_groups;
    int64_t n_terms;
    int n_qubits;
    int has_diagonal;
    int sector_filter;
    uint64_t spin_a0, spin_a1, spin_b0, spin_b1;
};

// Per-handle scratch for one batch.
struct DevScratch {
    void *slots;            // hash slots (layout depends on the word count)
    uint32_t *shx;          // [n] linear hash of each sample
    double *part;           // [n_chunks][n][2] partial E_loc per group chunk
    unsigned long long *counters;  // [4] pairs, probes, hits, terms
    int *err;               // first device-detected error (0 = none)
    int *mixed;             // set when samples span more than one sector
    uint32_t slot_mask;     // capacity - 1 (capacity is a power of two)
    uint32_t slot_shift;    // 32 - log2(capacity)
};

constexpr uint32_t kMetaInfeasibleBit = 1u << 16;
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

}  // namespace nqs

namespace nqs {

// Launch plan of one evaluation: sample tiles x group chunks.
struct EvalLaunch {
    int64_t n;
    int64_t n_chunks;
    int64_t chunk_len;
    int64_t g_first;
};

// Optional event recorded between the lookup and the finish kernels.
struct EvalStageEvents {
    hipEvent_t after_lookup;
};

EvalLaunch plan_eval(const DevTable &tab, int64_t n, bool dump);
hipError_t launch_reset(const DevScratch &sc, hipStream_t st);
hipError_t launch_hash(const DevTable &tab, const DevScratch &sc, uint32_t capacity,
                       const uint64_t *samples, const int64_t *weights, int64_t n,
                       hipStream_t st);
hipError_t launch_eloc(const DevTable &tab, const DevScratch &sc, const EvalLaunch &L,
                       const uint64_t *samples, const double *log_amp, const double *phase,
                       double *eloc, int precision, int32_t *hit_idx, uint8_t *sign_bits,
                       int64_t sign_stride, EvalStageEvents ev, hipStream_t st);
hipError_t launch_energy(const int64_t *w, const double *e, int64_t n, double *part,
                         double *result, double *out, hipStream_t st);
constexpr int kEnergyPartDoubles = 3 * 256;

}  // namespace nqs
