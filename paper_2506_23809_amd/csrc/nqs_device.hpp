// Device-side data structures shared by the kernels and the host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "nqs_table.hpp"

namespace nqs {

// The occupation-form diagonal for the matrix cores: digit tiles of the
// 16 x 16 x 64 int8 MFMA (64 lanes x 16 bytes each, kDiagLimbs byte planes:
// two per base-2^15 digit; see build_diag_tiles).  Column tile jt (qubits j in [16 jt, 16 jt + 16))
// needs the rows i <= j: one k-block of 64 rows for jt < 4, two after.
constexpr int kDiagTileBytes = 64 * 16;
__host__ __device__ constexpr int diag_mfma_tiles(int jtiles) {
    return jtiles <= 4 ? jtiles : 4 + 2 * (jtiles - 4);
}

// Pair join: at most this many qubit blocks (a table whose groups flip up to
// kJoinMaxBlocks - 1 qubits).
constexpr int kJoinMaxBlocks = 8;

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
    // flip enumeration
    int enum_ok;           // every in-sector group is a single or double excitation
    int k_alpha, k_beta;   // qubits per spin
    const uint8_t *spin_q; // [128]: alpha qubits at [0, k_alpha), beta at [64, 64 + k_beta)
    const uint32_t *gh;    // group index slots (0xFFFFFFFF = empty)
    uint32_t gh_shift;     // 32 - log2(slots)
    const uint8_t *qcls;   // [128] class of each qubit (filter partitions)
    // the X = 0 group in occupation form (when its Z strings have at most two
    // qubits): d[0], d[1 + j], d[1 + nq + j (j - 1) / 2 + i] for i < j; FP64
    // and FP32 (hi, lo) pairs
    int diag_occ;
    const double *diag;
    const float *diag32;
    // the same form for the matrix cores (see kDiagDigits): digit tiles
    // [diag_mfma_tiles(diag_jtiles)][kDiagLimbs][64][16], 2^-S, and the
    // column tiles (ceil(n_qubits / 16); 0 without the form)
    const int8_t *diag_q8;
    double diag_scale;
    int diag_jtiles;
    // pair join: the qubits split into join_blocks disjoint blocks (jmask);
    // two bit strings at Hamming distance at most max_flip < join_blocks
    // agree on at least one block (pigeonhole), so every connected pair of
    // samples shares the contents of some block
    int max_flip;          // largest popc(X) over the groups
    int join_blocks;       // max_flip + 1, or 0 when that exceeds kJoinMaxBlocks
    uint64_t jmask[kJoinMaxBlocks][2];
};

// ---- flip enumeration: shape of one round
//
// A block evaluates B samples per round.  Per sample it keeps in LDS a
// 64-byte record, its occupied/virtual qubit lists (4 x 64 bytes), one
// accumulator per wave (16 x 16 bytes), 128 bytes of bucket counts and
// offsets, and the row hashes (u32) of three lists, each padded to a multiple
// of 4 entries:
//   rows of A  = beta singles + none      (sorted by class)
//   rows of Ba = alpha occupied pairs
//   rows of Bb = beta occupied pairs      (sorted by class)
// and, in the block's area of device scratch, the flip codes (u16) of those
// rows and of the fourth list, whose hashes (u32) sit there too:
//   cols of Bb = beta virtual pairs       (sorted by class)
// (a column is read once per work unit, a row code only for a candidate its
// fingerprints do not settle).  The products are
//   A  = (beta singles + none) x (alpha singles + none), without (none, none)
//   Ba = alpha occupied pairs x alpha virtual pairs
//   Bb = beta occupied pairs x beta virtual pairs
// (alpha columns are computed in registers).  B is the largest count (at
// most 16) that fits beside the filter and the queues.
constexpr int kEnumThreads = 1024;
constexpr int kEnumWaves = kEnumThreads / 64;
constexpr int kEnumQueue = 64;     // (code, hash) entries per wave
constexpr int kEnumMaxB = 16;
constexpr int kEnumMaxParts = 8;   // filter partitions (sample classes)
// LDS of one CU (160 KB) less 64 bytes for the scalar variables of the
// persistent batch kernel; every enumeration block takes all of it: a static
// 128 KB filter (whatever its used size) and the dynamic rest
constexpr int kEnumLds = 160 * 1024 - 64;
constexpr int kEnumFilterWords = 1 << 15;
constexpr int kEnumDynLds = kEnumLds - 4 * kEnumFilterWords;
constexpr int kEnumScalars = 64;
constexpr int kEnumRowPad = 32;    // rows may be read 3 entries past the end
// dynamic LDS: hash words (512 B), qubit classes (128 B), queues, scalars,
// padding, then the per-sample records
constexpr int kEnumQueueOff = 512 + 128;
constexpr int kEnumScalarOff = kEnumQueueOff + kEnumWaves * kEnumQueue * 8;
constexpr int kEnumDynFixed = kEnumScalarOff + kEnumScalars + kEnumRowPad;
constexpr int kEnumPerSampleFixed = 64 + 256 + kEnumWaves * 16 + 128;

__host__ __device__ inline int enum_pairs(int m) { return m * (m - 1) / 2; }
__host__ __device__ inline int enum_pad4(int m) { return (m + 3) & ~3; }

// Row entries per sample (padded): rows of A, Ba and Bb.
__host__ __device__ inline int enum_row_entries(int ka, int kb, int na, int nb) {
    (void)ka;
    return enum_pad4(1 + nb * (kb - nb)) + enum_pad4(enum_pairs(na)) + enum_pad4(enum_pairs(nb));
}

// List entries per sample (padded): rows of A, Ba, Bb and columns of Bb.
__host__ __device__ inline int enum_list_entries(int ka, int kb, int na, int nb) {
    return enum_row_entries(ka, kb, na, nb) + enum_pad4(enum_pairs(kb - nb));
}

// Samples per round for the given occupation, 0 if one does not fit (16
// bytes stay free after the last sample: rows are read up to 3 entries past
// a list's end).
__host__ __device__ inline int enum_round_size(int ka, int kb, int na, int nb) {
    const int per = kEnumPerSampleFixed + 4 * enum_row_entries(ka, kb, na, nb);
    const int b = (kEnumDynLds - kEnumDynFixed - 16) / per;
    return b < kEnumMaxB ? b : kEnumMaxB;
}

// Device scratch of one block in its rounds: B x L flip codes (u16), then,
// 16-byte aligned, B x (Bb columns) hashes (u32).
__host__ __device__ inline int64_t enum_blk_codes_bytes(int B, int L) {
    return (2 * static_cast<int64_t>(B) * L + 15) & ~static_cast<int64_t>(15);
}
__host__ __device__ inline int64_t enum_blk_bytes(int ka, int kb, int na, int nb) {
    const int B = enum_round_size(ka, kb, na, nb);
    if (B <= 0) return 0;
    return enum_blk_codes_bytes(B, enum_list_entries(ka, kb, na, nb)) +
           4 * static_cast<int64_t>(B) * enum_pad4(enum_pairs(kb - nb));
}

// Solo rounds, for occupations whose lists are small (at most 32 qubits per
// spin and one filter partition): each wave evaluates its own samples, one at
// a time, with no block barrier after the filter load.  Per wave it keeps its
// sample's orbital lists (4 x 32 bytes) and the rows of A, Ba and Bb (hash
// u32, then flip code u16; columns are computed in registers); the queue is
// the wave's usual one.
constexpr int kEnumSoloLists = 128;
__host__ __device__ inline int enum_solo_bytes(int row_entries) {
    return (kEnumSoloLists + 6 * row_entries + 15) & ~15;
}
// After the waves' areas, shared by the block: the entry table (u16 per row
// list position) and the task table (u32 per lane and chunk).
__host__ __device__ inline int enum_solo_entry_off(int row_entries) {
    return kEnumDynFixed + kEnumWaves * enum_solo_bytes(row_entries);
}
__host__ __device__ inline int enum_solo_task_off(int row_entries) {
    return enum_solo_entry_off(row_entries) + ((2 * row_entries + 15) & ~15);
}

// Sector key of a group: (half popcount of its alpha flips) | (half popcount
// of its beta flips) << 8.  A flip x -> x ^ X keeps (N_alpha, N_beta) iff
// popc(x & X_alpha) | popc(x & X_beta) << 8 equals the key.  Flips with an
// odd alpha or beta popcount always leave the sector and get a key no sample
// can produce.
constexpr uint32_t kSectorNever = 0xFFFFu;

// Per-handle scratch for one batch.
struct DevScratch {
    uint64_t *skey;         // [capacity][words] sample keys (kFreeKey in the last word: free)
    int32_t *sidx;          // [capacity] sample index of each claimed slot (-1: free)
    uint32_t *sfp;          // [capacity] fingerprint h(key) | 1 of each claimed slot (0: free)
    uint32_t *shx;          // [n] linear hash of each sample
    uint32_t *filter;       // [1 << filter_log2 words] Bloom bitmap of sample hashes
    double *part;           // [n_chunks][n][2] partial E_loc per group chunk
    unsigned long long *counters;  // [8] pairs, probes, hits, terms, candidates
    int *err;               // first device-detected error (0 = none)
    int *mixed;             // set when samples span more than one sector
    uint32_t slot_mask;     // capacity - 1 (capacity is a power of two)
    uint32_t slot_shift;    // 32 - log2(capacity)
    int filter_log2;        // log2 of the filter size in 32-bit words
    // filter of the enumeration: 1 << eparts_log2 partitions (sample classes)
    // of 1 << efilter_log2 words; with one partition it is the filter above
    uint32_t *efilter;
    int eparts_log2;
    int efilter_log2;
    // the enumeration blocks' areas (codes and Bb columns of their rounds):
    // eblk_blocks areas of eblk_stride bytes
    char *eblk;
    int64_t eblk_stride;
    uint32_t eblk_blocks;
    // pair join (all null when the launch plans none).  A bucket is
    // (block b, slot of the hash of x's contents on b), key (b << join_log2m)
    // | slot; a partition is the buckets of one key prefix,
    // key >> join_lshift, join_parts of them
    uint32_t *jcnt;             // [parts] entries per partition
    unsigned long long *jreg;   // [parts][join_cap] each partition's entries, scatter order:
                                // fingerprint << 56 | (key & (2^join_lshift - 1)) << 32 | sample
    // entries by partition, then bucket, then fingerprint, then sample index
    uint32_t *jent;             // [blocks * n] the entry's sample
    unsigned long long *jrange; // [blocks * n] first entry of the entry's group (its bucket's
                                // members of its fingerprint) | group size << 32 | block << 48
    uint64_t *jkeys;            // [blocks * n][2] the entry's bit string (entries in a group
                                // of two or more)
    uint32_t *jhit;             // [ceil(blocks * n / 32)] bit b * n + i: entry (b, i) has a
                                // hit and wrote its partial
    unsigned long long *jstat;  // [parts][2] sum of squared group sizes, largest bucket
    unsigned long long *jctl;   // [kJoinCtl] see kJoinCtl*
    int join_log2m;
    int64_t join_n;             // samples of the launch (the partials' row length)
    int join_lshift;
    int join_parts;
    int join_tile;              // samples per tile of the grouping kernels
    int join_tiles;
    int join_cap;               // entries of a partition's region
    int join_force;             // 1: join whenever it can run, 0: when cheaper
};

// Pair-join control words (jctl): the enumeration's probe count, the join's
// ordered candidate pairs (sum of squared group sizes), the largest bucket,
// whether a partition exceeded kJoinPartCap, and the decision (1: the join
// runs); then 64 slots of the probe count.
enum { kJoinCtlProbes = 0, kJoinCtlCost = 1, kJoinCtlMax = 2, kJoinCtlOver = 3,
       kJoinCtlChosen = 4, kJoinCtlProbeSlots = 8, kJoinCtl = 8 + 64 };
// Largest partition the per-partition sorter holds in LDS; a larger one
// leaves the batch to the other strategies.
constexpr int kJoinPartCap = 8192;
// Largest batch the join is planned for: its partitions then have at most
// 2^11 buckets (the sorter's bucket counts in LDS).
constexpr int64_t kJoinMaxSamples = int64_t(1) << 21;

// Whether the pair join was chosen for this launch (device side).
__device__ __forceinline__ bool join_chosen(const DevScratch &sc) {
    return sc.jctl != nullptr && sc.jctl[kJoinCtlChosen] != 0ull;
}

constexpr uint32_t kGoldenMul = 0x9E3779B1u;

// The sample hash is probed a bucket at a time: a key starts at the first
// slot of bucket (h * golden) >> slot_shift and takes the first free slot
// from there on, so the occupied slots of a bucket form a prefix and one
// bucket load decides most lookups.  Keys and sample indices are separate
// arrays: a bucket is 64 bytes of keys (8 one-word or 4 two-word keys), the
// index is read only on a hit.  The table has at least 4 slots per sample.
// A third array holds a 4-byte fingerprint per slot, the key's linear hash
// with bit 0 set (0: free): a lookup whose hash matches no fingerprint of an
// open bucket is a miss without reading keys (the enumeration's candidates,
// nearly all misses, decide this from 32 or 16 bytes).
__host__ __device__ constexpr int bucket_log2(int words) { return words == 1 ? 3 : 2; }
constexpr int kSlotsPerSample = 4;
// A free slot holds all ones in its key's last word: bit 63 of that word is
// qubit 63 (one word, at most 63 qubits) or qubit 127 (two words, at most
// 127 qubits), never set in a sample.
constexpr uint64_t kFreeKey = ~0ull;

// Launch plan of one evaluation: sample tiles x group chunks.
struct EvalLaunch {
    int strategy;       // kStrategyStream or kStrategyEnum
    unsigned enum_blocks;  // persistent blocks of the enumeration kernel
    int64_t n;
    int64_t n_chunks;
    int64_t chunk_len;
    int64_t g_first;
    int threads;        // lookup kernel block size
    int filter_log2;    // filter words = 1 << filter_log2
    size_t lds_bytes;   // dynamic LDS of the lookup kernel
    int eparts_log2;    // enumeration filter: partitions ...
    int efilter_log2;   // ... of this many words (log2)
    int join;           // 1: the pair join is launched (the device decides whether it runs)
    int join_force;     // 1: it runs whenever it can (tuning asked for it)
    int join_log2m;     // log2 of the buckets per block
    // 1: only the join's kernels and the finish (no enumeration or streaming
    // launch); its result is valid only if the device chose the join, which
    // the caller checks (nqs_eloc_energy, after its previous call chose it)
    int join_only;
};

// Bytes of the pair join's scratch for n samples and the table's blocks
// (0 when the table has none).
size_t join_scratch_bytes(const DevTable &tab, int64_t n, int log2m);
// Bucket count per block for n samples: the power of two at or above n.
int join_log2m_for(int64_t n);
// Lay the join scratch out from base (256-byte aligned pieces).
void join_scratch_layout(const DevTable &tab, int64_t n, int log2m, char *base, DevScratch *sc);
// The join's grouping (counts, scatter, sort, then the decision) between
// the clear of its counters and the hash build, and its pair kernel; with
// clear_hash the grouping's first kernel also frees the hash slots and
// clears the Bloom bitmaps.  The grouping also makes the hash build's checks
// of every sample (register range, negative counts, mixed sectors).
hipError_t launch_join_prep(const DevTable &tab, const DevScratch &sc, const uint64_t *samples,
                            const int64_t *weights, int64_t n, int64_t g_eff, bool clear_hash,
                            hipStream_t st);
// With build (1), the same launch also carries the sample-hash build (checks,
// and the insertion when the join is not chosen) in blocks of its own; with
// build 0 none (a launch that only joins: the grouping made the checks).
hipError_t launch_join_pairs(const DevTable &tab, const DevScratch &sc, const uint64_t *samples,
                             const int64_t *weights, int build, const double *log_amp,
                             const double *phase, int64_t n, int precision, int32_t *hit_idx,
                             uint32_t *sign_bits, int64_t sign_words, hipStream_t st);

constexpr int kStrategyAuto = 0, kStrategyStream = 1, kStrategyEnum = 2, kStrategyJoin = 3;

// Optional event recorded between the lookup and the finish kernels.
struct EvalStageEvents {
    hipEvent_t after_lookup;
    hipEvent_t after_pairs;     // after the pair join's pair kernel (when launched)
    hipEvent_t after_grouping;  // after the pair join's grouping (before the hash build)
    hipEvent_t after_finish;    // after the finish kernel (before an energy's combining)
};

// Launch parameters chosen by the autotuner; 0 means the built-in default
// (1024 threads, 16 filter bits per sample, about 4 lookup blocks per CU's
// worth of 1024-thread blocks).
struct Tuning {
    int threads;        // lookup block size: 256, 512 or 1024
    int filter_bits;    // Bloom bits per sample (the bitmap is capped at 128 KB)
    int blocks_per_cu;  // target (tile, chunk) items per CU
    int strategy;       // kStrategyAuto: enumeration when the table allows it
};

EvalLaunch plan_eval(const DevTable &tab, int64_t n, bool dump, const Tuning *tune);
// With join_only (a launch of the join's kernels alone) the sample hash is
// neither cleared nor filled: nothing reads it.
hipError_t launch_hash(const DevTable &tab, const DevScratch &sc, uint32_t capacity,
                       const uint64_t *samples, const int64_t *weights, int64_t n,
                       hipStream_t st, hipEvent_t after_grouping = nullptr,
                       bool join_only = false);
// Eq. 1 taken beside an evaluation: the finish kernel writes one partial set
// (sum w, sum w Re E, sum w Im E, M2 about the block mean) per block to part
// (at least ceil(n / 256) sets), and one block combines them into out[4] =
// {mean re, mean im, variance, sum w}, copies the device's error word to
// *err_out and the join's decision to *chosen_out, then, with seq, publishes
// *seq + 1 (kept in *seq) to *seq_out
// (out, err_out and seq_out may be pinned host memory, which the host polls).
// part == nullptr: not taken.
struct EnergyFused {
    const int64_t *weights;
    double *part;
    double *out;
    int *err_out;
    unsigned *seq;
    unsigned *seq_out;
    unsigned *chosen_out;  // the join's decision (2: no join launched)
};
hipError_t launch_eloc(const DevTable &tab, const DevScratch &sc, const EvalLaunch &L,
                       const uint64_t *samples, const int64_t *weights, const double *log_amp,
                       const double *phase, double *eloc, int precision, int32_t *hit_idx,
                       uint32_t *sign_bits, int64_t sign_words, EvalStageEvents ev,
                       EnergyFused ef, hipStream_t st);
// Eq. 1: per-block partials, then one block combines them; out = {mean re,
// mean im, variance, sum w}.
hipError_t launch_energy(const int64_t *w, const double *e, int64_t n, double *part,
                         double *out, hipStream_t st);
constexpr int kEnergyPartDoubles = 4 * 256;  // (sum w, sum w Re E, sum w Im E, M2) per block
constexpr int kCounters = 8;
// The counters are kept in kCounterSlots copies, one 64-byte line each; a
// block adds to copy (blockIdx.x % kCounterSlots), so the device's atomics
// on them spread over that many lines (thousands of waves adding to one
// address serialise), and a reader sums the copies.
constexpr int kCounterSlots = 64;
__device__ __forceinline__ void count_add(unsigned long long *counters, int k,
                                          unsigned long long v) {
    if (v) atomicAdd(&counters[(blockIdx.x % kCounterSlots) * kCounters + k], v);
}

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
    int strategy;       // kStrategyEnum: enumeration rounds, streaming items only as fallback
    int pad;
};

struct WorkItem {
    int32_t job;
    int32_t chunk;      // -1: enumeration rounds tile, tile + stride, ...
    int32_t tile;
    int32_t stride;
};

constexpr int kEnumVariants = 4;
constexpr int kStreamCounter = kEnumVariants;  // after the enumeration counters
constexpr int kBatchCounters = kStreamCounter + 1;

struct BatchShape {
    int threads;          // lookup block size, shared by all jobs
    int max_filter_log2;  // largest Bloom bitmap (sets the dynamic LDS)
    int64_t max_n;        // largest batch
    int64_t max_clear;    // largest of slot capacity and filter words
    unsigned lookup_blocks;
    unsigned enum_blocks;  // persistent blocks of the enumeration kernels
    // the work list starts with the enumeration items, grouped by variant
    // v = (words - 1) + 2 * integral form: group v is [enum_begin[v], enum_begin[v + 1])
    int enum_begin[5];
};

// d_next: kBatchCounters counters (one per enumeration variant, then the
// streaming items).
// h_jobs: the host copy of the job descriptors (the pair join's per-job
// launches read their tables and scratch from it).
hipError_t launch_batch(const JobDesc *d_jobs, int n_jobs, const WorkItem *d_items, int n_items,
                        unsigned *d_next, const BatchShape &shape, int precision, hipStream_t st,
                        const JobDesc *h_jobs);
size_t batch_lds_bytes(int threads, int max_filter_log2);
// Set the dynamic-LDS limit of the batch kernels (outside any graph capture).
hipError_t prepare_batch_kernels();

}  // namespace nqs
