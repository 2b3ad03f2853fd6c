/*
 * nqs.h - C ABI of the MI355X local-energy library (libnqs.so).
 *
 * The library evaluates the sample-space local energy of a neural-network
 * quantum state for a qubit Hamiltonian given as Pauli strings:
 *
 *   E_loc(x) = sum_{x' in S} <x|H|x'> psi(x') / psi(x)      (Eq. 5)
 *
 * over a batch S of unique occupation-number samples, where psi is known
 * only on S (the psi lookup table of the sample-space energy, Sec. IV-C);
 * an x' outside S contributes nothing.  It also returns the count-weighted
 * energy mean and variance of Eq. 1.
 *
 * Conventions (all entry points):
 *  - Qubit j is bit (j % 64) of word (j / 64); masks and samples are two
 *    uint64 words per item, [n][2], word 0 holding qubits 0..63.  Bits at or
 *    above n_qubits must be zero.  With the molecular ordering of Sec. II-A,
 *    spin orbital (p, alpha) is qubit 2p and (p, beta) is qubit 2p + 1.
 *  - A Pauli term (x, z, c) is c * P with P = i^{popc(x & z)} X^x Z^z, so
 *    every P is Hermitian.  Terms with an odd number of Y factors
 *    (popc(x & z) odd) have purely imaginary matrix elements and cannot
 *    occur in a real molecular Hamiltonian; they are rejected.
 *  - psi(x) = exp(a(x) + i phi(x)): a is ln|psi| (not ln|psi|^2).
 *  - Buffers marked "device" are HIP device pointers on the current device;
 *    "host" buffers are ordinary host memory.  The caller owns every buffer
 *    it passes and must keep device buffers alive until the work enqueued on
 *    hip_stream has completed.  hip_stream is a hipStream_t (NULL = the
 *    default stream).
 *  - Return value: NQS_OK (0) or a negative NQS_E_* code; a description of
 *    the last error on the calling thread is available from
 *    nqs_last_error().  No exception crosses the ABI.  Errors found while
 *    device work runs (duplicate samples, bits out of range, negative
 *    counts) are latched on the handle and returned by the next nqs_sync().
 */
#ifndef NQS_H
#define NQS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    NQS_OK = 0,
    NQS_E_ARG = -1,       /* null pointer, negative size, unknown option, non-finite value */
    NQS_E_RANGE = -2,     /* n_qubits outside [1, 127], or a bit at or above n_qubits set */
    NQS_E_NONREAL = -3,   /* a term with an odd number of Y factors */
    NQS_E_DUPLICATE = -4, /* a sample occurs twice in one batch */
    NQS_E_NOMEM = -5,     /* host or device allocation failed */
    NQS_E_DEVICE = -6,    /* a HIP runtime call failed */
    NQS_E_STATE = -7      /* handle used in a state that does not allow the call */
};

enum {
    NQS_FP64 = 0,        /* every sum and product in FP64 */
    NQS_FP32_KAHAN = 1   /* term sums in FP32 with compensation; FP64 amplitude ratios */
};

typedef struct nqs_ham_s *nqs_ham; /* opaque, owned by the library */

/* Text of the last error reported on the calling thread ("" if none). */
const char *nqs_last_error(void);

/* ABI version of this header (major * 100 + minor). */
int nqs_version(void);

/*
 * Build the resident Pauli table of a Hamiltonian (Eq. 2 mapped to qubits).
 *
 *   x_masks, z_masks : host, [n_terms][2] uint64, the X and Z bits of each term.
 *   coeffs           : host, [n_terms] double, the real coefficients c_t.
 *   spin_masks       : host, [2][2] uint64 {alpha, beta} qubit masks, or NULL.
 *                      When both are non-zero and every sample of a batch has
 *                      the same (N_alpha, N_beta), flips that change either
 *                      count are skipped without a lookup (they cannot land
 *                      in S).  NULL or all-zero switches the filter off.
 *   hip_stream       : stream for the upload.
 *
 * Terms are validated (bits below n_qubits, finite coefficients, even Y
 * count), the phase i^{ny} is folded into the coefficient, equal strings
 * are merged by summing in input order, and the table is grouped by X
 * mask (ascending (X, Z) order; the X = 0 group, if present, is group 0).
 * No threshold is applied.  The host arrays may be freed when this call
 * returns.
 *
 * Errors: NQS_E_ARG (null out or arrays, n_terms < 0, non-finite c,
 * overlapping spin masks, 2^26 or more X groups), NQS_E_RANGE,
 * NQS_E_NONREAL, NQS_E_NOMEM, NQS_E_DEVICE.  On error *out is set to NULL.
 * The call returns after the upload has completed.  A spin mask covering
 * more than 64 qubits leaves the sector filter off.
 */
int nqs_ham_create(nqs_ham *out, int n_qubits, int64_t n_terms, const uint64_t *x_masks,
                   const uint64_t *z_masks, const double *coeffs, const uint64_t *spin_masks,
                   void *hip_stream);

/*
 * Integral form (the paper's own evaluator, Slater-Condon rules of Sec.
 * III-B): a handle whose matrix elements come from h_pq and the chemists'
 * (pq|rs) instead of Pauli terms, for the ONV ordering of Sec. II-A (spin
 * orbital (p, alpha) = qubit 2p, (p, beta) = qubit 2p + 1, n_qubits =
 * 2 n_orbitals <= 126).  The Hamiltonian is
 *   H = sum h_pq a+_{ps} a_{qs} + 1/2 sum (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs},
 * and the table holds the X = 0 group and every spin-conserving single and
 * double flip (the same groups as the Jordan-Wigner table of dense
 * integrals).  (pq|rs) is stored once per 8-fold orbit, so the resident
 * data are O(K^4 / 8) doubles instead of O(K^4) Pauli strings.
 *   h1e: host [K][K] double, symmetric.   eri: host [K][K][K][K] double with
 *   the 8-fold symmetry of real orbitals (checked to 1e-12 of the largest
 *   integral).
 * Evaluates in FP64 only (NQS_E_ARG for NQS_FP32_KAHAN); the debug dump
 * records lookups but no sign bits.  Errors: NQS_E_ARG, NQS_E_RANGE,
 * NQS_E_NOMEM, NQS_E_DEVICE.
 */
int nqs_ham_create_integrals(nqs_ham *out, int n_orbitals, const double *h1e, const double *eri,
                             void *hip_stream);

/* Group count G, merged term count T and device bytes held by the handle
 * (table plus scratch). */
int nqs_ham_info(nqs_ham h, int64_t *n_groups, int64_t *n_terms, int64_t *device_bytes);

/* Release the handle, its device table and its scratch.  Waits for the
 * handle's outstanding work first.  NULL is accepted. */
int nqs_ham_destroy(nqs_ham h);

/*
 * Host-only form of the table builder used by nqs_ham_create (no device
 * needed).  Call once with all output pointers NULL to obtain *n_groups and
 * *n_merged, then again with buffers of those sizes:
 *   group_x  [n_groups][2] uint64   X mask of each group
 *   group_off[n_groups + 1] int64   term range of each group
 *   term_z   [n_merged][2] uint64   Z mask of each merged term
 *   term_c   [n_merged] double      folded coefficient c * (-1)^{ny/2}
 * Same validation and errors as nqs_ham_create.
 */
int nqs_table_host(int n_qubits, int64_t n_terms, const uint64_t *x_masks,
                   const uint64_t *z_masks, const double *coeffs, int64_t *n_groups,
                   int64_t *n_merged, uint64_t *group_x, int64_t *group_off, uint64_t *term_z,
                   double *term_c);

/*
 * Host-only form of the occupation-form diagonal that the finish kernel
 * evaluates on the matrix cores (no device needed).  For a table whose X = 0
 * group has only Z strings of at most two qubits, Z_i = 1 - 2 n_i turns the
 * group into d0 + sum_{i <= j} n_i n_j U[j][i]; the U are stored as fixed
 * point (U 2^S rounded, S the largest integer keeping every |U| 2^S below
 * 2^59) in four base-2^15 digits, least significant first (the lower three
 * balanced in [-2^14, 2^14), the top one in [-2^14, 2^14]), each digit E as
 * two int8 byte planes a, b with E = a - 128 b, as 16 x 16 x 64 int8 MFMA
 * operand tiles: for column tile jt (j in [16 jt, 16 jt + 16),
 * ceil(n_qubits / 16) of them) its k-blocks kb of 64 rows i (one for jt < 4,
 * two after), then per digit its planes a and b, each 64 lanes x 16 bytes,
 * lane L byte b holding the plane's byte for U[16 jt + L % 16][64 kb + 16 (L / 16)
 * + b] (zero where i > j or outside the register).  Call with tiles NULL to
 * obtain *n_bytes (0: the table has no such form), then with a buffer of
 * that size.  *d0 receives d0 and *scale 2^-S.  Same arguments, validation
 * and errors as nqs_ham_create.
 */
int nqs_diag_tiles_host(int n_qubits, int64_t n_terms, const uint64_t *x_masks,
                        const uint64_t *z_masks, const double *coeffs,
                        const uint64_t *spin_masks, int64_t *n_bytes, int8_t *tiles,
                        double *d0, double *scale);

/*
 * Local energies of one batch (Eq. 5 over S, Alg. 3's per-sample outer loop).
 *
 *   samples : device, [n][2] uint64, unique bit strings, bits >= n_qubits zero.
 *   weights : device, [n] int64 counts >= 0, or NULL.  Counts do not change
 *             E_loc; when given they are checked for negatives.
 *   log_amp : device, [n] double, a(x) = ln|psi(x)|.
 *   phase   : device, [n] double, phi(x).
 *   eloc    : device, [n][2] double (re, im) output, caller-owned.
 *   precision: NQS_FP64 or NQS_FP32_KAHAN.
 *
 * Asynchronous on hip_stream (no host synchronisation).  The handle's
 * scratch (sample hash, partial sums) is reused; a handle may be used from
 * one stream at a time.  n = 0 is a no-op.  A call whose arguments (n,
 * pointers, precision) repeat the previous call's, with the same launch plan
 * and profiling off, is issued as one replay of a HIP graph captured on the
 * second such call (the buffers' contents are read at run time, as for an
 * eager call); the environment variable NQS_EVAL_GRAPHS=0, read when a
 * handle is created, keeps every call eager.  Errors: NQS_E_ARG, NQS_E_STATE
 * (bad handle), NQS_E_NOMEM, NQS_E_DEVICE synchronously; NQS_E_DUPLICATE and
 * NQS_E_RANGE (sample bits, negative counts) from the next nqs_sync().
 */
int nqs_eloc_eval(nqs_ham h, int64_t n, const uint64_t *samples, const int64_t *weights,
                  const double *log_amp, const double *phase, double *eloc, int precision,
                  void *hip_stream);

/*
 * nqs_eloc_eval for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results as nqs_eloc_eval (bit for bit, same launch
 * plan), but the evaluation scratch comes from one array of
 * NQS_NOALLOC_SCRATCH_BYTES held by the library on every device it runs on
 * for the life of the process, and the call makes no allocation of any kind
 * (it also never captures or replays a graph).
 *
 * The array is shared by every call on a device and keeps the last call's
 * contents; whatever must start cleared is cleared on the stream by the
 * call's own kernels.  Two calls that overlap on one device (different
 * streams, threads or handles) race on it and give undefined results: the
 * caller serialises them.  The scratch needed grows with n (at 100 qubits
 * and 262,144 samples about 160 MB, the pair join's partition regions and
 * entries included): a batch that needs more than the array holds returns
 * NQS_E_ARG before anything is launched.  Arguments, other
 * errors and asynchrony as nqs_eloc_eval; NQS_E_STATE also when the
 * handle's device is not the current one.
 */
#define NQS_NOALLOC_SCRATCH_BYTES (192ull << 20)
int nqs_eloc_eval_noalloc(nqs_ham h, int64_t n, const uint64_t *samples, const int64_t *weights,
                          const double *log_amp, const double *phase, double *eloc, int precision,
                          void *hip_stream);

/*
 * Count-weighted energy of Eq. 1 over unique samples:
 *   out[0] = Re E, out[1] = Im E with E = sum w E_loc / sum w,
 *   out[2] = sum w |E_loc - E|^2 / sum w (population variance),
 *   out[3] = sum w.
 * Two launches: each of up to 256 blocks sums a fixed strided set of
 * samples and their deviations about its own mean; one block combines them
 * in block order (per block, M2_b + W_b |mean_b - E|^2).
 * weights: device [n] int64; eloc: device [n][2] double; out: host [4].
 * The reduction order is fixed, so repeated calls give identical bits.
 * Calls are serialised per device (one scratch per device).
 * Synchronises hip_stream before returning.  Errors: NQS_E_ARG (n <= 0,
 * null pointers, sum w == 0), NQS_E_NOMEM, NQS_E_DEVICE.
 */
int nqs_energy(int64_t n, const int64_t *weights, const double *eloc, double out[4],
               void *hip_stream);

/*
 * One VMC step's evaluation: nqs_eloc_eval followed by Eq. 1 (§II-A) over
 * its result, in one launch sequence (replayed as one graph when the same
 * arguments repeat).  The finish kernel also writes each block's weighted
 * sums and its deviations about the block's own mean; one block combines
 * them in block order (M2_b + W_b |mean_b - E|^2 per block), so out[] is
 * the same quantity as nqs_energy's, summed in another fixed order (equal
 * to it within rounding; repeated calls give identical bits).
 *   eloc: device [n][2] double, written as by nqs_eloc_eval;
 *   out:  host [4] = {Re E, Im E, variance, sum w}, as nqs_energy.
 * weights are required (device [n] int64).  Returns once the result is on
 * the host: the last kernel writes it, with the device's error word and a
 * new sequence number, to a pinned buffer of the handle that this call
 * polls (all reads of the caller's arrays are done by then; later work on
 * hip_stream still runs after this call's kernels).  Reports the errors the
 * device latched during this call (NQS_E_DUPLICATE, NQS_E_RANGE) as
 * nqs_sync would.  Calls on one handle must not overlap.  Errors: those of
 * nqs_eloc_eval and nqs_energy (NQS_E_ARG for n <= 0, null weights or out,
 * sum w == 0).
 */
int nqs_eloc_energy(nqs_ham h, int64_t n, const uint64_t *samples, const int64_t *weights,
                    const double *log_amp, const double *phase, double *eloc, int precision,
                    double out[4], void *hip_stream);

/* Wait for hip_stream and return the first error latched by device work of
 * this handle since the previous nqs_sync (then clear it). */
int nqs_sync(nqs_ham h, void *hip_stream);

/*
 * Counters of the last nqs_eloc_eval on this handle (valid after nqs_sync):
 *   out[0] pairs      = n * G (sample, group) pair-evaluations
 *   out[1] probes     = pairs that passed the sector test (lookups of x')
 *   out[2] hits       = lookups that found x' in S (off-diagonal)
 *   out[3] terms      = Pauli terms evaluated (diagonal group plus hit groups)
 *   out[4] candidates = lookups that passed the on-chip filter and went to
 *                       the hash table in device memory (with the pair
 *                       join: the ordered pairs of samples sharing a group)
 *   out[5] rounds     = sample rounds run by the flip enumeration (0 when
 *                       the group-streaming kernel did the lookups)
 * With the enumeration, probes counts every spin-conserving single and
 * double flip of each sample, which equals the streaming count when the
 * table holds a group for each of them.
 */
int nqs_eval_stats(nqs_ham h, int64_t out[6]);

/*
 * Launch plan of the last nqs_eloc_eval (or nqs_eloc_eval_noalloc) on this
 * handle; out[0..6] are host-side and valid as soon as the call has
 * returned, out[7] after nqs_sync:
 *   out[0] strategy planned besides the pair join: NQS_STRATEGY_STREAM or
 *          NQS_STRATEGY_ENUM
 *   out[1] filter partitions (sample classes) of the enumeration filter:
 *          1, 2, 4 or 8 (0 when streaming is planned)
 *   out[2] 32-bit words per enumeration filter partition
 *   out[3] group chunks of the streaming kernel (0: no streaming launch)
 *   out[4] samples of the batch
 *   out[5] 32-bit words of the streaming kernel's Bloom bitmap
 *   out[6] qubit blocks of the pair join, 0 when no join was launched
 *   out[7] whether the device ran the pair join: 1, 0, or -1 (not launched)
 * Which of the others ran is in nqs_eval_stats (rounds > 0: enumeration).
 * Errors: NQS_E_STATE (bad handle, nothing evaluated yet), NQS_E_ARG,
 * NQS_E_DEVICE.
 */
int nqs_eval_plan(nqs_ham h, int64_t out[8]);

/*
 * Test hook: the k-th device allocation of evaluation scratch from now on
 * (block areas, filter partitions, sample hash, sample hashes, partial sums,
 * in that order within one growth) fails once as if the device were out of
 * memory, so the error path can be exercised: that evaluation returns
 * NQS_E_NOMEM and the handle stays usable (a later call allocates again).
 * k = 0 switches the hook off.  Process-wide.  Errors: NQS_E_ARG (k < 0).
 */
int nqs_debug_fail_allocs(int k);

/*
 * Kernel timing.  nqs_profile(h, 1) makes every later nqs_eloc_eval on h
 * record HIP events on its stream around each kernel stage; after the
 * stream has completed, nqs_last_kernel_ms(h, out) returns the durations in
 * milliseconds of the last evaluation:
 *   out[0] sample-hash build (clear + insert)
 *   out[1] E_loc lookup kernel (all non-diagonal groups)
 *   out[2] E_loc finish kernel (diagonal group + partial sums)
 * Errors: NQS_E_STATE (bad handle, profiling off, nothing recorded yet),
 * NQS_E_DEVICE.
 */
int nqs_profile(nqs_ham h, int enable);
int nqs_last_kernel_ms(nqs_ham h, float out[3]);

/*
 * Finer durations of the last profiled evaluation, in milliseconds, from
 * the same events plus two more (stages that did not run take ~0):
 *   out[0] clear and the pair join's grouping (bucket keys, fingerprints
 *          and the sample checks and, in the same launch, the hash clear;
 *          partition counts, placing, per-partition sort, the device's
 *          decision)
 *   out[1] sample-hash build (~0 when the join is launched: the build then
 *          runs inside the pair kernel's launch)
 *   out[2] the pair join's pair kernel (with the hash build, except in a
 *          launch that only joins)
 *   out[3] enumeration / streaming lookup kernels (return at once when the
 *          join runs)
 *   out[4] finish kernel (diagonal + partial sums)
 *   out[5] all of the evaluation
 * Errors as nqs_last_kernel_ms.
 */
int nqs_last_stage_ms(nqs_ham h, float out[6]);

/*
 * Test hook: nqs_eloc_eval with the lookup results recorded (same kernels,
 * extra stores switched on).
 *   hit_idx  : device [n][G] int32 or NULL.  For group g of sample i: the
 *              index j of x' = x_i ^ X_g in S, or -1 when x' is not in S or
 *              the group failed the sector test; the X = 0 group records i.
 *   sign_bits: device [n][(T + 31) / 32] uint32 or NULL, zero-filled by the
 *              caller.  Bit (t % 32) of word (t / 32) is popc(Z_t & x_i) & 1
 *              for every term t the kernel evaluated for sample i (X = 0
 *              group and hit groups); other bits stay zero.
 * Other arguments and errors as nqs_eloc_eval (FP64 only).
 */
int nqs_debug_dump(nqs_ham h, int64_t n, const uint64_t *samples, const double *log_amp,
                   const double *phase, double *eloc, int32_t *hit_idx, uint32_t *sign_bits,
                   void *hip_stream);


/* ------------------------------------------------------------------ tuning
 *
 * Launch parameters of the lookup stage.  Zero fields take the built-in
 * default.  They change speed only: results do not depend on threads or
 * filter_bits, while blocks_per_cu (group-chunk boundaries) and strategy
 * (the order in which a sample's hits are summed) reorder FP sums within
 * rounding.
 *
 * Strategies (Eq. 5 evaluated two ways, same hits and matrix elements):
 *   NQS_STRATEGY_STREAM: every X group passes every sample (exact sector
 *     test, Bloom filter, hash probe); works for any table.
 *   NQS_STRATEGY_ENUM: each sample's spin-conserving single and double
 *     flips are enumerated from its occupied and virtual orbitals, and only
 *     those are probed.  Needs spin masks covering every qubit and no group
 *     flipping more than four qubits; a batch whose samples span several
 *     sectors (or whose occupation does not fit the on-chip round) runs the
 *     streaming kernel instead, decided on the device.
 *   NQS_STRATEGY_JOIN: the pair join.  Every group of the table flips at
 *     most m qubits (m = 4 for molecular tables), so two samples a term
 *     connects agree on at least one of m + 1 disjoint qubit blocks; the
 *     samples are grouped by the contents of each block (a hash bucket,
 *     split by a content fingerprint), and only pairs of samples sharing a
 *     group are tested (Hamming distance, then the group index).  Its cost
 *     is the sum of squared group sizes, independent of the table's size:
 *     for samples spread over a large sector it is far below both others.  Needs m + 1 <= 8, at most 2^21 samples, and at
 *     most 8192 entries in one partition of 2^11 buckets (a hash range of
 *     the bucket keys; about two thousand entries each on average);
 *     otherwise (decided on the device) the enumeration or streaming
 *     strategy runs instead.
 *   NQS_STRATEGY_AUTO (0): the pair join is launched beside the enumeration
 *     (where the table allows it) or streaming, and the device runs the
 *     join when its counted cost (sum of squared group sizes plus a term
 *     per entry) is below the other strategy's (the
 *     enumeration's lookups, or half the sample-group pairs of streaming).
 *     Batches (nqs_batch_*) make the same decision per job: a job's
 *     grouping and pair kernels are launched around the persistent
 *     kernels, which skip the job when its device chose the join.  Served
 *     requests are planned as single evaluations are, the join included.
 */
enum { NQS_STRATEGY_AUTO = 0, NQS_STRATEGY_STREAM = 1, NQS_STRATEGY_ENUM = 2,
       NQS_STRATEGY_JOIN = 3 };

typedef struct {
    int32_t threads;       /* streaming block size: 256, 512 or 1024 (default 1024) */
    int32_t filter_bits;   /* on-chip filter bits per sample, 4..64 (default 16; the
                              bitmap is capped at 128 KB) */
    int32_t blocks_per_cu; /* streaming work items per compute unit, 1..64 (default 4) */
    int32_t strategy;      /* NQS_STRATEGY_* (default AUTO) */
} nqs_tuning;

/* Set (t != NULL) or clear (t == NULL) the handle's tuning.  NQS_E_ARG on a
 * value out of range. */
int nqs_set_tuning(nqs_ham h, const nqs_tuning *t);
/* The tuning the handle uses (defaults filled in). */
int nqs_get_tuning(nqs_ham h, nqs_tuning *out);

/*
 * Autotuner.  Times candidate tunings (streaming: threads x filter bits x
 * blocks per CU; enumeration, where allowed: filter bits) with HIP events on
 * hip_stream, evaluating this batch (arguments as
 * nqs_eloc_eval; eloc receives the last result), and keeps the fastest.  The
 * choice is cached per shape class (mask words, sector-test form, whether
 * enumeration applies, log2 of the batch size and of the group count,
 * precision) in a JSON file at
 * cache_path (NULL: no cache); a cached class is applied without timing.
 * The chosen tuning is set on the handle and returned in *best, with its
 * time in *best_ms (-1 when it came from the cache).  Synchronises the
 * stream.  Errors: as nqs_eloc_eval, plus NQS_E_STATE when the cache file
 * cannot be written.
 */
int nqs_autotune(nqs_ham h, int64_t n, const uint64_t *samples, const double *log_amp,
                 const double *phase, double *eloc, int precision, const char *cache_path,
                 nqs_tuning *best, double *best_ms, void *hip_stream);

/* ------------------------------------------------------------------ batched form
 *
 * Many Hamiltonians, each with its own uneven batch, in one pass: per-job
 * hash builds run as one (tile, job) grid, and all lookup work is one list
 * of (job, sample tile, group chunk) items drained by a single persistent
 * kernel (blocks take items from an atomic counter until the list is
 * empty); enumeration jobs add items of sample rounds.  Results equal those
 * of nqs_eloc_eval with the same tunings; a batch planned with threads other
 * than 1024 runs every job with the streaming strategy.  Integral-form jobs
 * (nqs_ham_create_integrals) evaluate in FP64 whatever the batch precision.
 */
typedef struct {
    nqs_ham ham;              /* distinct handles within one batch */
    int64_t n;                /* samples of this job (0 allowed) */
    const uint64_t *samples;  /* device [n][2] */
    const int64_t *weights;   /* device [n] or NULL */
    const double *log_amp;    /* device [n] */
    const double *phase;      /* device [n] */
    double *eloc;             /* device [n][2] output */
} nqs_batch_item;

typedef struct nqs_batch_s *nqs_batch; /* opaque, owned by the library */

/*
 * Plan a batch: grows each handle's scratch, builds and uploads the job
 * descriptors and the work list (synchronously, on hip_stream).  The buffer
 * pointers are recorded: later launches read whatever the buffers hold then.
 * threads: lookup block size for the whole batch (0 = default).  Each job
 * uses its handle's tuning for the filter size and chunking.  The handles
 * must outlive the batch and must not be used elsewhere while it runs.
 * Errors: NQS_E_ARG (no items, a repeated or invalid handle, bad sizes or
 * pointers), NQS_E_NOMEM, NQS_E_DEVICE.
 */
int nqs_batch_create(nqs_batch *out, int n_items, const nqs_batch_item *items, int precision,
                     int threads, void *hip_stream);
/* Enqueue one evaluation of the whole batch (asynchronous; no allocation). */
int nqs_batch_launch(nqs_batch b, void *hip_stream);
/* Capture one evaluation into a HIP graph held by the batch.  hip_stream
 * must not be the default (NULL) stream. */
int nqs_batch_capture(nqs_batch b, void *hip_stream);
/* Launch the captured graph (NQS_E_STATE if nothing was captured). */
int nqs_batch_replay(nqs_batch b, void *hip_stream);
/* Release the batch (waits for the device first).  NULL is accepted. */
int nqs_batch_destroy(nqs_batch b);

/* ------------------------------------------------------------------ serving
 *
 * A request loop with continuous batching.  Hamiltonians are registered
 * once (their tables stay resident).  The device is divided into lanes
 * (streams, 1..8): each lane owns evaluation scratch (sample hash, partial
 * sums, filters, pair-join buckets) sized for the largest request any
 * registered handle will send, plus its own counters and error latch, all
 * allocated at registration.  nqs_server_submit enqueues an E_loc request
 * (nqs_batch_item: handle, batch, amplitudes, output) and returns at once.
 * A dispatcher thread admits pending requests in arrival order into free
 * lanes, as long as the resident data plus the footprint of every request
 * on the device stays within hbm_budget_bytes, and launches each on its
 * lane with the plan nqs_eloc_eval would take (the device picks the pair
 * join, the enumeration or streaming).  Lanes run concurrently, so requests
 * that arrive while others run join the device's work as lanes free up,
 * whatever handle they use (two requests for one handle overlap on two
 * lanes); each request completes on its own lane event.  A request's result
 * is the same as its nqs_eloc_eval result, bit for bit (same kernels, same
 * plan).
 *
 * Footprint of a request: 56 bytes per sample (samples, log_amp, phase,
 * counts, output).  Resident: the tables and the lanes' scratch.  Requests
 * whose footprint plus the resident data exceed the budget are rejected at
 * submission (NQS_E_NOMEM).  Device-detected errors of a request
 * (duplicates, bits out of range) are latched on its handle and returned by
 * the next nqs_sync on that handle; the server goes on serving.
 */
typedef struct {
    int64_t hbm_budget_bytes; /* admission budget (> 0) */
    int32_t streams;          /* lanes: requests on the device at once, 1..8 (0 = 4) */
    int32_t precision;        /* NQS_FP64 or NQS_FP32_KAHAN */
} nqs_server_config;

typedef struct nqs_server_s *nqs_server; /* opaque, owned by the library */

/* Start a server (and its dispatcher thread) on the current device. */
int nqs_server_create(nqs_server *out, const nqs_server_config *cfg);
/* Register a handle: its table counts as resident, and every lane's scratch
 * is grown (when no request runs) to hold a request of max_samples for it.
 * NQS_E_NOMEM if the resident total would exceed the budget or the lanes'
 * scratch cannot be allocated; NQS_E_STATE if the lanes must grow while
 * requests run. */
int nqs_server_add_ham(nqs_server s, nqs_ham h, int64_t max_samples);
/* Enqueue a request (thread-safe).  *ticket identifies it in nqs_server_poll.
 * Errors: NQS_E_ARG (unregistered handle, more samples than its registered
 * max_samples, bad item), NQS_E_NOMEM (can never fit the budget),
 * NQS_E_STATE (server stopping or failed). */
int nqs_server_submit(nqs_server s, const nqs_batch_item *req, int64_t *ticket);
/* Move up to capacity finished requests out: their tickets and their
 * latencies in microseconds (submission to completion on its lane);
 * *n_out receives the count.  Returns the dispatcher's error, if any. */
int nqs_server_poll(nqs_server s, int64_t *tickets, double *latency_us, int capacity,
                    int *n_out);
/* Wait until every submitted request has finished, or timeout_s elapses
 * (NQS_E_STATE). */
int nqs_server_drain(nqs_server s, double timeout_s);
/* out[0] submitted, [1] completed, [2] rejected, [3] launches (one per
 * request), [4] most requests in flight at once, [5] the same (lanes busy at
 * once), [6] peak admitted bytes (resident + in flight), [7] resident bytes
 * (tables and lane scratch). */
int nqs_server_stats(nqs_server s, int64_t out[8]);
/* Finish outstanding requests, stop the dispatcher and release everything.
 * NULL is accepted. */
int nqs_server_destroy(nqs_server s);

#ifdef __cplusplus
}
#endif

#endif /* NQS_H */
