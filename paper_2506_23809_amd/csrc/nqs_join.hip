// Pair join: the local energy summed over pairs of samples (Eq. 5 with the
// kets taken from S, the loop structure of Alg. 3), for batches whose
// samples have few partners.
//
// Every group of the table flips at most max_flip qubits, so two samples
// that a term connects differ in at most max_flip bits.  With the qubits
// split into B = max_flip + 1 disjoint blocks, such a pair agrees on at
// least one block (pigeonhole).  Grouping the samples by the contents of
// each block (B buckets per sample, addressed by a hash of the contents)
// therefore puts every connected pair into a common bucket; a pair is taken
// in the first block on which it agrees, so it is counted once.  Inside a
// bucket every ordered pair (x, x') is tested: Hamming distance, first
// agreeing block, then the group index says whether a group with
// X = x ^ x' exists, and a hit adds <x|H|x'> psi(x')/psi(x) with the same
// sums as the other strategies.
//
// Grouping without global atomics per entry: the bucket keys are split into
// partitions by their high bits (about a thousand entries each).  A tile of
// samples counts its entries per partition in LDS and reserves its share
// of each partition with one atomic; the entries are then placed, each
// partition is sorted in LDS by (bucket, content fingerprint, sample), and
// the start and size of each entry's group (its bucket's members with its
// fingerprint: hash-colliding contents mostly fall apart) are written beside
// the entries.  The pair kernel then takes one lane per entry.
//
// Cost: the ordered pairs inside groups, the sum of squared group sizes.
// For samples spread over a large sector this is far below the
// enumeration's N x (connected states per sample) lookups.  The decision is
// taken on the device from the group sizes, between the hash clear and the
// hash build: when the join is cheaper it runs, and the hash build's
// insertion, the enumeration and the streaming kernels of the same launch
// stand down; otherwise those run and the pair kernel returns at once.
//
// Determinism: a partition is sorted by sample index within each group, so
// each sample's hits are added in a fixed order (one partial per block,
// partners in index order), and the finish kernel adds the block partials
// in block order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/nqs.h"
#include "nqs_dev_common.hpp"
#include "nqs_device.hpp"

namespace nqs {

namespace {

constexpr int kJoinGroupThreads = 1024;  // tile kernels
constexpr int kJoinPairThreads = 256;
constexpr int kJoinPairPer = 4;  // entries per lane of the pair kernel, at most
constexpr int kJoinSortThreads = 512;
// Largest bucket ranked by a pass over its members; a partition with a
// larger one is bitonic-sorted whole.
constexpr unsigned long long kJoinRankMax = 64;
constexpr int kJoinMaxParts = 8192;      // partitions of any planned launch
constexpr int kJoinMaxLocal = 2048;      // buckets per partition (2^join_lshift)
constexpr int kJoinTiles = 128;          // tiles of the grouping kernels, at most
constexpr int kScatterStash = 10240;     // bucket keys a scatter tile keeps in LDS
constexpr int kJoinFpShift = 56;         // fingerprint byte of a partition-region entry

inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// The 64-bit multiply-xorshift mix of block b's masked words (any hash
// serves: only equal contents must meet).
template <int W>
__device__ __forceinline__ uint64_t join_mix(const DevTable &tab, const Key<W> &x, int b) {
    uint64_t z = x.w[0] & tab.jmask[b][0];
    if constexpr (W == 2) z ^= (x.w[W - 1] & tab.jmask[b][1]) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The bucket key of block b of x (below 2^24: at most 8 blocks, 2^21
// buckets each) and, in the top byte, the content fingerprint: the mix's
// low byte, which the bucket does not use.  Equal contents have equal
// fingerprints, so a bucket splits into groups of equal fingerprint without
// separating any pair that agrees on the block.
template <int W>
__device__ __forceinline__ uint32_t join_key_fp(const DevTable &tab, const Key<W> &x, int b,
                                                int log2m) {
    const uint64_t z = join_mix<W>(tab, x, b);
    const uint32_t slot = static_cast<uint32_t>(z >> (64 - log2m));
    return ((static_cast<uint32_t>(b) << log2m) | slot) | (static_cast<uint32_t>(z) << 24);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ unsigned long long wave_max(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

// Inclusive prefix sum over the lanes of a wave.
__device__ __forceinline__ unsigned long long wave_scan(unsigned long long v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long o = __shfl_up(v, off);
        if (lane >= off) v += o;
    }
    return v;
}

// Exclusive prefix sum of v over the block (blockDim.x a multiple of 64, at
// most 1024 threads); *total receives the block's sum.  Synchronises.
__device__ __forceinline__ unsigned long long block_exclusive_scan(unsigned long long v,
                                                                  unsigned long long *total) {
    __shared__ unsigned long long wsum[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const unsigned long long inc = wave_scan(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    unsigned long long before = 0, all = 0;
    for (int w = 0; w < waves; ++w) {
        const unsigned long long s = wsum[w];
        if (w < wave) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// Sum and maximum over the block (blockDim.x a multiple of 64, at most
// 1024 threads), valid in thread 0.  Synchronises.
__device__ __forceinline__ void block_sum_max(unsigned long long &s, unsigned long long &m) {
    __shared__ unsigned long long red[2][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    s = wave_sum(s);
    m = wave_max(m);
    if (lane == 0) {
        red[0][wave] = s;
        red[1][wave] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long S = 0, M = 0;
        for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) {
            S += red[0][w];
            M = red[1][w] > M ? red[1][w] : M;
        }
        s = S;
        m = M;
    }
    __syncthreads();
}

// ---- kernels

// One block per tile of samples: the bucket key of every (block, sample),
// the tile's entries per partition (LDS), its range in each partition it
// touches (one global atomic per partition: the partition's count so far),
// then each entry written at its place in its partition's region (regions
// of join_cap entries, in partition order; a partition that outgrows its
// region keeps counting but writes nothing, and the join then stands down).
// Also whether the batch spans several (N_alpha, N_beta) sectors and the
// enumeration's lookups for it (its spin-conserving singles and doubles),
// summed for the decision.
template <int W>
__global__ __launch_bounds__(kJoinGroupThreads) void join_scatter_kernel(
    DevTable tab, DevScratch sc, const uint64_t *__restrict__ samples,
    const int64_t *__restrict__ weights, int64_t n) {
    __shared__ uint32_t cur[kJoinMaxParts];
    // the tile's first bucket keys and fingerprints, kept for the placing
    // pass (sample s of the tile, block b: stash[s * join_blocks + b]; keys
    // beyond it are computed again)
    __shared__ uint32_t stash[kScatterStash];
    if (blockIdx.x >= static_cast<unsigned>(sc.join_tiles)) {
        // blocks beyond the tiles free the hash slots and clear the Bloom
        // bitmaps that the hash build of this launch may fill
        const uint32_t cap = sc.slot_mask + 1u;
        const uint32_t fw = 1u << sc.filter_log2;
        const uint32_t efw = sc.eparts_log2 > 0 ? 1u << (sc.eparts_log2 + sc.efilter_log2) : 0u;
        uint32_t span = cap > fw ? cap : fw;
        span = span > efw ? span : efw;
        const uint32_t stride = (gridDim.x - static_cast<unsigned>(sc.join_tiles)) * blockDim.x;
        for (uint32_t s = (blockIdx.x - static_cast<unsigned>(sc.join_tiles)) * blockDim.x +
                          threadIdx.x;
             s < span; s += stride) {
            if (s < cap) {
                sc.sidx[s] = -1;
                sc.sfp[s] = 0u;
                sc.skey[static_cast<size_t>(s) * W + W - 1] = kFreeKey;
            }
            if (s < fw) sc.filter[s] = 0u;
            if (s < efw) sc.efilter[s] = 0u;
        }
        return;
    }
    const int parts = sc.join_parts, lshift = sc.join_lshift, log2m = sc.join_log2m;
    for (int p = threadIdx.x; p < parts; p += blockDim.x) cur[p] = 0u;
    __syncthreads();
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * sc.join_tile;
    const int64_t t1 = t0 + sc.join_tile < n ? t0 + sc.join_tile : n;
    unsigned long long probes = 0;
    const int nq = tab.n_qubits;
    const int nb = tab.join_blocks;
    for (int64_t i = t0 + threadIdx.x; i < t1; i += blockDim.x) {
        const Key<W> x = load_key<W>(samples, i);
        const int64_t at = (i - t0) * nb;
        for (int b = 0; b < nb; ++b) {
            const uint32_t v = join_key_fp<W>(tab, x, b, log2m);
            atomicAdd(&cur[(v & 0xFFFFFFu) >> lshift], 1u);
            if (at + b < kScatterStash) stash[at + b] = v;
        }
        // the checks of the sample-hash build (a launch that only joins has
        // no build): bits beyond the register, negative counts
        const uint64_t hw = samples[2 * i + 1];
        const bool bad = nq >= 64 ? (nq < 128 && (hw >> (nq - 64)) != 0)
                                  : ((x.w[0] >> nq) != 0 || hw != 0);
        if (bad || (weights && weights[i] < 0)) latch(sc.err, NQS_E_RANGE);
        if (tab.sector_filter) {
            const uint64_t w0 = x.w[0], w1 = W == 2 ? x.w[W - 1] : 0ull;
            const uint64_t s0 = samples[0], s1 = samples[1];
            const int na = __popcll(w0 & tab.spin_a0) + __popcll(w1 & tab.spin_a1);
            const int nbe = __popcll(w0 & tab.spin_b0) + __popcll(w1 & tab.spin_b1);
            const int ra = __popcll(s0 & tab.spin_a0) + __popcll(s1 & tab.spin_a1);
            const int rb = __popcll(s0 & tab.spin_b0) + __popcll(s1 & tab.spin_b1);
            if (na != ra || nbe != rb) atomicOr(sc.mixed, 1);
            if (tab.enum_ok) {
                const unsigned long long va = tab.k_alpha - na, vb = tab.k_beta - nbe;
                const unsigned long long a = na, bb = nbe;
                probes += a * va + bb * vb + (a * (a - 1) / 2) * (va * (va - 1) / 2) +
                          (bb * (bb - 1) / 2) * (vb * (vb - 1) / 2) + a * va * bb * vb;
            }
        }
    }
    __syncthreads();
    // the tile's first place in each partition it touches
    for (int p = threadIdx.x; p < parts; p += blockDim.x) {
        const uint32_t c = cur[p];
        if (c) cur[p] = atomicAdd(&sc.jcnt[p], c);
    }
    probes = wave_sum(probes);
    if ((threadIdx.x & 63) == 0 && probes)
        atomicAdd(&sc.jctl[kJoinCtlProbeSlots + (blockIdx.x * 16 + (threadIdx.x >> 6)) % 64],
                  probes);
    __syncthreads();
    // the entries (keys from the stash, or computed again past it)
    const uint32_t lmask = (1u << lshift) - 1u;
    const uint32_t cap = static_cast<uint32_t>(sc.join_cap);
    for (int64_t i = t0 + threadIdx.x; i < t1; i += blockDim.x) {
        const int64_t at = (i - t0) * nb;
        Key<W> x;
        if (at + nb > kScatterStash) x = load_key<W>(samples, i);
        for (int b = 0; b < nb; ++b) {
            const uint32_t v =
                at + b < kScatterStash ? stash[at + b] : join_key_fp<W>(tab, x, b, log2m);
            const uint32_t k = v & 0xFFFFFFu;
            const uint32_t part = k >> lshift;
            const uint32_t pos = atomicAdd(&cur[part], 1u);
            if (pos < cap)
                sc.jreg[static_cast<int64_t>(part) * cap + pos] =
                    (static_cast<unsigned long long>(v >> 24) << kJoinFpShift) |
                    (static_cast<unsigned long long>(k & lmask) << 32) |
                    static_cast<unsigned long long>(i);
        }
    }
}

// One partition (c entries, at most kJoinPartCap) ordered by (bucket,
// content fingerprint, sample); thread 0 writes its statistics.
template <int W>
__device__ __forceinline__ void join_sort_partition(const DevTable &tab, const DevScratch &sc,
                                                    const uint64_t *__restrict__ samples, int p,
                                                    uint32_t c, uint32_t s0) {
    __shared__ uint32_t buf[kJoinPartCap];
    __shared__ uint32_t cnt[kJoinMaxLocal];
    // each placed entry's content fingerprint (from the scatter)
    __shared__ uint8_t fpr[kJoinPartCap];
    // the partition's entries, in its region (scatter order)
    const unsigned long long *__restrict__ reg =
        sc.jreg + static_cast<int64_t>(p) * static_cast<uint32_t>(sc.join_cap);
    const int L = 1 << sc.join_lshift;
    const uint32_t lmask = static_cast<uint32_t>(L - 1);
    for (int u = threadIdx.x; u < L; u += blockDim.x) cnt[u] = 0u;
    __syncthreads();
    for (uint32_t u = threadIdx.x; u < c; u += blockDim.x)
        atomicAdd(&cnt[static_cast<uint32_t>(reg[u] >> 32) & lmask], 1u);
    __syncthreads();
    // bucket starts (exclusive scan of the counts), packed with the sizes
    const int per = (L + blockDim.x - 1) / blockDim.x;
    const int u0 = threadIdx.x * per;
    unsigned long long own = 0, mx = 0;
    for (int u = u0; u < u0 + per && u < L; ++u) {
        const unsigned long long v = cnt[u];
        own += v;
        mx = v > mx ? v : mx;
    }
    unsigned long long total;
    unsigned long long run = block_exclusive_scan(own, &total);
    for (int u = u0; u < u0 + per && u < L; ++u) {
        const uint32_t v = cnt[u];
        cnt[u] = static_cast<uint32_t>(run) | (v << 16);
        run += v;
    }
    // the partition's largest bucket (also decides the ordering method
    // below)
    unsigned long long none = 0;
    block_sum_max(none, mx);
    __shared__ unsigned long long s_mx;
    if (threadIdx.x == 0) s_mx = mx;
    __syncthreads();
    const unsigned long long mx_all = s_mx;
    // each entry at its bucket's next place: the low half of cnt[] serves as
    // the cursor (it ends at the bucket's end, below 2^16)
    for (uint32_t u = threadIdx.x; u < c; u += blockDim.x) {
        const unsigned long long e = reg[u];
        const uint32_t loc = static_cast<uint32_t>(e >> 32) & lmask;
        const uint32_t at = atomicAdd(&cnt[loc], 1u) & 0xFFFFu;
        buf[at] = (loc << 21) | static_cast<uint32_t>(e);
        fpr[at] = static_cast<uint8_t>(e >> kJoinFpShift);
    }
    __syncthreads();
    // large buckets (clustered samples: few distinct block contents): sort
    // the whole partition (bitonic, 4-byte keys in LDS) instead of ranking
    // each entry by a pass over its bucket, which would be quadratic
    const bool big = mx_all > kJoinRankMax;
    if (big) {
        uint32_t P2 = 2;
        while (P2 < c) P2 <<= 1;
        for (uint32_t u = c + threadIdx.x; u < P2; u += blockDim.x) buf[u] = 0xFFFFFFFFu;
        for (uint32_t k = 2; k <= P2; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                __syncthreads();
                for (uint32_t t = threadIdx.x; t < (P2 >> 1); t += blockDim.x) {
                    // the t-th index with bit j clear, and its partner
                    const uint32_t a = ((t & ~(j - 1u)) << 1) | (t & (j - 1u)), l = a + j;
                    const uint32_t va = buf[a], vl = buf[l];
                    if ((va > vl) == ((a & k) == 0)) {
                        buf[a] = vl;
                        buf[l] = va;
                    }
                }
            }
        }
        __syncthreads();
    }
    const int blk = p >> (sc.join_log2m - sc.join_lshift);
    const uint4 *__restrict__ src = reinterpret_cast<const uint4 *>(samples);
    uint4 *keys = reinterpret_cast<uint4 *>(sc.jkeys);
    // each entry's place: its bucket's start, the members of its bucket with
    // a smaller fingerprint, then those of its own fingerprint with a smaller
    // sample index; its range is its fingerprint group (the whole bucket for
    // a bitonic-sorted partition)
    unsigned long long pairs = 0;
    for (uint32_t u = threadIdx.x; u < c; u += blockDim.x) {
        const uint32_t v = buf[u];
        const uint32_t loc = v >> 21, me = v & 0x1FFFFFu;
        const uint32_t r = cnt[loc];
        const uint32_t m = r >> 16, bs = (r & 0xFFFFu) - m;
        uint32_t rank = 0, gs = bs, gm = m;
        if (big) {
            rank = u - bs;  // sorted: the place in the bucket is the offset
        } else if (m >= 2) {
            const uint32_t f = fpr[u];
            uint32_t below = 0, same = 0;
            for (uint32_t q = bs; q < bs + m; ++q) {
                const uint32_t fq = fpr[q], mq = buf[q] & 0x1FFFFFu;
                below += fq < f ? 1u : 0u;
                same += fq == f ? 1u : 0u;
                rank += (fq < f || (fq == f && mq < me)) ? 1u : 0u;
            }
            gs = bs + below;
            gm = same;
        }
        pairs += gm;
        const uint32_t dst = s0 + bs + rank;
        sc.jent[dst] = me;
        sc.jrange[dst] = (s0 + gs) | (static_cast<unsigned long long>(gm) << 32) |
                         (static_cast<unsigned long long>(blk) << 48);
        // (a sample alone in its group is never paired: no bit string)
        if (gm >= 2) keys[dst] = src[me];
    }
    // the partition's sum of squared group sizes (each entry adds its
    // group's size) and its largest bucket
    unsigned long long unused = 0;
    block_sum_max(pairs, unused);
    if (threadIdx.x == 0) {
        sc.jstat[2 * p] = pairs;
        sc.jstat[2 * p + 1] = mx_all;
    }
}

// The join's cost and largest bucket over the partitions, and the decision
// (by one whole block).
__device__ __forceinline__ void join_decide(const DevTable &tab, const DevScratch &sc,
                                            const uint64_t *__restrict__ samples, int64_t n,
                                            int64_t g_eff) {
    unsigned long long q = 0, m = 0;
    for (int p = threadIdx.x; p < sc.join_parts; p += blockDim.x) {
        q += sc.jstat[2 * p];
        const unsigned long long mm = sc.jstat[2 * p + 1];
        m = mm > m ? mm : m;
    }
    block_sum_max(q, m);
    if (threadIdx.x != 0) return;
    // the alternative: the enumeration's lookups when it can take this batch
    // (one sector, an occupation whose round fits on chip), else streaming
    // every group past every sample (cheaper per pair)
    bool enum_usable = tab.enum_ok && *sc.mixed == 0;
    if (enum_usable) {
        const uint64_t s0 = samples[0], s1 = samples[1];
        const int na = __popcll(s0 & tab.spin_a0) + __popcll(s1 & tab.spin_a1);
        const int nb = __popcll(s0 & tab.spin_b0) + __popcll(s1 & tab.spin_b1);
        enum_usable = enum_round_size(tab.k_alpha, tab.k_beta, na, nb) > 0;
    }
    unsigned long long probes = 0;
    for (int k = 0; k < 64; ++k) probes += sc.jctl[kJoinCtlProbeSlots + k];
    sc.jctl[kJoinCtlProbes] = probes;
    // costs in units of one enumeration probe, from MI355X timings of both
    // strategies over 64 molecule-shaped jobs (24..100 qubits, 10^3..2.6 10^5
    // samples): a candidate pair of the join costs about 4 probes, an entry
    // (its grouping and its share of the pair kernel) about 40, the join's
    // extra launches about 10^7; a probe against a filter split into class
    // partitions costs about 4 (each round walks the partitions).  Hits cost
    // the same in every strategy and do not enter.
    const double alt = enum_usable
                           ? static_cast<double>(probes) * (sc.eparts_log2 > 0 ? 4.0 : 1.0)
                           : 0.5 * static_cast<double>(n) * static_cast<double>(g_eff);
    const double entries = static_cast<double>(tab.join_blocks) * static_cast<double>(n);
    const double cand = static_cast<double>(q) > entries ? static_cast<double>(q) - entries : 0.0;
    const double cost = 4.0 * cand + 40.0 * entries + 1.0e7;
    const bool fits = sc.jctl[kJoinCtlOver] == 0ull;
    const bool chosen = fits && (sc.join_force != 0 || cost < alt);
    sc.jctl[kJoinCtlCost] = q;
    sc.jctl[kJoinCtlMax] = m;
    sc.jctl[kJoinCtlChosen] = chosen ? 1ull : 0ull;
}

// One block per partition: its entries ordered by (bucket, content
// fingerprint, sample) and written back, each with the range of its group
// (the members of its bucket with its fingerprint), its block and its bit
// string; the partition's sum of squared group sizes and largest bucket.  A
// counting sort by bucket (LDS counts, their scan, then each entry at its
// bucket's start plus a cursor in the same word) groups the buckets; an
// entry's place inside its bucket is then the number of members with a
// smaller content fingerprint (which the scatter put in the entry's top
// byte), or the same one and a smaller sample index (a pass over the
// bucket, as long as the pair kernel's).  Buckets of hash-colliding
// contents thus split, and the pair kernel tests only the pairs whose
// contents agree up to 2^-8.  LDS holds 4 bytes per entry (bucket << 21 |
// sample) and its fingerprint byte, so that several blocks share a CU.  A partition whose largest bucket needs the bitonic sort keeps
// whole buckets as its groups.  A partition of more than kJoinPartCap
// entries is only flagged (the join then does not run).
template <int W>
__global__ __launch_bounds__(kJoinSortThreads) void join_sort_kernel(
    DevTable tab, DevScratch sc, const uint64_t *__restrict__ samples) {
    const int p = blockIdx.x;
    const uint32_t c = sc.jcnt[p];
    // the partition's first output place: the entries of the partitions
    // before it (every sample has one entry per block, so they all fit)
    unsigned long long before = 0;
    for (int q = threadIdx.x; q < p; q += blockDim.x) before += sc.jcnt[q];
    unsigned long long s0;
    (void)block_exclusive_scan(before, &s0);
    if (c > static_cast<uint32_t>(kJoinPartCap)) {
        if (threadIdx.x == 0) {
            sc.jstat[2 * p] = static_cast<unsigned long long>(c) * c;
            sc.jstat[2 * p + 1] = c;
            sc.jctl[kJoinCtlOver] = 1ull;
        }
        return;
    }
    join_sort_partition<W>(tab, sc, samples, p, c, static_cast<uint32_t>(s0));
}

// One block: the decision, once every partition is sorted.  (Taking it in
// the sort kernel's last block would need a device-scope release fence in
// every block, which writes back the L2 of each XCD: far slower than a
// launch.)
__global__ __launch_bounds__(kJoinGroupThreads) void join_decide_kernel(
    DevTable tab, DevScratch sc, const uint64_t *__restrict__ samples, int64_t n, int64_t g_eff) {
    join_decide(tab, sc, samples, n, g_eff);
}

// The contribution of partner j (bit string y = x ^ d) to E_loc(x), or no
// hit when the table has no group with X = d.
template <int W, bool DUMP, int P, bool SCV>
__device__ __forceinline__ bool join_hit(const DevTable &tab, const Key<W> &x, const Key<W> &y,
                                         const Key<W> &d, int64_t i, int32_t j, double la,
                                         double ph, const double *__restrict__ log_amp,
                                         const double *__restrict__ phase,
                                         int32_t *__restrict__ hit_idx,
                                         uint32_t *__restrict__ sign_bits, int64_t sign_words,
                                         unsigned long long *terms, double &re, double &im,
                                         AccF32 &ar, AccF32 &ai) {
    // any pair within the distance bound is a candidate (in a batch that
    // spans several sectors also spin-changing ones), so the group index
    // decides in the integral form too
    const int64_t g = group_find<W>(tab, linear_hash<W>(d, tab.hr), d);
    if constexpr (DUMP) {
        if (hit_idx && g >= 0) hit_idx[i * tab.n_groups + g] = j;
    }
    if (g < 0) return false;
    if constexpr (P == NQS_FP64) {
        uint32_t *row = (DUMP && sign_bits) ? sign_bits + i * sign_words : nullptr;
        double hsum;
        if constexpr (SCV) {
            (void)row;
            hsum = sc_element<W>(tab, x, y);
        } else {
            hsum = group_sum<W, DUMP>(tab, g, x, row, terms);
        }
        const double2 rat = amp_ratio_f64(log_amp[j] - la, phase[j] - ph);
        re += hsum * rat.x;
        im += hsum * rat.y;
    } else {
        const AccF32 hs = group_sum_f32<W>(tab, g, x, terms);
        float rr, ri;
        ratio_f32(log_amp[j] - la, phase[j] - ph, rr, ri);
        const float pre = hs.s * rr, pim = hs.s * ri;
        ar.add(pre, fmaf(hs.s, rr, -pre) + hs.c * rr);
        ai.add(pim, fmaf(hs.s, ri, -pim) + hs.c * ri);
    }
    return true;
}

// One lane per entry with partners (block b, sample i; each wave gathers
// them from its per x 64 consecutive entries, so that with per > 1 lanes
// are not spent on the many entries alone in their group): the partners of
// i in its group, in index order; with a hit, its partial sum goes to
// part[b][i] and bit b * n + i of the hit map is set (the finish reads only
// flagged partials).  The first build_blocks blocks are the sample-hash
// build of the same launch instead (its checks always; its insertion when
// the join is not chosen): both need only the decision, so one launch
// carries both.
template <int W, bool DUMP, int P, bool SCV>
__global__ __launch_bounds__(kJoinPairThreads) void join_pair_kernel(
    DevTable tab, DevScratch sc, const uint64_t *__restrict__ samples,
    const int64_t *__restrict__ weights, const double *__restrict__ log_amp,
    const double *__restrict__ phase, int64_t n, unsigned build_blocks, int per,
    int32_t *__restrict__ hit_idx, uint32_t *__restrict__ sign_bits, int64_t sign_words) {
    if (blockIdx.x < build_blocks) {
        const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
        if (i < n) hash_build_one<W>(tab, sc, samples, weights, i);
        return;
    }
    if (!join_chosen(sc)) return;
    // each wave takes per x 64 consecutive entries (per <= kJoinPairPer)
    // and gathers those with partners into its lanes
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ uint32_t picks[kJoinPairThreads / 64][64 * kJoinPairPer];
    const int64_t entries = static_cast<int64_t>(tab.join_blocks) * n;
    const int64_t base =
        (static_cast<int64_t>(blockIdx.x - build_blocks) * (kJoinPairThreads / 64) + wave) *
        (64 * per);
    uint32_t listed = 0;
    for (int k = 0; k < per; ++k) {
        const int64_t p = base + 64 * k + lane;
        const bool grouped = p < entries && ((sc.jrange[p] >> 32) & 0xFFFFull) >= 2ull;
        const unsigned long long mask = __ballot(grouped);
        if (grouped)
            picks[wave][listed + __popcll(mask & ((1ull << lane) - 1ull))] =
                static_cast<uint32_t>(64 * k + lane);
        listed += static_cast<uint32_t>(__popcll(mask));
    }
    __syncthreads();
    const uint32_t *__restrict__ ent = sc.jent;
    const int maxf = tab.max_flip;
    unsigned long long n_cand = 0, n_probe = 0, n_hit = 0, n_term = 0;
    for (uint32_t t = static_cast<uint32_t>(lane); t < listed; t += 64) {
        const int64_t p = base + picks[wave][t];
        const int64_t i = ent[p];
        const unsigned long long r = sc.jrange[p];
        const uint32_t bs = static_cast<uint32_t>(r), m = static_cast<uint32_t>(r >> 32) & 0xFFFFu;
        const int b = static_cast<int>(r >> 48);
        const int64_t e = static_cast<int64_t>(b) * n + i;
        if (m >= 2) {
            const Key<W> x = load_key<W>(sc.jkeys, p);
            double re = 0.0, im = 0.0, la = 0.0, ph = 0.0;
            bool have_psi = false;
            AccF32 ar, ai;
            // one candidate: distance, first agreeing block, then the hit
            auto visit = [&](uint32_t q, const Key<W> &y) {
                if (q == static_cast<uint32_t>(p)) return;
                Key<W> d;
                int pop = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    d.w[w] = x.w[w] ^ y.w[w];
                    pop += __popcll(d.w[w]);
                }
                if (pop > maxf) return;
                // the first block on which x and y agree must be this one
                int first = tab.join_blocks;
#pragma unroll
                for (int cb = kJoinMaxBlocks - 1; cb >= 0; --cb) {
                    if (cb < tab.join_blocks) {
                        uint64_t v = d.w[0] & tab.jmask[cb][0];
                        if constexpr (W == 2) v |= d.w[W - 1] & tab.jmask[cb][1];
                        if (v == 0ull) first = cb;
                    }
                }
                if (first != b) return;
                if (pop == 0) {
                    latch(sc.err, NQS_E_DUPLICATE);
                    return;
                }
                const int32_t j = static_cast<int32_t>(ent[q]);
                ++n_probe;
                if (!have_psi) {
                    la = log_amp[i];
                    ph = phase[i];
                    have_psi = true;
                }
                if (join_hit<W, DUMP, P, SCV>(tab, x, y, d, i, j, la, ph, log_amp, phase, hit_idx,
                                              sign_bits, sign_words, &n_term, re, im, ar, ai))
                    ++n_hit;
            };
            // partners in index order; one-word bit strings four at a time
            // (large buckets wait on these loads; two-word strings would
            // cost the kernel a wave per SIMD in registers)
            uint32_t q = bs;
            if constexpr (W == 1) {
                for (; q + 4 <= bs + m; q += 4) {
                    const Key<W> y0 = load_key<W>(sc.jkeys, q), y1 = load_key<W>(sc.jkeys, q + 1);
                    const Key<W> y2 = load_key<W>(sc.jkeys, q + 2),
                                 y3 = load_key<W>(sc.jkeys, q + 3);
                    visit(q, y0);
                    visit(q + 1, y1);
                    visit(q + 2, y2);
                    visit(q + 3, y3);
                }
            }
            for (; q < bs + m; ++q) visit(q, load_key<W>(sc.jkeys, q));
            n_cand += m - 1;
            if (n_hit) {
                double2 sum;
                if constexpr (P == NQS_FP64) {
                    sum = make_double2(re, im);
                } else {
                    sum = make_double2(ar.value(), ai.value());
                }
                *reinterpret_cast<double2 *>(sc.part + 2 * e) = sum;
                atomicOr(&sc.jhit[e >> 5], 1u << (e & 31));
            }
        }
    }
    // one set of counter atomics per block
    __shared__ unsigned long long cnt[4][kJoinPairThreads / 64];
    n_cand = wave_sum(n_cand);
    n_probe = wave_sum(n_probe);
    n_hit = wave_sum(n_hit);
    n_term = wave_sum(n_term);
    if (lane == 0) {
        cnt[0][wave] = n_cand;
        cnt[1][wave] = n_probe;
        cnt[2][wave] = n_hit;
        cnt[3][wave] = n_term;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        unsigned long long v = 0;
        for (int w = 0; w < kJoinPairThreads / 64; ++w) v += cnt[threadIdx.x][w];
        const int slot[4] = {4, 1, 2, 3};
        if (v) count_add(sc.counters, slot[threadIdx.x], v);
    }
}

template <int W>
hipError_t launch_join_prep_w(const DevTable &tab, const DevScratch &sc,
                              const uint64_t *samples, const int64_t *weights, int64_t n,
                              int64_t g_eff, bool clear_hash, hipStream_t st) {
    const dim3 tiles(static_cast<unsigned>(sc.join_tiles));
    const dim3 blk(kJoinGroupThreads);
    // the hash clear rides along: four slots a thread in the blocks after
    // the tiles
    unsigned extra = 0;
    if (clear_hash) {
        const uint64_t cap = uint64_t(sc.slot_mask) + 1u, fw = uint64_t(1) << sc.filter_log2;
        const uint64_t efw = sc.eparts_log2 > 0 ? uint64_t(1) << (sc.eparts_log2 + sc.efilter_log2)
                                                : 0u;
        uint64_t span = cap > fw ? cap : fw;
        span = span > efw ? span : efw;
        extra = static_cast<unsigned>((span + 4 * kJoinGroupThreads - 1) / (4 * kJoinGroupThreads));
    }
    hipLaunchKernelGGL(join_scatter_kernel<W>, dim3(tiles.x + extra), blk, 0, st, tab, sc, samples,
                       weights, n);
    hipLaunchKernelGGL(join_sort_kernel<W>, dim3(static_cast<unsigned>(sc.join_parts)),
                       dim3(kJoinSortThreads), 0, st, tab, sc, samples);
    hipLaunchKernelGGL(join_decide_kernel, dim3(1), blk, 0, st, tab, sc, samples, n, g_eff);
    return hipGetLastError();
}

template <int W, bool D, int P, bool SCV>
hipError_t launch_pairs_w(const DevTable &tab, const DevScratch &sc, const uint64_t *samples,
                          const int64_t *weights, int build, const double *log_amp,
                          const double *phase, int64_t n, int32_t *hit_idx, uint32_t *sign_bits,
                          int64_t sign_words, hipStream_t st) {
    const int64_t entries = static_cast<int64_t>(tab.join_blocks) * n;
    const unsigned build_blocks =
        build ? static_cast<unsigned>((n + kJoinPairThreads - 1) / kJoinPairThreads) : 0u;
    // several entries a lane where most samples are alone in their groups:
    // blocks whose contents outnumber the samples (fewer waves, each
    // gathering its few entries with partners); one a lane where blocks
    // are short and groups large (every entry has work: parallelism first)
    int qmin = 128;
    for (int b = 0; b < tab.join_blocks; ++b) {
        const int q = __builtin_popcountll(tab.jmask[b][0]) + __builtin_popcountll(tab.jmask[b][1]);
        qmin = q < qmin ? q : qmin;
    }
    const int per = (qmin >= 62 || (int64_t(1) << qmin) >= 2 * n) ? kJoinPairPer : 1;
    const int64_t per_block = int64_t(kJoinPairThreads) * per;
    const dim3 grid(build_blocks + static_cast<unsigned>((entries + per_block - 1) / per_block));
    hipLaunchKernelGGL((join_pair_kernel<W, D, P, SCV>), grid, dim3(kJoinPairThreads), 0, st, tab,
                       sc, samples, weights, log_amp, phase, n, build_blocks, per, hit_idx,
                       sign_bits, sign_words);
    return hipGetLastError();
}

// Partitions and tiles of a launch of n samples with 2^log2m buckets per
// block: a partition covers 2^lshift buckets (2048, fewer for a small
// batch), about as many entries (fewer, larger partitions: the sorter's
// blocks all fit on the chip at once, and the tiles reserve fewer ranges);
// the grouping kernels take at most kJoinTiles tiles of a multiple of 1024
// samples.
struct JoinGeometry {
    int lshift, parts, tile, tiles, cap;
};

JoinGeometry join_geometry(const DevTable &tab, int64_t n, int log2m) {
    JoinGeometry g;
    g.lshift = log2m <= 11 ? log2m : (log2m <= 21 ? 11 : log2m - 10);
    g.parts = tab.join_blocks << (log2m - g.lshift);
    const int64_t per = (n + int64_t(kJoinTiles) * kJoinGroupThreads - 1) /
                        (int64_t(kJoinTiles) * kJoinGroupThreads);
    g.tile = static_cast<int>((per < 1 ? 1 : per) * kJoinGroupThreads);
    g.tiles = static_cast<int>((n + g.tile - 1) / g.tile);
    if (g.tiles < 1) g.tiles = 1;
    // a partition's region: as many entries as the sorter takes (a partition
    // belongs to one block, so it never has more than n)
    g.cap = static_cast<int>(n < kJoinPartCap ? n : kJoinPartCap);
    return g;
}

}  // namespace

int join_log2m_for(int64_t n) {
    int lg = 6;
    while ((int64_t(1) << lg) < n) ++lg;
    return lg;
}

namespace {

// Byte sizes of the join's pieces, in layout order.
constexpr int kJoinPieces = 8;
void join_sizes(const DevTable &tab, int64_t n, int log2m, size_t sizes[kJoinPieces]) {
    const JoinGeometry g = join_geometry(tab, n, log2m);
    const size_t entries = static_cast<size_t>(tab.join_blocks) * static_cast<size_t>(n);
    const size_t parts = static_cast<size_t>(g.parts);
    sizes[0] = 4 * parts;                                 // jcnt
    sizes[1] = 8 * parts * static_cast<size_t>(g.cap);    // jreg
    sizes[2] = 4 * entries;                               // jent
    sizes[3] = 8 * entries;                               // jrange
    sizes[4] = 16 * parts;                                // jstat
    sizes[5] = 8 * static_cast<size_t>(kJoinCtl);         // jctl
    sizes[6] = 16 * entries;                              // jkeys
    sizes[7] = 4 * ((entries + 31) / 32);                 // jhit
}

}  // namespace

size_t join_scratch_bytes(const DevTable &tab, int64_t n, int log2m) {
    if (tab.join_blocks <= 0 || n <= 0) return 0;
    size_t sizes[kJoinPieces];
    join_sizes(tab, n, log2m, sizes);
    size_t total = 0;
    for (size_t s : sizes) total = align256(total + s);
    return total;
}

void join_scratch_layout(const DevTable &tab, int64_t n, int log2m, char *base, DevScratch *sc) {
    size_t sizes[kJoinPieces];
    join_sizes(tab, n, log2m, sizes);
    size_t off[kJoinPieces];
    size_t total = 0;
    for (int k = 0; k < kJoinPieces; ++k) {
        off[k] = total;
        total = align256(total + sizes[k]);
    }
    const JoinGeometry g = join_geometry(tab, n, log2m);
    sc->jcnt = reinterpret_cast<uint32_t *>(base + off[0]);
    sc->jreg = reinterpret_cast<unsigned long long *>(base + off[1]);
    sc->jent = reinterpret_cast<uint32_t *>(base + off[2]);
    sc->jrange = reinterpret_cast<unsigned long long *>(base + off[3]);
    sc->jstat = reinterpret_cast<unsigned long long *>(base + off[4]);
    sc->jctl = reinterpret_cast<unsigned long long *>(base + off[5]);
    sc->jkeys = reinterpret_cast<uint64_t *>(base + off[6]);
    sc->jhit = reinterpret_cast<uint32_t *>(base + off[7]);
    sc->join_log2m = log2m;
    sc->join_n = n;
    sc->join_lshift = g.lshift;
    sc->join_parts = g.parts;
    sc->join_tile = g.tile;
    sc->join_tiles = g.tiles;
    sc->join_cap = g.cap;
}

hipError_t launch_join_prep(const DevTable &tab, const DevScratch &sc, const uint64_t *samples,
                            const int64_t *weights, int64_t n, int64_t g_eff, bool clear_hash,
                            hipStream_t st) {
    if (tab.n_qubits <= 63)
        return launch_join_prep_w<1>(tab, sc, samples, weights, n, g_eff, clear_hash, st);
    return launch_join_prep_w<2>(tab, sc, samples, weights, n, g_eff, clear_hash, st);
}

hipError_t launch_join_pairs(const DevTable &tab, const DevScratch &sc, const uint64_t *samples,
                             const int64_t *weights, int build, const double *log_amp,
                             const double *phase, int64_t n, int precision, int32_t *hit_idx,
                             uint32_t *sign_bits, int64_t sign_words, hipStream_t st) {
    const bool dump = hit_idx || sign_bits;
    const bool f32 = precision == NQS_FP32_KAHAN && !dump && !tab.sc;
    const bool w1 = tab.n_qubits <= 63;
#define NQS_PAIRS(Wd, D, Pr, SCI) \
    return launch_pairs_w<Wd, D, Pr, SCI>(tab, sc, samples, weights, build, log_amp, phase, n, \
                                          hit_idx, sign_bits, sign_words, st)
    if (tab.sc) {
        if (w1) {
            if (dump) NQS_PAIRS(1, true, NQS_FP64, true);
            NQS_PAIRS(1, false, NQS_FP64, true);
        }
        if (dump) NQS_PAIRS(2, true, NQS_FP64, true);
        NQS_PAIRS(2, false, NQS_FP64, true);
    }
    if (w1) {
        if (dump) NQS_PAIRS(1, true, NQS_FP64, false);
        if (f32) NQS_PAIRS(1, false, NQS_FP32_KAHAN, false);
        NQS_PAIRS(1, false, NQS_FP64, false);
    }
    if (dump) NQS_PAIRS(2, true, NQS_FP64, false);
    if (f32) NQS_PAIRS(2, false, NQS_FP32_KAHAN, false);
    NQS_PAIRS(2, false, NQS_FP64, false);
#undef NQS_PAIRS
}

}  // namespace nqs
