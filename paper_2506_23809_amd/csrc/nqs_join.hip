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
// Cost: the ordered pairs inside buckets, the sum of squared bucket sizes.
// For samples spread over a large sector this is far below the
// enumeration's N x (connected states per sample) lookups.  The decision is
// taken on the device from the bucket sizes, between the hash clear and the
// hash build: when the join is cheaper it runs, and the hash build's
// insertion, the enumeration and the streaming kernels of the same launch
// stand down; otherwise those run and the join's later kernels return at
// once.
//
// Determinism: the entries of a bucket are sorted by sample index before the
// pair kernel runs, so each sample's hits are added in a fixed order (one
// partial per block, partners in index order), and the finish kernel adds
// the block partials in block order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/nqs.h"
#include "nqs_dev_common.hpp"
#include "nqs_device.hpp"

namespace nqs {

namespace {

constexpr int kJoinThreads = 256;
constexpr int kJoinScanThreads = kJoinScanItems / 4;
constexpr int kJoinSmallSort = 32;  // buckets up to this size are sorted in registers
constexpr int kJoinSortThreads = 1024;

inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Bucket of block b of x: the block index in the top bits, a hash of the
// block's contents below (equal contents, equal bucket).
template <int W>
__device__ __forceinline__ uint32_t join_bucket(const DevTable &tab, const Key<W> &x, int b,
                                                int log2m) {
    uint32_t h = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        uint64_t v = x.w[q] & tab.jmask[b][q];
        while (v) {
            h ^= tab.hr[64 * q + __builtin_ctzll(v)];
            v &= v - 1;
        }
    }
    const uint32_t slot = log2m > 0 ? (h * kGoldenMul) >> (32 - log2m) : 0u;
    return (static_cast<uint32_t>(b) << log2m) | slot;
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

// In-register bitonic sort of N values (N a power of two; constant indices).
template <int N>
__device__ __forceinline__ void bitonic_regs(uint32_t (&v)[N]) {
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const uint32_t a = v[i], b = v[l];
                    const bool sw = ((i & k) == 0) ? (a > b) : (a < b);
                    v[i] = sw ? b : a;
                    v[l] = sw ? a : b;
                }
            }
        }
    }
}

// Entry p of the sorted bucket [s, e) of block b: sample j, its bit
// string, the range, the block.
__device__ __forceinline__ void join_put(const DevScratch &sc, const uint64_t *__restrict__ samples,
                                         uint32_t p, uint32_t j, uint32_t s, uint32_t e,
                                         uint32_t b) {
    sc.jent[p] = j;
    const uint4 key = reinterpret_cast<const uint4 *>(samples)[j];
    reinterpret_cast<uint4 *>(sc.jkeys)[p] = key;
    sc.jrange[p] = make_uint2(s, e);
    sc.jblk[p] = static_cast<uint8_t>(b);
}

template <int N>
__device__ __forceinline__ void join_sort_put(const DevScratch &sc,
                                              const uint64_t *__restrict__ samples, uint32_t s,
                                              uint32_t m, uint32_t b) {
    uint32_t v[N];
#pragma unroll
    for (int t = 0; t < N; ++t) v[t] = static_cast<uint32_t>(t) < m ? sc.jent[s + t] : 0xFFFFFFFFu;
    bitonic_regs<N>(v);
#pragma unroll
    for (int t = 0; t < N; ++t)
        if (static_cast<uint32_t>(t) < m) join_put(sc, samples, s + t, v[t], s, s + m, b);
}

// ---- kernels

// Per sample: its bucket in every block (counted), whether the batch spans
// several (N_alpha, N_beta) sectors, and the enumeration's lookups for it
// (its spin-conserving singles and doubles), summed for the decision.
template <int W>
__global__ __launch_bounds__(kJoinThreads) void join_count_kernel(DevTable tab, DevScratch sc,
                                                                  const uint64_t *__restrict__ samples,
                                                                  int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    unsigned long long probes = 0;
    if (i < n) {
        const Key<W> x = load_key<W>(samples, i);
        for (int b = 0; b < tab.join_blocks; ++b) {
            const uint32_t k = join_bucket<W>(tab, x, b, sc.join_log2m);
            sc.jkey[static_cast<int64_t>(b) * n + i] = k;
            atomicAdd(&sc.jcnt[k], 1u);
        }
        if (tab.sector_filter) {
            const uint64_t w0 = x.w[0], w1 = W == 2 ? x.w[W - 1] : 0ull;
            const uint64_t s0 = samples[0], s1 = samples[1];
            const int na = __popcll(w0 & tab.spin_a0) + __popcll(w1 & tab.spin_a1);
            const int nb = __popcll(w0 & tab.spin_b0) + __popcll(w1 & tab.spin_b1);
            const int ra = __popcll(s0 & tab.spin_a0) + __popcll(s1 & tab.spin_a1);
            const int rb = __popcll(s0 & tab.spin_b0) + __popcll(s1 & tab.spin_b1);
            if (na != ra || nb != rb) atomicOr(sc.mixed, 1);
            if (tab.enum_ok) {
                const unsigned long long va = tab.k_alpha - na, vb = tab.k_beta - nb;
                const unsigned long long a = na, bb = nb;
                probes = a * va + bb * vb + (a * (a - 1) / 2) * (va * (va - 1) / 2) +
                         (bb * (bb - 1) / 2) * (vb * (vb - 1) / 2) + a * va * bb * vb;
            }
        }
    }
    probes = wave_sum(probes);
    if ((threadIdx.x & 63) == 0 && probes)
        atomicAdd(&sc.jctl[kJoinCtlProbeSlots + blockIdx.x % 64], probes);
}

// Per scan block of kJoinScanItems bucket counts: the entries they take
// (buckets of two samples or more), the sum of their squares and the
// largest.
__global__ __launch_bounds__(kJoinScanThreads) void join_scan_sums_kernel(DevScratch sc,
                                                                          int64_t buckets) {
    __shared__ unsigned long long part[3][kJoinScanThreads / 64];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kJoinScanItems + 4 * threadIdx.x;
    unsigned long long s = 0, q = 0, m = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const unsigned long long v = base + t < buckets ? sc.jcnt[base + t] : 0u;
        s += v >= 2 ? v : 0;
        q += v * v;
        m = v > m ? v : m;
    }
    s = wave_sum(s);
    q = wave_sum(q);
    m = wave_max(m);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        part[0][wave] = s;
        part[1][wave] = q;
        part[2][wave] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long S = 0, Q = 0, M = 0;
        for (int w = 0; w < kJoinScanThreads / 64; ++w) {
            S += part[0][w];
            Q += part[1][w];
            M = part[2][w] > M ? part[2][w] : M;
        }
        const int64_t nb = gridDim.x;
        sc.jscan[blockIdx.x] = S;
        sc.jscan[nb + blockIdx.x] = Q;
        sc.jscan[2 * nb + blockIdx.x] = M;
    }
}

// One block: the exclusive scan of the scan blocks' sums (in place), the
// join's cost and largest bucket, and the decision.
__global__ __launch_bounds__(1024) void join_decide_kernel(DevTable tab, DevScratch sc,
                                                           const uint64_t *__restrict__ samples,
                                                           int64_t n, int64_t nscan,
                                                           int64_t g_eff) {
    __shared__ unsigned long long red[2][16];
    unsigned long long carry = 0, q = 0, m = 0;
    for (int64_t c0 = 0; c0 < nscan; c0 += blockDim.x) {
        const int64_t t = c0 + threadIdx.x;
        unsigned long long v = 0;
        if (t < nscan) {
            v = sc.jscan[t];
            q += sc.jscan[nscan + t];
            const unsigned long long mm = sc.jscan[2 * nscan + t];
            m = mm > m ? mm : m;
        }
        unsigned long long total;
        const unsigned long long ex = block_exclusive_scan(v, &total);
        if (t < nscan) sc.jscan[t] = carry + ex;
        carry += total;
    }
    q = wave_sum(q);
    m = wave_max(m);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = q;
        red[1][wave] = m;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    unsigned long long Q = 0, M = 0;
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) {
        Q += red[0][w];
        M = red[1][w] > M ? red[1][w] : M;
    }
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
    const double alt = enum_usable ? static_cast<double>(probes)
                                   : 0.5 * static_cast<double>(n) * static_cast<double>(g_eff);
    // the join's own fixed work: counting, scanning, scattering and sorting
    // the entries and buckets
    const double buckets = static_cast<double>(static_cast<int64_t>(tab.join_blocks)
                                               << sc.join_log2m);
    const double entries = static_cast<double>(tab.join_blocks) * static_cast<double>(n);
    const double cost = static_cast<double>(Q) + 4.0 * entries + 0.5 * buckets;
    const bool fits = M <= static_cast<unsigned long long>(kJoinMaxBucket);
    const bool chosen = fits && (sc.join_force != 0 || cost < alt);
    sc.jctl[kJoinCtlCost] = Q;
    sc.jctl[kJoinCtlMax] = M;
    sc.jctl[kJoinCtlEntries] = carry;
    sc.jctl[kJoinCtlChosen] = chosen ? 1ull : 0ull;
}

// Bucket start offsets: each scan block rescans its counts from the block's
// exclusive offset.
__global__ __launch_bounds__(kJoinScanThreads) void join_offsets_kernel(DevScratch sc,
                                                                        int64_t buckets) {
    if (!join_chosen(sc)) return;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kJoinScanItems + 4 * threadIdx.x;
    uint32_t v[4];
    unsigned long long own = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        v[t] = base + t < buckets ? sc.jcnt[base + t] : 0u;
        own += v[t] >= 2 ? v[t] : 0u;
    }
    unsigned long long total;
    unsigned long long off = sc.jscan[blockIdx.x] + block_exclusive_scan(own, &total);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (base + t < buckets) {
            sc.jcnt[base + t] = static_cast<uint32_t>(off);
            sc.jsize[base + t] = v[t];
        }
        off += v[t] >= 2 ? v[t] : 0u;
    }
}

// Entries into their buckets (any order; sorted next).  Afterwards jcnt[k]
// holds the end of bucket k, whose start is that less jsize[k].  A sample
// alone in its bucket has no partner in that block: its partial is zero,
// written here, and it takes no entry.
__global__ __launch_bounds__(kJoinThreads) void join_scatter_kernel(DevTable tab, DevScratch sc,
                                                                    int64_t n) {
    if (!join_chosen(sc)) return;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int b = 0; b < tab.join_blocks; ++b) {
        const uint32_t k = sc.jkey[static_cast<int64_t>(b) * n + i];
        if (sc.jsize[k] < 2u) {
            double *out = sc.part + 2 * (static_cast<int64_t>(b) * n + i);
            out[0] = 0.0;
            out[1] = 0.0;
            continue;
        }
        const uint32_t pos = atomicAdd(&sc.jcnt[k], 1u);
        sc.jent[pos] = static_cast<uint32_t>(i);
    }
}

// One thread per bucket: a bucket of up to kJoinSmallSort entries is sorted
// in registers and written out with its keys and range; a larger one goes to
// the block sorter's list.
__global__ __launch_bounds__(kJoinThreads) void join_sort_small_kernel(
    DevScratch sc, const uint64_t *__restrict__ samples, int64_t buckets) {
    if (!join_chosen(sc)) return;
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= buckets) return;
    const uint32_t m = sc.jsize[k];
    if (m < 2) return;  // no entry
    const uint32_t e = sc.jcnt[k], s = e - m;
    const uint32_t blk = static_cast<uint32_t>(k >> sc.join_log2m);
    if (m == 2) {
        const uint32_t a = sc.jent[s], b = sc.jent[s + 1];
        join_put(sc, samples, s, a < b ? a : b, s, e, blk);
        join_put(sc, samples, s + 1, a < b ? b : a, s, e, blk);
    } else if (m <= 4) {
        join_sort_put<4>(sc, samples, s, m, blk);
    } else if (m <= 8) {
        join_sort_put<8>(sc, samples, s, m, blk);
    } else if (m <= 16) {
        join_sort_put<16>(sc, samples, s, m, blk);
    } else if (m <= static_cast<uint32_t>(kJoinSmallSort)) {
        join_sort_put<32>(sc, samples, s, m, blk);
    } else {
        const unsigned long long t = atomicAdd(&sc.jctl[kJoinCtlBig], 1ull);
        sc.jbig[t] = static_cast<uint32_t>(k);
    }
}

// The listed buckets (more than kJoinSmallSort entries, at most
// kJoinMaxBucket: the decision guarantees it), one block each at a time:
// bitonic sort in LDS, then written out.
__global__ __launch_bounds__(kJoinSortThreads) void join_sort_big_kernel(
    DevScratch sc, const uint64_t *__restrict__ samples) {
    if (!join_chosen(sc)) return;
    __shared__ uint32_t buf[kJoinMaxBucket];
    const unsigned long long nbig = sc.jctl[kJoinCtlBig];
    for (unsigned long long t = blockIdx.x; t < nbig; t += gridDim.x) {
        const uint32_t k = sc.jbig[t];
        const uint32_t m = sc.jsize[k];
        const uint32_t e = sc.jcnt[k], s = e - m;
        const uint32_t blk = k >> sc.join_log2m;
        uint32_t P = 64;
        while (P < m) P <<= 1;
        for (uint32_t u = threadIdx.x; u < P; u += blockDim.x)
            buf[u] = u < m ? sc.jent[s + u] : 0xFFFFFFFFu;
        __syncthreads();
        for (uint32_t kk = 2; kk <= P; kk <<= 1) {
            for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
                for (uint32_t u = threadIdx.x; u < P; u += blockDim.x) {
                    const uint32_t l = u ^ j;
                    if (l > u) {
                        const uint32_t a = buf[u], b = buf[l];
                        const bool sw = ((u & kk) == 0) ? (a > b) : (a < b);
                        if (sw) {
                            buf[u] = b;
                            buf[l] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t u = threadIdx.x; u < m; u += blockDim.x)
            join_put(sc, samples, s + u, buf[u], s, e, blk);
        __syncthreads();
    }
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
        double sn, cs;
        sincos(phase[j] - ph, &sn, &cs);
        const double mag = exp(log_amp[j] - la);
        re += hsum * (mag * cs);
        im += hsum * (mag * sn);
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

// One lane per entry (block b, sample i): the partners of i in its bucket of
// block b, in index order; its partial sum goes to part[b][i].
template <int W, bool DUMP, int P, bool SCV>
__global__ __launch_bounds__(kJoinThreads) void join_pair_kernel(
    DevTable tab, DevScratch sc, const double *__restrict__ log_amp,
    const double *__restrict__ phase, int64_t n, int32_t *__restrict__ hit_idx,
    uint32_t *__restrict__ sign_bits, int64_t sign_words) {
    if (!join_chosen(sc)) return;
    // the entries of buckets of two samples or more
    const int64_t total = static_cast<int64_t>(sc.jctl[kJoinCtlEntries]);
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    unsigned long long n_cand = 0, n_probe = 0, n_hit = 0, n_term = 0;
    if (p < total) {
        const int b = sc.jblk[p];
        const int64_t i = sc.jent[p];
        const uint4 xk = reinterpret_cast<const uint4 *>(sc.jkeys)[p];
        Key<W> x;
        x.w[0] = (static_cast<uint64_t>(xk.y) << 32) | xk.x;
        if constexpr (W == 2) x.w[W - 1] = (static_cast<uint64_t>(xk.w) << 32) | xk.z;
        const uint2 r = sc.jrange[p];
        double re = 0.0, im = 0.0, la = 0.0, ph = 0.0;
        bool have_psi = false;
        AccF32 ar, ai;
        const int maxf = tab.max_flip;
        const uint4 *keys = reinterpret_cast<const uint4 *>(sc.jkeys);
        auto visit = [&](uint32_t q, uint4 yk) {
            Key<W> d;
            d.w[0] = x.w[0] ^ ((static_cast<uint64_t>(yk.y) << 32) | yk.x);
            int pop = __popcll(d.w[0]);
            if constexpr (W == 2) {
                d.w[W - 1] = x.w[W - 1] ^ ((static_cast<uint64_t>(yk.w) << 32) | yk.z);
                pop += __popcll(d.w[W - 1]);
            }
            if (pop > maxf || q == static_cast<uint32_t>(p)) return;
            // the first block on which x and y agree must be this one
            int first = tab.join_blocks;
#pragma unroll
            for (int c = kJoinMaxBlocks - 1; c >= 0; --c) {
                if (c < tab.join_blocks) {
                    uint64_t v = d.w[0] & tab.jmask[c][0];
                    if constexpr (W == 2) v |= d.w[W - 1] & tab.jmask[c][1];
                    if (v == 0ull) first = c;
                }
            }
            if (first != b) return;
            if (pop == 0) {
                latch(sc.err, NQS_E_DUPLICATE);
                return;
            }
            ++n_probe;
            if (!have_psi) {
                la = log_amp[i];
                ph = phase[i];
                have_psi = true;
            }
            Key<W> y;
#pragma unroll
            for (int w = 0; w < W; ++w) y.w[w] = x.w[w] ^ d.w[w];
            const int32_t j = static_cast<int32_t>(sc.jent[q]);
            if (join_hit<W, DUMP, P, SCV>(tab, x, y, d, i, j, la, ph, log_amp, phase, hit_idx,
                                          sign_bits, sign_words, &n_term, re, im, ar, ai))
                ++n_hit;
        };
        uint32_t q = r.x;
        // four partner keys in flight per step
        for (; q + 4 <= r.y; q += 4) {
            const uint4 k0 = keys[q], k1 = keys[q + 1], k2 = keys[q + 2], k3 = keys[q + 3];
            visit(q, k0);
            visit(q + 1, k1);
            visit(q + 2, k2);
            visit(q + 3, k3);
        }
        for (; q < r.y; ++q) visit(q, keys[q]);
        n_cand = r.y - r.x - 1;
        double *out = sc.part + 2 * (static_cast<int64_t>(b) * n + i);
        if constexpr (P == NQS_FP64) {
            out[0] = re;
            out[1] = im;
        } else {
            out[0] = ar.value();
            out[1] = ai.value();
        }
    }
    // one set of counter atomics per block
    __shared__ unsigned long long cnt[4][kJoinThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
        for (int w = 0; w < kJoinThreads / 64; ++w) v += cnt[threadIdx.x][w];
        const int slot[4] = {4, 1, 2, 3};
        count_add(sc.counters, slot[threadIdx.x], v);
    }
}

template <int W>
hipError_t launch_join_prep_w(const DevTable &tab, const DevScratch &sc,
                              const uint64_t *samples, int64_t n, int64_t g_eff, hipStream_t st) {
    const int64_t buckets = static_cast<int64_t>(tab.join_blocks) << sc.join_log2m;
    const int64_t nscan = (buckets + kJoinScanItems - 1) / kJoinScanItems;
    const dim3 sgrid(static_cast<unsigned>((n + kJoinThreads - 1) / kJoinThreads));
    hipLaunchKernelGGL(join_count_kernel<W>, sgrid, dim3(kJoinThreads), 0, st, tab, sc, samples, n);
    hipLaunchKernelGGL(join_scan_sums_kernel, dim3(static_cast<unsigned>(nscan)),
                       dim3(kJoinScanThreads), 0, st, sc, buckets);
    hipLaunchKernelGGL(join_decide_kernel, dim3(1), dim3(1024), 0, st, tab, sc, samples, n, nscan,
                       g_eff);
    hipLaunchKernelGGL(join_offsets_kernel, dim3(static_cast<unsigned>(nscan)),
                       dim3(kJoinScanThreads), 0, st, sc, buckets);
    hipLaunchKernelGGL(join_scatter_kernel, sgrid, dim3(kJoinThreads), 0, st, tab, sc, n);
    hipLaunchKernelGGL(join_sort_small_kernel,
                       dim3(static_cast<unsigned>((buckets + kJoinThreads - 1) / kJoinThreads)),
                       dim3(kJoinThreads), 0, st, sc, samples, buckets);
    // the listed buckets number at most entries / (kJoinSmallSort + 1)
    const int64_t max_big = static_cast<int64_t>(tab.join_blocks) * n / (kJoinSmallSort + 1);
    const int64_t big_grid = max_big < 1 ? 1 : (max_big < 2048 ? max_big : 2048);
    hipLaunchKernelGGL(join_sort_big_kernel, dim3(static_cast<unsigned>(big_grid)),
                       dim3(kJoinSortThreads), 0, st, sc, samples);
    return hipGetLastError();
}

template <int W, bool D, int P, bool SCV>
hipError_t launch_pairs_w(const DevTable &tab, const DevScratch &sc, const double *log_amp,
                          const double *phase, int64_t n, int32_t *hit_idx, uint32_t *sign_bits,
                          int64_t sign_words, hipStream_t st) {
    const int64_t total = static_cast<int64_t>(tab.join_blocks) * n;
    const dim3 grid(static_cast<unsigned>((total + kJoinThreads - 1) / kJoinThreads));
    hipLaunchKernelGGL((join_pair_kernel<W, D, P, SCV>), grid, dim3(kJoinThreads), 0, st, tab, sc,
                       log_amp, phase, n, hit_idx, sign_bits, sign_words);
    return hipGetLastError();
}

}  // namespace

int join_log2m_for(int64_t n) {
    int lg = 6;
    while ((int64_t(1) << lg) < n) ++lg;
    return lg;
}

namespace {

// Byte sizes of the join's pieces, in layout order.
constexpr int kJoinPieces = 9;
void join_sizes(const DevTable &tab, int64_t n, int log2m, size_t sizes[kJoinPieces]) {
    const size_t B = static_cast<size_t>(tab.join_blocks);
    const size_t buckets = B << log2m;
    const size_t entries = B * static_cast<size_t>(n);
    const size_t nscan = (buckets + kJoinScanItems - 1) / kJoinScanItems;
    sizes[0] = 4 * buckets;                    // jcnt
    sizes[1] = 4 * entries;                    // jkey, then the block sorter's list
    sizes[2] = 4 * entries;                    // jent
    sizes[3] = 8 * entries;                    // jrange
    sizes[4] = 16 * entries;                   // jkeys
    sizes[5] = 8 * 3 * nscan;                  // jscan
    sizes[6] = 8 * static_cast<size_t>(kJoinCtl);  // jctl
    sizes[7] = 4 * buckets;                    // jsize
    sizes[8] = entries;                        // jblk
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
    sc->jcnt = reinterpret_cast<uint32_t *>(base + off[0]);
    sc->jkey = reinterpret_cast<uint32_t *>(base + off[1]);
    sc->jbig = sc->jkey;  // the bucket keys are dead once the entries are scattered
    sc->jent = reinterpret_cast<uint32_t *>(base + off[2]);
    sc->jrange = reinterpret_cast<uint2 *>(base + off[3]);
    sc->jkeys = reinterpret_cast<uint64_t *>(base + off[4]);
    sc->jscan = reinterpret_cast<unsigned long long *>(base + off[5]);
    sc->jctl = reinterpret_cast<unsigned long long *>(base + off[6]);
    sc->jsize = reinterpret_cast<uint32_t *>(base + off[7]);
    sc->jblk = reinterpret_cast<uint8_t *>(base + off[8]);
    sc->join_log2m = log2m;
}

hipError_t launch_join_prep(const DevTable &tab, const DevScratch &sc, const uint64_t *samples,
                            int64_t n, int64_t g_eff, hipStream_t st) {
    if (tab.n_qubits <= 63) return launch_join_prep_w<1>(tab, sc, samples, n, g_eff, st);
    return launch_join_prep_w<2>(tab, sc, samples, n, g_eff, st);
}

hipError_t launch_join_pairs(const DevTable &tab, const DevScratch &sc, const uint64_t *samples,
                             const double *log_amp, const double *phase, int64_t n, int precision,
                             int32_t *hit_idx, uint32_t *sign_bits, int64_t sign_words,
                             hipStream_t st) {
    (void)samples;
    const bool dump = hit_idx || sign_bits;
    const bool f32 = precision == NQS_FP32_KAHAN && !dump && !tab.sc;
    const bool w1 = tab.n_qubits <= 63;
#define NQS_PAIRS(Wd, D, Pr, SCI) \
    return launch_pairs_w<Wd, D, Pr, SCI>(tab, sc, log_amp, phase, n, hit_idx, sign_bits, sign_words, st)
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
