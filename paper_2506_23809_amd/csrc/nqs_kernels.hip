// HIP kernels (gfx950) for the sample-space local energy.
//
//   E_loc(x) = sum_{x' in S} <x|H|x'> psi(x') / psi(x)           (Eq. 5)
//
// The per-sample outer loop of the multi-level scheme (Eq. 6, Alg. 3) is the
// GPU grid: one lane owns one sample x and keeps it in registers.  The inner
// loop over kets runs over the X groups of the Pauli table instead of over
// determinants: every term of group g connects x to x' = x ^ X_g, so one
// lookup of x' in the sample hash (the psi lookup table of the sample-space
// energy) decides the whole group.  A hit evaluates
//   <x|H|x'> = sum_{t in g} c~_t (-1)^{popc(Z_t & x)}
// with the folded coefficient c~ = c (-1)^{ny/2} (one popcount per term, the
// parity step of Alg. 3) and multiplies it by exp(a' - a) e^{i(phi' - phi)}.
//
// Lookup pipeline of the E_loc kernel, per (sample, group) pair:
//   1. sector test on compressed alpha/beta bit fields (flips that change
//      N_alpha or N_beta cannot land in S when all samples share a sector);
//   2. linear hash: h(x ^ X) = h(x) ^ h(X), one XOR;
//   3. two bits of one word of an LDS-resident blocked Bloom bitmap of the
//      sample hashes: most x' not in S stop here without touching global
//      memory;
//   4. survivors are compacted into a per-wave LDS queue (ballot + mbcnt)
//      and looked up 64 at a time in the global open-addressing hash.
// Group records stream through LDS in stages; the filter stays resident for
// the whole block.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "../../include/nqs.h"
#include "nqs_device.hpp"
#include "nqs_dev_common.hpp"

namespace nqs {

// ------------------------------------------------------------------ hash build

// Frees every slot (index -1, fingerprint 0, key's last word kFreeKey) and clears the
// Bloom bitmaps.
__global__ void hash_clear_kernel(uint64_t *__restrict__ skey, int32_t *__restrict__ sidx,
                                  uint32_t *__restrict__ sfp,
                                  int words, uint32_t capacity, uint32_t *__restrict__ filter,
                                  uint32_t filter_words, uint32_t *__restrict__ efilter,
                                  uint32_t efilter_words, unsigned long long *__restrict__ counters,
                                  int *__restrict__ mixed, uint32_t *__restrict__ jcnt,
                                  uint32_t jparts, unsigned long long *__restrict__ jctl,
                                  uint32_t *__restrict__ jhit, uint32_t jhit_words) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    // the batch's counters and sector flag start at zero as well, and so do
    // the pair join's partition counts and control words
    if (s < static_cast<uint32_t>(kCounters * kCounterSlots)) counters[s] = 0;
    if (s == 0) *mixed = 0;
    if (jctl && s < static_cast<uint32_t>(kJoinCtl)) jctl[s] = 0;
    if (s < jparts) jcnt[s] = 0u;
    if (s < jhit_words) jhit[s] = 0u;
    if (s < capacity) {
        sidx[s] = -1;
        sfp[s] = 0u;
        skey[static_cast<size_t>(s) * words + words - 1] = kFreeKey;
    }
    if (s < filter_words) filter[s] = 0u;
    if (s < efilter_words) efilter[s] = 0u;
}

template <int W>
__global__ void hash_build_kernel(DevTable tab, DevScratch sc,
                                  const uint64_t *__restrict__ samples,
                                  const int64_t *__restrict__ weights, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) hash_build_one<W>(tab, sc, samples, weights, i);
}

// ------------------------------------------------------------------ E_loc

constexpr int kLookupThreads = 1024;
constexpr int kStage = 512;      // group records per LDS stage (multiple of kUnroll)
constexpr int kQueueCap = 128;   // per-wave candidate queue (flushed at 64)
constexpr int kUnroll = 4;       // groups tested per inner iteration
constexpr uint32_t kPadKey = 0xFFFFFFFFu;  // stage padding: never a candidate
static_assert(kStage % kUnroll == 0, "stage must hold whole unrolled iterations");
// Largest dynamic LDS a lookup block asks for: 128 KB bitmap, 512 32-byte
// records, 16 queues of 128 entries (152 KB; the CU has 160 KB).
constexpr int kMaxLookupLds = (4 << 15) + kStage * 32 + 16 * kQueueCap * 4;

template <bool S32>
struct StageRec;
template <>
struct alignas(16) StageRec<true> {
    uint32_t ca, cb, hx, key;
};
template <>
struct alignas(16) StageRec<false> {
    uint64_t ca, cb;
    uint32_t hx, key, pad0, pad1;
};

size_t lookup_lds_bytes(bool s32, int filter_log2, int threads) {
    const size_t rec = s32 ? sizeof(StageRec<true>) : sizeof(StageRec<false>);
    return (size_t(4) << filter_log2) + kStage * rec + size_t(threads / 64) * kQueueCap * 4;
}

// Sum of one group's terms for bra x: sum_t c~_t (-1)^{popc(Z_t & x)}.
// One (sample tile, group chunk) work item on one block.  Each lane walks the
// groups of the chunk in order; hits are added to the owning lane in queue
// order, which is group order, so the partial sum does not depend on
// scheduling.  The X = 0 group is left to the finish kernel.  The caller
// has synchronised the block; load_filter = false reuses the bitmap already
// in LDS (same Hamiltonian and batch as the previous item).
template <int W, bool S32, bool SEC, bool DUMP, int P, bool SCV>
__device__ __forceinline__ void lookup_item(
    const DevTable &tab, const DevScratch &sc, const uint64_t *__restrict__ samples,
    const double *__restrict__ log_amp, const double *__restrict__ phase, int64_t n,
    int64_t tile, int64_t chunk, int64_t g_first, int64_t chunk_len, bool load_filter,
    int32_t *__restrict__ hit_idx, uint32_t *__restrict__ sign_bits, int64_t sign_words,
    uint4 *smem4) {
    using Rec = StageRec<S32>;
    const int fwords = 1 << sc.filter_log2;
    uint32_t *filt = reinterpret_cast<uint32_t *>(smem4);
    Rec *stage = reinterpret_cast<Rec *>(filt + fwords);
    const int lane = threadIdx.x & 63;
    uint32_t *queue = reinterpret_cast<uint32_t *>(stage + kStage) + (threadIdx.x >> 6) * kQueueCap;

    const int64_t tile0 = tile * blockDim.x;
    const int64_t wave0 = tile0 + (threadIdx.x & ~63);
    const int64_t i = tile0 + threadIdx.x;
    const bool active = i < n;
    const int64_t g0 = g_first + chunk * chunk_len;
    const int64_t g1 = min(g0 + chunk_len, tab.n_groups);

    // resident Bloom bitmap
    if (load_filter) {
        const uint4 *gf = reinterpret_cast<const uint4 *>(sc.filter);
        for (int k = threadIdx.x; k < (fwords >> 2); k += blockDim.x) smem4[k] = gf[k];
    }

    Key<W> x;
    uint32_t hx = 0;
    double la = 0.0, ph = 0.0;
    uint64_t xa = 0, xb = 0;
    if (active) {
        x = load_key<W>(samples, i);
        hx = sc.shx[i];
        la = log_amp[i];
        ph = phase[i];
        if (SEC && *sc.mixed == 0) {
            xa = compress<W>(x, tab.spin_a0, tab.spin_a1);
            xb = compress<W>(x, tab.spin_b0, tab.spin_b1);
        }
    } else {
#pragma unroll
        for (int q = 0; q < W; ++q) x.w[q] = 0;
    }

    double acc_re = 0.0, acc_im = 0.0;              // FP64 form
    AccF32 fre, fim;                                // FP32 form
    unsigned long long n_hit = 0, n_terms = 0;      // per lane
    unsigned long long w_probe = 0, w_cand = 0;     // per wave (identical in all lanes)
    uint32_t qn = 0;  // queue length, identical in all lanes of the wave
    const uint32_t fmask = static_cast<uint32_t>(fwords - 1);
    const uint64_t amask = __ballot(active);  // lanes that own a sample

    // Look up queue entries [0, m): lane k takes entry k; hits go back to
    // the owning lanes in entry order.
    auto flush = [&](uint32_t m) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const uint32_t e = lane < static_cast<int>(m) ? queue[lane] : 0u;
        const int l = static_cast<int>(e & 63u);
        const int64_t g = g0 + static_cast<int64_t>(e >> 6);
        Key<W> xl;
#pragma unroll
        for (int q = 0; q < W; ++q) xl.w[q] = shfl_u64(x.w[q], l);
        const uint32_t hxl = __shfl(hx, l);
        const double lal = shfl_f64(la, l), phl = shfl_f64(ph, l);
        double cre = 0.0, cim = 0.0;
        float pre = 0.f, ere = 0.f, pim = 0.f, eim = 0.f;
        bool hit = false;
        if (lane < static_cast<int>(m)) {
            Key<W> xp;
#pragma unroll
            for (int q = 0; q < W; ++q) xp.w[q] = xl.w[q] ^ tab.gx[2 * g + q];
            const uint32_t h = hxl ^ tab.ghm[2 * g];
            const int32_t j = hash_find<W>(sc.skey, sc.sidx, sc.slot_mask,
                                           slot_of(h, sc.slot_shift) << bucket_log2(W), xp);
            if constexpr (DUMP) {
                if (hit_idx) hit_idx[(wave0 + l) * tab.n_groups + g] = j;
            }
            if (j >= 0) {
                hit = true;
                ++n_hit;
                if constexpr (P == NQS_FP64) {
                    uint32_t *row =
                        (DUMP && sign_bits) ? sign_bits + (wave0 + l) * sign_words : nullptr;
                    double hsum;
                    if constexpr (SCV) {
                        (void)row;
                        hsum = sc_element<W>(tab, xl, xp);
                    } else {
                        hsum = group_sum<W, DUMP>(tab, g, xl, row, &n_terms);
                    }
                    const double2 rat = amp_ratio_f64(log_amp[j] - lal, phase[j] - phl);
                    cre = hsum * rat.x;
                    cim = hsum * rat.y;
                } else {
                    const AccF32 hs = group_sum_f32<W>(tab, g, xl, &n_terms);
                    float rr, ri;
                    ratio_f32(log_amp[j] - lal, phase[j] - phl, rr, ri);
                    pre = hs.s * rr;
                    ere = fmaf(hs.s, rr, -pre) + hs.c * rr;
                    pim = hs.s * ri;
                    eim = fmaf(hs.s, ri, -pim) + hs.c * ri;
                }
            }
        }
        uint64_t hm = __ballot(hit);
        while (hm) {
            const int q = __builtin_ctzll(hm);
            hm &= hm - 1;
            const int owner = __builtin_amdgcn_readlane(l, q);
            if constexpr (P == NQS_FP64) {
                const double r = readlane_f64(cre, q);
                const double im = readlane_f64(cim, q);
                if (lane == owner) {
                    acc_re += r;
                    acc_im += im;
                }
            } else {
                const float a0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pre), q));
                const float a1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ere), q));
                const float b0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pim), q));
                const float b1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(eim), q));
                if (lane == owner) {
                    fre.add(a0, a1);
                    fim.add(b0, b1);
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    };

    // The sector test applies only when every sample of the batch has the
    // same (N_alpha, N_beta); the hash build reports that in *sc.mixed.
    auto run = [&](auto sec_c) {
        constexpr bool SECV = decltype(sec_c)::value;
        for (int64_t sg = g0; sg < g1; sg += kStage) {
            const int cnt = static_cast<int>(min(static_cast<int64_t>(kStage), g1 - sg));
            const int cnt_pad = (cnt + kUnroll - 1) / kUnroll * kUnroll;
            __syncthreads();
            for (int k = threadIdx.x; k < cnt_pad; k += blockDim.x) {
                const int64_t g = sg + k;
                Rec r;
                if (k < cnt) {
                    if constexpr (S32) {
                        r.ca = static_cast<uint32_t>(tab.gsec[2 * g]);
                        r.cb = static_cast<uint32_t>(tab.gsec[2 * g + 1]);
                    } else {
                        r.ca = tab.gsec[2 * g];
                        r.cb = tab.gsec[2 * g + 1];
                        r.pad0 = r.pad1 = 0;
                    }
                    r.hx = tab.ghm[2 * g];
                    r.key = tab.ghm[2 * g + 1];
                } else {
                    r.ca = 0;
                    r.cb = 0;
                    if constexpr (!S32) r.pad0 = r.pad1 = 0;
                    r.hx = 0;
                    r.key = kPadKey;
                }
                stage[k] = r;
            }
            __syncthreads();
            for (int k = 0; k < cnt_pad; k += kUnroll) {
                // phase 1: the records of kUnroll groups (wave-uniform LDS reads)
                Rec r[kUnroll];
    #pragma unroll
                for (int u = 0; u < kUnroll; ++u) r[u] = stage[k + u];
                // phase 2: filter words of the flipped samples
                uint32_t h[kUnroll], fw[kUnroll];
    #pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    h[u] = hx ^ r[u].hx;
                    fw[u] = filt[filter_word(h[u], fmask)];
                }
                // phase 3: sector test and filter bits
                uint64_t ins_m[kUnroll], cand_m[kUnroll];
    #pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    bool ins;
                    if constexpr (SECV) {
                        uint32_t ca, cb;
                        if constexpr (S32) {
                            ca = __popc(static_cast<uint32_t>(xa) & r[u].ca);
                            cb = __popc(static_cast<uint32_t>(xb) & r[u].cb);
                        } else {
                            ca = __popcll(xa & r[u].ca);
                            cb = __popcll(xb & r[u].cb);
                        }
                        ins = (ca | (cb << 8)) == r[u].key;
                    } else {
                        ins = r[u].key != kPadKey;
                    }
                    const bool bits = filter_test(fw[u], h[u]) != 0u;
                    ins_m[u] = __ballot(ins) & amask;
                    cand_m[u] = __ballot(ins && bits) & amask;
                }
    #pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    w_probe += static_cast<unsigned long long>(__popcll(ins_m[u]));
                    const uint64_t cm = cand_m[u];
                    if constexpr (DUMP) {
                        if (active && !((cm >> lane) & 1ull) && hit_idx && k + u < cnt)
                            hit_idx[i * tab.n_groups + sg + k + u] = -1;
                    }
                    if (cm) {
                        w_cand += static_cast<unsigned long long>(__popcll(cm));
                        if ((cm >> lane) & 1ull)
                            queue[qn + lanes_below(cm)] =
                                (static_cast<uint32_t>(sg + k + u - g0) << 6) | static_cast<uint32_t>(lane);
                        qn += static_cast<uint32_t>(__popcll(cm));
                        if (qn >= 64) {
                            flush(64);
                            qn -= 64;
                            if (lane < static_cast<int>(qn)) queue[lane] = queue[64 + lane];
                        }
                    }
                }
            }
        }
    };
    if constexpr (SEC) {
        if (*sc.mixed == 0)
            run(std::true_type{});
        else
            run(std::false_type{});
    } else {
        run(std::false_type{});
    }
    if (qn > 0) flush(qn);

    if (active) {
        double *p = sc.part + 2 * (chunk * n + i);
        if constexpr (P == NQS_FP64) {
            p[0] = acc_re;
            p[1] = acc_im;
        } else {
            p[0] = fre.value();
            p[1] = fim.value();
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        n_hit += __shfl_xor(n_hit, off);
        n_terms += __shfl_xor(n_terms, off);
    }
    if (lane == 0) {
        count_add(sc.counters, 1, w_probe);
        count_add(sc.counters, 2, n_hit);
        count_add(sc.counters, 3, n_terms);
        count_add(sc.counters, 4, w_cand);
    }
}

// ------------------------------------------------------------------ flip enumeration
//
// The second lookup strategy, for tables whose in-sector groups are all
// single and double excitations (molecular Hamiltonians, every qubit with a
// spin).  Instead of passing every X group by every sample and discarding
// the out-of-sector ones, a block builds each sample's occupied and virtual
// orbital lists and enumerates exactly its spin-conserving flips:
//   A  = (beta singles + none) x (alpha singles + none), without (none, none)
//   Ba = alpha occupied pairs x alpha virtual pairs
//   Bb = beta occupied pairs x beta virtual pairs
// Each product is laid out as rows x columns: 64 columns sit in the lanes'
// registers (their hash already XORed with h(x)), rows stream from LDS as
// wave-uniform reads, so one probe is one XOR plus the Bloom test of the
// streaming kernel.  Filter survivors go through the same per-wave queue
// into the global sample hash; a hit finds its group through the group
// index (or, in the integral form, evaluates Slater-Condon directly).
// The result equals the streaming kernel's up to the order of the hit sums:
// groups a sample cannot reach (sector test false) are never visited.
//
// Flip codes: four 7-bit qubit fields (0x7F = none), columns fill fields 0
// and 1, rows fields 2 and 3, the round slot of the sample sits in bits 28+.

// Base of the dynamic LDS of the running kernel.
__device__ __forceinline__ char *dyn_lds() {
    extern __shared__ uint4 nqs_dyn_lds[];
    return reinterpret_cast<char *>(nqs_dyn_lds);
}

constexpr uint32_t kNoQubit = 0x7Fu;
constexpr uint32_t kNoPair = kNoQubit | (kNoQubit << 7);
constexpr int kEnumRowSeg = 64;  // rows per work unit (two 32-row lane masks)

// Row segments of a product of nrow rows: at most 64 rows each, of equal
// length rounded up to a multiple of 4.
__device__ __forceinline__ int seg_len(int nrow) {
    const int ns = (nrow + kEnumRowSeg - 1) / kEnumRowSeg;
    return ns ? (((nrow + ns - 1) / ns) + 3) & ~3 : 0;
}

struct alignas(16) EnumSample {
    uint64_t x0, x1;
    double la, ph;
    int64_t idx;
    uint32_t hx;
    uint32_t cx;     // class of x: the filter partition that holds it
    uint32_t pad[2];
};
static_assert(sizeof(EnumSample) == 64, "one 64-byte record per sample");

// Per-sample bucket counts and offsets (128 bytes): beta occupied / virtual
// orbitals per class, and for each sorted list the start of each class
// bucket (entry offsets within the list, kEnumMaxParts + 1 each), and the
// work units of each partition.
struct EnumMeta {
    uint8_t nocc[kEnumMaxParts], nvir[kEnumMaxParts];
    uint16_t offa[kEnumMaxParts + 1];   // rows of A
    uint16_t offb[kEnumMaxParts + 1];   // rows of Bb
    uint16_t offc[kEnumMaxParts + 1];   // columns of Bb
    uint16_t units[kEnumMaxParts];      // work units of each partition
    uint16_t pad[1];
};
static_assert(sizeof(EnumMeta) <= 128, "metadata fits its 128 bytes");

struct EnumShape {
    int B;               // samples per round, 0 = enumeration not usable
    int parts;           // filter partitions (sample classes)
    int na, nb, va, vb;  // occupied / virtual orbitals per spin
    int ra, rba, rbb;    // rows of A, Ba, Bb
    int ca, cba, cbb;    // columns of A, Ba, Bb (cbb: the Bb column list)
    int la, lba, lbb;    // list offsets (entries): rows of A at 0, Ba, Bb, then Bb columns
    int lcb;
    int L;               // padded list entries per sample
    int n_task;          // solo rounds: (product, row segment, column) tasks per sample
    int solo;            // 1: solo rounds (one wave per sample)
};

__device__ __forceinline__ int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Shape of the rounds of this batch, from the first sample's occupation.
// Usable when the table allows it and the hash build found one sector.
__device__ __forceinline__ EnumShape enum_shape(const DevTable &tab, const DevScratch &sc,
                                                const uint64_t *__restrict__ samples, int64_t n) {
    EnumShape s{};
    if (!tab.enum_ok || n <= 0 || *sc.mixed != 0) return s;
    const uint64_t w0 = samples[0], w1 = samples[1];
    s.na = __popcll(w0 & tab.spin_a0) + __popcll(w1 & tab.spin_a1);
    s.nb = __popcll(w0 & tab.spin_b0) + __popcll(w1 & tab.spin_b1);
    s.va = tab.k_alpha - s.na;
    s.vb = tab.k_beta - s.nb;
    s.B = enum_round_size(tab.k_alpha, tab.k_beta, s.na, s.nb);
    s.parts = 1 << sc.eparts_log2;
    s.ra = 1 + s.nb * s.vb;
    s.ca = 1 + s.na * s.va;
    s.rba = enum_pairs(s.na);
    s.cba = enum_pairs(s.va);
    s.rbb = enum_pairs(s.nb);
    s.cbb = enum_pairs(s.vb);
    s.la = 0;
    s.lba = enum_pad4(s.ra);
    s.lbb = s.lba + enum_pad4(s.rba);
    s.lcb = s.lbb + enum_pad4(s.rbb);
    s.L = s.lcb + enum_pad4(s.cbb);
    // solo rounds keep only the row lists (entries [0, lcb)) per wave, then
    // the block's pair table and task table
    s.n_task = ceil_div(s.ra, kEnumRowSeg) * s.ca + ceil_div(s.rba, kEnumRowSeg) * s.cba +
               ceil_div(s.rbb, kEnumRowSeg) * s.cbb;
    s.solo = (s.parts == 1 && tab.k_alpha <= 32 && tab.k_beta <= 32 &&
              enum_solo_task_off(s.lcb) + 4 * 64 * ceil_div(s.n_task, 64) <= kEnumDynLds) ? 1 : 0;
    return s;
}

// The shape as scalar values (its inputs may come through vector loads).
__device__ __forceinline__ EnumShape uniform_shape(EnumShape s) {
    int *f = reinterpret_cast<int *>(&s);
#pragma unroll
    for (int k = 0; k < static_cast<int>(sizeof(EnumShape) / sizeof(int)); ++k)
        f[k] = __builtin_amdgcn_readfirstlane(f[k]);
    return s;
}

// k-th pair (i < j) in the order (0,1), (0,2), (1,2), (0,3), ...: j is the
// largest with j (j - 1) / 2 <= k, from a float square root corrected by one
// step each way (exact for the k < 2016 of orbital lists of up to 64).
__device__ __forceinline__ void pair_of(int k, int &i, int &j) {
    int jj = static_cast<int>((1.0f + sqrtf(static_cast<float>(8 * k + 1))) * 0.5f);
    if (jj * (jj - 1) / 2 > k) --jj;
    if ((jj + 1) * jj / 2 <= k) ++jj;
    j = jj;
    i = k - jj * (jj - 1) / 2;
}

struct EnumCounts {
    unsigned long long probes = 0, cand = 0, rounds = 0;  // wave-uniform
    unsigned long long hits = 0, terms = 0;               // per lane
};

// Outcome of one queued candidate: whether x' is a sample with a group
// (a hit), and its contribution H_xx' psi(x')/psi(x), in FP64 (re, im) or
// in FP32 with the rounding errors kept (pre + ere, pim + eim).
struct EnumHit {
    bool hit = false;
    double re = 0.0, im = 0.0;
    float pre = 0.f, ere = 0.f, pim = 0.f, eim = 0.f;
};

// Fingerprints of one bucket: 8 (one-word keys, a and b) or 4 (two-word
// keys, a only).  The candidates load those of the first bucket of x' ahead
// of their lookups.
struct FpBucket {
    uint4 a, b;
};

template <int W>
__device__ __forceinline__ FpBucket enum_candidate_bucket(const DevScratch &sc, uint2 e) {
    const uint4 *p = reinterpret_cast<const uint4 *>(
        sc.sfp + (slot_of(e.y, sc.slot_shift) << bucket_log2(W)));
    FpBucket f;
    f.a = p[0];
    if constexpr (W == 1) f.b = p[1];
    else f.b = make_uint4(0u, 0u, 0u, 0u);
    return f;
}

// Whether a key of hash h may sit in the bucket (a fingerprint equals
// h | 1), and whether the bucket is open (its last slot free): a key that is
// present sits in its first bucket unless that bucket is full.
template <int W>
__device__ __forceinline__ bool fp_settles_miss(const FpBucket &f, uint32_t h) {
    const uint32_t w = h | 1u;
    uint32_t d = min(min(f.a.x ^ w, f.a.y ^ w), min(f.a.z ^ w, f.a.w ^ w));
    uint32_t last = f.a.w;
    if constexpr (W == 1) {
        d = min(d, min(min(f.b.x ^ w, f.b.y ^ w), min(f.b.z ^ w, f.b.w ^ w)));
        last = f.b.w;
    }
    return d != 0u && last == 0u;
}

// Candidate e = (flip code, h(x')) of sample x (hash hx, log amplitude la,
// phase ph, index idx), the fingerprints of the first bucket of x' already
// loaded (f0): look x' = x ^ X up in the sample hash and, on a hit, find its
// group (or evaluate Slater-Condon) and the amplitude ratio; c is left as it
// is (no hit) otherwise.
template <int W, bool DUMP, int P, bool SCV>
__device__ __forceinline__ void enum_candidate(
    const DevTable &tab, const DevScratch &sc,
    const Key<W> &x, uint32_t hx, double la, double ph, int64_t idx, uint2 e, const FpBucket &f0,
    const double *__restrict__ log_amp, const double *__restrict__ phase,
    int32_t *__restrict__ hit_idx, uint32_t *__restrict__ sign_bits, int64_t sign_words,
    EnumCounts &cnt, EnumHit &c) {
    // nearly every candidate is a filter false positive: its fingerprints
    // settle it before the flips are decoded or any key is read
    if (fp_settles_miss<W>(f0, e.y)) return;
    Key<W> X;
#pragma unroll
    for (int q = 0; q < W; ++q) X.w[q] = 0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const uint32_t q = (e.x >> (7 * f)) & kNoQubit;
        if (q != kNoQubit) {
            if constexpr (W == 1) {
                X.w[0] |= 1ull << q;
            } else {
                // constant indices keep X in registers
                const uint64_t bit = 1ull << (q & 63);
                if (q < 64) X.w[0] |= bit; else X.w[1] |= bit;
            }
        }
    }
    Key<W> xp;
#pragma unroll
    for (int q = 0; q < W; ++q) xp.w[q] = x.w[q] ^ X.w[q];
    const int32_t j = hash_find<W>(sc.skey, sc.sidx, sc.slot_mask,
                                   slot_of(e.y, sc.slot_shift) << bucket_log2(W), xp);
    if (j < 0) return;
    int64_t g = -1;
    if (!SCV || DUMP) g = group_find<W>(tab, e.y ^ hx, X);
    if constexpr (DUMP) {
        if (hit_idx && g >= 0) hit_idx[idx * tab.n_groups + g] = j;
    }
    if (!SCV && g < 0) return;
    c.hit = true;
    ++cnt.hits;
    if constexpr (P == NQS_FP64) {
        uint32_t *row = (DUMP && sign_bits) ? sign_bits + idx * sign_words : nullptr;
        double hsum;
        if constexpr (SCV) {
            (void)row;
            hsum = sc_element<W>(tab, x, xp);
        } else {
            hsum = group_sum<W, DUMP>(tab, g, x, row, &cnt.terms);
        }
        // (inline: this kernel's occupancy is set by its LDS, and a call
        // would only add a stack)
        double sn, cs;
        sincos(phase[j] - ph, &sn, &cs);
        const double mag = exp(log_amp[j] - la);
        c.re = hsum * (mag * cs);
        c.im = hsum * (mag * sn);
    } else {
        const AccF32 hs = group_sum_f32<W>(tab, g, x, &cnt.terms);
        float rr, ri;
        ratio_f32(log_amp[j] - la, phase[j] - ph, rr, ri);
        c.pre = hs.s * rr;
        c.ere = fmaf(hs.s, rr, -c.pre) + hs.c * rr;
        c.pim = hs.s * ri;
        c.eim = fmaf(hs.s, ri, -c.pim) + hs.c * ri;
    }
}

// Position of the pair (i < j) of a class-sorted orbital list in the pair
// list sorted by pair class (u ^ w): bucket s holds the blocks of class
// pairs (u, u ^ s), u <= u ^ s, in increasing u; pairs inside one class come
// in pair_of order, pairs across two classes row-major.
__device__ __forceinline__ int sorted_pair_pos(const uint8_t *cnt, const uint16_t *off, int parts,
                                               int i, int j, int u, int w) {
    int start_u = 0, start_w = 0;
    for (int c = 0; c < parts; ++c) {
        start_u += c < u ? cnt[c] : 0;
        start_w += c < w ? cnt[c] : 0;
    }
    const int s = u ^ w;
    int pre = 0;
    for (int c = 0; c < u; ++c) {
        const int d = c ^ s;
        if (s == 0) pre += enum_pairs(cnt[c]);
        else if (c < d) pre += cnt[c] * cnt[d];
    }
    const int il = i - start_u, jl = j - start_w;
    const int loc = (s == 0) ? jl * (jl - 1) / 2 + il : il * cnt[w] + jl;
    return off[s] + pre + loc;
}

// Rows [0, m) of rw (m at most 32) against the column hash, in groups of
// four (rows past m are probed too and left to the caller's mask): bit r of
// the result is the filter outcome of row r.  Each outcome is funnelled in at
// bit 31 (one alignbit per row, no masking of the shifted filter word), so
// the word ends up shifted by 32 less the rows probed.  Rows go two groups
// of four at a time: eight filter reads in flight per lane.
template <bool A16>
__device__ __forceinline__ uint4 row_group(const uint32_t *rw, int r) {
    if constexpr (A16) {
        return reinterpret_cast<const uint4 *>(rw)[r >> 2];
    } else {
        return make_uint4(rw[r], rw[r + 1], rw[r + 2], rw[r + 3]);
    }
}

__device__ __forceinline__ void filter_words(const char *filt_b, uint32_t fbytes_mask,
                                             const uint32_t h[4], uint32_t fw[4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
        // the filter word of h, as a byte offset
        fw[v] = *reinterpret_cast<const uint32_t *>(filt_b + (h[v] & fbytes_mask));
}

__device__ __forceinline__ uint32_t filter_funnel(uint32_t pm, const uint32_t h[4],
                                                  const uint32_t fw[4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
        pm = __builtin_amdgcn_alignbit((fw[v] >> ((h[v] >> 17) & 31)) &
                                           (fw[v] >> ((h[v] >> 24) & 31)),
                                       pm, 1u);
    return pm;
}

template <bool A16>
__device__ __forceinline__ void row_hashes(const uint32_t *rw, int r, uint32_t colh, uint32_t h[4]) {
    const uint4 q = row_group<A16>(rw, r);
    h[0] = colh ^ q.x;
    h[1] = colh ^ q.y;
    h[2] = colh ^ q.z;
    h[3] = colh ^ q.w;
}

template <bool A16>
__device__ __forceinline__ uint32_t probe_half(const char *filt_b, uint32_t fbytes_mask,
                                               uint32_t colh, const uint32_t *rw, int m) {
    uint32_t pm = 0;
    int r = 0;
    for (; r + 8 <= m; r += 8) {
        uint32_t ha[4], hb[4], fa[4], fb[4];
        row_hashes<A16>(rw, r, colh, ha);
        row_hashes<A16>(rw, r + 4, colh, hb);
        filter_words(filt_b, fbytes_mask, ha, fa);
        filter_words(filt_b, fbytes_mask, hb, fb);
        pm = filter_funnel(pm, ha, fa);
        pm = filter_funnel(pm, hb, fb);
    }
    for (; r < m; r += 4) {
        uint32_t ha[4], fa[4];
        row_hashes<A16>(rw, r, colh, ha);
        filter_words(filt_b, fbytes_mask, ha, fa);
        pm = filter_funnel(pm, ha, fa);
    }
    // r rows went in (m rounded up to 4)
    return r > 0 ? pm >> (32 - r) : 0u;
}

// Filter test of the rows [0, nrl) of a work unit (nrl <= 64, row hashes at
// rw, this lane's own rows [0, nr)) against this lane's column hash (h(x)
// and the column's flips folded in): bit r of the result is the outcome of
// row r, rows past nr (read from the next list or the padding) masked off.
// excl drops row 0 (the probe of x itself).  A16: rw is 16-byte aligned
// (one LDS read per 4 rows).
template <bool A16>
__device__ __forceinline__ uint64_t probe_rows(const char *filt_b, uint32_t fbytes_mask,
                                               uint32_t colh, const uint32_t *rw, int nrl, int nr,
                                               bool act, bool excl) {
    const int m0 = min(nrl, 32);
    const uint32_t pm0 = probe_half<A16>(filt_b, fbytes_mask, colh, rw, m0);
    const uint32_t pm1 = probe_half<A16>(filt_b, fbytes_mask, colh, rw + 32, nrl - m0);
    const int n0 = min(nr, 32), n1 = nr - n0;
    uint32_t keep0 = n0 >= 32 ? 0xFFFFFFFFu : ((1u << n0) - 1u);
    uint32_t keep1 = n1 >= 32 ? 0xFFFFFFFFu : ((1u << n1) - 1u);
    if (!act) keep0 = keep1 = 0u;
    if (excl) keep0 &= ~1u;
    return (static_cast<uint64_t>(pm1 & keep1) << 32) | (pm0 & keep0);
}


// One round: samples [round * B, round * B + B) of the batch, all filter
// partitions in turn (with one partition its filter is already in LDS).
// Partial sums of the hits go to sc.part[i] in a fixed order: per wave in
// queue order, then over the waves in wave order.
template <int W, bool DUMP, int P, bool SCV>
__device__ __forceinline__ void enum_round(uint32_t *filt, const DevTable &tab,
                                           const DevScratch &sc, const EnumShape &S,
                                           const uint64_t *__restrict__ samples,
                                           const double *__restrict__ log_amp,
                                           const double *__restrict__ phase, int64_t n,
                                           int64_t round, int32_t *__restrict__ hit_idx,
                                           uint32_t *__restrict__ sign_bits, int64_t sign_words,
                                           EnumCounts &cnt, int &loaded_part) {
    char *smem = dyn_lds();
    const int lane = threadIdx.x & 63;
    // wave-uniform (scalar) so that unit and row loops run on the scalar unit
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int parts = S.parts;
    uint32_t *hr = reinterpret_cast<uint32_t *>(smem);
    uint8_t *qcl = reinterpret_cast<uint8_t *>(smem + 512);
    uint2 *queue = reinterpret_cast<uint2 *>(smem + kEnumQueueOff) + wave * kEnumQueue;
    char *per = smem + kEnumDynFixed;
    const int B = S.B;
    const int L = S.L;
    EnumSample *smp = reinterpret_cast<EnumSample *>(per);
    uint8_t *ov = reinterpret_cast<uint8_t *>(per + 64 * B);                      // [B][256]
    char *accb = per + 320 * B;                                                    // [B][16][16 B]
    EnumMeta *meta = reinterpret_cast<EnumMeta *>(per + 320 * B + kEnumWaves * 16 * B);  // [B]
    // row hashes in LDS [B][Lr]; in the block's device area the flip codes
    // of all four lists [B][L] and the Bb column hashes [B][Lc]
    const int Lr = S.lcb, Lc = L - S.lcb;
    uint32_t *lh = reinterpret_cast<uint32_t *>(per + kEnumPerSampleFixed * B);
    char *blk = sc.eblk + static_cast<int64_t>(blockIdx.x) * sc.eblk_stride;
    uint16_t *lc = reinterpret_cast<uint16_t *>(blk);
    uint32_t *lch = reinterpret_cast<uint32_t *>(blk + enum_blk_codes_bytes(B, L));

    const int64_t s0 = round * B;
    const int nb = static_cast<int>(min(static_cast<int64_t>(B), n - s0));
    if (nb <= 0) return;
    if (blockIdx.x >= sc.eblk_blocks) {
        // no device area for this block (the grids have one block per CU)
        if (threadIdx.x == 0) latch(sc.err, NQS_E_STATE);
        return;
    }
    ++cnt.rounds;
    const uint32_t pmask = static_cast<uint32_t>(parts - 1);

    // stage 1: records, alpha lists, beta lists sorted by class (stable),
    // class counts, bucket offsets and work units; one wave per sample
    for (int b = wave; b < nb; b += kEnumWaves) {
        const int64_t i = s0 + b;
        const uint64_t w0 = samples[2 * i], w1 = samples[2 * i + 1];
        uint8_t *o = ov + 256 * b;
        EnumMeta &m = meta[b];
        uint32_t cx = 0;
        int my_no = 0, my_nv = 0;
        {
            const bool in = lane < tab.k_alpha;
            const int q = in ? tab.spin_q[lane] : 0;
            const bool occ = in && (((q < 64 ? w0 : w1) >> (q & 63)) & 1ull);
            const uint64_t mo = __ballot(occ), mv = __ballot(in && !occ);
            if (occ) o[lanes_below(mo)] = static_cast<uint8_t>(q);
            if (in && !occ) o[64 + lanes_below(mv)] = static_cast<uint8_t>(q);
        }
        {
            const bool in = lane < tab.k_beta;
            const int q = in ? tab.spin_q[64 + lane] : 0;
            const bool occ = in && (((q < 64 ? w0 : w1) >> (q & 63)) & 1ull);
            const uint32_t c = in ? (qcl[q] & pmask) : 0u;
            int no = 0, nv = 0;
            for (int u = 0; u < parts; ++u) {
                const uint64_t mo = __ballot(occ && c == static_cast<uint32_t>(u));
                const uint64_t mv = __ballot(in && !occ && c == static_cast<uint32_t>(u));
                if (occ && c == static_cast<uint32_t>(u)) o[128 + no + lanes_below(mo)] = static_cast<uint8_t>(q);
                if (in && !occ && c == static_cast<uint32_t>(u))
                    o[192 + nv + lanes_below(mv)] = static_cast<uint8_t>(q);
                if (lane == u) {
                    // lane u keeps the class-u counts
                    my_no = __popcll(mo);
                    my_nv = __popcll(mv);
                    m.nocc[u] = static_cast<uint8_t>(my_no);
                    m.nvir[u] = static_cast<uint8_t>(my_nv);
                }
                no += __popcll(mo);
                nv += __popcll(mv);
            }
            uint32_t v = occ ? c : 0u;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v ^= __shfl_xor(v, off);
            cx = v;
        }
        if (lane == 0) {
            EnumSample r;
            r.x0 = w0;
            r.x1 = w1;
            r.la = log_amp[i];
            r.ph = phase[i];
            r.idx = i;
            r.hx = sc.shx[i];
            r.cx = cx;
            r.pad[0] = r.pad[1] = 0;
            smp[b] = r;
        }
        if (lane < kEnumWaves) reinterpret_cast<uint4 *>(accb + kEnumWaves * 16 * b)[lane] =
            make_uint4(0u, 0u, 0u, 0u);
        // bucket sizes, offsets and work units, one lane per (t, u) pair of
        // classes: lane 8 t + u
        {
            const int gt = lane >> 3, gu = lane & 7;
            const bool gin = gt < parts && gu < parts;
            const int gd = (gu ^ gt) & 7;
            const int no_u = __shfl(my_no, gu), nv_u = __shfl(my_nv, gu);
            const int no_d = __shfl(my_no, gd), nv_d = __shfl(my_nv, gd);
            // bucket t of A rows: beta singles u -> u ^ t; of Bb rows / columns:
            // occupied / virtual pairs of classes (u, u ^ t)
            int sa = gin ? no_u * nv_d : 0, sb = 0, scc = 0;
            if (gin) {
                if (gt == 0) {
                    sb = enum_pairs(no_u);
                    scc = enum_pairs(nv_u);
                } else if (gu < gd) {
                    sb = no_u * no_d;
                    scc = nv_u * nv_d;
                }
            }
#pragma unroll
            for (int off = 1; off < 8; off <<= 1) {
                sa += __shfl_xor(sa, off);
                sb += __shfl_xor(sb, off);
                scc += __shfl_xor(scc, off);
            }
            if (gt == 0) sa += 1;  // the none row opens bucket 0 of A
            // every lane of group t holds the sizes of bucket t; offsets are
            // the sums over the buckets before t
            const int sa_u = __shfl(sa, 8 * gu), sb_u = __shfl(sb, 8 * gu), sc_u = __shfl(scc, 8 * gu);
            int pa = (gu < gt && gu < parts) ? sa_u : 0;
            int pb = (gu < gt && gu < parts) ? sb_u : 0;
            int pc = (gu < gt && gu < parts) ? sc_u : 0;
#pragma unroll
            for (int off = 1; off < 8; off <<= 1) {
                pa += __shfl_xor(pa, off);
                pb += __shfl_xor(pb, off);
                pc += __shfl_xor(pc, off);
            }
            if (gu == 0 && gt < parts) {
                m.offa[gt] = static_cast<uint16_t>(pa);
                m.offb[gt] = static_cast<uint16_t>(pb);
                m.offc[gt] = static_cast<uint16_t>(pc);
                if (gt == parts - 1) {
                    m.offa[parts] = static_cast<uint16_t>(pa + sa);
                    m.offb[parts] = static_cast<uint16_t>(pb + sb);
                    m.offc[parts] = static_cast<uint16_t>(pc + scc);
                }
            }
            // work units of partition p (lane group p): A rows of bucket t =
            // p ^ cx against all alpha columns, Ba when t = 0, and Bb column
            // bucket v against row bucket t ^ v
            const int t = (gt ^ static_cast<int>(cx)) & 7;
            const int sc_v = __shfl(scc, 8 * gu), sb_tv = __shfl(sb, 8 * ((t ^ gu) & 7));
            const int sa_t = __shfl(sa, 8 * t);
            int un = gin ? ceil_div(sc_v, 64) * ceil_div(sb_tv, kEnumRowSeg) : 0;
#pragma unroll
            for (int off = 1; off < 8; off <<= 1) un += __shfl_xor(un, off);
            if (gu == 0 && gt < parts) {
                const int cha = ceil_div(S.ca, 64);
                const int uba =
                    (S.rba && S.cba) ? ceil_div(S.cba, 64) * ceil_div(S.rba, kEnumRowSeg) : 0;
                un += cha * ceil_div(sa_t, kEnumRowSeg) + (t == 0 ? uba : 0);
                m.units[gt] = static_cast<uint16_t>(un);
            }
        }
    }
    __syncthreads();

    // stage 3: list entries (hash, code) at their sorted positions
    const int E = S.ra + S.rba + S.rbb + S.cbb;
    for (int t = threadIdx.x; t < nb * E; t += blockDim.x) {
        const int b = t / E;
        int e = t - b * E;
        const uint8_t *o = ov + 256 * b;
        const EnumMeta &m = meta[b];
        uint32_t qa, qb;
        int pos;
        if (e < S.ra) {
            if (e == 0) {
                lh[b * Lr] = 0u;
                lc[b * L] = static_cast<uint16_t>(kNoPair);
                continue;
            }
            // beta single (occupied i -> virtual a), both in class order
            const int k = e - 1;
            const int ii = k / S.vb, aa = k - ii * S.vb;
            qa = o[128 + ii];
            qb = o[192 + aa];
            const int u = qcl[qa] & pmask, d = qcl[qb] & pmask, tt = u ^ d;
            int su = 0, sd = 0, pre = 0;
            for (int c = 0; c < parts; ++c) {
                su += c < u ? m.nocc[c] : 0;
                sd += c < d ? m.nvir[c] : 0;
                pre += c < u ? m.nocc[c] * m.nvir[c ^ tt] : 0;
            }
            pos = S.la + m.offa[tt] + (tt == 0 ? 1 : 0) + pre + (ii - su) * m.nvir[d] + (aa - sd);
        } else if ((e -= S.ra) < S.rba) {
            int ii, jj;
            pair_of(e, ii, jj);
            qa = o[ii];
            qb = o[jj];
            pos = S.lba + e;
        } else if ((e -= S.rba) < S.rbb) {
            int ii, jj;
            pair_of(e, ii, jj);
            qa = o[128 + ii];
            qb = o[128 + jj];
            pos = S.lbb + sorted_pair_pos(m.nocc, m.offb, parts, ii, jj, qcl[qa] & pmask,
                                          qcl[qb] & pmask);
        } else {
            e -= S.rbb;
            int ii, jj;
            pair_of(e, ii, jj);
            qa = o[192 + ii];
            qb = o[192 + jj];
            pos = S.lcb + sorted_pair_pos(m.nvir, m.offc, parts, ii, jj, qcl[qa] & pmask,
                                          qcl[qb] & pmask);
        }
        const uint32_t hv = hr[qa] ^ hr[qb];
        if (pos < Lr) lh[b * Lr + pos] = hv;
        else lch[b * Lc + pos - Lr] = hv;
        lc[b * L + pos] = static_cast<uint16_t>(qa | (qb << 7));
    }
    __syncthreads();

    // stage 4: probes, partition by partition; work units round-robin over
    // the waves
    uint32_t qn = 0;

    auto flush = [&](uint32_t mcount) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const uint2 e = lane < static_cast<int>(mcount) ? queue[lane] : make_uint2(0u, 0u);
        const int b = static_cast<int>(e.x >> 28);
        EnumHit c;
        if (lane < static_cast<int>(mcount)) {
            const FpBucket f = enum_candidate_bucket<W>(sc, e);
            if (!fp_settles_miss<W>(f, e.y)) {
                // the row's code from its list position
                const uint32_t pos = (e.x >> 14) & 0x3FFFu;
                const uint32_t rc = lc[b * L + static_cast<int>(pos)];
                const uint2 ef = make_uint2((e.x & 0xF0003FFFu) | (rc << 14), e.y);
                const EnumSample rec = smp[b];
                Key<W> x;
                x.w[0] = rec.x0;
                if constexpr (W == 2) x.w[1] = rec.x1;
                enum_candidate<W, DUMP, P, SCV>(tab, sc, x, rec.hx, rec.la, rec.ph, rec.idx, ef, f,
                                                log_amp, phase, hit_idx, sign_bits, sign_words,
                                                cnt, c);
            }
        }
        const bool hit = c.hit;
        const double cre = c.re, cim = c.im;
        const float pre = c.pre, ere = c.ere, pim = c.pim, eim = c.eim;
        uint64_t hm = __ballot(hit);
        while (hm) {
            const int q = __builtin_ctzll(hm);
            hm &= hm - 1;
            const int bq = __builtin_amdgcn_readlane(b, q);
            char *slot = accb + kEnumWaves * 16 * bq + 16 * wave;
            if constexpr (P == NQS_FP64) {
                const double r = readlane_f64(cre, q);
                const double im = readlane_f64(cim, q);
                if (lane == 0) {
                    double *a = reinterpret_cast<double *>(slot);
                    a[0] += r;
                    a[1] += im;
                }
            } else {
                const float a0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pre), q));
                const float a1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ere), q));
                const float b0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pim), q));
                const float b1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(eim), q));
                if (lane == 0) {
                    float *a = reinterpret_cast<float *>(slot);  // re.s, re.c, im.s, im.c
                    AccF32 ar, ai;
                    ar.s = a[0]; ar.c = a[1]; ai.s = a[2]; ai.c = a[3];
                    ar.add(a0, a1);
                    ai.add(b0, b1);
                    a[0] = ar.s; a[1] = ar.c; a[2] = ai.s; a[3] = ai.c;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    };

    const uint32_t fbytes_mask = ((1u << sc.efilter_log2) - 1u) << 2;
    const char *filt_b = reinterpret_cast<const char *>(filt);
    const int cha = ceil_div(S.ca, 64);
    const int nseg_ba = ceil_div(S.rba, kEnumRowSeg);
    const int uba = (S.rba && S.cba) ? ceil_div(S.cba, 64) * nseg_ba : 0;
    for (int pi = 0; pi < parts; ++pi) {
        // odd rounds walk the partitions backwards: a round starts with the
        // partition the previous one ended with
        const int p = (round & 1) ? parts - 1 - pi : pi;
        if (parts > 1 && p != loaded_part) {
            // partition p of the filter: samples of class p
            __syncthreads();
            const uint4 *gf = reinterpret_cast<const uint4 *>(
                sc.efilter + (static_cast<size_t>(p) << sc.efilter_log2));
            uint4 *f4 = reinterpret_cast<uint4 *>(filt);
            const int n4 = (1 << sc.efilter_log2) >> 2;
            // eight 16-byte loads in flight per thread: a whole 128 KB
            // partition in one memory round trip
            int k = static_cast<int>(threadIdx.x);
            for (; k + 7 * kEnumThreads < n4; k += 8 * kEnumThreads) {
                const uint4 a0 = gf[k], a1 = gf[k + kEnumThreads];
                const uint4 a2 = gf[k + 2 * kEnumThreads], a3 = gf[k + 3 * kEnumThreads];
                const uint4 a4 = gf[k + 4 * kEnumThreads], a5 = gf[k + 5 * kEnumThreads];
                const uint4 a6 = gf[k + 6 * kEnumThreads], a7 = gf[k + 7 * kEnumThreads];
                f4[k] = a0;
                f4[k + kEnumThreads] = a1;
                f4[k + 2 * kEnumThreads] = a2;
                f4[k + 3 * kEnumThreads] = a3;
                f4[k + 4 * kEnumThreads] = a4;
                f4[k + 5 * kEnumThreads] = a5;
                f4[k + 6 * kEnumThreads] = a6;
                f4[k + 7 * kEnumThreads] = a7;
            }
            for (; k < n4; k += kEnumThreads) f4[k] = gf[k];
            __syncthreads();
            loaded_part = p;
        }
        int U = 0;
        for (int b = 0; b < nb; ++b) U += meta[b].units[p];
        U = __builtin_amdgcn_readfirstlane(U);
        int ub = 0, bb = 0;  // first unit of sample bb
        for (int u = wave; u < U; u += kEnumWaves) {
            // sample of unit u (units are sample-major)
            while (u >= ub + meta[bb].units[p]) {
                ub += meta[bb].units[p];
                ++bb;
            }
            const int b = __builtin_amdgcn_readfirstlane(bb);
            int l = u - __builtin_amdgcn_readfirstlane(ub);
            const EnumMeta &m = meta[b];
            const uint8_t *o = ov + 256 * b;
            const int t = p ^ static_cast<int>(smp[b].cx);
            // unit l of sample b: product, column chunk, row segment
            int prod, ch, seg, ncol, col0 = 0, row0, nrow;
            const int nra = m.offa[t + 1] - m.offa[t];
            const int ua = cha * ceil_div(nra, kEnumRowSeg);
            int ns;
            if (l < ua) {
                prod = 0;
                ns = ceil_div(nra, kEnumRowSeg);
                ch = l / ns;
                seg = l - ch * ns;
                ncol = S.ca;
                row0 = S.la + m.offa[t];
                nrow = nra;
            } else if (t == 0 && l < ua + uba) {
                prod = 1;
                l -= ua;
                ns = nseg_ba;
                ch = l / nseg_ba;
                seg = l - ch * nseg_ba;
                ncol = S.cba;
                row0 = S.lba;
                nrow = S.rba;
            } else {
                prod = 2;
                l -= ua + (t == 0 ? uba : 0);
                int v = 0, uv = 0;
                ns = 1;
                for (; v < parts; ++v) {
                    const int nc = m.offc[v + 1] - m.offc[v];
                    nrow = m.offb[(t ^ v) + 1] - m.offb[t ^ v];
                    ns = ceil_div(nrow, kEnumRowSeg);
                    uv = ceil_div(nc, 64) * ns;
                    if (l < uv) break;
                    l -= uv;
                }
                ch = l / ns;
                seg = l - ch * ns;
                ncol = m.offc[v + 1] - m.offc[v];
                col0 = S.lcb + m.offc[v];
                row0 = S.lbb + m.offb[t ^ v];
            }
            const int k = ch * 64 + lane;
            const bool act = k < ncol;
            // this lane's column: hash (with h(x)) and code in fields 0 and 1
            uint32_t colh = 0, colc = kNoPair;
            if (act) {
                if (prod == 2) {
                    colh = lch[b * Lc + col0 - Lr + k];
                    colc = lc[b * L + col0 + k];
                } else {
                    uint32_t qa = kNoQubit, qb = kNoQubit;
                    if (prod == 0) {
                        if (k > 0) {
                            const int e = k - 1;
                            const int ii = e / S.va;
                            qa = o[ii];
                            qb = o[64 + (e - ii * S.va)];
                        }
                    } else {
                        int ii, jj;
                        pair_of(k, ii, jj);
                        qa = o[64 + ii];
                        qb = o[64 + jj];
                    }
                    if (qa != kNoQubit) {
                        colh = hr[qa] ^ hr[qb];
                        colc = qa | (qb << 7);
                    }
                }
            }
            colh ^= smp[b].hx;
            colc |= static_cast<uint32_t>(b) << 28;
            const uint64_t colmask = __ballot(act);
            // (none, none) is x itself: never a probe
            const bool excl0 = prod == 0 && t == 0 && ch == 0 && seg == 0;
            // ns segments of equal length (a multiple of 4, at most 64)
            const int sl = (ceil_div(nrow, ns) + 3) & ~3;
            const int r0 = seg * sl;
            const int nr = min(nrow - r0, sl);
            const uint32_t *rw = lh + b * Lr + row0 + r0;
            // queue entry of row rr: its list position in place of its code
            const uint32_t colq = colc | (static_cast<uint32_t>(row0 + r0) << 14);
            cnt.probes += static_cast<unsigned long long>(__popcll(colmask)) * nr -
                          (excl0 ? 1ull : 0ull);
            uint64_t pm = probe_rows<false>(filt_b, fbytes_mask, colh, rw, nr, nr, act,
                                            excl0 && lane == 0);
            // filter survivors into the queue
            for (;;) {
                const uint64_t any = __ballot(pm != 0ull);
                if (!any) break;
                const bool has = pm != 0ull;
                const int bit = has ? __builtin_ctzll(pm) : 0;
                const int rr = bit;
                pm &= pm - 1ull;
                const uint32_t c = static_cast<uint32_t>(__popcll(any));
                cnt.cand += c;
                if (qn + c > static_cast<uint32_t>(kEnumQueue)) {
                    flush(qn);
                    qn = 0;
                }
                if (has)
                    queue[qn + lanes_below(any)] =
                        make_uint2(colq + (static_cast<uint32_t>(rr) << 14), colh ^ rw[rr]);
                qn += c;
            }
        }
    }
    if (qn > 0) flush(qn);
    __syncthreads();

    // stage 5: per-sample partial, waves in order
    if (threadIdx.x < static_cast<unsigned>(nb)) {
        const int b = threadIdx.x;
        const char *a = accb + kEnumWaves * 16 * b;
        double *pp = sc.part + 2 * (s0 + b);
        if constexpr (P == NQS_FP64) {
            double re = 0.0, im = 0.0;
            for (int w = 0; w < kEnumWaves; ++w) {
                re += reinterpret_cast<const double *>(a + 16 * w)[0];
                im += reinterpret_cast<const double *>(a + 16 * w)[1];
            }
            pp[0] = re;
            pp[1] = im;
        } else {
            AccF32 ar, ai;
            for (int w = 0; w < kEnumWaves; ++w) {
                const float *f = reinterpret_cast<const float *>(a + 16 * w);
                ar.add(f[0], f[1]);
                ai.add(f[2], f[3]);
            }
            pp[0] = ar.value();
            pp[1] = ai.value();
        }
    }
    __syncthreads();
}

// floor(a / b) for 0 <= a < 2^22 and b >= 1, with inv = 1.0f / b: the
// quotient (a + 1/2) / b lies at least 1 / (2 b) from an integer, more than
// the two float roundings of the product (at most (a + 1/2) / b * 2^-23).
__device__ __forceinline__ int div_small(int a, float inv) {
    return static_cast<int>((static_cast<float>(a) + 0.5f) * inv);
}

// Solo rounds: round r gives sample r * 16 + w to wave w, for r = first,
// first + step, ...  Each wave builds its own sample's lists and probes its
// products as tasks (product, row segment of at most 64 rows, column), 64
// tasks at a time, one per lane: a chunk may mix products, so that lanes are
// not left idle by column counts short of a multiple of 64.  Hits are added
// in queue order into registers; there is no block barrier, so one wave's
// memory waits overlap the other waves' probes.  The row lists of A, Ba and
// Bb (hash and flip code) sit in the wave's LDS, columns are computed in
// registers.  A lane reads its segment's rows; reads past them (up to the
// chunk's longest segment) stay inside the block's LDS (the next wave's area
// or the block's tables) and are masked off.
template <int W, bool DUMP, int P, bool SCV>
__device__ __forceinline__ void enum_solo(const uint32_t *filt, const DevTable &tab,
                                          const DevScratch &sc, const EnumShape &S,
                                          const uint64_t *__restrict__ samples,
                                          const double *__restrict__ log_amp,
                                          const double *__restrict__ phase, int64_t n,
                                          int64_t first, int64_t step,
                                          int32_t *__restrict__ hit_idx,
                                          uint32_t *__restrict__ sign_bits, int64_t sign_words,
                                          EnumCounts &cnt) {
    char *smem = dyn_lds();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t *hr = reinterpret_cast<const uint32_t *>(smem);
    uint2 *queue = reinterpret_cast<uint2 *>(smem + kEnumQueueOff) + wave * kEnumQueue;
    char *mine = smem + kEnumDynFixed + wave * enum_solo_bytes(S.lcb);
    uint8_t *o = reinterpret_cast<uint8_t *>(mine);  // alpha occ, alpha vir, beta occ, beta vir
    uint32_t *lh = reinterpret_cast<uint32_t *>(mine + kEnumSoloLists);
    uint16_t *lc = reinterpret_cast<uint16_t *>(mine + kEnumSoloLists + 4 * S.lcb);
    const uint32_t fbytes_mask = ((1u << sc.efilter_log2) - 1u) << 2;
    const char *filt_b = reinterpret_cast<const char *>(filt);
    // this lane's alpha and beta qubit, for the whole loop
    const bool ina = lane < tab.k_alpha, inb = lane < tab.k_beta;
    const int qa_l = ina ? tab.spin_q[lane] : 0;
    const int qb_l = inb ? tab.spin_q[64 + lane] : 0;
    const uint16_t *et = reinterpret_cast<const uint16_t *>(smem + enum_solo_entry_off(S.lcb));
    const uint32_t *tasks = reinterpret_cast<const uint32_t *>(smem + enum_solo_task_off(S.lcb));
    const int lcb = S.lcb;
    const int s_ca = S.ca, s_cba = S.cba, s_cbb = S.cbb;
    const int s_ra = S.ra, s_rba = S.rba, s_rbb = S.rbb;
    // per product: row segments of at most 64 rows, of equal length (a
    // multiple of 4), and the tasks (segment, column) they make
    const int ns_a = ceil_div(s_ra, kEnumRowSeg), ns_ba = ceil_div(s_rba, kEnumRowSeg);
    const int sl_a = seg_len(s_ra), sl_ba = seg_len(s_rba), sl_bb = seg_len(s_rbb);
    const int t_a = ns_a * s_ca, t_ba = ns_ba * s_cba;
    const int n_task = S.n_task;
    // every flip but (none, none)
    const unsigned long long n_probe = static_cast<unsigned long long>(s_ra) * s_ca +
                                       static_cast<unsigned long long>(s_rba) * s_cba +
                                       static_cast<unsigned long long>(s_rbb) * s_cbb - 1ull;
    const int64_t n_rounds = (n + kEnumWaves - 1) / kEnumWaves;
    for (int64_t r = first; r < n_rounds; r += step) {
        const int64_t i = r * kEnumWaves + wave;
        if (i >= n) break;  // later rounds only have larger indices
        if (wave == 0) ++cnt.rounds;
        Key<W> x;
        x.w[0] = samples[2 * i];
        if constexpr (W == 2) x.w[1] = samples[2 * i + 1];
        const uint64_t x1 = W == 2 ? x.w[W - 1] : 0ull;
        const double la = log_amp[i], ph = phase[i];
        const uint32_t hx = sc.shx[i];

        // orbital lists, in spin-qubit order
        {
            const bool oa = ina && (((qa_l < 64 ? x.w[0] : x1) >> (qa_l & 63)) & 1ull);
            const bool ob = inb && (((qb_l < 64 ? x.w[0] : x1) >> (qb_l & 63)) & 1ull);
            const uint64_t moa = __ballot(oa), mva = __ballot(ina && !oa);
            const uint64_t mob = __ballot(ob), mvb = __ballot(inb && !ob);
            if (oa) o[lanes_below(moa)] = static_cast<uint8_t>(qa_l);
            if (ina && !oa) o[32 + lanes_below(mva)] = static_cast<uint8_t>(qa_l);
            if (ob) o[64 + lanes_below(mob)] = static_cast<uint8_t>(qb_l);
            if (inb && !ob) o[96 + lanes_below(mvb)] = static_cast<uint8_t>(qb_l);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // row lists (hash, flip code) from the entry table: A rows (the none
        // row, then beta singles), alpha occupied pairs, beta occupied pairs
        for (int pos = lane; pos < lcb; pos += 64) {
            const uint32_t v = et[pos];
            const uint32_t ia = v & kNoQubit, ib = v >> 7;
            uint32_t h = 0u, c = kNoPair;
            if (ia != kNoQubit) {
                const uint32_t qa = o[ia], qb = o[ib];
                h = hr[qa] ^ hr[qb];
                c = qa | (qb << 7);
            }
            lh[pos] = h;
            lc[pos] = static_cast<uint16_t>(c);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");

        double acc_re = 0.0, acc_im = 0.0;
        AccF32 acc_r, acc_i;
        uint32_t qn = 0;
        auto flush = [&](uint32_t mcount) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            EnumHit c;
            if (lane < static_cast<int>(mcount)) {
                const uint2 e = queue[lane];
                enum_candidate<W, DUMP, P, SCV>(tab, sc, x, hx, la, ph, i, e,
                                                enum_candidate_bucket<W>(sc, e), log_amp, phase,
                                                hit_idx, sign_bits, sign_words, cnt, c);
            }
            uint64_t hm = __ballot(c.hit);
            while (hm) {
                const int q = __builtin_ctzll(hm);
                hm &= hm - 1;
                if constexpr (P == NQS_FP64) {
                    acc_re += readlane_f64(c.re, q);
                    acc_im += readlane_f64(c.im, q);
                } else {
                    acc_r.add(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(c.pre), q)),
                              __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c.ere), q)));
                    acc_i.add(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(c.pim), q)),
                              __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c.eim), q)));
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        };

        // lanes take (product, row segment, column) tasks, products and
        // segments in order: a chunk of 64 tasks may mix products, each lane
        // reading its own segment's rows (16-byte aligned)
        cnt.probes += n_probe;
        for (int c0 = 0; c0 < n_task; c0 += 64) {
            // this lane's task: rows [rb, rb + nr) of its product's list and
            // its column (alpha single or none, alpha or beta virtual pair)
            const uint32_t tv = tasks[c0 + lane];
            const int rb = static_cast<int>(tv & 0x7FFu);
            const int nr = static_cast<int>((tv >> 11) & 0x7Fu);
            const uint32_t ia = (tv >> 18) & kNoQubit, ib = tv >> 25;
            const bool act = nr > 0;
            uint32_t colh = 0u, colc = kNoPair;
            if (ia != kNoQubit) {
                const uint32_t qa = o[ia], qb = o[ib];
                colh = hr[qa] ^ hr[qb];
                colc = qa | (qb << 7);
            }
            colh ^= hx;
            // rows read by the chunk: the longest segment among its products
            const int tl = min(c0 + 63, n_task - 1);
            const int pf = c0 < t_a ? 0 : (c0 < t_a + t_ba ? 1 : 2);
            const int pl = tl < t_a ? 0 : (tl < t_a + t_ba ? 1 : 2);
            int nrl = 0;
            if (pf <= 0 && 0 <= pl) nrl = max(nrl, sl_a);
            if (pf <= 1 && 1 <= pl) nrl = max(nrl, sl_ba);
            if (pf <= 2 && 2 <= pl) nrl = max(nrl, sl_bb);
            const uint32_t *rw = lh + rb;
            const uint16_t *rc = lc + rb;
            // task 0 is (A, first segment, none column): its row 0 is x
            uint64_t pm = probe_rows<true>(filt_b, fbytes_mask, colh, rw, nrl, nr, act,
                                           c0 == 0 && lane == 0);
            for (;;) {
                const uint64_t any = __ballot(pm != 0ull);
                if (!any) break;
                const bool has = pm != 0ull;
                const int bit = has ? __builtin_ctzll(pm) : 0;
                const int rr = bit;
                pm &= pm - 1ull;
                const uint32_t c = static_cast<uint32_t>(__popcll(any));
                cnt.cand += c;
                if (qn + c > static_cast<uint32_t>(kEnumQueue)) {
                    flush(qn);
                    qn = 0;
                }
                if (has)
                    queue[qn + lanes_below(any)] = make_uint2(
                        colc | (static_cast<uint32_t>(rc[rr]) << 14), colh ^ rw[rr]);
                qn += c;
            }
        }
        if (qn > 0) flush(qn);
        if (lane == 0) {
            double *pp = sc.part + 2 * i;
            if constexpr (P == NQS_FP64) {
                pp[0] = acc_re;
                pp[1] = acc_im;
            } else {
                pp[0] = acc_r.value();
                pp[1] = acc_i.value();
            }
        }
    }
}

__device__ __forceinline__ void enum_flush_counts(const DevScratch &sc, EnumCounts &c) {
    unsigned long long h = c.hits, t = c.terms;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        h += __shfl_xor(h, off);
        t += __shfl_xor(t, off);
    }
    if ((threadIdx.x & 63) == 0) {
        count_add(sc.counters, 1, c.probes);
        count_add(sc.counters, 2, h);
        count_add(sc.counters, 3, t);
        count_add(sc.counters, 4, c.cand);
        if (threadIdx.x == 0) count_add(sc.counters, 6, c.rounds);
    }
    c = EnumCounts{};
}

// Hash words and qubit classes of a table into the enumeration's LDS (the
// caller synchronises before the first round).
__device__ __forceinline__ void load_enum_tables(const DevTable &tab) {
    char *smem = dyn_lds();
    uint32_t *hr = reinterpret_cast<uint32_t *>(smem);
    uint8_t *qcl = reinterpret_cast<uint8_t *>(smem + 512);
    for (int k = threadIdx.x; k < 128; k += blockDim.x) {
        hr[k] = tab.hr[k];
        qcl[k] = tab.qcls[k];
    }
}

// Entry table and task table of the solo rounds (the caller synchronises
// before use).  Entry table: for each position of a wave's row lists, the
// row's two qubits as indices into the wave's orbital lists (7 bits each,
// 0x7F: none, also for the padding): A rows (the none row, then beta
// occupied x beta virtual), alpha occupied pairs, beta occupied pairs.
// Task t of a sample, products and row segments in order: A = (none + alpha
// singles) columns x A rows, then Ba, then Bb; its word holds the first row
// (11 bits), the row count (7 bits) and the column's two qubits as orbital
// list indices (7 bits each, 0x7F: none).  Padding tasks up to a whole
// chunk have no rows and no qubits.
__device__ __forceinline__ void load_solo_tables(const EnumShape &S) {
    uint16_t *et = reinterpret_cast<uint16_t *>(dyn_lds() + enum_solo_entry_off(S.lcb));
    for (int pos = threadIdx.x; pos < S.lcb; pos += blockDim.x) {
        uint32_t ia = kNoQubit, ib = kNoQubit;
        if (pos < S.ra) {
            if (pos > 0) {
                const int kk = pos - 1, ii = kk / S.vb;
                ia = static_cast<uint32_t>(64 + ii);                // beta occupied
                ib = static_cast<uint32_t>(96 + kk - ii * S.vb);    // beta virtual
            }
        } else if (pos >= S.lba && pos < S.lba + S.rba) {
            int ii, jj;
            pair_of(pos - S.lba, ii, jj);                           // alpha occupied pair
            ia = static_cast<uint32_t>(ii);
            ib = static_cast<uint32_t>(jj);
        } else if (pos >= S.lbb && pos < S.lbb + S.rbb) {
            int ii, jj;
            pair_of(pos - S.lbb, ii, jj);                           // beta occupied pair
            ia = static_cast<uint32_t>(64 + ii);
            ib = static_cast<uint32_t>(64 + jj);
        }
        et[pos] = static_cast<uint16_t>(ia | (ib << 7));
    }
    uint32_t *tt = reinterpret_cast<uint32_t *>(dyn_lds() + enum_solo_task_off(S.lcb));
    const int ns_a = ceil_div(S.ra, kEnumRowSeg), ns_ba = ceil_div(S.rba, kEnumRowSeg);
    const int t_a = ns_a * S.ca, t_ba = ns_ba * S.cba;
    const int sl_a = seg_len(S.ra), sl_ba = seg_len(S.rba), sl_bb = seg_len(S.rbb);
    const int n_pad = 64 * ceil_div(S.n_task, 64);
    for (int t = threadIdx.x; t < n_pad; t += blockDim.x) {
        uint32_t rb = 0, nr = 0, ia = kNoQubit, ib = kNoQubit;
        if (t < S.n_task) {
            const int p = t < t_a ? 0 : (t < t_a + t_ba ? 1 : 2);
            const int u = t - (p == 0 ? 0 : (p == 1 ? t_a : t_a + t_ba));
            const int ncol = p == 0 ? S.ca : (p == 1 ? S.cba : S.cbb);
            const int sl = p == 0 ? sl_a : (p == 1 ? sl_ba : sl_bb);
            const int nrow = p == 0 ? S.ra : (p == 1 ? S.rba : S.rbb);
            const int row0 = p == 0 ? 0 : (p == 1 ? S.lba : S.lbb);
            const int seg = u / ncol, col = u - seg * ncol;
            rb = static_cast<uint32_t>(row0 + seg * sl);
            nr = static_cast<uint32_t>(min(nrow - seg * sl, sl));
            if (p == 0) {
                if (col > 0) {
                    const int kk = col - 1, ii = kk / S.va;
                    ia = static_cast<uint32_t>(ii);                  // alpha occupied
                    ib = static_cast<uint32_t>(32 + kk - ii * S.va);  // alpha virtual
                }
            } else {
                int ii, jj;
                pair_of(col, ii, jj);
                const int lb = p == 1 ? 32 : 96;                     // alpha / beta virtual
                ia = static_cast<uint32_t>(lb + ii);
                ib = static_cast<uint32_t>(lb + jj);
            }
        }
        tt[t] = rb | (nr << 11) | (ia << 18) | (ib << 25);
    }
}

__device__ __forceinline__ void load_filter_lds(const DevScratch &sc, uint4 *smem4) {
    // (also used with the static filter array of the enumeration kernels)
    const uint4 *gf = reinterpret_cast<const uint4 *>(sc.filter);
    const int n4 = (1 << sc.filter_log2) >> 2;
    for (int k = threadIdx.x; k < n4; k += blockDim.x) smem4[k] = gf[k];
}

// Persistent form: block b runs rounds b, b + grid, b + 2 grid, ...
template <int W, bool DUMP, int P, bool SCV>
__global__ __launch_bounds__(kEnumThreads) void eloc_enum_kernel(
    DevTable tab, DevScratch sc, const uint64_t *__restrict__ samples,
    const double *__restrict__ log_amp, const double *__restrict__ phase, int64_t n,
    int32_t *__restrict__ hit_idx, uint32_t *__restrict__ sign_bits, int64_t sign_words) {
    // the filter at LDS address 0 (a static array: its address folds into
    // the read); records, lists and queues in the dynamic rest
    __shared__ uint4 s_filter[kEnumFilterWords / 4];
    if (join_chosen(sc)) return;  // the pair join of this launch does the work
    const EnumShape S = enum_shape(tab, sc, samples, n);
    if (S.B <= 0) return;  // the streaming kernel of this launch does the work
    const int64_t n_rounds = (n + S.B - 1) / S.B;
    if (S.parts == 1) load_filter_lds(sc, s_filter);  // else each round loads its partitions
    load_enum_tables(tab);
    if (S.solo) load_solo_tables(S);
    __syncthreads();
    EnumCounts cnt;
    int loaded_part = -1;
    // rounds blockIdx.x, blockIdx.x + gridDim.x, ...: no counter, no barrier
    if (S.solo) {
        enum_solo<W, DUMP, P, SCV>(reinterpret_cast<uint32_t *>(s_filter), tab, sc, S, samples,
                                   log_amp, phase, n, blockIdx.x, gridDim.x, hit_idx, sign_bits,
                                   sign_words, cnt);
    } else {
        for (int64_t r = blockIdx.x; r < n_rounds; r += gridDim.x)
            enum_round<W, DUMP, P, SCV>(reinterpret_cast<uint32_t *>(s_filter), tab, sc, S,
                                        samples, log_amp, phase, n, r, hit_idx, sign_bits,
                                        sign_words, cnt, loaded_part);
    }
    enum_flush_counts(sc, cnt);
}

// Marks every (sample, group) pair of a dump as "no candidate" before an
// enumeration writes its hits.
__global__ void fill_i32_kernel(int32_t *__restrict__ p, int64_t count, int32_t v) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < count) p[k] = v;
}

// Grid form: (sample tiles of blockDim) x (group chunks), one item per block.
template <int W, bool S32, bool SEC, bool DUMP, int P, bool SCV>
__global__ __launch_bounds__(kLookupThreads) void eloc_lookup_kernel(
    DevTable tab, DevScratch sc, const uint64_t *__restrict__ samples,
    const double *__restrict__ log_amp, const double *__restrict__ phase, int64_t n,
    int64_t g_first, int64_t chunk_len, int32_t *__restrict__ hit_idx,
    uint32_t *__restrict__ sign_bits, int64_t sign_words, int fallback_only) {
    extern __shared__ uint4 smem4[];
    if (join_chosen(sc)) return;  // the pair join of this launch does the work
    // beside an enumeration launch this grid only runs when enumeration cannot
    if (fallback_only && enum_shape(tab, sc, samples, n).B > 0) return;
    lookup_item<W, S32, SEC, DUMP, P, SCV>(tab, sc, samples, log_amp, phase, n, blockIdx.x, blockIdx.y,
                                      g_first, chunk_len, true, hit_idx, sign_bits, sign_words,
                                      smem4);
}

// <x|H_diag|x> from the occupation form of the X = 0 group: d[0] plus, for
// each occupied qubit j in increasing order, d[1 + j] and the pair terms
// d[1 + nq + j (j - 1) / 2 + i] of the occupied i < j (d: FP64 values, or
// FP32 (hi, lo) pairs in the same 8 bytes for the compensated form).
// The next set bit of (lo, hi) in increasing order (lo first), cleared.
// Selects instead of branches: lanes whose sets have equally many bits run
// the same number of steps whichever words the bits sit in.
__device__ __forceinline__ int pop_lowest(uint64_t &lo, uint64_t &hi) {
    const bool in_lo = lo != 0ull;
    const uint64_t m = in_lo ? lo : hi;
    const int q = (in_lo ? 0 : 64) + __builtin_ctzll(m);
    const uint64_t cleared = m & (m - 1);
    lo = in_lo ? cleared : lo;
    hi = in_lo ? hi : cleared;
    return q;
}

// <x|H_diag|x> from the occupation form of the X = 0 group: d[0] plus, for
// each occupied qubit j in increasing order, d[1 + j] and the pair terms
// d[1 + nq + j (j - 1) / 2 + i] of the occupied i < j in increasing order
// (d: FP64 values, or FP32 (hi, lo) pairs in the same 8 bytes for the
// compensated form).  Every sample of a one-sector batch takes the same
// number of steps in both loops (the k-th occupied qubit has k below it).
template <int W, int P>
__device__ __forceinline__ double diag_occ_sum(const double *d, int nq, const Key<W> &x) {
    const double *d2 = d + 1 + nq;
    const uint64_t x0 = x.w[0], x1 = W == 2 ? x.w[W - 1] : 0ull;
    uint64_t a0 = x0, a1 = x1;
    if constexpr (P == NQS_FP64) {
        double acc = d[0];
        while (a0 | a1) {
            const int j = pop_lowest(a0, a1);
            const double *row = d2 + j * (j - 1) / 2;
            double t = d[1 + j];
            // the occupied qubits below j
            uint64_t b0 = j >= 64 ? x0 : (x0 & ((1ull << j) - 1ull));
            uint64_t b1 = j >= 64 ? (x1 & ((1ull << (j & 63)) - 1ull)) : 0ull;
            while (b0 | b1) t += row[pop_lowest(b0, b1)];
            acc += t;
        }
        return acc;
    } else {
        const float2 *f = reinterpret_cast<const float2 *>(d);
        const float2 *f2 = f + 1 + nq;
        AccF32 a;
        a.add(f[0].x, f[0].y);
        while (a0 | a1) {
            const int j = pop_lowest(a0, a1);
            const float2 *row = f2 + j * (j - 1) / 2;
            a.add(f[1 + j].x, f[1 + j].y);
            uint64_t b0 = j >= 64 ? x0 : (x0 & ((1ull << j) - 1ull));
            uint64_t b1 = j >= 64 ? (x1 & ((1ull << (j & 63)) - 1ull)) : 0ull;
            while (b0 | b1) {
                const float2 v = row[pop_lowest(b0, b1)];
                a.add(v.x, v.y);
            }
        }
        return a.value();
    }
}

typedef int diag_v4i __attribute__((ext_vector_type(4)));

// Bits b of a 16-bit value as 16 bytes of 0 or 1 (byte b = bit b): each
// nibble times 0x00204081 puts its bits 7 apart, one in each byte's bit 0.
__device__ __forceinline__ diag_v4i spread_bits16(uint32_t v) {
    diag_v4i r;
    r[0] = static_cast<int>(((v & 0xFu) * 0x00204081u) & 0x01010101u);
    r[1] = static_cast<int>((((v >> 4) & 0xFu) * 0x00204081u) & 0x01010101u);
    r[2] = static_cast<int>((((v >> 8) & 0xFu) * 0x00204081u) & 0x01010101u);
    r[3] = static_cast<int>((((v >> 12) & 0xFu) * 0x00204081u) & 0x01010101u);
    return r;
}

// The occupation-form diagonal of the 64 samples of a wave (each lane's x;
// zero for a lane without a sample) on the matrix cores, called by every
// lane of the wave together.  With n the 0/1 occupations and Q the
// fixed-point terms in base-2^15 digits E_l (see kDiagDigits), the value is
//   d0 + 2^-S sum_l 2^(15 l) sum_j n_j sum_{i <= j} n_i E_l[j][i].
// Per digit l, column tile jt and group of 16 samples: C = E_l N (16 x 16
// products over k = i; N the samples' bits, one column per sample), so
// C[j][s] = sum_i E_l[j][i] n_s[i].  E_l = a - 128 b is held as two int8
// byte planes: one chain of MFMAs multiplies plane a by N and plane b by
// -128 N (the bits as bytes 0x80) into the same accumulator, so C arrives
// whole in 32 bits; each lane masks its four C[j][s] by n_s[j] and adds them
// to its digit sum.  All of it is exact integer arithmetic (|C| <= 2^21,
// a digit sum below 2^28), the digits are recombined in 64-bit integers and
// the total is rounded once to FP64, so the result does not depend on any
// order of summation.  B holds the digit tiles (LDS or global memory).
//
// Lane layout of the instruction: lane L holds row L % 16 of A and column
// L % 16 of B, with k in [16 (L / 16), +16) of the 64-wide k-block (byte
// b = k); C row 4 (L / 16) + r, column L % 16 in its r-th value.  The digit
// tiles are stored in that A layout.
// One column tile jt of diag_occ_mfma for H groups of 16 samples: the
// digit tiles at B + t (KB k-blocks), the samples' bit operands N and M
// (-128 N), the row masks mk (bit 4 jt + r: n_s[j] for the lane's row
// j = 16 jt + 4 g + r), the digit sums T.
template <int H, int KB>
__device__ __forceinline__ void diag_mfma_tile(const diag_v4i *__restrict__ B, int t, int jt,
                                               int lane, const diag_v4i (&N)[H][2],
                                               const diag_v4i (&M)[H][2],
                                               const uint32_t (&mk)[H], int (&T)[H][kDiagDigits]) {
    const diag_v4i zero = {0, 0, 0, 0};
    // the row masks as 0/1 multipliers (hidden from the optimiser, so that
    // each masked add stays a 24-bit multiply-add)
    int bit[H][4];
#pragma unroll
    for (int h = 0; h < H; ++h) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            bit[h][r] = static_cast<int>((mk[h] >> (4 * jt + r)) & 1u);
            asm("" : "+v"(bit[h][r]));
        }
    }
#pragma unroll
    for (int l = 0; l < kDiagDigits; ++l) {
        diag_v4i a[KB], b[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            a[kb] = B[((t + kb) * kDiagLimbs + 2 * l) * 64 + lane];
            b[kb] = B[((t + kb) * kDiagLimbs + 2 * l + 1) * 64 + lane];
        }
#pragma unroll
        for (int h = 0; h < H; ++h) {
            // both planes of every k-block into one accumulator
            diag_v4i acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0], N[h][0], zero, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(b[0], M[h][0], acc, 0, 0, 0);
            if constexpr (KB == 2) {
                acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[1], N[h][1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(b[1], M[h][1], acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T[h][l] = __mul24(acc[r], bit[h][r]) + T[h][l];
                // one 24-bit multiply-add per value (not two products
                // summed by a three-input add)
                asm("" : "+v"(T[h][l]));
            }
        }
    }
}

template <int W>
__device__ __forceinline__ double diag_occ_mfma(const DevTable &tab, const Key<W> &x,
                                                const diag_v4i *__restrict__ B) {
    // all four groups of 16 samples in one pass over the digit tiles
    constexpr int H = 4;
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
    const uint64_t w0 = x.w[0], w1 = W == 2 ? x.w[W - 1] : 0ull;
    const int jtiles = tab.diag_jtiles;
    // the column samples 16 h + c: their bits as the B operands of both
    // k-blocks (bytes 0/1 in N, 0/0x80 in M), and the lane's row masks
    // (bits 16 jt + 4 g + r of them, packed as bit 4 jt + r)
    diag_v4i N[H][2], M[H][2];
    uint32_t mk[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const uint64_t m0 = __shfl(w0, 16 * h + c), m1 = __shfl(w1, 16 * h + c);
        N[h][0] = spread_bits16(static_cast<uint32_t>(m0 >> (16 * g)) & 0xFFFFu);
        N[h][1] = spread_bits16(static_cast<uint32_t>(m1 >> (16 * g)) & 0xFFFFu);
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int v = 0; v < 4; ++v) M[h][kb][v] = N[h][kb][v] << 7;
        // (row group g of tile jt: bits 16 jt + 4 g .. + 3, inside one
        // 32-bit half of the sample: one bit-field extract each)
        const uint32_t half[4] = {static_cast<uint32_t>(m0), static_cast<uint32_t>(m0 >> 32),
                                  static_cast<uint32_t>(m1), static_cast<uint32_t>(m1 >> 32)};
        uint32_t v = 0;
#pragma unroll
        for (int jt = 0; jt < 8; ++jt)
            v |= __builtin_amdgcn_ubfe(half[jt >> 1], 16 * (jt & 1) + 4 * g, 4) << (4 * jt);
        mk[h] = v;
    }
    int T[H][kDiagDigits];
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
        for (int l = 0; l < kDiagDigits; ++l) T[h][l] = 0;
    // column tiles 0..3 reach rows i < 64 (one k-block), later ones two
    const int j1 = jtiles < 4 ? jtiles : 4;
    for (int jt = 0; jt < j1; ++jt) diag_mfma_tile<H, 1>(B, jt, jt, lane, N, M, mk, T);
    for (int jt = 4; jt < jtiles; ++jt)
        diag_mfma_tile<H, 2>(B, 4 + 2 * (jt - 4), jt, lane, N, M, mk, T);
    double mine = 0.0;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        // digits 0, 1 and 2, 3 recombined (each pair below 2^44 in
        // magnitude), then summed over the four row groups of the lane's
        // column
        long long lo = static_cast<long long>(T[h][0]) + (static_cast<long long>(T[h][1]) << 15);
        long long hi = static_cast<long long>(T[h][2]) + (static_cast<long long>(T[h][3]) << 15);
        lo += __shfl_xor(lo, 16);
        hi += __shfl_xor(hi, 16);
        lo += __shfl_xor(lo, 32);
        hi += __shfl_xor(hi, 32);
        // both terms exact in FP64, one rounding of the exact total; the
        // lane of sample 16 h + c (row group h) keeps it
        const double v = static_cast<double>(lo) + static_cast<double>(hi) * 1073741824.0;
        if (g == h) mine = v;
    }
    return tab.diag[0] + mine * tab.diag_scale;
}

// The same sum from a staged occupation form, with the occupied qubits first
// written, in increasing order, as bytes into the lane's list in LDS
// (interleaved across the block: entries 4w..4w+3 of this lane are the word
// lst[w * stride]).  Four row entries are read per step, independently of
// each other (the bit scan of the loop above makes every read wait for the
// last), and added in the same order: the bits of the result are the same.
template <int W, int P>
__device__ __forceinline__ double diag_occ_sum_list(const double *d, int nq, const Key<W> &x,
                                                    uint32_t *lst, int stride) {
    uint64_t a0 = x.w[0], a1 = W == 2 ? x.w[W - 1] : 0ull;
    int cnt = 0;
    uint32_t word = 0;
    while (a0 | a1) {
        const int q = pop_lowest(a0, a1);
        word |= static_cast<uint32_t>(q) << (8 * (cnt & 3));
        if ((cnt & 3) == 3) {
            lst[(cnt >> 2) * stride] = word;
            word = 0;
        }
        ++cnt;
    }
    // the last word's unused bytes are 0 (a valid row index, never added)
    if (cnt & 3) lst[(cnt >> 2) * stride] = word;
    if constexpr (P == NQS_FP64) {
        const double *d2 = d + 1 + nq;
        double acc = d[0];
        for (int k = 0; k < cnt; ++k) {
            const int j = static_cast<int>((lst[(k >> 2) * stride] >> (8 * (k & 3))) & 0xFFu);
            const double *row = d2 + j * (j - 1) / 2;
            double t = d[1 + j];
            for (int m = 0; m < k; m += 4) {
                const uint32_t iw = lst[(m >> 2) * stride];
                const double r0 = row[iw & 0xFFu], r1 = row[(iw >> 8) & 0xFFu];
                const double r2 = row[(iw >> 16) & 0xFFu], r3 = row[iw >> 24];
                t += r0;
                if (m + 1 < k) t += r1;
                if (m + 2 < k) t += r2;
                if (m + 3 < k) t += r3;
            }
            acc += t;
        }
        return acc;
    } else {
        const float2 *f = reinterpret_cast<const float2 *>(d);
        const float2 *f2 = f + 1 + nq;
        AccF32 a;
        a.add(f[0].x, f[0].y);
        for (int k = 0; k < cnt; ++k) {
            const int j = static_cast<int>((lst[(k >> 2) * stride] >> (8 * (k & 3))) & 0xFFu);
            const float2 *row = f2 + j * (j - 1) / 2;
            a.add(f[1 + j].x, f[1 + j].y);
            for (int m = 0; m < k; m += 4) {
                const uint32_t iw = lst[(m >> 2) * stride];
                const float2 r0 = row[iw & 0xFFu], r1 = row[(iw >> 8) & 0xFFu];
                const float2 r2 = row[(iw >> 16) & 0xFFu], r3 = row[iw >> 24];
                a.add(r0.x, r0.y);
                if (m + 1 < k) a.add(r1.x, r1.y);
                if (m + 2 < k) a.add(r2.x, r2.y);
                if (m + 3 < k) a.add(r3.x, r3.y);
            }
        }
        return a.value();
    }
}

// E_loc(x) = diagonal group sum + sum of the chunk partials in chunk order.
template <int W, bool DUMP, int P, bool SCV>
__device__ __forceinline__ void finish_one(const DevTable &tab, const DevScratch &sc,
                                           const uint64_t *__restrict__ samples, int64_t n,
                                           int64_t n_chunks, bool enum_on,
                                           double *__restrict__ eloc,
                                           int32_t *__restrict__ hit_idx,
                                           uint32_t *__restrict__ sign_bits, int64_t sign_words,
                                           int64_t i, const uint64_t *dz = nullptr,
                                           const double *dc = nullptr, int nd = 0,
                                           const double *dq = nullptr,
                                           uint32_t *olist = nullptr, bool have_d = false,
                                           double dval = 0.0, double2 *value = nullptr) {
    unsigned long long n_terms = 0;
    // the pair join leaves one partial per block, an enumeration one per sample
    if (join_chosen(sc))
        n_chunks = tab.join_blocks;
    else if (enum_on && enum_shape(tab, sc, samples, n).B > 0)
        n_chunks = 1;
    if (i < n) {
        const Key<W> x = load_key<W>(samples, i);
        double re = 0.0, im = 0.0;
        if (tab.has_diagonal) {
            if constexpr (SCV) {
                re = sc_diagonal<W>(tab, x);
            } else if (have_d) {
                // the occupation form on the matrix cores (computed by the
                // caller for the whole wave)
                re = dval;
            } else if (dq) {
                // occupation form (the caller passes it staged or in place);
                // counted as the X = 0 group's terms it stands for
                re = olist ? diag_occ_sum_list<W, P>(dq, tab.n_qubits, x, olist + threadIdx.x,
                                                     static_cast<int>(blockDim.x))
                           : diag_occ_sum<W, P>(dq, tab.n_qubits, x);
                n_terms += static_cast<unsigned long long>(tab.goff[1] - tab.goff[0]);
            } else if (dz) {
                // the X = 0 group staged in LDS by the caller (same order, same sums)
                if constexpr (P == NQS_FP64) {
                    double acc = 0.0;
                    for (int t = 0; t < nd; ++t) {
                        int par = __popcll(dz[2 * t] & x.w[0]);
                        if constexpr (W == 2) par += __popcll(dz[2 * t + 1] & x.w[1]);
                        acc += (par & 1) ? -dc[t] : dc[t];
                    }
                    re = acc;
                } else {
                    AccF32 a;
                    const float2 *dc32 = reinterpret_cast<const float2 *>(dc);
                    for (int t = 0; t < nd; ++t) {
                        int par = __popcll(dz[2 * t] & x.w[0]);
                        if constexpr (W == 2) par += __popcll(dz[2 * t + 1] & x.w[1]);
                        const float2 cc = dc32[t];
                        a.add(flip_sign(cc.x, par), flip_sign(cc.y, par));
                    }
                    re = a.value();
                }
                n_terms += static_cast<unsigned long long>(nd);
            } else if constexpr (P == NQS_FP64) {
                uint32_t *row = (DUMP && sign_bits) ? sign_bits + i * sign_words : nullptr;
                re = group_sum<W, DUMP>(tab, 0, x, row, &n_terms);
            } else {
                re = group_sum_f32<W>(tab, 0, x, &n_terms).value();
            }
            if constexpr (DUMP) {
                if (hit_idx) hit_idx[i * tab.n_groups] = static_cast<int32_t>(i);
            }
        }
        if (join_chosen(sc)) {
            // the pair join: the blocks' partials in block order, only
            // those its hit map flags (the others were never written)
            uint32_t w[kJoinMaxBlocks];
#pragma unroll
            for (int b = 0; b < kJoinMaxBlocks; ++b) {
                const int64_t e = static_cast<int64_t>(b) * n + i;
                w[b] = b < n_chunks ? sc.jhit[e >> 5] : 0u;
            }
#pragma unroll
            for (int b = 0; b < kJoinMaxBlocks; ++b) {
                const int64_t e = static_cast<int64_t>(b) * n + i;
                if ((w[b] >> (e & 31)) & 1u) {
                    const double2 v = *reinterpret_cast<const double2 *>(sc.part + 2 * e);
                    re += v.x;
                    im += v.y;
                }
            }
            n_chunks = 0;
        }
        // the partials in chunk order, eight loads in flight at a time
        for (int64_t c0 = 0; c0 < n_chunks; c0 += 8) {
            double2 v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (c0 + k < n_chunks)
                    v[k] = *reinterpret_cast<const double2 *>(sc.part + 2 * ((c0 + k) * n + i));
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (c0 + k < n_chunks) {
                    re += v[k].x;
                    im += v[k].y;
                }
        }
        eloc[2 * i] = re;
        eloc[2 * i + 1] = im;
        if (value) *value = make_double2(re, im);
    }
    // every sample sums the whole X = 0 group: one count for the batch
    (void)n_terms;
    if (!SCV && tab.has_diagonal && blockIdx.x == 0 && threadIdx.x == 0)
        count_add(sc.counters, 3,
                  static_cast<unsigned long long>(n) * (tab.goff[1] - tab.goff[0]));
}

// Diagonal terms staged in LDS by the finish kernels (up to this many; a
// larger X = 0 group is read from device memory).
constexpr int kDiagLds = 1024;

// Copy the X = 0 group's Z masks and coefficients (FP64, or the FP32 hi/lo
// pair in the same 8 bytes) into LDS; returns the term count, or -1 when the
// group does not fit.  Synchronises the block.
template <int P>
__device__ __forceinline__ int stage_diagonal(const DevTable &tab, uint64_t *dz, double *dc) {
    if (!tab.has_diagonal) return -1;
    const int t0 = static_cast<int>(tab.goff[0]);
    const int nd = static_cast<int>(tab.goff[1]) - t0;
    if (nd > kDiagLds) return -1;
    for (int k = threadIdx.x; k < nd; k += blockDim.x) {
        dz[2 * k] = tab.tz[2 * static_cast<size_t>(t0 + k)];
        dz[2 * k + 1] = tab.tz[2 * static_cast<size_t>(t0 + k) + 1];
        if constexpr (P == NQS_FP64) {
            dc[k] = tab.tc[t0 + k];
        } else {
            const float2 cc = make_float2(tab.tc32[2 * static_cast<size_t>(t0 + k)],
                                          tab.tc32[2 * static_cast<size_t>(t0 + k) + 1]);
            dc[k] = *reinterpret_cast<const double *>(&cc);
        }
    }
    __syncthreads();
    return nd;
}

// The occupation form of the diagonal (its 1 + nq + nq (nq - 1) / 2 entries)
// in LDS when it fits the staging area of the term form, else in place;
// nullptr when the table has no such form.  Synchronises the block.
template <int P>
__device__ __forceinline__ const double *stage_diag_occ(const DevTable &tab, double *buf,
                                                        int cap = 3 * kDiagLds) {
    if (!tab.diag_occ) return nullptr;
    const int nq = tab.n_qubits;
    const int cnt = 1 + nq + nq * (nq - 1) / 2;
    const double *src = P == NQS_FP64 ? tab.diag : reinterpret_cast<const double *>(tab.diag32);
    if (cnt > cap) return src;
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) buf[k] = src[k];
    __syncthreads();
    return buf;
}

// Eq. 1 beside the finish: the weighted sums of one block's samples
// (w = 0 for a thread without a sample), W_b = sum w, sum w Re E,
// sum w Im E, and M2_b = sum w |E - m_b|^2 about the block's own mean m_b,
// written by thread 0 to part[0..3].  Sums over each wave by a fixed XOR
// pattern, then over the waves in order: the same bits on every call.
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ void energy_block_partial(double w, double re, double im, double *__restrict__ part) {
    __shared__ double red[16][3];
    __shared__ double mean[2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int waves = static_cast<int>(blockDim.x >> 6);
    const double sw = wave_sum_f64(w), sr = wave_sum_f64(w * re), si = wave_sum_f64(w * im);
    if (lane == 0) {
        red[wave][0] = sw;
        red[wave][1] = sr;
        red[wave][2] = si;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double W = 0.0, R = 0.0, I = 0.0;
        for (int k = 0; k < waves; ++k) {
            W += red[k][0];
            R += red[k][1];
            I += red[k][2];
        }
        part[0] = W;
        part[1] = R;
        part[2] = I;
        mean[0] = W != 0.0 ? R / W : 0.0;
        mean[1] = W != 0.0 ? I / W : 0.0;
    }
    __syncthreads();
    const double dr = re - mean[0], di = im - mean[1];
    const double sv = wave_sum_f64(w * (dr * dr + di * di));
    __syncthreads();  // every wave has read red[] and mean[]
    if (lane == 0) red[wave][0] = sv;
    __syncthreads();
    if (threadIdx.x == 0) {
        double V = 0.0;
        for (int k = 0; k < waves; ++k) V += red[k][0];
        part[3] = V;
    }
}

template <int W, bool DUMP, int P, bool SCV>
__global__ __launch_bounds__(256) void eloc_finish_kernel(
    DevTable tab, DevScratch sc, const uint64_t *__restrict__ samples, int64_t n,
    int64_t n_chunks, int enum_on, double *__restrict__ eloc, int32_t *__restrict__ hit_idx,
    uint32_t *__restrict__ sign_bits, int64_t sign_words, int stage_cap, int list_words,
    const int64_t *__restrict__ weights, double *__restrict__ epart) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    bool done = false;
    double2 v = make_double2(0.0, 0.0);
    if constexpr (!DUMP && !SCV) {
        // staging area (dynamic LDS of stage_cap doubles, at least
        // 3 kDiagLds): the diagonal's Z masks and coefficients, or its
        // occupation form
        double *stage = reinterpret_cast<double *>(dyn_lds());
        const double *dq = stage_diag_occ<P>(tab, stage, stage_cap);
        if (dq) {
            // staged: the occupied-qubit lists follow the stage (list_words
            // words per thread)
            uint32_t *olist = (dq == stage && list_words > 0)
                                  ? reinterpret_cast<uint32_t *>(stage + stage_cap)
                                  : nullptr;
            finish_one<W, DUMP, P, SCV>(tab, sc, samples, n, n_chunks, enum_on != 0, eloc,
                                        hit_idx, sign_bits, sign_words, i, nullptr, nullptr, 0,
                                        dq, olist, false, 0.0, &v);
            done = true;
        } else {
            uint64_t *dz = reinterpret_cast<uint64_t *>(stage);
            double *dc = stage + 2 * kDiagLds;
            const int nd = stage_diagonal<P>(tab, dz, dc);
            if (nd >= 0) {
                finish_one<W, DUMP, P, SCV>(tab, sc, samples, n, n_chunks, enum_on != 0, eloc,
                                            hit_idx, sign_bits, sign_words, i, dz, dc, nd,
                                            nullptr, nullptr, false, 0.0, &v);
                done = true;
            }
        }
    }
    if (!done)
        finish_one<W, DUMP, P, SCV>(tab, sc, samples, n, n_chunks, enum_on != 0, eloc, hit_idx,
                                    sign_bits, sign_words, i, nullptr, nullptr, 0, nullptr,
                                    nullptr, false, 0.0, &v);
    if (epart) {
        // this thread's E_loc, as just written (not read back)
        energy_block_partial(i < n ? static_cast<double>(weights[i]) : 0.0, v.x, v.y,
                             epart + 4 * static_cast<int64_t>(blockIdx.x));
    }
}

// The finish kernel of tables with the occupation-form diagonal (no debug
// dump, Pauli form): the digit tiles staged in LDS once per block, the
// diagonal of each wave's 64 samples on the matrix cores, then the partials.
constexpr int kFinishMfmaThreads = 1024;
constexpr int kDiagMaxTiles = diag_mfma_tiles(8);

template <int W, int P>
__global__ __launch_bounds__(kFinishMfmaThreads) void eloc_finish_mfma_kernel(
    DevTable tab, DevScratch sc, const uint64_t *__restrict__ samples, int64_t n,
    int64_t n_chunks, int enum_on, double *__restrict__ eloc, const int64_t *__restrict__ weights,
    double *__restrict__ epart) {
    __shared__ diag_v4i tiles[kDiagMaxTiles * kDiagLimbs * 64];
    // the sample first: its load overlaps the staging of the tiles
    Key<W> x;
#pragma unroll
    for (int w = 0; w < W; ++w) x.w[w] = 0ull;
    {
        const int64_t i0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
        if (i0 < n) x = load_key<W>(samples, i0);
    }
    const int words = diag_mfma_tiles(tab.diag_jtiles) * kDiagLimbs * 64;
    const diag_v4i *src = reinterpret_cast<const diag_v4i *>(tab.diag_q8);
    for (int k = threadIdx.x; k < words; k += blockDim.x) tiles[k] = src[k];
    __syncthreads();
    const double d = diag_occ_mfma<W>(tab, x, tiles);
    // the index again (two registers not held across the diagonal)
    unsigned tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + tid;
    double2 v = make_double2(0.0, 0.0);
    finish_one<W, false, P, false>(tab, sc, samples, n, n_chunks, enum_on != 0, eloc, nullptr,
                                   nullptr, 0, i, nullptr, nullptr, 0, nullptr, nullptr, true, d,
                                   &v);
    if (epart) {
        // this thread's E_loc, as just written (not read back)
        energy_block_partial(i < n ? static_cast<double>(weights[i]) : 0.0, v.x, v.y,
                             epart + 4 * static_cast<int64_t>(blockIdx.x));
    }
}

// ------------------------------------------------------------------ batched form
//
// Many Hamiltonians and uneven batches in one pass.  Small per-job kernels
// run on a (tile, job) grid; the lookup work of all jobs is one list of
// (job, tile, chunk) items drained by a persistent kernel: each block takes
// the next item from one atomic counter until the list is empty, and
// reloads the LDS Bloom bitmap only when the job changes.  Partials are
// per item, so the result does not depend on which block ran which item.

__global__ void batch_reset_kernel(const JobDesc *__restrict__ jobs, int n_jobs,
                                   unsigned *__restrict__ next) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n_jobs) {
        for (int k = 0; k < kCounters * kCounterSlots; ++k) jobs[j].sc.counters[k] = 0;
        *jobs[j].sc.mixed = 0;
    }
    if (j == 0)
        for (int k = 0; k < kBatchCounters; ++k) next[k] = 0u;
}

__global__ void batch_clear_kernel(const JobDesc *__restrict__ jobs) {
    const JobDesc &J = jobs[blockIdx.y];
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const int words = (J.kind & 1) + 1;
    if (s < J.capacity) {
        J.sc.sidx[s] = -1;
        J.sc.sfp[s] = 0u;
        J.sc.skey[static_cast<size_t>(s) * words + words - 1] = kFreeKey;
    }
    if (s < (1u << J.sc.filter_log2)) J.sc.filter[s] = 0u;
    if (J.sc.eparts_log2 > 0 && s < (1u << (J.sc.eparts_log2 + J.sc.efilter_log2)))
        J.sc.efilter[s] = 0u;
    if (J.sc.jctl) {
        if (s < static_cast<uint32_t>(J.sc.join_parts)) J.sc.jcnt[s] = 0u;
        if (s < static_cast<uint32_t>((J.tab.join_blocks * J.n + 31) / 32)) J.sc.jhit[s] = 0u;
        if (s < static_cast<uint32_t>(kJoinCtl)) J.sc.jctl[s] = 0ull;
    }
}

__global__ void batch_build_kernel(const JobDesc *__restrict__ jobs) {
    const JobDesc &J = jobs[blockIdx.y];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= J.n) return;
    if ((J.kind & 1) == 0)
        hash_build_one<1>(J.tab, J.sc, J.samples, J.weights, i);
    else
        hash_build_one<2>(J.tab, J.sc, J.samples, J.weights, i);
}

// Enumeration items: rounds tile, tile + stride, ... of one job.  One
// persistent kernel per variant (mask words, evaluator) drains the items of
// that variant; each job runs block rounds or solo rounds as its shape
// decides (the shape is known on the device only), exactly as a single
// launch would.  They run before the streaming kernel.
template <int W, int P, bool SCV>
__global__ __launch_bounds__(kEnumThreads) void batch_enum_kernel(
    const JobDesc *__restrict__ jobs, const WorkItem *__restrict__ items, int n_items,
    unsigned *__restrict__ next) {
    __shared__ uint4 s_filter[kEnumFilterWords / 4];
    __shared__ int cur;
    int last_job = -1;
    int loaded_part = -1;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) cur = static_cast<int>(atomicAdd(next, 1u));
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(cur);
        if (it >= n_items) break;  // every block reaches this once the list is drained
        const WorkItem w = items[it];
        const JobDesc &J = jobs[w.job];
        if (join_chosen(J.sc)) continue;  // the pair join does this job
        const EnumShape S = uniform_shape(enum_shape(J.tab, J.sc, J.samples, J.n));
        if (S.B <= 0) continue;  // the streaming items do this job
        const int per_round = S.solo ? kEnumWaves : S.B;
        const int64_t n_rounds = (J.n + per_round - 1) / per_round;
        if (w.tile >= n_rounds) continue;
        if (w.job != last_job) {
            // (with several partitions each round loads the ones it needs)
            if (S.parts == 1) load_filter_lds(J.sc, s_filter);
            load_enum_tables(J.tab);
            if (S.solo) load_solo_tables(S);
            loaded_part = -1;
            __syncthreads();
        }
        last_job = w.job;
        EnumCounts cnt;
        if (S.solo) {
            enum_solo<W, false, P, SCV>(reinterpret_cast<uint32_t *>(s_filter), J.tab, J.sc, S,
                                        J.samples, J.log_amp, J.phase, J.n, w.tile, w.stride,
                                        nullptr, nullptr, 0, cnt);
        } else {
            for (int64_t r = w.tile; r < n_rounds; r += w.stride)
                enum_round<W, false, P, SCV>(reinterpret_cast<uint32_t *>(s_filter), J.tab,
                                             J.sc, S, J.samples, J.log_amp, J.phase, J.n, r,
                                             nullptr, nullptr, 0, cnt, loaded_part);
        }
        enum_flush_counts(J.sc, cnt);
    }
}

// Streaming items; those of a job that is enumerated return at once (they
// run only when the job's samples span several sectors).
template <int P>
__global__ __launch_bounds__(kLookupThreads) void batch_lookup_kernel(
    const JobDesc *__restrict__ jobs, const WorkItem *__restrict__ items, int n_items,
    unsigned *__restrict__ next) {
    extern __shared__ uint4 smem4[];
    __shared__ int cur;
    int last_job = -1;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) cur = static_cast<int>(atomicAdd(next, 1u));
        __syncthreads();
        // block-uniform: scalar loads of the item and its job descriptor
        const int it = __builtin_amdgcn_readfirstlane(cur);
        if (it >= n_items) break;  // every block reaches this once the list is drained
        const WorkItem w = items[it];
        const JobDesc &J = jobs[w.job];
        if (join_chosen(J.sc)) continue;  // the pair join does this job
        if (J.strategy == kStrategyEnum && enum_shape(J.tab, J.sc, J.samples, J.n).B > 0)
            continue;  // enumerated instead
        const bool load = w.job != last_job;
        last_job = w.job;
#define NQS_ITEM(Wd, S, SE, Pr, SCI)                                                          \
    lookup_item<Wd, S, SE, false, Pr, SCI>(J.tab, J.sc, J.samples, J.log_amp, J.phase, J.n,      \
                                           w.tile, w.chunk, J.g_first, J.chunk_len, load, nullptr, \
                                           nullptr, 0, smem4)
        // integral-form jobs evaluate in FP64 whatever the batch precision
        switch (J.kind) {
            case kJobW1Nosec: NQS_ITEM(1, true, false, P, false); break;
            case kJobW1S32: NQS_ITEM(1, true, true, P, false); break;
            case kJobW1S64: NQS_ITEM(1, false, true, P, false); break;
            case kJobW2Nosec: NQS_ITEM(2, true, false, P, false); break;
            case kJobW2S32: NQS_ITEM(2, true, true, P, false); break;
            case kJobW2S64: NQS_ITEM(2, false, true, P, false); break;
            case kJobW1S32 + kJobIntegrals: NQS_ITEM(1, true, true, NQS_FP64, true); break;
            case kJobW2S32 + kJobIntegrals: NQS_ITEM(2, true, true, NQS_FP64, true); break;
            case kJobW2S64 + kJobIntegrals: NQS_ITEM(2, false, true, NQS_FP64, true); break;
            default: break;
        }
#undef NQS_ITEM
    }
}

template <int P>
__global__ __launch_bounds__(256) void batch_finish_kernel(const JobDesc *__restrict__ jobs) {
    const JobDesc &J = jobs[blockIdx.y];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (static_cast<int64_t>(blockIdx.x) * blockDim.x >= J.n) return;  // whole block past the end
    const int64_t chunks = J.chunk_len > 0 ? J.n_chunks : 0;
    const bool integrals = (J.kind & kJobIntegrals) != 0;
    const bool en = J.strategy == kStrategyEnum;
    if (integrals) {
        if ((J.kind & 1) == 0)
            finish_one<1, false, NQS_FP64, true>(J.tab, J.sc, J.samples, J.n, chunks, en, J.eloc,
                                                 nullptr, nullptr, 0, i);
        else
            finish_one<2, false, NQS_FP64, true>(J.tab, J.sc, J.samples, J.n, chunks, en, J.eloc,
                                                 nullptr, nullptr, 0, i);
        return;
    }
    // the same diagonal evaluation as the single-launch finish kernels
    if (J.tab.diag_jtiles > 0) {
        const diag_v4i *tiles = reinterpret_cast<const diag_v4i *>(J.tab.diag_q8);
        if ((J.kind & 1) == 0) {
            Key<1> x;
            x.w[0] = i < J.n ? J.samples[2 * i] : 0ull;
            const double d = diag_occ_mfma<1>(J.tab, x, tiles);
            finish_one<1, false, P, false>(J.tab, J.sc, J.samples, J.n, chunks, en, J.eloc,
                                           nullptr, nullptr, 0, i, nullptr, nullptr, 0, nullptr,
                                           nullptr, true, d);
        } else {
            Key<2> x;
            x.w[0] = i < J.n ? J.samples[2 * i] : 0ull;
            x.w[1] = i < J.n ? J.samples[2 * i + 1] : 0ull;
            const double d = diag_occ_mfma<2>(J.tab, x, tiles);
            finish_one<2, false, P, false>(J.tab, J.sc, J.samples, J.n, chunks, en, J.eloc,
                                           nullptr, nullptr, 0, i, nullptr, nullptr, 0, nullptr,
                                           nullptr, true, d);
        }
        return;
    }
    __shared__ double stage[3 * kDiagLds];
    const double *dq = stage_diag_occ<P>(J.tab, stage);
    uint64_t *dz = reinterpret_cast<uint64_t *>(stage);
    double *dc = stage + 2 * kDiagLds;
    const int nd = dq ? -1 : stage_diagonal<P>(J.tab, dz, dc);
    const uint64_t *z = nd >= 0 ? dz : nullptr;
    if ((J.kind & 1) == 0)
        finish_one<1, false, P, false>(J.tab, J.sc, J.samples, J.n, chunks, en, J.eloc, nullptr,
                                       nullptr, 0, i, z, dc, nd, dq);
    else
        finish_one<2, false, P, false>(J.tab, J.sc, J.samples, J.n, chunks, en, J.eloc, nullptr,
                                       nullptr, 0, i, z, dc, nd, dq);
}

size_t batch_lds_bytes(int threads, int max_filter_log2) {
    return lookup_lds_bytes(false, max_filter_log2, threads);
}

namespace {
// The enumeration kernel of variant v = (words - 1) + 2 * integral form.
template <int P>
const void *enum_variant(int v) {
    switch (v) {
        case 0: return reinterpret_cast<const void *>(&batch_enum_kernel<1, P, false>);
        case 1: return reinterpret_cast<const void *>(&batch_enum_kernel<2, P, false>);
        case 2: return reinterpret_cast<const void *>(&batch_enum_kernel<1, NQS_FP64, true>);
        default: return reinterpret_cast<const void *>(&batch_enum_kernel<2, NQS_FP64, true>);
    }
}
}  // namespace

hipError_t prepare_batch_kernels() {
    static bool done = false;
    if (done) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&batch_lookup_kernel<NQS_FP64>),
        hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLookupLds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&batch_lookup_kernel<NQS_FP32_KAHAN>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLookupLds);
    for (int v = 0; v < kEnumVariants && e == hipSuccess; ++v) {
        e = hipFuncSetAttribute(enum_variant<NQS_FP64>(v),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kEnumDynLds);
        if (e == hipSuccess && v < 2)
            e = hipFuncSetAttribute(enum_variant<NQS_FP32_KAHAN>(v),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, kEnumDynLds);
    }
    if (e == hipSuccess) done = true;
    return e;
}

hipError_t launch_batch(const JobDesc *d_jobs, int n_jobs, const WorkItem *d_items, int n_items,
                        unsigned *d_next, const BatchShape &shape, int precision,
                        hipStream_t st, const JobDesc *h_jobs) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3((n_jobs + 63) / 64), dim3(64), 0, st, d_jobs,
                       n_jobs, d_next);
    hipLaunchKernelGGL(batch_clear_kernel,
                       dim3(static_cast<unsigned>((shape.max_clear + 255) / 256), n_jobs),
                       dim3(256), 0, st, d_jobs);
    // the pair join's grouping and decision for the jobs that plan it
    // (the same kernels as a single launch; the build and the persistent
    // kernels below skip a job the join takes)
    for (int k = 0; h_jobs && k < n_jobs; ++k) {
        const JobDesc &J = h_jobs[k];
        if (!J.sc.jctl || J.n == 0) continue;
        const hipError_t e = launch_join_prep(J.tab, J.sc, J.samples, J.weights, J.n,
                                              J.tab.n_groups - (J.tab.has_diagonal ? 1 : 0),
                                              false, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(batch_build_kernel,
                       dim3(static_cast<unsigned>((shape.max_n + 255) / 256), n_jobs), dim3(256),
                       0, st, d_jobs);
    const size_t lds = batch_lds_bytes(shape.threads, shape.max_filter_log2);
    const hipError_t pe = prepare_batch_kernels();
    if (pe != hipSuccess) return pe;
    // items [enum_begin[v], enum_begin[v + 1]) are the enumeration rounds of
    // variant v; the streaming items follow
    const bool f32 = precision == NQS_FP32_KAHAN;
    for (int v = 0; v < kEnumVariants; ++v) {
        const int b0 = shape.enum_begin[v], cnt = shape.enum_begin[v + 1] - b0;
        if (cnt <= 0) continue;
        const WorkItem *it = d_items + b0;
        unsigned *nx = d_next + v;
#define NQS_EB(Wd, Pr, SCI)                                                                    \
    hipLaunchKernelGGL((batch_enum_kernel<Wd, Pr, SCI>), dim3(shape.enum_blocks),               \
                       dim3(kEnumThreads), kEnumDynLds, st, d_jobs, it, cnt, nx)
        switch (v) {
            case 0: if (f32) NQS_EB(1, NQS_FP32_KAHAN, false); else NQS_EB(1, NQS_FP64, false); break;
            case 1: if (f32) NQS_EB(2, NQS_FP32_KAHAN, false); else NQS_EB(2, NQS_FP64, false); break;
            case 2: NQS_EB(1, NQS_FP64, true); break;
            default: NQS_EB(2, NQS_FP64, true); break;
        }
#undef NQS_EB
    }
    for (int k = 0; h_jobs && k < n_jobs; ++k) {
        const JobDesc &J = h_jobs[k];
        if (!J.sc.jctl || J.n == 0) continue;
        const int pr = (J.kind & kJobIntegrals) ? NQS_FP64 : precision;
        const hipError_t e = launch_join_pairs(J.tab, J.sc, J.samples, J.weights, 0, J.log_amp,
                                               J.phase, J.n, pr, nullptr, nullptr, 0, st);
        if (e != hipSuccess) return e;
    }
    const int ne = shape.enum_begin[kEnumVariants];
    const WorkItem *s_items = d_items + ne;
    const int ns = n_items - ne;
    const dim3 fgrid(static_cast<unsigned>((shape.max_n + 255) / 256), n_jobs);
    if (f32) {
        if (ns > 0)
            hipLaunchKernelGGL(batch_lookup_kernel<NQS_FP32_KAHAN>, dim3(shape.lookup_blocks),
                               dim3(shape.threads), lds, st, d_jobs, s_items, ns,
                               d_next + kStreamCounter);
        hipLaunchKernelGGL(batch_finish_kernel<NQS_FP32_KAHAN>, fgrid, dim3(256), 0, st, d_jobs);
    } else {
        if (ns > 0)
            hipLaunchKernelGGL(batch_lookup_kernel<NQS_FP64>, dim3(shape.lookup_blocks),
                               dim3(shape.threads), lds, st, d_jobs, s_items, ns,
                               d_next + kStreamCounter);
        hipLaunchKernelGGL(batch_finish_kernel<NQS_FP64>, fgrid, dim3(256), 0, st, d_jobs);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ energy (Eq. 1)

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 256;

__device__ __forceinline__ double block_sum(double v, double *lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

// Eq. 1 in two launches.  Each block of the first takes a fixed strided set
// of samples: its sums W_b = sum w, sum w Re E, sum w Im E, its own mean m_b
// and M2_b = sum w |E - m_b|^2 about that mean (a second pass over the same
// samples, still in cache).  One block then combines the block partials in
// block order: the mean from the sums, and
//   sum_i w_i |E_i - mean|^2 = sum_b (M2_b + W_b |m_b - mean|^2),
// exact because each block's weighted deviations from its own mean sum to
// zero.  (Combining them in the first launch's last block would need a
// device-scope release fence in every block, which costs more than the
// launch on a chip of several L2s.)
__global__ __launch_bounds__(kRedThreads) void energy_block_kernel(
    const int64_t *__restrict__ w, const double *__restrict__ e, int64_t n,
    double *__restrict__ part) {
    __shared__ double lds[kRedThreads];
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kRedThreads + threadIdx.x;
    const int64_t step = static_cast<int64_t>(gridDim.x) * kRedThreads;
    double sw = 0.0, sr = 0.0, si = 0.0;
    for (int64_t i = i0; i < n; i += step) {
        const double wi = static_cast<double>(w[i]);
        sw += wi;
        sr += wi * e[2 * i];
        si += wi * e[2 * i + 1];
    }
    sw = block_sum(sw, lds);
    sr = block_sum(sr, lds);
    si = block_sum(si, lds);
    const double mr = sw != 0.0 ? sr / sw : 0.0, mi = sw != 0.0 ? si / sw : 0.0;
    double sv = 0.0;
    for (int64_t i = i0; i < n; i += step) {
        const double dr = e[2 * i] - mr, di = e[2 * i + 1] - mi;
        sv += static_cast<double>(w[i]) * (dr * dr + di * di);
    }
    sv = block_sum(sv, lds);
    if (threadIdx.x == 0) {
        double *pb = part + 4 * blockIdx.x;
        pb[0] = sw;
        pb[1] = sr;
        pb[2] = si;
        pb[3] = sv;
    }
}

// Single block: out = {mean re, mean im, variance, sum w} from nb block
// partials (thread t takes partials t, t + kRedThreads, ... in that order).
// out may be pinned host memory; with err, the device's error word is
// copied to *err_out beside it (the host reads both after one wait).
__global__ __launch_bounds__(kRedThreads) void energy_combine_kernel(
    const double *__restrict__ part, int64_t nb, double *__restrict__ out,
    const int *__restrict__ err, int *__restrict__ err_out, unsigned *__restrict__ seq,
    unsigned *__restrict__ seq_out, const unsigned long long *__restrict__ jctl,
    unsigned *__restrict__ chosen_out) {
    __shared__ double lds[kRedThreads];
    double bw = 0.0, br = 0.0, bi = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += kRedThreads) {
        bw += part[4 * b];
        br += part[4 * b + 1];
        bi += part[4 * b + 2];
    }
    const double SW = block_sum(bw, lds), SR = block_sum(br, lds), SI = block_sum(bi, lds);
    const double MR = SW != 0.0 ? SR / SW : 0.0, MI = SW != 0.0 ? SI / SW : 0.0;
    double c = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += kRedThreads) {
        const double w = part[4 * b];
        c += part[4 * b + 3];
        if (w != 0.0) {
            const double ur = part[4 * b + 1] / w - MR, ui = part[4 * b + 2] / w - MI;
            c += w * (ur * ur + ui * ui);
        }
    }
    const double SV = block_sum(c, lds);
    if (threadIdx.x == 0) {
        out[0] = MR;
        out[1] = MI;
        out[2] = SW != 0.0 ? SV / SW : 0.0;
        out[3] = SW;
        if (err) *err_out = *err;
        if (chosen_out) *chosen_out = jctl ? (jctl[kJoinCtlChosen] != 0ull ? 1u : 0u) : 2u;
        if (seq) {
            // a new sequence number, published after the results (system
            // scope: the host polls it)
            const unsigned v = *seq + 1u;
            *seq = v;
            __threadfence_system();
            *reinterpret_cast<volatile unsigned *>(seq_out) = v;
        }
    }
}

// ------------------------------------------------------------------ launchers



namespace {
int device_cus() {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cus[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        cus[dev] = v;
    }
    return cus[dev];
}
}  // namespace

EvalLaunch plan_eval(const DevTable &tab, int64_t n, bool dump, const Tuning *tune) {
    EvalLaunch L;
    L.n = n;
    const int want = tune ? tune->strategy : kStrategyAuto;
    L.strategy = (tab.enum_ok && want != kStrategyStream) ? kStrategyEnum : kStrategyStream;
    L.enum_blocks = static_cast<unsigned>(device_cus());
    L.threads = (tune && tune->threads) ? tune->threads : kLookupThreads;
    // Bloom bitmap: about 16 bits per sample unless tuned, 512 B .. 128 KB;
    // an enumeration whose batch outgrows one bitmap takes 32 bits per
    // sample in its class partitions
    int lg = 7;
    int64_t bits_per_sample = (tune && tune->filter_bits) ? tune->filter_bits : 16;
    if (!(tune && tune->filter_bits) && L.strategy == kStrategyEnum && 16 * n > (int64_t(1) << 20))
        bits_per_sample = 32;
    while (lg < 15 && (int64_t(1) << (lg + 5)) < bits_per_sample * n) ++lg;
    L.filter_log2 = lg;
    // enumeration filter: up to kEnumMaxParts partitions (sample classes) of
    // at most 128 KB each, so that every sample keeps its bits per sample
    int lp = 0;
    if (L.strategy == kStrategyEnum)
        while ((1 << lp) < kEnumMaxParts && (int64_t(1) << (lp + 20)) < bits_per_sample * n) ++lp;
    L.eparts_log2 = lp;
    if (lp == 0) {
        L.efilter_log2 = lg;
    } else {
        int le = 7;
        while (le < 15 && (int64_t(1) << (le + 5 + lp)) < bits_per_sample * n) ++le;
        L.efilter_log2 = le;
    }
    L.lds_bytes = lookup_lds_bytes(tab.sector32 != 0, lg, L.threads);
    L.g_first = tab.has_diagonal ? 1 : 0;
    const int64_t g_eff = tab.n_groups - L.g_first;
    const int64_t tiles = (n + L.threads - 1) / L.threads;
    int64_t chunks = 1;
    if (!dump && g_eff > 0) {
        const int64_t target = (tune && tune->blocks_per_cu) ? tune->blocks_per_cu : 4;
        const int64_t want = (target * 256 * 1024 / L.threads + tiles - 1) / tiles;
        const int64_t max_chunks = (g_eff + kStage - 1) / kStage;
        chunks = want < max_chunks ? want : max_chunks;
        if (chunks < 1) chunks = 1;
        if (chunks > 65535) chunks = 65535;
    }
    L.n_chunks = chunks;
    L.chunk_len = g_eff > 0 ? (g_eff + chunks - 1) / chunks : 0;
    // the pair join is launched beside the other strategy and decides on the
    // device whether it runs
    L.join = 0;
    L.join_force = 0;
    L.join_only = 0;
    L.join_log2m = 0;
    if (tab.join_blocks > 0 && (want == kStrategyAuto || want == kStrategyJoin) &&
        n <= kJoinMaxSamples) {
        L.join = 1;
        L.join_force = want == kStrategyJoin ? 1 : 0;
        L.join_log2m = join_log2m_for(n);
    }
    return L;
}

hipError_t launch_hash(const DevTable &tab, const DevScratch &sc, uint32_t capacity,
                       const uint64_t *samples, const int64_t *weights, int64_t n,
                       hipStream_t st, hipEvent_t after_grouping, bool join_only) {
    const int words = tab.n_qubits <= 63 ? 1 : 2;
    // with the pair join launched, its histogram kernel frees the hash slots
    // and clears the bitmaps in blocks of its own (the grouping does not use
    // them); this kernel then clears only the counters and control words
    const bool join = sc.jctl != nullptr;
    const uint32_t cap = join ? 0u : capacity;
    const uint32_t fwords = join ? 0u : 1u << sc.filter_log2;
    const uint32_t efwords =
        (join || sc.eparts_log2 <= 0) ? 0u : (1u << (sc.eparts_log2 + sc.efilter_log2));
    const uint32_t jparts = join ? static_cast<uint32_t>(sc.join_parts) : 0u;
    const uint32_t jhw = join ? static_cast<uint32_t>((tab.join_blocks * n + 31) / 32) : 0u;
    uint32_t span = cap > fwords ? cap : fwords;
    span = span > efwords ? span : efwords;
    span = span > jparts ? span : jparts;
    span = span > jhw ? span : jhw;
    const uint32_t n_counters = static_cast<uint32_t>(kCounters * kCounterSlots);
    span = span > n_counters ? span : n_counters;
    span = span > static_cast<uint32_t>(kJoinCtl) ? span : static_cast<uint32_t>(kJoinCtl);
    hipLaunchKernelGGL(hash_clear_kernel, dim3((span + 255) / 256), dim3(256), 0, st, sc.skey,
                       sc.sidx, sc.sfp, words, cap, sc.filter, fwords, sc.efilter, efwords,
                       sc.counters, sc.mixed, sc.jcnt, jparts, sc.jctl, sc.jhit, jhw);
    if (join) {
        // the pair join's grouping and decision come before the build, which
        // skips its insertion when the join runs
        const hipError_t e = launch_join_prep(tab, sc, samples, weights, n,
                                              tab.n_groups - (tab.has_diagonal ? 1 : 0),
                                              !join_only, st);
        if (e != hipSuccess) return e;
    }
    if (after_grouping) {
        const hipError_t e = hipEventRecord(after_grouping, st);
        if (e != hipSuccess) return e;
    }
    // with the join launched the build runs inside its pair kernel's launch
    if (join) return hipGetLastError();
    const dim3 grid(static_cast<unsigned>((n + 255) / 256));
    if (words == 1)
        hipLaunchKernelGGL(hash_build_kernel<1>, grid, dim3(256), 0, st, tab, sc, samples, weights, n);
    else
        hipLaunchKernelGGL(hash_build_kernel<2>, grid, dim3(256), 0, st, tab, sc, samples, weights, n);
    return hipGetLastError();
}

template <int W, bool S32, bool SEC, bool D, int P, bool SCV>
hipError_t launch_lookup(const DevTable &tab, const DevScratch &sc, const EvalLaunch &L,
                         const uint64_t *samples, const double *log_amp, const double *phase,
                         int32_t *hit_idx, uint32_t *sign_bits, int64_t sign_words,
                         int fallback_only, hipStream_t st) {
    static bool attr_set = false;
    if (!attr_set) {
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&eloc_lookup_kernel<W, S32, SEC, D, P, SCV>),
            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLookupLds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const dim3 grid(static_cast<unsigned>((L.n + L.threads - 1) / L.threads),
                    static_cast<unsigned>(L.n_chunks));
    hipLaunchKernelGGL((eloc_lookup_kernel<W, S32, SEC, D, P, SCV>), grid, dim3(L.threads), L.lds_bytes, st,
                       tab, sc, samples, log_amp, phase, L.n, L.g_first, L.chunk_len, hit_idx,
                       sign_bits, sign_words, fallback_only);
    return hipGetLastError();
}

template <int W, bool D, int P, bool SCV>
hipError_t launch_enum(const DevTable &tab, const DevScratch &sc, const EvalLaunch &L,
                       const uint64_t *samples, const double *log_amp, const double *phase,
                       int32_t *hit_idx, uint32_t *sign_bits, int64_t sign_words, hipStream_t st) {
    static bool attr_set = false;
    if (!attr_set) {
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&eloc_enum_kernel<W, D, P, SCV>),
            hipFuncAttributeMaxDynamicSharedMemorySize, kEnumDynLds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((eloc_enum_kernel<W, D, P, SCV>), dim3(L.enum_blocks), dim3(kEnumThreads),
                       kEnumDynLds, st, tab, sc, samples, log_amp, phase, L.n, hit_idx, sign_bits,
                       sign_words);
    return hipGetLastError();
}

// The finish kernel's dynamic LDS may pass 64 KB (a staged occupation form
// plus the threads' occupied-qubit lists): raise its limit once.
template <int W, bool D, int P>
hipError_t allow_finish_lds() {
    static bool done = false;
    if (done) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&eloc_finish_kernel<W, D, P, false>),
        hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    if (e == hipSuccess) done = true;
    return e;
}

hipError_t launch_eloc(const DevTable &tab, const DevScratch &sc, const EvalLaunch &L,
                       const uint64_t *samples, const int64_t *weights, const double *log_amp,
                       const double *phase, double *eloc, int precision, int32_t *hit_idx,
                       uint32_t *sign_bits, int64_t sign_words, EvalStageEvents ev,
                       EnergyFused ef, hipStream_t st) {
    const int words = tab.n_qubits <= 63 ? 1 : 2;
    const bool dump = hit_idx || sign_bits;
    const bool f32 = precision == NQS_FP32_KAHAN && !dump;
    const bool s32 = tab.sector32 != 0;
    const int64_t n = L.n;
    const bool en = L.strategy == kStrategyEnum;
    const int fb = en ? 1 : 0;
    hipError_t e = hipSuccess;
    if (sc.jctl) {
        // a dump marks every pair first; the join (or the enumeration) writes
        // only its hits
        if (hit_idx) {
            const int64_t cnt = n * tab.n_groups;
            hipLaunchKernelGGL(fill_i32_kernel, dim3(static_cast<unsigned>((cnt + 255) / 256)),
                               dim3(256), 0, st, hit_idx, cnt, -1);
        }
        // the hash build rides in the same launch (launch_hash left it out);
        // a join-only launch has none (its hash is not cleared, nothing would
        // read it, and the grouping made the sample checks)
        e = launch_join_pairs(tab, sc, samples, weights, L.join_only ? 0 : 1, log_amp, phase, n,
                              precision, hit_idx, sign_bits, sign_words, st);
        if (e != hipSuccess) return e;
    }
    if (ev.after_pairs) {
        e = hipEventRecord(ev.after_pairs, st);
        if (e != hipSuccess) return e;
    }
    if (en && !L.join_only) {
        // a dump marks every pair first; the enumeration writes only its hits
        // (done above when a join was launched too)
        if (hit_idx && !sc.jctl) {
            const int64_t cnt = n * tab.n_groups;
            hipLaunchKernelGGL(fill_i32_kernel, dim3(static_cast<unsigned>((cnt + 255) / 256)),
                               dim3(256), 0, st, hit_idx, cnt, -1);
        }
#define NQS_ENUM(Wd, D, Pr, SCI) \
    e = launch_enum<Wd, D, Pr, SCI>(tab, sc, L, samples, log_amp, phase, hit_idx, sign_bits, \
                                    sign_words, st)
        if (tab.sc) {
            if (words == 1) {
                if (dump) NQS_ENUM(1, true, NQS_FP64, true); else NQS_ENUM(1, false, NQS_FP64, true);
            } else {
                if (dump) NQS_ENUM(2, true, NQS_FP64, true); else NQS_ENUM(2, false, NQS_FP64, true);
            }
        } else if (words == 1) {
            if (dump) NQS_ENUM(1, true, NQS_FP64, false);
            else if (f32) NQS_ENUM(1, false, NQS_FP32_KAHAN, false);
            else NQS_ENUM(1, false, NQS_FP64, false);
        } else {
            if (dump) NQS_ENUM(2, true, NQS_FP64, false);
            else if (f32) NQS_ENUM(2, false, NQS_FP32_KAHAN, false);
            else NQS_ENUM(2, false, NQS_FP64, false);
        }
#undef NQS_ENUM
        if (e != hipSuccess) return e;
    }
    if (L.chunk_len > 0 && !L.join_only) {
#define NQS_LOOKUP(Wd, S, SE, D, Pr)                                                       \
    e = launch_lookup<Wd, S, SE, D, Pr, false>(tab, sc, L, samples, log_amp, phase, hit_idx,  \
                                               sign_bits, sign_words, fb, st)
#define NQS_LOOKUP_D(Wd, S, SE)                      \
    if (dump) NQS_LOOKUP(Wd, S, SE, true, NQS_FP64);  \
    else if (f32) NQS_LOOKUP(Wd, S, SE, false, NQS_FP32_KAHAN); \
    else NQS_LOOKUP(Wd, S, SE, false, NQS_FP64)
        // the sector test needs spin masks (and, checked on the device, one
        // (N_alpha, N_beta) over the batch)
        const bool sec = tab.sector_filter != 0;
        if (tab.sc) {
#define NQS_LOOKUP_SC(Wd, S, D) \
    e = launch_lookup<Wd, S, true, D, NQS_FP64, true>(tab, sc, L, samples, log_amp, phase, \
                                                     hit_idx, sign_bits, sign_words, fb, st)
            if (words == 1) {
                if (dump) NQS_LOOKUP_SC(1, true, true); else NQS_LOOKUP_SC(1, true, false);
            } else if (s32) {
                if (dump) NQS_LOOKUP_SC(2, true, true); else NQS_LOOKUP_SC(2, true, false);
            } else {
                if (dump) NQS_LOOKUP_SC(2, false, true); else NQS_LOOKUP_SC(2, false, false);
            }
#undef NQS_LOOKUP_SC
        } else if (words == 1) {
            if (!sec) { NQS_LOOKUP_D(1, true, false); }
            else if (s32) { NQS_LOOKUP_D(1, true, true); }
            else { NQS_LOOKUP_D(1, false, true); }
        } else {
            if (!sec) { NQS_LOOKUP_D(2, true, false); }
            else if (s32) { NQS_LOOKUP_D(2, true, true); }
            else { NQS_LOOKUP_D(2, false, true); }
        }
#undef NQS_LOOKUP_D
#undef NQS_LOOKUP
        if (e != hipSuccess) return e;
    }
    if (ev.after_lookup) {
        e = hipEventRecord(ev.after_lookup, st);
        if (e != hipSuccess) return e;
    }
    const int64_t chunks = L.chunk_len > 0 ? L.n_chunks : 0;
    const dim3 fgrid(static_cast<unsigned>((n + 255) / 256));
    // the occupation form staged whole when it fits 64 KB (100 qubits: 40 KB)
    const int occ_cnt = 1 + tab.n_qubits + tab.n_qubits * (tab.n_qubits - 1) / 2;
    const int stage_cap = (tab.diag_occ && occ_cnt > 3 * kDiagLds && occ_cnt * 8 <= 65536)
                              ? occ_cnt : 3 * kDiagLds;
    // and, after it, each thread's list of occupied qubits (bytes, 4 a word)
    const int list_words = tab.diag_occ ? (tab.n_qubits + 3) / 4 : 0;
    const size_t stage_bytes =
        (dump || tab.sc) ? 0
                         : sizeof(double) * stage_cap + (f32 ? size_t(256) * 4 * list_words : 0);
    if (!dump && !tab.sc && tab.diag_jtiles > 0) {
        // the occupation-form diagonal on the matrix cores
        // 1024-thread blocks once they fill every CU (each block stages the
        // digit tiles once), else 256-thread blocks to spread a small batch
        const int mth = n >= 256 * int64_t(kFinishMfmaThreads) ? kFinishMfmaThreads : 256;
        const dim3 mgrid(static_cast<unsigned>((n + mth - 1) / mth));
        const dim3 mblk(mth);
        if (words == 1) {
            if (f32)
                hipLaunchKernelGGL((eloc_finish_mfma_kernel<1, NQS_FP32_KAHAN>), mgrid, mblk, 0,
                                   st, tab, sc, samples, n, chunks, fb, eloc, ef.weights, ef.part);
            else
                hipLaunchKernelGGL((eloc_finish_mfma_kernel<1, NQS_FP64>), mgrid, mblk, 0, st, tab,
                                   sc, samples, n, chunks, fb, eloc, ef.weights, ef.part);
        } else {
            if (f32)
                hipLaunchKernelGGL((eloc_finish_mfma_kernel<2, NQS_FP32_KAHAN>), mgrid, mblk, 0,
                                   st, tab, sc, samples, n, chunks, fb, eloc, ef.weights, ef.part);
            else
                hipLaunchKernelGGL((eloc_finish_mfma_kernel<2, NQS_FP64>), mgrid, mblk, 0, st, tab,
                                   sc, samples, n, chunks, fb, eloc, ef.weights, ef.part);
        }
        if (ev.after_finish && (e = hipEventRecord(ev.after_finish, st)) != hipSuccess) return e;
        if (ef.part)
            hipLaunchKernelGGL(energy_combine_kernel, dim3(1), dim3(kRedThreads), 0, st, ef.part,
                               static_cast<int64_t>(mgrid.x), ef.out, sc.err, ef.err_out, ef.seq,
                               ef.seq_out, sc.jctl, ef.chosen_out);
        return hipGetLastError();
    }
    // (the energy partials only where no dump is taken)
    double *const ep = dump ? nullptr : ef.part;
#define NQS_FINISH(Wd, D, Pr)                                                                 \
    do {                                                                                      \
        if ((e = allow_finish_lds<Wd, D, Pr>()) != hipSuccess) return e;                     \
        hipLaunchKernelGGL((eloc_finish_kernel<Wd, D, Pr, false>), fgrid, dim3(256),          \
                           stage_bytes, st, tab, sc, samples, n, chunks, fb, eloc, hit_idx,   \
                           sign_bits, sign_words, stage_cap, list_words, ef.weights, ep);     \
    } while (0)
#define NQS_FINISH_SC(Wd, D)                                                                     \
    hipLaunchKernelGGL((eloc_finish_kernel<Wd, D, NQS_FP64, true>), fgrid, dim3(256), 0, st, tab, \
                       sc, samples, n, chunks, fb, eloc, hit_idx, sign_bits, sign_words, 0, 0,    \
                       ef.weights, ep)
    if (tab.sc) {
        if (words == 1) {
            if (dump) NQS_FINISH_SC(1, true); else NQS_FINISH_SC(1, false);
        } else {
            if (dump) NQS_FINISH_SC(2, true); else NQS_FINISH_SC(2, false);
        }
    } else if (words == 1) {
        if (dump) NQS_FINISH(1, true, NQS_FP64);
        else if (f32) NQS_FINISH(1, false, NQS_FP32_KAHAN);
        else NQS_FINISH(1, false, NQS_FP64);
    } else {
        if (dump) NQS_FINISH(2, true, NQS_FP64);
        else if (f32) NQS_FINISH(2, false, NQS_FP32_KAHAN);
        else NQS_FINISH(2, false, NQS_FP64);
    }
#undef NQS_FINISH
#undef NQS_FINISH_SC
    if (ev.after_finish && (e = hipEventRecord(ev.after_finish, st)) != hipSuccess) return e;
    if (ep)
        hipLaunchKernelGGL(energy_combine_kernel, dim3(1), dim3(kRedThreads), 0, st, ep,
                           static_cast<int64_t>(fgrid.x), ef.out, sc.err, ef.err_out, ef.seq,
                           ef.seq_out, sc.jctl, ef.chosen_out);
    return hipGetLastError();
}

hipError_t launch_energy(const int64_t *w, const double *e, int64_t n, double *part,
                         double *out, hipStream_t st) {
    int64_t blocks = (n + kRedThreads - 1) / kRedThreads;
    if (blocks > kRedBlocks) blocks = kRedBlocks;
    if (blocks < 1) blocks = 1;
    static_assert(4 * kRedBlocks <= kEnergyPartDoubles, "the block partials fit");
    hipLaunchKernelGGL(energy_block_kernel, dim3(blocks), dim3(kRedThreads), 0, st, w, e, n, part);
    hipLaunchKernelGGL(energy_combine_kernel, dim3(1), dim3(kRedThreads), 0, st, part, blocks, out,
                       nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    return hipGetLastError();
}

}  // namespace nqs
