// Device helpers shared by the kernel translation units: sample keys,
// the linear hash and Bloom bits, the bucketed sample hash, the group
// index, group term sums (FP64 and FP32 with compensation), the
// Slater-Condon element and the FP32 amplitude ratio.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/nqs.h"
#include "nqs_device.hpp"

namespace nqs {

// ------------------------------------------------------------------ helpers

template <int W>
struct Key {
    uint64_t w[W];
};

template <int W>
__device__ __forceinline__ Key<W> load_key(const uint64_t *__restrict__ p, int64_t i) {
    Key<W> k;
#pragma unroll
    for (int q = 0; q < W; ++q) k.w[q] = p[2 * i + q];
    return k;
}

template <int W>
__device__ __forceinline__ uint32_t linear_hash(const Key<W> &k, const uint32_t *__restrict__ hr) {
    uint32_t h = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        uint64_t v = k.w[q];
        while (v) {
            h ^= hr[64 * q + __builtin_ctzll(v)];
            v &= v - 1;
        }
    }
    return h;
}

// Bits of x selected by (m0, m1), packed to the low end in mask order.
template <int W>
__device__ __forceinline__ uint64_t compress(const Key<W> &x, uint64_t m0, uint64_t m1) {
    uint64_t r = 0;
    int k = 0;
    while (m0) {
        const int b = __builtin_ctzll(m0);
        r |= ((x.w[0] >> b) & 1ull) << k++;
        m0 &= m0 - 1;
    }
    if constexpr (W == 2) {
        while (m1) {
            const int b = __builtin_ctzll(m1);
            r |= ((x.w[1] >> b) & 1ull) << k++;
            m1 &= m1 - 1;
        }
    }
    return r;
}

__device__ __forceinline__ uint32_t slot_of(uint32_t h, uint32_t shift) {
    return (h * kGoldenMul) >> shift;
}

// One bucket of the sample hash: 64 bytes of keys (8 one-word or 4
// two-word), four independent 16-byte loads.
struct Bucket {
    uint4 q0, q1, q2, q3;
};

template <int W>
__device__ __forceinline__ Bucket bucket_load(const uint64_t *__restrict__ skey, uint32_t start) {
    const uint4 *p = reinterpret_cast<const uint4 *>(skey + static_cast<size_t>(start) * W);
    return Bucket{p[0], p[1], p[2], p[3]};
}

// Slot of the bucket holding k (or -1), and whether the bucket has a free
// slot.  Occupied slots form a prefix of a bucket (a key takes the first
// free slot from its start on, and nothing is removed), so the bucket is
// open iff its last slot is free; a key is stored once, so any slot that
// matches is the one.  The common case (no match) costs one XOR-OR per key
// word and a minimum.
template <int W>
__device__ __forceinline__ uint32_t slot_diff(const Bucket &b, int s, const Key<W> &k) {
    // zero iff slot s holds k (s a compile-time constant after unrolling)
    const uint32_t k0l = static_cast<uint32_t>(k.w[0]), k0h = static_cast<uint32_t>(k.w[0] >> 32);
    if constexpr (W == 1) {
        const uint4 &v = (s >> 1) == 0 ? b.q0 : (s >> 1) == 1 ? b.q1 : (s >> 1) == 2 ? b.q2 : b.q3;
        return (s & 1) ? ((v.z ^ k0l) | (v.w ^ k0h)) : ((v.x ^ k0l) | (v.y ^ k0h));
    } else {
        const uint32_t k1l = static_cast<uint32_t>(k.w[1]), k1h = static_cast<uint32_t>(k.w[1] >> 32);
        const uint4 &v = s == 0 ? b.q0 : s == 1 ? b.q1 : s == 2 ? b.q2 : b.q3;
        return (v.x ^ k0l) | (v.y ^ k0h) | (v.z ^ k1l) | (v.w ^ k1h);
    }
}

template <int W>
__device__ __forceinline__ int bucket_scan(const Bucket &b, const Key<W> &k, bool &empty) {
    constexpr int BK = 1 << bucket_log2(W);
    // the last slot's key (its last word) is the bucket's last word
    empty = (b.q3.z & b.q3.w) == 0xFFFFFFFFu;
    uint32_t m = slot_diff<W>(b, 0, k);
#pragma unroll
    for (int s = 1; s < BK; ++s) m = min(m, slot_diff<W>(b, s, k));
    if (m != 0u) return -1;
    // a match (rare): which slot
    int found = 0;
#pragma unroll
    for (int s = BK - 1; s > 0; --s)
        if (slot_diff<W>(b, s, k) == 0u) found = s;
    return found;
}

// Index of key k in the sample hash, or -1, with the bucket at start already
// loaded (b); the index array is read only for the slot that holds the key.
template <int W>
__device__ __forceinline__ int32_t hash_find_from(const uint64_t *__restrict__ skey,
                                                  const int32_t *__restrict__ sidx, uint32_t mask,
                                                  uint32_t start, const Key<W> &k, Bucket b) {
    constexpr int BK = 1 << bucket_log2(W);
    for (uint32_t probe = 0; probe <= mask; probe += BK) {
        bool empty;
        const int found = bucket_scan<W>(b, k, empty);
        if (found >= 0) return sidx[(start + static_cast<uint32_t>(found)) & mask];
        if (empty) return -1;
        start = (start + BK) & mask;
        b = bucket_load<W>(skey, start);
    }
    return -1;
}

// Index of key in the sample hash, or -1 (one memory round trip per bucket).
template <int W>
__device__ __forceinline__ int32_t hash_find(const uint64_t *__restrict__ skey,
                                             const int32_t *__restrict__ sidx, uint32_t mask,
                                             uint32_t start, const Key<W> &k) {
    return hash_find_from<W>(skey, sidx, mask, start, k, bucket_load<W>(skey, start));
}

__device__ __forceinline__ void latch(int *err, int code) { atomicCAS(err, 0, code); }

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const uint64_t u = static_cast<uint64_t>(__double_as_longlong(v));
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(u), lane);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(u >> 32), lane);
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int lane) {
    const uint32_t lo = __shfl(static_cast<uint32_t>(v), lane);
    const uint32_t hi = __shfl(static_cast<uint32_t>(v >> 32), lane);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ double shfl_f64(double v, int lane) {
    return __longlong_as_double(static_cast<long long>(
        shfl_u64(static_cast<uint64_t>(__double_as_longlong(v)), lane)));
}

// Number of set bits of mask below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// Blocked Bloom filter of the sample hashes: a key with hash h sets two bits
// of one 32-bit word, word (h >> 2) & (words - 1) and bits (h >> 17) & 31 and
// (h >> 24) & 31 (disjoint ranges of h for filters of up to 2^15 words).  The
// byte offset of the word is h & ((words - 1) << 2), which folds into the
// XOR forming h; the shift by (h >> 24) reads byte 3 of h in place (a
// sub-dword operand), so a probe costs one shift less.
__device__ __forceinline__ uint32_t filter_word(uint32_t h, uint32_t wmask) {
    return (h >> 2) & wmask;
}
__device__ __forceinline__ uint32_t filter_bits(uint32_t h) {
    return (1u << ((h >> 17) & 31)) | (1u << ((h >> 24) & 31));
}
__device__ __forceinline__ uint32_t filter_test(uint32_t fw, uint32_t h) {
    return (fw >> ((h >> 17) & 31)) & (fw >> ((h >> 24) & 31)) & 1u;
}

template <int W, bool DUMP>
__device__ __forceinline__ double group_sum(const DevTable &tab, int64_t g, const Key<W> &x,
                                            uint32_t *__restrict__ sign_row,
                                            unsigned long long *terms) {
    const uint32_t t0 = tab.goff[g], t1 = tab.goff[g + 1];
    double s = 0.0;
    for (uint32_t t = t0; t < t1; ++t) {
        int par = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) par += __popcll(tab.tz[2 * static_cast<size_t>(t) + q] & x.w[q]);
        const double c = tab.tc[t];
        s += (par & 1) ? -c : c;
        if constexpr (DUMP) {
            if (sign_row && (par & 1)) atomicOr(&sign_row[t >> 5], 1u << (t & 31));
        }
    }
    *terms += t1 - t0;
    return s;
}

// ---- integral form (Slater-Condon rules, the evaluator of Sec. III-B)
//
// <bra|H|ket> from h_pq and the chemists' (pq|rs) for determinants that
// differ by at most two spin orbitals; ONV ordering, so a ladder operator on
// spin orbital j carries (-1)^(occupied orbitals below j).

template <int W>
__device__ __forceinline__ int parity_below(const Key<W> &s, int j) {
    int c;
    if (j < 64) {
        c = __popcll(s.w[0] & ((1ull << j) - 1ull));
    } else {
        c = __popcll(s.w[0]);
        if constexpr (W == 2) c += __popcll(s.w[1] & ((1ull << (j - 64)) - 1ull));
    }
    return c & 1;
}

template <int W>
__device__ __forceinline__ void flip_bit(Key<W> &s, int j) {
    if (W == 1 || j < 64)
        s.w[0] ^= 1ull << (j & 63);
    else
        s.w[W - 1] ^= 1ull << (j & 63);
}

template <int W>
__device__ __forceinline__ int lowest(const Key<W> &s) {
    if (s.w[0]) return __builtin_ctzll(s.w[0]);
    if constexpr (W == 2) return 64 + __builtin_ctzll(s.w[1]);
    return 127;
}

__device__ __forceinline__ double eri_at(const DevTable &tab, int p, int q, int r, int s) {
    const int64_t pq = p > q ? int64_t(p) * (p + 1) / 2 + q : int64_t(q) * (q + 1) / 2 + p;
    const int64_t rs = r > s ? int64_t(r) * (r + 1) / 2 + s : int64_t(s) * (s + 1) / 2 + r;
    return tab.sc_eri[pq > rs ? pq * (pq + 1) / 2 + rs : rs * (rs + 1) / 2 + pq];
}

template <int W>
__device__ __forceinline__ double sc_element(const DevTable &tab, const Key<W> &bra,
                                             const Key<W> &ket) {
    Key<W> A, I;
    int na = 0, ni = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        A.w[q] = bra.w[q] & ~ket.w[q];  // created
        I.w[q] = ket.w[q] & ~bra.w[q];  // annihilated
        na += __popcll(A.w[q]);
        ni += __popcll(I.w[q]);
    }
    if (na != ni) return 0.0;
    const int K = tab.sc_k;
    if (na == 1) {
        const int i = lowest<W>(I), a = lowest<W>(A);
        if ((i & 1) != (a & 1)) return 0.0;
        Key<W> st = ket;
        int sg = parity_below<W>(st, i);
        flip_bit<W>(st, i);
        sg ^= parity_below<W>(st, a);
        const int as = a >> 1, is = i >> 1;
        double v = tab.sc_h1[as * K + is];
        // spectators: occupied in ket, except i
#pragma unroll
        for (int q = 0; q < W; ++q) {
            uint64_t m = ket.w[q] & ~I.w[q];
            while (m) {
                const int j = 64 * q + __builtin_ctzll(m);
                m &= m - 1;
                const int js = j >> 1;
                v += eri_at(tab, as, is, js, js);
                if ((j & 1) == (i & 1)) v -= eri_at(tab, as, js, js, is);
            }
        }
        return sg ? -v : v;
    }
    if (na == 2) {
        const int i = lowest<W>(I), a = lowest<W>(A);
        Key<W> I2 = I, A2 = A;
        flip_bit<W>(I2, i);
        flip_bit<W>(A2, a);
        const int j = lowest<W>(I2), b = lowest<W>(A2);
        // |bra> = G a+_a a+_b a_j a_i |ket>
        Key<W> st = ket;
        int sg = parity_below<W>(st, i);
        flip_bit<W>(st, i);
        sg ^= parity_below<W>(st, j);
        flip_bit<W>(st, j);
        sg ^= parity_below<W>(st, b);
        flip_bit<W>(st, b);
        sg ^= parity_below<W>(st, a);
        double v = 0.0;
        if (((a ^ i) & 1) == 0 && ((b ^ j) & 1) == 0) v += eri_at(tab, a >> 1, i >> 1, b >> 1, j >> 1);
        if (((a ^ j) & 1) == 0 && ((b ^ i) & 1) == 0) v -= eri_at(tab, a >> 1, j >> 1, b >> 1, i >> 1);
        return sg ? -v : v;
    }
    return 0.0;
}

template <int W>
__device__ __forceinline__ double sc_diagonal(const DevTable &tab, const Key<W> &x) {
    const int K = tab.sc_k;
    double d = 0.0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        uint64_t m = x.w[q];
        while (m) {
            const int i = 64 * q + __builtin_ctzll(m);
            m &= m - 1;
            const int is = i >> 1;
            d += tab.sc_h1[is * K + is];
            // partners above i
            Key<W> rest;
#pragma unroll
            for (int r = 0; r < W; ++r) rest.w[r] = r < q ? 0ull : (r == q ? m : x.w[r]);
#pragma unroll
            for (int r = 0; r < W; ++r) {
                uint64_t m2 = rest.w[r];
                while (m2) {
                    const int j = 64 * r + __builtin_ctzll(m2);
                    m2 &= m2 - 1;
                    const int js = j >> 1;
                    d += eri_at(tab, is, is, js, js);
                    if ((i & 1) == (j & 1)) d -= eri_at(tab, is, js, js, is);
                }
            }
        }
    }
    return d;
}

// ---- FP32 form with compensation (precision NQS_FP32_KAHAN)
//
// Coefficients are stored as FP32 pairs hi + lo (lo = c - hi rounded), the
// sign (-1)^{popc(Z & x)} is applied by flipping sign bits, the hi parts
// are added with Knuth's error-free TwoSum and the lo parts and the TwoSum
// errors go into a compensation term; a product H * r keeps its rounding
// error through fma.  The per-sample value s + c is widened to FP64 only
// when it leaves the lane.

__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float bp = s - a;
    e = (a - (s - bp)) + (b - bp);
}

__device__ __forceinline__ float flip_sign(float v, int par) {
    return __uint_as_float(__float_as_uint(v) ^ (static_cast<uint32_t>(par & 1) << 31));
}

struct AccF32 {
    float s = 0.f, c = 0.f;
    __device__ __forceinline__ void add(float v, float err) {
        float t, e;
        two_sum(s, v, t, e);
        s = t;
        c += e + err;
    }
    __device__ __forceinline__ double value() const {
        return static_cast<double>(s) + static_cast<double>(c);
    }
};

template <int W>
__device__ __forceinline__ AccF32 group_sum_f32(const DevTable &tab, int64_t g, const Key<W> &x,
                                                unsigned long long *terms) {
    const uint32_t t0 = tab.goff[g], t1 = tab.goff[g + 1];
    AccF32 a;
    for (uint32_t t = t0; t < t1; ++t) {
        int par = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) par += __popcll(tab.tz[2 * static_cast<size_t>(t) + q] & x.w[q]);
        a.add(flip_sign(tab.tc32[2 * static_cast<size_t>(t)], par),
              flip_sign(tab.tc32[2 * static_cast<size_t>(t) + 1], par));
    }
    *terms += t1 - t0;
    return a;
}

// psi(x') / psi(x) in FP64 from the log-amplitude and phase differences,
// out of line: inlined into a kernel's partner or probe loop, the exp and
// sincos constants stay in registers across the whole loop and cost it
// waves per SIMD (the call is made only on a hit).
static __device__ __noinline__ double2 amp_ratio_f64(double da, double dphi) {
    double sn, cs;
    sincos(dphi, &sn, &cs);
    const double mag = exp(da);
    return make_double2(mag * cs, mag * sn);
}

// psi(x') / psi(x) in FP32 from the FP64 log-psi difference; the phase
// difference is reduced to (-pi, pi] in FP64 before rounding.
__device__ __forceinline__ void ratio_f32(double da, double dphi, float &rr, float &ri) {
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    dphi -= kTwoPi * rint(dphi / kTwoPi);
    const float mag = expf(static_cast<float>(da));
    float sn, cs;
    sincosf(static_cast<float>(dphi), &sn, &cs);
    rr = mag * cs;
    ri = mag * sn;
}

// Index of the group with flip mask X, or -1 (the group index is keyed by
// h(X), which the caller has: h(x') ^ h(x)).
template <int W>
__device__ __forceinline__ int64_t group_find(const DevTable &tab, uint32_t hX, const Key<W> &X) {
    const uint32_t mask = 0xFFFFFFFFu >> tab.gh_shift;
    uint32_t slot = slot_of(hX, tab.gh_shift);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const uint32_t g = tab.gh[slot];
        if (g == 0xFFFFFFFFu) return -1;
        bool eq = tab.gx[2 * static_cast<size_t>(g)] == X.w[0];
        if constexpr (W == 2) eq = eq && tab.gx[2 * static_cast<size_t>(g) + 1] == X.w[1];
        if (eq) return g;
        slot = (slot + 1) & mask;
    }
    return -1;
}

// ------------------------------------------------------------------ hash build

// One thread per sample: range check, sector uniformity, counts >= 0, linear
// hash, Bloom bit, and insertion by CAS on the slot index.  A duplicate key
// is found by comparing against the sample that owns the slot.  With the
// pair join chosen only the checks run.
template <int W>
__device__ __forceinline__ void hash_build_one(const DevTable &tab, const DevScratch &sc,
                                               const uint64_t *__restrict__ samples,
                                               const int64_t *__restrict__ weights, int64_t i) {
    const uint64_t w0 = samples[2 * i], w1 = samples[2 * i + 1];
    bool bad;
    const int nq = tab.n_qubits;
    if (nq >= 64) {
        bad = (nq - 64 < 64) && ((w1 >> (nq - 64)) != 0);
    } else {
        bad = ((w0 >> nq) != 0) || (w1 != 0);
    }
    if (bad) latch(sc.err, NQS_E_RANGE);
    if (weights && weights[i] < 0) latch(sc.err, NQS_E_RANGE);
    if (tab.sector_filter) {
        const uint64_t s0 = samples[0], s1 = samples[1];
        const int na = __popcll(w0 & tab.spin_a0) + __popcll(w1 & tab.spin_a1);
        const int nb = __popcll(w0 & tab.spin_b0) + __popcll(w1 & tab.spin_b1);
        const int ra = __popcll(s0 & tab.spin_a0) + __popcll(s1 & tab.spin_a1);
        const int rb = __popcll(s0 & tab.spin_b0) + __popcll(s1 & tab.spin_b1);
        if (na != ra || nb != rb) atomicOr(sc.mixed, 1);
    }
    // the pair join, when it runs, needs neither the hash nor the filters
    if (join_chosen(sc) || bad) return;
    Key<W> k;
    k.w[0] = w0;
    if constexpr (W == 2) k.w[1] = w1;
    const uint32_t h = linear_hash<W>(k, tab.hr);
    sc.shx[i] = h;
    const uint32_t fmask = (1u << sc.filter_log2) - 1u;
    const uint32_t fbits = filter_bits(h);
    atomicOr(&sc.filter[filter_word(h, fmask)], fbits);
    if (sc.eparts_log2 > 0) {
        // the partition of the enumeration filter: class of x, the XOR of
        // the classes of its occupied beta qubits
        uint32_t c = 0;
        uint64_t m0 = w0 & tab.spin_b0, m1 = w1 & tab.spin_b1;
        while (m0) {
            c ^= tab.qcls[__builtin_ctzll(m0)];
            m0 &= m0 - 1;
        }
        while (m1) {
            c ^= tab.qcls[64 + __builtin_ctzll(m1)];
            m1 &= m1 - 1;
        }
        c &= (1u << sc.eparts_log2) - 1u;
        const uint32_t emask = (1u << sc.efilter_log2) - 1u;
        atomicOr(&sc.efilter[(c << sc.efilter_log2) + filter_word(h, emask)], fbits);
    }
    uint32_t slot = slot_of(h, sc.slot_shift) << bucket_log2(W);
    for (uint32_t probe = 0; probe <= sc.slot_mask; ++probe) {
        const int32_t old = atomicCAS(&sc.sidx[slot], -1, static_cast<int32_t>(i));
        if (old == -1) {
            sc.skey[static_cast<size_t>(slot) * W] = w0;
            if constexpr (W == 2) sc.skey[static_cast<size_t>(slot) * W + 1] = w1;
            sc.sfp[slot] = h | 1u;
            return;
        }
        bool same = samples[2 * old] == w0;
        if constexpr (W == 2) same = same && samples[2 * old + 1] == w1;
        if (same) {
            latch(sc.err, NQS_E_DUPLICATE);
            return;
        }
        slot = (slot + 1) & sc.slot_mask;
    }
}

}  // namespace nqs
