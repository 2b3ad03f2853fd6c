// HIP kernels (gfx950) for the sample-space local energy.
//
//   E_loc(x) = sum_{x' in S} <x|H|x'> psi(x') / psi(x)           (Eq. 5)
//
// The per-sample outer loop of the multi-level scheme (Eq. 6, Alg. 3) is the
// GPU grid: one lane owns one sample x and keeps it in registers.  The inner
// loop over kets runs over the X groups of the Pauli table instead of over
// determinants: every term of group g connects x to x' = x ^ X_g, so one
// lookup of x' in the sample hash (the psi lookup table of the sample-space
// energy) decides the whole group.  The group stream is wave-uniform, so it
// reaches the lanes through scalar loads.  A lookup hit evaluates
//   <x|H|x'> = sum_{t in g} c~_t (-1)^{popc(Z_t & x)}
// with the folded coefficient c~ = c (-1)^{ny/2}, and multiplies it by
// exp(a' - a) e^{i(phi' - phi)}.
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

__device__ __forceinline__ uint32_t slot_of(uint32_t h, uint32_t shift) {
    return (h * kGoldenMul) >> shift;
}

template <int W>
struct SlotT;
template <>
struct SlotT<1> {
    using type = Slot1;
};
template <>
struct SlotT<2> {
    using type = Slot2;
};

template <int W>
__device__ __forceinline__ bool key_eq(const typename SlotT<W>::type &s, const Key<W> &k) {
    if constexpr (W == 1) {
        return s.k0 == k.w[0];
    } else {
        return s.k0 == k.w[0] && s.k1 == k.w[1];
    }
}

// Index of key in the sample hash, or -1.
template <int W>
__device__ __forceinline__ int32_t hash_find(const typename SlotT<W>::type *__restrict__ slots,
                                             uint32_t mask, uint32_t slot, const Key<W> &k) {
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const typename SlotT<W>::type s = slots[slot];
        if (s.idx < 0) return -1;
        if (key_eq<W>(s, k)) return s.idx;
        slot = (slot + 1) & mask;
    }
    return -1;
}

__device__ __forceinline__ void latch(int *err, int code) { atomicCAS(err, 0, code); }

// ------------------------------------------------------------------ hash build

__global__ void hash_clear_kernel(int32_t *__restrict__ idx_words, int stride_words,
                                  uint32_t capacity) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < capacity) idx_words[static_cast<size_t>(s) * stride_words] = -1;
}

// One thread per sample: range check, sector uniformity, counts >= 0, linear
// hash, and insertion by CAS on the slot index.  A duplicate key is found
// by comparing against the sample that owns the slot.
template <int W>
__global__ void hash_build_kernel(DevTable tab, DevScratch sc,
                                  const uint64_t *__restrict__ samples,
                                  const int64_t *__restrict__ weights, int64_t n) {
    using S = typename SlotT<W>::type;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t w0 = samples[2 * i], w1 = samples[2 * i + 1];
    // bits at or above n_qubits
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
    Key<W> k;
    k.w[0] = w0;
    if constexpr (W == 2) k.w[1] = w1;
    if (W == 1 && w1 != 0) return;  // already latched as out of range
    const uint32_t h = linear_hash<W>(k, tab.hr);
    sc.shx[i] = h;
    S *slots = static_cast<S *>(sc.slots);
    uint32_t slot = slot_of(h, sc.slot_shift);
    for (uint32_t probe = 0; probe <= sc.slot_mask; ++probe) {
        const int32_t old = atomicCAS(&slots[slot].idx, -1, static_cast<int32_t>(i));
        if (old == -1) {
            slots[slot].k0 = w0;
            if constexpr (W == 2) slots[slot].k1 = w1;
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

// ------------------------------------------------------------------ E_loc

constexpr int kProbeThreads = 256;

// Sum of one group's terms for bra x: sum_t c~_t (-1)^{popc(Z_t & x)}.
template <int W, bool DUMP>
__device__ __forceinline__ double group_sum(const DevTable &tab, int64_t g, const Key<W> &x,
                                            uint8_t *__restrict__ sign_row,
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
            if (par & 1) sign_row[t >> 3] |= static_cast<uint8_t>(1u << (t & 7));
        }
    }
    *terms += t1 - t0;
    return s;
}

// Grid: (sample tiles of 256) x (group chunks).  Each lane walks the groups of
// its chunk in order and writes one partial sum, so the result does not
// depend on scheduling.  The X = 0 group is left to the finish kernel.
template <int W, bool DUMP>
__global__ __launch_bounds__(kProbeThreads) void eloc_probe_kernel(
    DevTable tab, DevScratch sc, const uint64_t *__restrict__ samples,
    const double *__restrict__ log_amp, const double *__restrict__ phase, int64_t n,
    int64_t g_first, int64_t chunk_len, int32_t *__restrict__ hit_idx,
    uint8_t *__restrict__ sign_bits, int64_t sign_stride) {
    using S = typename SlotT<W>::type;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kProbeThreads + threadIdx.x;
    const bool active = i < n;
    const int64_t chunk = blockIdx.y;
    const int64_t g0 = g_first + chunk * chunk_len;
    const int64_t g1 = min(g0 + chunk_len, tab.n_groups);
    const bool filter = tab.sector_filter && (*sc.mixed == 0);
    const S *__restrict__ slots = static_cast<const S *>(sc.slots);

    Key<W> x;
    uint32_t hx = 0;
    double la = 0.0, ph = 0.0;
    if (active) {
        x = load_key<W>(samples, i);
        hx = sc.shx[i];
        la = log_amp[i];
        ph = phase[i];
    } else {
#pragma unroll
        for (int q = 0; q < W; ++q) x.w[q] = 0;
    }
    uint8_t *sign_row = DUMP && active && sign_bits ? sign_bits + i * sign_stride : nullptr;

    double acc_re = 0.0, acc_im = 0.0;
    unsigned long long n_probe = 0, n_hit = 0, n_terms = 0;
    for (int64_t g = g0; g < g1; ++g) {
        bool ok = active;
        if (filter) {
            int ca = 0, cb = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                ca += __popcll(x.w[q] & tab.gxa[2 * g + q]);
                cb += __popcll(x.w[q] & tab.gxb[2 * g + q]);
            }
            const uint32_t meta = tab.gmeta[g];
            ok = ok && ((static_cast<uint32_t>(ca) | (static_cast<uint32_t>(cb) << 8)) ==
                        (meta & 0xFFFFu)) && !(meta & kMetaInfeasibleBit);
        }
        int32_t j = -1;
        if (ok) {
            ++n_probe;
            Key<W> xp;
#pragma unroll
            for (int q = 0; q < W; ++q) xp.w[q] = x.w[q] ^ tab.gx[2 * g + q];
            const uint32_t h = hx ^ tab.ghx[g];
            j = hash_find<W>(slots, sc.slot_mask, slot_of(h, sc.slot_shift), xp);
            if (j >= 0) {
                ++n_hit;
                const double hsum = group_sum<W, DUMP>(tab, g, x, sign_row, &n_terms);
                double sn, cs;
                sincos(phase[j] - ph, &sn, &cs);
                const double mag = exp(log_amp[j] - la);
                acc_re += hsum * (mag * cs);
                acc_im += hsum * (mag * sn);
            }
        }
        if constexpr (DUMP) {
            if (active && hit_idx) hit_idx[i * tab.n_groups + g] = j;
        }
    }
    if (active) {
        double *p = sc.part + 2 * (chunk * n + i);
        p[0] = acc_re;
        p[1] = acc_im;
    }
    // counters: one atomic per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        n_probe += __shfl_xor(n_probe, off);
        n_hit += __shfl_xor(n_hit, off);
        n_terms += __shfl_xor(n_terms, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&sc.counters[1], n_probe);
        atomicAdd(&sc.counters[2], n_hit);
        atomicAdd(&sc.counters[3], n_terms);
    }
}

// E_loc(x) = diagonal group sum + sum of the chunk partials in chunk order.
template <int W, bool DUMP>
__global__ __launch_bounds__(256) void eloc_finish_kernel(
    DevTable tab, DevScratch sc, const uint64_t *__restrict__ samples, int64_t n,
    int64_t n_chunks, double *__restrict__ eloc, int32_t *__restrict__ hit_idx,
    uint8_t *__restrict__ sign_bits, int64_t sign_stride) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    unsigned long long n_terms = 0;
    if (i < n) {
        const Key<W> x = load_key<W>(samples, i);
        double re = 0.0, im = 0.0;
        if (tab.has_diagonal) {
            uint8_t *sign_row = DUMP && sign_bits ? sign_bits + i * sign_stride : nullptr;
            re = group_sum<W, DUMP>(tab, 0, x, sign_row, &n_terms);
            if constexpr (DUMP) {
                if (hit_idx) hit_idx[i * tab.n_groups] = static_cast<int32_t>(i);
            }
        }
        for (int64_t c = 0; c < n_chunks; ++c) {
            const double *p = sc.part + 2 * (c * n + i);
            re += p[0];
            im += p[1];
        }
        eloc[2 * i] = re;
        eloc[2 * i + 1] = im;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n_terms += __shfl_xor(n_terms, off);
    if ((threadIdx.x & 63) == 0 && n_terms) atomicAdd(&sc.counters[3], n_terms);
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

// Pass 1: per-block sum w, sum w Re E, sum w Im E over a fixed strided set.
__global__ __launch_bounds__(kRedThreads) void energy_pass1_kernel(
    const int64_t *__restrict__ w, const double *__restrict__ e, int64_t n,
    double *__restrict__ part) {
    __shared__ double lds[kRedThreads];
    double sw = 0.0, sr = 0.0, si = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRedThreads + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRedThreads) {
        const double wi = static_cast<double>(w[i]);
        sw += wi;
        sr += wi * e[2 * i];
        si += wi * e[2 * i + 1];
    }
    sw = block_sum(sw, lds);
    sr = block_sum(sr, lds);
    si = block_sum(si, lds);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = sw;
        part[3 * blockIdx.x + 1] = sr;
        part[3 * blockIdx.x + 2] = si;
    }
}

// Single block: combine pass-1 partials in block order; result[0..2] =
// sum w, mean re, mean im.
__global__ __launch_bounds__(kRedThreads) void energy_mean_kernel(const double *__restrict__ part,
                                                                  int nparts,
                                                                  double *__restrict__ result) {
    __shared__ double lds[kRedThreads];
    double sw = 0.0, sr = 0.0, si = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kRedThreads) {
        sw += part[3 * b];
        sr += part[3 * b + 1];
        si += part[3 * b + 2];
    }
    sw = block_sum(sw, lds);
    sr = block_sum(sr, lds);
    si = block_sum(si, lds);
    if (threadIdx.x == 0) {
        result[0] = sw;
        result[1] = sw != 0.0 ? sr / sw : 0.0;
        result[2] = sw != 0.0 ? si / sw : 0.0;
    }
}

// Pass 2: per-block sum w |E - mean|^2.
__global__ __launch_bounds__(kRedThreads) void energy_pass2_kernel(
    const int64_t *__restrict__ w, const double *__restrict__ e, int64_t n,
    const double *__restrict__ result, double *__restrict__ part) {
    __shared__ double lds[kRedThreads];
    const double mr = result[1], mi = result[2];
    double sv = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRedThreads + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRedThreads) {
        const double dr = e[2 * i] - mr, di = e[2 * i + 1] - mi;
        sv += static_cast<double>(w[i]) * (dr * dr + di * di);
    }
    sv = block_sum(sv, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = sv;
}

// Single block: out = {mean re, mean im, var, sum w}.
__global__ __launch_bounds__(kRedThreads) void energy_var_kernel(const double *__restrict__ part,
                                                                 int nparts,
                                                                 const double *__restrict__ result,
                                                                 double *__restrict__ out) {
    __shared__ double lds[kRedThreads];
    double sv = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kRedThreads) sv += part[b];
    sv = block_sum(sv, lds);
    if (threadIdx.x == 0) {
        const double sw = result[0];
        out[0] = result[1];
        out[1] = result[2];
        out[2] = sw != 0.0 ? sv / sw : 0.0;
        out[3] = sw;
    }
}

// ------------------------------------------------------------------ launchers

__global__ void reset_kernel(unsigned long long *counters, int *mixed) {
    if (threadIdx.x < 4) counters[threadIdx.x] = 0;
    if (threadIdx.x == 0) *mixed = 0;
}

hipError_t launch_reset(const DevScratch &sc, hipStream_t st) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, st, sc.counters, sc.mixed);
    return hipGetLastError();
}

EvalLaunch plan_eval(const DevTable &tab, int64_t n, bool dump) {
    EvalLaunch L;
    L.n = n;
    L.g_first = tab.has_diagonal ? 1 : 0;
    const int64_t g_eff = tab.n_groups - L.g_first;
    const int64_t tiles = (n + kProbeThreads - 1) / kProbeThreads;
    int64_t chunks = 1;
    if (!dump && g_eff > 0) {
        const int64_t want = (2048 + tiles - 1) / tiles;
        const int64_t max_chunks = (g_eff + 255) / 256;
        chunks = want < max_chunks ? want : max_chunks;
        if (chunks < 1) chunks = 1;
        if (chunks > 65535) chunks = 65535;
    }
    L.n_chunks = chunks;
    L.chunk_len = g_eff > 0 ? (g_eff + chunks - 1) / chunks : 0;
    return L;
}

hipError_t launch_hash(const DevTable &tab, const DevScratch &sc, uint32_t capacity,
                       const uint64_t *samples, const int64_t *weights, int64_t n,
                       hipStream_t st) {
    const int words = tab.n_qubits <= 63 ? 1 : 2;
    const int stride = words == 1 ? sizeof(Slot1) / 4 : sizeof(Slot2) / 4;
    int32_t *idx0 = reinterpret_cast<int32_t *>(static_cast<char *>(sc.slots) +
                                                (words == 1 ? offsetof(Slot1, idx)
                                                            : offsetof(Slot2, idx)));
    hipLaunchKernelGGL(hash_clear_kernel, dim3((capacity + 255) / 256), dim3(256), 0, st, idx0,
                       stride, capacity);
    const dim3 grid(static_cast<unsigned>((n + 255) / 256));
    if (words == 1)
        hipLaunchKernelGGL(hash_build_kernel<1>, grid, dim3(256), 0, st, tab, sc, samples, weights, n);
    else
        hipLaunchKernelGGL(hash_build_kernel<2>, grid, dim3(256), 0, st, tab, sc, samples, weights, n);
    return hipGetLastError();
}

hipError_t launch_eloc(const DevTable &tab, const DevScratch &sc, const EvalLaunch &L,
                       const uint64_t *samples, const double *log_amp, const double *phase,
                       double *eloc, int precision, int32_t *hit_idx, uint8_t *sign_bits,
                       int64_t sign_stride, EvalStageEvents ev, hipStream_t st) {
    (void)precision;
    const int words = tab.n_qubits <= 63 ? 1 : 2;
    const bool dump = hit_idx || sign_bits;
    const int64_t n = L.n;
    const dim3 pgrid(static_cast<unsigned>((n + kProbeThreads - 1) / kProbeThreads),
                     static_cast<unsigned>(L.n_chunks));
    const dim3 fgrid(static_cast<unsigned>((n + 255) / 256));
    if (L.chunk_len > 0) {
#define NQS_PROBE(Wd, D)                                                                       \
    hipLaunchKernelGGL((eloc_probe_kernel<Wd, D>), pgrid, dim3(kProbeThreads), 0, st, tab, sc, \
                       samples, log_amp, phase, n, L.g_first, L.chunk_len, hit_idx, sign_bits,  \
                       sign_stride)
        if (words == 1) {
            if (dump) NQS_PROBE(1, true); else NQS_PROBE(1, false);
        } else {
            if (dump) NQS_PROBE(2, true); else NQS_PROBE(2, false);
        }
#undef NQS_PROBE
    }
    if (ev.after_lookup) {
        const hipError_t e = hipEventRecord(ev.after_lookup, st);
        if (e != hipSuccess) return e;
    }
    const int64_t chunks = L.chunk_len > 0 ? L.n_chunks : 0;
#define NQS_FINISH(Wd, D)                                                                        \
    hipLaunchKernelGGL((eloc_finish_kernel<Wd, D>), fgrid, dim3(256), 0, st, tab, sc, samples, n, \
                       chunks, eloc, hit_idx, sign_bits, sign_stride)
    if (words == 1) {
        if (dump) NQS_FINISH(1, true); else NQS_FINISH(1, false);
    } else {
        if (dump) NQS_FINISH(2, true); else NQS_FINISH(2, false);
    }
#undef NQS_FINISH
    return hipGetLastError();
}

hipError_t launch_energy(const int64_t *w, const double *e, int64_t n, double *part,
                         double *result, double *out, hipStream_t st) {
    int64_t blocks = (n + kRedThreads - 1) / kRedThreads;
    if (blocks > kRedBlocks) blocks = kRedBlocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(energy_pass1_kernel, dim3(blocks), dim3(kRedThreads), 0, st, w, e, n, part);
    hipLaunchKernelGGL(energy_mean_kernel, dim3(1), dim3(kRedThreads), 0, st, part,
                       static_cast<int>(blocks), result);
    hipLaunchKernelGGL(energy_pass2_kernel, dim3(blocks), dim3(kRedThreads), 0, st, w, e, n,
                       result, part);
    hipLaunchKernelGGL(energy_var_kernel, dim3(1), dim3(kRedThreads), 0, st, part,
                       static_cast<int>(blocks), result, out);
    return hipGetLastError();
}

}  // namespace nqs
