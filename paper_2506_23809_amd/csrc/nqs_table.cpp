// Host-side Pauli table builder (no device code).
//
// The terms of H = sum_t c_t i^{ny_t} X^{x_t} Z^{z_t} enter as packed masks.
// For a real Hamiltonian ny is even, and the matrix element between basis
// states x (bra) and x' = x ^ X_t (ket) is
//   <x| i^{ny} X^X Z^Z |x'> = <x| (-i)^{ny} Z^Z X^X |x'> = (-1)^{ny/2} (-1)^{popc(Z & x)},
// using X^X Z^Z = (-1)^{ny} Z^Z X^X.  The constant (-1)^{ny/2} is folded into
// the stored coefficient, so a kernel needs one popcount per term.  Terms are
// grouped by X because every term of a group connects x to the same x'
// (the per-ket inner loop of Alg. 3 becomes a loop over groups).
#include "nqs_table.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

#include "../../include/nqs.h"

namespace nqs {

namespace {

inline int popc2(uint64_t a, uint64_t b) { return __builtin_popcountll(a) + __builtin_popcountll(b); }

inline bool above(uint64_t w0, uint64_t w1, int nq) {
    // true if any bit at index >= nq is set
    if (nq >= 128) return false;
    if (nq >= 64) {
        int k = nq - 64;
        return k < 64 && (w1 >> k) != 0;
    }
    return (w0 >> nq) != 0 || w1 != 0;
}

uint64_t splitmix64(uint64_t *s) {
    uint64_t z = (*s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

}  // namespace

uint64_t compress_bits(uint64_t w0, uint64_t w1, uint64_t m0, uint64_t m1) {
    uint64_t r = 0;
    int k = 0;
    while (m0) {
        const int b = __builtin_ctzll(m0);
        r |= ((w0 >> b) & 1ull) << k++;
        m0 &= m0 - 1;
    }
    while (m1) {
        const int b = __builtin_ctzll(m1);
        r |= ((w1 >> b) & 1ull) << k++;
        m1 &= m1 - 1;
    }
    return r;
}

LinearHash::LinearHash() {
    uint64_t s = 0x6e71735f68617368ull;  // fixed seed: tables are reproducible
    for (int j = 0; j < 128; ++j) r[j] = static_cast<uint32_t>(splitmix64(&s) >> 32);
}

uint32_t LinearHash::operator()(uint64_t w0, uint64_t w1) const {
    uint32_t h = 0;
    while (w0) {
        h ^= r[__builtin_ctzll(w0)];
        w0 &= w0 - 1;
    }
    while (w1) {
        h ^= r[64 + __builtin_ctzll(w1)];
        w1 &= w1 - 1;
    }
    return h;
}

int build_table(int n_qubits, int64_t n_terms, const uint64_t *x, const uint64_t *z,
                const double *c, const uint64_t *spin_masks, HostTable *out, std::string *err) {
    if (!out) { *err = "null output"; return NQS_E_ARG; }
    if (n_qubits < 1 || n_qubits > kMaxQubits) {
        *err = "n_qubits must be in [1, 127], got " + std::to_string(n_qubits);
        return NQS_E_RANGE;
    }
    if (n_terms < 0) { *err = "n_terms < 0"; return NQS_E_ARG; }
    if (n_terms > 0 && (!x || !z || !c)) { *err = "null term arrays"; return NQS_E_ARG; }
    if (n_terms >= (int64_t(1) << 32)) { *err = "more than 2^32 terms"; return NQS_E_ARG; }

    HostTable &T = *out;
    T = HostTable();
    T.n_qubits = n_qubits;
    T.words = n_qubits <= 63 ? 1 : 2;

    if (spin_masks) {
        for (int k = 0; k < 4; ++k) T.spin[k / 2][k % 2] = spin_masks[k];
        for (int s = 0; s < 2; ++s)
            if (above(T.spin[s][0], T.spin[s][1], n_qubits)) {
                *err = "spin mask has bits at or above n_qubits";
                return NQS_E_RANGE;
            }
        if ((T.spin[0][0] & T.spin[1][0]) || (T.spin[0][1] & T.spin[1][1])) {
            *err = "alpha and beta spin masks overlap";
            return NQS_E_ARG;
        }
        bool a = T.spin[0][0] | T.spin[0][1], b = T.spin[1][0] | T.spin[1][1];
        const int wa = popc2(T.spin[0][0], T.spin[0][1]);
        const int wb = popc2(T.spin[1][0], T.spin[1][1]);
        // the compressed sector test works on one 64-bit word per spin
        T.sector_filter = a && b && wa <= 64 && wb <= 64;
        T.sector32 = T.sector_filter && wa <= 32 && wb <= 32;
        if (!(a || b)) {
            T.spin[0][0] = T.spin[0][1] = T.spin[1][0] = T.spin[1][1] = 0;
        } else if (!(a && b)) {
            *err = "spin masks: give both alpha and beta, or neither";
            return NQS_E_ARG;
        }
    }

    std::vector<double> folded(static_cast<size_t>(n_terms));
    for (int64_t t = 0; t < n_terms; ++t) {
        const uint64_t x0 = x[2 * t], x1 = x[2 * t + 1], z0 = z[2 * t], z1 = z[2 * t + 1];
        if (above(x0, x1, n_qubits) || above(z0, z1, n_qubits)) {
            *err = "term " + std::to_string(t) + " has a bit at or above n_qubits";
            return NQS_E_RANGE;
        }
        if (!std::isfinite(c[t])) {
            *err = "term " + std::to_string(t) + " has a non-finite coefficient";
            return NQS_E_ARG;
        }
        const int ny = popc2(x0 & z0, x1 & z1);
        if (ny & 1) {
            *err = "term " + std::to_string(t) + " has an odd number of Y factors";
            return NQS_E_NONREAL;
        }
        folded[t] = (ny & 2) ? -c[t] : c[t];
    }

    // stable order by (X hi, X lo, Z hi, Z lo): equal strings keep input order
    std::vector<int64_t> ord(static_cast<size_t>(n_terms));
    std::iota(ord.begin(), ord.end(), int64_t(0));
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
        if (x[2 * a + 1] != x[2 * b + 1]) return x[2 * a + 1] < x[2 * b + 1];
        if (x[2 * a] != x[2 * b]) return x[2 * a] < x[2 * b];
        if (z[2 * a + 1] != z[2 * b + 1]) return z[2 * a + 1] < z[2 * b + 1];
        return z[2 * a] < z[2 * b];
    });

    const LinearHash lh;
    T.tz.reserve(2 * static_cast<size_t>(n_terms));
    T.tc.reserve(static_cast<size_t>(n_terms));
    uint64_t px0 = 0, px1 = 0, pz0 = 0, pz1 = 0;
    bool first = true;
    for (int64_t k = 0; k < n_terms; ++k) {
        const int64_t t = ord[k];
        const uint64_t x0 = x[2 * t], x1 = x[2 * t + 1], z0 = z[2 * t], z1 = z[2 * t + 1];
        const bool same_x = !first && x0 == px0 && x1 == px1;
        if (same_x && z0 == pz0 && z1 == pz1) {
            T.tc.back() += folded[t];  // merge equal strings
            continue;
        }
        if (!same_x) {
            T.gx.push_back(x0);
            T.gx.push_back(x1);
            T.goff.push_back(static_cast<int64_t>(T.tc.size()));
        }
        T.tz.push_back(z0);
        T.tz.push_back(z1);
        T.tc.push_back(folded[t]);
        px0 = x0; px1 = x1; pz0 = z0; pz1 = z1;
        first = false;
    }
    T.n_groups = static_cast<int64_t>(T.gx.size() / 2);
    T.n_terms = static_cast<int64_t>(T.tc.size());
    T.goff.push_back(T.n_terms);
    T.has_diagonal = T.n_groups > 0 && T.gx[0] == 0 && T.gx[1] == 0;

    T.gsec.resize(2 * T.n_groups);
    T.ghm.resize(2 * T.n_groups);
    for (int64_t g = 0; g < T.n_groups; ++g) {
        const uint64_t x0 = T.gx[2 * g], x1 = T.gx[2 * g + 1];
        const uint64_t a0 = x0 & T.spin[0][0], a1 = x1 & T.spin[0][1];
        const uint64_t b0 = x0 & T.spin[1][0], b1 = x1 & T.spin[1][1];
        const int pa = popc2(a0, a1), pb = popc2(b0, b1);
        T.gsec[2 * g] = T.sector_filter ? compress_bits(x0, x1, T.spin[0][0], T.spin[0][1]) : 0;
        T.gsec[2 * g + 1] = T.sector_filter ? compress_bits(x0, x1, T.spin[1][0], T.spin[1][1]) : 0;
        uint32_t key = static_cast<uint32_t>(pa / 2) | (static_cast<uint32_t>(pb / 2) << 8);
        if ((pa & 1) || (pb & 1)) key = kSectorNeverKey;
        T.ghm[2 * g] = lh(x0, x1);
        T.ghm[2 * g + 1] = key;
        T.max_group_terms =
            std::max(T.max_group_terms, static_cast<int>(T.goff[g + 1] - T.goff[g]));
    }
    build_enum_index(&T);
    build_diag_occ(&T);
    return NQS_OK;
}

int build_flip_table(int K, HostTable *out, std::string *err) {
    if (K < 1 || 2 * K > kMaxQubits) {
        *err = "n_orbitals must be in [1, 63]";
        return NQS_E_RANGE;
    }
    HostTable &T = *out;
    T = HostTable();
    const int nq = 2 * K;
    T.n_qubits = nq;
    T.words = nq <= 63 ? 1 : 2;
    for (int p = 0; p < K; ++p) {
        const int a = 2 * p, b = 2 * p + 1;
        if (a < 64) T.spin[0][0] |= 1ull << a; else T.spin[0][1] |= 1ull << (a - 64);
        if (b < 64) T.spin[1][0] |= 1ull << b; else T.spin[1][1] |= 1ull << (b - 64);
    }
    T.sector_filter = K <= 64;
    T.sector32 = K <= 32;
    struct M { uint64_t lo, hi; };
    auto bit = [](int q) { return q < 64 ? M{1ull << q, 0} : M{0, 1ull << (q - 64)}; };
    auto orr = [](M x, M y) { return M{x.lo | y.lo, x.hi | y.hi}; };
    std::vector<M> flips;
    flips.push_back(M{0, 0});
    for (int s = 0; s < 2; ++s) {
        for (int p = 0; p < K; ++p)
            for (int q = p + 1; q < K; ++q) {
                flips.push_back(orr(bit(2 * p + s), bit(2 * q + s)));
                for (int r = q + 1; r < K; ++r)
                    for (int t = r + 1; t < K; ++t)
                        flips.push_back(orr(orr(bit(2 * p + s), bit(2 * q + s)),
                                            orr(bit(2 * r + s), bit(2 * t + s))));
            }
    }
    for (int p = 0; p < K; ++p)
        for (int q = p + 1; q < K; ++q)
            for (int r = 0; r < K; ++r)
                for (int t = r + 1; t < K; ++t)
                    flips.push_back(orr(orr(bit(2 * p), bit(2 * q)), orr(bit(2 * r + 1), bit(2 * t + 1))));
    std::sort(flips.begin(), flips.end(), [](const M &x, const M &y) {
        return x.hi != y.hi ? x.hi < y.hi : x.lo < y.lo;
    });
    const LinearHash lh;
    T.n_groups = static_cast<int64_t>(flips.size());
    T.n_terms = 0;
    T.has_diagonal = true;
    T.gx.resize(2 * T.n_groups);
    T.gsec.resize(2 * T.n_groups);
    T.ghm.resize(2 * T.n_groups);
    T.goff.assign(T.n_groups + 1, 0);
    for (int64_t g = 0; g < T.n_groups; ++g) {
        const uint64_t x0 = flips[g].lo, x1 = flips[g].hi;
        T.gx[2 * g] = x0;
        T.gx[2 * g + 1] = x1;
        const int pa = popc2(x0 & T.spin[0][0], x1 & T.spin[0][1]);
        const int pb = popc2(x0 & T.spin[1][0], x1 & T.spin[1][1]);
        T.gsec[2 * g] = compress_bits(x0, x1, T.spin[0][0], T.spin[0][1]);
        T.gsec[2 * g + 1] = compress_bits(x0, x1, T.spin[1][0], T.spin[1][1]);
        T.ghm[2 * g] = lh(x0, x1);
        T.ghm[2 * g + 1] = static_cast<uint32_t>(pa / 2) | (static_cast<uint32_t>(pb / 2) << 8);
    }
    build_enum_index(&T);
    return NQS_OK;
}

void build_enum_index(HostTable *T) {
    uint64_t cap = 64;
    while (cap < 2 * static_cast<uint64_t>(T->n_groups)) cap <<= 1;
    int lg = 0;
    while ((uint64_t(1) << lg) < cap) ++lg;
    T->gh.assign(cap, 0xFFFFFFFFu);
    T->gh_shift = static_cast<uint32_t>(32 - lg);
    T->max_flip = 0;
    const uint32_t mask = static_cast<uint32_t>(cap - 1);
    for (int64_t g = 0; g < T->n_groups; ++g) {
        T->max_flip = std::max(T->max_flip, popc2(T->gx[2 * g], T->gx[2 * g + 1]));
        uint32_t slot = (T->ghm[2 * g] * 0x9E3779B1u) >> T->gh_shift;
        while (T->gh[slot] != 0xFFFFFFFFu) slot = (slot + 1) & mask;
        T->gh[slot] = static_cast<uint32_t>(g);
    }
    T->k_alpha = T->k_beta = 0;
    uint64_t seed = 0x6e71735f636c6173ull;  // fixed: the partition of a sample is reproducible
    for (int q = 0; q < 128; ++q) {
        const uint8_t v = static_cast<uint8_t>(splitmix64(&seed) >> 61);
        const int w = q >> 6;
        T->qcls[q] = (q < T->n_qubits && (T->spin[1][w] >> (q & 63)) & 1ull) ? v : 0;
    }
    for (int q = 0; q < T->n_qubits; ++q) {
        const int w = q >> 6;
        const uint64_t b = 1ull << (q & 63);
        if (T->spin[0][w] & b) T->spin_q[T->k_alpha++] = static_cast<uint8_t>(q);
        else if (T->spin[1][w] & b) T->spin_q[64 + T->k_beta++] = static_cast<uint8_t>(q);
    }
    T->enum_ok = T->sector_filter && T->k_alpha + T->k_beta == T->n_qubits &&
                 T->k_alpha <= 64 && T->k_beta <= 64 && T->max_flip <= 4;
}

void build_diag_occ(HostTable *T) {
    T->diag_occ = false;
    T->diag.clear();
    if (!T->has_diagonal) return;
    const int nq = T->n_qubits;
    std::vector<double> d(1 + nq + static_cast<size_t>(nq) * (nq - 1) / 2, 0.0);
    for (int64_t t = T->goff[0]; t < T->goff[1]; ++t) {
        const uint64_t z0 = T->tz[2 * t], z1 = T->tz[2 * t + 1];
        const double c = T->tc[t];
        int q[2], w = 0;
        for (int b = 0; b < 128 && w <= 2; ++b) {
            if (((b < 64 ? z0 >> b : z1 >> (b - 64)) & 1ull) == 0) continue;
            if (w < 2) q[w] = b;
            ++w;
        }
        if (w > 2) return;  // a Z string on three or more qubits: keep the term form
        // c Z_i Z_j = c (1 - 2 n_i)(1 - 2 n_j), c Z_i = c (1 - 2 n_i)
        d[0] += c;
        if (w >= 1) d[1 + q[0]] -= 2.0 * c;
        if (w == 2) {
            d[1 + q[1]] -= 2.0 * c;
            d[1 + nq + static_cast<size_t>(q[1]) * (q[1] - 1) / 2 + q[0]] += 4.0 * c;
        }
    }
    T->diag = std::move(d);
    T->diag_occ = true;
}

void build_diag_tiles(const HostTable &T, std::vector<int8_t> *out, double *scale) {
    out->clear();
    *scale = 1.0;
    if (!T.diag_occ) return;
    const int nq = T.n_qubits;
    const int jtiles = (nq + 15) / 16;
    auto u = [&](int j, int i) -> double {
        if (j >= nq || i > j) return 0.0;
        return i == j ? T.diag[1 + j] : T.diag[1 + nq + size_t(j) * (j - 1) / 2 + i];
    };
    double maxabs = 0.0;
    for (int j = 0; j < nq; ++j)
        for (int i = 0; i <= j; ++i) maxabs = std::max(maxabs, std::fabs(u(j, i)));
    int e = 0;
    if (maxabs > 0.0) std::frexp(maxabs, &e);  // maxabs < 2^e
    const int S = maxabs > 0.0 ? kDiagBits - e : 0;
    *scale = std::ldexp(1.0, -S);
    const int tiles = jtiles <= 4 ? jtiles : 4 + 2 * (jtiles - 4);
    out->assign(size_t(tiles) * kDiagLimbs * 64 * 16, 0);
    int t = 0;
    for (int jt = 0; jt < jtiles; ++jt) {
        const int nkb = jt < 4 ? 1 : 2;
        for (int kb = 0; kb < nkb; ++kb, ++t) {
            for (int L = 0; L < 64; ++L) {
                for (int b = 0; b < 16; ++b) {
                    const int j = 16 * jt + L % 16, i = 64 * kb + 16 * (L / 16) + b;
                    // |q| < 2^kDiagBits (a double below 2^59 is at most
                    // 2^59 - 64, so rounding keeps it there)
                    int64_t q = std::llround(std::ldexp(u(j, i), S));
                    for (int l = 0; l < kDiagDigits; ++l) {
                        // base-2^15 digit: balanced for the lower three, the
                        // rest for the top one (then within [-2^14, 2^14])
                        int64_t E = q;
                        if (l + 1 < kDiagDigits) {
                            E = ((q + 16384) & 32767) - 16384;
                            q = (q - E) / 32768;
                        }
                        // E = a - 128 b with a, b int8: b the nearest
                        // multiple's quotient, kept in range at E = -2^14
                        int64_t bq = -((E + 64) >> 7);
                        if (bq > 127) bq = 127;
                        const int64_t a = E + 128 * bq;
                        const size_t at = (size_t(t) * kDiagLimbs + 2 * l) * 64 + L;
                        (*out)[at * 16 + b] = static_cast<int8_t>(a);
                        (*out)[(at + 64) * 16 + b] = static_cast<int8_t>(bq);
                    }
                }
            }
        }
    }
}

}  // namespace nqs
