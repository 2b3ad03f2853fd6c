// Host-side Pauli table: validation, phase folding, merge and group-by-X.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace nqs {

namespace detail {
// Record msg as the calling thread's last error and return code (nqs_host.cpp).
int fail(int code, const std::string &msg);
}  // namespace detail

// Maximum supported register width: samples and masks are two 64-bit words.
constexpr int kMaxQubits = 127;

// 32-bit GF(2)-linear hash of a bit string: the XOR of one random word per
// set bit.  Linearity gives h(x ^ X) = h(x) ^ h(X), so the hash of a flipped
// sample is one XOR away from the hash of the sample.
struct LinearHash {
    uint32_t r[128];
    LinearHash();
    uint32_t operator()(uint64_t w0, uint64_t w1) const;
};

struct HostTable {
    int n_qubits = 0;
    int words = 1;                 // 1 when n_qubits <= 63, else 2
    int64_t n_groups = 0;
    int64_t n_terms = 0;
    bool has_diagonal = false;     // group 0 has X = 0
    bool sector_filter = false;    // spin masks given, non-zero, each at most 64 qubits
    bool sector32 = false;         // both spin masks hold at most 32 qubits
    uint64_t spin[2][2] = {{0, 0}, {0, 0}};
    // groups, ascending by X
    std::vector<uint64_t> gx;      // [G][2] flip mask
    std::vector<uint64_t> gsec;    // [G][2] alpha flips and beta flips, each compressed
                                   // to consecutive bits (order of the spin mask)
    std::vector<uint32_t> ghm;     // [G][2] (linear hash of X, sector key)
    std::vector<int64_t> goff;     // [G + 1]
    // merged terms, ascending by (X, Z)
    std::vector<uint64_t> tz;      // [T][2]
    std::vector<double> tc;        // [T] c * (-1)^{ny/2}
    int max_group_terms = 0;
    // flip enumeration (the alternative to streaming every group past each
    // sample): valid when every qubit has a spin, the sector test applies and
    // no group flips more than four qubits, so the in-sector groups of a
    // sample are among its single and double excitations
    int max_flip = 0;              // largest popc(X) over the groups
    bool enum_ok = false;
    int k_alpha = 0, k_beta = 0;   // qubits per spin
    uint8_t spin_q[128] = {};      // alpha qubits at [0, k_alpha), beta qubits at [64, 64 + k_beta)
    // class of each qubit (random 3-bit values on beta qubits, 0 on alpha):
    // the class of a bit string, the XOR over its set qubits, picks the
    // filter partition of a sample; alpha flips leave it unchanged
    uint8_t qcls[128] = {};
    // group index by X: open addressing on (h(X) * golden) >> gh_shift,
    // linear probing, 0xFFFFFFFF = empty; keys are compared through gx
    std::vector<uint32_t> gh;
    uint32_t gh_shift = 0;
    // the X = 0 group in occupation form, when all its Z strings have at
    // most two qubits (Z_i = 1 - 2 n_i):
    //   <x|H_diag|x> = d[0] + sum_{j occ} (d[1 + j] + sum_{i occ, i < j} d[1 + nq + j (j - 1) / 2 + i])
    bool diag_occ = false;
    std::vector<double> diag;
};

// Fill max_flip, enum_ok, the spin qubit lists and the group index.
void build_enum_index(HostTable *T);

// Fill diag_occ and diag from the X = 0 group.
void build_diag_occ(HostTable *T);

// The occupation form as the digit tiles of the matrix-core diagonal: the
// terms U[j][i] (i <= j < nq; i == j: d[1 + j], the single terms; i < j:
// the pair terms) times 2^S, with S the largest integer keeping every
// |U| 2^S below 2^kDiagBits, rounded to integers q and written in
// kDiagDigits base-2^15 digits E_l (least significant first; the lower ones
// balanced in [-2^14, 2^14), the top one in [-2^14, 2^14]), each digit as two
// int8 byte planes, E = a - 128 b.  The MFMA multiplies plane a by the
// samples' 0/1 bits and plane b by the same bits times -128 into one
// accumulator, so that one 32-bit sum per digit carries both planes.
// Tiles: for column tile jt (j in [16 jt, 16 jt + 16), ceil(nq / 16) of
// them) the k-blocks kb of 64 rows i (one for jt < 4, two after), in that
// order; per tile, digit l and plane p (a, then b: plane 2 l + p), lane L
// holds in byte b the plane's byte for U[16 jt + L % 16][64 kb + 16 (L / 16)
// + b] (the A-operand layout of the 16 x 16 x 64 int8 MFMA).  *scale =
// 2^-S.  Empty without the form.
constexpr int kDiagDigits = 4;
constexpr int kDiagLimbs = 2 * kDiagDigits;  // byte planes
constexpr int kDiagBits = 59;
void build_diag_tiles(const HostTable &T, std::vector<int8_t> *out, double *scale);

// Sector key: half of popc(X & alpha) | half of popc(X & beta) << 8, or
// kSectorNeverKey when either popcount is odd (the flip always leaves the
// sector).
constexpr uint32_t kSectorNeverKey = 0xFFFFu;

// Bits of w selected by mask, packed to the low end in mask order.
uint64_t compress_bits(uint64_t w0, uint64_t w1, uint64_t m0, uint64_t m1);

// Flip table of a molecular Hamiltonian in the ONV ordering (spin orbital
// (p, alpha) = qubit 2p, (p, beta) = qubit 2p + 1): the X = 0 group and every
// spin-conserving single and double flip, as groups without Pauli terms.
// Matrix elements then come from the integrals (Slater-Condon rules).
int build_flip_table(int n_orbitals, HostTable *out, std::string *err);

// Returns 0 or a negative NQS_E_* code with *err describing it.
int build_table(int n_qubits, int64_t n_terms, const uint64_t *x, const uint64_t *z,
                const double *c, const uint64_t *spin_masks, HostTable *out, std::string *err);

}  // namespace nqs
