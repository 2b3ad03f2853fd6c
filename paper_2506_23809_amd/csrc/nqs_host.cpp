// Host-only part of the C ABI: the per-thread error text, the version, and
// the host form of the table builder.  Plain C++ (no device code), so it can
// also be built, with the table builder, into a CPU-only library (the
// sanitizer test does that).
#include <cstring>
#include <new>
#include <string>

#include "../../include/nqs.h"
#include "nqs_table.hpp"

namespace nqs {
namespace detail {

namespace {
thread_local std::string g_last_error;
}  // namespace

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

const char *last_error() { return g_last_error.c_str(); }

}  // namespace detail
}  // namespace nqs

extern "C" {

const char *nqs_last_error(void) { return nqs::detail::last_error(); }

int nqs_version(void) { return 101; }

int nqs_table_host(int n_qubits, int64_t n_terms, const uint64_t *x_masks,
                   const uint64_t *z_masks, const double *coeffs, int64_t *n_groups,
                   int64_t *n_merged, uint64_t *group_x, int64_t *group_off, uint64_t *term_z,
                   double *term_c) {
    using nqs::detail::fail;
    if (!n_groups || !n_merged) return fail(NQS_E_ARG, "null count outputs");
    nqs::HostTable T;
    std::string err;
    int rc;
    try {
        rc = nqs::build_table(n_qubits, n_terms, x_masks, z_masks, coeffs, nullptr, &T, &err);
    } catch (const std::bad_alloc &) {
        return fail(NQS_E_NOMEM, "host allocation failed");
    }
    if (rc) return fail(rc, err);
    *n_groups = T.n_groups;
    *n_merged = T.n_terms;
    // (an empty table has empty vectors, whose data() may be null: memcpy
    // from a null pointer is undefined even for zero bytes)
    if (group_x && !T.gx.empty())
        std::memcpy(group_x, T.gx.data(), sizeof(uint64_t) * T.gx.size());
    if (group_off && !T.goff.empty())
        std::memcpy(group_off, T.goff.data(), sizeof(int64_t) * T.goff.size());
    if (term_z && !T.tz.empty()) std::memcpy(term_z, T.tz.data(), sizeof(uint64_t) * T.tz.size());
    if (term_c && !T.tc.empty()) std::memcpy(term_c, T.tc.data(), sizeof(double) * T.tc.size());
    return NQS_OK;
}

int nqs_diag_tiles_host(int n_qubits, int64_t n_terms, const uint64_t *x_masks,
                        const uint64_t *z_masks, const double *coeffs,
                        const uint64_t *spin_masks, int64_t *n_bytes, int8_t *tiles,
                        double *d0, double *scale) {
    using nqs::detail::fail;
    if (!n_bytes) return fail(NQS_E_ARG, "null size output");
    nqs::HostTable T;
    std::string err;
    std::vector<int8_t> q8;
    double sc = 1.0;
    int rc;
    try {
        rc = nqs::build_table(n_qubits, n_terms, x_masks, z_masks, coeffs, spin_masks, &T, &err);
        if (rc == 0) nqs::build_diag_tiles(T, &q8, &sc);
    } catch (const std::bad_alloc &) {
        return fail(NQS_E_NOMEM, "host allocation failed");
    }
    if (rc) return fail(rc, err);
    *n_bytes = static_cast<int64_t>(q8.size());
    if (tiles && !q8.empty()) std::memcpy(tiles, q8.data(), q8.size());
    if (d0) *d0 = T.diag_occ ? T.diag[0] : 0.0;
    if (scale) *scale = sc;
    return NQS_OK;
}

}  // extern "C"
