/*
 * CPU FP64 oracle for the local energy.  TEST INFRASTRUCTURE ONLY: it is
 * called by the tests, the smoke check and the CPU-baseline leg of the
 * benchmark, never by the library.  It shares no code with the GPU path.
 *
 * What it computes (Eq. 5 restricted to the sample set, the sample-space
 * energy of Sec. IV-C with a psi lookup table over the unique samples):
 *
 *   E_loc(x) = sum_{x' in S} <x|H|x'> psi(x') / psi(x),
 *   psi(x)   = exp(a(x) + i phi(x)),
 *   H        = sum_t c_t P_t,  P_t = i^{popc(X_t & Z_t)} X^{X_t} Z^{Z_t}.
 *
 * Matrix element, read straight from the operator: Z^{Z} |x'> =
 * (-1)^{popc(Z & x')} |x'>, then X^{X} flips to |x' ^ X>, so
 *   <x|P_t|x'> = i^{ny_t} (-1)^{popc(Z_t & x')}  if x ^ x' == X_t, else 0.
 * A state x' outside S contributes nothing (the lookup table holds S only).
 *
 * Algorithm: the literal double loop over (x, x') in S x S.  A pair is
 * skipped only when popc(x ^ x') exceeds the largest popc(X_t) of the term
 * list (no term can connect it); otherwise the terms with X_t = x ^ x' are
 * found by binary search in an X-sorted index and summed.  Sums use
 * Neumaier compensation.  OpenMP over x.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    uint64_t x0, x1;
    int64_t lo, hi; /* range in the X-sorted term order */
} ogroup;

typedef struct {
    int64_t n_terms;
    int64_t n_groups;
    int maxpop;
    int64_t *order;   /* term indices sorted by X */
    ogroup *groups;
    const uint64_t *x, *z;
    const double *cre, *cim;
} oterms;

typedef struct {
    double s, c;
} neu;

static inline void neu_add(neu *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static inline double neu_val(const neu *a) { return a->s + a->c; }

static const uint64_t *g_sort_x;

static int cmp_by_x(const void *pa, const void *pb) {
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    uint64_t a1 = g_sort_x[2 * a + 1], b1 = g_sort_x[2 * b + 1];
    if (a1 != b1) return a1 < b1 ? -1 : 1;
    uint64_t a0 = g_sort_x[2 * a], b0 = g_sort_x[2 * b];
    if (a0 != b0) return a0 < b0 ? -1 : 1;
    return a < b ? -1 : (a > b);
}

static int terms_init(oterms *T, int64_t nt, const uint64_t *x, const uint64_t *z,
                      const double *cre, const double *cim) {
    memset(T, 0, sizeof(*T));
    T->n_terms = nt;
    T->x = x; T->z = z; T->cre = cre; T->cim = cim;
    T->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nt ? nt : 1));
    T->groups = (ogroup *)malloc(sizeof(ogroup) * (size_t)(nt ? nt : 1));
    if (!T->order || !T->groups) return -1;
    for (int64_t i = 0; i < nt; ++i) T->order[i] = i;
    g_sort_x = x; /* qsort has no context argument; the oracle sorts once, serially */
    qsort(T->order, (size_t)nt, sizeof(int64_t), cmp_by_x);
    int64_t g = -1;
    T->maxpop = 0;
    for (int64_t k = 0; k < nt; ++k) {
        int64_t t = T->order[k];
        if (g < 0 || T->groups[g].x0 != x[2 * t] || T->groups[g].x1 != x[2 * t + 1]) {
            ++g;
            T->groups[g].x0 = x[2 * t];
            T->groups[g].x1 = x[2 * t + 1];
            T->groups[g].lo = k;
            int p = __builtin_popcountll(x[2 * t]) + __builtin_popcountll(x[2 * t + 1]);
            if (p > T->maxpop) T->maxpop = p;
        }
        T->groups[g].hi = k + 1;
    }
    T->n_groups = g + 1;
    return 0;
}

static void terms_free(oterms *T) {
    free(T->order);
    free(T->groups);
}

static const ogroup *find_group(const oterms *T, uint64_t d0, uint64_t d1) {
    int64_t lo = 0, hi = T->n_groups;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        const ogroup *g = &T->groups[mid];
        if (g->x1 < d1 || (g->x1 == d1 && g->x0 < d0))
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo < T->n_groups && T->groups[lo].x0 == d0 && T->groups[lo].x1 == d1) return &T->groups[lo];
    return NULL;
}

/* <bra|H|ket> for the terms of group g (bra ^ ket == X of g).  Also returns
 * sum |c_t| over the group in *abs_out. */
static void group_element(const oterms *T, const ogroup *g, uint64_t k0, uint64_t k1,
                          double *re, double *im, double *abs_out) {
    neu sr = {0, 0}, si = {0, 0}, sa = {0, 0};
    for (int64_t k = g->lo; k < g->hi; ++k) {
        int64_t t = T->order[k];
        uint64_t X0 = T->x[2 * t], X1 = T->x[2 * t + 1];
        uint64_t Z0 = T->z[2 * t], Z1 = T->z[2 * t + 1];
        int ny = (__builtin_popcountll(X0 & Z0) + __builtin_popcountll(X1 & Z1)) & 3;
        int zs = (__builtin_popcountll(Z0 & k0) + __builtin_popcountll(Z1 & k1)) & 1;
        double cr = T->cre[t], ci = T->cim ? T->cim[t] : 0.0;
        /* multiply c by i^ny */
        double pr, pi;
        switch (ny) {
            case 0: pr = cr; pi = ci; break;
            case 1: pr = -ci; pi = cr; break;
            case 2: pr = -cr; pi = -ci; break;
            default: pr = ci; pi = -cr; break;
        }
        if (zs) { pr = -pr; pi = -pi; }
        neu_add(&sr, pr);
        neu_add(&si, pi);
        neu_add(&sa, hypot(cr, ci));
    }
    *re = neu_val(&sr);
    *im = neu_val(&si);
    if (abs_out) *abs_out = neu_val(&sa);
}

/*
 * eloc[2i], eloc[2i+1]: real and imaginary part of E_loc(s_i).
 * absum[i] (optional): sum over connected x' in S of |psi(x')/psi(x)| times
 * sum_{t in group} |c_t|, the absolute scale of the sum.
 * n_conn[i] (optional): number of x' in S with a non-empty group (x itself
 * included when the X = 0 group exists).
 * Returns 0, or -1 on allocation failure.
 */
int oracle_eloc(int n_qubits, int64_t n_terms, const uint64_t *x, const uint64_t *z,
                const double *c_re, const double *c_im, int64_t n_samples, const uint64_t *s,
                const double *log_amp, const double *phase, double *eloc, double *absum,
                int64_t *n_conn, int n_threads) {
    (void)n_qubits;
    oterms T;
    if (terms_init(&T, n_terms, x, z, c_re, c_im)) { terms_free(&T); return -1; }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_samples; ++i) {
        const uint64_t b0 = s[2 * i], b1 = s[2 * i + 1];
        neu er = {0, 0}, ei = {0, 0}, ea = {0, 0};
        int64_t nc = 0;
        for (int64_t j = 0; j < n_samples; ++j) {
            uint64_t d0 = b0 ^ s[2 * j], d1 = b1 ^ s[2 * j + 1];
            if (__builtin_popcountll(d0) + __builtin_popcountll(d1) > T.maxpop) continue;
            const ogroup *g = find_group(&T, d0, d1);
            if (!g) continue;
            double hr, hi, ha;
            group_element(&T, g, s[2 * j], s[2 * j + 1], &hr, &hi, &ha);
            double mag = exp(log_amp[j] - log_amp[i]);
            double ang = phase[j] - phase[i];
            double rr = mag * cos(ang), ri = mag * sin(ang);
            neu_add(&er, hr * rr - hi * ri);
            neu_add(&ei, hr * ri + hi * rr);
            neu_add(&ea, ha * mag);
            ++nc;
        }
        eloc[2 * i] = neu_val(&er);
        eloc[2 * i + 1] = neu_val(&ei);
        if (absum) absum[i] = neu_val(&ea);
        if (n_conn) n_conn[i] = nc;
    }
    terms_free(&T);
    return 0;
}

/*
 * Same double loop on a subset of rows: E_loc for rows[k], k < n_rows, with
 * x' still ranging over all of S.  Used to check sampled outputs at full
 * sizes and for the bounded CPU baseline.
 */
int oracle_eloc_rows(int n_qubits, int64_t n_terms, const uint64_t *x, const uint64_t *z,
                     const double *c_re, const double *c_im, int64_t n_samples,
                     const uint64_t *s, const double *log_amp, const double *phase,
                     int64_t n_rows, const int64_t *rows, double *eloc, double *absum,
                     int64_t *n_conn, int n_threads) {
    (void)n_qubits;
    oterms T;
    if (terms_init(&T, n_terms, x, z, c_re, c_im)) { terms_free(&T); return -1; }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < n_rows; ++k) {
        const int64_t i = rows[k];
        const uint64_t b0 = s[2 * i], b1 = s[2 * i + 1];
        neu er = {0, 0}, ei = {0, 0}, ea = {0, 0};
        int64_t nc = 0;
        for (int64_t j = 0; j < n_samples; ++j) {
            uint64_t d0 = b0 ^ s[2 * j], d1 = b1 ^ s[2 * j + 1];
            if (__builtin_popcountll(d0) + __builtin_popcountll(d1) > T.maxpop) continue;
            const ogroup *g = find_group(&T, d0, d1);
            if (!g) continue;
            double hr, hi, ha;
            group_element(&T, g, s[2 * j], s[2 * j + 1], &hr, &hi, &ha);
            double mag = exp(log_amp[j] - log_amp[i]);
            double ang = phase[j] - phase[i];
            double rr = mag * cos(ang), ri = mag * sin(ang);
            neu_add(&er, hr * rr - hi * ri);
            neu_add(&ei, hr * ri + hi * rr);
            neu_add(&ea, ha * mag);
            ++nc;
        }
        eloc[2 * k] = neu_val(&er);
        eloc[2 * k + 1] = neu_val(&ei);
        if (absum) absum[k] = neu_val(&ea);
        if (n_conn) n_conn[k] = nc;
    }
    terms_free(&T);
    return 0;
}

/*
 * Connected pairs: every (i, j) with a non-empty group for s_i ^ s_j, in
 * row-major order.  With pairs == NULL only the count is returned.
 */
int64_t oracle_pairs(int64_t n_terms, const uint64_t *x, int64_t n_samples, const uint64_t *s,
                     int64_t *pairs, int64_t cap) {
    oterms T;
    if (terms_init(&T, n_terms, x, x, NULL, NULL)) { terms_free(&T); return -1; }
    int64_t n = 0;
    for (int64_t i = 0; i < n_samples; ++i)
        for (int64_t j = 0; j < n_samples; ++j) {
            uint64_t d0 = s[2 * i] ^ s[2 * j], d1 = s[2 * i + 1] ^ s[2 * j + 1];
            if (__builtin_popcountll(d0) + __builtin_popcountll(d1) > T.maxpop) continue;
            if (!find_group(&T, d0, d1)) continue;
            if (pairs && n < cap) {
                pairs[2 * n] = i;
                pairs[2 * n + 1] = j;
            }
            ++n;
        }
    terms_free(&T);
    return n;
}

/* <bra|H|ket> for one pair of basis states (0 if no term connects them). */
void oracle_hij(int64_t n_terms, const uint64_t *x, const uint64_t *z, const double *c_re,
                const double *c_im, const uint64_t *bra, const uint64_t *ket, double *out) {
    oterms T;
    out[0] = out[1] = 0.0;
    if (terms_init(&T, n_terms, x, z, c_re, c_im)) { terms_free(&T); return; }
    const ogroup *g = find_group(&T, bra[0] ^ ket[0], bra[1] ^ ket[1]);
    if (g) group_element(&T, g, ket[0], ket[1], &out[0], &out[1], NULL);
    terms_free(&T);
}

/* Batched <bra_k|H|ket_k>, with the index built once. */
int oracle_hij_batch(int64_t n_terms, const uint64_t *x, const uint64_t *z, const double *c_re,
                     const double *c_im, int64_t n, const uint64_t *bra, const uint64_t *ket,
                     double *out) {
    oterms T;
    if (terms_init(&T, n_terms, x, z, c_re, c_im)) { terms_free(&T); return -1; }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        out[2 * k] = out[2 * k + 1] = 0.0;
        const ogroup *g = find_group(&T, bra[2 * k] ^ ket[2 * k], bra[2 * k + 1] ^ ket[2 * k + 1]);
        if (g) group_element(&T, g, ket[2 * k], ket[2 * k + 1], &out[2 * k], &out[2 * k + 1], NULL);
    }
    terms_free(&T);
    return 0;
}

/* Number of distinct X masks in the term list. */
int64_t oracle_n_groups(int64_t n_terms, const uint64_t *x) {
    oterms T;
    if (terms_init(&T, n_terms, x, x, NULL, NULL)) { terms_free(&T); return -1; }
    int64_t g = T.n_groups;
    terms_free(&T);
    return g;
}
