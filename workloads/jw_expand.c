/*
 * Jordan-Wigner expansion of a spin-orbital molecular Hamiltonian into
 * merged Pauli strings.  Part of the seeded input producer: it turns the
 * integrals of the second-quantised Hamiltonian (Eq. 2, written here in the
 * chemists' form) into the Pauli-term list that both the oracle and the GPU
 * library consume.  It holds none of the local-energy arithmetic.
 *
 *   H = sum_{pq,s} h_pq a+_{ps} a_{qs}
 *     + 1/2 sum_{pqrs,s,t} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}
 *
 * Spin orbital (p, s) is qubit 2p + s (s = 0 alpha, 1 beta), following the
 * ONV ordering of Sec. II-A.  Qubit j lives in word j/64, bit j%64.
 *
 * Ladder operators (occupied = |1>):
 *   a+_j = X_j Z_{<j} |0><0|_j = 1/2 X^{e_j} Z^{m_{<j}} + 1/2 X^{e_j} Z^{m_{<=j}}
 *   a_j  = X_j Z_{<j} |1><1|_j = 1/2 X^{e_j} Z^{m_{<j}} - 1/2 X^{e_j} Z^{m_{<=j}}
 * where X^x Z^z is the "raw" product with all X factors to the left.  Raw
 * strings multiply as
 *   (X^{x1} Z^{z1})(X^{x2} Z^{z2}) = (-1)^{popc(z1 & x2)} X^{x1^x2} Z^{z1^z2}.
 * A raw string c X^x Z^z equals c (-i)^{ny} P with ny = popc(x & z) and
 * P = i^{ny} X^x Z^z the Hermitian Pauli string; the output coefficient is
 * therefore c (-i)^{ny}.  Strings with odd ny carry imaginary coefficients
 * that cancel exactly in a real Hamiltonian; by default they are dropped as
 * they are produced (keep_odd=1 keeps them so that a test can watch them
 * cancel).
 *
 * Merging is done in per-partition open-addressing tables; a string always
 * lands in the same partition and receives its contributions in the same
 * loop order, so the merged values do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    uint64_t x0, x1, z0, z1;
    double re, im;
    int used;
} jw_entry;

typedef struct {
    jw_entry *slots;
    uint64_t cap;   /* power of two */
    uint64_t count;
} jw_table;

typedef struct {
    int n_parts;
    jw_table *parts;
    int64_t n_out;
    uint64_t *ox, *oz;
    double *oc, *oc_im;
} jw_result;

static inline uint64_t mix64(uint64_t v) {
    v ^= v >> 30; v *= 0xbf58476d1ce4e5b9ull;
    v ^= v >> 27; v *= 0x94d049bb133111ebull;
    v ^= v >> 31;
    return v;
}

static inline uint64_t key_hash(uint64_t x0, uint64_t x1, uint64_t z0, uint64_t z1) {
    return mix64(x0 ^ mix64(x1 ^ mix64(z0 ^ mix64(z1 + 0x9e3779b97f4a7c15ull))));
}

static int table_init(jw_table *t, uint64_t cap) {
    t->cap = cap;
    t->count = 0;
    t->slots = (jw_entry *)calloc(cap, sizeof(jw_entry));
    return t->slots ? 0 : -1;
}

static int table_add(jw_table *t, uint64_t x0, uint64_t x1, uint64_t z0, uint64_t z1,
                     double re, double im);

static int table_grow(jw_table *t) {
    jw_table n;
    if (table_init(&n, t->cap * 2)) return -1;
    for (uint64_t i = 0; i < t->cap; ++i) {
        jw_entry *e = &t->slots[i];
        if (e->used) table_add(&n, e->x0, e->x1, e->z0, e->z1, e->re, e->im);
    }
    free(t->slots);
    *t = n;
    return 0;
}

static int table_add(jw_table *t, uint64_t x0, uint64_t x1, uint64_t z0, uint64_t z1,
                     double re, double im) {
    if ((t->count + 1) * 10 > t->cap * 6) {
        if (table_grow(t)) return -1;
    }
    uint64_t mask = t->cap - 1;
    uint64_t h = key_hash(x0, x1, z0, z1) & mask;
    for (;;) {
        jw_entry *e = &t->slots[h];
        if (!e->used) {
            e->used = 1;
            e->x0 = x0; e->x1 = x1; e->z0 = z0; e->z1 = z1;
            e->re = re; e->im = im;
            t->count++;
            return 0;
        }
        if (e->x0 == x0 && e->x1 == x1 && e->z0 == z0 && e->z1 == z1) {
            e->re += re;
            e->im += im;
            return 0;
        }
        h = (h + 1) & mask;
    }
}

/* One raw string: coef * X^x Z^z. */
typedef struct {
    uint64_t x[2], z[2];
    double c;
} raw_t;

static inline int popc2(uint64_t a0, uint64_t a1) {
    return __builtin_popcountll(a0) + __builtin_popcountll(a1);
}

static inline void ladder(int j, int creation, raw_t out[2]) {
    /* bits strictly below j */
    uint64_t lo0, lo1;
    if (j < 64) {
        lo0 = (j == 0) ? 0 : ((1ull << j) - 1);
        lo1 = 0;
    } else {
        lo0 = ~0ull;
        lo1 = (j == 64) ? 0 : ((1ull << (j - 64)) - 1);
    }
    uint64_t e0 = (j < 64) ? (1ull << j) : 0, e1 = (j < 64) ? 0 : (1ull << (j - 64));
    out[0].x[0] = e0; out[0].x[1] = e1;
    out[0].z[0] = lo0; out[0].z[1] = lo1;
    out[0].c = 0.5;
    out[1].x[0] = e0; out[1].x[1] = e1;
    out[1].z[0] = lo0 | e0; out[1].z[1] = lo1 | e1;
    out[1].c = creation ? 0.5 : -0.5;
}

static inline raw_t raw_mul(raw_t a, raw_t b) {
    raw_t r;
    int s = popc2(a.z[0] & b.x[0], a.z[1] & b.x[1]) & 1;
    r.x[0] = a.x[0] ^ b.x[0]; r.x[1] = a.x[1] ^ b.x[1];
    r.z[0] = a.z[0] ^ b.z[0]; r.z[1] = a.z[1] ^ b.z[1];
    r.c = a.c * b.c * (s ? -1.0 : 1.0);
    return r;
}

/* Add coef * raw to the table with the (-i)^ny conversion. */
static inline int emit(jw_table *t, raw_t r, double coef, int keep_odd) {
    int ny = popc2(r.x[0] & r.z[0], r.x[1] & r.z[1]) & 3;
    double v = coef * r.c;
    /* (-i)^ny: 0 -> 1, 1 -> -i, 2 -> -1, 3 -> +i */
    switch (ny) {
        case 0: return table_add(t, r.x[0], r.x[1], r.z[0], r.z[1], v, 0.0);
        case 2: return table_add(t, r.x[0], r.x[1], r.z[0], r.z[1], -v, 0.0);
        case 1: return keep_odd ? table_add(t, r.x[0], r.x[1], r.z[0], r.z[1], 0.0, -v) : 0;
        default: return keep_odd ? table_add(t, r.x[0], r.x[1], r.z[0], r.z[1], 0.0, v) : 0;
    }
}

static inline int part_of(uint64_t x0, uint64_t x1, int n_parts) {
    return (int)(mix64(x0 * 0x9e3779b97f4a7c15ull ^ x1) % (uint64_t)n_parts);
}

static int expand_part(int part, int n_parts, int K, const double *h, const double *eri,
                       int keep_odd, jw_table *t) {
    const int nso = 2 * K;
    (void)nso;
    /* one-body */
    for (int s = 0; s < 2; ++s)
        for (int p = 0; p < K; ++p)
            for (int q = 0; q < K; ++q) {
                double v = h[p * K + q];
                if (v == 0.0) continue;
                int P = 2 * p + s, Q = 2 * q + s;
                raw_t A[2], B[2];
                ladder(P, 1, A);
                ladder(Q, 0, B);
                uint64_t x0 = A[0].x[0] ^ B[0].x[0], x1 = A[0].x[1] ^ B[0].x[1];
                if (part_of(x0, x1, n_parts) != part) continue;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        if (emit(t, raw_mul(A[a], B[b]), v, keep_odd)) return -1;
            }
    /* two-body: index u = (s*K + p)*K + q for the (p,q,s) pair, w likewise for
     * (r,s,t).  The terms for (u,w) and (w,u) are the same operator with the
     * same coefficient, so only u <= w is expanded, doubled when u < w. */
    const int64_t npair = 2LL * K * K;
    for (int64_t u = 0; u < npair; ++u) {
        int s = (int)(u / ((int64_t)K * K));
        int p = (int)((u / K) % K), q = (int)(u % K);
        int P = 2 * p + s, Q = 2 * q + s;
        raw_t A[2], D[2];
        ladder(P, 1, A);
        ladder(Q, 0, D);
        for (int64_t w = u; w < npair; ++w) {
            int tt = (int)(w / ((int64_t)K * K));
            int r = (int)((w / K) % K), ss = (int)(w % K);
            int R = 2 * r + tt, S = 2 * ss + tt;
            if (P == R || Q == S) continue;
            double v = eri[(((int64_t)p * K + q) * K + r) * K + ss];
            if (v == 0.0) continue;
            v *= (u == w) ? 0.5 : 1.0;
            uint64_t x0 = A[0].x[0] ^ D[0].x[0], x1 = A[0].x[1] ^ D[0].x[1];
            if (R < 64) x0 ^= 1ull << R; else x1 ^= 1ull << (R - 64);
            if (S < 64) x0 ^= 1ull << S; else x1 ^= 1ull << (S - 64);
            if (part_of(x0, x1, n_parts) != part) continue;
            raw_t B[2], C[2];
            ladder(R, 1, B);
            ladder(S, 0, C);
            /* operator a+_P a+_R a_S a_Q */
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    raw_t ab = raw_mul(A[a], B[b]);
                    for (int c = 0; c < 2; ++c) {
                        raw_t abc = raw_mul(ab, C[c]);
                        for (int d = 0; d < 2; ++d)
                            if (emit(t, raw_mul(abc, D[d]), v, keep_odd)) return -1;
                    }
                }
        }
    }
    return 0;
}

typedef struct {
    uint64_t x0, x1, z0, z1;
    double re, im;
} jw_out;

static int out_cmp(const void *pa, const void *pb) {
    const jw_out *a = (const jw_out *)pa, *b = (const jw_out *)pb;
    if (a->x1 != b->x1) return a->x1 < b->x1 ? -1 : 1;
    if (a->x0 != b->x0) return a->x0 < b->x0 ? -1 : 1;
    if (a->z1 != b->z1) return a->z1 < b->z1 ? -1 : 1;
    if (a->z0 != b->z0) return a->z0 < b->z0 ? -1 : 1;
    return 0;
}

/* Sort the merged terms by (x_hi, x_lo, z_hi, z_lo). */
static void sort_output(jw_result *res) {
    int64_t n = res->n_out;
    jw_out *tmp = (jw_out *)malloc(sizeof(jw_out) * (size_t)(n ? n : 1));
    if (!tmp) return;
    for (int64_t k = 0; k < n; ++k) {
        tmp[k].x0 = res->ox[2 * k]; tmp[k].x1 = res->ox[2 * k + 1];
        tmp[k].z0 = res->oz[2 * k]; tmp[k].z1 = res->oz[2 * k + 1];
        tmp[k].re = res->oc[k]; tmp[k].im = res->oc_im[k];
    }
    qsort(tmp, (size_t)n, sizeof(jw_out), out_cmp);
    for (int64_t k = 0; k < n; ++k) {
        res->ox[2 * k] = tmp[k].x0; res->ox[2 * k + 1] = tmp[k].x1;
        res->oz[2 * k] = tmp[k].z0; res->oz[2 * k + 1] = tmp[k].z1;
        res->oc[k] = tmp[k].re; res->oc_im[k] = tmp[k].im;
    }
    free(tmp);
}

/*
 * Expand and merge.  h is [K][K], eri is [K][K][K][K] in chemists' order
 * (pq|rs).  Terms with |c| < thresh after merging are dropped.  Returns an
 * opaque result (NULL on failure); its size is jw_count().
 */
void *jw_build(int K, const double *h, const double *eri, double thresh, int keep_odd,
               int n_parts) {
    if (K <= 0 || 2 * K > 128 || n_parts <= 0) return NULL;
    jw_result *res = (jw_result *)calloc(1, sizeof(jw_result));
    if (!res) return NULL;
    res->n_parts = n_parts;
    res->parts = (jw_table *)calloc((size_t)n_parts, sizeof(jw_table));
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
    for (int part = 0; part < n_parts; ++part) {
        if (table_init(&res->parts[part], 1u << 16)) { fail |= 1; continue; }
        if (expand_part(part, n_parts, K, h, eri, keep_odd, &res->parts[part])) fail |= 1;
    }
    int64_t n = 0;
    for (int part = 0; part < n_parts && !fail; ++part) {
        jw_table *t = &res->parts[part];
        for (uint64_t i = 0; i < t->cap; ++i) {
            jw_entry *e = &t->slots[i];
            if (e->used && hypot(e->re, e->im) >= thresh) ++n;
        }
    }
    if (!fail) {
        res->ox = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)(n ? n : 1));
        res->oz = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)(n ? n : 1));
        res->oc = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
        res->oc_im = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
        if (!res->ox || !res->oz || !res->oc || !res->oc_im) fail = 1;
    }
    if (!fail) {
        int64_t k = 0;
        for (int part = 0; part < n_parts; ++part) {
            jw_table *t = &res->parts[part];
            for (uint64_t i = 0; i < t->cap; ++i) {
                jw_entry *e = &t->slots[i];
                if (!(e->used && hypot(e->re, e->im) >= thresh)) continue;
                res->ox[2 * k] = e->x0; res->ox[2 * k + 1] = e->x1;
                res->oz[2 * k] = e->z0; res->oz[2 * k + 1] = e->z1;
                res->oc[k] = e->re;
                res->oc_im[k] = e->im;
                ++k;
            }
        }
        res->n_out = n;
        sort_output(res);
    }
    for (int part = 0; part < n_parts; ++part) free(res->parts[part].slots);
    free(res->parts);
    res->parts = NULL;
    if (fail) {
        free(res->ox); free(res->oz); free(res->oc); free(res->oc_im); free(res);
        return NULL;
    }
    return res;
}

int64_t jw_count(void *r) { return r ? ((jw_result *)r)->n_out : -1; }

void jw_fetch(void *r, uint64_t *x, uint64_t *z, double *c_re, double *c_im) {
    jw_result *res = (jw_result *)r;
    memcpy(x, res->ox, sizeof(uint64_t) * 2 * (size_t)res->n_out);
    memcpy(z, res->oz, sizeof(uint64_t) * 2 * (size_t)res->n_out);
    memcpy(c_re, res->oc, sizeof(double) * (size_t)res->n_out);
    memcpy(c_im, res->oc_im, sizeof(double) * (size_t)res->n_out);
}

void jw_free(void *r) {
    jw_result *res = (jw_result *)r;
    if (!res) return;
    free(res->ox); free(res->oz); free(res->oc); free(res->oc_im);
    free(res);
}
