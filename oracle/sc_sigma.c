/*
 * CPU oracle (test infrastructure only): row-driven Slater-Condon sigma.
 *
 * Computes sigma_L = sum_K <L|H|K> c_K over an explicit, sorted list of
 * determinants (occupation bitstrings over M <= 64 spin-orbitals), for
 *   H = e_core + sum_pq h_pq a+_p a_q + 1/2 sum_pqrs (pq|rs) a+_p a+_r a_s a_q
 * restricted to the listed determinants (sigma = P H P c, P the projector on
 * the listed space).  This is the plain definition of the product that the
 * categorical sigma build evaluates (the sigma equations of the Methods
 * section; the build is lossless, so its result is exactly this product).
 *
 * Determinant |b> = a+_{i1} ... a+_{iN}|0> with i1 < ... < iN.  Every sign is
 * obtained by applying the annihilation/creation operators one at a time to
 * the bitstring and counting occupied orbitals below the acted-on index.
 * Matrix elements use the textbook Slater-Condon rules in their general form
 * (no integral symmetry assumed):
 *   diagonal:  sum_i h_ii + 1/2 sum_{i!=j} [(ii|jj) - (ij|ji)]
 *   single  (L = a+_p a_q K): s * [h_pq + 1/2 sum_{j in K, j!=q}
 *               ((pq|jj) + (jj|pq) - (pj|jq) - (jq|pj))]
 *   double  (L = a+_p a+_r a_s a_q K): s * 1/2 [(pq|rs) + (rs|pq) - (ps|rq) - (rq|ps)]
 * where s is the sign of the operator string acting on K.
 *
 * Shares no code with the GPU library.  Complex arithmetic throughout (real
 * inputs simply carry zero imaginary parts).
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static inline int popc(uint64_t x) { return __builtin_popcountll(x); }

/* a_q |b>: returns 0 if q not occupied; else sets *out and multiplies *sgn. */
static inline int annih(uint64_t b, int q, uint64_t* out, int* sgn) {
    uint64_t bit = 1ULL << q;
    if (!(b & bit)) return 0;
    if (popc(b & (bit - 1)) & 1) *sgn = -*sgn;
    *out = b ^ bit;
    return 1;
}

/* a+_p |b> */
static inline int creat(uint64_t b, int p, uint64_t* out, int* sgn) {
    uint64_t bit = 1ULL << p;
    if (b & bit) return 0;
    if (popc(b & (bit - 1)) & 1) *sgn = -*sgn;
    *out = b | bit;
    return 1;
}

static inline int64_t find_det(const uint64_t* dets, int64_t n, uint64_t key) {
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        uint64_t v = dets[mid];
        if (v == key) return mid;
        if (v < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

typedef struct {
    int M;
    const cplx* h; /* [M][M] */
    const cplx* g; /* [M][M][M][M], (pq|rs) */
    double e_core;
} ham_t;

static inline cplx H1(const ham_t* H, int p, int q) { return H->h[p * H->M + q]; }
static inline cplx G(const ham_t* H, int p, int q, int r, int s) {
    int M = H->M;
    return H->g[(((size_t)p * M + q) * M + r) * M + s];
}

static int occ_list(uint64_t b, int* occ) {
    int n = 0;
    while (b) { int i = __builtin_ctzll(b); occ[n++] = i; b &= b - 1; }
    return n;
}

static cplx diag_elem(const ham_t* H, uint64_t b) {
    int occ[64];
    int n = occ_list(b, occ);
    cplx e = H->e_core;
    for (int a = 0; a < n; ++a) e += H1(H, occ[a], occ[a]);
    cplx t = 0;
    for (int a = 0; a < n; ++a)
        for (int c = 0; c < n; ++c) {
            if (a == c) continue;
            int i = occ[a], j = occ[c];
            t += G(H, i, i, j, j) - G(H, i, j, j, i);
        }
    return e + 0.5 * t;
}

/* <L| H |K> for L = a+_p a_q K (p != q), sign s given. */
static cplx single_elem(const ham_t* H, uint64_t K, int p, int q) {
    cplx v = H1(H, p, q);
    cplx t = 0;
    uint64_t rest = K & ~(1ULL << q);
    while (rest) {
        int j = __builtin_ctzll(rest);
        rest &= rest - 1;
        t += G(H, p, q, j, j) + G(H, j, j, p, q) - G(H, p, j, j, q) - G(H, j, q, p, j);
    }
    return v + 0.5 * t;
}

static cplx double_elem(const ham_t* H, int p, int q, int r, int s) {
    return 0.5 * (G(H, p, q, r, s) + G(H, r, s, p, q) - G(H, p, s, r, q) - G(H, r, q, p, s));
}

/* One row: sigma_L = sum_K <L|H|K> c_K over listed K. */
static cplx row_sigma(const ham_t* H, const uint64_t* dets, int64_t n, uint64_t L, const cplx* c) {
    int M = H->M;
    int occ[64], vir[64];
    int no = occ_list(L, occ);
    int nv = 0;
    for (int i = 0; i < M; ++i) if (!(L & (1ULL << i))) vir[nv++] = i;
    int64_t il = find_det(dets, n, L);
    cplx acc = diag_elem(H, L) * c[il];
    /* singles: K = a+_q a_p L (p in L, q not in L); then L = a+_p a_q K */
    for (int a = 0; a < no; ++a)
        for (int b = 0; b < nv; ++b) {
            int p = occ[a], q = vir[b];
            uint64_t K = (L & ~(1ULL << p)) | (1ULL << q);
            int64_t ik = find_det(dets, n, K);
            if (ik < 0) continue;
            /* sign of a+_p a_q acting on K */
            int s2 = 1;
            uint64_t u1 = 0, u2 = 0;
            annih(K, q, &u1, &s2);
            creat(u1, p, &u2, &s2);
            acc += (double)s2 * single_elem(H, K, p, q) * c[ik];
        }
    /* doubles: K = L - {p, r} + {q, s}, p < r in L, q < s not in L */
    for (int a = 0; a < no; ++a)
        for (int a2 = a + 1; a2 < no; ++a2)
            for (int b = 0; b < nv; ++b)
                for (int b2 = b + 1; b2 < nv; ++b2) {
                    int p = occ[a], r = occ[a2], q = vir[b], s = vir[b2];
                    uint64_t K = (L & ~((1ULL << p) | (1ULL << r))) | (1ULL << q) | (1ULL << s);
                    int64_t ik = find_det(dets, n, K);
                    if (ik < 0) continue;
                    /* sign of a+_p a+_r a_s a_q acting on K */
                    int sg = 1;
                    uint64_t t1 = 0, t2 = 0, t3 = 0, t4 = 0;
                    annih(K, q, &t1, &sg);
                    annih(t1, s, &t2, &sg);
                    creat(t2, r, &t3, &sg);
                    creat(t3, p, &t4, &sg);
                    acc += (double)sg * double_elem(H, p, q, r, s) * c[ik];
                }
    return acc;
}

/* Full sigma over all listed determinants. h, g, c, sigma: interleaved complex. */
void oracle_sigma(int M, int64_t n, const uint64_t* dets, const double* h, const double* g,
                  double e_core, const double* c, double* sigma, int nthreads) {
    ham_t H = {M, (const cplx*)h, (const cplx*)g, e_core};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i)
        ((cplx*)sigma)[i] = row_sigma(&H, dets, n, dets[i], (const cplx*)c);
}

/* Selected rows only: sigma_rows[j] = sigma_{rows[j]}. */
void oracle_sigma_rows(int M, int64_t n, const uint64_t* dets, const double* h, const double* g,
                       double e_core, const double* c, const int64_t* rows, int64_t nrows,
                       double* out, int nthreads) {
    ham_t H = {M, (const cplx*)h, (const cplx*)g, e_core};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t j = 0; j < nrows; ++j)
        ((cplx*)out)[j] = row_sigma(&H, dets, n, dets[rows[j]], (const cplx*)c);
}

/* Row j of H as a list of (column index, value); returns the count written
 * (at most cap).  Used to build dense matrices of small spaces. */
int64_t oracle_h_row(int M, int64_t n, const uint64_t* dets, const double* h, const double* g,
                     double e_core, int64_t row, double* vals, int64_t cap) {
    ham_t H = {M, (const cplx*)h, (const cplx*)g, e_core};
    uint64_t L = dets[row];
    int occ[64], vir[64];
    int no = occ_list(L, occ), nv = 0;
    for (int i = 0; i < M; ++i) if (!(L & (1ULL << i))) vir[nv++] = i;
    int64_t w = 0; /* each entry: (column index, re, im) as three doubles */
#define EMIT(idx, val) do { if (w < cap) { ((double*)vals)[3 * w] = (double)(idx); \
        ((double*)vals)[3 * w + 1] = creal(val); ((double*)vals)[3 * w + 2] = cimag(val); } ++w; } while (0)
    EMIT(row, diag_elem(&H, L));
    for (int a = 0; a < no; ++a)
        for (int b = 0; b < nv; ++b) {
            int p = occ[a], q = vir[b];
            uint64_t K = (L & ~(1ULL << p)) | (1ULL << q);
            int64_t ik = find_det(dets, n, K);
            if (ik < 0) continue;
            int s2 = 1;
            uint64_t u1 = 0, u2 = 0;
            annih(K, q, &u1, &s2);
            creat(u1, p, &u2, &s2);
            EMIT(ik, (double)s2 * single_elem(&H, K, p, q));
        }
    for (int a = 0; a < no; ++a)
        for (int a2 = a + 1; a2 < no; ++a2)
            for (int b = 0; b < nv; ++b)
                for (int b2 = b + 1; b2 < nv; ++b2) {
                    int p = occ[a], r = occ[a2], q = vir[b], s = vir[b2];
                    uint64_t K = (L & ~((1ULL << p) | (1ULL << r))) | (1ULL << q) | (1ULL << s);
                    int64_t ik = find_det(dets, n, K);
                    if (ik < 0) continue;
                    int sg = 1;
                    uint64_t t1 = 0, t2 = 0, t3 = 0, t4 = 0;
                    annih(K, q, &t1, &sg);
                    annih(t1, s, &t2, &sg);
                    creat(t2, r, &t3, &sg);
                    creat(t3, p, &t4, &sg);
                    EMIT(ik, (double)sg * double_elem(&H, p, q, r, s));
                }
#undef EMIT
    return w;
}

/* Row L of P H P for a windowed space given by its subspaces (contiguous,
 * sizes sub[k], electron windows [lo[k], hi[k]]), without a determinant list:
 * every determinant reached from L by at most two electron moves is kept when
 * its subspace occupations lie in the windows.  Writes (bits, re, im) triples
 * (bits stored through a uint64 view) and returns the count (at most cap are
 * written).  Used on spaces too large to enumerate. */
static int in_windows(uint64_t b, int K, const int* sub, const int* lo, const int* hi) {
    int off = 0;
    for (int k = 0; k < K; ++k) {
        uint64_t m = (sub[k] >= 64) ? ~0ULL : (((1ULL << sub[k]) - 1ULL) << off);
        int n = popc(b & m);
        if (n < lo[k] || n > hi[k]) return 0;
        off += sub[k];
    }
    return 1;
}

int64_t oracle_h_row_window(int M, int K, const int* sub, const int* lo, const int* hi, const double* h,
                            const double* g, double e_core, uint64_t L, uint64_t* bits, double* vals, int64_t cap) {
    ham_t H = {M, (const cplx*)h, (const cplx*)g, e_core};
    int occ[64], vir[64];
    int no = occ_list(L, occ), nv = 0;
    for (int i = 0; i < M; ++i) if (!(L & (1ULL << i))) vir[nv++] = i;
    int64_t w = 0;
#define EMITB(b, val) do { if (w < cap) { bits[w] = (b); vals[2 * w] = creal(val); vals[2 * w + 1] = cimag(val); } \
        ++w; } while (0)
    EMITB(L, diag_elem(&H, L));
    for (int a = 0; a < no; ++a)
        for (int b = 0; b < nv; ++b) {
            int p = occ[a], q = vir[b];
            uint64_t Kd = (L & ~(1ULL << p)) | (1ULL << q);
            if (!in_windows(Kd, K, sub, lo, hi)) continue;
            int s2 = 1;
            uint64_t u1 = 0, u2 = 0;
            annih(Kd, q, &u1, &s2);
            creat(u1, p, &u2, &s2);
            EMITB(Kd, (double)s2 * single_elem(&H, Kd, p, q));
        }
    for (int a = 0; a < no; ++a)
        for (int a2 = a + 1; a2 < no; ++a2)
            for (int b = 0; b < nv; ++b)
                for (int b2 = b + 1; b2 < nv; ++b2) {
                    int p = occ[a], r = occ[a2], q = vir[b], s = vir[b2];
                    uint64_t Kd = (L & ~((1ULL << p) | (1ULL << r))) | (1ULL << q) | (1ULL << s);
                    if (!in_windows(Kd, K, sub, lo, hi)) continue;
                    int sg = 1;
                    uint64_t t1 = 0, t2 = 0, t3 = 0, t4 = 0;
                    annih(Kd, q, &t1, &sg);
                    annih(t1, s, &t2, &sg);
                    creat(t2, r, &t3, &sg);
                    creat(t3, p, &t4, &sg);
                    EMITB(Kd, (double)sg * double_elem(&H, p, q, r, s));
                }
#undef EMITB
    return w;
}

/* Diagonal elements <b|H|b> for a list of determinants (real part). */
void oracle_diag(int M, int64_t n, const uint64_t* dets, const double* h, const double* g,
                 double e_core, double* out, int nthreads) {
    ham_t H = {M, (const cplx*)h, (const cplx*)g, e_core};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) out[i] = creal(diag_elem(&H, dets[i]));
}
