/*
 * Plain CPU oracle for the order-statistics approximate nearest-neighbour
 * search of Verdoliva, Cozzolino and Poggi (arXiv 1509.03453, "ROSANNA").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the GPU library; the product path never calls it.
 *
 * It is written for a reader checking it against the paper by eye: plain
 * loops, no blocking, no reordering of any sum.  Notation follows the paper:
 *   K    vector length                                  (Table I)
 *   G    number of largest-magnitude components hashed (Table I)
 *   N_C  number of cones, C(K,G) * 2^G                  (Section 2, Table I)
 * Indices are 0-based here; the paper counts from 1.
 *
 * Readings taken where the paper is silent (each one is pinned or listed as
 * unpinned by the test-suite):
 *   R1  equal magnitudes: the lower component index ranks first.
 *   R2  the sign bit of a component is 1 unless the value is < 0, so zero and
 *       negative zero count as non-negative (Fig. 2 caption: c=0 holds the
 *       negative values, c=1 "the others").
 *   R3  cone id = colex rank of the profile (the G indices in ascending order)
 *       times 2^G, plus the sign bits with the lowest index as most
 *       significant bit (Fig. 2, right table).
 *   R4  probe order (Section 3.B): L-subsets T of query rank positions in
 *       lexicographic order with the query's own signs (phase A), then the
 *       same subsets with h = 1..G signs flipped (phase B).  Lexicographic
 *       order on T is non-decreasing in the paper's profile distance.
 *   R5  the search budget B is met with whole cones: probing stops after the
 *       first cone at which the running candidate count reaches B.
 *   R6  arg-min over (FP32 distance, original row) in lexicographic order.
 *   R9  several bases: coordinates in basis r are M_r times the vector, in
 *       FP32 term by term (ascending j); distances stay on the original
 *       vectors (a rotation preserves them).
 *   R10 several bases: the l-th cone of every basis (empty cones included)
 *       forms level l; the budget counts the rows of visited cones, rows seen
 *       again in another basis included; ncand counts distinct rows.
 *   R11 PCA front-end (Section 4.B): the key of a vector is P (x - mu), the
 *       first k principal coordinates of the centred vector, in FP32 term by
 *       term (the difference, each product and each sum rounded, ascending
 *       j); cones come from the keys, distances from the full original
 *       vectors (the paper computes them over all components of the rotated
 *       vectors, which is the same distance).
 *   R12 coarse clusters (ROSANNA+, Section 4.B): Lloyd k-means from given
 *       initial centroids, a fixed number of iterations; a row goes to the
 *       centroid at the smallest FP32 term-by-term squared distance (lower
 *       centroid on ties); a centroid becomes the float64 mean of its rows
 *       (summed in ascending row order) rounded to FP32, and keeps its value
 *       when no row is assigned.  The table buckets rows by (cluster, cone of
 *       the residual x - c in FP32).  A query takes the nprobe centroids
 *       nearest to it (FP32 distance, lower centroid on ties); in each it
 *       walks the cones of its residual with budget ceil(B / nprobe); every
 *       row met is compared on the full vectors; ncand sums the clusters'
 *       candidates.
 *   R13 fixed-C mode (Section 3, Table III): the budget counts cones
 *       instead of rows: the first C cones of the walk (empty ones included)
 *       are visited, per basis (several bases: levels 0..C-1 of every basis)
 *       and per searched cluster.  When every cone taken is empty the search
 *       has no candidate: the row is -1 and the distance +inf.
 *   R14 structured bases (Section 3.D, Walsh-Hadamard matrices in place of
 *       pseudo-random ones): basis r is H diag(s_r) / sqrt(K), H the
 *       Sylvester-ordered Hadamard matrix (K a power of two), s_r a vector
 *       of signs.  Coordinates come from the fast transform (sign flips,
 *       then butterflies with strides 1, 2, 4, ..., each (a, b) -> (a + b,
 *       a - b) rounded in FP32), left unnormalised: the positive factor
 *       1/sqrt(K) changes neither the order of the magnitudes nor the signs,
 *       so the cones are those of the orthonormal basis.
 *   R15 sparse table (Section 4: a second-level hash table manages the
 *       tables when the number of cones is very large): only the non-empty
 *       cones are stored, as a list of distinct cone ids in ascending order
 *       with the offsets of their rows (rows sorted by cone, then by row
 *       id); a cone of the walk that is not in the list is empty.  The walk
 *       and the stopping rules are those of the dense table (row budget:
 *       reading R5; fixed C: reading R13), so both tables give the same
 *       search; a budget of at least N (or C >= N_C) takes every row.  A
 *       walk takes at most 2^22 positions: a row budget not met by then (or
 *       a C beyond it) stops there, which bounds the work of a walk through
 *       mostly empty cones.
 *
 * Precision: distances are produced both in double (the definition, eq. (1))
 * and in FP32 evaluated term by term in ascending component order with each
 * subtraction, product and sum rounded separately (the precision in which the
 * arg-min decision is taken).  Built with -ffp-contract=off and without
 * -ffast-math so that no operation is fused or re-associated.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_F32 = 0, ORC_F16 = 1, ORC_U8 = 2 };

/* ------------------------------------------------------------------------ */
/* Scalars                                                                    */
/* ------------------------------------------------------------------------ */

/* IEEE 754 binary16 -> binary32, exact (every half is a float). */
static float half_to_float(uint16_t h)
{
    int s = (h >> 15) & 1;
    int e = (h >> 10) & 0x1f;
    int m = h & 0x3ff;
    float v;
    if (e == 0)
        v = ldexpf((float)m, -24);              /* zero and subnormals      */
    else if (e == 31)
        v = m ? NAN : INFINITY;
    else
        v = ldexpf((float)(m | 0x400), e - 25); /* (1 + m/1024) 2^(e-15)    */
    return s ? -v : v;
}

/* Component i of row n, converted exactly to float. */
static float elem(const void *X, int dtype, int64_t n, int K, int i)
{
    int64_t at = n * (int64_t)K + i;
    if (dtype == ORC_F16)
        return half_to_float(((const uint16_t *)X)[at]);
    if (dtype == ORC_U8)
        return (float)((const uint8_t *)X)[at];
    return ((const float *)X)[at];
}

static void load_row(const void *X, int dtype, int64_t n, int K, float *out)
{
    for (int i = 0; i < K; i++)
        out[i] = elem(X, dtype, n, K, i);
}

/* Binomial coefficient C(n,k); 0 when k > n or n < 0. */
int64_t orc_binom(int n, int k)
{
    if (k < 0 || n < 0 || k > n)
        return 0;
    int64_t c = 1;
    for (int t = 0; t < k; t++)
        c = c * (n - t) / (t + 1);
    return c;
}

/* Section 2, Table I: N_C = C(K,G) 2^G. */
int64_t orc_num_cones(int K, int G)
{
    return orc_binom(K, G) << G;
}

/* ------------------------------------------------------------------------ */
/* Hashing (Section 2, eq. (2), Fig. 2)                                      */
/* ------------------------------------------------------------------------ */

/* True when component i comes before component j in decreasing-magnitude
 * order (reading R1 breaks ties by the lower index). */
static int mag_before(const float *v, int i, int j)
{
    float ai = fabsf(v[i]), aj = fabsf(v[j]);
    if (ai != aj)
        return ai > aj;
    return i < j;
}

/* Full decreasing-magnitude order of one vector: order[0] is the index of
 * the largest |v_i|.  Insertion sort, K <= 256. */
void orc_rank_order(const float *v, int K, int32_t *order)
{
    for (int i = 0; i < K; i++) {
        int at = i;
        while (at > 0 && mag_before(v, i, order[at - 1])) {
            order[at] = order[at - 1];
            at--;
        }
        order[at] = i;
    }
}

/* Sign bit of a component under reading R2. */
static int sign_bit(float x)
{
    return x < 0.0f ? 0 : 1;
}

/* Cone id of a profile given as G distinct component indices (any order)
 * with one sign bit each (reading R3): the indices are sorted ascending,
 * p_1 < ... < p_G, the profile's colex rank is sum_j C(p_j, j), and the sign
 * bits follow in ascending index order, most significant first. */
static int64_t cone_id(const int32_t *idx, const int *sgn, int G)
{
    int32_t p[256];
    int s[256];
    for (int j = 0; j < G; j++) {
        p[j] = idx[j];
        s[j] = sgn[j];
    }
    for (int a = 1; a < G; a++)          /* insertion sort, carrying signs */
        for (int b = a; b > 0 && p[b - 1] > p[b]; b--) {
            int32_t tp = p[b]; p[b] = p[b - 1]; p[b - 1] = tp;
            int ts = s[b]; s[b] = s[b - 1]; s[b - 1] = ts;
        }
    int64_t rank = 0;
    for (int j = 0; j < G; j++)
        rank += orc_binom(p[j], j + 1);
    int64_t bits = 0;
    for (int j = 0; j < G; j++)
        bits = (bits << 1) | s[j];
    return (rank << G) | bits;
}

/* Hash every row: the G largest-magnitude components in decreasing order
 * (top_idx[n*G + j]), their sign bits (top_sign) and the row's cone id. */
int orc_hash(const void *X, int dtype, int64_t N, int K, int G,
             int32_t *top_idx, uint8_t *top_sign, int64_t *cone)
{
    if (K < 1 || K > 256 || G < 1 || G > K)
        return -1;
    for (int64_t n = 0; n < N; n++) {
        float v[256];
        int32_t order[256];
        int s[256];
        load_row(X, dtype, n, K, v);
        orc_rank_order(v, K, order);
        for (int j = 0; j < G; j++) {
            s[j] = sign_bit(v[order[j]]);
            if (top_idx)
                top_idx[n * G + j] = order[j];
            if (top_sign)
                top_sign[n * G + j] = (uint8_t)s[j];
        }
        cone[n] = cone_id(order, s, G);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Bucketing: one hash table, rows grouped by cone (Section 4)               */
/* ------------------------------------------------------------------------ */

/* Counting sort of row ids by cone, stable (rows of one cone stay in
 * ascending original order).  offsets has NC+1 entries; bucket c occupies
 * perm[offsets[c] .. offsets[c+1]). */
int orc_bucket(const int64_t *cone, int64_t N, int64_t NC, int64_t *offsets, int64_t *perm)
{
    for (int64_t c = 0; c <= NC; c++)
        offsets[c] = 0;
    for (int64_t n = 0; n < N; n++) {
        if (cone[n] < 0 || cone[n] >= NC)
            return -1;
        offsets[cone[n] + 1]++;
    }
    for (int64_t c = 0; c < NC; c++)
        offsets[c + 1] += offsets[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(NC > 0 ? NC : 1));
    if (!fill)
        return -2;
    for (int64_t c = 0; c < NC; c++)
        fill[c] = offsets[c];
    for (int64_t n = 0; n < N; n++)
        perm[fill[cone[n]]++] = n;
    free(fill);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Probe order (Section 3.B, Algorithm 1)                                    */
/* ------------------------------------------------------------------------ */

/* Lexicographic successor of a G-subset t[0] < ... < t[G-1] of {0..K-1};
 * returns 0 when t was the last one. */
static int lex_next(int32_t *t, int K, int G)
{
    int j = G - 1;
    while (j >= 0 && t[j] == K - G + j)
        j--;
    if (j < 0)
        return 0;
    t[j]++;
    for (int a = j + 1; a < G; a++)
        t[a] = t[a - 1] + 1;
    return 1;
}

static int popcount_int(int m)
{
    int c = 0;
    while (m) {
        c += m & 1;
        m >>= 1;
    }
    return c;
}

/* Walks the cones of one query in probe order and calls visit(cone) for each
 * one; stops early when visit returns nonzero.  Phase A: subsets T of query
 * rank positions in lexicographic order, profile {order[t_j]}, the query's
 * own signs.  Phase B: h = 1..G flipped signs; for each T in lexicographic
 * order, flip masks of popcount h in ascending value, mask bit (G-1-j)
 * flipping the sign of component order[t_j].  Phase A alone covers each
 * profile once; A and B together cover all N_C cones once. */
typedef int (*visit_fn)(int64_t cone, void *ctx);

static void walk_cones(const float *y, int K, int G, visit_fn visit, void *ctx)
{
    int32_t order[256], t[256], idx[256];
    int s[256];
    orc_rank_order(y, K, order);
    for (int h = 0; h <= G; h++) {
        for (int j = 0; j < G; j++)
            t[j] = j;
        do {
            for (int mask = 0; mask < (1 << G); mask++) {
                if (popcount_int(mask) != h)
                    continue;
                for (int j = 0; j < G; j++) {
                    idx[j] = order[t[j]];
                    s[j] = sign_bit(y[idx[j]]) ^ ((mask >> (G - 1 - j)) & 1);
                }
                if (visit(cone_id(idx, s, G), ctx))
                    return;
            }
        } while (lex_next(t, K, G));
    }
}

struct collect_ctx {
    int64_t *out;
    int64_t cap, n;
};

static int collect_all(int64_t cone, void *vctx)
{
    struct collect_ctx *c = (struct collect_ctx *)vctx;
    if (c->n < c->cap)
        c->out[c->n] = cone;
    c->n++;
    return 0;
}

/* Every cone in the query's probe order, empty or not (N_C entries). */
int64_t orc_walk(const float *y, int K, int G, int64_t *cones, int64_t cap)
{
    struct collect_ctx c = { cones, cap, 0 };
    walk_cones(y, K, G, collect_all, &c);
    return c.n;
}

struct budget_ctx {
    const int64_t *offsets;
    int64_t B, cum;
    int64_t *probes;
    int64_t cap, n;
};

/* Reading R5: empty cones are skipped; whole cones are added until the
 * running count of candidates reaches B. */
static int take_until_budget(int64_t cone, void *vctx)
{
    struct budget_ctx *c = (struct budget_ctx *)vctx;
    int64_t size = c->offsets[cone + 1] - c->offsets[cone];
    if (size == 0)
        return 0;
    if (c->n < c->cap)
        c->probes[c->n] = cone;
    c->n++;
    c->cum += size;
    return c->cum >= c->B;
}

/* Probe list of one query: the non-empty cones visited within budget B, in
 * order.  Returns the number of probes (entries beyond cap are counted but
 * not stored); *ncand receives the number of candidates they hold. */
int64_t orc_probe(const float *y, int K, int G, const int64_t *offsets, int64_t B,
                  int64_t *probes, int64_t cap, int64_t *ncand)
{
    struct budget_ctx c = { offsets, B, 0, probes, cap, 0 };
    walk_cones(y, K, G, take_until_budget, &c);
    *ncand = c.cum;
    return c.n;
}

struct cones_ctx {
    const int64_t *offsets;
    int64_t C, seen, cum;
    int64_t *probes;
    int64_t cap, n;
};

/* Reading R13: the first C cones of the walk, empty ones included; the
 * non-empty ones are the probes. */
static int take_first_cones(int64_t cone, void *vctx)
{
    struct cones_ctx *c = (struct cones_ctx *)vctx;
    if (c->seen >= c->C)
        return 1;
    c->seen++;
    int64_t size = c->offsets[cone + 1] - c->offsets[cone];
    if (size > 0) {
        if (c->n < c->cap)
            c->probes[c->n] = cone;
        c->n++;
        c->cum += size;
    }
    return c->seen >= c->C;
}

/* Probe list of one query in fixed-C mode. */
int64_t orc_probe_cones(const float *y, int K, int G, const int64_t *offsets, int64_t C,
                        int64_t *probes, int64_t cap, int64_t *ncand)
{
    struct cones_ctx c = { offsets, C, 0, 0, probes, cap, 0 };
    walk_cones(y, K, G, take_first_cones, &c);
    *ncand = c.cum;
    return c.n;
}

/* ------------------------------------------------------------------------ */
/* Distance and arg-min (eq. (1), Algorithm 1)                               */
/* ------------------------------------------------------------------------ */

/* Squared Euclidean distance: in FP32 term by term (i ascending, each
 * operation rounded) and in double. */
static void dist2(const float *x, const float *y, int K, float *d32, double *d64)
{
    float acc = 0.0f;
    double acc64 = 0.0;
    for (int i = 0; i < K; i++) {
        float diff = x[i] - y[i];
        float sq = diff * diff;
        acc = acc + sq;
        double e = (double)x[i] - (double)y[i];
        acc64 += e * e;
    }
    *d32 = acc;
    *d64 = acc64;
}

/* Keeps the smaller of (d, row) pairs in lexicographic order (reading R6). */
static void argmin_update(float d, int64_t row, float *best_d, int64_t *best_row)
{
    if (d < *best_d || (d == *best_d && row < *best_row)) {
        *best_d = d;
        *best_row = row;
    }
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Approximate NN search with one basis (Algorithm 1 with R = 1), with the
 * cones taken from keys (reading R11): the table was built from the rows'
 * keys of length Kk; each query walks the cones of its key (row q of Yk, or
 * the query itself when Yk is NULL, Kk = K), its probes are visited in order
 * until B candidates are reached (with cones set, reading R13: the first B
 * cones of the walk), and every row of those cones is compared with the
 * query on all K components.  Outputs per query: the row (out_idx),
 * its FP32 and double distances, and the number of candidates. */
int orc_search_keyed(const void *X, int xdtype, int64_t N, int K, int Kk, int G,
                     const int64_t *offsets, const int64_t *perm,
                     const void *Y, int ydtype, const float *Yk, int64_t Q, int64_t B,
                     int64_t *out_idx, float *out_d32, double *out_d64, int64_t *out_ncand,
                     int nthreads, int cones)
{
    (void)N;
    if (K < 1 || K > 256 || Kk < 1 || Kk > 256 || G < 1 || G > Kk || B < 1)
        return -1;
    if (!Yk && Kk != K)
        return -1;
    int64_t NC = orc_num_cones(Kk, G);
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < Q; q++) {
        float y[256], yk[256], x[256];
        load_row(Y, ydtype, q, K, y);
        if (Yk)
            memcpy(yk, Yk + q * Kk, sizeof(float) * (size_t)Kk);
        else
            memcpy(yk, y, sizeof(float) * (size_t)K);
        int64_t *probes = (int64_t *)malloc(sizeof(int64_t) * (size_t)NC);
        if (!probes) {
#pragma omp atomic write
            bad = 1;
            continue;
        }
        int64_t ncand = 0;
        int64_t np = cones ? orc_probe_cones(yk, Kk, G, offsets, B, probes, NC, &ncand)
                           : orc_probe(yk, Kk, G, offsets, B, probes, NC, &ncand);
        float best_d = INFINITY;
        int64_t best_row = INT64_MAX;
        double best_d64 = INFINITY;
        for (int64_t k = 0; k < np; k++) {
            int64_t c = probes[k];
            for (int64_t pos = offsets[c]; pos < offsets[c + 1]; pos++) {
                int64_t row = perm[pos];
                float d32;
                double d64;
                load_row(X, xdtype, row, K, x);
                dist2(x, y, K, &d32, &d64);
                int64_t before = best_row;
                argmin_update(d32, row, &best_d, &best_row);
                if (best_row != before)
                    best_d64 = d64;
            }
        }
        out_idx[q] = best_row == INT64_MAX ? -1 : best_row;  /* -1: no candidate (R13) */
        out_d32[q] = best_d;
        out_d64[q] = best_d64;
        out_ncand[q] = ncand;
        free(probes);
    }
    return bad ? -2 : 0;
}

/* Approximate NN search with one basis (Algorithm 1 with R = 1): the query's
 * cones are probed in order until B candidates are reached, and every row
 * of those cones is compared with the query. */
int orc_search(const void *X, int xdtype, int64_t N, int K, int G,
               const int64_t *offsets, const int64_t *perm,
               const void *Y, int ydtype, int64_t Q, int64_t B,
               int64_t *out_idx, float *out_d32, double *out_d64, int64_t *out_ncand,
               int nthreads)
{
    return orc_search_keyed(X, xdtype, N, K, K, G, offsets, perm, Y, ydtype, NULL, Q, B,
                            out_idx, out_d32, out_d64, out_ncand, nthreads, 0);
}

/* Exact NN by linear search over all rows (eq. (1)).  idx32/d32 take the
 * arg-min decision on FP32 distances; idx64/d64 on double distances (ground
 * truth for recall: a result is right when its double distance equals d64). */
int orc_exhaustive(const void *X, int xdtype, int64_t N, int K,
                   const void *Y, int ydtype, int64_t Q,
                   int64_t *idx32, float *d32_out, int64_t *idx64, double *d64_out,
                   int nthreads)
{
    if (K < 1 || K > 256)
        return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < Q; q++) {
        float y[256], x[256];
        load_row(Y, ydtype, q, K, y);
        float b32 = INFINITY;
        int64_t r32 = INT64_MAX, r64 = INT64_MAX;
        double b64 = INFINITY;
        for (int64_t n = 0; n < N; n++) {
            float d32;
            double d64;
            load_row(X, xdtype, n, K, x);
            dist2(x, y, K, &d32, &d64);
            argmin_update(d32, n, &b32, &r32);
            if (d64 < b64 || (d64 == b64 && n < r64)) {
                b64 = d64;
                r64 = n;
            }
        }
        idx32[q] = r32;
        d32_out[q] = b32;
        idx64[q] = r64;
        d64_out[q] = b64;
    }
    return 0;
}

/* Double distance of given (query, row) pairs; used to score recall. */
int orc_pair_d64(const void *X, int xdtype, int K, const void *Y, int ydtype,
                 const int64_t *rows, int64_t Q, double *out)
{
    for (int64_t q = 0; q < Q; q++) {
        float y[256], x[256];
        float d32;
        load_row(Y, ydtype, q, K, y);
        load_row(X, xdtype, rows[q], K, x);
        dist2(x, y, K, &d32, &out[q]);
    }
    return 0;
}

/* FP32 distance of given (query, row) pairs, same evaluation as the search. */
int orc_pair_d32(const void *X, int xdtype, int K, const void *Y, int ydtype,
                 const int64_t *rows, int64_t Q, float *out)
{
    for (int64_t q = 0; q < Q; q++) {
        float y[256], x[256];
        double d64;
        load_row(Y, ydtype, q, K, y);
        load_row(X, xdtype, rows[q], K, x);
        dist2(x, y, K, &out[q], &d64);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Screened search with an exact re-rank (reading R7)                        */
/* ------------------------------------------------------------------------ */
/*
 * Reading R7 (not in the paper; the paper always computes exact distances on
 * the original vectors, Section 1 and Algorithm 1): candidates are first
 * ranked by d~ = ||x^||^2 - 2 q^.x^, where x^ and q^ are x and q rounded to
 * a short format (bfloat16, or binary16 for binary16 data) with round to
 * nearest, ties to even; the R smallest (d~, row) pairs survive and the
 * exact FP32 distance of eq. (1) decides among them.  d~ is evaluated in
 * double on the rounded values.
 */

/* Round to `bits` significant bits (nearest, ties to even) with the
 * exponent range of the target format: smallest normal 2^emin, values below
 * it quantised to 2^(emin - bits + 1); overflow past the largest finite
 * value gives infinity. */
static double round_sig(double x, int bits, int emin, double maxfin)
{
    if (x == 0.0 || !isfinite(x))
        return x;
    int e = ilogb(x);
    if (e < emin)
        e = emin;
    double q = ldexp(1.0, e - bits + 1);   /* spacing of the format at |x| */
    double r = nearbyint(x / q) * q;       /* default mode: ties to even */
    if (fabs(r) > maxfin)
        return copysign(INFINITY, x);
    return r;
}

/* bfloat16: 8 significant bits, exponent range of binary32. */
static double to_bf16(float x)
{
    return round_sig((double)x, 8, -126, 3.3895313892515355e38);
}

/* binary16: 11 significant bits, smallest normal 2^-14, largest 65504. */
static double to_f16(float x)
{
    return round_sig((double)x, 11, -14, 65504.0);
}

struct cand {
    double dt;
    int64_t row;
};

static int cand_less(const struct cand *a, const struct cand *b)
{
    return a->dt < b->dt || (a->dt == b->dt && a->row < b->row);
}

/* Screened search: same probe walk and candidates as orc_search; out_dt_R
 * receives the R-th smallest d~ (infinity with fewer than R candidates) and
 * out_top (Q x R, may be NULL) the surviving rows in (d~, row) order, -1 padded. */
int orc_search_tiled(const void *X, int xdtype, int64_t N, int K, int G,
                     const int64_t *offsets, const int64_t *perm,
                     const void *Y, int ydtype, int64_t Q, int64_t B, int R, int use_f16,
                     int64_t *out_idx, float *out_d32, double *out_d64, int64_t *out_ncand,
                     double *out_dt_R, int64_t *out_top, int nthreads, int cones,
                     const float *Yk, int Kk)
{
    (void)N;
    if (!Yk)
        Kk = K;
    if (K < 1 || K > 256 || Kk < 1 || Kk > 256 || G < 1 || G > Kk || B < 1 || R < 1 || R > 64)
        return -1;
    int64_t NC = orc_num_cones(Kk, G);
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < Q; q++) {
        float y[256], x[256];
        double yh[256];
        load_row(Y, ydtype, q, K, y);
        for (int i = 0; i < K; i++)
            yh[i] = use_f16 ? to_f16(y[i]) : to_bf16(y[i]);
        int64_t *probes = (int64_t *)malloc(sizeof(int64_t) * (size_t)NC);
        if (!probes) {
#pragma omp atomic write
            bad = 1;
            continue;
        }
        int64_t ncand = 0;
        const float *yw = Yk ? Yk + q * Kk : y;  /* the walk runs on the keys of a keyed table (R11) */
        int64_t np = cones ? orc_probe_cones(yw, Kk, G, offsets, B, probes, NC, &ncand)
                           : orc_probe(yw, Kk, G, offsets, B, probes, NC, &ncand);
        struct cand top[64];
        int kept = 0;
        for (int64_t k = 0; k < np; k++) {
            int64_t c = probes[k];
            for (int64_t pos = offsets[c]; pos < offsets[c + 1]; pos++) {
                int64_t row = perm[pos];
                load_row(X, xdtype, row, K, x);
                double n2 = 0.0, dot = 0.0;
                for (int i = 0; i < K; i++) {
                    double xh = use_f16 ? to_f16(x[i]) : to_bf16(x[i]);
                    n2 += xh * xh;
                    dot += yh[i] * xh;
                }
                struct cand cd = { n2 - 2.0 * dot, row };
                /* keep the R smallest (d~, row), sorted (insertion) */
                if (kept < R || cand_less(&cd, &top[kept - 1])) {
                    int at = kept < R ? kept++ : R - 1;
                    while (at > 0 && cand_less(&cd, &top[at - 1])) {
                        top[at] = top[at - 1];
                        at--;
                    }
                    top[at] = cd;
                }
            }
        }
        float best_d = INFINITY;
        int64_t best_row = INT64_MAX;
        double best_d64 = INFINITY;
        for (int t = 0; t < kept; t++) {
            float d32;
            double d64;
            load_row(X, xdtype, top[t].row, K, x);
            dist2(x, y, K, &d32, &d64);
            int64_t before = best_row;
            argmin_update(d32, top[t].row, &best_d, &best_row);
            if (best_row != before)
                best_d64 = d64;
        }
        out_idx[q] = best_row == INT64_MAX ? -1 : best_row;  /* -1: no candidate (R13) */
        out_d32[q] = best_d;
        out_d64[q] = best_d64;
        out_ncand[q] = ncand;
        if (out_dt_R)
            out_dt_R[q] = kept == R ? top[R - 1].dt : INFINITY;
        if (out_top)
            for (int t = 0; t < R; t++)
                out_top[q * R + t] = t < kept ? top[t].row : -1;
        free(probes);
    }
    return bad ? -2 : 0;
}

/* d~ of given (query, row) pairs, as in orc_search_tiled. */
int orc_pair_dtilde(const void *X, int xdtype, int K, const void *Y, int ydtype,
                    const int64_t *rows, int64_t Q, int use_f16, double *out)
{
    for (int64_t q = 0; q < Q; q++) {
        float y[256], x[256];
        load_row(Y, ydtype, q, K, y);
        load_row(X, xdtype, rows[q], K, x);
        double n2 = 0.0, dot = 0.0;
        for (int i = 0; i < K; i++) {
            double xh = use_f16 ? to_f16(x[i]) : to_bf16(x[i]);
            double yh = use_f16 ? to_f16(y[i]) : to_bf16(y[i]);
            n2 += xh * xh;
            dot += yh * xh;
        }
        out[q] = n2 - 2.0 * dot;
    }
    return 0;
}

/* Rounded value of each element (for pinning the rounding). */
int orc_round_short(const float *x, int64_t n, int use_f16, double *out)
{
    for (int64_t i = 0; i < n; i++)
        out[i] = use_f16 ? to_f16(x[i]) : to_bf16(x[i]);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Several bases (Section 3.A, Algorithm 1)                                   */
/* ------------------------------------------------------------------------ */

/* Coordinates of rows in another basis (reading R9): out[n][i] =
 * sum_j M[i][j] x[n][j] with M a K x K row-major matrix, evaluated in FP32
 * in ascending j with each product and sum rounded separately. */
int orc_rotate(const void *X, int dtype, int64_t N, int K, const float *M, float *out)
{
    if (K < 1 || K > 256)
        return -1;
    for (int64_t n = 0; n < N; n++) {
        float x[256];
        load_row(X, dtype, n, K, x);
        for (int i = 0; i < K; i++) {
            float acc = 0.0f;
            for (int j = 0; j < K; j++) {
                float pr = M[(int64_t)i * K + j] * x[j];
                acc = acc + pr;
            }
            out[n * K + i] = acc;
        }
    }
    return 0;
}

/* Coordinates in a structured basis (reading R14): for each row, v = s * x
 * (sign flips, exact), then for strides h = 1, 2, ..., K/2 every pair (j,
 * j + h) with j & h == 0 becomes (v_j + v_{j+h}, v_j - v_{j+h}) in FP32: the
 * fast Walsh-Hadamard transform, out = H diag(s) x without the 1/sqrt(K). */
int orc_wht(const void *X, int dtype, int64_t N, int K, const float *signs, float *out)
{
    if (K < 1 || K > 256 || (K & (K - 1)))
        return -1;
    for (int64_t n = 0; n < N; n++) {
        float v[256];
        load_row(X, dtype, n, K, v);
        for (int j = 0; j < K; j++)
            v[j] = signs[j] * v[j];
        for (int h = 1; h < K; h <<= 1)
            for (int j = 0; j < K; j++)
                if (!(j & h)) {
                    float a = v[j], b = v[j + h];
                    v[j] = a + b;
                    v[j + h] = a - b;
                }
        memcpy(out + n * K, v, sizeof(float) * (size_t)K);
    }
    return 0;
}

/* The search with R bases (Section 3.A).  Basis r has its own table
 * (offsets_r, perm_r built from the rows' coordinates in that basis by
 * orc_hash/orc_bucket); rot holds the R matrices (wht set: R sign vectors of
 * length K, the bases of reading R14).  A query's candidates are the rows of
 * the cones it reaches when it visits, level by level, the l-th cone of every
 * basis's Section 3.B order (empty cones included), each row analyzed once;
 * reading R10 says where that visit stops: when the rows of the visited
 * cones, a row in several of them counted each time, reach B (with cones set,
 * reading R13: after level B-1 of every basis).  Distances are taken on the
 * original vectors; ncand is the number of distinct candidates. */
int orc_search_rot(const void *X, int xdtype, int64_t N, int K, int G, int R, const float *rot,
                   const int64_t *offsets, const int64_t *perms,
                   const void *Y, int ydtype, int64_t Q, int64_t B,
                   int64_t *out_idx, float *out_d32, double *out_d64, int64_t *out_ncand,
                   int nthreads, int cones, int wht)
{
    /* Section 3.A with R bases, in the reading R10, stated as a set:
     *   slot k of a query's schedule is (level l, basis r) = (k / R, k % R),
     *   its cone the l-th of basis r's Section 3.B walk of the query's
     *   coordinates in that basis;
     *   the search takes the shortest prefix of the schedule whose cones hold
     *   at least B rows, a row in several of them counted each time (all
     *   slots if they never do), or with `cones` the first C = B levels;
     *   the candidates are the distinct rows of the prefix's cones, the result
     *   their arg-min on (FP32 distance, row), ncand their number. */
    if (K < 1 || K > 256 || G < 1 || G > K || B < 1 || R < 1 || (wht && (K & (K - 1))))
        return -1;
    int64_t NC = orc_num_cones(K, G);
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 2)
    for (int64_t q = 0; q < Q; q++) {
        float y[256], yr[256], x[256];
        load_row(Y, ydtype, q, K, y);
        int64_t *walks = (int64_t *)malloc(sizeof(int64_t) * (size_t)(NC * R));
        unsigned char *member = (unsigned char *)calloc((size_t)N, 1);
        if (!walks || !member) {
            free(walks);
            free(member);
#pragma omp atomic write
            bad = 1;
            continue;
        }
        for (int r = 0; r < R; r++) {
            if (wht)
                orc_wht(y, ORC_F32, 1, K, rot + (int64_t)r * K, yr);
            else
                orc_rotate(y, ORC_F32, 1, K, rot + (int64_t)r * K * K, yr);
            orc_walk(yr, K, G, walks + (int64_t)r * NC, NC);
        }
        /* the length of the prefix */
        const int64_t nslots = NC * R;
        int64_t take = nslots;
        if (cones) {
            take = (B < NC ? B : NC) * R;
        } else {
            int64_t rows = 0;
            for (int64_t k = 0; k < nslots; k++) {
                const int64_t r = k % R, c = walks[r * NC + k / R];
                const int64_t *off = offsets + r * (NC + 1);
                rows += off[c + 1] - off[c];
                if (rows >= B) {
                    take = k + 1;
                    break;
                }
            }
        }
        /* the candidate set */
        for (int64_t k = 0; k < take; k++) {
            const int64_t r = k % R, c = walks[r * NC + k / R];
            const int64_t *off = offsets + r * (NC + 1);
            const int64_t *perm = perms + r * N;
            for (int64_t pos = off[c]; pos < off[c + 1]; pos++)
                member[perm[pos]] = 1;
        }
        /* the arg-min over it */
        float best_d = INFINITY;
        int64_t best_row = INT64_MAX;
        double best_d64 = INFINITY;
        int64_t ncand = 0;
        for (int64_t row = 0; row < N; row++) {
            if (!member[row])
                continue;
            float d32;
            double d64;
            load_row(X, xdtype, row, K, x);
            dist2(x, y, K, &d32, &d64);
            int64_t before = best_row;
            argmin_update(d32, row, &best_d, &best_row);
            if (best_row != before)
                best_d64 = d64;
            ncand++;
        }
        out_idx[q] = best_row == INT64_MAX ? -1 : best_row;  /* -1: no candidate (R13) */
        out_d32[q] = best_d;
        out_d64[q] = best_d64;
        out_ncand[q] = ncand;
        free(walks);
        free(member);
    }
    return bad ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* PCA front-end (Section 4.B)                                                */
/* ------------------------------------------------------------------------ */

/* Keys in a reduced basis (reading R11): out[n][i] = sum_j P[i][j] (x[n][j] -
 * mu[j]) for i < k, with P a k x K row-major matrix and mu of length K (NULL:
 * no centring), in FP32 with ascending j and the difference, each product
 * and each sum rounded separately. */
int orc_project(const void *X, int dtype, int64_t N, int K, const float *mu, const float *P, int k, float *out)
{
    if (K < 1 || K > 256 || k < 1 || k > 256)
        return -1;
    for (int64_t n = 0; n < N; n++) {
        float x[256];
        load_row(X, dtype, n, K, x);
        for (int i = 0; i < k; i++) {
            float acc = 0.0f;
            for (int j = 0; j < K; j++) {
                float c = mu ? x[j] - mu[j] : x[j];
                float pr = P[(int64_t)i * K + j] * c;
                acc = acc + pr;
            }
            out[n * k + i] = acc;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Coarse clusters (ROSANNA+, Section 4.B)                                    */
/* ------------------------------------------------------------------------ */

/* Nearest centroid of each row (reading R12): FP32 term-by-term squared
 * distance, lower centroid on ties.  cent is C x K row-major FP32. */
int orc_assign(const void *X, int dtype, int64_t N, int K, const float *cent, int C, int32_t *out)
{
    if (K < 1 || K > 256 || C < 1)
        return -1;
    for (int64_t n = 0; n < N; n++) {
        float x[256];
        load_row(X, dtype, n, K, x);
        float best = INFINITY;
        int bc = 0;
        for (int c = 0; c < C; c++) {
            float d32;
            double d64;
            dist2(x, cent + (int64_t)c * K, K, &d32, &d64);
            if (d32 < best) {
                best = d32;
                bc = c;
            }
        }
        out[n] = bc;
    }
    return 0;
}

/* Lloyd update (reading R12): centroid c = float64 sum of its rows in
 * ascending row order, divided by their count, rounded to FP32; unchanged
 * when the cluster is empty. */
int orc_kmeans_update(const void *X, int dtype, int64_t N, int K, const int32_t *assign, int C,
                      const float *old_cent, float *new_cent)
{
    if (K < 1 || K > 256 || C < 1)
        return -1;
    double *sum = (double *)calloc((size_t)C * K, sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)C, sizeof(int64_t));
    if (!sum || !cnt) {
        free(sum);
        free(cnt);
        return -2;
    }
    for (int64_t n = 0; n < N; n++) {
        float x[256];
        load_row(X, dtype, n, K, x);
        int c = assign[n];
        for (int j = 0; j < K; j++)
            sum[(int64_t)c * K + j] += (double)x[j];
        cnt[c]++;
    }
    for (int c = 0; c < C; c++)
        for (int j = 0; j < K; j++)
            new_cent[(int64_t)c * K + j] = cnt[c] ? (float)(sum[(int64_t)c * K + j] / (double)cnt[c])
                                                  : old_cent[(int64_t)c * K + j];
    free(sum);
    free(cnt);
    return 0;
}

/* Search in clusters (reading R12).  offsets has C * N_C + 1 entries: bucket
 * (c, cone) is c * N_C + cone; perm maps sorted positions to rows. */
int orc_search_ivf(const void *X, int xdtype, int64_t N, int K, int G, const float *cent, int C,
                   const int64_t *offsets, const int64_t *perm, const void *Y, int ydtype, int64_t Q,
                   int64_t B, int nprobe, int64_t *out_idx, float *out_d32, double *out_d64,
                   int64_t *out_ncand, int nthreads, int cones)
{
    (void)N;
    if (K < 1 || K > 256 || G < 1 || G > K || B < 1 || nprobe < 1 || nprobe > C)
        return -1;
    int64_t NC = orc_num_cones(K, G);
    int64_t Bc = (B + nprobe - 1) / nprobe;
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < Q; q++) {
        float y[256], r[256], x[256];
        load_row(Y, ydtype, q, K, y);
        int64_t *probes = (int64_t *)malloc(sizeof(int64_t) * (size_t)NC);
        float *cd = (float *)malloc(sizeof(float) * (size_t)C);
        char *taken = (char *)calloc((size_t)C, 1);
        if (!probes || !cd || !taken) {
#pragma omp atomic write
            bad = 1;
            free(probes);
            free(cd);
            free(taken);
            continue;
        }
        for (int c = 0; c < C; c++) {
            double d64;
            dist2(y, cent + (int64_t)c * K, K, &cd[c], &d64);
        }
        float best_d = INFINITY;
        int64_t best_row = INT64_MAX;
        double best_d64 = INFINITY;
        int64_t ncand = 0;
        for (int t = 0; t < nprobe; t++) {
            int bc = -1;
            for (int c = 0; c < C; c++)
                if (!taken[c] && (bc < 0 || cd[c] < cd[bc]))
                    bc = c;
            taken[bc] = 1;
            for (int j = 0; j < K; j++)
                r[j] = y[j] - cent[(int64_t)bc * K + j];
            const int64_t *off = offsets + (int64_t)bc * NC;
            int64_t nc_c = 0;
            int64_t np = cones ? orc_probe_cones(r, K, G, off, B, probes, NC, &nc_c)
                               : orc_probe(r, K, G, off, Bc, probes, NC, &nc_c);
            ncand += nc_c;
            for (int64_t k = 0; k < np; k++) {
                int64_t cone = probes[k];
                for (int64_t pos = off[cone]; pos < off[cone + 1]; pos++) {
                    int64_t row = perm[pos];
                    float d32;
                    double d64;
                    load_row(X, xdtype, row, K, x);
                    dist2(x, y, K, &d32, &d64);
                    int64_t before = best_row;
                    argmin_update(d32, row, &best_d, &best_row);
                    if (best_row != before)
                        best_d64 = d64;
                }
            }
        }
        out_idx[q] = best_row == INT64_MAX ? -1 : best_row;  /* -1: every cluster searched was empty */
        out_d32[q] = best_d;
        out_d64[q] = best_d64;
        out_ncand[q] = ncand;
        free(probes);
        free(cd);
        free(taken);
    }
    return bad ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* Sparse table (Section 4, second-level hash; reading R15)                  */
/* ------------------------------------------------------------------------ */

struct cone_row {
    int64_t cone, row;
};

static int cone_row_cmp(const void *a, const void *b)
{
    const struct cone_row *x = (const struct cone_row *)a, *y = (const struct cone_row *)b;
    if (x->cone != y->cone)
        return x->cone < y->cone ? -1 : 1;
    return x->row < y->row ? -1 : (x->row > y->row);
}

/* Rows sorted by (cone, row) into perm; keys[u] is the u-th distinct cone in
 * ascending order and its rows are perm[offsets[u] .. offsets[u+1]).
 * keys, offsets and perm hold N, N + 1 and N entries.  Returns the number
 * of distinct cones, or -1 when out of memory. */
int64_t orc_bucket_sparse(const int64_t *cone, int64_t N, int64_t *keys, int64_t *offsets, int64_t *perm)
{
    struct cone_row *cr = (struct cone_row *)malloc(sizeof(struct cone_row) * (size_t)(N > 0 ? N : 1));
    if (!cr)
        return -1;
    for (int64_t n = 0; n < N; n++) {
        cr[n].cone = cone[n];
        cr[n].row = n;
    }
    qsort(cr, (size_t)N, sizeof(struct cone_row), cone_row_cmp);
    int64_t u = 0;
    for (int64_t i = 0; i < N; i++) {
        if (i == 0 || cr[i].cone != cr[i - 1].cone) {
            keys[u] = cr[i].cone;
            offsets[u] = i;
            u++;
        }
        perm[i] = cr[i].row;
    }
    offsets[u] = N;
    free(cr);
    return u;
}

/* Position of cone in keys[0..n) (ascending), or -1 if absent (empty cone). */
static int64_t sparse_find(const int64_t *keys, int64_t n, int64_t cone)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] < cone)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < n && keys[lo] == cone ? lo : -1;
}

#define ORC_SPARSE_WALK_CAP ((int64_t)1 << 22)

struct sparse_ctx {
    const int64_t *keys, *offsets;
    int64_t n_keys;
    int cones;
    int64_t B, limit, seen, cum;
    int64_t *probes;
    int64_t cap, n;
};

/* One walk position: the row budget of reading R5 or the first B cones of
 * reading R13, with the cone's rows looked up in the sparse table. */
static int take_sparse(int64_t cone, void *vctx)
{
    struct sparse_ctx *c = (struct sparse_ctx *)vctx;
    if (c->seen >= c->limit)
        return 1;
    c->seen++;
    int64_t u = sparse_find(c->keys, c->n_keys, cone);
    int64_t size = u < 0 ? 0 : c->offsets[u + 1] - c->offsets[u];
    if (size > 0) {
        if (c->n < c->cap)
            c->probes[c->n] = u;
        c->n++;
        c->cum += size;
    }
    if (c->cones)
        return c->seen >= c->limit;
    return (size > 0 && c->cum >= c->B) || c->seen >= c->limit;
}

/* The walk's first n positions (cones, empty or not); returns how many were
 * written (fewer only when N_C < n). */
struct prefix_ctx {
    int64_t *out;
    int64_t cap, n;
};

static int take_prefix(int64_t cone, void *vctx)
{
    struct prefix_ctx *c = (struct prefix_ctx *)vctx;
    c->out[c->n++] = cone;
    return c->n >= c->cap;
}

int64_t orc_walk_prefix(const float *y, int K, int G, int64_t *cones, int64_t n)
{
    if (n < 1)
        return 0;
    struct prefix_ctx c = { cones, n, 0 };
    walk_cones(y, K, G, take_prefix, &c);
    return c.n;
}

/* Probe list of one query on a sparse table: bucket numbers u (positions in
 * keys) of the non-empty cones taken, in walk order; *ncand their rows. */
int64_t orc_probe_sparse(const float *y, int K, int G, const int64_t *keys, int64_t n_keys,
                         const int64_t *offsets, int64_t N, int64_t B, int cones, int64_t *probes, int64_t cap,
                         int64_t *ncand)
{
    int64_t NC = orc_num_cones(K, G);
    if ((!cones && B >= N) || (cones && B >= NC)) {  /* every row */
        for (int64_t u = 0; u < n_keys && u < cap; u++)
            probes[u] = u;
        *ncand = offsets[n_keys];
        return n_keys;
    }
    int64_t limit = NC < ORC_SPARSE_WALK_CAP ? NC : ORC_SPARSE_WALK_CAP;
    if (cones && B < limit)
        limit = B;
    struct sparse_ctx c = { keys, offsets, n_keys, cones, B, limit, 0, 0, probes, cap, 0 };
    walk_cones(y, K, G, take_sparse, &c);
    *ncand = c.cum;
    return c.n;
}

/* Algorithm 1 with one basis on a sparse table (reading R15); outputs as in
 * orc_search_keyed (row -1 and +inf when there is no candidate). */
int orc_search_sparse(const void *X, int xdtype, int64_t N, int K, int G, const int64_t *keys, int64_t n_keys,
                      const int64_t *offsets, const int64_t *perm, const void *Y, int ydtype, int64_t Q, int64_t B,
                      int cones, int64_t *out_idx, float *out_d32, double *out_d64, int64_t *out_ncand, int nthreads)
{
    if (K < 1 || K > 256 || G < 1 || G > K || B < 1 || n_keys < 1)
        return -1;
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < Q; q++) {
        float y[256], x[256];
        load_row(Y, ydtype, q, K, y);
        int64_t *probes = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_keys);
        if (!probes) {
#pragma omp atomic write
            bad = 1;
            continue;
        }
        int64_t ncand = 0;
        int64_t np = orc_probe_sparse(y, K, G, keys, n_keys, offsets, N, B, cones, probes, n_keys, &ncand);
        float best_d = INFINITY;
        int64_t best_row = INT64_MAX;
        double best_d64 = INFINITY;
        for (int64_t k = 0; k < np; k++) {
            int64_t u = probes[k];
            for (int64_t pos = offsets[u]; pos < offsets[u + 1]; pos++) {
                int64_t row = perm[pos];
                float d32;
                double d64;
                load_row(X, xdtype, row, K, x);
                dist2(x, y, K, &d32, &d64);
                int64_t before = best_row;
                argmin_update(d32, row, &best_d, &best_row);
                if (best_row != before)
                    best_d64 = d64;
            }
        }
        out_idx[q] = best_row == INT64_MAX ? -1 : best_row;
        out_d32[q] = best_d;
        out_d64[q] = best_d64;
        out_ncand[q] = ncand;
        free(probes);
    }
    return bad ? -2 : 0;
}

