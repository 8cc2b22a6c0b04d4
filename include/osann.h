/*
 * osann.h -- C ABI of the MI355X (gfx950) order-statistics approximate
 * nearest-neighbour search library (libosann.so).
 *
 * The method is that of Verdoliva, Cozzolino and Poggi, "A reliable
 * order-statistics-based approximate nearest neighbor search algorithm"
 * (arXiv 1509.03453, ROSANNA), with one basis (the original coordinates):
 *
 *   problem     (Section 2, eq. (1)) given N database vectors x_n in R^D
 *               and a query y, find argmin_n ||x_n - y||^2;
 *   hashing     (Section 2, eq. (2), Fig. 2) every vector is classified by
 *               the indices of its L largest-magnitude components (its
 *               profile) and the signs of those components (its cone);
 *               there are N_C = C(D,L) * 2^L cones;
 *   index       (Section 4) the database is bucketed by cone;
 *   search      (Algorithm 1, Section 3.B) the query's own cone is scanned
 *               first, then neighbouring cones in order of the paper's
 *               profile distance, with exact Euclidean distances and a
 *               running arg-min.
 *
 * The paper's K (vector length) is D here and its G (number of components
 * hashed) is L.
 *
 * Conventions shared by every call:
 *   - Array pointers are HIP device pointers on the current device unless a
 *     comment says otherwise (e.g. torch.Tensor.data_ptr() of a CUDA tensor).
 *   - `stream` arguments are hipStream_t passed as void*; NULL is the null
 *     stream.
 *   - Calls returning int give OS_ANN_OK (0) or a negative code below;
 *     calls returning a pointer give NULL on error.  In both cases
 *     os_ann_last_error() / os_ann_last_error_message() describe the last
 *     failure of the calling thread.
 *   - Keys follow these rules: equal magnitudes rank the lower component
 *     index first; a component's sign bit is 1 unless its value is < 0
 *     (zero and -0.0 are non-negative, Fig. 2 caption); the cone id is
 *     colex_rank(profile indices ascending) * 2^L + sign bits, lowest index
 *     most significant (Fig. 2, right table).
 *   - Distances are squared Euclidean in FP32, evaluated term by term in
 *     ascending component order with each subtraction, product and sum
 *     rounded separately; ties in distance go to the lower original row.
 */
#ifndef OSANN_H
#define OSANN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define OS_ANN_OK          0
#define OS_ANN_EINVAL     -1  /* null pointer; N < 1 or N >= 2^31; D < 1 or D > 256;
                                 L < 1 or L > min(D, 7); max_candidates < 1; Q < 0;
                                 bad dtype or mode; workspace too small */
#define OS_ANN_ENOMEM     -2  /* device allocation failed */
#define OS_ANN_EDEVICE    -3  /* a HIP runtime call or kernel launch failed */
#define OS_ANN_ENOTSUP    -4  /* N_C = C(D,L) * 2^L above 2^24 for a table kind without a
                                 sparse form; tiled mode with more non-empty cones than
                                 its LDS cone list holds, or on a sparse table */
#define OS_ANN_ENONFINITE -5  /* NaN or infinity in the database (build only) */

/* Storage types of database rows and queries. */
#define OS_ANN_F32 0
#define OS_ANN_F16 1
#define OS_ANN_U8  2

/* Search modes.
 *   FP32   every candidate's exact FP32 distance; arg-min on (distance, row).
 *   TILED  the same candidates are screened on the matrix cores with
 *          d~ = ||x^||^2 - 2 q^.x^ (x^, q^ rounded to BF16, or kept as FP16
 *          for FP16 data; FP32 accumulation), the rerank_r smallest (d~, row)
 *          survive, and their exact FP32 distances (as in FP32 mode) decide
 *          the result.  out_dist is always the exact FP32 distance of out_idx. */
#define OS_ANN_MODE_FP32   0
#define OS_ANN_MODE_TILED  1

/* Search flags. */
#define OS_ANN_FLAG_TIME_KERNELS 1  /* record HIP events around each kernel launch */
#define OS_ANN_FLAG_GRAPH        2  /* run the search as a hipGraph of its shape class
                                       (stream, Q rounded up to one of 8 steps per
                                       octave, query type, mode, R, cone budget, budget),
                                       captured on the class's first call and replayed on
                                       later calls with any buffers: the queries are
                                       copied into buffers the index keeps per stream,
                                       the results out of them; `workspace` is not used.
                                       Needs a non-null stream that is not being
                                       captured (else OS_ANN_EINVAL) */
#define OS_ANN_FLAG_BUDGET_CONES 4  /* fixed-C mode (Section 3, Table III): max_candidates
                                       is the number C of cones each walk takes, empty
                                       ones included, not a number of rows; with several
                                       bases the search takes levels 0..C-1 of every
                                       basis, on a clustered table the first C cones of
                                       each searched cluster.  out_ncand is then the rows
                                       the search compared (distinct rows with several
                                       bases; 0 and out_idx = -1, out_dist = +inf when
                                       every cone taken is empty) */

/* Kernel ids of os_ann_kernel_time. */
#define OS_ANN_KERNEL_PROBE  0  /* query classification + walk state */
#define OS_ANN_KERNEL_SCAN   1  /* FP32 candidate scan + arg-min */
#define OS_ANN_KERNEL_SCREEN 2  /* tiled mode: matrix-core screening, per-query top-R */
#define OS_ANN_KERNEL_FINISH 3  /* tiled mode: merge of top-R lists + FP32 re-rank */
#define OS_ANN_KERNEL_GRAPH  4  /* a replayed hipGraph, as one unit */
#define OS_ANN_KERNEL_COUNT  5

typedef struct os_ann_index os_ann_index;

typedef struct os_ann_build_opts {
    int32_t dtype;      /* OS_ANN_F32 / OS_ANN_F16 / OS_ANN_U8 storage of db rows */
    int32_t want_lowp;  /* nonzero: also keep the BF16/FP16 copy used by
                           OS_ANN_MODE_TILED (built on first tiled search otherwise) */
    void *stream;       /* stream the build runs on (NULL = null stream) */
} os_ann_build_opts;

typedef struct os_ann_search_opts {
    int32_t mode;         /* OS_ANN_MODE_FP32 or OS_ANN_MODE_TILED */
    int32_t rerank_r;     /* tiled mode: survivors re-ranked in FP32: 4, 8 or 16 (0 = 8) */
    int32_t query_dtype;  /* OS_ANN_F32 / OS_ANN_F16 / OS_ANN_U8 */
    int32_t flags;        /* OS_ANN_FLAG_* bits */
    void *stream;         /* stream the search runs on (NULL = null stream) */
    void *workspace;      /* optional caller-owned device scratch, >= os_ann_workspace_bytes;
                             NULL: the index's own scratch (not for concurrent calls) */
    int64_t workspace_bytes;
    int64_t *walks_capped;  /* optional device int64: sparse tables only, set to the number of
                               walks the 2^22-position cap stopped (a row budget not met
                               although cones remained, or a C beyond the cap); ignored
                               (left untouched) for other tables */
} os_ann_search_opts;

/*
 * Build an index over N FP32 rows of D components (row-major db[N][D]).
 * Hashes every row (Section 2, eq. (2)), buckets the rows by cone with a
 * stable sort (rows of one cone keep ascending original order; Section 4)
 * and keeps a bucket-contiguous, permuted copy of the rows.
 * Synchronous: returns when the index is ready.  The library copies the
 * rows, so the caller may free db as soon as the call returns.  The index
 * owns all its device memory until os_ann_free.
 * Errors: EINVAL, ENOMEM, EDEVICE, ENOTSUP, ENONFINITE (returns NULL).
 */
os_ann_index *os_ann_build(const float *db, int64_t N, int32_t D, int32_t L);

/* As os_ann_build with rows stored as opts->dtype (FP32, FP16 or uint8) and
 * the build enqueued on opts->stream (still synchronous).  opts may be NULL
 * (FP32, null stream).
 *
 * Sparse table (Section 4: a second-level hash table manages the table when
 * the cones are very many): when N_C = C(D,L) 2^L exceeds 2^24 (os_ann_build
 * too), only the non-empty cones are kept: the rows' 64-bit cone ids sorted
 * (rows of a cone in ascending order), the distinct ids with their row
 * offsets, and a hash table from id to bucket.  Searches walk the same
 * Section 3.B order (a cone missing from the table is empty) with the same
 * row budget or fixed-C rule, except that a walk takes at most 2^22
 * positions (a row budget not met by then stops there); a budget of at
 * least N, or C >= N_C, takes every row.  FP32 mode only (tiled, and
 * opts->want_lowp: ENOTSUP); os_ann_classify: ENOTSUP; os_ann_export gives
 * row tops and perm only, the rest comes from os_ann_export_sparse. */
os_ann_index *os_ann_build_ex(const void *db, int64_t N, int32_t D, int32_t L,
                              const os_ann_build_opts *opts);

/*
 * Build an index with several bases (Section 3.A; Algorithm 1 with R
 * rotations).  rot holds n_rot (1..16) D x D FP32 matrices, row-major, device
 * memory: the coordinates of a vector y in basis r are rot[r] y, evaluated in
 * FP32 term by term (ascending j, each product and sum rounded).  Every basis
 * gets its own table (hashing and bucketing of the rows' coordinates in that
 * basis) holding the original rows; distances are always taken on the
 * original rows.  Passing the identity as rot[0] keeps the original basis.
 * The matrices need not be orthonormal (the result is then still the arg-min
 * over the visited rows, but the cones no longer describe rotated space).
 * Searches on such an index run in OS_ANN_MODE_FP32 only (tiled: ENOTSUP);
 * opts->want_lowp must be 0.  Synchronous; the library copies db and rot.
 * Errors: EINVAL, ENOMEM, EDEVICE, ENOTSUP, ENONFINITE (returns NULL).
 */
os_ann_index *os_ann_build_rot(const void *db, int64_t N, int32_t D, int32_t L, const float *rot,
                               int32_t n_rot, const os_ann_build_opts *opts);

/*
 * Several structured bases (Section 3.D: Walsh-Hadamard matrices in place of
 * pseudo-random ones, which cuts the rotation cost from D^2 to D log2 D per
 * vector).  Basis r is H diag(signs[r]) / sqrt(D), H the Sylvester-ordered
 * D x D Hadamard matrix (entry (i, j) = (-1)^popcount(i & j)); signs holds
 * n_rot (1..16) vectors of D entries, each exactly +1 or -1, FP32, device
 * memory.  D must be a power of two.  Coordinates come from the fast
 * transform: the sign flips, then butterflies with strides 1, 2, ..., D/2,
 * each pair (a, b) becoming (a + b, a - b) rounded in FP32, without the
 * 1/sqrt(D) factor (a positive scale changes neither the order of the
 * magnitudes nor the signs, so the cones are those of the orthonormal
 * basis).  Everything else is as in os_ann_build_rot: one table per basis
 * over the original rows, distances on the original rows, FP32 mode only.
 * Errors: EINVAL (also D not a power of two, a sign other than +-1), ENOMEM,
 * EDEVICE, ENOTSUP, ENONFINITE (returns NULL).
 */
os_ann_index *os_ann_build_wht(const void *db, int64_t N, int32_t D, int32_t L, const float *signs,
                               int32_t n_rot, const os_ann_build_opts *opts);

/*
 * Approximate NN of Q FP32 queries (row-major queries[Q][D]), Algorithm 1
 * with one basis: each query's cones are visited in the Section 3.B order
 * (own cone first; then the other profiles that share the query's signs, in
 * lexicographic order of the query's rank positions, which is non-decreasing
 * in the paper's profile distance; then the same profiles with 1..L signs
 * flipped), skipping empty cones, until the cones visited hold at least
 * max_candidates rows (whole cones only; every cone when max_candidates >= N).
 * Every candidate's distance is computed and the arg-min kept.
 * out_idx[q] in [0, N) is the original row of the nearest candidate and
 * out_dist[q] its squared distance (FP32).
 * Asynchronous on the null stream: outputs are valid after the stream
 * synchronises; the caller owns queries and outputs and keeps them alive
 * until then.  Q = 0 is a no-op.  Uses the index's own scratch, so two
 * calls on one index must not overlap (use os_ann_search_ex with distinct
 * workspaces for concurrent searches).
 * Errors: EINVAL, ENOMEM, EDEVICE.
 */
int os_ann_search(const os_ann_index *idx, const float *queries, int64_t Q,
                  int64_t max_candidates, int64_t *out_idx, float *out_dist);

/* As os_ann_search with options (mode, query dtype, stream, workspace,
 * flags) and the per-query candidate count out_ncand[Q] (int64, may be
 * NULL).  opts may be NULL (FP32 mode, FP32 queries, null stream).  The
 * first tiled search of a new shape (Q, budget, index) times the candidate
 * work splits and keeps the fastest (in memory, and appended to the file
 * named by the OSANN_TUNE_FILE environment variable if set); this first call
 * synchronises the stream.  Results never depend on the split or on the
 * batch a query arrives in. */
int os_ann_search_ex(const os_ann_index *idx, const void *queries, int64_t Q,
                     int64_t max_candidates, const os_ann_search_opts *opts,
                     int64_t *out_idx, float *out_dist, int64_t *out_ncand);

/*
 * For callers that can not allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP32
 * search of os_ann_search_ex, allocating nothing.  Its scratch (the queries'
 * FP32 copies and walk state, O(D) bytes per query) is a fixed 64 MiB device
 * array inside the library, one copy per GPU, held until the process ends;
 * the call makes no hipMalloc, hipFree or other allocating call.  The caller
 * still passes the queries and the outputs (device memory, as for
 * os_ann_search_ex; out_ncand may be NULL).
 * opts may be NULL; its mode must be OS_ANN_MODE_FP32 (tiled: ENOTSUP), its
 * workspace NULL and its flags at most OS_ANN_FLAG_BUDGET_CONES (EINVAL
 * otherwise).  Any index kind searchable in FP32 mode works.  A batch whose
 * scratch exceeds 64 MiB (about 160,000 queries at D = 64, 43,000 at
 * D = 256; os_ann_workspace_bytes in FP32 mode gives the need) is rejected
 * with EINVAL: split it.  Asynchronous on opts->stream.  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads, or one issued before the previous one's stream has
 * finished reading it) race and give wrong results; serialise them.  No
 * part of the array needs to start at zero.
 * Errors: EINVAL, ENOTSUP, EDEVICE.
 */
int os_ann_search_static(const os_ann_index *idx, const void *queries, int64_t Q,
                         int64_t max_candidates, const os_ann_search_opts *opts,
                         int64_t *out_idx, float *out_dist, int64_t *out_ncand);

/*
 * Principal axes of the database, for the PCA front-end of Section 4.B
 * (classify on the first principal components, compare on all of them).
 * The float64 mean and covariance (sum of the centred outer products divided
 * by N) are computed on the device in fixed order; the covariance is
 * diagonalised on the host (cyclic Jacobi, float64).  Outputs, host memory:
 * mean_out[D] (FP32 mean), basis_out[k][D] (the k axes of largest variance in
 * decreasing order, FP32, one per row, each signed so that its
 * largest-magnitude component, lowest index on ties, is positive), var_out[k]
 * (their variances, float64; may be NULL).  db is device memory of
 * opts->dtype.  Synchronous.  Errors: EINVAL (null pointers, k outside
 * [1, D]), ENOMEM, EDEVICE, ENONFINITE.
 */
int os_ann_pca(const void *db, int64_t N, int32_t D, int32_t k, const os_ann_build_opts *opts,
               float *mean_out, float *basis_out, double *var_out);

/*
 * Build an index whose cones come from keys (the PCA front-end of Section
 * 4.B): the key of a vector x is P (x - mean), the k components
 * sum_j P[i][j] (x[j] - mean[j]) evaluated in FP32 term by term (ascending
 * j; the difference, each product and each sum rounded).  basis (k x D,
 * row-major) and mean (D, or NULL for no centring) are FP32 device memory,
 * copied by the library; typically the output of os_ann_pca.  The table
 * hashes the rows' keys (L <= min(k, 7)) and holds the original rows; a
 * search projects each query the same way, walks the cones of its key and
 * compares candidates on all D components (exact FP32 distances, as for any
 * index).  Both search modes apply: OS_ANN_MODE_TILED walks the keys and
 * screens the full queries against the full rows (the low-precision copy is
 * built on the first tiled search; opts->want_lowp must be 0 here);
 * os_ann_classify is not available (ENOTSUP).  Synchronous.  Errors: EINVAL,
 * ENOMEM, EDEVICE, ENOTSUP, ENONFINITE (returns NULL).
 */
os_ann_index *os_ann_build_proj(const void *db, int64_t N, int32_t D, int32_t L, const float *mean,
                                const float *basis, int32_t k, const os_ann_build_opts *opts);

/*
 * Lloyd k-means for the coarse clusters of ROSANNA+ (Section 4.B): from the
 * C initial centroids init[C][D] (FP32, device), iters times: every row goes
 * to the centroid at the smallest FP32 squared distance (evaluated term by
 * term, lower centroid on ties), then every centroid becomes the float64 mean
 * of its rows (summed in ascending row order) rounded to FP32, or keeps its
 * value if no row is assigned.  out[C][D] (FP32, device) receives the
 * result; db is device memory of opts->dtype.  Synchronous.
 * Errors: EINVAL (null pointers, C outside [1, 4096], iters < 0), ENOMEM,
 * EDEVICE.
 */
int os_ann_kmeans(const void *db, int64_t N, int32_t D, int32_t C, int32_t iters, const float *init,
                  const os_ann_build_opts *opts, float *out);

/*
 * Build a clustered index (ROSANNA+, Section 4.B): every row goes to its
 * nearest centroid (as in os_ann_kmeans) and is hashed on its residual
 * x - c (FP32); the table's buckets are (cluster, cone), bucket id
 * cluster * C(D,L) 2^L + cone (os_ann_info reports their count as n_cones,
 * os_ann_export their offsets).  centroids[C][D] is FP32 device memory,
 * copied.  A search compares each query with every centroid (FP32 distance,
 * lower centroid on ties), and in each of the nprobe nearest clusters walks
 * the cones of the query's residual with budget ceil(max_candidates /
 * nprobe); the rows met are compared on the full vectors and the best
 * (distance, row) wins; ncand sums the clusters' candidates (-1 as the row
 * if every searched cluster is empty).  FP32 mode only (tiled: ENOTSUP);
 * opts->want_lowp must be 0; os_ann_classify: ENOTSUP.  Requires
 * 1 <= nprobe <= min(C, 64), C <= 1024 and C * C(D,L) 2^L <= 2^24.
 * Synchronous.  Errors: EINVAL, ENOMEM, EDEVICE, ENOTSUP, ENONFINITE
 * (returns NULL).
 */
os_ann_index *os_ann_build_ivf(const void *db, int64_t N, int32_t D, int32_t L, const float *centroids,
                               int32_t C, int32_t nprobe, const os_ann_build_opts *opts);

/* Change the number of clusters a clustered index searches per query (same
 * limits as os_ann_build_ivf).  Not to be called while a search on the index
 * is in flight.  Errors: EINVAL. */
int os_ann_set_nprobe(os_ann_index *idx, int32_t nprobe);

/* Bytes of device scratch a search with these arguments needs (>= 0), or a
 * negative error code.  Used to size caller-owned workspaces and by
 * admission control. */
int64_t os_ann_workspace_bytes(const os_ann_index *idx, int64_t Q, int64_t max_candidates,
                               const os_ann_search_opts *opts);

/*
 * Classify Q queries without scanning (Section 2 hashing, Section 3.B
 * probing): q_cone[Q] (uint32) own cone id, q_top[Q] (uint64) the L largest
 * components in decreasing magnitude packed as 9-bit pairs (bits 0-7
 * component index, bit 8 sign bit; pair j at bit 9*j), q_ncand[Q] (int64)
 * candidates within max_candidates.  Any output may be NULL.  Asynchronous
 * on `stream`; uses the index's scratch.
 */
int os_ann_classify(const os_ann_index *idx, const void *queries, int32_t query_dtype,
                    int64_t Q, int64_t max_candidates, uint32_t *q_cone, uint64_t *q_top,
                    int64_t *q_ncand, void *stream);

/*
 * Copy out the index for inspection: row_cone[N] (uint32) cone of each
 * original row, row_top[N] (uint64) packed top-L pairs as in
 * os_ann_classify, offsets[n_cones+1] (int64; bucket c holds sorted
 * positions offsets[c] .. offsets[c+1]-1, offsets[n_cones] = N), perm[N]
 * (int64; original row at each sorted position).  Any output may be NULL.
 * Asynchronous on `stream`.
 */
int os_ann_export(const os_ann_index *idx, uint32_t *row_cone, uint64_t *row_top,
                  int64_t *offsets, int64_t *perm, void *stream);

/* As os_ann_export for basis r (0 <= r < n_rot) of an index built with
 * os_ann_build_rot; r = 0 for any other index. */
int os_ann_export_basis(const os_ann_index *idx, int32_t r, uint32_t *row_cone, uint64_t *row_top,
                        int64_t *offsets, int64_t *perm, void *stream);

/* Sparse table only (EINVAL otherwise): cone_ids[n_nonempty] (uint64, the
 * distinct non-empty cones in ascending order; n_nonempty from
 * os_ann_info), offsets[n_nonempty+1] (int64; the rows of cone_ids[u] sit
 * at sorted positions offsets[u] .. offsets[u+1]-1) and perm[N] (int64).
 * Any output may be NULL.  Asynchronous on `stream`. */
int os_ann_export_sparse(const os_ann_index *idx, uint64_t *cone_ids, int64_t *offsets, int64_t *perm,
                         void *stream);

/* Copy out the permuted rows, converted exactly to FP32: rows[N][D] with
 * rows[pos] = db[perm[pos]].  Asynchronous on `stream`. */
int os_ann_export_rows(const os_ann_index *idx, float *rows, void *stream);

/*
 * Per-kernel device time of the searches made on this index with
 * OS_ANN_FLAG_TIME_KERNELS: HIP events are recorded on the search's stream
 * immediately before and after each kernel launch.  Waits for the recorded
 * events, then returns (host pointers) the number of launches and their
 * summed duration in milliseconds, and forgets them.  kernel is an
 * OS_ANN_KERNEL_* id.  Errors: EINVAL, EDEVICE.
 */
int os_ann_kernel_time(const os_ann_index *idx, int32_t kernel, int64_t *launches, double *total_ms);

/* Host-side facts about an index (host pointers, any may be NULL):
 * N, D, L, number of cones, number of non-empty cones, device bytes held. */
int os_ann_info(const os_ann_index *idx, int64_t *N, int32_t *D, int32_t *L,
                int64_t *n_cones, int64_t *n_nonempty, int64_t *device_bytes);

/* Graph replay statistics of an index (OS_ANN_FLAG_GRAPH): graphs captured
 * so far, graph replays so far, and graphs currently kept (at most 512 per
 * index; the least recently replayed is dropped first).  Any output may be
 * NULL.  Host-side counters; no device work. */
int os_ann_graph_stats(const os_ann_index *idx, int64_t *captured, int64_t *replayed, int64_t *cached);

/* Tiling of the last tiled-mode search enqueued on the index (Section
 * 3.D's short-list scan as matrix-core tiles, as the autotuner chose it):
 * kernel 0 = query-tile screen, 1 = cone-major screen; order 0 = queries by
 * own cone, 1 = by their walk's first cones; groups = 16-query MFMA groups
 * per tile (per pass for the cone-major screen); splits = lists per query.
 * -1 / 0 before any tiled search.  Any output may be NULL.  Host-side; no
 * device work. */
int os_ann_last_tiling(const os_ann_index *idx, int32_t *kernel, int32_t *order, int32_t *groups,
                       int32_t *splits);

/* Release the index.  The caller makes sure no search on it is in flight.
 * Waits for the device to finish its work (as hipFree does); the index's
 * device blocks then stay with the library, idle, for later builds and
 * searches of the same sizes (at most 8 GiB of idle blocks in all). */
void os_ann_free(os_ann_index *idx);

/* Return every idle device block kept by the library to the HIP runtime
 * (for a caller that needs the memory elsewhere).  Blocks of live indexes
 * are not touched.  Never fails: returns OS_ANN_OK. */
int os_ann_trim(void);

/*
 * Device memory from the caller's allocator, so that a host framework such as
 * PyTorch can supply the device memory; the paper's problem statement
 * (Section 2, eq. (1)) puts no constraint on where the index lives.
 *
 * alloc(bytes, stream, ctx) must return a block of at least `bytes` bytes of
 * device memory on the current device, aligned to 256 bytes, usable by work
 * enqueued on `stream` (the stream of the library call that asks; NULL is the
 * null stream), or NULL when it can not.  free(ptr, stream, ctx) takes back a
 * block with the stream it was asked for; the library calls it only once the
 * device has finished every use of the block.
 *
 * Once set, every device allocation of the library goes through alloc:
 * index memory (os_ann_free returns it), the index's own search scratch and
 * low-precision copy, and the temporaries of builds, PCA and k-means.  A NULL
 * from alloc makes the call fail with OS_ANN_ENOMEM after it has returned
 * every block it obtained; an index built earlier stays usable.  A block not
 * aligned to 256 bytes is handed back at once and the call fails with
 * OS_ANN_ENOMEM.  Blocks always go back to the allocator that made them, even
 * after the hook changes.  Passing NULL for both functions restores the
 * library's own allocation (the HIP runtime behind an idle-block cache); one
 * NULL and one function is EINVAL.  Setting a hook also returns the idle
 * blocks of the library's own cache to the runtime.  Process-wide; not to be
 * called while another library call is running.
 *
 * Caller-owned workspaces (os_ann_search_opts.workspace) never come from the
 * hook: the caller allocates them.
 */
typedef void *(*os_ann_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*os_ann_free_fn)(void *ptr, void *stream, void *ctx);
int os_ann_set_allocator(os_ann_alloc_fn alloc, os_ann_free_fn free, void *ctx);

/* Last error code / message of the calling thread (OS_ANN_OK / "" if none). */
int os_ann_last_error(void);
const char *os_ann_last_error_message(void);

/* Library version string (host pointer, static storage). */
const char *os_ann_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OSANN_H */
