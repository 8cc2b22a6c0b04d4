// Internal interface between the host ABI layer (osann_abi.cpp) and the HIP
// kernels for gfx950.  Not installed; the public interface is include/osann.h.
//
// Device data layout of an index (N rows of D components, storage type T):
//   row_cone[N]   u32  cone id of each original row
//   row_top[N]    u64  top-L (index, sign) pairs, 9 bits each, decreasing |x|
//   perm[N]       u32  original row at each bucket-sorted position
//   offsets[NC+1] u32  bucket c = sorted positions [offsets[c], offsets[c+1])
//   planes        16-byte chunks, component-chunk major:
//                 planes[k*N + pos] holds components [k*E, k*E+E) of the row
//                 at sorted position pos (E = 16/sizeof(T), zero padded past D).
//                 A wave reading 64 consecutive positions of one chunk reads
//                 1 KiB of contiguous memory, and each lane still sees its own
//                 row's components in ascending order.
//   lexsub[C(D,L)][L] u8  L-subsets of rank positions in lexicographic order
//   maskord[2^L]  u8   sign-flip masks ordered by (popcount, value)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osann {

constexpr int kMaxD = 256;
constexpr int kMaxL = 7;
constexpr int64_t kMaxCones = int64_t(1) << 24;

// Storage type codes (same values as the public OS_ANN_F32 / F16 / U8).
enum DType : int { kF32 = 0, kF16 = 1, kU8 = 2 };

inline int elem_bytes(int dtype) { return dtype == kF32 ? 4 : dtype == kF16 ? 2 : 1; }
inline int chunk_elems(int dtype) { return 16 / elem_bytes(dtype); }

// C(n, k) on the host (0 when k > n).
inline int64_t binom_host(int n, int k) {
    if (k < 0 || n < 0 || k > n) return 0;
    int64_t c = 1;
    for (int t = 0; t < k; ++t) c = c * (n - t) / (t + 1);
    return c;
}

// ---- launchers (each enqueues on `s`, returns the hipError_t of the launch) ----

// Key kernel: top-L pairs, cone id, non-finite flag (atomic OR of 1).
hipError_t launch_row_keys(const void* X, int dtype, int64_t N, int D, int L,
                           uint32_t* row_cone, uint64_t* row_top, uint32_t* nonfinite,
                           hipStream_t s);

// Stable LSD radix sort of (cone, row) by cone; writes perm and sorted cones.
// tmp must hold 4 arrays of N u32 plus radix_hist_words(N) u32.  The scan of
// the per-block digit counts uses launch_exclusive_scan.
int64_t radix_hist_words(int64_t N);
hipError_t launch_sort_by_cone(const uint32_t* row_cone, int64_t N, int64_t n_cones,
                               uint32_t* tmp, uint32_t* perm_out, uint32_t* sorted_cone_out,
                               hipStream_t s);

// The same stable sort on 64-bit keys, by bits [0, end_bit) (1..64): row ids
// (0..N-1) by key to perm_out, sorted keys to key_out.  tmp holds
// radix_sort_u64_tmp_bytes(N) bytes.
size_t radix_sort_u64_tmp_bytes(int64_t N);
hipError_t launch_radix_sort_u64(const uint64_t* key_in, int64_t N, int end_bit, void* tmp, uint64_t* key_out,
                                 uint32_t* perm_out, hipStream_t s);

// Bucket offsets from the sorted cones.
hipError_t launch_offsets(const uint32_t* sorted_cone, int64_t N, int64_t n_cones,
                          uint32_t* offsets, hipStream_t s);

// Permuted, chunk-major copy of the rows.
hipError_t launch_gather_planes(const void* X, int dtype, int64_t N, int D,
                                const uint32_t* perm, void* planes, hipStream_t s);

// Probe-order tables and the non-empty cone count.
hipError_t launch_probe_tables(int D, int L, uint8_t* lexsub, uint8_t* maskord, hipStream_t s);
hipError_t launch_count_nonempty(const uint32_t* offsets, int64_t n_cones, uint32_t* count,
                                 hipStream_t s);

// Export helpers.
hipError_t launch_widen_u32(const uint32_t* in, int64_t n, int64_t* out, hipStream_t s);
hipError_t launch_planes_to_rows(const void* planes, int dtype, int64_t N, int D,
                                 float* rows, hipStream_t s);

// Exclusive prefix sum: out[0..n] (out[n] = total); tmp holds
// exclusive_scan_tmp_words(n) words.
int64_t exclusive_scan_tmp_words(int64_t n);
hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* tmp,
                                 hipStream_t s);

// jstop value meaning "every row is a candidate" (budget >= N).
constexpr uint32_t kWalkAll = 0xFFFFFFFFu;

// Query classification and walk state (Section 3.B).  Per query the kernel
// stores its decreasing-magnitude order and sign bits and the length of the
// walk prefix that meets the budget; consumers regenerate the probed cones
// from that state (probe_cone), so no per-probe list is materialised.
struct ProbeArgs {
    const void* Y;          // queries [Q][D], dtype qtype
    int qtype;
    int64_t Q;
    int D, L;
    const uint32_t* offsets;
    int64_t n_cones, n_sub; // N_C and C(D,L)
    int64_t N;
    int64_t budget;         // max_candidates
    const uint8_t* lexsub;
    const uint8_t* maskord;
    const uint32_t* binom;  // [256*8] C(n, k)
    // outputs (any may be null)
    float* yf;              // [Q][dpad] FP32 copy of the queries (zero padded)
    int dpad;
    uint16_t* ql;           // [Q][dk] BF16 (or FP16) copy for the matrix-core path
    int dk;
    int ql_f16;             // 1: FP16 rounding, 0: BF16 rounding
    uint8_t* order;         // [Q][D] components by decreasing magnitude
    uint8_t* sbit;          // [Q][D] sign bit of each component
    uint32_t* jstop;        // [Q] walk positions taken (kWalkAll: every row)
    uint32_t* nprobe;       // [Q] non-empty cones probed
    int64_t* ncand;         // [Q]
    uint32_t* q_cone;       // [Q]
    uint64_t* q_top;        // [Q]
    // optional bitmap of the probed non-empty cones, [Q][nw] words
    uint64_t* qbits;
    int64_t nw;
    const uint32_t* ne_id;  // cone -> rank among the non-empty cones
    int64_t n_ne;
    const uint32_t* cone_base;  // [Q] first bucket of each query's cone ids in offsets (null: 0)
};
hipError_t launch_probe(const ProbeArgs& a, hipStream_t s);

// FP32 candidate scan + arg-min (eq. (1), Algorithm 1).
struct ScanArgs {
    const void* planes;
    int dtype;
    int64_t N;
    int D, L, nch;          // nch = number of 16-byte chunks per row
    const float* yf;        // [Q][nch*E]
    int64_t Q;
    const uint8_t* order;
    const uint8_t* sbit;
    const uint32_t* jstop;
    const uint32_t* offsets;
    int64_t n_sub;
    const uint8_t* lexsub;
    const uint8_t* maskord;
    const uint32_t* binom;
    const uint32_t* perm;
    int64_t* out_idx;
    float* out_dist;
    int waves_per_query;    // 1, 2 or 4
    const uint32_t* cone_base;  // [Q] first bucket of each query's cone ids in offsets (null: 0)
};
hipError_t launch_scan_fp32(const ScanArgs& a, hipStream_t s);

// Several bases: one table per basis over the same original rows.
constexpr int kMaxRot = 16;
struct RotArgs {
    int64_t N;
    int D, L, R, nch, dtype, dpad;
    int64_t n_cones, n_sub;
    const uint32_t* offsets;          // [R][n_cones+1]
    const uint32_t* perm;             // [R][N] original row at each position of basis r's table
    const uint64_t* xtop;             // [R][R][N] packed top-L pairs, in basis r2, of basis r's rows
    const uint4* const* planes_tab;   // [R] device pointers: basis r's table, original rows, chunk-major
    const uint8_t* lexsub;
    const uint8_t* maskord;
    const uint32_t* binom;
    int64_t Q, budget;
    const float* yr;                  // [R][Q][D] query coordinates in each basis
    const float* yf;                  // [Q][dpad] FP32 queries
    uint8_t* order;                   // [Q][R][D] walk state per basis
    uint8_t* sbit;                    // [Q][R][D]
    uint32_t* kstop;                  // [Q] schedule slots visited
    int64_t* visited;                 // [Q] rows of the visited cones (repeats counted), may be null
    int64_t* out_idx;
    float* out_dist;
    int64_t* out_ncand;               // distinct rows analyzed, may be null
    int waves_per_query;              // 1, 2 or 4
};
hipError_t launch_rotate(const void* X, int dtype, int64_t N, int D, const float* M, float* out, hipStream_t s);

// PCA front-end (Section 4.B): keys P (x - mu) (mu may be null), and the
// float64 mean and covariance of the rows (scratch: moments_scratch_doubles).
hipError_t launch_project(const void* X, int dtype, int64_t N, int D, const float* mu, const float* P, int k,
                          float* out, hipStream_t s);
size_t moments_scratch_doubles(int64_t N, int D);
hipError_t launch_moments(const void* X, int dtype, int64_t N, int D, double* mean, double* cov, double* scratch,
                          hipStream_t s);
hipError_t launch_probe_rot(const RotArgs& a, hipStream_t s);
hipError_t launch_scan_rot(const RotArgs& a, hipStream_t s);
hipError_t launch_gather_top(const uint32_t* perm, int64_t N, const uint64_t* top2, uint64_t* xt, hipStream_t s);

}  // namespace osann
