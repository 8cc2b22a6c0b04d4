// Internal interface of the sparse table (Section 4: a second-level hash
// table manages the tables when the cones are very many).  Only the
// non-empty cones are stored: their 64-bit cone ids in ascending order, the
// offsets of their rows in the bucket order (rows sorted by cone, then by
// row id), and an open-addressing hash table from cone id to bucket number.
// A walk position whose cone is not in the table is an empty cone.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osann {

constexpr uint64_t kSparseEmpty = ~0ull;        // free hash slot (no cone id reaches 2^63)
constexpr uint64_t kSparseAll = ~0ull;          // walk length meaning "every row"
constexpr uint64_t kSparseWalkCap = 1ull << 22; // walk positions a sparse walk takes at most

struct SparseTable {
    const uint64_t* hkeys;    // [hmask + 1] cone id per slot (kSparseEmpty: free)
    const uint32_t* hval;     // [hmask + 1] bucket number per slot
    uint64_t hmask;
    // One-hash bit filter in front of the table (no false negatives): bit
    // (mix(id) >> 32) & fmask is set for every non-empty cone id.  At 32 bits
    // per key (at most 4 MB) it stays in the caches and answers most probes of empty
    // cones (about 3% of them pass it).
    const uint64_t* filt;     // [(fmask + 1) / 64] words
    uint64_t fmask;
    const uint32_t* offsets;  // [n_ne + 1] first row position of each bucket
    const uint64_t* binom;    // [257][8] C(n, k)
    const uint8_t* maskord;   // [128] flip masks by popcount, then value
    int64_t n_sub;            // C(D, L)
    int64_t n_cones;          // C(D, L) 2^L
    int64_t N;
    int D, L;
};

// 64-bit cone id of every row from its packed top-L pairs.
hipError_t launch_sparse_keys(const uint64_t* row_top, int64_t N, int L, const uint64_t* binom, uint64_t* key,
                              hipStream_t s);
// Stable sort of the rows by cone id (row ids ascending within a cone):
// sorted ids to key_out, row ids to perm.  tmp holds sparse_sort_tmp_bytes.
size_t sparse_sort_tmp_bytes(int64_t N, int end_bit);
hipError_t launch_sparse_sort(const uint64_t* key_in, uint64_t* key_out, uint32_t* perm, int64_t N, int end_bit,
                              void* tmp, size_t tmp_bytes, hipStream_t s);
// flag[i] = 1 where sorted[i] starts a new cone.
hipError_t launch_sparse_heads(const uint64_t* sorted, int64_t N, uint32_t* flag, hipStream_t s);
// From the exclusive scan pos[0..N] of the flags: keys[pos[i]] and
// offsets[pos[i]] = i at every head, offsets[pos[N]] = N.
hipError_t launch_sparse_compact(const uint64_t* sorted, const uint32_t* flag, const uint32_t* pos, int64_t N,
                                 uint64_t* keys, uint32_t* offsets, hipStream_t s);
// Hash table of n distinct keys in cap (a power of two >= 2n) slots, and
// their filter of fbits bits (a power of two, 64 to 2^32).
hipError_t launch_sparse_hash(const uint64_t* keys, int64_t n, uint64_t* hkeys, uint32_t* hval, uint64_t cap,
                              uint64_t* filt, uint64_t fbits, hipStream_t s);
// Filter size for n keys: a power of two >= 32 n bits, from 2^12 to 2^25.
uint64_t sparse_filter_bits(int64_t n);

// Search: walk (row budget, the first C cones, or at most kSparseWalkCap
// positions) and FP32 scan with arg-min in one pass per query, from the
// walk state the probe kernel wrote.
struct SparseSearchArgs {
    SparseTable t;
    const void* planes;    // chunk-major rows in bucket order
    int dtype, nch;
    const float* yf;       // [Q][dpad]
    int dpad;
    const uint8_t* order;  // [Q][D]
    const uint8_t* sbit;   // [Q][D]
    const uint32_t* perm;
    int64_t Q, budget;
    int cones;             // 1: budget is the number C of cones
    int64_t* out_idx;
    float* out_dist;
    int64_t* out_ncand;    // rows compared (may be null)
    unsigned long long* out_capped;  // walks stopped by the kSparseWalkCap limit: added to (may be null)
};
hipError_t launch_sparse_search(const SparseSearchArgs& a, hipStream_t s);

}  // namespace osann
