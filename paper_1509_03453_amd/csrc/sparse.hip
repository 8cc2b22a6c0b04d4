// Sparse table (Section 4: a second-level hash table manages the tables when
// the cones are very many).  With C(D,L) 2^L above what a dense offsets
// array can address, only the non-empty cones are kept: the rows' 64-bit
// cone ids are sorted (stable, so the rows of a cone keep ascending ids),
// the distinct ids get bucket numbers and row offsets, and an
// open-addressing hash table maps a cone id to its bucket number.
//
// Searching walks the Section 3.B order as the dense path does, but walk
// position j is decoded without the dense subset table: the subset of rank
// positions is unranked from its lexicographic rank through the colex rank
// of the reflected subset (greedy, one binary search over C(s, k) per
// element), then the cone id is looked up; a missing id is an empty cone.
// Walk and scan run in one pass, since the cones of a sparse table hold few
// rows and a second walk would cost as much as the first.

#include "osann_device.h"
#include "osann_kernels.h"
#include "osann_sparse.h"

namespace osann {

namespace {

// SplitMix64 output function (Steele, Lea and Flood, 2014) as the hash.
__device__ inline uint64_t sparse_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Bucket number of a cone id, or -1 for an empty cone.  At least half the
// slots are free, so every probe sequence ends at a free slot.
__device__ inline int64_t sparse_lookup(const SparseTable& t, uint64_t key) {
    const uint64_t m = sparse_mix(key);
    const uint64_t b = (m >> 32) & t.fmask;
    if (!((t.filt[b >> 6] >> (b & 63)) & 1ull)) return -1;  // not in the filter: an empty cone
    uint64_t h = m & t.hmask;
    for (uint64_t step = 0; step <= t.hmask; ++step) {
        const uint64_t k = t.hkeys[h];
        if (k == key) return t.hval[h];
        if (k == kSparseEmpty) return -1;
        h = (h + 1) & t.hmask;
    }
    return -1;
}

// 64-bit cone id of up to 7 (index, sign bit) pairs; entries beyond L hold
// index 0x7FFF so that they sort last.  Colex rank of the ascending index
// set times 2^L, plus the sign bits in ascending index order, the lowest
// index most significant.
// LT > 0: L is LT, known at compile time, and only the first LT entries
// are sorted (the rest hold 0x7FFF and stay last); LT = 0: L at run time.
// BT: element type of the binomial table (uint32_t where every binomial
// read is below 2^32).
template <int LT = 0, typename BT = uint64_t>
__device__ inline uint64_t sparse_cone_id(int L, int (&idx)[7], int (&sg)[7], const BT* __restrict__ binom) {
    constexpr int NS = LT > 0 ? LT : 7;
    if (LT > 0) L = LT;
#pragma unroll
    for (int a = 1; a < NS; ++a)
#pragma unroll
        for (int b = NS - 1; b >= a; --b)
            if (idx[b - 1] > idx[b]) {
                int u = idx[b]; idx[b] = idx[b - 1]; idx[b - 1] = u;
                u = sg[b]; sg[b] = sg[b - 1]; sg[b - 1] = u;
            }
    BT rank = 0;
    uint64_t bits = 0;
#pragma unroll
    for (int j = 0; j < NS; ++j)
        if (j < L) {
            rank += binom[idx[j] * 8 + j + 1];
            bits = (bits << 1) | (uint64_t)sg[j];
        }
    return ((uint64_t)rank << L) | bits;
}

// Cone at walk position j: block h of C(D,L) C(L,h) positions (flipped
// signs), the lexicographic L-subset T of rank positions and the flip mask;
// T is unranked from the colex rank C(D,L) - 1 - t of {D-1-T_b}, whose
// k-th largest element s_k is the largest s with C(s, k) <= the remaining
// rank.  T_b = D-1-s_{L-b}, and mask bit L-1-b (= k-1) flips the sign of
// component order[T_b].
template <int LT, typename BT>
__device__ inline uint64_t sparse_walk_cone(uint64_t j, const SparseTable& t, const BT* __restrict__ bn,
                                            const uint8_t* order, const uint8_t* sbit) {
    const int L = LT > 0 ? LT : t.L, D = t.D;
    const uint64_t nsub = (uint64_t)t.n_sub;
    uint64_t tt = j;
    int mask = 0;
    if (j >= nsub) {
        uint64_t base = nsub, cl = 1;
        int mstart = 1;
        for (int h = 1; h <= L; ++h) {
            cl = (uint64_t)bn[L * 8 + h];
            const uint64_t sz = nsub * cl;
            if (j < base + sz) break;
            base += sz;
            mstart += (int)cl;
        }
        const uint64_t jj = j - base;
        tt = jj / cl;
        mask = t.maskord[mstart + (int)(jj % cl)];
    }
    BT r = (BT)(nsub - 1 - tt);
    int idx[7], sg[7];
#pragma unroll
    for (int k = 7; k >= 1; --k) {
        idx[k - 1] = 0x7FFF;
        sg[k - 1] = 0;
        if (k <= L) {
            int lo = k - 1, hi = D - 1;  // C(k-1, k) = 0 <= r
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (bn[mid * 8 + k] <= r)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            r -= bn[lo * 8 + k];
            const int c = order[D - 1 - lo];
            idx[k - 1] = c;
            sg[k - 1] = sbit[c] ^ ((mask >> (k - 1)) & 1);
        }
    }
    return sparse_cone_id<LT, BT>(L, idx, sg, bn);
}

__global__ void sparse_keys_kernel(const uint64_t* __restrict__ row_top, int64_t N, int L,
                                   const uint64_t* __restrict__ binom, uint64_t* __restrict__ key) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const uint64_t top = row_top[n];
    int idx[7], sg[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        idx[j] = 0x7FFF;
        sg[j] = 0;
        if (j < L) {
            const uint32_t pr = (uint32_t)(top >> (9 * j)) & 0x1FFu;
            idx[j] = (int)(pr & 0xFFu);
            sg[j] = (int)(pr >> 8);
        }
    }
    key[n] = sparse_cone_id(L, idx, sg, binom);
}

__global__ void sparse_heads_kernel(const uint64_t* __restrict__ sorted, int64_t N, uint32_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) flag[i] = (i == 0 || sorted[i] != sorted[i - 1]) ? 1u : 0u;
}

__global__ void sparse_compact_kernel(const uint64_t* __restrict__ sorted, const uint32_t* __restrict__ flag,
                                      const uint32_t* __restrict__ pos, int64_t N, uint64_t* __restrict__ keys,
                                      uint32_t* __restrict__ offsets) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (flag[i]) {
        keys[pos[i]] = sorted[i];
        offsets[pos[i]] = (uint32_t)i;
    }
    if (i == N - 1) offsets[pos[N]] = (uint32_t)N;
}

__global__ void sparse_fill_kernel(uint64_t* __restrict__ p, uint64_t n, uint64_t v) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void sparse_insert_kernel(const uint64_t* __restrict__ keys, int64_t n, uint64_t* hkeys,
                                     uint32_t* __restrict__ hval, uint64_t mask, uint64_t* filt, uint64_t fmask) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const uint64_t key = keys[u];
    const uint64_t m = sparse_mix(key);
    const uint64_t b = (m >> 32) & fmask;
    atomicOr(reinterpret_cast<unsigned long long*>(filt + (b >> 6)), 1ull << (b & 63));
    uint64_t h = m & mask;
    for (uint64_t step = 0; step <= mask; ++step) {
        const unsigned long long prev =
            atomicCAS(reinterpret_cast<unsigned long long*>(hkeys + h), (unsigned long long)kSparseEmpty,
                      (unsigned long long)key);
        if (prev == (unsigned long long)kSparseEmpty) {
            hval[h] = (uint32_t)u;
            return;
        }
        h = (h + 1) & mask;
    }
}

constexpr int kSparseWaves = 4;

// One wave per query, 64 walk positions at a time: each lane decodes its
// position and looks the cone up; a wave prefix sum of the bucket sizes
// finds where the row budget is met (row budget) or the positions end
// (first C cones, or the walk cap); the rows of the taken cones go to the
// lanes through a cursor over the running counts; FP32 distance term by
// term and arg-min on (distance, original row).  The binomials and the walk
// state sit in LDS.
template <typename E, int LT, typename BT>
__global__ __launch_bounds__(64 * kSparseWaves) void sparse_search_kernel(SparseSearchArgs a) {
    __shared__ BT s_binom[257 * 8];
    __shared__ uint8_t order[kSparseWaves][kMaxD];
    __shared__ uint8_t sbit[kSparseWaves][kMaxD];
    __shared__ float ys[kSparseWaves][kMaxD];
    __shared__ uint32_t s_start[kSparseWaves][64];
    __shared__ uint32_t s_incl[kSparseWaves][64];
    const int w = threadIdx.x / 64, l = lane_id();
    const int64_t q = (int64_t)blockIdx.x * kSparseWaves + w;
    const bool qv = q < a.Q;
    for (int i = threadIdx.x; i < 257 * 8; i += 64 * kSparseWaves) s_binom[i] = (BT)a.t.binom[i];
    const SparseTable t = a.t;
    const int D = t.D;
    for (int i = l; i < a.dpad; i += 64) ys[w][i] = qv ? a.yf[q * a.dpad + i] : 0.0f;
    for (int i = l; i < D; i += 64) {
        order[w][i] = qv ? a.order[q * D + i] : 0;
        sbit[w][i] = qv ? a.sbit[q * D + i] : 0;
    }
    __syncthreads();
    if (!qv) return;  // no block barrier below this point
    const float* y = ys[w];
    const uint4* planes = static_cast<const uint4*>(a.planes);
    float best = __builtin_huge_valf();
    uint32_t brow = 0xFFFFFFFFu;
    auto visit = [&](int64_t p) {
        const float d = row_dist_fp32<E>(planes, t.N, a.nch, p, y);
        if (d <= best) {
            const uint32_t row = a.perm[p];
            if (d < best || row < brow) {
                best = d;
                brow = row;
            }
        }
    };
    const uint64_t nc = (uint64_t)t.n_cones, budget = (uint64_t)a.budget;
    uint64_t carry = 0;
    bool capped = false;
    if ((!a.cones && budget >= (uint64_t)t.N) || (a.cones && budget >= nc)) {  // every row
        for (int64_t p = l; p < t.N; p += 64) visit(p);
        carry = (uint64_t)t.N;
    } else {
        uint64_t limit = nc < kSparseWalkCap ? nc : kSparseWalkCap;
        if (a.cones && budget < limit) limit = budget;
        uint32_t* st = s_start[w];
        uint32_t* in = s_incl[w];
        bool done = false;
        for (uint64_t j0 = 0; j0 < limit && !done; j0 += 64) {
            const uint64_t j = j0 + l;
            uint32_t start = 0, len = 0;
            if (j < limit) {
                const int64_t u = sparse_lookup(t, sparse_walk_cone<LT, BT>(j, t, s_binom, order[w], sbit[w]));
                if (u >= 0) {
                    start = t.offsets[u];
                    len = t.offsets[u + 1] - start;
                }
            }
            uint32_t incl = wave_incl_scan(len);  // distinct cones: 64 of them hold at most N rows
            if (!a.cones) {
                const uint64_t reached = __ballot(j < limit && carry + incl >= budget);
                if (reached) {  // positions after the one that meets the budget are not taken
                    const int sl = __ffsll((unsigned long long)reached) - 1;
                    const uint32_t at = shfl_u32(incl, sl);
                    if (l > sl) incl = at;
                    done = true;
                }
            }
            st[l] = start;
            in[l] = incl;
            const uint32_t total = shfl_u32(incl, 63);
            carry += total;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            uint32_t k = 0;
            for (uint32_t f = l; f < total; f += 64) {
                while (in[k] <= f) ++k;
                const uint32_t before = k ? in[k - 1] : 0u;
                visit((int64_t)st[k] + (f - before));
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        // stopped by the position cap: a row budget not met although cones
        // remained, or a C beyond the cap
        capped = a.cones ? limit == kSparseWalkCap && budget > limit && nc > limit : !done && limit < nc;
    }
    wave_argmin(best, brow);
    if (l == 0) {
        a.out_idx[q] = brow == 0xFFFFFFFFu ? -1 : (int64_t)brow;
        a.out_dist[q] = best;
        if (a.out_ncand) a.out_ncand[q] = (int64_t)carry;
        if (capped && a.out_capped) atomicAdd(a.out_capped, 1ull);
    }
}

inline dim3 grid_for(int64_t n, int b) { return dim3((unsigned)((n + b - 1) / b)); }

}  // namespace

hipError_t launch_sparse_keys(const uint64_t* row_top, int64_t N, int L, const uint64_t* binom, uint64_t* key,
                              hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (L < 1 || L > 7) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sparse_keys_kernel, grid_for(N, 256), dim3(256), 0, s, row_top, N, L, binom, key);
    return hipGetLastError();
}

size_t sparse_sort_tmp_bytes(int64_t N, int end_bit) {
    (void)end_bit;
    return radix_sort_u64_tmp_bytes(N);
}

hipError_t launch_sparse_sort(const uint64_t* key_in, uint64_t* key_out, uint32_t* perm, int64_t N, int end_bit,
                              void* tmp, size_t tmp_bytes, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (tmp_bytes < radix_sort_u64_tmp_bytes(N)) return hipErrorInvalidValue;
    return launch_radix_sort_u64(key_in, N, end_bit, tmp, key_out, perm, s);
}

hipError_t launch_sparse_heads(const uint64_t* sorted, int64_t N, uint32_t* flag, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(sparse_heads_kernel, grid_for(N, 256), dim3(256), 0, s, sorted, N, flag);
    return hipGetLastError();
}

hipError_t launch_sparse_compact(const uint64_t* sorted, const uint32_t* flag, const uint32_t* pos, int64_t N,
                                 uint64_t* keys, uint32_t* offsets, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(sparse_compact_kernel, grid_for(N, 256), dim3(256), 0, s, sorted, flag, pos, N, keys, offsets);
    return hipGetLastError();
}

uint64_t sparse_filter_bits(int64_t n) {
    uint64_t bits = uint64_t(1) << 12;
    while (bits < 32 * (uint64_t)(n > 0 ? n : 0) && bits < (uint64_t(1) << 25)) bits <<= 1;
    return bits;
}

hipError_t launch_sparse_hash(const uint64_t* keys, int64_t n, uint64_t* hkeys, uint32_t* hval, uint64_t cap,
                              uint64_t* filt, uint64_t fbits, hipStream_t s) {
    if (cap == 0 || (cap & (cap - 1)) || cap < 2 * (uint64_t)n) return hipErrorInvalidValue;
    if (fbits < 64 || (fbits & (fbits - 1)) || fbits > (uint64_t(1) << 32) || filt == nullptr)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(sparse_fill_kernel, grid_for((int64_t)cap, 256), dim3(256), 0, s, hkeys, cap, kSparseEmpty);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sparse_fill_kernel, grid_for((int64_t)(fbits / 64), 256), dim3(256), 0, s, filt, fbits / 64,
                       uint64_t(0));
    e = hipGetLastError();
    if (e != hipSuccess || n <= 0) return e;
    hipLaunchKernelGGL(sparse_insert_kernel, grid_for(n, 256), dim3(256), 0, s, keys, n, hkeys, hval, cap - 1, filt,
                       fbits - 1);
    return hipGetLastError();
}

// Whether every binomial the walk reads (C(n, k), n < D, k <= L) and the
// subset ranks (< C(D, L)) are below 2^32.
static bool binom_fits_32(int D, int L) {
    uint64_t c = 1, top = 0;
    for (int k = 1; k <= L; ++k) {  // C(D-1, k) from C(D-1, k-1); exact in 64 bits for D <= 256, k <= 7
        c = c * (uint64_t)(D - k) / (uint64_t)k;
        if (c > top) top = c;
    }
    uint64_t nsub = 1;
    for (int k = 1; k <= L; ++k) nsub = nsub * (uint64_t)(D - k + 1) / (uint64_t)k;
    return top < (uint64_t(1) << 32) && nsub < (uint64_t(1) << 32);
}

// The walk compiled for each L (1 to 7) and binomial width.
template <typename E, typename BT>
static hipError_t search_lb(const SparseSearchArgs& a, dim3 grid, dim3 block, hipStream_t s) {
    switch (a.t.L) {
        case 1: hipLaunchKernelGGL((sparse_search_kernel<E, 1, BT>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((sparse_search_kernel<E, 2, BT>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((sparse_search_kernel<E, 3, BT>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((sparse_search_kernel<E, 4, BT>), grid, block, 0, s, a); break;
        case 5: hipLaunchKernelGGL((sparse_search_kernel<E, 5, BT>), grid, block, 0, s, a); break;
        case 6: hipLaunchKernelGGL((sparse_search_kernel<E, 6, BT>), grid, block, 0, s, a); break;
        case 7: hipLaunchKernelGGL((sparse_search_kernel<E, 7, BT>), grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename E>
static hipError_t search_l(const SparseSearchArgs& a, dim3 grid, dim3 block, hipStream_t s) {
    return binom_fits_32(a.t.D, a.t.L) ? search_lb<E, uint32_t>(a, grid, block, s)
                                       : search_lb<E, uint64_t>(a, grid, block, s);
}

hipError_t launch_sparse_search(const SparseSearchArgs& a, hipStream_t s) {
    if (a.Q <= 0) return hipSuccess;
    if (a.t.D < 1 || a.t.D > kMaxD || a.t.L < 1 || a.t.L > 7 || a.dpad > kMaxD || a.budget < 1)
        return hipErrorInvalidValue;
    const dim3 grid = grid_for(a.Q, kSparseWaves), block(64 * kSparseWaves);
    switch (a.dtype) {
        case kF32: return search_l<F32>(a, grid, block, s);
        case kF16: return search_l<F16>(a, grid, block, s);
        case kU8: return search_l<U8>(a, grid, block, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace osann
