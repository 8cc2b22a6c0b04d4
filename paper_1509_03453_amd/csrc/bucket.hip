// Bucket build: one cone-bucketed table of the database (Section 4).
//
//  * sort_by_cone   stable LSD radix sort of row ids by cone, 8-bit digits
//                   (also on 64-bit keys, for the sparse second-level table).
//                   Each block owns a contiguous chunk of the input; the rank
//                   of an element inside its block comes from wave ballots
//                   (lanes of equal digit below it) plus per-wave counts in
//                   LDS, in position order, so no atomic ever decides an
//                   order and rows of one cone keep ascending original ids.
//  * offsets        bucket starts read off the sorted cones.
//  * gather_planes  permuted, chunk-major copy of the rows (layout in
//                   osann_kernels.h), staged through LDS so that both the row
//                   reads and the plane writes are contiguous.
//  * probe tables   lexicographic L-subsets and sign-flip masks used by the
//                   query walk (Section 3.B).
#include "osann_device.h"
#include "osann_kernels.h"

namespace osann {

constexpr int kRadixThreads = 256;
constexpr int kRadixChunk = 2048;  // elements per block (8 tiles of 256)

static inline int64_t radix_blocks(int64_t N) { return (N + kRadixChunk - 1) / kRadixChunk; }
int64_t radix_hist_words(int64_t N) {
    const int64_t h = 256 * radix_blocks(N);
    return 2 * h + 1 + exclusive_scan_tmp_words(h);  // counts, scanned counts, scan scratch
}

template <typename K>
__global__ __launch_bounds__(kRadixThreads) void radix_hist_kernel(const K* __restrict__ keys, int64_t N, int shift,
                                                                   uint32_t* __restrict__ hist, int64_t nb) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixChunk;
    for (int t = 0; t < kRadixChunk; t += kRadixThreads) {
        int64_t i = base + t + threadIdx.x;
        if (i < N) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);  // counts only
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

template <typename K>
__global__ __launch_bounds__(kRadixThreads) void radix_scatter_kernel(
    const K* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, int64_t N, int shift,
    const uint32_t* __restrict__ hist, int64_t nb, K* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
    constexpr int kWaves = kRadixThreads / 64;
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kWaves][256];
    const int tid = threadIdx.x, w = tid / 64;
    run[tid] = hist[(int64_t)tid * nb + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kRadixChunk;
    for (int t = 0; t < kRadixChunk; t += kRadixThreads) {
#pragma unroll
        for (int a = 0; a < kWaves; ++a) wcnt[a][tid] = 0;
        __syncthreads();
        const int64_t i = base + t + tid;
        const bool valid = i < N;
        const K key = valid ? keys_in[i] : K(0);
        const uint32_t val = valid ? (vals_in ? vals_in[i] : (uint32_t)i) : 0u;
        const uint32_t dig = (uint32_t)(key >> shift) & 255u;
        // lanes of this wave holding the same digit
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t ones = __ballot((dig >> b) & 1u);
            same &= ((dig >> b) & 1u) ? ones : ~ones;
        }
        const uint32_t below = (uint32_t)__popcll(same & lanemask_lt());
        if (valid && below == 0) wcnt[w][dig] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t off = run[dig] + below;
            for (int a = 0; a < w; ++a) off += wcnt[a][dig];
            keys_out[off] = key;
            vals_out[off] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int a = 0; a < kWaves; ++a) add += wcnt[a][tid];
        run[tid] += add;
        __syncthreads();
    }
}

// The same sort for short inputs (a search's queries, small tables) in one
// block of 1024 threads and one launch, held in LDS.  Wave w owns the
// contiguous segment [w S, (w + 1) S) of the positions (S a multiple of 64),
// its lane l the items w S + 64 j + l, in registers.  Every pass:
//   1. each wave counts its segment's digits, 64 items at a time, into its
//      own LDS counts (one add per distinct digit, by the lowest lane
//      holding it: no atomics, no order taken from timing);
//   2. the counts are scanned digit-major, wave-minor, into each wave's
//      start per digit (earlier segments first: the sort stays stable);
//   3. each wave walks its segment again in order, each item's place being
//      its wave's running start for its digit plus the lanes of equal digit
//      below it (wave ballots), and scatters it into the LDS arrays;
// then the items are reloaded from there.  Only block barriers separate
// the steps; inside a step each wave works alone.
constexpr int kSmallSortThreads = 1024;
constexpr int kSmallSortItems = 16;  // per thread
constexpr int64_t kSmallSortMax = (int64_t)kSmallSortThreads * kSmallSortItems;

__global__ __launch_bounds__(kSmallSortThreads) void radix_small_kernel(const uint32_t* __restrict__ keys_in,
                                                                        int64_t N, int passes,
                                                                        uint32_t* __restrict__ keys_out,
                                                                        uint32_t* __restrict__ vals_out) {
    constexpr int kWaves = kSmallSortThreads / 64;
    __shared__ uint32_t s_key[kSmallSortMax];
    __shared__ uint32_t s_val[kSmallSortMax];
    __shared__ uint32_t cnt[kWaves][256];  // per wave: digit counts, then running starts
    __shared__ uint32_t tot[256];
    const int tid = threadIdx.x, w = tid / 64, l = tid % 64;
    const int64_t seg = ((N + kWaves * 64 - 1) / (kWaves * 64)) * 64;  // positions per wave
    const int groups = (int)(seg / 64);                                  // <= kSmallSortItems
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    };
    uint32_t key[kSmallSortItems], val[kSmallSortItems];
#pragma unroll
    for (int j = 0; j < kSmallSortItems; ++j) {
        const int64_t e = w * seg + 64 * j + l;
        const bool v = j < groups && e < N;
        key[j] = v ? keys_in[e] : 0u;
        val[j] = (uint32_t)e;
    }
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        for (int q = l; q < 256; q += 64) cnt[w][q] = 0;
        wave_sync();
#pragma unroll
        for (int j = 0; j < kSmallSortItems; ++j) {
            if (j >= groups) break;
            const int64_t e = w * seg + 64 * j + l;
            const bool valid = e < N;
            const uint32_t dig = (key[j] >> shift) & 255u;
            uint64_t same = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const uint64_t ones = __ballot((dig >> b) & 1u);
                same &= ((dig >> b) & 1u) ? ones : ~ones;
            }
            if (valid && (same & lanemask_lt()) == 0) cnt[w][dig] += (uint32_t)__popcll(same);
            wave_sync();
        }
        __syncthreads();
        if (tid < 256) {  // digit tid: prefix over the waves, then the total
            uint32_t c[kWaves], sum = 0;
#pragma unroll
            for (int a = 0; a < kWaves; ++a) c[a] = cnt[a][tid];
#pragma unroll
            for (int a = 0; a < kWaves; ++a) {
                cnt[a][tid] = sum;
                sum += c[a];
            }
            tot[tid] = sum;
        }
        __syncthreads();
        if (w == 0) {  // exclusive scan of the 256 totals: 4 per lane, then across the wave
            uint32_t c[4], sum = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                c[q] = tot[4 * l + q];
                sum += c[q];
            }
            uint32_t incl = sum;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t up = (uint32_t)__shfl_up((int)incl, d, 64);
                if (l >= d) incl += up;
            }
            uint32_t at = incl - sum;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                tot[4 * l + q] = at;
                at += c[q];
            }
        }
        __syncthreads();
        for (int q = l; q < 256; q += 64) cnt[w][q] += tot[q];  // this wave's start per digit
        wave_sync();
#pragma unroll
        for (int j = 0; j < kSmallSortItems; ++j) {
            if (j >= groups) break;
            const int64_t e = w * seg + 64 * j + l;
            const bool valid = e < N;
            const uint32_t dig = (key[j] >> shift) & 255u;
            uint64_t same = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const uint64_t ones = __ballot((dig >> b) & 1u);
                same &= ((dig >> b) & 1u) ? ones : ~ones;
            }
            const uint64_t below = same & lanemask_lt();
            if (valid) {
                const uint32_t off = cnt[w][dig] + (uint32_t)__popcll(below);
                s_key[off] = key[j];
                s_val[off] = val[j];
            }
            wave_sync();
            if (valid && below == 0) cnt[w][dig] += (uint32_t)__popcll(same);
            wave_sync();
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSmallSortItems; ++j) {
            const int64_t e = w * seg + 64 * j + l;
            if (j < groups && e < N) {
                key[j] = s_key[e];
                val[j] = s_val[e];
            }
        }
        __syncthreads();  // every item read before the next pass scatters
    }
#pragma unroll
    for (int j = 0; j < kSmallSortItems; ++j) {
        const int64_t e = w * seg + 64 * j + l;
        if (j < groups && e < N) {
            keys_out[e] = key[j];
            vals_out[e] = val[j];
        }
    }
}

hipError_t launch_sort_by_cone(const uint32_t* row_cone, int64_t N, int64_t n_cones, uint32_t* tmp,
                               uint32_t* perm_out, uint32_t* sorted_cone_out, hipStream_t s) {
    int bits = 1;
    while ((int64_t(1) << bits) < n_cones) ++bits;
    const int passes = (bits + 7) / 8;
    const int64_t nb = radix_blocks(N);
    uint32_t* ka = tmp;
    uint32_t* va = tmp + N;
    uint32_t* kb = tmp + 2 * N;
    uint32_t* vb = tmp + 3 * N;
    if (N > 0 && N <= kSmallSortMax) {
        hipLaunchKernelGGL(radix_small_kernel, dim3(1), dim3(kSmallSortThreads), 0, s, row_cone, N, passes,
                           sorted_cone_out, perm_out);
        return hipGetLastError();
    }
    const int64_t hw = 256 * nb;
    uint32_t* hist = tmp + 4 * N;        // per (digit, block) counts
    uint32_t* hscan = hist + hw;         // their exclusive scan (hw + 1 words)
    uint32_t* stmp = hscan + hw + 1;     // scan scratch
    const uint32_t* kin = row_cone;
    const uint32_t* vin = nullptr;  // identity on the first pass
    for (int p = 0; p < passes; ++p) {
        const bool last = p == passes - 1;
        uint32_t* kout = last ? sorted_cone_out : ((p & 1) ? kb : ka);
        uint32_t* vout = last ? perm_out : ((p & 1) ? vb : va);
        hipLaunchKernelGGL(radix_hist_kernel<uint32_t>, dim3((unsigned)nb), dim3(kRadixThreads), 0, s, kin, N,
                           8 * p, hist, nb);
        hipError_t e = launch_exclusive_scan(hist, hw, hscan, stmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(radix_scatter_kernel<uint32_t>, dim3((unsigned)nb), dim3(kRadixThreads), 0, s, kin,
                           vin, N, 8 * p, hscan, nb, kout, vout);
        kin = kout;
        vin = vout;
    }
    return hipGetLastError();
}

// The same sort on 64-bit keys (bits [0, end_bit) decide the order): row
// ids by key, ties in ascending row id.  tmp layout, in bytes: two key
// arrays of N u64, two id arrays of N u32, then the digit counts.
size_t radix_sort_u64_tmp_bytes(int64_t N) {
    return (size_t)N * 24 + (size_t)radix_hist_words(N) * 4;
}

hipError_t launch_radix_sort_u64(const uint64_t* key_in, int64_t N, int end_bit, void* tmp, uint64_t* key_out,
                                 uint32_t* perm_out, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (end_bit < 1 || end_bit > 64 || N > 0xFFFFFFFFll) return hipErrorInvalidValue;
    const int passes = (end_bit + 7) / 8;
    const int64_t nb = radix_blocks(N);
    uint64_t* ka = static_cast<uint64_t*>(tmp);
    uint64_t* kb = ka + N;
    uint32_t* va = reinterpret_cast<uint32_t*>(kb + N);
    uint32_t* vb = va + N;
    const int64_t hw = 256 * nb;
    uint32_t* hist = vb + N;
    uint32_t* hscan = hist + hw;
    uint32_t* stmp = hscan + hw + 1;
    const uint64_t* kin = key_in;
    const uint32_t* vin = nullptr;  // identity on the first pass
    for (int p = 0; p < passes; ++p) {
        const bool last = p == passes - 1;
        uint64_t* kout = last ? key_out : ((p & 1) ? kb : ka);
        uint32_t* vout = last ? perm_out : ((p & 1) ? vb : va);
        hipLaunchKernelGGL(radix_hist_kernel<uint64_t>, dim3((unsigned)nb), dim3(kRadixThreads), 0, s, kin, N,
                           8 * p, hist, nb);
        hipError_t e = launch_exclusive_scan(hist, hw, hscan, stmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(radix_scatter_kernel<uint64_t>, dim3((unsigned)nb), dim3(kRadixThreads), 0, s, kin,
                           vin, N, 8 * p, hscan, nb, kout, vout);
        kin = kout;
        vin = vout;
    }
    return hipGetLastError();
}

// offsets[c] = first sorted position whose cone is >= c; offsets[NC] = N.
__global__ void offsets_kernel(const uint32_t* __restrict__ sc, int64_t N, int64_t nc,
                               uint32_t* __restrict__ off) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > N) return;
    const int64_t lo = p == 0 ? 0 : (int64_t)sc[p - 1] + 1;
    const int64_t hi = p == N ? nc : (int64_t)sc[p];
    for (int64_t c = lo; c <= hi; ++c) off[c] = (uint32_t)p;
}

hipError_t launch_offsets(const uint32_t* sorted_cone, int64_t N, int64_t n_cones, uint32_t* offsets,
                          hipStream_t s) {
    const int64_t n = N + 1;
    hipLaunchKernelGGL(offsets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, sorted_cone,
                       N, n_cones, offsets);
    return hipGetLastError();
}

// 64 sorted positions per block: rows read element-wise (contiguous within a
// row), parked in LDS as 16-byte chunks, then written plane by plane.
template <typename E>
__global__ __launch_bounds__(256) void gather_planes_kernel(const typename E::raw* __restrict__ X,
                                                            int64_t N, int D, int nch,
                                                            const uint32_t* __restrict__ perm,
                                                            uint4* __restrict__ planes) {
    constexpr int EPC = 16 / E::bytes;  // elements per chunk
    extern __shared__ uint4 tile[];     // [nch][64]
    typename E::raw* te = reinterpret_cast<typename E::raw*>(tile);
    const int64_t p0 = (int64_t)blockIdx.x * 64;
    const int per_row = nch * EPC;
    for (int f = threadIdx.x; f < 64 * per_row; f += blockDim.x) {
        const int r = f / per_row, i = f % per_row;
        typename E::raw v = 0;
        if (p0 + r < N && i < D) v = X[(int64_t)perm[p0 + r] * D + i];
        te[((i / EPC) * 64 + r) * EPC + (i % EPC)] = v;
    }
    __syncthreads();
    for (int f = threadIdx.x; f < nch * 64; f += blockDim.x) {
        const int k = f / 64, r = f % 64;
        if (p0 + r < N) planes[(int64_t)k * N + p0 + r] = tile[k * 64 + r];
    }
}

// Rows of whole 16-byte chunks (D * element size a multiple of 16, rows
// 16-byte aligned): each block moves 64 rows as chunks, reading every row's
// chunks with consecutive lanes and writing every chunk plane with
// consecutive lanes, through an LDS tile [nch][65] (the pad keeps the
// chunks of one row in different banks).
__global__ __launch_bounds__(256) void gather_chunks_kernel(const uint4* __restrict__ X, int64_t N, int nch,
                                                            const uint32_t* __restrict__ perm,
                                                            uint4* __restrict__ planes) {
    extern __shared__ uint4 tile[];  // [nch][65]
    const int64_t p0 = (int64_t)blockIdx.x * 64;
    for (int f = threadIdx.x; f < 64 * nch; f += blockDim.x) {
        const int r = f / nch, k = f - r * nch;
        if (p0 + r < N) tile[k * 65 + r] = X[(int64_t)perm[p0 + r] * nch + k];
    }
    __syncthreads();
    for (int f = threadIdx.x; f < nch * 64; f += blockDim.x) {
        const int k = f >> 6, r = f & 63;
        if (p0 + r < N) planes[(int64_t)k * N + p0 + r] = tile[k * 65 + r];
    }
}

hipError_t launch_gather_planes(const void* X, int dtype, int64_t N, int D, const uint32_t* perm,
                                void* planes, hipStream_t s) {
    const int epc = chunk_elems(dtype);
    const int nch = (D + epc - 1) / epc;
    const dim3 grid((unsigned)((N + 63) / 64));
    const size_t lds = (size_t)nch * 64 * 16;
    auto out = static_cast<uint4*>(planes);
    if (D % epc == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0) {
        hipLaunchKernelGGL(gather_chunks_kernel, grid, dim3(256), (size_t)nch * 65 * 16, s,
                           static_cast<const uint4*>(X), N, nch, perm, out);
        return hipGetLastError();
    }
    switch (dtype) {
        case kF32:
            hipLaunchKernelGGL(gather_planes_kernel<F32>, grid, dim3(256), lds, s,
                               static_cast<const uint32_t*>(X), N, D, nch, perm, out);
            break;
        case kF16:
            hipLaunchKernelGGL(gather_planes_kernel<F16>, grid, dim3(256), lds, s,
                               static_cast<const uint16_t*>(X), N, D, nch, perm, out);
            break;
        case kU8:
            hipLaunchKernelGGL(gather_planes_kernel<U8>, grid, dim3(256), lds, s,
                               static_cast<const uint8_t*>(X), N, D, nch, perm, out);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// lexsub[j] = j-th L-subset of {0..D-1} in lexicographic order (unranked by
// counting the subsets that start with each candidate value).
__global__ void lexsub_kernel(int D, int L, int64_t count, uint8_t* __restrict__ lexsub) {
    // C(n, k) for n < D, k < L, computed once per block (the walk below
    // would otherwise redo each with k divisions)
    __shared__ uint64_t cb[kMaxD * 8];
    for (int i = threadIdx.x; i < D * L; i += blockDim.x) cb[(i / L) * 8 + i % L] = binom_dev(i / L, i % L);
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    uint64_t rem = (uint64_t)j;
    int prev = -1;
    for (int a = 0; a < L; ++a) {
        for (int v = prev + 1; v < D; ++v) {
            const uint64_t cnt = cb[(D - 1 - v) * 8 + (L - 1 - a)];
            if (rem < cnt) {
                lexsub[j * L + a] = (uint8_t)v;
                prev = v;
                break;
            }
            rem -= cnt;
        }
    }
}

// maskord = all L-bit masks ordered by (popcount, value).
__global__ void maskord_kernel(int L, uint8_t* __restrict__ maskord) {
    const int m = threadIdx.x;
    if (m >= (1 << L)) return;
    int rank = 0;
    for (int o = 0; o < (1 << L); ++o) {
        const int po = __popc(o), pm = __popc(m);
        rank += (po < pm) || (po == pm && o < m);
    }
    maskord[rank] = (uint8_t)m;
}

hipError_t launch_probe_tables(int D, int L, uint8_t* lexsub, uint8_t* maskord, hipStream_t s) {
    const int64_t count = binom_host(D, L);
    hipLaunchKernelGGL(lexsub_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, D, L,
                       count, lexsub);
    hipLaunchKernelGGL(maskord_kernel, dim3(1), dim3(128), 0, s, L, maskord);
    return hipGetLastError();
}

__global__ void count_nonempty_kernel(const uint32_t* __restrict__ off, int64_t nc,
                                      uint32_t* __restrict__ count) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ne = c < nc && off[c + 1] > off[c];
    const uint64_t m = __ballot(ne);
    if (lane_id() == 0 && m) atomicAdd(count, (uint32_t)__popcll(m));
}

hipError_t launch_count_nonempty(const uint32_t* offsets, int64_t n_cones, uint32_t* count,
                                 hipStream_t s) {
    hipLaunchKernelGGL(count_nonempty_kernel, dim3((unsigned)((n_cones + 255) / 256)), dim3(256), 0, s,
                       offsets, n_cones, count);
    return hipGetLastError();
}

__global__ void widen_kernel(const uint32_t* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int64_t)in[i];
}

hipError_t launch_widen_u32(const uint32_t* in, int64_t n, int64_t* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(widen_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}

template <typename E>
__global__ void planes_to_rows_kernel(const typename E::raw* __restrict__ planes, int64_t N, int D,
                                      float* __restrict__ rows) {
    constexpr int EPC = 16 / E::bytes;
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= N * D) return;
    const int64_t pos = f / D;
    const int i = (int)(f % D);
    rows[f] = E::val(planes[((int64_t)(i / EPC) * N + pos) * EPC + (i % EPC)]);
}

hipError_t launch_planes_to_rows(const void* planes, int dtype, int64_t N, int D, float* rows,
                                 hipStream_t s) {
    const int64_t n = N * D;
    const dim3 grid((unsigned)((n + 255) / 256));
    switch (dtype) {
        case kF32:
            hipLaunchKernelGGL(planes_to_rows_kernel<F32>, grid, dim3(256), 0, s,
                               static_cast<const uint32_t*>(planes), N, D, rows);
            break;
        case kF16:
            hipLaunchKernelGGL(planes_to_rows_kernel<F16>, grid, dim3(256), 0, s,
                               static_cast<const uint16_t*>(planes), N, D, rows);
            break;
        case kU8:
            hipLaunchKernelGGL(planes_to_rows_kernel<U8>, grid, dim3(256), 0, s,
                               static_cast<const uint8_t*>(planes), N, D, rows);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace osann
