// Exclusive prefix sum of u32 values in three passes (block sums, scan of the
// block sums, block-local scans), used for padded bucket offsets and for the
// per-tile probe totals of the tiled search.
#include "osann_device.h"
#include "osann_kernels.h"

namespace osann {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;  // elements per block

int64_t exclusive_scan_tmp_words(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* warp_tot, uint32_t* total) {
    const int w = threadIdx.x / 64, l = lane_id();
    const uint32_t incl = wave_incl_scan(v);
    if (l == 63) warp_tot[w] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int a = 0; a < kScanThreads / 64; ++a) {
        if (a < w) before += warp_tot[a];
        all += warp_tot[a];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_block_sums(const uint32_t* __restrict__ in, int64_t n,
                                                                uint32_t* __restrict__ bsum) {
    __shared__ uint32_t wt[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    uint32_t s = 0;
#pragma unroll
    for (int e = 0; e < kScanPer; ++e)
        if (base + e < n) s += in[base + e];
    uint32_t tot;
    block_excl_scan(s, wt, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void scan_spine(uint32_t* __restrict__ bsum, int64_t nb) {
    __shared__ uint32_t wt[kScanThreads / 64];
    const int64_t seg = (nb + kScanThreads - 1) / kScanThreads;
    const int64_t b = threadIdx.x * seg, e = b + seg < nb ? b + seg : nb;
    uint32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += bsum[i];
    uint32_t tot;
    uint32_t run = block_excl_scan(s, wt, &tot);
    for (int64_t i = b; i < e; ++i) {
        const uint32_t x = bsum[i];
        bsum[i] = run;
        run += x;
    }
    if (threadIdx.x == 0) bsum[nb] = tot;
}

__global__ __launch_bounds__(kScanThreads) void scan_apply(const uint32_t* __restrict__ in, int64_t n,
                                                           const uint32_t* __restrict__ bsum, int64_t nb,
                                                           uint32_t* __restrict__ out) {
    __shared__ uint32_t wt[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer], s = 0;
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
        v[e] = base + e < n ? in[base + e] : 0u;
        s += v[e];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(s, wt, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) {
        if (base + e < n) out[base + e] = run;
        run += v[e];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bsum[nb];
}

hipError_t launch_exclusive_scan(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* tmp,
                                 hipStream_t s) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        hipLaunchKernelGGL(scan_spine, dim3(1), dim3(kScanThreads), 0, s, tmp, (int64_t)0);
        hipLaunchKernelGGL(scan_apply, dim3(1), dim3(kScanThreads), 0, s, in, n, tmp, (int64_t)0, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(scan_block_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, tmp);
    hipLaunchKernelGGL(scan_spine, dim3(1), dim3(kScanThreads), 0, s, tmp, nb);
    hipLaunchKernelGGL(scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, tmp, nb, out);
    return hipGetLastError();
}

}  // namespace osann
