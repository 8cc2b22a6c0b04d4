// Structured bases (Section 3.D): coordinates in H diag(s) by the fast
// Walsh-Hadamard transform, O(D log D) per row instead of the O(D^2) of a
// dense basis.  One wave64 per row: component j sits in lane j % 64,
// register j / 64.  Strides below 64 pair lanes (a cross-lane exchange),
// strides of 64 and more pair registers of one lane.  The lower element of
// each pair keeps a + b, the upper a - b, each rounded in FP32, so the
// result does not depend on how the butterflies are scheduled.
#include "osann_device.h"
#include "osann_kernels.h"
#include "osann_wht.h"

namespace osann {

constexpr int kWhtWaves = 4;

template <typename E>
__global__ __launch_bounds__(64 * kWhtWaves) void wht_kernel(const void* __restrict__ X, int64_t N, int D,
                                                           const float* __restrict__ signs,
                                                           float* __restrict__ out) {
#pragma clang fp contract(off)
    const int l = lane_id();
    const int64_t n = (int64_t)blockIdx.x * kWhtWaves + threadIdx.x / 64;
    if (n >= N) return;  // no barrier in this kernel
    auto x = static_cast<const typename E::raw*>(X) + n * D;
    float v[kMaxD / 64];
#pragma unroll
    for (int m = 0; m < kMaxD / 64; ++m) {
        const int j = l + 64 * m;
        v[m] = j < D ? signs[j] * E::val(x[j]) : 0.0f;
    }
    const int lane_strides = D < 64 ? D : 64;
    for (int h = 1; h < lane_strides; h <<= 1) {
        const bool upper = (l & h) != 0;
#pragma unroll
        for (int m = 0; m < kMaxD / 64; ++m) {
            const float p = __shfl_xor(v[m], h, 64);
            v[m] = upper ? p - v[m] : v[m] + p;
        }
    }
    for (int hm = 1; 64 * hm < D; hm <<= 1) {
#pragma unroll
        for (int m = 0; m < kMaxD / 64; ++m) {
            if ((m & hm) == 0 && m + hm < kMaxD / 64) {
                const float a = v[m], b = v[m + hm];
                v[m] = a + b;
                v[m + hm] = a - b;
            }
        }
    }
#pragma unroll
    for (int m = 0; m < kMaxD / 64; ++m) {
        const int j = l + 64 * m;
        if (j < D) out[n * D + j] = v[m];
    }
}

hipError_t launch_wht(const void* X, int dtype, int64_t N, int D, const float* signs, float* out, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (D < 1 || D > kMaxD || (D & (D - 1))) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((N + kWhtWaves - 1) / kWhtWaves)), block(64 * kWhtWaves);
    switch (dtype) {
        case kF32: hipLaunchKernelGGL(wht_kernel<F32>, grid, block, 0, s, X, N, D, signs, out); break;
        case kF16: hipLaunchKernelGGL(wht_kernel<F16>, grid, block, 0, s, X, N, D, signs, out); break;
        case kU8: hipLaunchKernelGGL(wht_kernel<U8>, grid, block, 0, s, X, N, D, signs, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace osann
