// Device helpers shared by the two matrix-core screening kernels (query-tile
// and cone-major): top-R list operations in the total order (d~, original
// row), order-preserving float bits for atomic minima, and the MFMA step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osann {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

__device__ inline bool pair_less(float d, uint32_t r, float e, uint32_t s) {
    return d < e || (d == e && r < s);
}

// Merge this lane's sorted list with lane^m's into the R smallest, sorted.
template <int R>
__device__ inline void merge_with(float (&d)[R], uint32_t (&r)[R], int m) {
    float pd[R];
    uint32_t pr[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        pd[k] = __shfl_xor(d[k], m, 64);
        pr[k] = (uint32_t)__shfl_xor((int)r[k], m, 64);
    }
#pragma unroll
    for (int k = 0; k < R; ++k)
        if (pair_less(pd[R - 1 - k], pr[R - 1 - k], d[k], r[k])) {
            d[k] = pd[R - 1 - k];
            r[k] = pr[R - 1 - k];
        }
#pragma unroll
    for (int j = R / 2; j > 0; j >>= 1)
#pragma unroll
        for (int k = 0; k < R; ++k)
            if ((k & j) == 0 && pair_less(d[k + j], r[k + j], d[k], r[k])) {
                const float td = d[k];
                d[k] = d[k + j];
                d[k + j] = td;
                const uint32_t tr = r[k];
                r[k] = r[k + j];
                r[k + j] = tr;
            }
}

template <int R>
__device__ inline void list_insert(float (&d)[R], uint32_t (&r)[R], float nd, uint32_t nr) {
    bool placed = false;
#pragma unroll
    for (int k = R - 1; k >= 1; --k) {
        if (!placed) {
            if (pair_less(nd, nr, d[k - 1], r[k - 1])) {
                d[k] = d[k - 1];
                r[k] = r[k - 1];
            } else {
                d[k] = nd;
                r[k] = nr;
                placed = true;
            }
        }
    }
    if (!placed) {
        d[0] = nd;
        r[0] = nr;
    }
}

// Order-preserving map of a non-NaN float to 32 bits (and back); 0xFFFFFFFF
// (above every float) stands for "no candidate yet".
__device__ inline uint32_t ord_bits(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float ord_float(uint32_t u) {
    if (u == 0xFFFFFFFFu) return __builtin_huge_valf();
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

// A value every lane of the wave holds alike, moved to scalar registers.
__device__ inline uint4 uni4(uint4 v) {
    return make_uint4(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y),
                      __builtin_amdgcn_readfirstlane(v.z), __builtin_amdgcn_readfirstlane(v.w));
}

template <bool F16IN>
__device__ inline f32x4_t mfma16(const uint4& a, const uint4& b, f32x4_t acc) {
    if (F16IN)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, b),
                                                      acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                   acc, 0, 0, 0);
}

constexpr int kHitCap = 64;   // hit buffer entries per wave (one full ballot)

}  // namespace osann
