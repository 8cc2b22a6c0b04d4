// Device helpers shared by the gfx950 kernels: element decoding, the
// magnitude order of components, cone ids and wave64 primitives.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osann {

// ---------------------------------------------------------------------------
// Elements.  Magnitudes are compared as unsigned integers: for finite IEEE
// values the bit pattern without its sign bit is monotone in |v|, so the
// order is exact and needs no floating-point arithmetic.
// ---------------------------------------------------------------------------
struct F32 {
    using raw = uint32_t;
    static constexpr int bytes = 4;
    __device__ static uint32_t mag(raw b) { return b & 0x7FFFFFFFu; }
    __device__ static bool neg(raw b) { return (b >> 31) && mag(b); }
    __device__ static bool nonfinite(raw b) { return mag(b) >= 0x7F800000u; }
    __device__ static float val(raw b) { return __uint_as_float(b); }
};
struct F16 {
    using raw = uint16_t;
    static constexpr int bytes = 2;
    __device__ static uint32_t mag(raw b) { return b & 0x7FFFu; }
    __device__ static bool neg(raw b) { return (b >> 15) && mag(b); }
    __device__ static bool nonfinite(raw b) { return mag(b) >= 0x7C00u; }
    __device__ static float val(raw b) { return (float)__builtin_bit_cast(_Float16, b); }
};
struct U8 {
    using raw = uint8_t;
    static constexpr int bytes = 1;
    __device__ static uint32_t mag(raw b) { return b; }
    __device__ static bool neg(raw) { return false; }
    __device__ static bool nonfinite(raw) { return false; }
    __device__ static float val(raw b) { return (float)b; }
};

// Sort key of component i: larger key = earlier in decreasing-magnitude
// order, ties to the lower index.  Bit 0 carries the sign bit (1 unless the
// value is negative); it never decides the order since indices are unique.
__device__ inline uint64_t comp_key(uint32_t mag, int i, bool neg) {
    return ((uint64_t)mag << 9) | ((uint64_t)(255 - i) << 1) | (neg ? 0u : 1u);
}
__device__ inline int key_index(uint64_t k) { return 255 - (int)((k >> 1) & 0xFF); }
__device__ inline int key_sign(uint64_t k) { return (int)(k & 1); }

// C(n, k) for the small arguments of cone ids (k <= 7, n <= 255).
__device__ inline uint64_t binom_dev(int n, int k) {
    if (k < 0 || n < k) return 0;
    uint64_t c = 1;
    for (int t = 0; t < k; ++t) c = c * (uint64_t)(n - t) / (uint64_t)(t + 1);
    return c;
}

// Cone id of L (index, sign bit) pairs in any order: colex rank of the
// ascending index set times 2^L, plus the sign bits with the lowest index as
// most significant bit.
template <int L>
__device__ inline uint32_t cone_of(int (&idx)[L], int (&sg)[L]) {
#pragma unroll
    for (int a = 1; a < L; ++a)
#pragma unroll
        for (int b = L - 1; b >= a; --b)
            if (idx[b - 1] > idx[b]) {
                int t = idx[b]; idx[b] = idx[b - 1]; idx[b - 1] = t;
                t = sg[b]; sg[b] = sg[b - 1]; sg[b - 1] = t;
            }
    uint64_t rank = 0;
    uint32_t bits = 0;
#pragma unroll
    for (int j = 0; j < L; ++j) {
        rank += binom_dev(idx[j], j + 1);
        bits = (bits << 1) | (uint32_t)sg[j];
    }
    return (uint32_t)((rank << L) | bits);
}

// ---------------------------------------------------------------------------
// wave64 primitives
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return (int)__lane_id(); }

__device__ inline uint64_t lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = (uint32_t)__shfl_xor((int)lo, m, 64);
    hi = (uint32_t)__shfl_xor((int)hi, m, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint32_t shfl_u32(uint32_t v, int src) {
    return (uint32_t)__shfl((int)v, src, 64);
}

// Inclusive prefix sum over the wave (Kogge-Stone with shuffles).
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    int l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = (uint32_t)__shfl_up((int)v, o, 64);
        if (l >= o) v += t;
    }
    return v;
}

// Lexicographic minimum of (d, row) over the wave; every lane gets it.
__device__ inline void wave_argmin(float& d, uint32_t& row) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        float od = __shfl_xor(d, o, 64);
        uint32_t orow = (uint32_t)__shfl_xor((int)row, o, 64);
        if (od < d || (od == d && orow < row)) {
            d = od;
            row = orow;
        }
    }
}

}  // namespace osann
