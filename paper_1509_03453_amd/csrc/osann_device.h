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

// Same as cone_of for a run-time L <= kMaxL (fixed-size arrays, guarded
// loops, so the arrays stay in registers); binomials from a table
// binom[n*8 + k] = C(n, k).
__device__ inline uint32_t cone_of_rt(int L, int (&idx)[7], int (&sg)[7], const uint32_t* __restrict__ binom) {
#pragma unroll
    for (int a = 1; a < 7; ++a)
#pragma unroll
        for (int b = 6; b >= a; --b)
            if (b < L && idx[b - 1] > idx[b]) {
                int t = idx[b]; idx[b] = idx[b - 1]; idx[b - 1] = t;
                t = sg[b]; sg[b] = sg[b - 1]; sg[b - 1] = t;
            }
    uint64_t rank = 0;
    uint32_t bits = 0;
#pragma unroll
    for (int j = 0; j < 7; ++j)
        if (j < L) {
            rank += binom[idx[j] * 8 + j + 1];
            bits = (bits << 1) | (uint32_t)sg[j];
        }
    return (uint32_t)((rank << L) | bits);
}

// Walk position j of a query -> cone (Section 3.B order).  The walk is laid
// out in blocks h = 0..L of C(D,L)*C(L,h) positions: block h takes the
// L-subsets T of rank positions in lexicographic order (lexsub) and, inside
// each T, the sign-flip masks of popcount h in ascending value (maskord);
// mask bit L-1-b flips the sign of component order[T_b].  order[] lists the
// query's components by decreasing magnitude and sbit[] holds the query's
// sign bits by component.
__device__ inline uint32_t probe_cone(int64_t j, int L, const uint8_t* order, const uint8_t* sbit,
                                      int64_t n_sub, const uint8_t* __restrict__ lexsub,
                                      const uint8_t* __restrict__ maskord, const uint32_t* __restrict__ binom) {
    int64_t t = j;
    int mask = 0;
    if (j >= n_sub) {  // phase B: some signs flipped
        int64_t base = n_sub;
        int mstart = 1;
        uint64_t cl = 1;
        for (int h = 1; h <= L; ++h) {
            cl = binom[L * 8 + h];
            const int64_t sz = n_sub * (int64_t)cl;
            if (j < base + sz) break;
            base += sz;
            mstart += (int)cl;
        }
        const int64_t jj = j - base;
        int64_t r;
        if (jj < (int64_t(1) << 32)) {  // 32-bit division (a short sequence; 64-bit is a long one)
            const uint32_t q32 = (uint32_t)jj / (uint32_t)cl;
            t = q32;
            r = (uint32_t)jj - q32 * (uint32_t)cl;
        } else {
            t = jj / (int64_t)cl;
            r = jj - t * (int64_t)cl;
        }
        mask = maskord[mstart + (int)r];
    }
    int idx[7], sg[7];
#pragma unroll
    for (int b = 0; b < 7; ++b) {
        if (b < L) {
            idx[b] = order[lexsub[t * L + b]];
            sg[b] = sbit[idx[b]] ^ ((mask >> (L - 1 - b)) & 1);
        } else {
            idx[b] = 0;
            sg[b] = 0;
        }
    }
    return cone_of_rt(L, idx, sg, binom);
}

// 16-byte chunk of stored components -> FP32 values (exact).
template <typename E>
struct Unpack;
template <>
struct Unpack<F32> {
    static constexpr int n = 4;
    __device__ static void run(const uint4& v, float (&o)[4]) {
        o[0] = __uint_as_float(v.x);
        o[1] = __uint_as_float(v.y);
        o[2] = __uint_as_float(v.z);
        o[3] = __uint_as_float(v.w);
    }
};
template <>
struct Unpack<F16> {
    static constexpr int n = 8;
    __device__ static void run(const uint4& v, float (&o)[8]) {
        const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            o[2 * k] = F16::val((uint16_t)(wv[k] & 0xFFFFu));
            o[2 * k + 1] = F16::val((uint16_t)(wv[k] >> 16));
        }
    }
};
template <>
struct Unpack<U8> {
    static constexpr int n = 16;
    __device__ static void run(const uint4& v, float (&o)[16]) {
        const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int b = 0; b < 4; ++b) o[4 * k + b] = (float)((wv[k] >> (8 * b)) & 0xFFu);
    }
};

// Squared distance between the row at sorted position `pos` of the
// chunk-major planes and the FP32 query y (zero padded to nch chunks): in
// ascending component order, subtraction, product and sum each rounded.
template <typename E>
__device__ inline float row_dist_fp32(const uint4* __restrict__ planes, int64_t N, int nch, int64_t pos,
                                      const float* y) {
#pragma clang fp contract(off)
    constexpr int EPC = Unpack<E>::n;
    float acc = 0.0f;
    for (int c = 0; c < nch; ++c) {
        float x[EPC];
        Unpack<E>::run(planes[(int64_t)c * N + pos], x);
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            const float d = x[e] - y[c * EPC + e];
            const float sq = d * d;
            acc = acc + sq;
        }
    }
    return acc;
}

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
__device__ inline uint16_t bf16_rne(float f) {
    const uint32_t b = __float_as_uint(f);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
// Round-to-nearest-even FP32 -> FP16 bits.
__device__ inline uint16_t f16_rne(float f) {
    return __builtin_bit_cast(uint16_t, (_Float16)f);
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
