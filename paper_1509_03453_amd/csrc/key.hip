// Key kernel: for every database row, the L largest-magnitude components
// (index and sign, decreasing magnitude) and the row's cone id
// (Section 2, eq. (2); Fig. 2).
//
// Work split: S lanes of a wave64 share one row (S = power of two), lane t
// reading components t, t+S, t+2S, ... so that the wave's loads are
// contiguous.  Each lane keeps its own top-L list in registers; the group
// then runs L rounds of a shuffle max-reduction on the packed component keys
// and the winning lane drops its head.  Integer compares only, so the result
// is exact and independent of the lane split.
#include "osann_device.h"
#include "osann_kernels.h"

namespace osann {

template <typename E, int L>
__global__ __launch_bounds__(256) void row_keys_kernel(const typename E::raw* __restrict__ X,
                                                       int64_t N, int D, int S, int vec,
                                                       uint32_t* __restrict__ row_cone,
                                                       uint64_t* __restrict__ row_top,
                                                       uint32_t* __restrict__ nonfinite) {
    const int t = threadIdx.x % S;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / S) + threadIdx.x / S;
    const bool valid = row < N;

    uint64_t top[L];
#pragma unroll
    for (int j = 0; j < L; ++j) top[j] = 0;  // every real key is >= 1
    bool bad = false;
    // keys carry the component index, so they are distinct and the
    // insertion order does not matter
    auto insert = [&](typename E::raw b, int i) __attribute__((always_inline)) {
        bad |= E::nonfinite(b);
        const uint64_t k = comp_key(E::mag(b), i, E::neg(b));
#pragma unroll
        for (int j = L - 1; j >= 0; --j) {  // into the descending list
            const uint64_t above = j > 0 ? top[j - 1] : ~0ull;
            if (k > top[j]) top[j] = (k > above) ? above : k;
        }
    };
    struct alignas(4 * sizeof(typename E::raw)) Raw4 {
        typename E::raw v[4];
    };
    if (valid && vec) {
        // D a multiple of 4, rows aligned: components 4t .. 4t + 3 and
        // 4t + 4S .. 4t + 4S + 3 (then 8S further ...), two loads per lane
        // issued before either is inserted
        const typename E::raw* xr = X + row * (int64_t)D;
        for (int i0 = 4 * t; i0 < D; i0 += 8 * S) {
            const bool two = i0 + 4 * S < D;
            const Raw4 v0 = *reinterpret_cast<const Raw4*>(xr + i0);
            Raw4 v1{};
            if (two) v1 = *reinterpret_cast<const Raw4*>(xr + i0 + 4 * S);
#pragma unroll
            for (int u = 0; u < 4; ++u) insert(v0.v[u], i0 + u);
            if (two)
#pragma unroll
                for (int u = 0; u < 4; ++u) insert(v1.v[u], i0 + 4 * S + u);
        }
    } else if (valid) {
        const typename E::raw* xr = X + row * (int64_t)D;
        // four components per step, loaded before any is inserted
        constexpr int U = 4;
        for (int i0 = t; i0 < D; i0 += U * S) {
            typename E::raw b[U];
#pragma unroll
            for (int u = 0; u < U; ++u) b[u] = i0 + u * S < D ? xr[i0 + u * S] : typename E::raw(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (i0 + u * S >= D) break;
                insert(b[u], i0 + u * S);
            }
        }
    }
    if (bad) atomicOr(nonfinite, 1u);

    uint64_t win[L];
#pragma unroll
    for (int j = 0; j < L; ++j) {
        uint64_t m = top[0];
        for (int o = 1; o < S; o <<= 1) {
            uint64_t other = shfl_xor_u64(m, o);
            m = other > m ? other : m;
        }
        win[j] = m;
        if (top[0] == m) {  // exactly one lane of the group holds it
#pragma unroll
            for (int a = 0; a < L - 1; ++a) top[a] = top[a + 1];
            top[L - 1] = 0;
        }
    }

    if (valid && t == 0) {
        int idx[L], sg[L];
        uint64_t packed = 0;
#pragma unroll
        for (int j = 0; j < L; ++j) {
            idx[j] = key_index(win[j]);
            sg[j] = key_sign(win[j]);
            packed |= (uint64_t)((uint32_t)idx[j] | ((uint32_t)sg[j] << 8)) << (9 * j);
        }
        row_top[row] = packed;
        row_cone[row] = cone_of<L>(idx, sg);
    }
}

template <typename E>
static hipError_t dispatch_keys(const void* X, int64_t N, int D, int L, uint32_t* cone,
                                uint64_t* top, uint32_t* flag, hipStream_t s) {
    auto x = static_cast<const typename E::raw*>(X);
    const int vec = D % 4 == 0 && reinterpret_cast<uintptr_t>(X) % (4 * sizeof(typename E::raw)) == 0;
    int S = 1;
    // about four components per lane, eight with the vector loads
    while (S * 2 <= D / (vec ? 8 : 4) && S < 64) S *= 2;
    const int threads = 256;
    const int64_t rows_per_block = threads / S;
    const dim3 grid((unsigned)((N + rows_per_block - 1) / rows_per_block));
    switch (L) {
#define OSANN_KEY_CASE(LL)                                                                        \
    case LL:                                                                                      \
        hipLaunchKernelGGL((row_keys_kernel<E, LL>), grid, dim3(threads), 0, s, x, N, D, S, vec, \
                           cone, top, flag);                                                      \
        break;
        OSANN_KEY_CASE(1) OSANN_KEY_CASE(2) OSANN_KEY_CASE(3) OSANN_KEY_CASE(4)
        OSANN_KEY_CASE(5) OSANN_KEY_CASE(6) OSANN_KEY_CASE(7)
#undef OSANN_KEY_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_row_keys(const void* X, int dtype, int64_t N, int D, int L, uint32_t* row_cone,
                           uint64_t* row_top, uint32_t* nonfinite, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    switch (dtype) {
        case kF32: return dispatch_keys<F32>(X, N, D, L, row_cone, row_top, nonfinite, s);
        case kF16: return dispatch_keys<F16>(X, N, D, L, row_cone, row_top, nonfinite, s);
        case kU8: return dispatch_keys<U8>(X, N, D, L, row_cone, row_top, nonfinite, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace osann
