// Matrix-core screening of the candidates with an exact FP32 re-rank.
//
// Queries are sorted by their own cone and cut into tiles of 64 (four waves
// of 16).  A work item is (tile, split): split s owns a contiguous range of
// the non-empty cones.  The block first marks, in an LDS table over that
// range, which of its 64 queries probe each cone (each wave regenerates its
// queries' walks, Section 3.B); then for every marked cone it streams the
// cone's rows in 16-row MFMA tiles (bucket sizes are padded to 16 rows in
// the low-precision copy).  With the rows as the MFMA A operand and the
// wave's 16 queries as B, lane l holds the dot products of query l%16 with 4
// rows, so each lane keeps a private top-R list of (d~, row) for one query,
// where d~ = ||x^||^2 - 2 q^.x^ ranks candidates like the squared distance
// of the rounded vectors.  The four lanes of a query merge their lists with
// shuffles (bitonic), and the split's list goes to a per-query slot.  A
// finishing pass merges the splits, recomputes the exact FP32 distance of
// the R survivors and keeps the arg-min on (distance, row).  The order in
// which candidates are met never matters: lists are kept in the total order
// (d~, row), so results do not depend on the batch or the split.
#include "osann_device.h"
#include "osann_kernels.h"
#include "osann_tiled.h"

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

template <bool F16IN, int KS, int R>
__global__ __launch_bounds__(256) void tiled_screen_kernel(TiledArgs a) {
    extern __shared__ uint64_t tab[];
    __shared__ uint8_t s_order[4][kMaxD];
    __shared__ uint8_t s_sbit[4][kMaxD];
    __shared__ uint32_t s_item;
    const int w = threadIdx.x / 64, l = lane_id();
    const int64_t total = a.T * a.S;
    const int64_t span = (a.n_ne + a.S - 1) / a.S;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1u);
        __syncthreads();
        const int64_t item = s_item;
        __syncthreads();
        if (item >= total) break;
        const int64_t t = item / a.S;
        const int s = (int)(item % a.S);
        const int64_t n0 = s * span;
        const int64_t n1 = n0 + span < a.n_ne ? n0 + span : a.n_ne;
        const int nspan = n1 > n0 ? (int)(n1 - n0) : 0;

        // 1. which of the tile's queries probe each cone of the split
        for (int i = threadIdx.x; i < nspan; i += blockDim.x) tab[i] = 0;
        __syncthreads();
        for (int c = 0; c < 16; ++c) {
            const int slot = 16 * w + c;
            const int64_t qs = t * kTileQ + slot;
            if (qs >= a.Q) break;
            const uint32_t q = a.qorder[qs];
            const uint32_t js = a.jstop[q];
            const unsigned long long bit = 1ull << slot;
            if (js == kWalkAll) {
                for (int i = l; i < nspan; i += 64) atomicOr((unsigned long long*)&tab[i], bit);
                continue;
            }
            for (int i = l; i < a.D; i += 64) {
                s_order[w][i] = a.order[(int64_t)q * a.D + i];
                s_sbit[w][i] = a.sbit[(int64_t)q * a.D + i];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            for (uint32_t j0 = 0; j0 < js; j0 += 64) {
                const uint32_t j = j0 + l;
                if (j < js) {
                    const uint32_t cone =
                        probe_cone(j, a.L, s_order[w], s_sbit[w], a.n_sub, a.lexsub, a.maskord, a.binom);
                    if (a.offsets[cone + 1] > a.offsets[cone]) {
                        const int64_t e = a.ne_id[cone];
                        if (e >= n0 && e < n1) atomicOr((unsigned long long*)&tab[e - n0], bit);
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        __syncthreads();

        // 2. this wave's 16 queries as the MFMA B operand
        const int64_t myslot = t * kTileQ + 16 * w + (l % 16);
        const bool qok = myslot < a.Q;
        const uint32_t myq = qok ? a.qorder[myslot] : 0u;
        uint4 bq[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            bq[ks] = qok ? *reinterpret_cast<const uint4*>(a.ql + (int64_t)myq * a.dk + ks * 32 + 8 * (l / 16))
                         : make_uint4(0, 0, 0, 0);

        float ld[R];
        uint32_t lr[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            ld[k] = __builtin_huge_valf();
            lr[k] = 0xFFFFFFFFu;
        }

        // 3. stream the marked cones' rows through the matrix cores
        for (int i = 0; i < nspan; ++i) {
            const uint64_t m = tab[i];
            const uint32_t wm = (uint32_t)(m >> (16 * w)) & 0xFFFFu;
            if (wm == 0) continue;
            const bool probed = (wm >> (l % 16)) & 1u;
            const uint32_t cone = a.ne_cone[n0 + i];
            const uint32_t p1 = a.poff[cone + 1];
            for (uint32_t p = a.poff[cone]; p < p1; p += 16) {
                f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
                const uint16_t* arow = a.xl + (int64_t)(p + (l % 16)) * a.dk + 8 * (l / 16);
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const uint4 av = *reinterpret_cast<const uint4*>(arow + ks * 32);
                    if (F16IN)
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8_t, av),
                                                                    __builtin_bit_cast(f16x8_t, bq[ks]), acc, 0,
                                                                    0, 0);
                    else
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, av),
                                                                     __builtin_bit_cast(bf16x8_t, bq[ks]), acc, 0,
                                                                     0, 0);
                }
                const int64_t rb = (int64_t)p + 4 * (l / 16);
                const float4 nv = *reinterpret_cast<const float4*>(a.nrm + rb);
                const float nn[4] = {nv.x, nv.y, nv.z, nv.w};
#pragma unroll
                for (int ii = 0; ii < 4; ++ii) {
                    const float d = nn[ii] - 2.0f * acc[ii];
                    if (probed && d <= ld[R - 1]) {
                        const uint32_t row = a.prow[rb + ii];
                        if (d < ld[R - 1] || row < lr[R - 1]) list_insert<R>(ld, lr, d, row);
                    }
                }
            }
        }

        // 4. merge the four lanes of each query, store the split's list
        merge_with<R>(ld, lr, 16);
        merge_with<R>(ld, lr, 32);
        if (l < 16 && qok) {
            uint2* dst = a.part + ((int64_t)myq * a.S + s) * R;
#pragma unroll
            for (int k = 0; k < R; ++k) dst[k] = make_uint2(__float_as_uint(ld[k]), lr[k]);
        }
        __syncthreads();
    }
}

// One group of G lanes per query: merge the S split lists, re-rank the R
// survivors with the exact FP32 distance, arg-min on (distance, row).
template <typename E, int R, int G>
__global__ __launch_bounds__(256) void tiled_finish_kernel(FinishArgs f) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t q = gid / G;
    const int g = (int)(gid % G);
    const bool qv = q < f.Q;
    float ld[R];
    uint32_t lr[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        ld[k] = __builtin_huge_valf();
        lr[k] = 0xFFFFFFFFu;
        if (qv && g < f.S) {
            const uint2 e = f.part[(q * f.S + g) * R + k];
            ld[k] = __uint_as_float(e.x);
            lr[k] = e.y;
        }
    }
#pragma unroll
    for (int m = 1; m < G; m <<= 1) merge_with<R>(ld, lr, m);
    uint32_t cr = 0xFFFFFFFFu;
#pragma unroll
    for (int k = 0; k < R; ++k)
        if (k == g) cr = lr[k];
    float cd = __builtin_huge_valf();
    if (qv && cr != 0xFFFFFFFFu)
        cd = row_dist_fp32<E>(static_cast<const uint4*>(f.planes), f.N, f.nch, f.iperm[cr], f.yf + q * f.dpad);
#pragma unroll
    for (int m = 1; m < G; m <<= 1) {
        const float od = __shfl_xor(cd, m, 64);
        const uint32_t orr = (uint32_t)__shfl_xor((int)cr, m, 64);
        if (pair_less(od, orr, cd, cr)) {
            cd = od;
            cr = orr;
        }
    }
    if (qv && g == 0) {
        f.out_idx[q] = cr == 0xFFFFFFFFu ? -1 : (int64_t)cr;
        f.out_dist[q] = cd;
    }
}

template <bool F16IN, int R>
static hipError_t screen_ks(const TiledArgs& a, int ks, dim3 grid, size_t lds, hipStream_t s) {
    switch (ks) {
        case 1: hipLaunchKernelGGL((tiled_screen_kernel<F16IN, 1, R>), grid, dim3(256), lds, s, a); break;
        case 2: hipLaunchKernelGGL((tiled_screen_kernel<F16IN, 2, R>), grid, dim3(256), lds, s, a); break;
        case 4: hipLaunchKernelGGL((tiled_screen_kernel<F16IN, 4, R>), grid, dim3(256), lds, s, a); break;
        case 8: hipLaunchKernelGGL((tiled_screen_kernel<F16IN, 8, R>), grid, dim3(256), lds, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tiled_screen(const TiledArgs& a, int R, int f16in, int blocks, hipStream_t s) {
    const int ks = a.dk / 32;
    const int64_t span = (a.n_ne + a.S - 1) / a.S;
    const size_t lds = (size_t)(span > 0 ? span : 1) * sizeof(uint64_t);
    const dim3 grid((unsigned)blocks);
    if (f16in) {
        if (R == 4) return screen_ks<true, 4>(a, ks, grid, lds, s);
        if (R == 8) return screen_ks<true, 8>(a, ks, grid, lds, s);
        if (R == 16) return screen_ks<true, 16>(a, ks, grid, lds, s);
    } else {
        if (R == 4) return screen_ks<false, 4>(a, ks, grid, lds, s);
        if (R == 8) return screen_ks<false, 8>(a, ks, grid, lds, s);
        if (R == 16) return screen_ks<false, 16>(a, ks, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

template <typename E, int R>
static hipError_t finish_g(const FinishArgs& f, hipStream_t s) {
    const int G = f.S > R ? f.S : R;
    const int64_t threads = f.Q * G;
    const dim3 grid((unsigned)((threads + 255) / 256));
    switch (G) {
        case 4: hipLaunchKernelGGL((tiled_finish_kernel<E, R, 4>), grid, dim3(256), 0, s, f); break;
        case 8: hipLaunchKernelGGL((tiled_finish_kernel<E, R, 8>), grid, dim3(256), 0, s, f); break;
        case 16: hipLaunchKernelGGL((tiled_finish_kernel<E, R, 16>), grid, dim3(256), 0, s, f); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename E>
static hipError_t finish_r(const FinishArgs& f, int R, hipStream_t s) {
    if (R == 4) return finish_g<E, 4>(f, s);
    if (R == 8) return finish_g<E, 8>(f, s);
    if (R == 16) return finish_g<E, 16>(f, s);
    return hipErrorInvalidValue;
}

hipError_t launch_tiled_finish(const FinishArgs& f, int R, hipStream_t s) {
    if (f.Q <= 0) return hipSuccess;
    switch (f.dtype) {
        case kF32: return finish_r<F32>(f, R, s);
        case kF16: return finish_r<F16>(f, R, s);
        case kU8: return finish_r<U8>(f, R, s);
    }
    return hipErrorInvalidValue;
}

hipError_t tiled_screen_max_lds(size_t bytes) {
    hipError_t e = hipSuccess;
#define OSANN_SET_LDS(F16IN, KS, R)                                                                        \
    if (e == hipSuccess)                                                                                   \
        e = hipFuncSetAttribute((const void*)tiled_screen_kernel<F16IN, KS, R>,                            \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
#define OSANN_SET_LDS_R(F16IN, KS) OSANN_SET_LDS(F16IN, KS, 4) OSANN_SET_LDS(F16IN, KS, 8) OSANN_SET_LDS(F16IN, KS, 16)
#define OSANN_SET_LDS_KS(F16IN) \
    OSANN_SET_LDS_R(F16IN, 1) OSANN_SET_LDS_R(F16IN, 2) OSANN_SET_LDS_R(F16IN, 4) OSANN_SET_LDS_R(F16IN, 8)
    OSANN_SET_LDS_KS(true)
    OSANN_SET_LDS_KS(false)
#undef OSANN_SET_LDS_KS
#undef OSANN_SET_LDS_R
#undef OSANN_SET_LDS
    return e;
}

int tiled_screen_occupancy(int R, int f16in, int ks, size_t lds) {
    int nb = 0;
    const void* fn = nullptr;
#define OSANN_PICK(F16IN, KS, RR) \
    if (f16in == (int)F16IN && ks == KS && R == RR) fn = (const void*)tiled_screen_kernel<F16IN, KS, RR>;
#define OSANN_PICK_R(F16IN, KS) OSANN_PICK(F16IN, KS, 4) OSANN_PICK(F16IN, KS, 8) OSANN_PICK(F16IN, KS, 16)
#define OSANN_PICK_KS(F16IN) OSANN_PICK_R(F16IN, 1) OSANN_PICK_R(F16IN, 2) OSANN_PICK_R(F16IN, 4) OSANN_PICK_R(F16IN, 8)
    OSANN_PICK_KS(true)
    OSANN_PICK_KS(false)
#undef OSANN_PICK_KS
#undef OSANN_PICK_R
#undef OSANN_PICK
    if (!fn) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, lds) != hipSuccess) return 0;
    return nb;
}

}  // namespace osann
