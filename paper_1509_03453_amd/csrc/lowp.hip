// Low-precision copy of an index for the matrix-core screening pass.
//
// Buckets are re-laid out with their size rounded up to 16 rows, so that a
// 16-row MFMA tile never straddles two buckets:
//   poff[c]        padded start of bucket c (poff[NC] = NP)
//   xl[p][dk]      row at padded position p, BF16 (round to nearest even) for
//                  FP32 and uint8 data, FP16 as stored for FP16 data; dk = D
//                  rounded up to 32 (one MFMA K step); zero padded
//   nrm[p]         FP32 sum of squares of the rounded row (ascending component
//                  order), NaN on padding rows
//   ppos[p]        sorted position of the row (exact FP32 re-rank from the
//                  planes), 0xFFFFFFFF on padding rows
//   prow[p]        original row at padded position p, 0xFFFFFFFF on padding
//                  rows (the screen orders equal d~ by original row)
//   ipos[r]        padded position of original row r (inverse of prow)
//   ne_id[c]       rank of cone c among the non-empty cones; ne_cone is its inverse
#include "osann_device.h"
#include "osann_kernels.h"

namespace osann {

__global__ void binom_table_kernel(uint32_t* __restrict__ tab) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 256 * 8) return;
    const int n = i / 8, k = i % 8;
    const uint64_t c = binom_dev(n, k);
    tab[i] = c > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)c;
}

hipError_t launch_binom_table(uint32_t* tab, hipStream_t s) {
    hipLaunchKernelGGL(binom_table_kernel, dim3(8), dim3(256), 0, s, tab);
    return hipGetLastError();
}

__global__ void lowp_sizes_kernel(const uint32_t* __restrict__ off, int64_t nc, uint32_t* __restrict__ psz,
                                  uint32_t* __restrict__ nef) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const uint32_t len = off[c + 1] - off[c];
    psz[c] = (len + 15u) & ~15u;
    nef[c] = len > 0;
}

__global__ void ne_cone_kernel(const uint32_t* __restrict__ off, int64_t nc, const uint32_t* __restrict__ ne_id,
                               uint32_t* __restrict__ ne_cone) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nc && off[c + 1] > off[c]) ne_cone[ne_id[c]] = (uint32_t)c;
}

// The same layout for up to 65,536 cones in one block and one launch:
// thread t takes a run of consecutive cones, sums their padded sizes and
// non-empty flags, the block scans the 1024 sums (wave scans, then the
// waves' totals), and each thread walks its run again writing the starts.
constexpr int kLayoutThreads = 1024;
constexpr int64_t kLayoutSmallMax = 65536;

__global__ __launch_bounds__(kLayoutThreads) void lowp_layout_small_kernel(const uint32_t* __restrict__ off,
                                                                           int64_t nc, uint32_t* __restrict__ poff,
                                                                           uint32_t* __restrict__ ne_id,
                                                                           uint32_t* __restrict__ ne_cone) {
    __shared__ uint32_t wsum_p[kLayoutThreads / 64], wsum_n[kLayoutThreads / 64];
    const int t = threadIdx.x, w = t / 64, l = t % 64;
    const int64_t per = (nc + kLayoutThreads - 1) / kLayoutThreads;
    const int64_t c0 = (int64_t)t * per, c1 = c0 + per < nc ? c0 + per : nc;
    // a thread's bucket lengths, 8 at a time, the 9 offsets of a batch
    // loaded together
    auto lengths = [&](int64_t c, uint32_t (&len)[8]) __attribute__((always_inline)) {
        uint32_t o[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) o[i] = c + i <= c1 ? off[c + i] : 0u;
#pragma unroll
        for (int i = 0; i < 8; ++i) len[i] = c + i < c1 ? o[i + 1] - o[i] : 0u;
    };
    uint32_t sp = 0, sn = 0;
    for (int64_t c = c0; c < c1; c += 8) {
        uint32_t len[8];
        lengths(c, len);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            sp += (len[i] + 15u) & ~15u;
            sn += len[i] > 0;
        }
    }
    // inclusive wave scans, then the waves' totals
    uint32_t ip = sp, in = sn;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t up = (uint32_t)__shfl_up((int)ip, d, 64), un = (uint32_t)__shfl_up((int)in, d, 64);
        if (l >= d) {
            ip += up;
            in += un;
        }
    }
    if (l == 63) {
        wsum_p[w] = ip;
        wsum_n[w] = in;
    }
    __syncthreads();
    uint32_t bp = 0, bn = 0, tp = 0, tn = 0;
    for (int a = 0; a < kLayoutThreads / 64; ++a) {
        if (a < w) {
            bp += wsum_p[a];
            bn += wsum_n[a];
        }
        tp += wsum_p[a];
        tn += wsum_n[a];
    }
    uint32_t rp = bp + ip - sp, rn = bn + in - sn;  // exclusive starts of this thread's run
    for (int64_t c = c0; c < c1; c += 8) {
        uint32_t len[8];
        lengths(c, len);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (c + i >= c1) break;
            poff[c + i] = rp;
            ne_id[c + i] = rn;
            if (len[i] > 0) ne_cone[rn] = (uint32_t)(c + i);
            rp += (len[i] + 15u) & ~15u;
            rn += len[i] > 0;
        }
    }
    if (t == 0) {
        poff[nc] = tp;
        ne_id[nc] = tn;
    }
}

hipError_t launch_lowp_layout(const uint32_t* offsets, int64_t n_cones, uint32_t* psz_tmp, uint32_t* nef_tmp,
                              uint32_t* scan_tmp, uint32_t* poff, uint32_t* ne_id, uint32_t* ne_cone,
                              hipStream_t s) {
    if (n_cones > 0 && n_cones <= kLayoutSmallMax) {
        hipLaunchKernelGGL(lowp_layout_small_kernel, dim3(1), dim3(kLayoutThreads), 0, s, offsets, n_cones, poff, ne_id,
                           ne_cone);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((n_cones + 255) / 256));
    hipLaunchKernelGGL(lowp_sizes_kernel, grid, dim3(256), 0, s, offsets, n_cones, psz_tmp, nef_tmp);
    hipError_t e = launch_exclusive_scan(psz_tmp, n_cones, poff, scan_tmp, s);
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan(nef_tmp, n_cones, ne_id, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ne_cone_kernel, grid, dim3(256), 0, s, offsets, n_cones, ne_id, ne_cone);
    return hipGetLastError();
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// The padding rows of the copy (the slots past a cone's rows up to its
// multiple of 16, and every row from the last cone's end to np_total): zero
// components, no position, NaN norm.  Thread g < 16 nc takes slot g % 16 of
// cone g / 16; the others take the tail, which starts at or after N.
__global__ void lowp_pad_kernel(const uint32_t* __restrict__ off, const uint32_t* __restrict__ poff, int64_t nc,
                                int dk, uint16_t* __restrict__ xl, uint32_t* __restrict__ ppos,
                                uint32_t* __restrict__ prow, float* __restrict__ nrm, int64_t np_total) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t p = -1;
    if (g < 16 * nc) {
        const int64_t c = g / 16;
        const int64_t q = (int64_t)poff[c] + (int64_t)(off[c + 1] - off[c]) + g % 16;
        if (q < (int64_t)poff[c + 1]) p = q;
    } else {
        const int64_t q = (int64_t)poff[nc] + (g - 16 * nc);
        if (q < np_total) p = q;
    }
    if (p < 0) return;
    uint4* xr = reinterpret_cast<uint4*>(xl + p * dk);
    for (int k = 0; k < dk / 8; ++k) xr[k] = make_uint4(0u, 0u, 0u, 0u);
    ppos[p] = 0xFFFFFFFFu;
    prow[p] = 0xFFFFFFFFu;
    nrm[p] = __uint_as_float(0x7FC00000u);
}

// Rounded value of one component and its 16-bit code.
__device__ inline uint16_t lowp_code(float x, int to_f16, float* v) {
    const uint16_t b = to_f16 ? f16_rne(x) : bf16_rne(x);
    *v = to_f16 ? F16::val(b) : __uint_as_float((uint32_t)b << 16);
    return b;
}

// One thread per sorted position (coalesced reads of the chunk-major
// planes): rounds the row into an LDS tile of the block's 256 rows and
// stores the FP32 sum of squares of the rounded values taken in ascending
// component order, and the position map; then the block writes the tile's
// rows to their padded positions with consecutive lanes on consecutive
// 16-byte units (rows of a cone are consecutive there).  The tile's row
// stride is dk/2 + 1 words, so the lanes of the first phase, one row each,
// hit different banks.
template <typename E>
__global__ __launch_bounds__(256) void lowp_rows_kernel(const uint4* __restrict__ planes, int64_t N, int D, int nch,
                                                        const uint32_t* __restrict__ sorted_cone,
                                                        const uint32_t* __restrict__ off,
                                                        const uint32_t* __restrict__ poff,
                                                        const uint32_t* __restrict__ perm, int dk, int to_f16,
                                                        uint16_t* __restrict__ xl, uint32_t* __restrict__ ppos,
                                                        uint32_t* __restrict__ prow, uint32_t* __restrict__ ipos,
                                                        float* __restrict__ nrm) {
#pragma clang fp contract(off)
    constexpr int EPC = Unpack<E>::n;             // components per 16-byte chunk of the planes
    constexpr int CPU = (EPC >= 8 ? 1 : 8 / EPC) * 4;  // chunks per step (32 or 64 components, loaded together)
    constexpr int NU = CPU * EPC / 8;             // output units per step
    extern __shared__ uint32_t tile[];            // [256][dk/2 + 1]
    __shared__ int64_t s_p[256];
    const int words = dk / 2, stride = words + 1;
    const int64_t pos0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t pos = pos0 + threadIdx.x;
    uint32_t* row = tile + threadIdx.x * stride;
    if (pos < N) {
        const uint32_t c = sorted_cone[pos];
        const int64_t p = (int64_t)poff[c] + (pos - (int64_t)off[c]);
        s_p[threadIdx.x] = p;
        for (int wd = nch * EPC / 2; wd < words; ++wd) row[wd] = 0u;  // columns past the planes' chunks
        float acc = 0.0f;
        for (int k0 = 0; k0 < nch; k0 += CPU) {
            float x[CPU * EPC];
#pragma unroll
            for (int j = 0; j < CPU; ++j) {
                float t[EPC];
                if (k0 + j < nch) {
                    Unpack<E>::run(planes[(int64_t)(k0 + j) * N + pos], t);
                } else {
#pragma unroll
                    for (int e = 0; e < EPC; ++e) t[e] = 0.0f;
                }
#pragma unroll
                for (int e = 0; e < EPC; ++e) x[j * EPC + e] = t[e];
            }
#pragma unroll
            for (int u = 0; u < NU; ++u) {
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    uint16_t code[2];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int e = u * 8 + 2 * h + q;
                        const int i = k0 * EPC + e;
                        code[q] = 0;
                        if (i < D) {
                            float v;
                            code[q] = lowp_code(x[e], to_f16, &v);
                            const float sq = v * v;
                            acc = acc + sq;
                        }
                    }
                    const int wd = (k0 * EPC) / 2 + u * 4 + h;
                    if (wd < words) row[wd] = (uint32_t)code[0] | ((uint32_t)code[1] << 16);
                }
            }
        }
        const uint32_t r = perm[pos];
        ppos[p] = (uint32_t)pos;
        prow[p] = r;
        ipos[r] = (uint32_t)p;
        nrm[p] = acc;
    } else {
        s_p[threadIdx.x] = -1;
    }
    __syncthreads();
    // 16-byte stores: dk is a multiple of 32, so a row is a whole number of
    // 16-byte units and every row starts on one
    uint4* xq = reinterpret_cast<uint4*>(xl);
    const int quads = words / 4;
    for (int f = threadIdx.x; f < 256 * quads; f += 256) {
        const int r = f / quads, qd = f - r * quads;
        const int64_t p = s_p[r];
        if (p >= 0) {
            const uint32_t* t = tile + r * stride + 4 * qd;
            xq[p * quads + qd] = make_uint4(t[0], t[1], t[2], t[3]);
        }
    }
}

hipError_t launch_lowp_rows(const void* planes, int dtype, int64_t N, int D, int nch, const uint32_t* sorted_cone,
                            const uint32_t* offsets, int64_t n_cones, const uint32_t* poff, const uint32_t* perm,
                            int dk, int to_f16, uint16_t* xl, uint32_t* ppos, uint32_t* prow, uint32_t* ipos,
                            float* nrm, int64_t np_total, hipStream_t s) {
    // padding rows: zero components, no position, NaN norm (fails every
    // comparison); the real rows are written whole below
    hipError_t e = hipSuccess;
    if (16 * n_cones <= np_total) {
        const int64_t threads = 16 * n_cones + (np_total - N);
        hipLaunchKernelGGL(lowp_pad_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, offsets, poff,
                           n_cones, dk, xl, ppos, prow, nrm, np_total);
        e = hipGetLastError();
    } else {
        e = launch_fill_u32(reinterpret_cast<uint32_t*>(xl), np_total * dk / 2, 0u, s);
        if (e == hipSuccess) e = launch_fill_u32(ppos, np_total, 0xFFFFFFFFu, s);
        if (e == hipSuccess) e = launch_fill_u32(prow, np_total, 0xFFFFFFFFu, s);
        if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t*>(nrm), np_total, 0x7FC00000u, s);
    }
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)((N + 255) / 256));
    auto pl = static_cast<const uint4*>(planes);
    const size_t lds = (size_t)256 * (dk / 2 + 1) * 4;
    if (dk % 32 != 0 || dk < nch * chunk_elems(dtype) || lds > 150 * 1024) return hipErrorInvalidValue;
    switch (dtype) {
        case kF32:
            e = hipFuncSetAttribute((const void*)lowp_rows_kernel<F32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(lowp_rows_kernel<F32>, grid, dim3(256), lds, s, pl, N, D, nch, sorted_cone, offsets,
                               poff, perm, dk, to_f16, xl, ppos, prow, ipos, nrm);
            break;
        case kF16:
            e = hipFuncSetAttribute((const void*)lowp_rows_kernel<F16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(lowp_rows_kernel<F16>, grid, dim3(256), lds, s, pl, N, D, nch, sorted_cone, offsets,
                               poff, perm, dk, to_f16, xl, ppos, prow, ipos, nrm);
            break;
        case kU8:
            e = hipFuncSetAttribute((const void*)lowp_rows_kernel<U8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(lowp_rows_kernel<U8>, grid, dim3(256), lds, s, pl, N, D, nch, sorted_cone, offsets,
                               poff, perm, dk, to_f16, xl, ppos, prow, ipos, nrm);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace osann
