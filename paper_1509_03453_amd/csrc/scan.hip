// FP32 candidate scan with running arg-min (eq. (1); Algorithm 1, the
// short-list search that Section 3.D names as the critical cost).
//
// One to four waves per query.  The query sits in LDS (FP32, zero padded to
// whole 16-byte chunks).  Lane f of the query's waves takes candidates f,
// f + 64*w, ... of the query's flattened candidate list; a per-lane cursor
// over the probe descriptors turns the flat index into a sorted position.
// Each lane then reads its row chunk by chunk from the chunk-major planes:
// for a fixed chunk, 64 lanes on consecutive positions read 1 KiB of
// contiguous memory, and each lane accumulates its own row's squared
// distance in ascending component order with separately rounded
// subtract/multiply/add, which makes the result bit-identical to the plain
// definition evaluated term by term.  The arg-min is over (distance,
// original row), so the visiting order never changes the result; the
// original row id is fetched only when a lane's best improves or ties.
#include "osann_device.h"
#include "osann_kernels.h"

namespace osann {

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

template <typename E, int NCH>
__global__ __launch_bounds__(256) void scan_fp32_kernel(ScanArgs a) {
#pragma clang fp contract(off)
    constexpr int EPC = Unpack<E>::n;
    __shared__ float ys[4][kMaxD];
    __shared__ float red_d[4];
    __shared__ uint32_t red_r[4];
    const int nch = NCH ? NCH : a.nch;
    const int wpq = a.waves_per_query;
    const int qpb = 4 / wpq;
    const int w = threadIdx.x / 64, l = lane_id();
    const int slot = w / wpq, sub = w % wpq;
    const int64_t q = (int64_t)blockIdx.x * qpb + slot;
    const bool qv = q < a.Q;
    const int dp = nch * EPC;

    for (int i = sub * 64 + l; i < dp; i += wpq * 64) ys[slot][i] = qv ? a.yf[q * dp + i] : 0.0f;
    __syncthreads();

    float best = __builtin_huge_valf();
    uint32_t brow = 0xFFFFFFFFu;
    if (qv) {
        const uint2* dq = a.desc + q * a.cap;
        const uint32_t np = a.nprobe[q];
        const uint32_t total = np ? dq[np - 1].y : 0u;
        const uint4* planes = static_cast<const uint4*>(a.planes);
        const float* y = ys[slot];
        uint32_t k = 0, prev = 0;
        uint2 cur = np ? dq[0] : make_uint2(0u, 0u);
        for (uint32_t f = sub * 64 + l; f < total; f += wpq * 64) {
            while (cur.y <= f) {
                prev = cur.y;
                cur = dq[++k];
            }
            const int64_t pos = (int64_t)cur.x + (f - prev);
            float acc = 0.0f;
            if (NCH) {
                uint4 v[NCH ? NCH : 1];
#pragma unroll
                for (int c = 0; c < NCH; ++c) v[c] = planes[(int64_t)c * a.N + pos];
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    float x[EPC];
                    Unpack<E>::run(v[c], x);
#pragma unroll
                    for (int e = 0; e < EPC; ++e) {
                        const float d = x[e] - y[c * EPC + e];
                        const float sq = d * d;
                        acc = acc + sq;
                    }
                }
            } else {
                for (int c = 0; c < nch; ++c) {
                    float x[EPC];
                    Unpack<E>::run(planes[(int64_t)c * a.N + pos], x);
#pragma unroll
                    for (int e = 0; e < EPC; ++e) {
                        const float d = x[e] - y[c * EPC + e];
                        const float sq = d * d;
                        acc = acc + sq;
                    }
                }
            }
            if (acc < best) {
                best = acc;
                brow = a.perm[pos];
            } else if (acc == best) {
                const uint32_t r = a.perm[pos];
                brow = r < brow ? r : brow;
            }
        }
    }
    wave_argmin(best, brow);
    if (wpq > 1) {
        if (l == 0) {
            red_d[w] = best;
            red_r[w] = brow;
        }
        __syncthreads();
        if (sub == 0 && l == 0) {
            for (int o = 1; o < wpq; ++o) {
                const float od = red_d[w + o];
                const uint32_t orow = red_r[w + o];
                if (od < best || (od == best && orow < brow)) {
                    best = od;
                    brow = orow;
                }
            }
        }
    }
    if (qv && sub == 0 && l == 0) {
        a.out_idx[q] = brow == 0xFFFFFFFFu ? -1 : (int64_t)brow;
        a.out_dist[q] = best;
    }
}

template <typename E>
static hipError_t dispatch_scan(const ScanArgs& a, hipStream_t s) {
    const int qpb = 4 / a.waves_per_query;
    const dim3 grid((unsigned)((a.Q + qpb - 1) / qpb)), block(256);
    switch (a.nch) {
#define OSANN_SCAN_CASE(C)                                                   \
    case C:                                                                  \
        hipLaunchKernelGGL((scan_fp32_kernel<E, C>), grid, block, 0, s, a);  \
        break;
        OSANN_SCAN_CASE(1) OSANN_SCAN_CASE(2) OSANN_SCAN_CASE(4) OSANN_SCAN_CASE(8)
        OSANN_SCAN_CASE(16)
#undef OSANN_SCAN_CASE
        default:
            hipLaunchKernelGGL((scan_fp32_kernel<E, 0>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_scan_fp32(const ScanArgs& a, hipStream_t s) {
    if (a.Q <= 0) return hipSuccess;
    if (a.waves_per_query != 1 && a.waves_per_query != 2 && a.waves_per_query != 4)
        return hipErrorInvalidValue;
    switch (a.dtype) {
        case kF32: return dispatch_scan<F32>(a, s);
        case kF16: return dispatch_scan<F16>(a, s);
        case kU8: return dispatch_scan<U8>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace osann
