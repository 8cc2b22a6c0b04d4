// FP32 candidate scan with running arg-min (eq. (1); Algorithm 1, the
// short-list search that Section 3.D names as the critical cost).
//
// One to four waves per query.  The query sits in LDS (FP32, zero padded to
// whole 16-byte chunks) with its walk state.  Each wave regenerates the
// query's probed cones 64 walk positions at a time (probe_cone), keeps the
// buckets' starts and running candidate counts in LDS, and lane f of the
// query's waves takes candidates f, f + 64*w, ... of that chunk; a per-lane
// cursor over the running counts turns the flat index into a sorted position.
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

// Distance of the candidate at sorted position pos, then the running
// arg-min on (distance, original row).
template <typename E, int NCH>
__device__ inline void visit(const ScanArgs& a, const uint4* __restrict__ planes, const float* y, int64_t pos,
                             float& best, uint32_t& brow) {
#pragma clang fp contract(off)
    constexpr int EPC = Unpack<E>::n;
    float acc;
    if (NCH) {
        acc = 0.0f;
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
        acc = row_dist_fp32<E>(planes, a.N, a.nch, pos, y);
    }
    if (acc < best) {
        best = acc;
        brow = a.perm[pos];
    } else if (acc == best) {
        const uint32_t r = a.perm[pos];
        brow = r < brow ? r : brow;
    }
}

template <typename E, int NCH>
__global__ __launch_bounds__(256) void scan_fp32_kernel(ScanArgs a) {
    __shared__ float ys[4][kMaxD];
    __shared__ uint8_t s_order[4][kMaxD];
    __shared__ uint8_t s_sbit[4][kMaxD];
    __shared__ uint32_t s_start[4][64];
    __shared__ uint32_t s_incl[4][64];
    __shared__ float red_d[4];
    __shared__ uint32_t red_r[4];
    constexpr int EPC = Unpack<E>::n;
    const int nch = NCH ? NCH : a.nch;
    const int wpq = a.waves_per_query;
    const int qpb = 4 / wpq;
    const int w = threadIdx.x / 64, l = lane_id();
    const int slot = w / wpq, sub = w % wpq;
    const int64_t q = (int64_t)blockIdx.x * qpb + slot;
    const bool qv = q < a.Q;
    const int dp = nch * EPC;

    for (int i = sub * 64 + l; i < dp; i += wpq * 64) ys[slot][i] = qv ? a.yf[q * dp + i] : 0.0f;
    for (int i = sub * 64 + l; i < a.D; i += wpq * 64) {
        s_order[slot][i] = qv ? a.order[q * a.D + i] : 0;
        s_sbit[slot][i] = qv ? a.sbit[q * a.D + i] : 0;
    }
    __syncthreads();

    float best = __builtin_huge_valf();
    uint32_t brow = 0xFFFFFFFFu;
    const uint4* planes = static_cast<const uint4*>(a.planes);
    const float* y = ys[slot];
    const uint32_t jstop = qv ? a.jstop[q] : 0u;
    if (jstop == kWalkAll) {
        for (int64_t f = sub * 64 + l; f < a.N; f += wpq * 64) visit<E, NCH>(a, planes, y, f, best, brow);
    } else {
        uint32_t* st = s_start[w];
        uint32_t* in = s_incl[w];
        const uint32_t* offs = a.offsets + (qv && a.cone_base ? a.cone_base[q] : 0u);  // this query's buckets
        for (uint32_t j0 = 0; j0 < jstop; j0 += 64) {
            // this wave's copy of the chunk's bucket starts and running counts
            const uint32_t j = j0 + l;
            uint32_t start = 0, len = 0;
            if (j < jstop) {
                const uint32_t c = probe_cone(j, a.L, s_order[slot], s_sbit[slot], a.n_sub, a.lexsub, a.maskord, a.binom);
                start = offs[c];
                len = offs[c + 1] - start;
            }
            const uint32_t incl = wave_incl_scan(len);
            st[l] = start;
            in[l] = incl;
            const uint32_t total = shfl_u32(incl, 63);
            // make the wave's LDS writes visible to its other lanes
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            uint32_t k = 0;
            for (uint32_t f = sub * 64 + l; f < total; f += wpq * 64) {
                while (in[k] <= f) ++k;
                const uint32_t before = k ? in[k - 1] : 0u;
                visit<E, NCH>(a, planes, y, (int64_t)st[k] + (f - before), best, brow);
            }
            // every lane is done reading before the next chunk overwrites
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
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
