// Query classification and probe list (Section 2 hashing of the query;
// Section 3.B order of cones; Algorithm 1 with one basis).
//
// One wave64 per query.  The wave ranks the query's components by decreasing
// magnitude (all-pairs integer compares of packed keys, ties to the lower
// index), derives the query's own cone, then walks the probe sequence 64
// entries at a time:
//   probe j -> (number of flipped signs h, lexicographic L-subset T of rank
//   positions, flip mask) -> profile {order[t] : t in T} with the query's
//   signs, flipped by the mask -> cone -> bucket (start, size).
// A wave prefix sum of the bucket sizes finds the first probe at which the
// running candidate count reaches the budget; the non-empty probes up to it
// are compacted with a ballot and written as (start, cumulative count).
#include "osann_device.h"
#include "osann_kernels.h"

namespace osann {

constexpr int kProbeWaves = 4;

template <typename E, int L>
__global__ __launch_bounds__(64 * kProbeWaves) void probe_kernel(ProbeArgs a) {
    __shared__ uint64_t keys[kProbeWaves][kMaxD];
    __shared__ uint8_t order[kProbeWaves][kMaxD];
    __shared__ uint8_t sbit[kProbeWaves][kMaxD];
    const int w = threadIdx.x / 64, l = lane_id();
    const int64_t q = (int64_t)blockIdx.x * kProbeWaves + w;
    const bool qv = q < a.Q;
    const int D = a.D;
    auto Y = static_cast<const typename E::raw*>(a.Y);

    // 1. load the query, keep an FP32 copy, stage the component keys
    uint64_t mine[kMaxD / 64];
#pragma unroll
    for (int m = 0; m < kMaxD / 64; ++m) {
        const int i = l + 64 * m;
        uint64_t k = 0;
        if (qv && i < D) {
            const typename E::raw b = Y[q * D + i];
            k = comp_key(E::mag(b), i, E::neg(b));
            if (a.yf) a.yf[q * a.dpad + i] = E::val(b);
            keys[w][i] = k;
        } else if (qv && a.yf && i < a.dpad) {
            a.yf[q * a.dpad + i] = 0.0f;
        }
        mine[m] = k;
    }
    __syncthreads();

    // 2. rank = number of components with a larger key
#pragma unroll
    for (int m = 0; m < kMaxD / 64; ++m) {
        const int i = l + 64 * m;
        if (qv && i < D) {
            int rank = 0;
            for (int j = 0; j < D; ++j) rank += keys[w][j] > mine[m];
            order[w][rank] = (uint8_t)i;
            sbit[w][i] = (uint8_t)key_sign(mine[m]);
        }
    }
    __syncthreads();
    if (!qv) return;  // no barrier below this point

    // 3. own cone and packed top-L pairs
    if (l == 0) {
        int idx[L], sg[L];
        uint64_t packed = 0;
#pragma unroll
        for (int j = 0; j < L; ++j) {
            idx[j] = order[w][j];
            sg[j] = sbit[w][idx[j]];
            packed |= (uint64_t)((uint32_t)idx[j] | ((uint32_t)sg[j] << 8)) << (9 * j);
        }
        if (a.q_top) a.q_top[q] = packed;
        const uint32_t own = cone_of<L>(idx, sg);
        if (a.q_cone) a.q_cone[q] = own;
    }
    if (!a.desc && !a.ncand && !a.nprobe) return;

    // 4. a budget of at least N takes every cone: one descriptor for all rows
    if (a.budget >= a.N) {
        if (l == 0) {
            if (a.desc) a.desc[q * a.cap] = make_uint2(0u, (uint32_t)a.N);
            if (a.nprobe) a.nprobe[q] = 1;
            if (a.ncand) a.ncand[q] = a.N;
        }
        return;
    }

    // 5. walk the probe sequence until the budget is met
    const uint64_t budget = (uint64_t)a.budget;
    uint64_t carry = 0;
    uint32_t np = 0;
    for (int64_t j0 = 0; j0 < a.n_cones; j0 += 64) {
        const int64_t j = j0 + l;
        uint32_t start = 0, len = 0;
        if (j < a.n_cones) {
            // block h of the sequence holds C(D,L)*C(L,h) probes with h flips
            int64_t base = 0;
            int h = 0, mstart = 0;
            uint64_t cl = 1;
            for (; h <= L; ++h) {
                cl = binom_dev(L, h);
                const int64_t sz = a.n_sub * (int64_t)cl;
                if (j < base + sz) break;
                base += sz;
                mstart += (int)cl;
            }
            const int64_t jj = j - base;
            const int64_t t = jj / (int64_t)cl;
            const int mask = a.maskord[mstart + (int)(jj % (int64_t)cl)];
            int idx[L], sg[L];
#pragma unroll
            for (int b = 0; b < L; ++b) {
                idx[b] = order[w][a.lexsub[t * L + b]];
                sg[b] = sbit[w][idx[b]] ^ ((mask >> (L - 1 - b)) & 1);
            }
            const uint32_t c = cone_of<L>(idx, sg);
            start = a.offsets[c];
            len = a.offsets[c + 1] - start;
        }
        const uint32_t incl = wave_incl_scan(len);
        const uint64_t tot = carry + incl;
        const uint64_t reached = __ballot(j < a.n_cones && tot >= budget);
        const int stop = reached ? __ffsll((unsigned long long)reached) - 1 : 63;
        const bool take = j < a.n_cones && l <= stop && len > 0;
        const uint64_t tm = __ballot(take);
        const uint32_t slot = np + (uint32_t)__popcll(tm & lanemask_lt());
        if (take && a.desc && slot < a.cap) a.desc[q * a.cap + slot] = make_uint2(start, (uint32_t)tot);
        np += (uint32_t)__popcll(tm);
        carry += shfl_u32(incl, stop);
        if (reached) break;
    }
    if (l == 0) {
        if (a.nprobe) a.nprobe[q] = np;
        if (a.ncand) a.ncand[q] = (int64_t)carry;
    }
}

template <typename E>
static hipError_t dispatch_probe(const ProbeArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((a.Q + kProbeWaves - 1) / kProbeWaves)), block(64 * kProbeWaves);
    switch (a.L) {
#define OSANN_PROBE_CASE(LL)                                                  \
    case LL:                                                                  \
        hipLaunchKernelGGL((probe_kernel<E, LL>), grid, block, 0, s, a);      \
        break;
        OSANN_PROBE_CASE(1) OSANN_PROBE_CASE(2) OSANN_PROBE_CASE(3) OSANN_PROBE_CASE(4)
        OSANN_PROBE_CASE(5) OSANN_PROBE_CASE(6) OSANN_PROBE_CASE(7)
#undef OSANN_PROBE_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_probe(const ProbeArgs& a, hipStream_t s) {
    if (a.Q <= 0) return hipSuccess;
    switch (a.qtype) {
        case kF32: return dispatch_probe<F32>(a, s);
        case kF16: return dispatch_probe<F16>(a, s);
        case kU8: return dispatch_probe<U8>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace osann
