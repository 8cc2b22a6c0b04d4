// Fixed-C walk lengths (Section 3, Table III).  One wave64 per walk: the
// walk state (the components by decreasing magnitude and their signs) comes
// from the probe kernel; the wave regenerates walk positions 0..C-1, 64 at a
// time, and counts the non-empty cones and the rows they hold (optionally
// also marking them in a per-walk bitmap over the non-empty cones, built in
// LDS).  The scans then take exactly the first min(C, N_C) positions.
#include "osann_device.h"
#include "osann_fixedc.h"
#include "osann_kernels.h"

namespace osann {

constexpr int kConesWaves = 4;

__global__ __launch_bounds__(64 * kConesWaves) void cones_kernel(ConesArgs a) {
    extern __shared__ unsigned long long cb_all[];  // [kConesWaves][nw] when a.qbits
    __shared__ uint8_t order[kConesWaves][kMaxD];
    __shared__ uint8_t sbit[kConesWaves][kMaxD];
    const int w = threadIdx.x / 64, l = lane_id();
    const int64_t q = (int64_t)blockIdx.x * kConesWaves + w;
    if (q >= a.Q) return;  // no block barrier in this kernel
    const int D = a.D;
    for (int i = l; i < D; i += 64) {
        order[w][i] = a.order[q * D + i];
        sbit[w][i] = a.sbit[q * D + i];
    }
    unsigned long long* qb = cb_all + (int64_t)w * a.nw;
    if (a.qbits)
        for (int64_t k = l; k < a.nw; k += 64) qb[k] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

    const int64_t stop = a.take < a.n_cones ? a.take : a.n_cones;
    const uint32_t* offs = a.offsets + (a.cone_base ? a.cone_base[q] : 0u);
    uint64_t rows = 0;
    uint32_t np = 0;
    for (int64_t j0 = 0; j0 < stop; j0 += 64) {
        const int64_t j = j0 + l;
        uint32_t len = 0;
        if (j < stop) {
            const uint32_t c = probe_cone(j, a.L, order[w], sbit[w], a.n_sub, a.lexsub, a.maskord, a.binom);
            len = offs[c + 1] - offs[c];
            if (a.qbits && len > 0) {
                const uint32_t e = a.ne_id[c];
                atomicOr(&qb[e >> 6], 1ull << (e & 63));
            }
        }
        // distinct cones of one walk: 64 of them hold at most every row
        rows += shfl_u32(wave_incl_scan(len), 63);
        np += (uint32_t)__popcll(__ballot(len > 0));
    }
    if (l == 0) {
        if (a.jstop) a.jstop[q] = (uint32_t)stop;
        if (a.nprobe) a.nprobe[q] = np;
        if (a.ncand) a.ncand[q] = (int64_t)rows;
    }
    if (a.qbits) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        for (int64_t k = l; k < a.nw; k += 64) a.qbits[q * a.nw + k] = qb[k];
    }
}

hipError_t launch_cones(const ConesArgs& a, hipStream_t s) {
    if (a.Q <= 0) return hipSuccess;
    if (a.D < 1 || a.D > kMaxD || a.take < 1 || !a.order || !a.sbit) return hipErrorInvalidValue;
    if (a.qbits && (a.nw < 1 || a.nw > 512 || !a.ne_id)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.Q + kConesWaves - 1) / kConesWaves)), block(64 * kConesWaves);
    const size_t lds = a.qbits ? (size_t)kConesWaves * a.nw * 8 : 0;
    hipLaunchKernelGGL(cones_kernel, grid, block, lds, s, a);
    return hipGetLastError();
}

}  // namespace osann
