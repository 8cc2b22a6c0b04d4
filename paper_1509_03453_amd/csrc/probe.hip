// Query classification and probe list (Section 2 hashing of the query;
// Section 3.B order of cones; Algorithm 1 with one basis).
//
// One wave64 per query.  The wave ranks the query's components by decreasing
// magnitude (all-pairs integer compares of packed keys, ties to the lower
// index), derives the query's own cone, then walks the probe sequence 64
// positions at a time:
//   position j -> (number of flipped signs h, lexicographic L-subset T of
//   rank positions, flip mask) -> profile {order[t] : t in T} with the
//   query's signs, flipped by the mask -> cone -> bucket size.
// A wave prefix sum of the bucket sizes finds the first position at which
// the running candidate count reaches the budget.  The kernel stores the
// query's order, sign bits and that walk length; the scans regenerate the
// probed cones from them, so the probe list costs O(D) bytes per query.
#include "osann_device.h"
#include "osann_kernels.h"

namespace osann {

constexpr int kProbeWaves = 4;

// Long walks read the walk's tables from LDS: the binomial rows it uses (0
// .. max(D - 1, L)), the flip-mask order and, where it takes at most 16 KB,
// the lexicographic L-subsets.  A walk is long when a query is expected to
// take at least 256 positions (budget x cones / rows: the walk passes empty
// cones too); a block of short walks would spend more copying the tables than
// reading them.  Dynamic LDS layout: the probe bitmaps of the block's waves
// (when kept), then those tables.
__host__ __device__ inline int probe_binom_rows(int D, int L) { return D > L + 1 ? D : L + 1; }
__host__ __device__ inline bool probe_lex_in_lds(int64_t n_sub, int L) { return n_sub * L <= 16384; }
__host__ __device__ inline bool probe_tables_in_lds(const ProbeArgs& a) {
    return (a.jstop || a.ncand || a.nprobe) && a.budget < a.N && a.budget * a.n_cones >= 256 * a.N;
}
__host__ __device__ inline int64_t probe_qb_bytes(const ProbeArgs& a) {
    return a.qbits ? (int64_t)kProbeWaves * a.nw * 8 : 0;
}

template <typename E, int L>
__global__ __launch_bounds__(64 * kProbeWaves) void probe_kernel(ProbeArgs a) {
    extern __shared__ __align__(16) unsigned char probe_lds[];
    unsigned long long* qb_all = reinterpret_cast<unsigned long long*>(probe_lds);  // [kProbeWaves][nw] when a.qbits
    uint32_t* s_binom = reinterpret_cast<uint32_t*>(probe_lds + probe_qb_bytes(a));
    uint8_t* s_mask = reinterpret_cast<uint8_t*>(s_binom + probe_binom_rows(a.D, L) * 8);
    uint8_t* s_lex = s_mask + 128;
    __shared__ uint64_t keys[kProbeWaves][kMaxD];
    __shared__ uint8_t order[kProbeWaves][kMaxD];
    __shared__ uint8_t sbit[kProbeWaves][kMaxD];
    const int w = threadIdx.x / 64, l = lane_id();
    const int64_t q = (int64_t)blockIdx.x * kProbeWaves + w;
    const bool qv = q < a.Q;
    const int D = a.D;
    auto Y = static_cast<const typename E::raw*>(a.Y);
    // the same for every thread of the launch: whether the tables are copied
    const bool tab = probe_tables_in_lds(a);
    const bool lex_lds = tab && probe_lex_in_lds(a.n_sub, L);
    if (tab) {
        for (int i = threadIdx.x; i < probe_binom_rows(D, L) * 8; i += blockDim.x) s_binom[i] = a.binom[i];
        for (int i = threadIdx.x; i < 128; i += blockDim.x) s_mask[i] = a.maskord[i];
        if (lex_lds)
            for (int64_t i = threadIdx.x; i < a.n_sub * L; i += blockDim.x) s_lex[i] = a.lexsub[i];
    }

    // 1. load the query, keep FP32 and low-precision copies, stage the keys
    uint64_t mine[kMaxD / 64];
#pragma unroll
    for (int m = 0; m < kMaxD / 64; ++m) {
        const int i = l + 64 * m;
        uint64_t k = 0;
        if (qv && i < D) {
            const typename E::raw b = Y[q * D + i];
            k = comp_key(E::mag(b), i, E::neg(b));
            const float v = E::val(b);
            if (a.yf) a.yf[q * a.dpad + i] = v;
            if (a.ql) a.ql[q * a.dk + i] = a.ql_f16 ? f16_rne(v) : bf16_rne(v);
            keys[w][i] = k;
        } else if (qv) {
            if (a.yf && i < a.dpad) a.yf[q * a.dpad + i] = 0.0f;
            if (a.ql && i < a.dk) a.ql[q * a.dk + i] = 0;
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

    // 3. walk state, own cone and packed top-L pairs
    for (int i = l; i < D; i += 64) {
        if (a.order) a.order[q * D + i] = order[w][i];
        if (a.sbit) a.sbit[q * D + i] = sbit[w][i];
    }
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
    if (!a.jstop && !a.ncand && !a.nprobe) return;

    // 4. a budget of at least N takes every cone
    if (a.budget >= a.N) {
        if (l == 0) {
            if (a.jstop) a.jstop[q] = kWalkAll;
            if (a.nprobe) a.nprobe[q] = 0xFFFFFFFFu;
            if (a.ncand) a.ncand[q] = a.N;
        }
        if (a.qbits)
            for (int64_t k = l; k < a.nw; k += 64) {
                const int64_t rem = a.n_ne - 64 * k;
                a.qbits[q * a.nw + k] = rem >= 64 ? ~0ull : ((1ull << rem) - 1);
            }
        return;
    }
    unsigned long long* qb = qb_all + (int64_t)w * a.nw;
    if (a.qbits) {
        for (int64_t k = l; k < a.nw; k += 64) qb[k] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }

    // 5. walk the probe sequence 64 positions at a time until the budget is
    // met; in a long walk two steps' cones are generated and their bucket
    // bounds (and non-empty ids) loaded before either is scanned, so their
    // loads are in flight together
    const uint64_t budget = (uint64_t)a.budget;
    const uint32_t* offs = a.offsets + (a.cone_base ? a.cone_base[q] : 0u);  // this query's buckets
    uint64_t carry = 0;
    uint32_t np = 0, stop_at = 0;
    // one step at j0: false once the budget is met
    auto step = [&](int64_t j0, uint32_t len, uint32_t e) __attribute__((always_inline)) {
        const int64_t j = j0 + l;
        const uint32_t incl = wave_incl_scan(len);
        const uint64_t tot = carry + incl;
        const uint64_t reached = __ballot(j < a.n_cones && tot >= budget);
        const int stop = reached ? __ffsll((unsigned long long)reached) - 1 : 63;
        const bool taken = j < a.n_cones && l <= stop && len > 0;
        const uint64_t tm = __ballot(taken);
        if (a.qbits && taken) atomicOr(&qb[e >> 6], 1ull << (e & 63));
        np += (uint32_t)__popcll(tm);
        carry += shfl_u32(incl, stop);
        if (reached) {
            stop_at = (uint32_t)(j0 + stop + 1);
            return false;
        }
        stop_at = (uint32_t)(j0 + 64 < a.n_cones ? j0 + 64 : a.n_cones);
        return true;
    };
    // a short walk takes one step at a time (it mostly ends in its first)
    for (int64_t j0 = 0; !tab && j0 < a.n_cones; j0 += 64) {
        const int64_t ja = j0 + l;
        uint32_t ca = 0, lena = 0, ea = 0;
        if (ja < a.n_cones) {
            ca = probe_cone(ja, L, order[w], sbit[w], a.n_sub, a.lexsub, a.maskord, a.binom);
            lena = offs[ca + 1] - offs[ca];
            if (a.qbits) ea = a.ne_id[ca];
        }
        if (!step(j0, lena, ea)) break;
    }
    for (int64_t j0 = 0; tab && j0 < a.n_cones; j0 += 128) {
        const int64_t ja = j0 + l, jb = j0 + 64 + l;
        uint32_t ca = 0, cb = 0, lena = 0, lenb = 0, ea = 0, eb = 0;
        const uint8_t* lex = lex_lds ? s_lex : a.lexsub;
        const uint8_t* mask = tab ? s_mask : a.maskord;
        const uint32_t* bin = tab ? s_binom : a.binom;
        if (ja < a.n_cones) ca = probe_cone(ja, L, order[w], sbit[w], a.n_sub, lex, mask, bin);
        if (jb < a.n_cones) cb = probe_cone(jb, L, order[w], sbit[w], a.n_sub, lex, mask, bin);
        if (ja < a.n_cones) {
            lena = offs[ca + 1] - offs[ca];
            if (a.qbits) ea = a.ne_id[ca];
        }
        if (jb < a.n_cones) {
            lenb = offs[cb + 1] - offs[cb];
            if (a.qbits) eb = a.ne_id[cb];
        }
        if (!step(j0, lena, ea)) break;
        if (j0 + 64 >= a.n_cones || !step(j0 + 64, lenb, eb)) break;
    }
    if (l == 0) {
        if (a.jstop) a.jstop[q] = stop_at;
        if (a.nprobe) a.nprobe[q] = np;
        if (a.ncand) a.ncand[q] = (int64_t)carry;
    }
    if (a.qbits) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        for (int64_t k = l; k < a.nw; k += 64) a.qbits[q * a.nw + k] = qb[k];
    }
}

template <typename E>
static hipError_t dispatch_probe(const ProbeArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((a.Q + kProbeWaves - 1) / kProbeWaves)), block(64 * kProbeWaves);
    const size_t lds = (size_t)probe_qb_bytes(a) +
                       (probe_tables_in_lds(a) ? (size_t)probe_binom_rows(a.D, a.L) * 8 * 4 + 128 +
                                                     (probe_lex_in_lds(a.n_sub, a.L) ? (size_t)(a.n_sub * a.L) : 0)
                                               : 0);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    switch (a.L) {
#define OSANN_PROBE_CASE(LL)                                                  \
    case LL:                                                                  \
        hipLaunchKernelGGL((probe_kernel<E, LL>), grid, block, lds, s, a);    \
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
