// Matrix-core screening of the candidates with an exact FP32 re-rank.
//
// Queries are sorted by their own cone and cut into tiles of 4 waves x 16G
// queries.  A work item is (tile, split): split s owns a contiguous range of
// the non-empty cones.  The block first marks, in an LDS table over that
// range, which of its queries probe each cone (from the probe pass's bitmaps,
// or by regenerating the walks of Section 3.B); then for every marked cone it
// streams the cone's rows through LDS in batches of up to 128 and screens
// them in 16-row MFMA tiles (bucket sizes are padded to 16 rows in the
// low-precision copy).  With the rows as the MFMA A operand and 16 queries
// as B, lane l holds the products of query l%16 with 4 rows, from which it
// forms d~ = ||x^||^2 - 2 q^.x^, which ranks candidates like the squared
// distance of the rounded vectors.
//
// Each query keeps, per split, a top-R list of (d~, padded position) in
// LDS.  The tile loop only compares d~ with a per-query bound; the few
// candidates at or below it go to a per-wave hit buffer, which is merged
// into the lists (one lane per query) when it fills and after every batch.
//
// Pruning: a candidate whose d~ exceeds an upper bound of the query's final
// R-th value can never be kept.  Two bounds are used: the R-th entry of the
// split's list of the query, and a bound shared by all splits: every kept
// candidate lowers the minimum of its class (padded position mod R) in a
// per-query array, and R distinct candidates lie at or below the largest
// class minimum, so that value bounds the R-th.  A pass before the screen
// seeds the class minima from the query's own cone.  Bounds only ever
// discard candidates outside the final top R, so the result is the same
// whatever the timing of the splits.
//
// A finishing pass merges the S split lists, recomputes the exact FP32
// distance of the R survivors and keeps the arg-min on (distance, row).
// Lists are kept in the total order (d~, position), so results do not
// depend on the batch or the split.
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

// Order-preserving map of a non-NaN float to 32 bits (and back); 0xFFFFFFFF
// (above every float) stands for "no candidate yet".
__device__ inline uint32_t ord_bits(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float ord_float(uint32_t u) {
    if (u == 0xFFFFFFFFu) return __builtin_huge_valf();
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

template <bool F16IN>
__device__ inline f32x4_t mfma16(const uint4& a, const uint4& b, f32x4_t acc) {
    if (F16IN)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, b),
                                                      acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                   acc, 0, 0, 0);
}

constexpr int kBatchRows = 128;  // rows staged in LDS per batch (8 MFMA row tiles)
constexpr int kHitCap = 64;      // hit buffer entries per wave (one full ballot)

// Exclusive prefix sum of one value per thread over the 256-thread block.
__device__ inline uint32_t block_scan256(uint32_t v, uint32_t* wsum, uint32_t* total) {
    const int w = threadIdx.x / 64, l = lane_id();
    const uint32_t incl = wave_incl_scan(v);
    if (l == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        before += k < w ? wsum[k] : 0u;
        all += wsum[k];
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// LDS slot (16-byte unit) of unit c of row r: XOR swizzle inside each row so
// that the 16 rows an MFMA A-fragment read touches fall in different banks.
template <int CPR>
__device__ inline int swz(int r, int c) {
    constexpr int M = CPR < 8 ? CPR - 1 : 7;
    return r * CPR + (c ^ (r & M));
}

// Marked cone of a split: padded rows [p0, p1) and, per wave, which of its
// queries probe the cone.
struct ListEntry {
    uint32_t p0, p1, pad0, pad1;
    uint64_t m[4];
};

template <bool F16IN, int KS, int R, int G>
__global__ __launch_bounds__(256, 2) void tiled_screen_kernel(TiledArgs a) {
    constexpr int QW = 16 * G;              // queries per wave
    constexpr int MQ = 4 * QW;              // queries per tile
    constexpr int CPR = KS * 4;             // 16-byte units per row (dk = 32*KS)
    constexpr int KU = kBatchRows * CPR / 256;  // units each thread stages per batch
    extern __shared__ uint64_t dyn[];
    // dyn: list[span] | scratch: first the cone table tab[span][4], then
    //      (once the list is built) rows[2][128*CPR] (uint4) and nrm[2][128]
    __shared__ uint8_t s_order[4][kMaxD];
    __shared__ uint8_t s_sbit[4][kMaxD];
    __shared__ uint32_t s_item, s_nlist, s_wsum[4];
    __shared__ uint2 s_list[4][QW * R];     // per wave: top-R list of each query slot
    __shared__ uint4 s_hit[4][kHitCap];     // per wave: (d~ bits, padded position, slot) hits
    const int w = threadIdx.x / 64, l = lane_id();
    const int64_t total = a.T * a.S;
    ListEntry* list = reinterpret_cast<ListEntry*>(dyn);
    uint64_t* tab = dyn + 6 * a.span;
    uint4* rows = reinterpret_cast<uint4*>(tab);
    float* nrmb = reinterpret_cast<float*>(rows + 2 * kBatchRows * CPR);
    // this thread's staging units: global element offset inside a batch and LDS slot
    int goff[KU], gslot[KU], grow[KU];
#pragma unroll
    for (int k = 0; k < KU; ++k) {
        const int u = threadIdx.x + 256 * k;
        grow[k] = u / CPR;
        goff[k] = grow[k] * a.dk + 8 * (u % CPR);
        gslot[k] = swz<CPR>(grow[k], u % CPR);
    }
    int aslot[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) aslot[ks] = swz<CPR>(l % 16, l / 16 + 4 * ks);
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1u);
        __syncthreads();
        const int64_t item = s_item;
        __syncthreads();
        if (item >= total) break;
        const int64_t t = item / a.S;
        const int s = (int)(item % a.S);
        const int64_t n0 = s * a.span;
        const int64_t n1 = n0 + a.span < a.n_ne ? n0 + a.span : a.n_ne;
        const int nspan = n1 > n0 ? (int)(n1 - n0) : 0;
        const int64_t wslot0 = t * MQ + (int64_t)w * QW;  // first tile slot of this wave

        // 1. per cone of the split: which of this wave's queries probe it
        if (a.qbits) {
            // transpose the queries' probed-cone bitmaps with ballots
            const bool mine = l < QW && wslot0 + l < a.Q;
            const uint32_t q = mine ? a.qorder[wslot0 + l] : 0u;
            for (int64_t k = n0 >> 6; k * 64 < n1; ++k) {
                const uint64_t word = mine ? a.qbits[(int64_t)q * a.nw + k] : 0ull;
                uint64_t col = 0;
#pragma unroll 8
                for (int c = 0; c < 64; ++c) {
                    const uint64_t m = __ballot((word >> c) & 1ull);
                    col = c == l ? m : col;
                }
                const int64_t e = k * 64 + l;
                if (e >= n0 && e < n1) tab[(e - n0) * 4 + w] = col;
            }
        } else {
            for (int i = l; i < nspan; i += 64) tab[i * 4 + w] = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            for (int c = 0; c < QW; ++c) {
                if (wslot0 + c >= a.Q) break;
                const uint32_t q = a.qorder[wslot0 + c];
                const uint32_t js = a.jstop[q];
                const unsigned long long bit = 1ull << c;
                if (js == kWalkAll) {
                    for (int i = l; i < nspan; i += 64) atomicOr((unsigned long long*)&tab[i * 4 + w], bit);
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
                            if (e >= n0 && e < n1) atomicOr((unsigned long long*)&tab[(e - n0) * 4 + w], bit);
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
        }
        __syncthreads();

        // 2. compact list of the cones some query of the tile probes
        if (threadIdx.x == 0) s_nlist = 0;
        __syncthreads();
        for (int base = 0; base < nspan; base += 256) {
            const int i = base + threadIdx.x;
            uint64_t m[4] = {0, 0, 0, 0};
            if (i < nspan)
#pragma unroll
                for (int k = 0; k < 4; ++k) m[k] = tab[i * 4 + k];
            const bool hit = (m[0] | m[1] | m[2] | m[3]) != 0;
            uint32_t cnt;
            const uint32_t at = block_scan256(hit ? 1u : 0u, s_wsum, &cnt);
            if (hit) {
                const uint32_t cone = a.ne_cone[n0 + i];
                ListEntry e;
                e.p0 = a.poff[cone];
                e.p1 = a.poff[cone + 1];
                e.pad0 = e.pad1 = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) e.m[k] = m[k];
                list[s_nlist + at] = e;
            }
            __syncthreads();
            if (threadIdx.x == 0) s_nlist += cnt;
            __syncthreads();
        }
        const int nlist = (int)s_nlist;  // the table is dead from here on: its space holds the row batches

        // 3. B operands: group g of this wave = query slots 16g .. 16g+15 of the
        //    wave; lane l works on slot 16g + l%16 of every group
        uint4 bq[G][KS];
        bool qok[G];
        uint32_t myq[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t slot = wslot0 + 16 * g + (l % 16);
            qok[g] = slot < a.Q;
            myq[g] = qok[g] ? a.qorder[slot] : 0u;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                bq[g][ks] = qok[g] ? *reinterpret_cast<const uint4*>(a.ql + (int64_t)myq[g] * a.dk + ks * 32 +
                                                                     8 * (l / 16))
                                   : make_uint4(0, 0, 0, 0);
        }
        // The split's top-R list of every query of the wave lives in LDS
        // (wlist[slot][k], ascending (d~, padded position)); lane l owns slot l
        // when lists are updated.  Candidates that pass the bound go to a hit
        // buffer first and are merged in bulk, which keeps the tile loop free
        // of list code.
        uint2* wl = s_list[w];
        for (int k = l; k < QW * R; k += 64) wl[k] = make_uint2(0x7F800000u, 0xFFFFFFFFu);
        uint32_t nhit = 0;
        // shared bound of slot l's query (owner view) and of slot 16g + l%16
        const uint32_t own_q = l < QW && wslot0 + l < a.Q ? a.qorder[wslot0 + l] : 0u;
        const bool own_ok = l < QW && wslot0 + l < a.Q;
        auto class_bound = [&](uint32_t q) {
            uint32_t c = 0;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const uint32_t v =
                    __hip_atomic_load(a.cmin + (int64_t)q * R + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                c = v > c ? v : c;
            }
            return c;
        };
        // thr[g]: no candidate of slot 16g + l%16 above it can enter the final
        // top R: the minimum of the slot's list R-th entry and the shared bound
        float thr[G];
        uint32_t ownb = own_ok ? class_bound(own_q) : 0xFFFFFFFFu;
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): operands and bounds landed
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        auto refresh_thr = [&]() {
            // owner lane l: bound of slot l; everyone: bound of its 4 slots
            const float ob = fminf(ord_float(ownb), __uint_as_float(wl[l % QW * R + R - 1].x));
#pragma unroll
            for (int g = 0; g < G; ++g) thr[g] = __shfl(ob, 16 * g + (l % 16), 64);
        };
        refresh_thr();
        // merge the hit buffer into the lists: lane l takes the hits of slot l
        auto flush = [&]() {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            float ld[R];
            uint32_t lr[R];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const uint2 e = wl[(l % QW) * R + k];
                ld[k] = __uint_as_float(e.x);
                lr[k] = e.y;
            }
            bool changed = false;
            for (uint32_t h = 0; h < nhit; ++h) {
                const uint4 e = s_hit[w][h];
                const float d = __uint_as_float(e.x);
                if (e.z == (uint32_t)l && pair_less(d, e.y, ld[R - 1], lr[R - 1])) {
                    list_insert<R>(ld, lr, d, e.y);
                    changed = true;
                    __hip_atomic_fetch_min(a.cmin + (int64_t)own_q * R + (e.y & (R - 1)), ord_bits(d),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            if (changed && l < QW)
#pragma unroll
                for (int k = 0; k < R; ++k) wl[l * R + k] = make_uint2(__float_as_uint(ld[k]), lr[k]);
            nhit = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            refresh_thr();
        };

        // 4. batches of up to 128 rows staged in LDS; the next batch is loaded
        //    into registers while the current one is on the matrix cores.
        uint4 stage[KU];
        float nst = 0.0f;
        auto issue = [&](uint32_t p, uint32_t n) {
            const uint16_t* src = a.xl + (int64_t)p * a.dk;
#pragma unroll
            for (int k = 0; k < KU; ++k)
                stage[k] = (uint32_t)grow[k] < n ? *reinterpret_cast<const uint4*>(src + goff[k])
                                                 : make_uint4(0, 0, 0, 0);
            nst = a.nrm[(int64_t)p + (threadIdx.x < n ? threadIdx.x : n - 1)];
        };
        auto park = [&](int buf) {
            uint4* dst = rows + buf * kBatchRows * CPR;
#pragma unroll
            for (int k = 0; k < KU; ++k) dst[gslot[k]] = stage[k];
            if (threadIdx.x < kBatchRows) nrmb[buf * kBatchRows + threadIdx.x] = nst;
        };
        int li = 0;          // list entry of the staged batch
        uint32_t bp = 0;     // its first padded row
        uint32_t bn = 0;     // its rows
        if (nlist > 0) {
            bp = list[0].p0;
            bn = list[0].p1 - bp < kBatchRows ? list[0].p1 - bp : kBatchRows;
            issue(bp, bn);
            park(0);
        }
        __syncthreads();
        int buf = 0;
        while (li < nlist) {
            // next batch: rest of this cone, else the next listed cone
            const uint32_t cur_p1 = list[li].p1;
            const uint64_t mk = list[li].m[w];
            int nli = li;
            uint32_t np = bp + bn, nn = 0;
            if (np >= cur_p1) {
                nli = li + 1;
                if (nli < nlist) np = list[nli].p0;
            }
            if (nli < nlist) {
                const uint32_t end = list[nli].p1;
                nn = end - np < kBatchRows ? end - np : kBatchRows;
                issue(np, nn);
            }
            // the shared class minima of slot l's query, read now and folded
            // into the bound after the batch.  Plain loads: a cached copy may
            // be stale, but every value ever stored there is a valid bound
            // (the words only decrease), and cached reads keep the batch
            // pipeline short.
            uint32_t cmv[R];
#pragma unroll
            for (int k = 0; k < R; ++k) cmv[k] = a.cmin[(int64_t)own_q * R + k];
            // screen the staged batch
            if (mk != 0) {
                const uint4* rb = rows + buf * kBatchRows * CPR;
                const float* nb = nrmb + buf * kBatchRows + 4 * (l / 16);
                float pthr[G];  // thr, or -inf for slots that do not probe this cone
                auto set_pthr = [&]() {
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const bool probed = (mk >> (16 * g + (l % 16))) & 1ull;
                        pthr[g] = probed ? thr[g] : -__builtin_huge_valf();
                    }
                };
                set_pthr();
                // software pipeline: tile r0's products are on the matrix
                // cores while tile r0-16's d~ are formed and compared, and
                // tile r0+16's fragments are read from LDS
                auto frag = [&](uint32_t r0, uint4 (&av)[KS], float4& nv4) {
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks) av[ks] = rb[aslot[ks] + r0 * CPR];
                    nv4 = *reinterpret_cast<const float4*>(nb + r0);
                };
                auto products = [&](const uint4 (&av)[KS], f32x4_t (&acc)[G]) {
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        acc[g] = mfma16<F16IN>(av[0], bq[g][0], f32x4_t{0.0f, 0.0f, 0.0f, 0.0f});
#pragma unroll
                        for (int ks = 1; ks < KS; ++ks) acc[g] = mfma16<F16IN>(av[ks], bq[g][ks], acc[g]);
                    }
                };
                uint4 av[KS];
                float4 nv4;
                f32x4_t acc[G];
                frag(0, av, nv4);
                products(av, acc);
                float4 nv_cur = nv4;
                for (uint32_t r0 = 0; r0 < bn; r0 += 16) {
                    const bool more = r0 + 16 < bn;
                    f32x4_t acc_next[G];
                    float4 nv_next = nv_cur;
                    if (more) {
                        frag(r0 + 16, av, nv_next);
                        products(av, acc_next);
                    }
                    const float nv[4] = {nv_cur.x, nv_cur.y, nv_cur.z, nv_cur.w};
                    // d~ of the lane's 4 rows for each group; a NaN norm marks
                    // a padding row and never passes
                    // (fminf drops NaN operands, so padding rows fall out of
                    // the minimum; a -inf threshold makes the margin +inf)
                    float d[G][4];
                    float margin = __builtin_huge_valf();
#pragma unroll
                    for (int g = 0; g < G; ++g) {
#pragma unroll
                        for (int ii = 0; ii < 4; ++ii) d[g][ii] = nv[ii] - 2.0f * acc[g][ii];
                        const float m4 = fminf(fminf(d[g][0], d[g][1]), fminf(d[g][2], d[g][3]));
                        margin = fminf(margin, m4 - pthr[g]);
                    }
                    if (__ballot(margin <= 0.0f) != 0) {  // rare once the bounds have settled
#pragma unroll
                        for (int g = 0; g < G; ++g)
#pragma unroll
                            for (int ii = 0; ii < 4; ++ii) {
                                const bool pass = d[g][ii] <= pthr[g];
                                const uint64_t m = __ballot(pass);
                                if (m == 0) continue;
                                if (nhit + (uint32_t)__popcll(m) > (uint32_t)kHitCap) flush();
                                if (pass) {
                                    const uint32_t at = nhit + (uint32_t)__popcll(m & lanemask_lt());
                                    s_hit[w][at] = make_uint4(__float_as_uint(d[g][ii]), bp + r0 + 4 * (l / 16) + ii,
                                                              16 * g + (l % 16), 0u);
                                }
                                nhit += (uint32_t)__popcll(m);
                            }
                        set_pthr();
                    }
                    if (more) {
#pragma unroll
                        for (int g = 0; g < G; ++g) acc[g] = acc_next[g];
                        nv_cur = nv_next;
                    }
                }
            }
            if (nhit > 0) flush();
            if (own_ok) {
                uint32_t c = 0;
#pragma unroll
                for (int k = 0; k < R; ++k) c = cmv[k] > c ? cmv[k] : c;
                ownb = c;
            }
            refresh_thr();
            if (nli < nlist) park(buf ^ 1);
            __syncthreads();
            buf ^= 1;
            li = nli;
            bp = np;
            bn = nn;
        }

        // 5. store the split's lists
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (own_ok) {
            uint2* dst = a.part + ((int64_t)own_q * a.S + s) * R;
#pragma unroll
            for (int k = 0; k < R; ++k) dst[k] = wl[l * R + k];
        }
        __syncthreads();
    }
}

// Seeds the shared class minima before the screen, so that no split starts
// without a bound.  One wave per query; each lane takes one row of the
// query's own cone (the first kSeedRows rows at most), computes d~ on the
// vector units and raises it by a bound on the difference to any FP32
// accumulation of the same products (the matrix cores add them in another
// order): each of the two sums is off by at most dk*u*S with S the sum of
// |products|, and the final subtraction by u*(|n| + 2|q.x|), so
// (4dk + 8)*u*(n + 2S) covers both (u = 2^-24), with a margin.  The raised
// value is at least the screen's d~ of a real candidate of its class, so the
// largest-class-minimum rule stays a valid bound.
constexpr int kSeedRows = 256;

template <bool F16IN, int R>
__global__ __launch_bounds__(256) void tiled_seed_kernel(SeedArgs a) {
#pragma clang fp contract(off)
    const int64_t q = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    const int l = lane_id();
    if (q >= a.Q) return;
    const uint32_t c = a.q_cone[q];
    const uint32_t p0 = a.poff[c], p1 = a.poff[c + 1];
    const uint32_t pend = p1 - p0 > (uint32_t)kSeedRows ? p0 + kSeedRows : p1;
    const float gamma = (float)(4 * a.dk + 8) * 5.9604645e-08f * 1.01f;
    for (uint32_t p = p0 + l; p < pend; p += 64) {
        const float n = a.nrm[p];
        if (!(n < __builtin_huge_valf())) continue;  // padding row (NaN norm)
        const uint4* xr = reinterpret_cast<const uint4*>(a.xl + (int64_t)p * a.dk);
        const uint4* qr = reinterpret_cast<const uint4*>(a.ql + q * a.dk);
        float dot = 0.0f, sabs = 0.0f;
        for (int k = 0; k < a.dk / 8; ++k) {
            const uint4 xv = xr[k], qv = qr[k];
            const uint32_t xw[4] = {xv.x, xv.y, xv.z, xv.w}, qw[4] = {qv.x, qv.y, qv.z, qv.w};
#pragma unroll
            for (int h = 0; h < 4; ++h)
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const uint16_t xb = (uint16_t)(xw[h] >> (16 * e)), qb = (uint16_t)(qw[h] >> (16 * e));
                    const float xf = F16IN ? F16::val(xb) : __uint_as_float((uint32_t)xb << 16);
                    const float qf = F16IN ? F16::val(qb) : __uint_as_float((uint32_t)qb << 16);
                    const float pr = xf * qf;
                    dot = dot + pr;
                    sabs = sabs + fabsf(pr);
                }
        }
        const float d = n - 2.0f * dot;
        const float tol = gamma * (n + 2.0f * sabs);
        __hip_atomic_fetch_min(a.cmin + q * R + (p & (R - 1)), ord_bits(d + tol), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

hipError_t launch_tiled_seed(const SeedArgs& a, int R, int f16in, hipStream_t s) {
    if (a.Q <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.Q + 3) / 4));
#define OSANN_SEED(F, RR)                                                                     \
    if ((f16in != 0) == F && R == RR) {                                                       \
        hipLaunchKernelGGL((tiled_seed_kernel<F, RR>), grid, dim3(256), 0, s, a);             \
        return hipGetLastError();                                                             \
    }
    OSANN_SEED(true, 4) OSANN_SEED(true, 8) OSANN_SEED(true, 16)
    OSANN_SEED(false, 4) OSANN_SEED(false, 8) OSANN_SEED(false, 16)
#undef OSANN_SEED
    return hipErrorInvalidValue;
}

// One group of G lanes per query: merge the S split lists (ordered by
// (d~, padded position)), re-rank the R survivors with the exact FP32
// distance, arg-min on (distance, original row).
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
    uint32_t cp = 0xFFFFFFFFu;
#pragma unroll
    for (int k = 0; k < R; ++k)
        if (k == g) cp = lr[k];
    float cd = __builtin_huge_valf();
    uint32_t cr = 0xFFFFFFFFu;
    if (qv && cp != 0xFFFFFFFFu) {
        const uint32_t pos = f.ppos[cp];
        if (pos != 0xFFFFFFFFu) {  // a padding row never enters a list; checked anyway
            cr = f.perm[pos];
            cd = row_dist_fp32<E>(static_cast<const uint4*>(f.planes), f.N, f.nch, pos, f.yf + q * f.dpad);
        }
    }
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
    constexpr int G = R <= 8 ? 4 : 2;
    switch (ks) {
        case 1: hipLaunchKernelGGL((tiled_screen_kernel<F16IN, 1, R, G>), grid, dim3(256), lds, s, a); break;
        case 2: hipLaunchKernelGGL((tiled_screen_kernel<F16IN, 2, R, G>), grid, dim3(256), lds, s, a); break;
        case 4: hipLaunchKernelGGL((tiled_screen_kernel<F16IN, 4, R, G>), grid, dim3(256), lds, s, a); break;
        case 8: hipLaunchKernelGGL((tiled_screen_kernel<F16IN, 8, R, G>), grid, dim3(256), lds, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Dynamic LDS of the screen kernel: marked-cone list (48 B per cone), then
// the larger of the cone table (32 B per cone) and the two staged row
// batches with their norms.
size_t tiled_screen_lds(int64_t span, int dk) {
    const size_t sp = (size_t)(span > 0 ? span : 1);
    const size_t batches = (size_t)2 * kBatchRows * dk * 2 + 2 * kBatchRows * 4;
    return sp * 48 + (sp * 32 > batches ? sp * 32 : batches);
}

hipError_t launch_tiled_screen(const TiledArgs& a, int R, int f16in, int blocks, hipStream_t s) {
    const int ks = a.dk / 32;
    const size_t lds = tiled_screen_lds(a.span, a.dk);
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

#define OSANN_EACH_SCREEN(X)                                                                        \
    X(true, 1, 4, 4) X(true, 2, 4, 4) X(true, 4, 4, 4) X(true, 8, 4, 4) X(true, 1, 8, 4) X(true, 2, 8, 4)    \
    X(true, 4, 8, 4) X(true, 8, 8, 4) X(true, 1, 16, 2) X(true, 2, 16, 2) X(true, 4, 16, 2)                  \
    X(true, 8, 16, 2) X(false, 1, 4, 4) X(false, 2, 4, 4) X(false, 4, 4, 4) X(false, 8, 4, 4)               \
    X(false, 1, 8, 4) X(false, 2, 8, 4) X(false, 4, 8, 4) X(false, 8, 8, 4) X(false, 1, 16, 2)              \
    X(false, 2, 16, 2) X(false, 4, 16, 2) X(false, 8, 16, 2)

size_t tiled_screen_static_lds(int R) {
    const size_t qw = 16 * (size_t)tile_groups(R);
    return 4 * qw * R * 8 + 4 * (size_t)kHitCap * 16 + 2 * 4 * kMaxD + 512;
}

// Lets every screen kernel take all the LDS its static arrays leave free.
hipError_t tiled_screen_max_lds() {
    hipError_t e = hipSuccess;
#define OSANN_SET_LDS(F16IN, KS, R, G)                                                                     \
    if (e == hipSuccess) {                                                                                 \
        hipFuncAttributes fa{};                                                                            \
        e = hipFuncGetAttributes(&fa, (const void*)tiled_screen_kernel<F16IN, KS, R, G>);                  \
        if (e == hipSuccess)                                                                               \
            e = hipFuncSetAttribute((const void*)tiled_screen_kernel<F16IN, KS, R, G>,                     \
                                    hipFuncAttributeMaxDynamicSharedMemorySize,                            \
                                    (int)(kLdsPerBlock - fa.sharedSizeBytes));                             \
    }
    OSANN_EACH_SCREEN(OSANN_SET_LDS)
#undef OSANN_SET_LDS
    return e;
}

int tiled_screen_occupancy(int R, int f16in, int ks, size_t lds) {
    int nb = 0;
    const void* fn = nullptr;
#define OSANN_PICK(F16IN, KS, RR, G) \
    if (f16in == (int)F16IN && ks == KS && R == RR) fn = (const void*)tiled_screen_kernel<F16IN, KS, RR, G>;
    OSANN_EACH_SCREEN(OSANN_PICK)
#undef OSANN_PICK
    if (!fn) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, lds) != hipSuccess) return 0;
    return nb;
}

}  // namespace osann
