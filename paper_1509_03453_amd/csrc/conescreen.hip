// Cone-major matrix-core screening: the tiled mode's screen when queries
// probe many cones (the probe pass then leaves one bit per (query, non-empty
// cone)).
//
// The query-tile screen computes, for every cone any query of a 64-query
// tile probes, the products of all 64 queries; where a query probes a third
// of the cones, two thirds of those products are masked.  Here the unit of
// work is a cone and the queries that probe it:
//
//   * a block takes a query block (128 consecutive slots of the sorted query
//     order) and a group of four 64-cone words of the non-empty cones; it
//     stages the block's low-precision queries in LDS once, then each of its
//     four waves takes one word alone (no further barrier);
//   * from the probe bitmaps the wave forms, for each cone of its word, the
//     mask of the block's queries that probe it (ballot transpose), and for
//     the cone it is screening, the list of those slots;
//   * it streams the cone's rows, 16 at a time, into the MFMA A operand and
//     takes the listed queries 16 at a time as B operands (up to four groups
//     per pass over the rows; a cone probed by more than 64 of the block's
//     queries is streamed again for the next 64), so every product is a
//     probed (query, row) pair apart from the padding of the last group and
//     of the bucket's last 16-row tile.
//
// Blocks are dealt to the chiplets in turn; chiplet x takes the word groups
// x, x + 8, ... each with every query block in turn, so the rows of one word
// group are read by one chiplet while they sit in its L2.
//
// Everything downstream is the query-tile screen's: each (query, word) keeps
// a top-R list of (d~, original row) in LDS, filled from a per-wave hit
// buffer; candidates are pruned against the list's R-th entry and against
// the largest of the query's R class minima, shared by all words and seeded
// from the query's own cone; the lists go to part[query][word] and the finish
// pass merges the words' lists.  Bounds only discard candidates outside the
// final top R, so the result does not depend on the schedule and equals the
// query-tile screen's.
#include "osann_device.h"
#include "osann_kernels.h"
#include "osann_screen.h"
#include "osann_tiled.h"

namespace osann {

constexpr int kConeQB = 128;  // query slots per block: two per lane

// Lane `lane`'s 64-bit value, in scalar registers (the readlane builtin
// returns a signed 32-bit int: each half is taken as unsigned before the
// two are joined, so the low half is never sign-extended into the high one).
__device__ inline uint64_t readlane_u64(uint64_t v, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}
constexpr int kConeG = 4;     // MFMA B groups (16 queries each) per pass over a cone's rows

// Waves per SIMD the kernel is register-capped for: three where the block's
// LDS (short rows) lets three blocks share a compute unit, else two.
template <int KS>
constexpr int cone_waves_per_simd() { return KS <= 2 ? 3 : 2; }

template <bool F16IN, int KS, int R>
__global__ __launch_bounds__(256, cone_waves_per_simd<KS>()) void cone_screen_kernel(TiledArgs a, int64_t nqb) {
    constexpr int QB = kConeQB;
    constexpr int G = kConeG;
    constexpr int UNITS = 4 * KS;         // 16-byte units of one query's codes (dk = 32 KS)
    extern __shared__ uint4 s_q[];        // [QB][UNITS] the block's queries
    __shared__ uint2 s_list[4][R * QB];   // per wave: top-R list per slot, ascending (d~, original row);
                                          // entry r of slot s at r * QB + s
    __shared__ uint3 s_hit[4][kHitCap];   // per wave: (d~ bits, padded position, slot); a flush
                                          // rewrites .y as the original row and .z as
                                          // slot | class << 8 | previous hit << 16
    __shared__ uint8_t s_sel[4][QB];      // per wave: slots probing the cone being screened
    __shared__ uint8_t s_head[4][QB];     // per wave, during a flush: last hit of each slot (0xFF: none)
    const int w = threadIdx.x / 64, l = lane_id();
    const int64_t ncg = (a.nw + 3) / 4;
    const int64_t xq = blockIdx.x % kXcd, jj = blockIdx.x / kXcd;
    const int64_t cg = xq + kXcd * (jj / nqb);
    const int64_t qb = jj % nqb;
    if (cg >= ncg) return;  // the whole block
    const int64_t slot0 = qb * QB;
    const int nq = (int)(a.Q - slot0 < QB ? a.Q - slot0 : QB);
    for (int t = threadIdx.x; t < QB * UNITS; t += 256) {
        const int s = t / UNITS, u = t % UNITS;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (s < nq) v = *reinterpret_cast<const uint4*>(a.ql + (int64_t)a.qorder[slot0 + s] * a.dk + 8 * u);
        s_q[t] = v;
    }
    __syncthreads();  // the only block barrier
    const int64_t k = cg * 4 + w;  // this wave's word of non-empty cones
    if (k >= a.nw) return;
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    };
    uint2* wl = s_list[w];
    uint3* hit = s_hit[w];
    uint8_t* sel = s_sel[w];
    // bound of slots l and 64 + l (lane l's own); other lanes read them by shuffle
    float thr[2] = {__builtin_huge_valf(), __builtin_huge_valf()};
    for (int t = l; t < QB * R; t += 64) wl[t] = make_uint2(0x7F800000u, 0xFFFFFFFFu);
    // bound of each slot: the largest of its R class minima (+inf while a class is empty)
    auto shared_bounds = [&]() {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int s = 64 * h + l;
            uint32_t b = 0xFFFFFFFFu;
            if (s < nq) {
                b = 0u;
#pragma unroll
                for (int c = 0; c < R; ++c) {
                    const uint32_t v = __hip_atomic_load(a.cmin + (int64_t)c * a.Q + slot0 + s, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    b = v > b ? v : b;
                }
            }
            thr[h] = fminf(thr[h], ord_float(b));
        }
    };
    shared_bounds();

    // lane c: masks over the block's 128 slots of the queries that probe
    // non-empty cone 64k + c, and that cone's padded rows
    uint64_t mk[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int s = 64 * h + l;
        const uint64_t word = s < nq ? a.qbits[(int64_t)a.qorder[slot0 + s] * a.nw + k] : 0ull;
        uint64_t col = 0;
#pragma unroll 8
        for (int c = 0; c < 64; ++c) {
            const uint64_t bm = __ballot((word >> c) & 1ull);
            col = c == l ? bm : col;
        }
        mk[h] = col;
    }
    const int64_t e = k * 64 + l;
    uint32_t lp0 = 0, lp1 = 0;
    if (e < a.n_ne) {
        const uint32_t cone = a.ne_cone[e];
        lp0 = a.poff[cone];
        lp1 = a.poff[cone + 1];
    }
    uint64_t rem = __ballot((mk[0] | mk[1]) != 0ull && lp1 > lp0);  // cones left to screen
    wave_sync();

    // ---- hits -> lists: lane l owns slots l and 64 + l ----
    // A flush chains each buffered hit to the previous hit of the same slot
    // (found by matching slot bits across the wave: the last hit of a slot
    // becomes its head), so each lane then walks only its own slots' hits (a
    // few) instead of the whole buffer; the merge keeps the R smallest (d~,
    // row) and the class minima, neither of which depends on the order.
    uint8_t* head = s_head[w];
    head[l] = 0xFFu;
    head[64 + l] = 0xFFu;
    uint32_t nhit = 0;
    auto flush = [&]() {
        wave_sync();
        const bool mine = (uint32_t)l < nhit;
        const uint3 en = hit[l];  // entries past nhit are stale but never used
        const uint32_t sl = en.z & 0xFFu;
        uint64_t same = __ballot(mine);
#pragma unroll
        for (int b = 0; b < 7; ++b) {
            const bool bit = (sl >> b) & 1u;
            const uint64_t ones = __ballot(bit);
            same &= bit ? ones : ~ones;
        }
        if (mine) {
            const uint64_t before = same & lanemask_lt();
            const uint32_t prev = before ? 63u - (uint32_t)__clzll((unsigned long long)before) : 0xFFu;
            hit[l] = make_uint3(en.x, a.prow[en.y], sl | ((en.y & (uint32_t)(R - 1)) << 8) | (prev << 16));
            if ((same >> l) == 1ull) head[sl] = (uint8_t)l;  // no later hit of this slot
        }
        wave_sync();
        auto merge = [&](int h) __attribute__((always_inline)) {
            const int s = 64 * h + l;
            uint32_t j = head[s];
            if (j == 0xFFu) return;
            float ld[R];
            uint32_t lr[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint2 e = wl[r * QB + s];
                ld[r] = __uint_as_float(e.x);
                lr[r] = e.y;
            }
            bool ch = false;
            for (; j != 0xFFu;) {
                const uint3 he = hit[j];
                const float d = __uint_as_float(he.x);
                if (pair_less(d, he.y, ld[R - 1], lr[R - 1])) {
                    list_insert<R>(ld, lr, d, he.y);
                    ch = true;
                    __hip_atomic_fetch_min(a.cmin + (int64_t)((he.z >> 8) & 0xFFu) * a.Q + slot0 + s, ord_bits(d),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                j = (he.z >> 16) & 0xFFu;
            }
            head[s] = 0xFFu;  // empty for the next flush
            if (ch) {
#pragma unroll
                for (int r = 0; r < R; ++r) wl[r * QB + s] = make_uint2(__float_as_uint(ld[r]), lr[r]);
                thr[h] = fminf(thr[h], ld[R - 1]);
            }
        };
        merge(0);
        merge(1);
        nhit = 0;
        wave_sync();
    };

    // ---- the (cone, pass, tile) sequence: uniform cursor ----
    struct Tile {
        int c;          // lane holding the cone's masks and rows, -1: past the end
        int base;       // first listed query of the pass
        uint32_t p;     // padded position of the tile's first row
    };
    int cur_c = -1, cur_base = 0, cur_nc = 0;
    uint32_t cur_p0 = 0, cur_p1 = 0, cur_p = 0;
    auto next_tile = [&](Tile& t) __attribute__((always_inline)) {
        if (cur_c >= 0) {
            cur_p += 16;
            if (cur_p >= cur_p1) {
                cur_base += 64;
                if (cur_base < cur_nc) cur_p = cur_p0;
                else cur_c = -1;
            }
        }
        if (cur_c < 0 && rem) {
            cur_c = __ffsll((unsigned long long)rem) - 1;
            rem &= rem - 1;
            cur_p0 = (uint32_t)__builtin_amdgcn_readlane((int)lp0, cur_c);
            cur_p1 = (uint32_t)__builtin_amdgcn_readlane((int)lp1, cur_c);
            const uint64_t m0 = readlane_u64(mk[0], cur_c), m1 = readlane_u64(mk[1], cur_c);
            cur_nc = __popcll(m0) + __popcll(m1);
            cur_base = 0;
            cur_p = cur_p0;
        }
        t.c = cur_c;
        t.base = cur_base;
        t.p = cur_p;
    };
    const int lane_off = (l % 16) * a.dk + 8 * (l / 16);
    auto load = [&](uint32_t pp, uint4 (&av)[KS], float4& nv) __attribute__((always_inline)) {
        const uint16_t* src = a.xl + (int64_t)pp * a.dk;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) av[ks] = *reinterpret_cast<const uint4*>(src + lane_off + 32 * ks);
        nv = *reinterpret_cast<const float4*>(a.nrm + pp + 4 * (l / 16));
    };

    // ---- the pass being screened: its queries as B operands ----
    int unit_c = -1, unit_base = -1, unit_nc = 0, ng = 0, cones_done = 0;
    uint4 bq[G][KS];
    float pthr[G];      // -bound/2 of the lane's query in group g (the accumulators hold -d~/2); +inf: none
    uint32_t bslot[G];  // its slot, 0xFF: none
    auto set_pthr = [&]() {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int src = (int)(bslot[g] & 63u);
            const float t0 = __shfl(thr[0], src, 64), t1 = __shfl(thr[1], src, 64);
            pthr[g] = bslot[g] != 0xFFu ? -0.5f * (bslot[g] < 64u ? t0 : t1) : __builtin_huge_valf();
        }
    };
    auto setup = [&](int c, int base) __attribute__((always_inline)) {
        if (c != unit_c) {
            if (++cones_done % 8 == 0) shared_bounds();  // the other words' progress
            const uint64_t m0 = readlane_u64(mk[0], c), m1 = readlane_u64(mk[1], c);
            const int n0 = __popcll(m0);
            wave_sync();
            if ((m0 >> l) & 1ull) sel[__popcll(m0 & lanemask_lt())] = (uint8_t)l;
            if ((m1 >> l) & 1ull) sel[n0 + __popcll(m1 & lanemask_lt())] = (uint8_t)(64 + l);
            wave_sync();
            unit_c = c;
            unit_nc = n0 + __popcll(m1);
        }
        unit_base = base;
        const int left = unit_nc - base;
        ng = left >= 16 * G ? G : (left + 15) / 16;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int idx = base + 16 * g + (l % 16);
            const bool v = g < ng && idx < unit_nc;
            const uint32_t slot = v ? sel[idx] : 0u;
            bslot[g] = v ? slot : 0xFFu;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                bq[g][ks] = v ? s_q[slot * UNITS + 4 * ks + (l / 16)] : make_uint4(0, 0, 0, 0);
        }
        set_pthr();
    };
    auto screen = [&](const Tile& t, const uint4 (&av)[KS], const float4& nv) __attribute__((always_inline)) {
        if (t.c != unit_c || t.base != unit_base) setup(t.c, t.base);
        const f32x4_t c0 = {-0.5f * nv.x, -0.5f * nv.y, -0.5f * nv.z, -0.5f * nv.w};
        // every group, used or not: straight-line code (a group past the
        // pass's queries holds zero operands and a +inf bound, so it never
        // passes the test)
        f32x4_t acc[G];
        float margin = -__builtin_huge_valf();
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = mfma16<F16IN>(av[0], bq[g][0], c0);
#pragma unroll
        for (int ks = 1; ks < KS; ++ks)
#pragma unroll
            for (int g = 0; g < G; ++g) acc[g] = mfma16<F16IN>(av[ks], bq[g][ks], acc[g]);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const float m4 = fmaxf(fmaxf(acc[g][0], acc[g][1]), fmaxf(acc[g][2], acc[g][3]));
            margin = fmaxf(margin, m4 - pthr[g]);
        }
        if (__ballot(margin >= 0.0f) != 0) {  // rare once the bounds have settled
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (g >= ng) break;
#pragma unroll
                for (int ii = 0; ii < 4; ++ii) {
                    const bool pass = acc[g][ii] >= pthr[g];
                    const uint64_t m = __ballot(pass);
                    if (m == 0) continue;
                    if (nhit + (uint32_t)__popcll(m) > (uint32_t)kHitCap) {
                        flush();
                        set_pthr();
                    }
                    if (pass) {
                        const uint32_t at = nhit + (uint32_t)__popcll(m & lanemask_lt());
                        hit[at] = make_uint3(__float_as_uint(-2.0f * acc[g][ii]), t.p + 4 * (l / 16) + ii, bslot[g]);
                    }
                    nhit += (uint32_t)__popcll(m);
                }
            }
        }
    };

    // three register buffers rotated by name: no register with a load in
    // flight is ever copied, and the next two tiles (of this cone or the
    // next ones) are in flight while the current one is screened (164
    // VGPRs, still three waves per SIMD).  Every step issues its loads (a
    // cursor past the end reloads padded position 0, a valid tile), so the
    // number of loads in flight is fixed and the wait before a tile's
    // products covers that tile's loads only.
    Tile tA, tB, tC;
    uint4 avA[KS], avB[KS], avC[KS];
    float4 nvA, nvB, nvC;
    next_tile(tA);
    load(tA.c >= 0 ? tA.p : 0u, avA, nvA);
    next_tile(tB);
    load(tB.c >= 0 ? tB.p : 0u, avB, nvB);
    while (tA.c >= 0) {
        next_tile(tC);
        load(tC.c >= 0 ? tC.p : 0u, avC, nvC);
        screen(tA, avA, nvA);
        if (tB.c < 0) break;
        next_tile(tA);
        load(tA.c >= 0 ? tA.p : 0u, avA, nvA);
        screen(tB, avB, nvB);
        if (tC.c < 0) break;
        next_tile(tB);
        load(tB.c >= 0 ? tB.p : 0u, avB, nvB);
        screen(tC, avC, nvC);
    }
    if (nhit > 0) flush();

    // the word's lists of the block's queries
    wave_sync();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int s = 64 * h + l;
        if (s < nq) {
            uint2* dst = a.part + ((int64_t)a.qorder[slot0 + s] * a.S + k) * R;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[r] = wl[r * QB + s];
        }
    }
}

template <bool F16IN, int R>
static hipError_t cone_ks(const TiledArgs& a, int ks, dim3 grid, size_t lds, int64_t nqb, hipStream_t s) {
    switch (ks) {
        case 1: hipLaunchKernelGGL((cone_screen_kernel<F16IN, 1, R>), grid, dim3(256), lds, s, a, nqb); break;
        case 2: hipLaunchKernelGGL((cone_screen_kernel<F16IN, 2, R>), grid, dim3(256), lds, s, a, nqb); break;
        case 4: hipLaunchKernelGGL((cone_screen_kernel<F16IN, 4, R>), grid, dim3(256), lds, s, a, nqb); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// dk and R whose instantiation fits its registers (R = 16 keeps two 16-entry
// lists per lane live in the merge: only with short rows)
bool cone_screen_ok(int dk, int R) { return (dk == 32 || dk == 64 || dk == 128) && (R <= 8 || dk == 32); }

size_t cone_screen_lds(int dk) { return (size_t)kConeQB * dk * 2; }

hipError_t launch_cone_screen(const TiledArgs& a, int R, int f16in, hipStream_t s) {
    if (!cone_screen_ok(a.dk, R) || a.S != a.nw || !a.qbits) return hipErrorInvalidValue;
    const int ks = a.dk / 32;
    const int64_t nqb = (a.Q + kConeQB - 1) / kConeQB;
    const int64_t ncg = (a.nw + 3) / 4;
    const int64_t blocks = (int64_t)kXcd * ((ncg + kXcd - 1) / kXcd) * nqb;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    const size_t lds = cone_screen_lds(a.dk);
    const dim3 grid((unsigned)blocks);
#define OSANN_CONE_PICK(F, RR) \
    if ((f16in != 0) == F && R == RR) return cone_ks<F, RR>(a, ks, grid, lds, nqb, s);
    OSANN_CONE_PICK(true, 4) OSANN_CONE_PICK(true, 8) OSANN_CONE_PICK(true, 16)
    OSANN_CONE_PICK(false, 4) OSANN_CONE_PICK(false, 8) OSANN_CONE_PICK(false, 16)
#undef OSANN_CONE_PICK
    return hipErrorInvalidValue;
}

// Lets every cone-major screen kernel take the dynamic LDS its static arrays leave free.
hipError_t cone_screen_max_lds() {
    hipError_t e = hipSuccess;
#define OSANN_CONE_LDS(F, KS, RR)                                                                        \
    if (e == hipSuccess) {                                                                               \
        hipFuncAttributes fa{};                                                                          \
        e = hipFuncGetAttributes(&fa, (const void*)cone_screen_kernel<F, KS, RR>);                       \
        if (e == hipSuccess)                                                                             \
            e = hipFuncSetAttribute((const void*)cone_screen_kernel<F, KS, RR>,                          \
                                    hipFuncAttributeMaxDynamicSharedMemorySize,                          \
                                    (int)(kLdsPerBlock - fa.sharedSizeBytes));                           \
    }
    OSANN_CONE_LDS(true, 1, 4) OSANN_CONE_LDS(true, 2, 4) OSANN_CONE_LDS(true, 4, 4)
    OSANN_CONE_LDS(true, 1, 8) OSANN_CONE_LDS(true, 2, 8) OSANN_CONE_LDS(true, 4, 8)
    OSANN_CONE_LDS(true, 1, 16) OSANN_CONE_LDS(true, 2, 16) OSANN_CONE_LDS(true, 4, 16)
    OSANN_CONE_LDS(false, 1, 4) OSANN_CONE_LDS(false, 2, 4) OSANN_CONE_LDS(false, 4, 4)
    OSANN_CONE_LDS(false, 1, 8) OSANN_CONE_LDS(false, 2, 8) OSANN_CONE_LDS(false, 4, 8)
    OSANN_CONE_LDS(false, 1, 16) OSANN_CONE_LDS(false, 2, 16) OSANN_CONE_LDS(false, 4, 16)
#undef OSANN_CONE_LDS
    return e;
}

}  // namespace osann
