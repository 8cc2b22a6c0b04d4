// Matrix-core screening of the candidates with an exact FP32 re-rank.
//
// Queries are sorted by their own cone and cut into wave tiles of 16G
// queries.  A work item is (wave tile, split): split s owns a contiguous
// range of the non-empty cones, and one wave takes the item alone.  It
// first lists the cones of its range that some query of the tile probes,
// with the mask of those queries (from the probe pass's bitmaps, or by
// regenerating the walks of Section 3.B, one lane per query); then it
// streams every listed cone's rows, 16 at a time, straight from memory into
// the MFMA A operand (bucket sizes are padded to 16 rows in the
// low-precision copy).  With the rows as the MFMA A operand and 16 queries
// as B, lane l holds the products of query l%16 with 4 rows; the
// accumulators start at -||x^||^2/2, so they end at -d~/2 with
// d~ = ||x^||^2 - 2 q^.x^, which ranks candidates like the squared distance
// of the rounded vectors.  No wave waits for another: a wave only
// reads the cones its own queries probe.
//
// Each query keeps, per split, a top-R list of (d~, original row) in LDS,
// the order the exact definition of the screen uses, so equal d~ resolve to
// the lower original row.  The tile loop only compares d~ with a per-query
// bound; the few candidates at or below it go to a per-wave hit buffer,
// which is merged into the lists (one lane per query) when it fills and at
// the end of the item.
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
// Lists are kept in the total order (d~, original row), so results do not
// depend on the order of the tiles or on the split.
#include "osann_device.h"
#include "osann_kernels.h"
#include "osann_tiled.h"
#include "osann_screen.h"

namespace osann {


// One wave works on one item at a time: (wave tile of 16G queries, split),
// taking the split's cones kChunk at a time.  Dynamic LDS holds, per wave,
// the marked-cone list of one chunk: (p0, p1, probe mask lo, hi) over the
// padded rows [p0, p1) of each listed cone.  While the walks are
// regenerated, a cone table (one probe mask per cone of the chunk) sits in
// the list's upper half and is compacted into the list in place (entry i is
// written at 16i bytes, table word j is read at 8*kChunk + 8j bytes, j >= i,
// and a chunk of 64 table words is read before its entries are written).
template <bool F16IN, int KS, int R, int G>
__global__ __launch_bounds__(256, 2) void tiled_screen_kernel(TiledArgs a) {
    constexpr int QW = 16 * G;              // queries per wave tile
    constexpr int U = KS <= 2 ? 2 : 1;      // row tiles per load group
    extern __shared__ uint64_t dyn[];
    __shared__ uint2 s_list[4][QW * R];     // per wave: top-R list of each query slot
    __shared__ uint4 s_hit[4][kHitCap];     // per wave: (d~ bits, padded position, slot, original row) hits
    __shared__ uint32_t s_head[4][64];      // per wave, during a flush: last hit of each slot (~0: none)
    __shared__ uint32_t s_next[4][kHitCap];  // the hit chained before it for the same slot
    __shared__ uint32_t s_walk[4][64 * kWalkCache];  // per wave, lane l: ranks of the non-empty cones its query probes
    const int w = threadIdx.x / 64, l = lane_id();
    s_head[w][l] = ~0u;
    // Work queue of this block's chiplet (blocks are dealt to the kXcd chiplets
    // in turn, and each has its own L2): with 8 splits or more, chiplet x
    // takes the splits x, x + kXcd, ... one after the other, so the waves
    // of a chiplet stream the same cones at about the same time; else it
    // takes the tiles x, x + kXcd, ... (tiles in order of their queries'
    // cones, so all chiplets work on neighbouring cones and balance).  The
    // mapping only steers locality: every item belongs to exactly one
    // queue, and every queue is drained by the blocks with that index mod
    // kXcd.
    const int xq = (int)(blockIdx.x % kXcd);
    const bool by_split = a.S >= kXcd;
    const int64_t total = by_split ? (int64_t)(a.S / kXcd) * a.T
                                   : (a.T > xq ? (a.T - xq + kXcd - 1) / kXcd : 0) * a.S;
    uint4* wlist = reinterpret_cast<uint4*>(dyn) + (size_t)w * kChunk;
    uint64_t* tab = reinterpret_cast<uint64_t*>(wlist) + kChunk;
    uint2* wl = s_list[w];
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    };
    for (;;) {
        uint32_t got = 0;
        if (l == 0) got = atomicAdd(a.counter + xq, 1u);
        const int64_t item = (int64_t)__builtin_amdgcn_readfirstlane(__shfl((int)got, 0, 64)) & 0xFFFFFFFFll;
        if (item >= total) break;
        const int64_t t = by_split ? item % a.T : xq + kXcd * (item / a.S);
        const int s = by_split ? xq + kXcd * (int)(item / a.T) : (int)(item % a.S);
        const int64_t n0 = s * a.span;
        const int64_t n1 = n0 + a.span < a.n_ne ? n0 + a.span : a.n_ne;
        const int64_t slot0 = t * QW;  // first query slot of the wave tile
        const bool own_ok = l < QW && slot0 + l < a.Q;
        const uint32_t own_q = own_ok ? a.qorder[slot0 + l] : 0u;
        const int64_t own_slot = own_ok ? slot0 + l : 0;  // class minima are stored by tile slot
        // Without bitmaps, each query lane decodes its walk once per item and
        // keeps the ranks of the non-empty cones it probes (up to kWalkCache;
        // a lane with more decodes its walk again for every chunk of cones).
        uint32_t* wc = s_walk[w] + l * kWalkCache;
        uint32_t nwc = 0;
        bool wover = false;
        const uint32_t walk_len = !a.qbits && own_ok ? a.jstop[own_q] : 0u;
        if (!a.qbits && own_ok && walk_len != kWalkAll) {
            const uint8_t* qo = a.order + (int64_t)own_q * a.D;
            const uint8_t* qs = a.sbit + (int64_t)own_q * a.D;
            for (uint32_t j = 0; j < walk_len; ++j) {
                const uint32_t cone = probe_cone(j, a.L, qo, qs, a.n_sub, a.lexsub, a.maskord, a.binom);
                if (a.offsets[cone + 1] <= a.offsets[cone]) continue;
                if (nwc == (uint32_t)kWalkCache) {
                    wover = true;
                    break;
                }
                wc[nwc++] = a.ne_id[cone];
            }
        }

        // 1. B operands: group g = query slots 16g .. 16g+15 of the tile;
        //    lane l works on slot 16g + l%16 of every group
        uint4 bq[G][KS];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t slot = slot0 + 16 * g + (l % 16);
            const uint32_t q = slot < a.Q ? a.qorder[slot] : 0u;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                bq[g][ks] = slot < a.Q ? *reinterpret_cast<const uint4*>(a.ql + (int64_t)q * a.dk + ks * 32 + 8 * (l / 16))
                                       : make_uint4(0, 0, 0, 0);
        }
        // The split's top-R list of every query of the tile lives in LDS
        // (wl[slot][k], ascending (d~, original row)); lane l owns slot l
        // when lists are updated.  Candidates that pass the bound go to a hit
        // buffer first and are merged in bulk, which keeps the tile loop free
        // of list code.
        for (int k = l; k < QW * R; k += 64) wl[k] = make_uint2(0x7F800000u, 0xFFFFFFFFu);
        uint32_t nhit = 0;
        uint32_t ownb = 0xFFFFFFFFu;  // shared bound of slot l's query (owner view)
        if (own_ok)
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const uint32_t v = __hip_atomic_load(a.cmin + (int64_t)k * a.Q + own_slot, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                ownb = k == 0 || v > ownb ? v : ownb;
            }
        wave_sync();
        // thr[g]: no candidate of slot 16g + l%16 above it can enter the final
        // top R: the minimum of the slot's list R-th entry and the shared bound
        float thr[G];
        auto refresh_thr = [&]() {
            const float ob = fminf(ord_float(ownb), __uint_as_float(wl[l % QW * R + R - 1].x));
#pragma unroll
            for (int g = 0; g < G; ++g) thr[g] = __shfl(ob, 16 * g + (l % 16), 64);
        };
        refresh_thr();
        // merge the hit buffer into the lists: first every lane looks up the
        // original row of up to one hit (one parallel gather) and chains the
        // hit into its slot's list in LDS (one exchange), then lane l walks
        // the hits of slot l only (the merge does not depend on their order)
        auto flush = [&]() {
            wave_sync();
            if ((uint32_t)l < nhit) {
                const uint4 e = s_hit[w][l];
                s_hit[w][l].w = a.prow[e.y];
                s_next[w][l] = atomicExch(&s_head[w][e.z], (uint32_t)l);
            }
            wave_sync();
            float ld[R];
            uint32_t lr[R];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const uint2 e = wl[(l % QW) * R + k];
                ld[k] = __uint_as_float(e.x);
                lr[k] = e.y;
            }
            bool changed = false;
            if (l < QW) {
                for (uint32_t h = s_head[w][l]; h != ~0u; h = s_next[w][h]) {
                    const uint4 e = s_hit[w][h];
                    const float d = __uint_as_float(e.x);
                    if (pair_less(d, e.w, ld[R - 1], lr[R - 1])) {
                        list_insert<R>(ld, lr, d, e.w);
                        changed = true;
                        __hip_atomic_fetch_min(a.cmin + (int64_t)(e.y & (R - 1)) * a.Q + own_slot, ord_bits(d),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                s_head[w][l] = ~0u;  // empty for the next flush
            }
            if (changed && l < QW)
#pragma unroll
                for (int k = 0; k < R; ++k) wl[l * R + k] = make_uint2(__float_as_uint(ld[k]), lr[k]);
            nhit = 0;
            wave_sync();
            refresh_thr();
        };

        // 3. the listed cones' rows, 16 at a time, straight from memory into
        //    the MFMA A operand (lane l: row l%16, columns 8(l/16)+32ks ..);
        //    the next tile's loads are in flight while the current one is
        //    screened.  One word of the query's class minima is read per
        //    tile; the largest of R consecutive reads (one per class) is a
        //    valid shared bound (the words only decrease), so it replaces
        //    the owner's bound every R tiles.  Plain loads: a cached copy may
        //    be stale, which only makes the bound looser.
        const int lane_off = (l % 16) * a.dk + 8 * (l / 16);
        auto load = [&](uint32_t pp, uint4 (&av)[KS], float4& nv) {  // pp: uniform
            const uint16_t* src = a.xl + (int64_t)pp * a.dk;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) av[ks] = *reinterpret_cast<const uint4*>(src + lane_off + 32 * ks);
            nv = *reinterpret_cast<const float4*>(a.nrm + pp + 4 * (l / 16));
        };
        uint32_t it = 0, run = 0;  // tiles screened in the item, largest class minimum read in the window
        for (int64_t c0 = n0; c0 < n1; c0 += kChunk) {
            const int64_t c1 = c0 + kChunk < n1 ? c0 + kChunk : n1;
            const int nchunk = (int)(c1 - c0);
            // 2. the chunk's cones that some query of the tile probes, with
            //    the mask of those queries
            uint32_t nlist = 0;
            auto append = [&](int64_t e, uint64_t m) {  // e: non-empty cone rank, m: its mask (this lane)
                const bool hit = m != 0;
                const uint64_t b = __ballot(hit);
                if (hit) {
                    const uint32_t cone = a.ne_cone[e];
                    wlist[nlist + (uint32_t)__popcll(b & lanemask_lt())] =
                        make_uint4(a.poff[cone], a.poff[cone + 1], (uint32_t)m, (uint32_t)(m >> 32));
                }
                nlist += (uint32_t)__popcll(b);
            };
            if (a.qbits) {
                // transpose the queries' probed-cone bitmaps with ballots
                for (int64_t k = c0 >> 6; k * 64 < c1; ++k) {
                    const uint64_t word = own_ok ? a.qbits[(int64_t)own_q * a.nw + k] : 0ull;
                    uint64_t col = 0;
#pragma unroll 8
                    for (int c = 0; c < 64; ++c) {
                        const uint64_t m = __ballot((word >> c) & 1ull);
                        col = c == l ? m : col;
                    }
                    const int64_t e = k * 64 + l;
                    append(e, e >= c0 && e < c1 ? col : 0ull);
                }
            } else {
                // one lane per query regenerates its walk; a query that probes
                // every cone sets its bit everywhere
                const uint32_t js = walk_len;
                const uint64_t all = __ballot(own_ok && js == kWalkAll);
                for (int i = l; i < nchunk; i += 64) tab[i] = all;
                wave_sync();
                if (own_ok && js != kWalkAll && !wover) {
                    const unsigned long long bit = 1ull << l;
                    for (uint32_t k = 0; k < nwc; ++k) {
                        const int64_t e = wc[k];
                        if (e >= c0 && e < c1) atomicOr((unsigned long long*)&tab[e - c0], bit);
                    }
                } else if (own_ok && js != kWalkAll) {
                    const uint8_t* qo = a.order + (int64_t)own_q * a.D;
                    const uint8_t* qs = a.sbit + (int64_t)own_q * a.D;
                    const unsigned long long bit = 1ull << l;
                    for (uint32_t j = 0; j < js; ++j) {
                        const uint32_t cone = probe_cone(j, a.L, qo, qs, a.n_sub, a.lexsub, a.maskord, a.binom);
                        const int64_t e = a.ne_id[cone];
                        if (e >= c0 && e < c1 && a.offsets[cone + 1] > a.offsets[cone])
                            atomicOr((unsigned long long*)&tab[e - c0], bit);
                    }
                }
                wave_sync();
                for (int base = 0; base < nchunk; base += 64) {
                    const int i = base + l;
                    const uint64_t m = i < nchunk ? tab[i] : 0ull;
                    append(c0 + i, m);
                }
            }
            wave_sync();

            if (nlist > 0) {
                // load cursor: the next tile to load (lli == nlist: past the end)
                uint32_t lli = 0;
                uint4 lent = uni4(wlist[0]);
                uint32_t lp = lent.x;
                const uint32_t p_any = lp;  // a valid tile, reloaded by a cursor past the end
                auto advance = [&]() {
                    if (lli >= nlist) return;
                    lp += 16;
                    if (lp >= lent.y) {
                        ++lli;
                        if (lli < nlist) {
                            lent = uni4(wlist[lli]);
                            lp = lent.x;
                        }
                    }
                };
                // a group: up to U consecutive tiles of the list, with their
                // padded positions and probe masks; n valid (a prefix)
                struct Group {
                    uint32_t pos[U], mlo[U], mhi[U];
                    uint32_t n;
                };
                auto fill = [&](Group& gr, uint4 (&av)[U][KS], float4 (&nv)[U]) __attribute__((always_inline)) {
                    gr.n = 0;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const bool v = lli < nlist;
                        gr.pos[u] = v ? lp : p_any;
                        gr.mlo[u] = lent.z;
                        gr.mhi[u] = lent.w;
                        gr.n += v ? 1u : 0u;
                        load(gr.pos[u], av[u], nv[u]);
                        advance();
                    }
                };
                // -thr/2 (the accumulators hold -d~/2), or +inf for slots that do
                // not probe the tile's cone
                float pthr[G];
                uint32_t cmlo = 0, cmhi = 0;  // the probe mask pthr was set for
                auto set_pthr = [&]() {
                    const uint64_t mk = ((uint64_t)cmhi << 32) | cmlo;
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const bool probed = (mk >> (16 * g + (l % 16))) & 1ull;
                        pthr[g] = probed ? -0.5f * thr[g] : __builtin_huge_valf();
                    }
                };
                // One group step: issue the next group's loads into the other
                // buffer (and one word of the class minima), then screen this
                // group.  The loop below alternates two register buffers by
                // name, so no register with a load in flight is ever copied,
                // and U tiles share each wait for memory.
                auto group = [&](const Group& gr, const uint4 (&av)[U][KS], const float4 (&nv)[U], uint32_t cw,
                                 Group& grn, uint4 (&avn)[U][KS], float4 (&nvn)[U],
                                 uint32_t& cwn) __attribute__((always_inline)) -> bool {
                    fill(grn, avn, nvn);
                    cwn = a.cmin[(int64_t)(it & (R - 1)) * a.Q + own_slot];
                    // fold the class read one group earlier; a window of R reads starts with class 0
                    run = ((it - 1) & (R - 1)) == 0 ? cw : (cw > run ? cw : run);
                    // products of every tile of the group first, then their bound
                    // tests, so the matrix work of one tile overlaps the vector
                    // work of the other
                    f32x4_t acc[U][G];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if ((uint32_t)u >= gr.n) break;
                        const f32x4_t c0 = {-0.5f * nv[u].x, -0.5f * nv[u].y, -0.5f * nv[u].z, -0.5f * nv[u].w};
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            acc[u][g] = mfma16<F16IN>(av[u][0], bq[g][0], c0);
#pragma unroll
                            for (int ks = 1; ks < KS; ++ks)
                                acc[u][g] = mfma16<F16IN>(av[u][ks], bq[g][ks], acc[u][g]);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if ((uint32_t)u >= gr.n) break;
                        const uint32_t p = gr.pos[u];
                        if (gr.mlo[u] != cmlo || gr.mhi[u] != cmhi) {
                            cmlo = gr.mlo[u];
                            cmhi = gr.mhi[u];
                            set_pthr();
                        }
                        float margin = -__builtin_huge_valf();
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            const float m4 = fmaxf(fmaxf(acc[u][g][0], acc[u][g][1]), fmaxf(acc[u][g][2], acc[u][g][3]));
                            margin = fmaxf(margin, m4 - pthr[g]);
                        }
                        if (__ballot(margin >= 0.0f) != 0) {  // rare once the bounds have settled
#pragma unroll
                            for (int g = 0; g < G; ++g)
#pragma unroll
                                for (int ii = 0; ii < 4; ++ii) {
                                    const bool pass = acc[u][g][ii] >= pthr[g];
                                    const uint64_t m = __ballot(pass);
                                    if (m == 0) continue;
                                    if (nhit + (uint32_t)__popcll(m) > (uint32_t)kHitCap) flush();
                                    if (pass) {
                                        const uint32_t at = nhit + (uint32_t)__popcll(m & lanemask_lt());
                                        s_hit[w][at] = make_uint4(__float_as_uint(-2.0f * acc[u][g][ii]),
                                                                  p + 4 * (l / 16) + ii, 16 * g + (l % 16), 0u);
                                    }
                                    nhit += (uint32_t)__popcll(m);
                                }
                            set_pthr();
                        }
                    }
                    // reads of classes 0 .. R-1 folded by now: a fresh shared bound
                    if ((it & (R - 1)) == 0 && it > 0) {
                        if (own_ok) ownb = run < ownb ? run : ownb;
                        refresh_thr();
                        set_pthr();
                    }
                    ++it;
                    return grn.n > 0;
                };
                Group gA, gB;
                uint4 avA[U][KS], avB[U][KS];
                float4 nvA[U], nvB[U];
                uint32_t cwA = 0xFFFFFFFFu, cwB;
                fill(gA, avA, nvA);
                cmlo = gA.mlo[0];
                cmhi = gA.mhi[0];
                set_pthr();
                while (group(gA, avA, nvA, cwA, gB, avB, nvB, cwB) && group(gB, avB, nvB, cwB, gA, avA, nvA, cwA)) {
                }
            }
        }
        if (nhit > 0) flush();

        // 4. store the split's lists
        wave_sync();
        if (own_ok) {
            uint2* dst = a.part + ((int64_t)own_q * a.S + s) * R;
#pragma unroll
            for (int k = 0; k < R; ++k) dst[k] = wl[l * R + k];
        }
        wave_sync();
    }
}

// Seeds the shared class minima before the screen, so that no split or word
// starts without a bound.  One wave per query takes the rows of the first
// cones of its walk (its own cone, then the next positions of Section 3.B's
// order: the most promising candidates), at most a.rows padded rows; a group
// of dk/8 lanes (rounded up to a power of two) reads one row in one
// coalesced load, 8 components per lane, and several rows' loads are issued
// before their products; it computes d~ on the vector units and raises it by a
// bound on the difference to any FP32 accumulation of the same products (the
// matrix cores add them in another order): each of the two sums is off by at
// most dk*u*S with S the sum of |products| (in any order of the additions),
// and the final subtraction by
// u*(|n| + 2|q.x|), so (4dk + 8)*u*(n + 2S) covers both (u = 2^-24), with a
// margin.  The R-th smallest raised value T is at least the screen's d~ of
// R distinct candidates, so it bounds the query's final R-th d~; it is put
// into every class, where it stays valid: the largest class minimum is at
// least T while any class keeps it, else every class holds a real candidate
// of its own.
constexpr int kSeedMaxRows = 1024;  // 16 rows per lane

template <bool F16IN, int R>
__global__ __launch_bounds__(256) void tiled_seed_kernel(SeedArgs a) {
#pragma clang fp contract(off)
    __shared__ uint32_t s_start[4][64], s_incl[4][64];
    __shared__ float s_raised[4][kSeedMaxRows];  // per wave: raised d~ of each seeded row
    const int w = threadIdx.x / 64, l = lane_id();
    const int64_t slot = (int64_t)blockIdx.x * 4 + w;
    if (slot >= a.Q) return;  // the whole wave; no block barrier below
    const int64_t q = a.qorder[slot];
    // the walk's first positions (at most 64) while their rows stay within a.rows
    const uint32_t js = a.jstop[q];
    const int64_t walk = js == kWalkAll ? a.n_cones : (int64_t)js;
    const int npos = (int)(walk < 64 ? walk : 64);
    uint32_t start = 0, len = 0;
    if (l < npos) {
        const uint32_t c = probe_cone(l, a.L, a.order + q * a.D, a.sbit + q * a.D, a.n_sub, a.lexsub, a.maskord,
                                      a.binom);
        start = a.poff[c];
        len = a.poff[c + 1] - start;
    }
    const uint32_t incl = wave_incl_scan(len);
    const bool take = l < npos && incl - len < (uint32_t)a.rows;  // the first position always
    s_start[w][l] = start;
    s_incl[w][l] = take ? incl : 0xFFFFFFFFu;
    const uint64_t tk = __ballot(take);
    const uint32_t last = tk ? shfl_u32(incl, 63 - __clzll((unsigned long long)tk)) : 0u;
    const uint32_t total = last < (uint32_t)a.rows ? last : (uint32_t)a.rows;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const float gamma = (float)(4 * a.dk + 8) * 5.9604645e-08f * 1.01f;
    const int units = a.dk / 8;  // 16-byte units of a row
    int gs = 4;                  // lanes per row
    while (gs < units) gs *= 2;
    const int rps = 64 / gs;     // rows per step
    const int sub = l % gs, grp = l / gs;
    float qf[8];
    {
        const uint4 qv = sub < units ? reinterpret_cast<const uint4*>(a.ql + q * a.dk)[sub] : make_uint4(0, 0, 0, 0);
        const uint32_t qw[4] = {qv.x, qv.y, qv.z, qv.w};
#pragma unroll
        for (int h = 0; h < 4; ++h)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const uint16_t qb = (uint16_t)(qw[h] >> (16 * e));
                qf[2 * h + e] = F16IN ? F16::val(qb) : __uint_as_float((uint32_t)qb << 16);
            }
    }
    float* raised_rows = s_raised[w];
    uint32_t k = 0;  // walk position of the lane's current row (the lane's rows ascend)
    auto locate = [&](uint32_t r) {
        while (s_incl[w][k] <= r) ++k;
        const uint32_t before = k ? s_incl[w][k - 1] : 0u;
        return s_start[w][k] + (r - before);
    };
    constexpr int U = 4;  // steps whose loads are in flight together
    for (uint32_t r0 = 0; r0 < total; r0 += (uint32_t)(rps * U)) {
        uint4 xv[U];
        float nv[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint32_t r = r0 + (uint32_t)(i * rps + grp);
            const bool ok = r < total;
            const uint32_t p = ok ? locate(r) : 0u;
            xv[i] = ok && sub < units ? reinterpret_cast<const uint4*>(a.xl + (int64_t)p * a.dk)[sub]
                                      : make_uint4(0, 0, 0, 0);
            nv[i] = ok ? a.nrm[p] : __builtin_nanf("");
        }
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint32_t xw[4] = {xv[i].x, xv[i].y, xv[i].z, xv[i].w};
            float dot = 0.0f, sabs = 0.0f;
#pragma unroll
            for (int h = 0; h < 4; ++h)
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const uint16_t xb = (uint16_t)(xw[h] >> (16 * e));
                    const float xf = F16IN ? F16::val(xb) : __uint_as_float((uint32_t)xb << 16);
                    const float pr = xf * qf[2 * h + e];
                    dot = dot + pr;
                    sabs = sabs + fabsf(pr);
                }
            for (int o = gs / 2; o > 0; o >>= 1) {  // the row's lanes: the same sums in every one
                dot = dot + __shfl_xor(dot, o, 64);
                sabs = sabs + __shfl_xor(sabs, o, 64);
            }
            const uint32_t r = r0 + (uint32_t)(i * rps + grp);
            if (sub == 0 && r < total) {
                const float n = nv[i];
                // padding rows (NaN norm) never count
                raised_rows[r] = n < __builtin_huge_valf() ? (n - 2.0f * dot) + gamma * (n + 2.0f * sabs)
                                                           : __builtin_huge_valf();
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    constexpr int PER = kSeedMaxRows / 64;
    float raised[PER];  // this lane's share of the raised values
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const uint32_t r = (uint32_t)l + 64u * i;
        raised[i] = r < total ? raised_rows[r] : __builtin_huge_valf();
    }
    // the R-th smallest: R rounds of a wave minimum, each removing one occurrence
    float T = __builtin_huge_valf();
    for (int rr = 0; rr < R; ++rr) {
        float lm = raised[0];
#pragma unroll
        for (int i = 1; i < PER; ++i) lm = fminf(lm, raised[i]);
        float m = lm;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fminf(m, __shfl_xor(m, o, 64));
        if (!(m < __builtin_huge_valf())) {  // fewer than R seeded rows
            T = __builtin_huge_valf();
            break;
        }
        const uint64_t who = __ballot(lm == m);
        if (l == __ffsll((unsigned long long)who) - 1) {
            bool done = false;
#pragma unroll
            for (int i = 0; i < PER; ++i)
                if (!done && raised[i] == m) {
                    raised[i] = __builtin_huge_valf();
                    done = true;
                }
        }
        T = m;
    }
    if (T < __builtin_huge_valf() && l < R)
        __hip_atomic_fetch_min(a.cmin + (int64_t)l * a.Q + slot, ord_bits(T), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

hipError_t launch_tiled_seed(const SeedArgs& a, int R, int f16in, hipStream_t s) {
    if (a.Q <= 0) return hipSuccess;
    if (a.rows < 64 || a.rows > kSeedMaxRows || a.rows % 64 != 0 || a.L < 1 || a.L > 7) return hipErrorInvalidValue;
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

// The FP32 squared distance of the row at padded position p from its
// row-major codes, where they hold the table's values exactly: the same
// operations in the same ascending order as row_dist_fp32 over the planes
// (the zero components past D add +0), but one contiguous read of the row
// instead of one scattered 16-B read per plane.  dpad is a multiple of 8.
template <bool F16CODES>
__device__ inline float code_row_dist_fp32(const uint16_t* __restrict__ xl, int dk, int64_t p, int dpad,
                                           const float* __restrict__ y) {
#pragma clang fp contract(off)
    const uint4* row = reinterpret_cast<const uint4*>(xl + p * dk);
    const int nu = dpad / 8;  // 16-B units of 8 components
    float acc = 0.0f;
    for (int u0 = 0; u0 < nu; u0 += 8) {
        uint4 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = u0 + j < nu ? row[u0 + j] : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (u0 + j < nu) {
                const uint32_t wv[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint16_t b = (uint16_t)(wv[e / 2] >> (16 * (e & 1)));
                    const float x = F16CODES ? F16::val(b) : __uint_as_float((uint32_t)b << 16);
                    const float d = x - y[(u0 + j) * 8 + e];
                    const float sq = d * d;
                    acc = acc + sq;
                }
            }
        }
    }
    return acc;
}

// One group of G lanes per query: merge the S split lists (ordered by
// (d~, original row)), re-rank the R survivors with the exact FP32
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
    }
    // lane g takes the split lists g, g + G, ... into its own list, two at
    // a time, each list's R entries in 16-byte loads issued together
    auto load_list = [&](int sp, uint4 (&v)[R / 2]) __attribute__((always_inline)) {
        const uint4* src = reinterpret_cast<const uint4*>(f.part + (q * f.S + sp) * R);
#pragma unroll
        for (int i = 0; i < R / 2; ++i) v[i] = src[i];
    };
    auto fold_list = [&](const uint4 (&v)[R / 2]) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const uint32_t db = (k & 1) ? v[k / 2].z : v[k / 2].x, r = (k & 1) ? v[k / 2].w : v[k / 2].y;
            const float d = __uint_as_float(db);
            if (!pair_less(d, r, ld[R - 1], lr[R - 1])) break;  // the list is sorted
            list_insert<R>(ld, lr, d, r);
        }
    };
    for (int sp = g; qv && sp < f.S; sp += 2 * G) {
        uint4 va[R / 2], vb[R / 2];
        const bool two = sp + G < f.S;
        load_list(sp, va);
        if (two) load_list(sp + G, vb);
        fold_list(va);
        if (two) fold_list(vb);
    }
#pragma unroll
    for (int m = 1; m < G; m <<= 1) merge_with<R>(ld, lr, m);
    uint32_t row = 0xFFFFFFFFu;
#pragma unroll
    for (int k = 0; k < R; ++k)
        if (k == g) row = lr[k];
    float cd = __builtin_huge_valf();
    uint32_t cr = 0xFFFFFFFFu;
    if (qv && row != 0xFFFFFFFFu) {
        const uint32_t cp = f.ipos[row];
        const uint32_t pos = f.ppos[cp];
        if (pos != 0xFFFFFFFFu) {  // a padding row never enters a list; checked anyway
            cr = row;
            const float* y = f.yf + q * f.dpad;
            if (f.xl_codes == 1)
                cd = code_row_dist_fp32<true>(f.xl, f.dk, cp, f.dpad, y);
            else if (f.xl_codes == 2)
                cd = code_row_dist_fp32<false>(f.xl, f.dk, cp, f.dpad, y);
            else
                cd = row_dist_fp32<E>(static_cast<const uint4*>(f.planes), f.N, f.nch, pos, y);
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

template <bool F16IN, int R, int G>
static hipError_t screen_ks(const TiledArgs& a, int ks, dim3 grid, size_t lds, hipStream_t s) {
    switch (ks) {
        case 1: hipLaunchKernelGGL((tiled_screen_kernel<F16IN, 1, R, G>), grid, dim3(256), lds, s, a); break;
        case 2: hipLaunchKernelGGL((tiled_screen_kernel<F16IN, 2, R, G>), grid, dim3(256), lds, s, a); break;
        case 4: hipLaunchKernelGGL((tiled_screen_kernel<F16IN, 4, R, G>), grid, dim3(256), lds, s, a); break;
        case 8: hipLaunchKernelGGL((tiled_screen_kernel<F16IN, 8, R, G>), grid, dim3(256), lds, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Dynamic LDS of the screen kernel: per wave, the marked-cone list of one
// chunk of cones (16 B per cone).
size_t tiled_screen_lds() { return (size_t)4 * kChunk * 16; }

hipError_t launch_tiled_screen(const TiledArgs& a, int R, int G, int f16in, int blocks, hipStream_t s) {
    const int ks = a.dk / 32;
    const size_t lds = tiled_screen_lds();
    const dim3 grid((unsigned)blocks);
    if (!tile_groups_ok(R, G)) return hipErrorInvalidValue;
#define OSANN_SCREEN_PICK(F16IN, RR, GG) \
    if (f16in == (int)F16IN && R == RR && G == GG) return screen_ks<F16IN, RR, GG>(a, ks, grid, lds, s);
    OSANN_SCREEN_PICK(true, 4, 4) OSANN_SCREEN_PICK(true, 4, 2) OSANN_SCREEN_PICK(true, 8, 4)
    OSANN_SCREEN_PICK(true, 8, 2) OSANN_SCREEN_PICK(true, 16, 2) OSANN_SCREEN_PICK(false, 4, 4)
    OSANN_SCREEN_PICK(false, 4, 2) OSANN_SCREEN_PICK(false, 8, 4) OSANN_SCREEN_PICK(false, 8, 2)
    OSANN_SCREEN_PICK(false, 16, 2)
#undef OSANN_SCREEN_PICK
    return hipErrorInvalidValue;
}

template <typename E, int R>
static hipError_t finish_g(const FinishArgs& f, hipStream_t s) {
    // lanes per query: a power of two (the lists are merged over xor partners);
    // lanes past the S lists fold nothing
    const int G = f.S > R ? 16 : R;
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
    if (f.xl_codes != 0 && (f.xl == nullptr || f.dpad % 8 != 0 || f.dpad > f.dk ||
                            f.xl_codes != (f.dtype == kF16 ? 1 : f.dtype == kU8 ? 2 : -1)))
        return hipErrorInvalidValue;
    switch (f.dtype) {
        case kF32: return finish_r<F32>(f, R, s);
        case kF16: return finish_r<F16>(f, R, s);
        case kU8: return finish_r<U8>(f, R, s);
    }
    return hipErrorInvalidValue;
}

#define OSANN_EACH_SCREEN_IN(X, F)                                                                  \
    X(F, 1, 4, 4) X(F, 2, 4, 4) X(F, 4, 4, 4) X(F, 8, 4, 4) X(F, 1, 4, 2) X(F, 2, 4, 2) X(F, 4, 4, 2)          \
    X(F, 8, 4, 2) X(F, 1, 8, 4) X(F, 2, 8, 4) X(F, 4, 8, 4) X(F, 8, 8, 4) X(F, 1, 8, 2) X(F, 2, 8, 2)          \
    X(F, 4, 8, 2) X(F, 8, 8, 2) X(F, 1, 16, 2) X(F, 2, 16, 2) X(F, 4, 16, 2) X(F, 8, 16, 2)
#define OSANN_EACH_SCREEN(X) OSANN_EACH_SCREEN_IN(X, true) OSANN_EACH_SCREEN_IN(X, false)

size_t tiled_screen_static_lds(int R, int G) {
    const size_t qw = 16 * (size_t)G;
    return 4 * qw * R * 8 + 4 * (size_t)kHitCap * 16 + 4 * (64 + (size_t)kHitCap) * 4 + 4 * 64 * kWalkCache * 4 + 512;
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

int tiled_screen_occupancy(int R, int G, int f16in, int ks, size_t lds) {
    int nb = 0;
    const void* fn = nullptr;
#define OSANN_PICK(F16IN, KS, RR, GG) \
    if (f16in == (int)F16IN && ks == KS && R == RR && G == GG) fn = (const void*)tiled_screen_kernel<F16IN, KS, RR, GG>;
    OSANN_EACH_SCREEN(OSANN_PICK)
#undef OSANN_PICK
    if (!fn) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, lds) != hipSuccess) return 0;
    return nb;
}

}  // namespace osann
