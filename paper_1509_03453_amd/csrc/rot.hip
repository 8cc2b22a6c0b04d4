// Several bases (Section 3.A; Algorithm 1 with R rotations).
//
// Every basis r has its own table, built from the rows' coordinates in that
// basis (row_keys + radix sort + offsets), holding the original rows in its
// bucket order.  A search visits, for l = 0, 1, ... and r = 0..R-1, the l-th
// cone of basis r in the query's Section 3.B order (empty cones included),
// and stops after the cone at which the rows of the visited cones, a row met
// again counting again, reach the budget.  A row is analyzed once: at the
// first (l, r) of that schedule whose cone holds it.  Instead of a per-query
// mark per row, the scan tells that first visit from the row's cones in the
// other bases: the position of a cone in the query's probe order of basis r'
// has a closed form (the inverse of the walk), so the row is skipped when
// some basis r' reaches it at an earlier level, or at the same level with
// r' < r.  Skipping duplicates never changes the arg-min; it saves their
// distances.
#include "osann_device.h"
#include "osann_kernels.h"

namespace osann {

// out[n][i] = sum_j M[i][j] x[n][j] in FP32, ascending j, each product and
// sum rounded separately.  A block of 256 threads takes 64 rows and 64
// output components; for each chunk of 32 j it stages the chunk of the 64
// rows and of the 64 matrix rows in LDS (each element read from memory
// once per block), and thread (tr, ti) adds the chunk's terms, in ascending
// j, to its 4 x 4 sums: rows tr + 16a, components ti + 16b.  Only j < D
// terms are added, so every sum is the same sequence of roundings as the
// plain loop.
constexpr int kRotTile = 64;
constexpr int kRotChunk = 32;

template <typename E>
__global__ __launch_bounds__(256) void rotate_kernel(const void* __restrict__ X, int64_t N, int D,
                                                     const float* __restrict__ M, float* __restrict__ out) {
#pragma clang fp contract(off)
    __shared__ float sx[kRotTile][kRotChunk + 1];  // +1: rows fall in different banks
    __shared__ float sm[kRotTile][kRotChunk + 1];
    const int t = threadIdx.x, ti = t % 16, tr = t / 16;
    const int64_t n0 = (int64_t)blockIdx.x * kRotTile;
    const int i0 = (int)blockIdx.y * kRotTile;
    auto x = static_cast<const typename E::raw*>(X);
    float acc[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[q][b] = 0.0f;
    for (int j0 = 0; j0 < D; j0 += kRotChunk) {
        const int jn = D - j0 < kRotChunk ? D - j0 : kRotChunk;
        for (int e = t; e < kRotTile * kRotChunk; e += 256) {
            const int r = e / kRotChunk, jj = e % kRotChunk;
            const int64_t n = n0 + r;
            const int i = i0 + r;
            sx[r][jj] = n < N && jj < jn ? E::val(x[n * D + j0 + jj]) : 0.0f;
            sm[r][jj] = i < D && jj < jn ? M[(int64_t)i * D + j0 + jj] : 0.0f;
        }
        __syncthreads();
        for (int jj = 0; jj < jn; ++jj) {
            float xv[4], mv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) xv[q] = sx[tr + 16 * q][jj];
#pragma unroll
            for (int b = 0; b < 4; ++b) mv[b] = sm[ti + 16 * b][jj];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const float pr = mv[b] * xv[q];
                    acc[q][b] = acc[q][b] + pr;
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t n = n0 + tr + 16 * q;
        if (n >= N) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + ti + 16 * b;
            if (i < D) out[n * D + i] = acc[q][b];
        }
    }
}

hipError_t launch_rotate(const void* X, int dtype, int64_t N, int D, const float* M, float* out, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (D <= 0 || (N + kRotTile - 1) / kRotTile > 0x7FFFFFFF) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((N + kRotTile - 1) / kRotTile), (unsigned)((D + kRotTile - 1) / kRotTile));
    switch (dtype) {
        case kF32: hipLaunchKernelGGL(rotate_kernel<F32>, grid, dim3(256), 0, s, X, N, D, M, out); break;
        case kF16: hipLaunchKernelGGL(rotate_kernel<F16>, grid, dim3(256), 0, s, X, N, D, M, out); break;
        case kU8: hipLaunchKernelGGL(rotate_kernel<U8>, grid, dim3(256), 0, s, X, N, D, M, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

constexpr int kRotWaves = 4;

// Ranks the D components of one FP32 vector (decreasing magnitude, ties to
// the lower index) into order[rank] = component, sbit[component] = sign bit
// and rank_of[component] = rank.  Called by a whole wave.
__device__ inline void rank_vector(const float* __restrict__ y, int D, uint64_t* keys, uint8_t* order,
                                   uint8_t* sbit, uint8_t* rank_of) {
    const int l = lane_id();
    for (int i = l; i < D; i += 64) {
        const uint32_t b = __float_as_uint(y[i]);
        keys[i] = comp_key(F32::mag(b), i, F32::neg(b));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    for (int i = l; i < D; i += 64) {
        const uint64_t k = keys[i];
        int rank = 0;
        for (int j = 0; j < D; ++j) rank += keys[j] > k;
        order[rank] = (uint8_t)i;
        sbit[i] = (uint8_t)key_sign(k);
        if (rank_of) rank_of[i] = (uint8_t)rank;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// One wave per query: rank the query in every basis (walk state to
// a.order/a.sbit, [Q][R][D]) and find the schedule length: the first slot
// k = l*R + r at which the visited rows reach the budget, plus one.
__global__ __launch_bounds__(64 * kRotWaves) void probe_rot_kernel(RotArgs a) {
    __shared__ uint64_t keys[kRotWaves][kMaxD];
    __shared__ uint8_t order[kRotWaves][kMaxRot][kMaxD];
    __shared__ uint8_t sbit[kRotWaves][kMaxRot][kMaxD];
    const int w = threadIdx.x / 64, l = lane_id();
    const int64_t q = (int64_t)blockIdx.x * kRotWaves + w;
    if (q >= a.Q) return;  // no block barrier in this kernel
    const int D = a.D, R = a.R;
    for (int r = 0; r < R; ++r) {
        rank_vector(a.yr + ((int64_t)r * a.Q + q) * D, D, keys[w], order[w][r], sbit[w][r], nullptr);
        for (int i = l; i < D; i += 64) {
            a.order[(q * R + r) * D + i] = order[w][r][i];
            a.sbit[(q * R + r) * D + i] = sbit[w][r][i];
        }
    }
    const int64_t nslots = (int64_t)R * a.n_cones;
    const uint64_t budget = (uint64_t)a.budget;
    uint64_t carry = 0;
    uint32_t stop_at = (uint32_t)nslots;
    for (int64_t k0 = 0; k0 < nslots; k0 += 64) {
        const int64_t k = k0 + l;
        uint32_t len = 0;
        if (k < nslots) {
            const int r = (int)(k % R);
            const int64_t lv = k / R;
            const uint32_t c = probe_cone(lv, a.L, order[w][r], sbit[w][r], a.n_sub, a.lexsub, a.maskord, a.binom);
            const uint32_t* off = a.offsets + (int64_t)r * (a.n_cones + 1);
            len = off[c + 1] - off[c];
        }
        const uint32_t incl = wave_incl_scan(len);
        const uint64_t reached = __ballot(k < nslots && carry + incl >= budget);
        if (reached) {
            stop_at = (uint32_t)(k0 + __ffsll((unsigned long long)reached));
            carry += shfl_u32(incl, __ffsll((unsigned long long)reached) - 1);
            break;
        }
        carry += shfl_u32(incl, 63);
    }
    if (l == 0) {
        a.kstop[q] = stop_at;
        if (a.visited) a.visited[q] = (int64_t)carry;
    }
}

// Position of a row's cone in the query's probe order of one basis (the
// inverse of probe_cone): top = the row's L largest components in that basis
// (packed 9-bit (index, sign bit) pairs), rank_of/sbit = the query's ranks
// and sign bits by component in that basis.  With T = the row's components'
// query ranks in ascending order and the mask of signs that differ from the
// query's (bit L-1-b for T_b): block h = popcount(mask) starts at
// C(D,L) * (C(L,0) + .. + C(L,h-1)); inside it, T's lexicographic rank times
// C(L,h) plus the mask's rank among the masks of popcount h.
__device__ inline int64_t walk_position(uint64_t top, int L, int D, const uint8_t* rank_of, const uint8_t* sbit,
                                        int64_t n_sub, const uint32_t* __restrict__ binom, const uint8_t* mrank,
                                        const uint32_t* hstart) {
    int t[7], f[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        t[j] = 0x7FFF;
        f[j] = 0;
        if (j < L) {
            const uint32_t pr = (uint32_t)(top >> (9 * j)) & 0x1FFu;
            const int idx = (int)(pr & 0xFFu);
            t[j] = rank_of[idx];
            f[j] = (int)(pr >> 8) ^ (int)sbit[idx];
        }
    }
#pragma unroll
    for (int x = 1; x < 7; ++x)
#pragma unroll
        for (int y = 6; y >= x; --y)
            if (t[y - 1] > t[y]) {
                int u = t[y]; t[y] = t[y - 1]; t[y - 1] = u;
                u = f[y]; f[y] = f[y - 1]; f[y - 1] = u;
            }
    int mask = 0;
    int64_t colex = 0;
#pragma unroll
    for (int j = 0; j < 7; ++j)
        if (j < L) {
            mask |= f[j] << (L - 1 - j);
            // lexicographic rank of T = C(D,L) - 1 - colex rank of {D-1-T}
            colex += binom[(D - 1 - t[L - 1 - j]) * 8 + j + 1];
        }
    const int h = __popc(mask);
    const int64_t lex = n_sub - 1 - colex;
    return n_sub * (int64_t)hstart[h] + lex * (int64_t)binom[L * 8 + h] + mrank[mask];
}

// The NCH 16-byte chunks of the row at position pos of a chunk-major table.
template <int NCH>
__device__ inline void rot_row_load(const uint4* __restrict__ planes, int64_t N, int64_t pos, uint4 (&v)[NCH]) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) v[c] = planes[(int64_t)c * N + pos];
}

// Squared FP32 distance of loaded chunks to y (term by term, ascending
// components, each subtraction, product and sum rounded).
template <typename E, int NCH>
__device__ inline float rot_row_dist(const uint4 (&v)[NCH], const float* y) {
#pragma clang fp contract(off)
    constexpr int EPC = Unpack<E>::n;
    float acc = 0.0f;
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
    return acc;
}

// Cross-basis tops fetched together with the row (the others, if R > kRotPre + 1,
// as the checks reach them).
constexpr int kRotPre = 3;

// One to four waves per query.  The schedule's slots are taken 64 at a time
// (cone starts and running row counts in LDS); lane f of the query's waves
// takes rows f, f + 64*wpq, ... of that chunk through a cursor over the
// running counts.  A row is skipped if another basis reaches it first, else
// its FP32 distance feeds the arg-min on (distance, original row).  The
// walk state of the block's queries (order, sign bits and ranks per basis,
// 3 * R * D bytes per query) sits in dynamic LDS sized for this R and D, so
// that many blocks share a compute unit; registers are capped for four waves
// per SIMD (the row chunks of a visit are in flight together with its tops).
template <typename E, int NCH>
__global__ __launch_bounds__(256, 4) void scan_rot_kernel(RotArgs a) {
    extern __shared__ uint8_t walk_lds[];  // [qpb][3][R][D]
    __shared__ float ys[4][kMaxD];
    __shared__ const uint4* s_planes[kMaxRot];
    __shared__ uint32_t s_start[4][64];
    __shared__ uint32_t s_incl[4][64];
    __shared__ uint8_t mrank[128];
    __shared__ uint32_t hstart[8];
    __shared__ float red_d[4];
    __shared__ uint32_t red_r[4], red_n[4];
    const int wpq = a.waves_per_query;
    const int qpb = 4 / wpq;
    const int w = threadIdx.x / 64, l = lane_id();
    const int slot = w / wpq, sub = w % wpq;
    const int64_t q = (int64_t)blockIdx.x * qpb + slot;
    const bool qv = q < a.Q;
    const int D = a.D, R = a.R, L = a.L;
    uint8_t* const w_order = walk_lds + (size_t)slot * 3 * R * D;
    uint8_t* const w_sbit = w_order + R * D;
    uint8_t* const w_rank = w_sbit + R * D;
    if (threadIdx.x < 128) {  // rank of each mask among the masks of its popcount
        const int m = threadIdx.x;
        int c = 0;
        for (int v = 0; v < m; ++v) c += __popc(v) == __popc(m);
        mrank[m] = (uint8_t)c;
    }
    if (threadIdx.x < R) s_planes[threadIdx.x] = a.planes_tab[threadIdx.x];
    if (threadIdx.x < 8) {
        uint32_t s = 0;
        for (int h = 0; h < (int)threadIdx.x; ++h) s += a.binom[L * 8 + h];
        hstart[threadIdx.x] = s;
    }
    for (int i = sub * 64 + l; i < a.dpad; i += wpq * 64) ys[slot][i] = qv ? a.yf[q * a.dpad + i] : 0.0f;
    for (int r = 0; r < R; ++r)
        for (int i = sub * 64 + l; i < D; i += wpq * 64) {
            const uint8_t o = qv ? a.order[(q * R + r) * D + i] : (uint8_t)i;
            w_order[r * D + i] = o;
            w_rank[r * D + o] = (uint8_t)i;
            w_sbit[r * D + i] = qv ? a.sbit[(q * R + r) * D + i] : 0;
        }
    __syncthreads();
    const float* y = ys[slot];
    const int64_t kstop = qv ? a.kstop[q] : 0;
    float best = __builtin_huge_valf();
    uint32_t brow = 0xFFFFFFFFu;
    uint32_t analyzed = 0;
    uint32_t* st = s_start[w];
    uint32_t* in = s_incl[w];
    for (int64_t k0 = 0; k0 < kstop; k0 += 64) {
        const int64_t kl = k0 + l;
        uint32_t start = 0, len = 0;
        if (kl < kstop) {
            const int r = (int)(kl % R);
            const uint32_t c = probe_cone(kl / R, L, w_order + r * D, w_sbit + r * D, a.n_sub, a.lexsub, a.maskord,
                                          a.binom);
            const uint32_t* off = a.offsets + (int64_t)r * (a.n_cones + 1);
            start = off[c];
            len = off[c + 1] - start;
        }
        const uint32_t incl = wave_incl_scan(len);
        st[l] = start;
        in[l] = incl;
        const uint32_t total = shfl_u32(incl, 63);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        uint32_t k = 0;
        for (uint32_t f = sub * 64 + l; f < total; f += wpq * 64) {
            while (in[k] <= f) ++k;
            const uint32_t before = k ? in[k - 1] : 0u;
            const int64_t kk = k0 + k;
            const int r = (int)(kk % R);
            const int64_t lv = kk / R;
            const int64_t p = (int64_t)st[k] + (f - before);
            // every load of this visit at once: the row's tops in (up to
            // kRotPre) other bases and, speculatively, the row itself
            const uint64_t* xt = a.xtop + (int64_t)r * R * a.N + p;
            uint64_t tops[kRotPre];
#pragma unroll
            for (int t = 0; t < kRotPre; ++t) {
                const int r2 = t < r ? t : t + 1;  // the t-th basis other than r
                tops[t] = r2 < R ? xt[(int64_t)r2 * a.N] : 0;
            }
            uint4 v[NCH ? NCH : 1];
            if (NCH) rot_row_load<NCH ? NCH : 1>(s_planes[r], a.N, p, v);
            // a row is analyzed at its first visit: no other basis r2 reaches
            // it at an earlier level, or at this level with r2 < r
            bool first = true;
            auto check = [&](int r2, uint64_t top) {
                const int64_t pos2 = walk_position(top, L, D, w_rank + r2 * D, w_sbit + r2 * D, a.n_sub, a.binom,
                                                   mrank, hstart);
                first = !(pos2 < lv || (pos2 == lv && r2 < r));
            };
#pragma unroll
            for (int t = 0; t < kRotPre; ++t)
                if (first && t < R - 1) check(t < r ? t : t + 1, tops[t]);
            for (int t = kRotPre; t < R - 1 && first; ++t) {
                const int r2 = t < r ? t : t + 1;
                check(r2, xt[(int64_t)r2 * a.N]);
            }
            if (!first) continue;
            ++analyzed;
            const float d = NCH ? rot_row_dist<E, NCH ? NCH : 1>(v, y)
                                : row_dist_fp32<E>(s_planes[r], a.N, a.nch, p, y);
            if (d <= best) {
                const uint32_t row = a.perm[(int64_t)r * a.N + p];
                if (d < best || row < brow) {
                    best = d;
                    brow = row;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    wave_argmin(best, brow);
    uint32_t tot = analyzed;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) tot += (uint32_t)__shfl_xor((int)tot, o, 64);
    if (wpq > 1) {
        if (l == 0) {
            red_d[w] = best;
            red_r[w] = brow;
            red_n[w] = tot;
        }
        __syncthreads();
        if (sub == 0 && l == 0)
            for (int o = 1; o < wpq; ++o) {
                const float od = red_d[w + o];
                const uint32_t orow = red_r[w + o];
                tot += red_n[w + o];
                if (od < best || (od == best && orow < brow)) {
                    best = od;
                    brow = orow;
                }
            }
    }
    if (qv && sub == 0 && l == 0) {
        a.out_idx[q] = brow == 0xFFFFFFFFu ? -1 : (int64_t)brow;
        a.out_dist[q] = best;
        if (a.out_ncand) a.out_ncand[q] = tot;
    }
}

hipError_t launch_probe_rot(const RotArgs& a, hipStream_t s) {
    if (a.Q <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.Q + kRotWaves - 1) / kRotWaves));
    hipLaunchKernelGGL(probe_rot_kernel, grid, dim3(64 * kRotWaves), 0, s, a);
    return hipGetLastError();
}

template <typename E>
static hipError_t dispatch_scan_rot(const RotArgs& a, hipStream_t s) {
    const int qpb = 4 / a.waves_per_query;
    const dim3 grid((unsigned)((a.Q + qpb - 1) / qpb)), block(256);
    const size_t lds = (size_t)qpb * 3 * a.R * a.D;
    switch (a.nch) {
#define OSANN_ROT_CASE(C)                                                     \
    case C:                                                                   \
        hipLaunchKernelGGL((scan_rot_kernel<E, C>), grid, block, lds, s, a);  \
        break;
        OSANN_ROT_CASE(1) OSANN_ROT_CASE(2) OSANN_ROT_CASE(4) OSANN_ROT_CASE(8) OSANN_ROT_CASE(16)
#undef OSANN_ROT_CASE
        default:
            hipLaunchKernelGGL((scan_rot_kernel<E, 0>), grid, block, lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_scan_rot(const RotArgs& a, hipStream_t s) {
    if (a.Q <= 0) return hipSuccess;
    if (a.waves_per_query != 1 && a.waves_per_query != 2 && a.waves_per_query != 4) return hipErrorInvalidValue;
    switch (a.dtype) {
        case kF32: return dispatch_scan_rot<F32>(a, s);
        case kF16: return dispatch_scan_rot<F16>(a, s);
        case kU8: return dispatch_scan_rot<U8>(a, s);
    }
    return hipErrorInvalidValue;
}

// Gathers, for the rows of basis r's table in its order, their packed top-L
// pairs in basis r2: xt[p] = top2[perm[p]].
__global__ void gather_top_kernel(const uint32_t* __restrict__ perm, int64_t N, const uint64_t* __restrict__ top2,
                                  uint64_t* __restrict__ xt) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) xt[p] = top2[perm[p]];
}

hipError_t launch_gather_top(const uint32_t* perm, int64_t N, const uint64_t* top2, uint64_t* xt, hipStream_t s) {
    hipLaunchKernelGGL(gather_top_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, perm, N, top2, xt);
    return hipGetLastError();
}

}  // namespace osann
