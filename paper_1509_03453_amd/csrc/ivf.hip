// Coarse clusters (ROSANNA+, Section 4.B): the database is split by k-means,
// each row is hashed on its residual to its centroid, and the buckets are
// (cluster, cone).  A query is compared with every centroid, and each of the
// nprobe nearest clusters is searched as its own "virtual query" (the
// query's residual walks that cluster's cones, the scan compares full
// vectors); a last pass keeps the best of the virtual results.
//
// Every floating-point decision (nearest centroid, residuals, centroid
// means) follows one fixed order, so results do not depend on timing.
#include "osann_device.h"
#include "osann_kernels.h"
#include "osann_ivf.h"

namespace osann {

// Squared distance of an FP32 vector to a row in FP32, ascending j, each
// subtraction, product and sum rounded.
template <typename E>
__global__ void assign_kernel(const void* __restrict__ X, int64_t N, int D, const float* __restrict__ cent, int C,
                              uint32_t* __restrict__ out) {
#pragma clang fp contract(off)
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    auto x = static_cast<const typename E::raw*>(X) + n * D;
    float best = __builtin_huge_valf();
    uint32_t bc = 0;
    for (int c = 0; c < C; ++c) {
        const float* m = cent + (int64_t)c * D;
        float acc = 0.0f;
        for (int j = 0; j < D; ++j) {
            const float df = E::val(x[j]) - m[j];
            const float sq = df * df;
            acc = acc + sq;
        }
        if (acc < best) {
            best = acc;
            bc = (uint32_t)c;
        }
    }
    out[n] = bc;
}

// The same decision with the row held in registers and the centroids staged
// through LDS 32 at a time (every lane reads the same centroid element: a
// broadcast); the j loop runs over the row's D components in order.
template <typename E, int DMAX>
__global__ __launch_bounds__(256) void assign_reg_kernel(const void* __restrict__ X, int64_t N, int D,
                                                         const float* __restrict__ cent, int C,
                                                         uint32_t* __restrict__ out) {
#pragma clang fp contract(off)
    constexpr int CT = 32;
    __shared__ float sc[CT][DMAX];
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = n < N;
    float xr[DMAX];
    auto x = static_cast<const typename E::raw*>(X) + (valid ? n : 0) * D;
#pragma unroll
    for (int j = 0; j < DMAX; ++j) xr[j] = j < D && valid ? E::val(x[j]) : 0.0f;
    float best = __builtin_huge_valf();
    uint32_t bc = 0;
    for (int c0 = 0; c0 < C; c0 += CT) {
        const int nt = C - c0 < CT ? C - c0 : CT;
        __syncthreads();
        for (int e = threadIdx.x; e < nt * D; e += blockDim.x) sc[e / D][e % D] = cent[(int64_t)c0 * D + e];
        __syncthreads();
        if (valid)
            for (int ci = 0; ci < nt; ++ci) {
                float acc = 0.0f;
#pragma unroll
                for (int j = 0; j < DMAX; ++j)
                    if (j < D) {
                        const float df = xr[j] - sc[ci][j];
                        const float sq = df * df;
                        acc = acc + sq;
                    }
                if (acc < best) {
                    best = acc;
                    bc = (uint32_t)(c0 + ci);
                }
            }
    }
    if (valid) out[n] = bc;
}

template <typename E>
static void assign_t(const void* X, int64_t N, int D, const float* cent, int C, uint32_t* out, hipStream_t s) {
    const dim3 grid((unsigned)((N + 255) / 256));
    if (D <= 64)
        hipLaunchKernelGGL((assign_reg_kernel<E, 64>), grid, dim3(256), 0, s, X, N, D, cent, C, out);
    else if (D <= 128)
        hipLaunchKernelGGL((assign_reg_kernel<E, 128>), grid, dim3(256), 0, s, X, N, D, cent, C, out);
    else
        hipLaunchKernelGGL(assign_kernel<E>, grid, dim3(256), 0, s, X, N, D, cent, C, out);
}

hipError_t launch_assign(const void* X, int dtype, int64_t N, int D, const float* cent, int C, uint32_t* out,
                         hipStream_t s) {
    if (N <= 0) return hipSuccess;
    switch (dtype) {
        case kF32: assign_t<F32>(X, N, D, cent, C, out, s); break;
        case kF16: assign_t<F16>(X, N, D, cent, C, out, s); break;
        case kU8: assign_t<U8>(X, N, D, cent, C, out, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// One block per cluster, one thread per component: the members are visited
// in ascending row order (a stable sort by cluster keeps it).
template <typename E>
__global__ __launch_bounds__(256) void centroid_update_kernel(const void* __restrict__ X, int D,
                                                              const uint32_t* __restrict__ members,
                                                              const uint32_t* __restrict__ offsets,
                                                              const float* __restrict__ old_cent,
                                                              float* __restrict__ new_cent) {
    const int c = blockIdx.x;
    const uint32_t b = offsets[c], e = offsets[c + 1];
    auto x = static_cast<const typename E::raw*>(X);
    for (int j = threadIdx.x; j < D; j += blockDim.x) {
        double acc = 0.0;
        for (uint32_t i = b; i < e; ++i) acc += (double)E::val(x[(int64_t)members[i] * D + j]);
        new_cent[(int64_t)c * D + j] = e > b ? (float)(acc / (double)(e - b)) : old_cent[(int64_t)c * D + j];
    }
}

hipError_t launch_centroid_update(const void* X, int dtype, int64_t N, int D, const uint32_t* members,
                                  const uint32_t* offsets, int C, const float* old_cent, float* new_cent,
                                  hipStream_t s) {
    (void)N;
    if (C <= 0) return hipSuccess;
    const dim3 grid((unsigned)C);
    switch (dtype) {
        case kF32:
            hipLaunchKernelGGL(centroid_update_kernel<F32>, grid, dim3(256), 0, s, X, D, members, offsets, old_cent,
                               new_cent);
            break;
        case kF16:
            hipLaunchKernelGGL(centroid_update_kernel<F16>, grid, dim3(256), 0, s, X, D, members, offsets, old_cent,
                               new_cent);
            break;
        case kU8:
            hipLaunchKernelGGL(centroid_update_kernel<U8>, grid, dim3(256), 0, s, X, D, members, offsets, old_cent,
                               new_cent);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename E>
__global__ void residual_rows_kernel(const void* __restrict__ X, int64_t N, int D, const float* __restrict__ cent,
                                     const uint32_t* __restrict__ assign, float* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * D) return;
    const int64_t n = t / D;
    const int j = (int)(t % D);
    out[t] = E::val(static_cast<const typename E::raw*>(X)[t]) - cent[(int64_t)assign[n] * D + j];
}

hipError_t launch_residual_rows(const void* X, int dtype, int64_t N, int D, const float* cent,
                                const uint32_t* assign, float* out, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const dim3 grid((unsigned)((N * D + 255) / 256));
    switch (dtype) {
        case kF32: hipLaunchKernelGGL(residual_rows_kernel<F32>, grid, dim3(256), 0, s, X, N, D, cent, assign, out); break;
        case kF16: hipLaunchKernelGGL(residual_rows_kernel<F16>, grid, dim3(256), 0, s, X, N, D, cent, assign, out); break;
        case kU8: hipLaunchKernelGGL(residual_rows_kernel<U8>, grid, dim3(256), 0, s, X, N, D, cent, assign, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

__global__ void compose_cones_kernel(uint32_t* __restrict__ cone, const uint32_t* __restrict__ group, int64_t N,
                                     int64_t n_cones) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) cone[n] = (uint32_t)((int64_t)group[n] * n_cones + cone[n]);
}

hipError_t launch_compose_cones(uint32_t* cone, const uint32_t* group, int64_t N, int64_t n_cones, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(compose_cones_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, cone, group, N,
                       n_cones);
    return hipGetLastError();
}

constexpr int kMaxProbeClusters = 64;

// One wave per query: lanes compute the distances to centroids l, l + 64,
// ... once into LDS; the nprobe nearest are then picked one at a time by a
// wave arg-min on (distance, id) over the centroids not yet picked.
__global__ __launch_bounds__(256) void ivf_queries_kernel(IvfQueryArgs a) {
#pragma clang fp contract(off)
    __shared__ float s_dist[4][kMaxClusters];
    __shared__ int s_sel[4][kMaxProbeClusters];
    const int w = threadIdx.x / 64, l = lane_id();
    const int64_t q = (int64_t)blockIdx.x * 4 + w;
    if (q >= a.Q) return;
    const float* y = a.yf + q * a.dpad;
    for (int c = l; c < a.C; c += 64) {
        const float* m = a.cent + (int64_t)c * a.D;
        float acc = 0.0f;
        for (int j = 0; j < a.D; ++j) {
            const float df = y[j] - m[j];
            const float sq = df * df;
            acc = acc + sq;
        }
        s_dist[w][c] = acc;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    uint32_t taken = 0;  // per lane: bit i = centroid l + 64 i already picked (C <= 64 * 32)
    for (int t = 0; t < a.nprobe; ++t) {
        float bd = __builtin_huge_valf();
        int bc = 0x7FFFFFFF;
        for (int c = l, i = 0; c < a.C; c += 64, ++i) {
            if ((taken >> i) & 1u) continue;
            const float d = s_dist[w][c];
            if (d < bd || (d == bd && c < bc)) {
                bd = d;
                bc = c;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const float od = __shfl_xor(bd, o, 64);
            const int oc = __shfl_xor(bc, o, 64);
            if (od < bd || (od == bd && oc < bc)) {
                bd = od;
                bc = oc;
            }
        }
        if (bc % 64 == l) taken |= 1u << (bc / 64);
        if (l == 0) s_sel[w][t] = bc;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    for (int t = 0; t < a.nprobe; ++t) {
        const int c = s_sel[w][t];
        const int64_t v = q * a.nprobe + t;
        const float* m = a.cent + (int64_t)c * a.D;
        for (int j = l; j < a.D; j += 64) a.yr[v * a.D + j] = y[j] - m[j];
        for (int j = l; j < a.dpad; j += 64) a.yfv[v * a.dpad + j] = y[j];
        if (l == 0) a.cone_base[v] = (uint32_t)((int64_t)c * a.n_cones);
    }
}

hipError_t launch_ivf_queries(const IvfQueryArgs& a, hipStream_t s) {
    if (a.Q <= 0) return hipSuccess;
    if (a.nprobe < 1 || a.nprobe > kMaxProbeClusters || a.nprobe > a.C || a.C > kMaxClusters)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(ivf_queries_kernel, dim3((unsigned)((a.Q + 3) / 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

__global__ void ivf_combine_kernel(const int64_t* __restrict__ vidx, const float* __restrict__ vdist,
                                   const int64_t* __restrict__ vncand, int64_t Q, int nprobe,
                                   int64_t* __restrict__ out_idx, float* __restrict__ out_dist,
                                   int64_t* __restrict__ out_ncand) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    float bd = __builtin_huge_valf();
    int64_t bi = -1;
    int64_t nc = 0;
    for (int t = 0; t < nprobe; ++t) {
        const int64_t v = q * nprobe + t;
        const float d = vdist[v];
        const int64_t i = vidx[v];
        nc += vncand[v];
        if (i < 0) continue;
        if (bi < 0 || d < bd || (d == bd && i < bi)) {
            bd = d;
            bi = i;
        }
    }
    out_idx[q] = bi;
    out_dist[q] = bd;
    if (out_ncand) out_ncand[q] = nc;
}

hipError_t launch_ivf_combine(const int64_t* vidx, const float* vdist, const int64_t* vncand, int64_t Q, int nprobe,
                              int64_t* out_idx, float* out_dist, int64_t* out_ncand, hipStream_t s) {
    if (Q <= 0) return hipSuccess;
    hipLaunchKernelGGL(ivf_combine_kernel, dim3((unsigned)((Q + 255) / 256)), dim3(256), 0, s, vidx, vdist, vncand,
                       Q, nprobe, out_idx, out_dist, out_ncand);
    return hipGetLastError();
}

}  // namespace osann
