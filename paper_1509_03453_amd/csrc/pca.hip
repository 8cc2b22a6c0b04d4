// PCA front-end (Section 4.B): the principal axes of the database, and keys
// made of the first k principal coordinates of the centred vectors.
//
// Moments: the float64 mean, then the float64 covariance of the centred rows
// (sum of outer products divided by N), each in two fixed-order passes
// (per-block partial sums over row ranges, then one sum over the blocks),
// so the result does not depend on timing.  The eigen-decomposition of the
// D x D covariance runs on the host.
//
// Keys: out[n][i] = sum_j P[i][j] (x[n][j] - mu[j]) in FP32 with ascending
// j, the difference, each product and each sum rounded separately.
#include "osann_device.h"
#include "osann_kernels.h"

namespace osann {

template <typename E>
__global__ void project_kernel(const void* __restrict__ X, int64_t N, int D, const float* __restrict__ mu,
                               const float* __restrict__ P, int k, float* __restrict__ out) {
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * k) return;
    const int64_t n = t / k;
    const int i = (int)(t % k);
    auto x = static_cast<const typename E::raw*>(X) + n * D;
    const float* p = P + (int64_t)i * D;
    float acc = 0.0f;
    for (int j = 0; j < D; ++j) {
        const float c = mu ? E::val(x[j]) - mu[j] : E::val(x[j]);
        const float pr = p[j] * c;
        acc = acc + pr;
    }
    out[t] = acc;
}

hipError_t launch_project(const void* X, int dtype, int64_t N, int D, const float* mu, const float* P, int k,
                          float* out, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const int64_t n = N * k;
    const dim3 grid((unsigned)((n + 255) / 256));
    switch (dtype) {
        case kF32: hipLaunchKernelGGL(project_kernel<F32>, grid, dim3(256), 0, s, X, N, D, mu, P, k, out); break;
        case kF16: hipLaunchKernelGGL(project_kernel<F16>, grid, dim3(256), 0, s, X, N, D, mu, P, k, out); break;
        case kU8: hipLaunchKernelGGL(project_kernel<U8>, grid, dim3(256), 0, s, X, N, D, mu, P, k, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Rows [b*rpb, (b+1)*rpb) of block b: part[b][j] = sum of component j, in
// row order (one thread per component).
template <typename E>
__global__ __launch_bounds__(256) void column_sums_kernel(const void* __restrict__ X, int64_t N, int D, int64_t rpb,
                                                          double* __restrict__ part) {
    const int64_t r0 = (int64_t)blockIdx.x * rpb;
    const int64_t r1 = r0 + rpb < N ? r0 + rpb : N;
    auto x = static_cast<const typename E::raw*>(X);
    for (int j = threadIdx.x; j < D; j += blockDim.x) {
        double acc = 0.0;
        for (int64_t r = r0; r < r1; ++r) acc += (double)E::val(x[r * D + j]);
        part[(int64_t)blockIdx.x * D + j] = acc;
    }
}

constexpr int kCovRows = 32;  // centred rows staged in LDS at a time
constexpr int kCovJ = 64;     // covariance entries (one row i, kCovJ columns j) per thread

// Rows [b*rpb, (b+1)*rpb) of block b (grid x): part[b][i][j] = sum over the
// rows of (x_i - mu_i)(x_j - mu_j) in float64, rows in order.  Thread t of
// grid-y block y takes the pair (i, j0 .. j0 + kCovJ - 1) number
// y * blockDim.x + t of the D x ceil(D / kCovJ) pairs.
template <typename E>
__global__ __launch_bounds__(256) void cov_partial_kernel(const void* __restrict__ X, int64_t N, int D,
                                                          const double* __restrict__ mu, int64_t rpb,
                                                          double* __restrict__ part) {
    __shared__ double c[kCovRows][kMaxD];
    const int jblocks = (D + kCovJ - 1) / kCovJ;
    const int pair = blockIdx.y * blockDim.x + threadIdx.x;
    const bool active = pair < D * jblocks;
    const int i = active ? pair / jblocks : 0;
    const int j0 = active ? (pair % jblocks) * kCovJ : 0;
    const int64_t r0 = (int64_t)blockIdx.x * rpb;
    const int64_t r1 = r0 + rpb < N ? r0 + rpb : N;
    auto x = static_cast<const typename E::raw*>(X);
    double acc[kCovJ];
#pragma unroll
    for (int m = 0; m < kCovJ; ++m) acc[m] = 0.0;
    for (int64_t rb = r0; rb < r1; rb += kCovRows) {
        const int nr = (int)(r1 - rb < kCovRows ? r1 - rb : kCovRows);
        __syncthreads();
        for (int e = threadIdx.x; e < nr * D; e += blockDim.x) {
            const int rr = e / D, jj = e % D;
            c[rr][jj] = (double)E::val(x[(rb + rr) * D + jj]) - mu[jj];
        }
        __syncthreads();
        if (active)
            for (int rr = 0; rr < nr; ++rr) {
                const double ci = c[rr][i];
#pragma unroll
                for (int m = 0; m < kCovJ; ++m)
                    if (j0 + m < D) acc[m] += ci * c[rr][j0 + m];
            }
    }
    if (active)
#pragma unroll
        for (int m = 0; m < kCovJ; ++m)
            if (j0 + m < D) part[((int64_t)blockIdx.x * D + i) * D + j0 + m] = acc[m];
}

// out[e] = scale * sum over b < nb of part[b][e], b in order.
__global__ void sum_blocks_kernel(const double* __restrict__ part, int nb, int64_t ne, double scale,
                                  double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += part[(int64_t)b * ne + e];
    out[e] = acc * scale;
}

int moments_blocks(int64_t N) { return (int)(N < 256 ? 1 : N / 256 < 240 ? N / 256 : 240); }

size_t moments_scratch_doubles(int64_t N, int D) {
    return (size_t)moments_blocks(N) * D * D + (size_t)D;
}

template <typename E>
static hipError_t moments_t(const void* X, int64_t N, int D, double* mean, double* cov, double* scratch,
                            hipStream_t s) {
    const int nb = moments_blocks(N);
    const int64_t rpb = (N + nb - 1) / nb;
    hipLaunchKernelGGL(column_sums_kernel<E>, dim3(nb), dim3(256), 0, s, X, N, D, rpb, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_blocks_kernel, dim3((D + 255) / 256), dim3(256), 0, s, scratch, nb, (int64_t)D,
                       1.0 / (double)N, mean);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int pairs = D * ((D + kCovJ - 1) / kCovJ);
    hipLaunchKernelGGL(cov_partial_kernel<E>, dim3(nb, (pairs + 255) / 256), dim3(256), 0, s, X, N, D, mean, rpb,
                       scratch);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t ne = (int64_t)D * D;
    hipLaunchKernelGGL(sum_blocks_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, scratch, nb, ne,
                       1.0 / (double)N, cov);
    return hipGetLastError();
}

hipError_t launch_moments(const void* X, int dtype, int64_t N, int D, double* mean, double* cov, double* scratch,
                          hipStream_t s) {
    if (N <= 0) return hipErrorInvalidValue;
    switch (dtype) {
        case kF32: return moments_t<F32>(X, N, D, mean, cov, scratch, s);
        case kF16: return moments_t<F16>(X, N, D, mean, cov, scratch, s);
        case kU8: return moments_t<U8>(X, N, D, mean, cov, scratch, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace osann
