// Roofline calibration probes for bench.py (measurement only; not part of
// the search library).
//
//   calib_read_stream  reads a device buffer (several times per launch if
//                      asked) with 16-byte loads spread over the whole chip:
//                      the achievable read bandwidth of HBM (buffer far above
//                      the 256 MB last-level cache) or of that cache (buffer
//                      well below, read many times).
//   calib_mfma         every wave issues back-to-back BF16/FP16 matrix
//                      instructions into independent accumulators, with no
//                      memory traffic: the achievable dense matrix-core rate.
//
// Both return the best time over their repetitions, measured with HIP events
// on a stream of their own.
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

// `passes` passes over the buffer in one launch (a small buffer is read
// many times, so the timed interval is long next to the launch); pass k
// starts k threads' worth of elements further on, so no load repeats the
// previous pass's address in the same thread.
__global__ __launch_bounds__(256) void read_stream_kernel(const uint4* __restrict__ p, size_t n16, int passes,
                                                          uint32_t* __restrict__ sink) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    uint4 a = make_uint4(0, 0, 0, 0), b = a, c = a, d = a;
    for (int k = 0; k < passes; ++k) {
        const size_t shift = ((size_t)k * 256) % n16;
        auto at = [&](size_t j) { j += shift; return j < n16 ? j : j - n16; };
        size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
        for (; i + 3 * stride < n16; i += 4 * stride) {
            const uint4 x0 = p[at(i)], x1 = p[at(i + stride)], x2 = p[at(i + 2 * stride)], x3 = p[at(i + 3 * stride)];
            a.x ^= x0.x; a.y ^= x0.y; a.z ^= x0.z; a.w ^= x0.w;
            b.x ^= x1.x; b.y ^= x1.y; b.z ^= x1.z; b.w ^= x1.w;
            c.x ^= x2.x; c.y ^= x2.y; c.z ^= x2.z; c.w ^= x2.w;
            d.x ^= x3.x; d.y ^= x3.y; d.z ^= x3.z; d.w ^= x3.w;
        }
        for (; i < n16; i += stride) {
            const uint4 x = p[at(i)];
            a.x ^= x.x; a.y ^= x.y; a.z ^= x.z; a.w ^= x.w;
        }
    }
    const uint32_t v = a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
    if (v == 0x9E3779B9u) sink[blockIdx.x % 1024] = v;  // keeps the loads; the buffer's pattern never folds to it
}

template <int SHAPE, bool F16>
__global__ __launch_bounds__(256) void mfma_loop_kernel(int iters, float* __restrict__ sink) {
    constexpr int K = 8;  // independent accumulators per wave, more than the instruction's latency in issues
    const uint32_t l = threadIdx.x % 64;
    const uint4 av = make_uint4(0x3F803F80u ^ l, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u ^ (l << 3));
    const uint4 bv = make_uint4(0x3C003C00u, 0x3C003C00u ^ l, 0x3C003C00u, 0x3C003C00u);
    float total = 0.0f;
    if (SHAPE == 16) {
        f32x4_t acc[K];
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (F16)
                    acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8_t, av),
                                                                    __builtin_bit_cast(f16x8_t, bv), acc[k], 0, 0, 0);
                else
                    acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, av),
                                                                     __builtin_bit_cast(bf16x8_t, bv), acc[k], 0, 0, 0);
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) total += acc[k][0] + acc[k][3];
    } else {
        f32x16_t acc[K / 2];
#pragma unroll
        for (int k = 0; k < K / 2; ++k)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[k][e] = 0.0f;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < K / 2; ++k) {
                if (F16)
                    acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, av),
                                                                    __builtin_bit_cast(f16x8_t, bv), acc[k], 0, 0, 0);
                else
                    acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, av),
                                                                     __builtin_bit_cast(bf16x8_t, bv), acc[k], 0, 0, 0);
            }
        }
#pragma unroll
        for (int k = 0; k < K / 2; ++k) total += acc[k][0] + acc[k][15];
    }
    if (total == 1234.5f) sink[blockIdx.x % 1024] = total;
}

static int num_cu() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return n;
}

template <typename F>
static int best_time(int reps, F&& launch, double* best_ms) {
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipStreamCreate(&s);
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    double best = 1e30;
    for (int r = 0; r <= reps && e == hipSuccess; ++r) {  // r == 0 warms up
        e = hipEventRecord(a, s);
        if (e == hipSuccess) e = launch(s);
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && r > 0 && ms < best) best = ms;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (s) (void)hipStreamDestroy(s);
    *best_ms = best;
    return e == hipSuccess ? 0 : -3;
}

extern "C" {

// Best time of `passes` passes over `bytes` (a multiple of 16) in one
// launch of blocks_per_cu * CUs blocks of 256 threads.
int calib_read_stream(size_t bytes, int passes, int reps, int blocks_per_cu, double* best_ms) {
    const int ncu = num_cu();
    if (!best_ms || bytes < 16 || bytes % 16 || passes < 1 || reps < 1 || blocks_per_cu < 1 || ncu < 1) return -1;
    void* buf = nullptr;
    uint32_t* sink = nullptr;
    if (hipMalloc(&buf, bytes) != hipSuccess) return -2;
    if (hipMalloc((void**)&sink, 4096) != hipSuccess) {
        (void)hipFree(buf);
        return -2;
    }
    int rc = hipMemset(buf, 0x5A, bytes) == hipSuccess && hipDeviceSynchronize() == hipSuccess ? 0 : -3;
    const unsigned blocks = (unsigned)(blocks_per_cu * ncu);
    if (!rc)
        rc = best_time(reps, [&](hipStream_t s) {
            hipLaunchKernelGGL(read_stream_kernel, dim3(blocks), dim3(256), 0, s, (const uint4*)buf, bytes / 16, passes,
                               sink);
            return hipGetLastError();
        }, best_ms);
    (void)hipFree(buf);
    (void)hipFree(sink);
    return rc;
}

// Best time of `iters` loop trips on waves_per_simd * 4 * CUs waves;
// flops_out receives the matrix flops of one launch.
int calib_mfma(int shape, int f16, int iters, int waves_per_simd, int reps, double* best_ms, double* flops_out) {
    const int ncu = num_cu();
    if (!best_ms || !flops_out || (shape != 16 && shape != 32) || iters < 1 || waves_per_simd < 1 ||
        waves_per_simd > 8 || reps < 1 || ncu < 1)
        return -1;
    float* sink = nullptr;
    if (hipMalloc((void**)&sink, 4096) != hipSuccess) return -2;
    const unsigned blocks = (unsigned)(waves_per_simd * ncu);  // 4 waves (one per SIMD) per block
    // per instruction: 16x16x32 and 32x32x16 both take 2*16*16*32 resp. 2*32*32*16 flops
    const double per_instr = shape == 16 ? 2.0 * 16 * 16 * 32 : 2.0 * 32 * 32 * 16;
    const double instr_per_wave = (double)iters * (shape == 16 ? 8 : 4);
    *flops_out = per_instr * instr_per_wave * 4.0 * blocks;
    const int rc = best_time(reps, [&](hipStream_t s) {
        if (shape == 16 && f16) hipLaunchKernelGGL((mfma_loop_kernel<16, true>), dim3(blocks), dim3(256), 0, s, iters, sink);
        if (shape == 16 && !f16) hipLaunchKernelGGL((mfma_loop_kernel<16, false>), dim3(blocks), dim3(256), 0, s, iters, sink);
        if (shape == 32 && f16) hipLaunchKernelGGL((mfma_loop_kernel<32, true>), dim3(blocks), dim3(256), 0, s, iters, sink);
        if (shape == 32 && !f16) hipLaunchKernelGGL((mfma_loop_kernel<32, false>), dim3(blocks), dim3(256), 0, s, iters, sink);
        return hipGetLastError();
    }, best_ms);
    (void)hipFree(sink);
    return rc;
}

}  // extern "C"
