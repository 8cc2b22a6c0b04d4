// Query order of the tiled path: the key that groups queries into wave tiles.
#include "osann_batch.h"

namespace osann {

__global__ void query_key_kernel(const uint32_t* __restrict__ q_cone, const uint8_t* __restrict__ order,
                                 const uint8_t* __restrict__ sbit, int64_t Q, int D, int L, int mode,
                                 uint32_t* __restrict__ key) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    if (mode == 1) {
        uint32_t k = 0;
        const int nb = query_sign_bits(D, Q);
        for (int i = 0; i < nb; ++i) k = (k << 1) | sbit[q * D + i];
        key[q] = k;
        return;
    }
    const int c = order[q * D + L];
    key[q] = q_cone[q] * (uint32_t)(2 * D) + (uint32_t)(2 * c + sbit[q * D + c]);
}

hipError_t launch_query_key(const uint32_t* q_cone, const uint8_t* order, const uint8_t* sbit, int64_t Q, int D,
                            int L, int mode, uint32_t* key, hipStream_t s) {
    if (Q <= 0) return hipSuccess;
    if (L < 1 || L >= D || mode < 0 || mode > 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(query_key_kernel, dim3((unsigned)((Q + 255) / 256)), dim3(256), 0, s, q_cone, order, sbit, Q, D,
                       L, mode, key);
    return hipGetLastError();
}

}  // namespace osann
