// Internal interface: the order in which the tiled path batches queries.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osann {

// Sort key of each query for cutting the batch into wave tiles.
//   mode 0: its own cone, then its (L+1)-th largest component and that
//     component's sign bit, key = q_cone * 2D + 2 * order[L] + sbit[order[L]]
//     (D > L): queries with equal keys share the start of their walks.
//   mode 1: the sign bits of components 0 .. query_sign_bits(D, Q) - 1, the
//     first the most significant: where a query probes a large share of the
//     cones, its walk covers most pairs of components with its own signs, so
//     queries that agree on many signs probe many of the same cones.
// Sign bits of the mode-1 key: 24 for up to 65,536 queries (about 128 pairs
// of them share 24 random sign bits; one radix pass less), else 32; at most D.
__host__ __device__ inline int query_sign_bits(int D, int64_t Q) {
    const int b = Q <= 65536 ? 24 : 32;
    return D < b ? D : b;
}
hipError_t launch_query_key(const uint32_t* q_cone, const uint8_t* order, const uint8_t* sbit, int64_t Q, int D,
                            int L, int mode, uint32_t* key, hipStream_t s);

}  // namespace osann
