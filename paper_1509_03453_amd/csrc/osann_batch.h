// Internal interface: the order in which the tiled path batches queries.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osann {

// Sort key of each query for cutting the batch into wave tiles.
//   mode 0: its own cone, then its (L+1)-th largest component and that
//     component's sign bit, key = q_cone * 2D + 2 * order[L] + sbit[order[L]]
//     (D > L): queries with equal keys share the start of their walks.
//   mode 1: the sign bits of components 0 .. min(D, 32) - 1, the first the
//     most significant: where a query probes a large share of the cones, its
//     walk covers most pairs of components with its own signs, so queries
//     that agree on many signs probe many of the same cones.
hipError_t launch_query_key(const uint32_t* q_cone, const uint8_t* order, const uint8_t* sbit, int64_t Q, int D,
                            int L, int mode, uint32_t* key, hipStream_t s);

}  // namespace osann
