// Internal interface: the order in which the tiled path batches queries.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osann {

// Sort key of each query for cutting the batch into wave tiles: its own cone,
// then its (L+1)-th largest component and that component's sign bit,
// key = q_cone * 2D + 2 * order[L] + sbit[order[L]] (D > L).  Queries with
// equal keys share the start of their walks more than queries that only
// share a cone, so a tile's queries probe more of the same cones.
hipError_t launch_query_key(const uint32_t* q_cone, const uint8_t* order, const uint8_t* sbit, int64_t Q, int D,
                            int L, uint32_t* key, hipStream_t s);

}  // namespace osann
