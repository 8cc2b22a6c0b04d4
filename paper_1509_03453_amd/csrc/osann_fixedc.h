// Internal interface of the fixed-C cone mode (Section 3, Table III): the
// walk of a query takes a fixed number C of cones, empty ones included,
// instead of stopping when the rows of the probed cones reach a budget.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osann {

struct ConesArgs {
    int64_t Q;               // walks (queries, or (query, cluster) pairs)
    int D, L;                // length of the walk state, cone size
    int64_t n_cones, n_sub;  // N_C and C(D,L)
    int64_t take;            // C: walk positions taken (>= 1)
    const uint32_t* offsets;
    const uint32_t* cone_base;  // [Q] first bucket of each walk's cone ids (null: 0)
    const uint8_t* lexsub;
    const uint8_t* maskord;
    const uint32_t* binom;
    const uint8_t* order;    // [Q][D] walk state written by the probe kernel
    const uint8_t* sbit;     // [Q][D]
    // outputs (any may be null)
    uint32_t* jstop;         // [Q] min(C, N_C)
    uint32_t* nprobe;        // [Q] non-empty cones among them
    int64_t* ncand;          // [Q] rows of those cones
    // optional bitmap of the taken non-empty cones, [Q][nw] words (bit e:
    // the cone whose rank among the non-empty cones is e)
    uint64_t* qbits;
    int64_t nw;
    const uint32_t* ne_id;   // cone -> rank among the non-empty cones
};
hipError_t launch_cones(const ConesArgs& a, hipStream_t s);

}  // namespace osann
