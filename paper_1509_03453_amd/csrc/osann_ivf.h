// Internal interface of the coarse-cluster path (ROSANNA+, Section 4.B).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osann {

constexpr int kMaxClusters = 1024;  // centroids of a clustered table (search keeps their distances in LDS)

// Nearest centroid of each row: FP32 term-by-term squared distance, the lower
// centroid on ties.  cent is C x D row-major FP32.
hipError_t launch_assign(const void* X, int dtype, int64_t N, int D, const float* cent, int C, uint32_t* out,
                         hipStream_t s);
// New centroids: float64 sum of each cluster's rows in ascending row order
// (members[offsets[c] .. offsets[c+1]) lists them), divided by their count,
// rounded to FP32; an empty cluster keeps its old centroid.
hipError_t launch_centroid_update(const void* X, int dtype, int64_t N, int D, const uint32_t* members,
                                  const uint32_t* offsets, int C, const float* old_cent, float* new_cent,
                                  hipStream_t s);
// Residual keys of the rows: out[n][j] = x[n][j] - cent[assign[n]][j] (FP32).
hipError_t launch_residual_rows(const void* X, int dtype, int64_t N, int D, const float* cent,
                                const uint32_t* assign, float* out, hipStream_t s);
// Bucket ids of the clustered table: cone[n] += group[n] * n_cones.
hipError_t launch_compose_cones(uint32_t* cone, const uint32_t* group, int64_t N, int64_t n_cones, hipStream_t s);

struct IvfQueryArgs {
    const float* yf;     // [Q][dpad] FP32 queries
    int dpad, D;
    int64_t Q;
    const float* cent;   // [C][D]
    int C, nprobe;
    int64_t n_cones;
    // outputs, per virtual query v = q * nprobe + t (t-th nearest centroid)
    float* yr;           // [Q*nprobe][D] residual y - c
    float* yfv;          // [Q*nprobe][dpad] copy of the query
    uint32_t* cone_base; // [Q*nprobe] c * n_cones
};
// Per query: the nprobe nearest centroids (FP32 distance, lower id on
// ties), in increasing distance, and the virtual queries' inputs.
hipError_t launch_ivf_queries(const IvfQueryArgs& a, hipStream_t s);
// Per query: the smallest (distance, row) of its nprobe virtual results and
// the sum of their candidate counts.
hipError_t launch_ivf_combine(const int64_t* vidx, const float* vdist, const int64_t* vncand, int64_t Q, int nprobe,
                              int64_t* out_idx, float* out_dist, int64_t* out_ncand, hipStream_t s);

}  // namespace osann
