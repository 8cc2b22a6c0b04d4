// Internal interface of the structured bases (Section 3.D: Walsh-Hadamard
// matrices in place of pseudo-random ones).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osann {

// Coordinates of N rows (dtype storage, D a power of two <= 256) in the
// basis H diag(signs): sign flips, then the fast Walsh-Hadamard transform
// (butterflies with strides 1, 2, ..., D/2, each (a, b) -> (a + b, a - b)
// in FP32), without the 1/sqrt(D) factor.  out is [N][D] FP32.
hipError_t launch_wht(const void* X, int dtype, int64_t N, int D, const float* signs, float* out, hipStream_t s);

}  // namespace osann
