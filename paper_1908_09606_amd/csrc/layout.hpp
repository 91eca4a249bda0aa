// Operand layout adapter (layout.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cosma {

// out (cols x rows, dense) = in^T for `in` of rows x cols with leading
// dimension ld_in.
hipError_t launch_transpose_f64(const double* in, int64_t rows, int64_t cols, int64_t ld_in,
                                double* out, hipStream_t s);
hipError_t launch_transpose_f32(const float* in, int64_t rows, int64_t cols, int64_t ld_in,
                                float* out, hipStream_t s);

}  // namespace cosma
