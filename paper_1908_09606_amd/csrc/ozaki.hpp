// FP64-accurate product from int8 digit slices (Ozaki scheme).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/cosma_mi355.h"

namespace cosma {

int run_ozaki(const cosma_plan_info& plan, double alpha, const void* A, int64_t lda,
              const void* B, int64_t ldb, double beta, void* C, int64_t ldc, void* workspace,
              hipStream_t stream);

}  // namespace cosma
