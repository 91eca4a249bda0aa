// FP64-accurate products on the int8 and bf16 matrix cores: digit slices
// (Ozaki scheme, int8 or bf16 digits) and modular residues (Ozaki scheme II).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/cosma_mi355.h"

namespace cosma {

// Digit-slice path (dtype COSMA_F64_OZAKI_I8).
int run_ozaki(const cosma_plan_info& plan, double alpha, const void* A, int64_t lda,
              const void* B, int64_t ldb, double beta, void* C, int64_t ldc, void* workspace,
              hipStream_t stream);

// Modular path (dtype COSMA_F64_OZAKI2_I8).
int run_ozaki2(const cosma_plan_info& plan, double alpha, const void* A, int64_t lda,
               const void* B, int64_t ldb, double beta, void* C, int64_t ldc, void* workspace,
               hipStream_t stream);

// Digit-slice path on the bf16 matrix cores (dtype COSMA_F64_OZAKI_BF16).
int run_ozaki_bf16(const cosma_plan_info& plan, double alpha, const void* A, int64_t lda,
                   const void* B, int64_t ldb, double beta, void* C, int64_t ldc,
                   void* workspace, hipStream_t stream);

// Row exponents of A (e[i]: max_t |A[i][t]| < 2^e[i]) and column exponents
// of B (f[j]); all-zero rows and columns get 0, rows and columns holding a
// NaN or an infinity get OZAKI_NONFINITE (their digits / residues are then
// zero and their row / column of C is NaN).  Shared by both paths.
constexpr int OZAKI_NONFINITE = 0x7fffffff;
hipError_t launch_ozaki_exponents(const double* A, int64_t m, int64_t k, int64_t lda,
                                  const double* B, int64_t n, int64_t ldb, int* e, int* f,
                                  hipStream_t stream);

}  // namespace cosma
