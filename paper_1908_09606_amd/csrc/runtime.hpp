// Internal runtime interface shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/cosma_mi355.h"

namespace cosma {

int current_device();
cosma_device_facts device_facts(int* status);
bool workspace_for_current(void** ptr, size_t* bytes);
// Plan for the current device; a_pitch_bytes = lda * element size (0: dense).
int plan_cached(int64_t m, int64_t n, int64_t k, int dtype, cosma_plan_info* out,
                int64_t a_pitch_bytes = 0);
int check_plan(const cosma_plan_info* p);
int map_hip(hipError_t e);
int run_plan(const cosma_plan_info& plan, double alpha, const void* A, int64_t lda, const void* B,
             int64_t ldb, double beta, void* C, int64_t ldc, hipStream_t stream);
int run_plan_ws(const cosma_plan_info& plan, double alpha, const void* A, int64_t lda,
                const void* B, int64_t ldb, double beta, void* C, int64_t ldc, void* ws,
                size_t ws_bytes, hipStream_t stream);
int check_args(int64_t m, int64_t n, int64_t k, double alpha, const void* A, int64_t lda,
               const void* B, int64_t ldb, double beta, const void* C, int64_t ldc, int dtype);

}  // namespace cosma
