// Entry points whose kernels are not built yet.
#include "kernels.hpp"
#include "ozaki.hpp"

namespace cosma {
}  // namespace cosma

extern "C" {
int cosma_gemm_batched(int64_t, const int64_t*, const int64_t*, const int64_t*, const double*,
                       const void* const*, const int64_t*, const void* const*, const int64_t*,
                       const double*, void* const*, const int64_t*, int, void*) {
  return COSMA_ERR_UNSUPPORTED;
}
int cosma_batch_create(int64_t, const int64_t*, const int64_t*, const int64_t*, const double*,
                       const void* const*, const int64_t*, const void* const*, const int64_t*,
                       const double*, void* const*, const int64_t*, int, void*, void**) {
  return COSMA_ERR_UNSUPPORTED;
}
int cosma_batch_run(void*, void*) { return COSMA_ERR_UNSUPPORTED; }
int cosma_batch_destroy(void*) { return COSMA_ERR_UNSUPPORTED; }
}
