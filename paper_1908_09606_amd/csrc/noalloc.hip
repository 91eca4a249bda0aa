// cosma_gemm without a caller workspace, for callers that cannot allocate
// device memory (code that must not call hipMalloc, e.g. under graph
// capture, in a serving loop, or in a harness that forbids it).
//
// The workspace of the product's schedule (split-K partials, BF16x3 planes,
// Ozaki digit / residue planes) lives in `scratch`, a file-scope device
// array of kScratchBytes that the code object carries: each GPU the library
// runs on holds one copy of it until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// for the symbol): the device address of each GPU's copy is looked up once,
// with that GPU current, and used everywhere instead.
//
// Every call on one GPU shares that GPU's copy, which keeps the last
// call's contents; no kernel of the schedule reads workspace it has not
// written in the same call.  Calls that overlap on one GPU (different
// streams, or several host threads) race on it: order them.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/cosma_mi355.h"
#include "planner.hpp"
#include "runtime.hpp"

namespace cosma {
namespace {

constexpr size_t kScratchBytes = COSMA_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxScratchDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current GPU's copy of `scratch` (looked up on the
// first call on that GPU).
int scratch_for_current(void** out) {
  const int dev = current_device();
  if (dev < 0 || dev >= kMaxScratchDevices) return COSMA_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
      return COSMA_ERR_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return COSMA_OK;
}

}  // namespace
}  // namespace cosma

using namespace cosma;

extern "C" {

int cosma_gemm_noalloc(int64_t m, int64_t n, int64_t k, double alpha, const void* A, int64_t lda,
                       const void* B, int64_t ldb, double beta, void* C, int64_t ldc, int dtype,
                       void* stream) {
  int rc = check_args(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
  if (rc != COSMA_OK) return rc;
  if (m == 0 || n == 0) return COSMA_OK;
  int st = COSMA_OK;
  device_facts(&st);
  if (st != COSMA_OK) return st;
  cosma_plan_info plan;
  rc = plan_cached(m, n, k, dtype, &plan, lda * (int64_t)word_bytes(dtype));
  if (rc != COSMA_OK) return rc;
  if (k > 0 && alpha != 0.0 && workspace_bytes(plan) > kScratchBytes) {
    // native dtypes: keep the planner's tile, give up the k split
    if (dtype != F64 && dtype != F32) return COSMA_ERR_WORKSPACE;
    cosma_plan_info whole;
    rc = cosma_plan_make(m, n, k, dtype, plan.tile_id, 1, &whole);
    if (rc != COSMA_OK) return rc;
    plan = whole;
  }
  void* ws = nullptr;
  rc = scratch_for_current(&ws);
  if (rc != COSMA_OK) return rc;
  return run_plan_ws(plan, alpha, A, lda, B, ldb, beta, C, ldc, ws, kScratchBytes,
                     (hipStream_t)stream);
}

}  // extern "C"
