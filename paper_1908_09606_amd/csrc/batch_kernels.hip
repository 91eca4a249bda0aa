// Small kernels around the persistent batched GEMM launches: problem
// descriptors written from kernel arguments, the item -> problem map, and
// the split-K reduction of a batch's split problems.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "tiles.hpp"

namespace cosma {
namespace {

// One block copies the staged descriptors, eight bytes per thread.
__global__ __launch_bounds__(256) void batch_stage_kernel(BatchStage st) {
  constexpr int words = (int)(sizeof(BatchProblem) / sizeof(uint64_t));
  static_assert(sizeof(BatchProblem) % sizeof(uint64_t) == 0, "descriptor size");
  const int total = st.count * words;
  const uint64_t* src = reinterpret_cast<const uint64_t*>(st.p);
  uint64_t* dst = reinterpret_cast<uint64_t*>(st.dst);
  for (int i = threadIdx.x; i < total; i += blockDim.x) dst[i] = src[i];
}

// Block p writes the problem index over its item range.
__global__ __launch_bounds__(256) void batch_expand_kernel(const BatchProblem* __restrict__ probs,
                                                           int32_t* __restrict__ map) {
  const int64_t p = blockIdx.x;
  const BatchProblem& q = probs[p];
  const int64_t items = (int64_t)q.tiles_m * q.tiles_n * q.splits;
  for (int64_t i = threadIdx.x; i < items; i += blockDim.x) map[q.first + i] = (int32_t)p;
}

// blockIdx.y: listed problem; blocks along x stride over its m * n entries.
template <typename T>
__global__ __launch_bounds__(256) void batch_reduce_kernel(BatchReduceArgs r) {
  const BatchProblem& q = r.probs[r.idx[blockIdx.y]];
  const int64_t m = q.m, n = q.n, total = m * n;
  const T* __restrict__ P = static_cast<const T*>(q.P);
  T* __restrict__ C = static_cast<T*>(q.C);
  const T alpha = (T)q.alpha, beta = (T)q.beta;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t row = e / n, col = e - row * n;
    const T* p = P + row * n + col;
    T s = p[0];
    for (int64_t sp = 1; sp < q.splits; ++sp) s += p[sp * total];
    T* c = C + row * q.ldc + col;
    const T v = alpha * s;
    *c = beta != T(0) ? v + beta * *c : v;
  }
}

}  // namespace

hipError_t launch_batch_stage(const BatchStage& st, hipStream_t s) {
  if (st.count <= 0) return hipSuccess;
  if (st.count > kStageProblems) return hipErrorInvalidValue;
  hipLaunchKernelGGL(batch_stage_kernel, dim3(1), dim3(256), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_batch_expand(const BatchProblem* probs, int64_t nprobs, int32_t* map,
                               hipStream_t s) {
  if (nprobs <= 0) return hipSuccess;
  if (nprobs > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(batch_expand_kernel, dim3((unsigned)nprobs), dim3(256), 0, s, probs, map);
  return hipGetLastError();
}

hipError_t launch_batch_reduce(int dtype, const BatchReduceArgs& r, int64_t max_elems,
                               hipStream_t s) {
  if (r.count <= 0) return hipSuccess;
  if (r.count > kReduceList) return hipErrorInvalidValue;
  int64_t bx = (max_elems + 255) / 256;
  if (bx > 2048) bx = 2048;
  if (bx < 1) bx = 1;
  const dim3 grid((unsigned)bx, (unsigned)r.count);
  if (dtype == F64)
    hipLaunchKernelGGL(batch_reduce_kernel<double>, grid, dim3(256), 0, s, r);
  else
    hipLaunchKernelGGL(batch_reduce_kernel<float>, grid, dim3(256), 0, s, r);
  return hipGetLastError();
}

}  // namespace cosma
