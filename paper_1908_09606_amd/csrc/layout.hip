// Operand layout adapter: out = in^T for row-major matrices, so that
// transposed operands of the CBLAS-style entry point reach the row-major
// kernels as op(A) (m x k) and op(B) (k x n).
#include <hip/hip_runtime.h>

#include "layout.hpp"
#include "tiles.hpp"

namespace cosma {
namespace {

constexpr int TT = 64;  // tile edge

// Workgroup per 64 x 64 tile of `in` (rows x cols, leading dimension ld_in),
// flattened grid.  Reads are coalesced along in's rows, writes along out's
// rows (out is cols x rows with leading dimension rows); the LDS tile is
// padded by one element against bank conflicts.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ in, int64_t rows,
                                                        int64_t cols, int64_t ld_in,
                                                        T* __restrict__ out) {
  __shared__ T tile[TT][TT + 1];
  const int64_t tiles_c = ceil_div(cols, TT);
  const int64_t r0 = (int64_t)(blockIdx.x / tiles_c) * TT;
  const int64_t c0 = (int64_t)(blockIdx.x % tiles_c) * TT;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < TT; i += 4) {
    const int64_t r = r0 + i, c = c0 + tx;
    if (r < rows && c < cols) tile[i][tx] = in[r * ld_in + c];
  }
  __syncthreads();
  for (int i = ty; i < TT; i += 4) {
    const int64_t c = c0 + i, r = r0 + tx;  // out row c, column r
    if (c < cols && r < rows) out[c * rows + r] = tile[tx][i];
  }
}

template <typename T>
hipError_t launch_transpose(const T* in, int64_t rows, int64_t cols, int64_t ld_in, T* out,
                            hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int64_t blocks = ceil_div(rows, TT) * ceil_div(cols, TT);
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(transpose_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, in, rows, cols,
                     ld_in, out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_transpose_f64(const double* in, int64_t rows, int64_t cols, int64_t ld_in,
                                double* out, hipStream_t s) {
  return launch_transpose<double>(in, rows, cols, ld_in, out, s);
}

hipError_t launch_transpose_f32(const float* in, int64_t rows, int64_t cols, int64_t ld_in,
                                float* out, hipStream_t s) {
  return launch_transpose<float>(in, rows, cols, ld_in, out, s);
}

}  // namespace cosma
