// Device fill of seeded synthetic matrices.  Test and benchmark input
// infrastructure only: it holds none of the matrix-multiplication arithmetic.
//
// Implements the counter-based splitmix64 generator described in
// synth/__init__.py (Steele, Lea & Flood, OOPSLA 2014) independently of the
// numpy version; both are bit-checked against each other on sampled indices.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

enum Dist { UNIFORM_F64 = 0, UNIFORM_F32 = 1, WIDE_F64 = 2, INT_F64 = 3, INT_F32 = 4 };

__device__ inline double value_f64(uint64_t h, uint64_t h_exp, int dist, int64_t r) {
  if (dist == UNIFORM_F64) return (double)(h >> 11) * 0x1p-52 - 1.0;
  if (dist == WIDE_F64) {
    double mant = 1.0 + (double)((h >> 11) & ((1ull << 52) - 1)) * 0x1p-52;
    int e = (int)(h_exp % 41ull) - 20;
    double v = ldexp(mant, e);
    return (h >> 63) ? -v : v;
  }
  return (double)((int64_t)(h % (uint64_t)(2 * r + 1)) - r);  // INT_F64
}

__device__ inline float value_f32(uint64_t h, int dist, int64_t r) {
  if (dist == UNIFORM_F32) return (float)(h >> 40) * 0x1p-23f - 1.0f;
  return (float)((int64_t)(h % (uint64_t)(2 * r + 1)) - r);  // INT_F32
}

__global__ void fill_kernel(void* dst, int64_t rows, int64_t cols, int64_t ld, uint64_t key,
                            uint64_t key_exp, int dist, int64_t param) {
  const int64_t total = rows * cols;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t r = i / cols, c = i - r * cols;
    const uint64_t ctr = (uint64_t)(i + 1) * kGamma;
    const uint64_t h = mix64(key + ctr);
    if (dist == UNIFORM_F32 || dist == INT_F32) {
      static_cast<float*>(dst)[r * ld + c] = value_f32(h, dist, param);
    } else {
      const uint64_t he = dist == WIDE_F64 ? mix64(key_exp + ctr) : 0;
      static_cast<double*>(dst)[r * ld + c] = value_f64(h, he, dist, param);
    }
  }
}

}  // namespace

extern "C" {

// Fill the rows x cols matrix at device pointer dst (leading dimension ld,
// elements of the distribution's type) on the given HIP stream.
// Returns 0 on success, -1 on bad arguments, -2 on a HIP error.
int synth_fill(void* dst, int64_t rows, int64_t cols, int64_t ld, uint64_t seed, uint32_t stream,
               int dist, int64_t param, void* hip_stream) {
  if (rows < 0 || cols < 0 || ld < cols || dist < 0 || dist > INT_F32 || param < 0) return -1;
  if (rows == 0 || cols == 0) return 0;
  if (!dst) return -1;
  const uint64_t key = mix64((4 * seed + stream + 1) * kGamma);
  const uint64_t key_exp = mix64((4 * seed + (stream + 8) + 1) * kGamma);
  const int64_t total = rows * cols;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream,
                     dst, rows, cols, ld, key, key_exp, dist, param);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"
