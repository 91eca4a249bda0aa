// FP64-accurate GEMM from int8 digit slices (Ozaki, Ogita, Oishi & Rump,
// "Error-free transformations of matrix multiplication by using fast
// routines of matrix multiplication", Numer. Algorithms 2012; int8 form as in
// Ootomo, Ozaki & Yokota, IJHPCA 2024).
//
//   1. Exponents: e_i with max_t |A[i][t]| < 2^e_i for every row of A and
//      f_j with max_t |B[t][j]| < 2^f_j for every column of B (binary64).
//   2. Digits: x = A[i][t] 2^-e_i lies in (-1, 1); with r_0 = x,
//      d_u = trunc(2^7 r_(u-1)), r_u = 2^7 r_(u-1) - d_u (all exact in
//      binary64), so x = sum_u d_u 2^-7u + r_s 2^-7s and |d_u| <= 127.
//      Same for the columns of B.  Digit planes are int8, k padded to a
//      multiple of 64 with zeros; A planes are [u][row][k], B planes are
//      stored transposed, [u][col][k], so both MFMA operands are
//      k-contiguous 16-byte runs.
//   3. Products: C[i][j] ~ 2^(e_i + f_j) sum_{u+v <= s+1} 2^-7(u+v) (A_u B_v)[i][j].
//      Every A_u B_v is exact in int32 (v_mfma_i32_16x16x64_i8); the pairs of
//      one anti-diagonal d = u + v share the scale 2^-7d, so they accumulate
//      in one int32 register block.  Every 8192 k (|sum| < s 127^2 8192 <
//      2^31) the s diagonal blocks are converted to binary64, scaled and
//      added, smallest scale first, to the binary64 accumulators.
//
// The GEMM keeps its block of C resident and streams k in LDS-staged rounds
// like the other kernels (Algorithm 1 / section 5); binary64 is used only for
// the exponents, the digit extraction, the summation of the int32 products
// and the split-K reduction.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstring>

#include "kernels.hpp"
#include "ozaki.hpp"
#include "planner.hpp"
#include "runtime.hpp"
#include "tiles.hpp"

namespace cosma {
namespace {

typedef int i4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int KPAD = 64;          // digit planes: k padded to a multiple of 64
constexpr int64_t FLUSH_K = 8192;  // int32 diagonal sums flushed every 8192 k

// ---------------------------------------------------------------- exponents
// One wave per row of A: e[i] = exponent of max_t |A[i][t]| (frexp form,
// so max < 2^e); an all-zero row gets 0.
__global__ __launch_bounds__(256) void row_exp_kernel(const double* __restrict__ A, int64_t m,
                                                      int64_t k, int64_t lda, int* __restrict__ e) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= m) return;
  double mx = 0.0;
  for (int64_t t = lane; t < k; t += 64) mx = fmax(mx, fabs(A[row * lda + t]));
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) {
    int ex = 0;
    if (mx > 0.0) frexp(mx, &ex);
    e[row] = ex;
  }
}

__global__ __launch_bounds__(256) void fill_int_kernel(int* __restrict__ p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = v;
}

// Columns of B: thread per column (coalesced across the wave), blockIdx.y
// per chunk of 1024 rows; partial maxima meet in an atomic max.
__global__ __launch_bounds__(256) void col_exp_kernel(const double* __restrict__ B, int64_t k,
                                                      int64_t n, int64_t ldb, int* __restrict__ f) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= n) return;
  const int64_t t0 = (int64_t)blockIdx.y * 1024;
  const int64_t t1 = min64(k, t0 + 1024);
  double mx = 0.0;
  for (int64_t t = t0; t < t1; ++t) mx = fmax(mx, fabs(B[t * ldb + col]));
  int ex = 0;
  if (mx > 0.0) frexp(mx, &ex);
  atomicMax(f + col, ex);
}

// Columns that are entirely zero end with INT_MIN from the fill: use 0.
__global__ __launch_bounds__(256) void fix_exp_kernel(int* __restrict__ f, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < n && f[j] == INT_MIN) f[j] = 0;
}

// ---------------------------------------------------------------- digits
// 16 consecutive values of one row (A) or one column (B) -> s planes of 16
// int8 digits each.
__device__ __forceinline__ void digits16(double (&x)[16], int s, int8_t* __restrict__ out,
                                         int64_t plane_stride) {
  for (int u = 0; u < s; ++u) {
    int8_t d[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const double y = x[e] * 128.0;
      const double q = trunc(y);
      d[e] = (int8_t)(int)q;
      x[e] = y - q;
    }
    i4 packed;
    std::memcpy(&packed, d, 16);
    *reinterpret_cast<i4*>(out + u * plane_stride) = packed;
  }
}

// A: thread per (row, 16-wide k chunk); writes planes[u][row][kc..kc+15].
__global__ __launch_bounds__(256) void slice_a_kernel(const double* __restrict__ A, int64_t m,
                                                      int64_t k, int64_t lda,
                                                      const int* __restrict__ e, int s,
                                                      int8_t* __restrict__ planes, int64_t kp) {
  const int64_t chunks = kp / 16;
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= m * chunks) return;
  const int64_t row = id / chunks, kc = (id - row * chunks) * 16;
  const int sh = -e[row];
  double x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i)
    x[i] = (kc + i < k) ? ldexp(A[row * lda + kc + i], sh) : 0.0;
  digits16(x, s, planes + row * kp + kc, m * kp);
}

// B: thread per (column, 16-wide k chunk), columns fastest across the wave;
// writes the transposed planes[u][col][kc..kc+15].
__global__ __launch_bounds__(256) void slice_b_kernel(const double* __restrict__ B, int64_t k,
                                                      int64_t n, int64_t ldb,
                                                      const int* __restrict__ f, int s,
                                                      int8_t* __restrict__ planes, int64_t kp) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t chunks = kp / 16;
  if (id >= n * chunks) return;
  const int64_t kc = (id / n) * 16, col = id - (id / n) * n;
  const int sh = -f[col];
  double x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i)
    x[i] = (kc + i < k) ? ldexp(B[(kc + i) * ldb + col], sh) : 0.0;
  digits16(x, s, planes + col * kp + kc, n * kp);
}

// ---------------------------------------------------------------- GEMM
// Work item: a 64 x 64 block of C, 4 waves of 32 x 32 (2 x 2 MFMA blocks).
// LDS stage: s planes of A (64 rows) and of B (64 columns), 64 k each, rows
// padded to 80 bytes.
constexpr int OZ_BM = 64, OZ_BN = 64, OZ_BK = 64, OZ_ROW = 80;

struct OzArgs {
  const int8_t* a_planes;  // [s][m][kp]
  const int8_t* b_planes;  // [s][n][kp]
  const int* e;            // row exponents of A
  const int* f;            // column exponents of B
  double* C;
  double* P;
  int64_t m, n, k, kp, ldc;
  int64_t k_split, tiles_m, tiles_n, splits, ldp, split_stride;
  double alpha, beta;
  int group_m, num_xcds;
};

template <int S>
__global__ __launch_bounds__(256) void ozaki_gemm_kernel(OzArgs g) {
  constexpr int PLANE = OZ_BM * OZ_ROW;   // bytes per plane in LDS (BM == BN)
  constexpr int STAGE = 2 * S * PLANE;
  __shared__ __attribute__((aligned(16))) int8_t lds[2][STAGE];

  const int64_t l = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x, g.num_xcds);
  const ItemCoord ic = item_coord(l, g.tiles_m, g.tiles_n, g.group_m);
  const int64_t row0 = ic.tile_row * OZ_BM, col0 = ic.tile_col * OZ_BN;
  const int64_t kbeg = ic.split * g.k_split;
  const int64_t kend = min64(g.k, kbeg + g.k_split);
  const int64_t nk = ceil_div(kend - kbeg, OZ_BK);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;

  // staging map: thread -> (row/col r, 16-byte k chunk)
  const int sr = t >> 2, sk = (t & 3) * 16;
  const bool a_in = row0 + sr < g.m, b_in = col0 + sr < g.n;
  const int8_t* a_src = g.a_planes + (row0 + sr) * g.kp + sk;
  const int8_t* b_src = g.b_planes + (col0 + sr) * g.kp + sk;
  const int64_t a_plane = g.m * g.kp, b_plane = g.n * g.kp;

  i4 acc[S][2][2];
  d4 sum[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      sum[i][j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int d = 0; d < S; ++d) acc[d][i][j] = i4{0, 0, 0, 0};
    }

  i4 ra[S], rb[S];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < S; ++u) {
      ra[u] = a_in ? *reinterpret_cast<const i4*>(a_src + u * a_plane + k0) : i4{0, 0, 0, 0};
      rb[u] = b_in ? *reinterpret_cast<const i4*>(b_src + u * b_plane + k0) : i4{0, 0, 0, 0};
    }
  };
  auto store = [&](int8_t* st) {
#pragma unroll
    for (int u = 0; u < S; ++u) {
      *reinterpret_cast<i4*>(st + u * PLANE + sr * OZ_ROW + sk) = ra[u];
      *reinterpret_cast<i4*>(st + (S + u) * PLANE + sr * OZ_ROW + sk) = rb[u];
    }
  };
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int d = S - 1; d >= 0; --d) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            sum[i][j][v] += ldexp((double)acc[d][i][j][v], -7 * (d + 2));
          acc[d][i][j] = i4{0, 0, 0, 0};
        }
      }
  };

  if (nk > 0) {
    load(kbeg);
    store(lds[0]);
  }
  __syncthreads();
  const int64_t rounds_per_flush = FLUSH_K / OZ_BK;
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    const bool more = kt + 1 < nk;
    if (more) load(kbeg + (kt + 1) * OZ_BK);
    const int8_t* st = lds[cur];
    i4 bfr[S][2];
#pragma unroll
    for (int v = 0; v < S; ++v)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        bfr[v][j] = *reinterpret_cast<const i4*>(st + (S + v) * PLANE +
                                                 (wn * 32 + j * 16 + lr) * OZ_ROW + lg * 16);
#pragma unroll
    for (int u = 0; u < S; ++u) {
      i4 afr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        afr[i] = *reinterpret_cast<const i4*>(st + u * PLANE + (wm * 32 + i * 16 + lr) * OZ_ROW +
                                              lg * 16);
#pragma unroll
      for (int v = 0; v + u < S; ++v)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[u + v][i][j] =
                __builtin_amdgcn_mfma_i32_16x16x64_i8(afr[i], bfr[v][j], acc[u + v][i][j], 0, 0, 0);
    }
    if (more) store(lds[cur ^ 1]);
    if ((kt + 1) % rounds_per_flush == 0) flush();
    __syncthreads();
  }
  flush();

  // epilogue: scale by 2^(e_i + f_j); standard 16x16 output layout
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = col0 + wn * 32 + j * 16 + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + wm * 32 + i * 16 + lg * 4 + v;
        if (row < g.m && col < g.n) {
          const double r = ldexp(sum[i][j][v], g.e[row] + g.f[col]);
          if (g.splits == 1) {
            double* p = g.C + row * g.ldc + col;
            const double y = g.alpha * r;
            *p = g.beta != 0.0 ? y + g.beta * *p : y;
          } else {
            g.P[ic.split * g.split_stride + row * g.ldp + col] = r;
          }
        }
      }
    }
}

unsigned blocks_for(int64_t threads) {
  int64_t b = (threads + 255) / 256;
  return (unsigned)(b < 1 ? 1 : b);
}

template <int S>
hipError_t launch_oz(const OzArgs& g, hipStream_t s) {
  const int64_t items = g.tiles_m * g.tiles_n * g.splits;
  if (items <= 0) return hipSuccess;
  if (items > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ozaki_gemm_kernel<S>, dim3((unsigned)items), dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace

int run_ozaki(const cosma_plan_info& plan, double alpha, const void* A, int64_t lda,
              const void* B, int64_t ldb, double beta, void* C, int64_t ldc, void* workspace,
              hipStream_t stream) {
  const int64_t m = plan.m, n = plan.n, k = plan.k;
  const int s = plan.slices;
  if (s < 1 || s > 8 || plan.tile_m != OZ_BM || plan.tile_n != OZ_BN || plan.tile_k != OZ_BK)
    return COSMA_ERR_INVALID_ARG;
  if (m > INT_MAX / 4 || n > INT_MAX / 4) return COSMA_ERR_UNSUPPORTED;
  const int64_t kp = ceil_div(k, KPAD) * KPAD;
  // workspace layout (matches workspace_bytes): partials | A planes, B planes | e, f
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  char* w = static_cast<char*>(workspace);
  const size_t part = plan.p_k > 1 ? up((size_t)plan.p_k * m * n * sizeof(double)) : 0;
  int8_t* a_planes = reinterpret_cast<int8_t*>(w + part);
  int8_t* b_planes = a_planes + (size_t)s * m * kp;
  int* e = reinterpret_cast<int*>(w + part + up((size_t)s * kp * (m + n)));
  int* f = e + m;
  hipError_t err;

  hipLaunchKernelGGL(row_exp_kernel, dim3((unsigned)ceil_div(m, 4)), dim3(256), 0, stream,
                     static_cast<const double*>(A), m, k, lda, e);
  hipLaunchKernelGGL(fill_int_kernel, dim3(blocks_for(n) > 4096 ? 4096 : blocks_for(n)), dim3(256),
                     0, stream, f, n, INT_MIN);
  hipLaunchKernelGGL(col_exp_kernel, dim3(blocks_for(n), (unsigned)ceil_div(k, 1024)), dim3(256), 0,
                     stream, static_cast<const double*>(B), k, n, ldb, f);
  hipLaunchKernelGGL(fix_exp_kernel, dim3(blocks_for(n)), dim3(256), 0, stream, f, n);
  hipLaunchKernelGGL(slice_a_kernel, dim3(blocks_for(m * (kp / 16))), dim3(256), 0, stream,
                     static_cast<const double*>(A), m, k, lda, e, s, a_planes, kp);
  hipLaunchKernelGGL(slice_b_kernel, dim3(blocks_for(n * (kp / 16))), dim3(256), 0, stream,
                     static_cast<const double*>(B), k, n, ldb, f, s, b_planes, kp);
  if ((err = hipGetLastError()) != hipSuccess) return COSMA_ERR_HIP;

  OzArgs g;
  g.a_planes = a_planes;
  g.b_planes = b_planes;
  g.e = e;
  g.f = f;
  g.C = static_cast<double*>(C);
  g.P = reinterpret_cast<double*>(w);
  g.m = m;
  g.n = n;
  g.k = k;
  g.kp = kp;
  g.ldc = ldc;
  g.k_split = plan.k_split;
  g.tiles_m = plan.p_m;
  g.tiles_n = plan.p_n;
  g.splits = plan.p_k;
  g.ldp = n;
  g.split_stride = m * n;
  g.alpha = alpha;
  g.beta = beta;
  g.group_m = plan.group_m > 0 ? plan.group_m : 1;
  int st = COSMA_OK;
  g.num_xcds = device_facts(&st).num_xcds;
  switch (s) {
    case 1: err = launch_oz<1>(g, stream); break;
    case 2: err = launch_oz<2>(g, stream); break;
    case 3: err = launch_oz<3>(g, stream); break;
    case 4: err = launch_oz<4>(g, stream); break;
    case 5: err = launch_oz<5>(g, stream); break;
    case 6: err = launch_oz<6>(g, stream); break;
    case 7: err = launch_oz<7>(g, stream); break;
    default: err = launch_oz<8>(g, stream); break;
  }
  if (err != hipSuccess) return COSMA_ERR_HIP;
  if (plan.p_k > 1) {
    err = launch_splitk_reduce_f64(g.P, m * n, n, plan.p_k, static_cast<double*>(C), ldc, m, n,
                                   alpha, beta, stream);
    if (err != hipSuccess) return COSMA_ERR_HIP;
  }
  return COSMA_OK;
}

}  // namespace cosma
