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
//      Same for the columns of B.  Digit planes are int8, stored in the
//      GEMM's staging order (one contiguous block per slice, tile and k
//      round; B transposed so that both MFMA operands are k-contiguous).
//   3. Products: C[i][j] ~ 2^(e_i + f_j) sum_{u+v <= s+1} 2^-7(u+v) (A_u B_v)[i][j].
//      Every A_u B_v is exact in int32 (v_mfma_i32_16x16x64_i8); the pairs of
//      one anti-diagonal d = u + v share the scale 2^-7d, so they accumulate
//      in one int32 register block.  A work item covers at most 8192 k
//      (|sum| <= s 127^2 8192 < 2^31); at its end the s diagonal blocks are
//      converted to binary64, scaled and added, smallest scale first.
//      Longer reductions are split and summed by the FP64 split-K reduction.
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

constexpr int64_t MAX_K_ITEM = 8192;  // reduction length per work item (int32 exactness)
constexpr int64_t COL_CHUNK = 256; // rows of B per block of the column-exponent pass

// ---------------------------------------------------------------- exponents
// One wave per row of A: e[i] = exponent of max_t |A[i][t]| (frexp form,
// so max < 2^e); an all-zero row gets 0, a row with a NaN or an infinity
// OZAKI_NONFINITE.
__global__ __launch_bounds__(256) void row_exp_kernel(const double* __restrict__ A, int64_t m,
                                                      int64_t k, int64_t lda, int* __restrict__ e) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= m) return;
  double mx = 0.0;
  bool bad = false;
#pragma unroll 16
  for (int64_t t = lane; t < k; t += 64) {  // unrolled: 16 loads in flight per lane
    const double v = A[row * lda + t];
    bad |= !isfinite(v);
    mx = fmax(mx, fabs(v));
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  bad = __any(bad);
  if (lane == 0) {
    int ex = 0;
    if (mx > 0.0) frexp(mx, &ex);
    e[row] = bad ? OZAKI_NONFINITE : ex;
  }
}

__global__ __launch_bounds__(256) void fill_int_kernel(int* __restrict__ p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = v;
}

// Columns of B: thread per column (coalesced across the wave), blockIdx.y
// per chunk of COL_CHUNK rows; partial maxima meet in an atomic max.
__global__ __launch_bounds__(256) void col_exp_kernel(const double* __restrict__ B, int64_t k,
                                                      int64_t n, int64_t ldb, int* __restrict__ f) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= n) return;
  const int64_t t0 = (int64_t)blockIdx.y * COL_CHUNK;
  const int64_t t1 = min64(k, t0 + COL_CHUNK);
  double mx = 0.0;
  bool bad = false;
#pragma unroll 16
  for (int64_t t = t0; t < t1; ++t) {  // unrolled: 16 loads in flight per thread
    const double v = B[t * ldb + col];
    bad |= !isfinite(v);
    mx = fmax(mx, fabs(v));
  }
  int ex = 0;
  if (mx > 0.0) frexp(mx, &ex);
  atomicMax(f + col, bad ? OZAKI_NONFINITE : ex);  // the marker dominates
}

// Columns that are entirely zero end with INT_MIN from the fill: use 0.
__global__ __launch_bounds__(256) void fix_exp_kernel(int* __restrict__ f, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < n && f[j] == INT_MIN) f[j] = 0;
}

// ---------------------------------------------------------------- digits
// Digit planes are stored in the order the GEMM consumes them.  For slice u,
// row tile T (OZ_BM rows of A, or OZ_BN columns of B) and k round R (OZ_BK
// values) there is one contiguous block, made of 1 KiB operand fragments of
// v_mfma_i32_16x16x64_i8: fragment f covers 16 rows (columns of B) and the
// round's 64 k, and lane l = 16 g + r of the instruction takes bytes
// [16 l, 16 l + 16) = digits of row 16 f + r, k = 64 R + 16 g .. + 15:
//   A: ((u * tiles_a + T) * rounds + R) * OZ_BM * OZ_BK
//        + ((row % OZ_BM) / 16) * 1024 + (16 g + row % 16) * 16 + k % 16
//   B: likewise with col for row, OZ_BN for OZ_BM
// Rows of padded tiles and k beyond the matrix hold zero digits.
constexpr int OZ_BM = 128, OZ_BN = 64, OZ_BK = 64;

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

// Byte offset, inside a tile's block, of the 16 digits of row (or column)
// rr of the tile and k chunk g (k % 64 in [16 g, 16 g + 16)).
__device__ __forceinline__ int frag_offset(int rr, int g) {
  return (rr >> 4) * 1024 + (g * 16 + (rr & 15)) * 16;
}

// Stage of the A slicing passes: rows r0 .. r0 + 127, k0 .. k0 + 31 of A,
// scaled by 2^-e[row], into tile.  Thread t takes the k pair 2 (t % 16) of
// rows t / 16 + 16 j (j < 8): each pair of loads of a wave covers 256
// contiguous bytes of four rows, and all 16 loads of a thread are in flight
// at once (entries outside A read A[0] and become zero).  The loads do not
// wait for the exponent: a row marked non-finite is zeroed after them.
template <int LD>
__device__ __forceinline__ void slice_a_stage(const double* __restrict__ A, int64_t m, int64_t k,
                                              int64_t lda, const int* __restrict__ e, int64_t r0,
                                              int64_t k0, double (&tile)[128][LD]) {
  const int kk = (threadIdx.x & 15) * 2, rq = threadIdx.x >> 4;
  const bool ok0 = k0 + kk < k, ok1 = k0 + kk + 1 < k;
  double a0[8], a1[8];
  int ex[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t row = r0 + rq + 16 * j;
    const bool rok = row < m;
    const int64_t at = row * lda + k0 + kk;
    a0[j] = A[rok && ok0 ? at : 0];
    a1[j] = A[rok && ok1 ? at + 1 : 0];
    ex[j] = e[rok ? row : 0];
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const bool use = r0 + rq + 16 * j < m && ex[j] != OZAKI_NONFINITE;
    tile[rq + 16 * j][kk] = use && ok0 ? ldexp(a0[j], -ex[j]) : 0.0;
    tile[rq + 16 * j][kk + 1] = use && ok1 ? ldexp(a1[j], -ex[j]) : 0.0;
  }
}

// A: one workgroup per (row tile, k round, half of the round): the 128 x 32
// values are read as described at slice_a_stage, scaled and transposed
// through LDS (34 KiB, so that
// several workgroups share a CU); then each of the 256 chunks of 16
// consecutive k is digitised by one thread and its 16 digit bytes per slice
// go to their fragment slot (chunks 2 h, 2 h + 1 of the round: a wave writes
// 512 contiguous bytes per slice).
constexpr int SA_K = OZ_BK / 2;
__global__ __launch_bounds__(256) void slice_a_kernel(const double* __restrict__ A, int64_t m,
                                                      int64_t k, int64_t lda,
                                                      const int* __restrict__ e, int s,
                                                      int8_t* __restrict__ planes, int64_t rows,
                                                      int64_t kp) {
  __shared__ double tile[OZ_BM][SA_K + 1];
  const int64_t rounds = kp / OZ_BK;
  const int64_t blk = blockIdx.x >> 1;  // row_tile * rounds + round
  const int half = blockIdx.x & 1;
  const int64_t r0 = (blk / rounds) * OZ_BM, k0 = (blk % rounds) * OZ_BK + half * SA_K;
  slice_a_stage(A, m, k, lda, e, r0, k0, tile);
  __syncthreads();
  // 256 chunks of 16 values (128 rows x 2): one per thread
  const int c = threadIdx.x;
  const int r = c >> 1, g = half * 2 + (c & 1);
  double x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = tile[r][(c & 1) * 16 + i];
  digits16(x, s, planes + blk * (OZ_BM * OZ_BK) + frag_offset(r, g), rows * kp);
}

// B: thread per (column, 16-wide k chunk), columns fastest across the wave.
__global__ __launch_bounds__(256) void slice_b_kernel(const double* __restrict__ B, int64_t k,
                                                      int64_t n, int64_t ldb,
                                                      const int* __restrict__ f, int s,
                                                      int8_t* __restrict__ planes, int64_t cols,
                                                      int64_t kp) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t chunks = kp / 16;
  if (id >= cols * chunks) return;
  const int64_t kc = (id / cols) * 16, col = id - (id / cols) * cols;
  double x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {  // entries outside B read B[0] and become zero
    const bool ok = col < n && kc + i < k;
    const double v = B[ok ? (kc + i) * ldb + col : 0];
    x[i] = ok ? v : 0.0;
  }
  // a column marked non-finite is zeroed after the loads (they do not wait
  // for the exponent)
  const int fc = col < n ? f[col] : 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = fc != OZAKI_NONFINITE ? ldexp(x[i], -fc) : 0.0;
  const int64_t rounds = kp / OZ_BK;
  const int64_t off = ((col / OZ_BN) * rounds + kc / OZ_BK) * (OZ_BN * OZ_BK) +
                      frag_offset((int)(col % OZ_BN), (int)((kc % OZ_BK) / 16));
  digits16(x, s, planes + off, cols * kp);
}

// ---------------------------------------------------------------- GEMM
// Work item: a 128 x 64 block of C; up to s = 7, 8 waves (two per SIMD) of
// 64 x 16, for s = 8 (whose accumulators need more registers) 4 waves of
// 64 x 32; blocks of 16 x 16 on v_mfma_i32_16x16x64_i8: lane l (r = l % 16,
// g = l / 16)
// supplies A[r][16g .. 16g+15] and B[16g .. 16g+15][r] and holds
// D[4g + v][r] in element v.  One round = 64 k.
//
// The s planes of A (8 KiB each per round) go through two LDS stages, moved
// by 16-byte global-to-LDS DMA (no registers, no conversion: the planes are
// already fragments, and each wave instruction moves one 1 KiB fragment);
// the next round's stage fills while the MFMAs run on the current one.  The
// B fragments of each plane that a wave needs are loaded straight into
// registers one round ahead.  LDS per block: 2 s 8 KiB (112 KiB at s = 7).
template <int S>
constexpr int oz_waves() {
  return S <= 7 ? 8 : 4;
}
typedef __attribute__((address_space(3))) void* lds_ptr;

struct OzArgs {
  const int8_t* a_planes;
  const int8_t* b_planes;
  const int* e;            // row exponents of A
  const int* f;            // column exponents of B
  double* C;
  double* P;
  int64_t m, n, k, kp, ldc;
  int64_t a_rows, b_cols;  // padded rows of A / columns of B (plane extents)
  int64_t k_split, tiles_m, tiles_n, splits, ldp, split_stride;
  double alpha, beta;
  int group_m, num_xcds;
};

template <int S>
__global__ __launch_bounds__(oz_waves<S>() * 64) void ozaki_gemm_kernel(OzArgs g) {
  constexpr int OZ_WAVES = oz_waves<S>();
  constexpr int WN = OZ_WAVES / 2;       // waves along n (2 along m)
  constexpr int NJ = OZ_BN / 16 / WN;    // 16-column blocks per wave
  constexpr int A_BLK = OZ_BM * OZ_BK, B_BLK = OZ_BN * OZ_BK;
  constexpr int STAGE = S * A_BLK;
  constexpr int A_FRAGS = S * (A_BLK / 1024);  // 1 KiB fragments per stage
  static_assert(A_FRAGS % OZ_WAVES == 0, "fragments per wave");
  __shared__ __attribute__((aligned(1024))) int8_t lds[2 * STAGE];

  const int64_t l = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x, g.num_xcds);
  const ItemCoord ic = item_coord(l, g.tiles_m, g.tiles_n, g.group_m);
  const int64_t row0 = ic.tile_row * OZ_BM, col0 = ic.tile_col * OZ_BN;
  const int64_t kbeg = ic.split * g.k_split;
  const int64_t kend = min64(g.k, kbeg + g.k_split);
  const int64_t nk = ceil_div(kend - kbeg, OZ_BK);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave / WN, wn = wave % WN;  // rows 64 wm .., columns 16 NJ wn ..
  const int lr = lane & 15, lg = lane >> 4;

  const int64_t rounds = g.kp / OZ_BK;
  const int64_t a_plane = g.a_rows * g.kp, b_plane = g.b_cols * g.kp;
  const int64_t rbeg = kbeg / OZ_BK;
  // this lane's 16 bytes of fragment 0 of round 0 of the work item
  const int8_t* a_src = g.a_planes + (ic.tile_row * rounds + rbeg) * A_BLK + lane * 16;
  const int8_t* b_src =
      g.b_planes + (ic.tile_col * rounds + rbeg) * B_BLK + wn * NJ * 1024 + lane * 16;

  i4 acc[S][4][NJ];
#pragma unroll
  for (int d = 0; d < S; ++d)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[d][i][j] = i4{0, 0, 0, 0};

  // wave w moves fragments w, w + OZ_WAVES, ... of the stage (fragment q:
  // slice q / 8, rows 16 (q % 8) ..)
  auto stage_a = [&](int64_t kt, int st) {
#pragma unroll
    for (int h = 0; h < A_FRAGS / OZ_WAVES; ++h) {
      const int q = wave + OZ_WAVES * h;
      const int u = q / (A_BLK / 1024), fr = q % (A_BLK / 1024);
      __builtin_amdgcn_global_load_lds(
          (const void*)(a_src + u * a_plane + kt * A_BLK + fr * 1024),
          (lds_ptr)(lds + st * STAGE + u * A_BLK + fr * 1024), 16, 0, 0);
    }
  };
  // B fragments of the current round (bc) and of the next (bn)
  i4 bc[S][NJ], bn[S][NJ];
  auto load_b = [&](int64_t kt) {
#pragma unroll
    for (int v = 0; v < S; ++v)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        bn[v][j] = *reinterpret_cast<const i4*>(b_src + v * b_plane + kt * B_BLK + j * 1024);
  };

  if (nk > 0) {
    stage_a(0, 0);
    load_b(0);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // round kt computes from LDS stage kt % 2 while round kt + 1 fills the
  // other stage and bn (issued between the products of slice 0); the DMA
  // writes must have landed before the barrier that opens the next round
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int st = (int)(kt & 1);
#pragma unroll
    for (int v = 0; v < S; ++v)
#pragma unroll
      for (int j = 0; j < NJ; ++j) bc[v][j] = bn[v][j];
    const bool more = kt + 1 < nk;
    // A fragments of slice u + 1 are read while the products of slice u
    // run: issued after its first two products, so that the wait before
    // those covers only fragments already needed
    const int8_t* a_frag = lds + st * STAGE + (wm * 4) * 1024 + lane * 16;
    i4 afr[2][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) afr[0][i] = *reinterpret_cast<const i4*>(a_frag + i * 1024);
    // the next round's loads (A_FRAGS / OZ_WAVES DMA fragments, S * NJ B
    // fragments) go out one by one between the products of slice 0 (load t
    // before product q with q LOADS <= t Q0 < (q + 1) LOADS), so the wave's
    // matrix unit keeps working while it issues them.  (Written out here
    // rather than through a helper: that form compiled to a rolled slice
    // loop with its register arrays in scratch memory.)
    constexpr int A_PW = A_FRAGS / OZ_WAVES, LOADS = A_PW + S * NJ, Q0 = S * 4 * NJ;
#pragma unroll
    for (int u = 0; u < S; ++u) {
#pragma unroll
      for (int q = 0; q < (S - u) * 4 * NJ; ++q) {
        if (u == 0) {
          const int t = q * LOADS / Q0;  // loads t .. of this gap
#pragma unroll
          for (int tt = t; tt < LOADS && tt * Q0 < (q + 1) * LOADS; ++tt) {
            if (tt * Q0 < q * LOADS) continue;
            __builtin_amdgcn_sched_barrier(0);
            if (more) {
              if (tt < A_PW) {
                const int qq = wave + OZ_WAVES * tt;
                const int uu = qq / (A_BLK / 1024), fr = qq % (A_BLK / 1024);
                __builtin_amdgcn_global_load_lds(
                    (const void*)(a_src + uu * a_plane + (kt + 1) * A_BLK + fr * 1024),
                    (lds_ptr)(lds + (st ^ 1) * STAGE + uu * A_BLK + fr * 1024), 16, 0, 0);
              } else {
                const int v = (tt - A_PW) / NJ, j = (tt - A_PW) % NJ;
                bn[v][j] =
                    *reinterpret_cast<const i4*>(b_src + v * b_plane + (kt + 1) * B_BLK + j * 1024);
              }
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        if (q == 2 && u + 1 < S) {
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int i = 0; i < 4; ++i)
            afr[(u + 1) & 1][i] =
                *reinterpret_cast<const i4*>(a_frag + (u + 1) * A_BLK + i * 1024);
          __builtin_amdgcn_sched_barrier(0);
        }
        const int v = q / (4 * NJ), i = (q / NJ) % 4, j = q % NJ;
        acc[u + v][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(afr[u & 1][i], bc[v][j],
                                                                 acc[u + v][i][j], 0, 0, 0);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  // epilogue: diagonal sums to binary64 (smallest scale first), scale by
  // 2^(e_i + f_j); 16 x 16 output layout
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t col = col0 + (wn * NJ + j) * 16 + lr;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + wm * 64 + i * 16 + lg * 4 + v;
        if (row < g.m && col < g.n) {
          double x = 0.0;
#pragma unroll
          for (int d = S - 1; d >= 0; --d) x += ldexp((double)acc[d][i][j][v], -7 * (d + 2));
          const int er = g.e[row], fc = g.f[col];
          const double r = (er == OZAKI_NONFINITE || fc == OZAKI_NONFINITE)
                               ? __builtin_nan("")
                               : ldexp(x, er + fc);
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
  hipLaunchKernelGGL(ozaki_gemm_kernel<S>, dim3((unsigned)items), dim3(oz_waves<S>() * 64), 0, s,
                     g);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ozaki_exponents(const double* A, int64_t m, int64_t k, int64_t lda,
                                  const double* B, int64_t n, int64_t ldb, int* e, int* f,
                                  hipStream_t stream) {
  hipLaunchKernelGGL(row_exp_kernel, dim3((unsigned)ceil_div(m, 4)), dim3(256), 0, stream, A, m, k,
                     lda, e);
  hipLaunchKernelGGL(fill_int_kernel, dim3(blocks_for(n) > 4096 ? 4096 : blocks_for(n)), dim3(256),
                     0, stream, f, n, INT_MIN);
  hipLaunchKernelGGL(col_exp_kernel, dim3(blocks_for(n), (unsigned)ceil_div(k, COL_CHUNK)),
                     dim3(256), 0, stream, B, k, n, ldb, f);
  hipLaunchKernelGGL(fix_exp_kernel, dim3(blocks_for(n)), dim3(256), 0, stream, f, n);
  return hipGetLastError();
}

int run_ozaki(const cosma_plan_info& plan, double alpha, const void* A, int64_t lda,
              const void* B, int64_t ldb, double beta, void* C, int64_t ldc, void* workspace,
              hipStream_t stream) {
  const int64_t m = plan.m, n = plan.n, k = plan.k;
  const int s = plan.slices;
  if (s < 1 || s > 8 || plan.tile_m != OZ_BM || plan.tile_n != OZ_BN || plan.tile_k != OZ_BK ||
      plan.k_split > MAX_K_ITEM)
    return COSMA_ERR_INVALID_ARG;
  if (m > INT_MAX / 4 || n > INT_MAX / 4) return COSMA_ERR_UNSUPPORTED;
  const int64_t kp = ceil_div(k, OZ_BK) * OZ_BK;
  const int64_t a_rows = ceil_div(m, OZ_BM) * OZ_BM, b_cols = ceil_div(n, OZ_BN) * OZ_BN;
  // the slice kernels' grids: two blocks per (row tile, round) for A, one
  // thread per (column, 16 k) for B
  if (2 * (a_rows / OZ_BM) * (kp / OZ_BK) > 0x7fffffffLL || b_cols * (kp / 16) / 256 > 0x7fffffffLL)
    return COSMA_ERR_UNSUPPORTED;
  // workspace layout (matches workspace_bytes): partials | A planes, B planes | e, f
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  char* w = static_cast<char*>(workspace);
  const size_t part = plan.p_k > 1 ? up((size_t)plan.p_k * m * n * sizeof(double)) : 0;
  int8_t* a_planes = reinterpret_cast<int8_t*>(w + part);
  int8_t* b_planes = a_planes + (size_t)s * a_rows * kp;
  int* e = reinterpret_cast<int*>(w + part + up((size_t)s * kp * (a_rows + b_cols)));
  int* f = e + m;
  hipError_t err;

  if ((err = launch_ozaki_exponents(static_cast<const double*>(A), m, k, lda,
                                    static_cast<const double*>(B), n, ldb, e, f, stream)) !=
      hipSuccess)
    return COSMA_ERR_HIP;
  hipLaunchKernelGGL(slice_a_kernel, dim3((unsigned)(2 * (a_rows / OZ_BM) * (kp / OZ_BK))),
                     dim3(256), 0, stream,
                     static_cast<const double*>(A), m, k, lda, e, s, a_planes, a_rows, kp);
  hipLaunchKernelGGL(slice_b_kernel, dim3(blocks_for(b_cols * (kp / 16))), dim3(256), 0, stream,
                     static_cast<const double*>(B), k, n, ldb, f, s, b_planes, b_cols, kp);
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
  g.a_rows = a_rows;
  g.b_cols = b_cols;
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
