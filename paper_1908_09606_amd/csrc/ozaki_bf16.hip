// FP64-accurate GEMM from bf16 digit slices (Ozaki, Ogita, Oishi & Rump,
// "Error-free transformations of matrix multiplication by using fast
// routines of matrix multiplication", Numer. Algorithms 2012), on the bf16
// matrix cores with fp32 accumulation.
//
//   1. Exponents: e_i with max_t |A[i][t]| < 2^e_i per row of A and f_j per
//      column of B, as for the int8 digit path.
//   2. Digits (rounded to nearest, a signed-digit expansion): x = A[i][t] 2^-e_i
//      lies in (-1, 1); with r_0 = x, d_u = rint(2^8 r_(u-1)),
//      r_u = 2^8 r_(u-1) - d_u (exact in binary64), so
//      x = sum_u d_u 2^-8u + r_s 2^-8s with |r_u| <= 1/2, |d_1| <= 256 and
//      |d_u| <= 128 for u >= 2.  Integers of at most 8 significant bits are
//      bf16 values, so each digit plane is an exact bf16 matrix (8 bits per
//      slice against the int8 form's 7).
//   3. Products: C[i][j] ~ 2^(e_i + f_j) sum_{u+v <= s+1} 2^-8(u+v) (A_u B_v)[i][j]
//      with v_mfma_f32_16x16x32_bf16.  A digit product is an integer of at
//      most 17 bits, exact in fp32; the pairs of one anti-diagonal d = u + v
//      share the scale 2^-8d and accumulate in one fp32 block, and fp32 adds
//      integers exactly while every partial sum stays within 2^24.  Per k,
//      diagonal d collects at most 256^2 (d = 2) or
//      2 * 256 * 128 + (d - 3) * 128^2 <= 2^17 + 2^15 (3 <= d <= s + 1 <= 9)
//      in absolute value, so a round of 32 k stays below 2^23.  After each round every diagonal block is
//      converted to binary64, scaled and added to one binary64 accumulator
//      (each as soon as its last pair of the round is issued), and the next
//      round's first product restarts it from zero.  The reduction length of
//      a work item is therefore unbounded.
//
//      Keeping the fp32 blocks over several rounds (they would stay exact
//      for 4 rounds up to s = 6) moves the conversion off most rounds, but
//      then all s blocks are live across the round boundary and the
//      register allocation of this kernel spills heavily; measured, the
//      per-round conversion costs about a fifth of the launch at s = 6.
//
// Relative to the int8 form, a slice carries one more bit but a bf16
// product runs at half the int8 rate, and the per-round conversion costs
// vector ALU time: the int8 form is the faster of the two on this GPU; this
// one keeps the whole computation in floating-point units.
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
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- digits
// Digit planes in the GEMM's consumption order.  For slice u, row tile T
// (OB_BM rows of A, or OB_BN columns of B) and k round R (OB_BK values) there
// is one contiguous block of 1 KiB operand fragments of
// v_mfma_f32_16x16x32_bf16: fragment f covers 16 rows (columns of B) and the
// round's 32 k; lane l = 16 g + r of the instruction takes bytes
// [16 l, 16 l + 16) = the bf16 digits of row 16 f + r, k = 32 R + 8 g .. + 7:
//   A: ((u * tiles_a + T) * rounds + R) * OB_BM * OB_BK * 2
//        + ((row % OB_BM) / 16) * 1024 + (16 g + row % 16) * 16 + (k % 8) * 2
//   B: likewise with col for row, OB_BN for OB_BM
// Rows of padded tiles and k beyond the matrix hold zero digits.
constexpr int OB_BM = 128, OB_BN = 64, OB_BK = 32;
constexpr int A_BLK = OB_BM * OB_BK * 2, B_BLK = OB_BN * OB_BK * 2;  // bytes per slice and round

// 2^-8d as a constant of the unrolled loops.
__host__ __device__ constexpr double pow2_neg8(int d) { return d == 0 ? 1.0 : pow2_neg8(d - 1) / 256.0; }

// bf16 encoding of an integer-valued float with |q| <= 256: the float's
// significand has at most 8 significant bits, so its upper half is the bf16
// value exactly (no rounding involved).
__device__ __forceinline__ unsigned bf16_bits_exact(float q) {
  return __float_as_uint(q) >> 16;
}

__device__ __forceinline__ void digits8(double (&x)[8], int s, unsigned char* __restrict__ out,
                                        int64_t plane_stride) {
  for (int u = 0; u < s; ++u) {
    unsigned h[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const double y = x[e] * 256.0;
      const double q = rint(y);
      h[e] = bf16_bits_exact((float)q);
      x[e] = y - q;
    }
    const i4 packed = {(int)(h[0] | (h[1] << 16)), (int)(h[2] | (h[3] << 16)),
                       (int)(h[4] | (h[5] << 16)), (int)(h[6] | (h[7] << 16))};
    *reinterpret_cast<i4*>(out + u * plane_stride) = packed;
  }
}

// Byte offset, inside a tile's block, of the 8 digits of row (or column) rr
// of the tile and k chunk g (k % 32 in [8 g, 8 g + 8)).
__device__ __forceinline__ int frag_offset(int rr, int g) {
  return (rr >> 4) * 1024 + (g * 16 + (rr & 15)) * 16;
}

// A: one workgroup per (row tile, k round): 128 x 32 values read in 8-byte
// loads (each pair of loads of a wave covers 256 contiguous bytes of four
// rows), scaled and transposed through LDS; then each chunk of 8 consecutive k is
// digitised and its 16 bytes per slice go to their fragment slot (a wave's
// 64 chunks fill one 1 KiB fragment).
__global__ __launch_bounds__(256) void slice_a_bf16_kernel(const double* __restrict__ A, int64_t m,
                                                           int64_t k, int64_t lda,
                                                           const int* __restrict__ e, int s,
                                                           unsigned char* __restrict__ planes,
                                                           int64_t rows, int64_t kp) {
  __shared__ double tile[OB_BM][OB_BK + 1];
  const int64_t rounds = kp / OB_BK;
  const int64_t blk = blockIdx.x;  // row_tile * rounds + round
  const int64_t r0 = (blk / rounds) * OB_BM, k0 = (blk % rounds) * OB_BK;
  // rows r0 .. r0 + 127 and k0 .. k0 + 31, read as in the int8 slicing
  // pass: thread t takes k pair 2 (t % 16) of rows t / 16 + 16 j, all 16
  // loads in flight at once (entries outside A read A[0] and become zero;
  // a row marked non-finite is zeroed after the loads)
  {
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
  __syncthreads();
  // 512 chunks of 8 values (128 rows x 4): two per thread
  for (int h = 0; h < 2; ++h) {
    const int c = threadIdx.x + 256 * h;
    const int r = c >> 2, g = c & 3;
    double x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = tile[r][g * 8 + i];
    digits8(x, s, planes + blk * A_BLK + frag_offset(r, g), rows * kp * 2);
  }
}

// B: thread per (column, 8-wide k chunk), columns fastest across the wave.
__global__ __launch_bounds__(256) void slice_b_bf16_kernel(const double* __restrict__ B, int64_t k,
                                                           int64_t n, int64_t ldb,
                                                           const int* __restrict__ f, int s,
                                                           unsigned char* __restrict__ planes,
                                                           int64_t cols, int64_t kp) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t chunks = kp / 8;
  if (id >= cols * chunks) return;
  const int64_t kc = (id / cols) * 8, col = id - (id / cols) * cols;
  double x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {  // entries outside B read B[0] and become zero
    const bool ok = col < n && kc + i < k;
    const double v = B[ok ? (kc + i) * ldb + col : 0];
    x[i] = ok ? v : 0.0;
  }
  // a column marked non-finite is zeroed after the loads (they do not wait
  // for the exponent)
  const int fc = col < n ? f[col] : 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) x[i] = fc != OZAKI_NONFINITE ? ldexp(x[i], -fc) : 0.0;
  const int64_t rounds = kp / OB_BK;
  const int64_t off = ((col / OB_BN) * rounds + kc / OB_BK) * B_BLK +
                      frag_offset((int)(col % OB_BN), (int)((kc % OB_BK) / 8));
  digits8(x, s, planes + off, cols * kp * 2);
}

// ---------------------------------------------------------------- GEMM
// Work item: a 128 x 64 block of C.  Up to s = 6: 8 waves (two per SIMD) of
// 64 x 16; s = 7, 8 (more accumulator registers): 4 waves of 64 x 32, one
// per SIMD with the accumulators in the AGPR half of the register file.  Blocks of
// 16 x 16: lane l (r = l % 16, g = l / 16) supplies A[r][8g .. 8g+7] and
// B[8g .. 8g+7][r] and holds D[4g + v][r] in element v.  One round = 32 k.
//
// The s planes of A (8 KiB each per round) go through two LDS stages by
// 16-byte global-to-LDS DMA (each wave instruction moves one 1 KiB
// fragment); the next round's stage fills while the current one feeds the
// matrix cores.  The B fragments a wave needs are loaded into registers one
// round ahead.  LDS per block: 2 s 8 KiB (112 KiB at s = 7).
template <int S>
constexpr int ob_waves() {
  return S <= 6 ? 8 : 4;
}
typedef __attribute__((address_space(3))) void* lds_ptr;

struct ObArgs {
  const unsigned char* a_planes;
  const unsigned char* b_planes;
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
__global__ __launch_bounds__(ob_waves<S>() * 64) void ozaki_bf16_gemm_kernel(ObArgs g) {
  constexpr int NW = ob_waves<S>();
  constexpr int WN = NW / 2;           // waves along n (2 along m)
  constexpr int NJ = OB_BN / 16 / WN;  // 16-column blocks per wave
  constexpr int STAGE = S * A_BLK;
  constexpr int A_FRAGS = S * (A_BLK / 1024);  // 1 KiB fragments per stage
  static_assert(A_FRAGS % NW == 0, "fragments per wave");
  static_assert(2 * STAGE <= 160 * 1024, "LDS budget");
  __shared__ __attribute__((aligned(1024))) unsigned char lds[2 * STAGE];

  const int64_t l = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x, g.num_xcds);
  const ItemCoord ic = item_coord(l, g.tiles_m, g.tiles_n, g.group_m);
  const int64_t row0 = ic.tile_row * OB_BM, col0 = ic.tile_col * OB_BN;
  const int64_t kbeg = ic.split * g.k_split;
  const int64_t kend = min64(g.k, kbeg + g.k_split);
  const int64_t nk = ceil_div(kend - kbeg, OB_BK);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave / WN, wn = wave % WN;  // rows 64 wm .., columns 16 NJ wn ..
  const int lr = lane & 15, lg = lane >> 4;

  const int64_t rounds = g.kp / OB_BK;
  const int64_t a_plane = g.a_rows * g.kp * 2, b_plane = g.b_cols * g.kp * 2;
  const int64_t rbeg = kbeg / OB_BK;
  // this lane's 16 bytes of fragment 0 of round 0 of the work item
  const unsigned char* a_src = g.a_planes + (ic.tile_row * rounds + rbeg) * A_BLK + lane * 16;
  const unsigned char* b_src =
      g.b_planes + (ic.tile_col * rounds + rbeg) * B_BLK + wn * NJ * 1024 + lane * 16;

  const f4 zero = {0.f, 0.f, 0.f, 0.f};
  f4 acc[S][4][NJ];      // fp32 diagonal sums of the current round
  double sum[4][NJ][4];  // binary64 total over the rounds so far
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
#pragma unroll
      for (int d = 0; d < S; ++d) acc[d][i][j] = zero;
#pragma unroll
      for (int v = 0; v < 4; ++v) sum[i][j][v] = 0.0;
    }

  // wave w moves fragments w, w + NW, ... of the stage (fragment q: slice
  // q / 8, rows 16 (q % 8) ..)
  auto stage_a = [&](int64_t kt, int st) {
#pragma unroll
    for (int h = 0; h < A_FRAGS / NW; ++h) {
      const int q = wave + NW * h;
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
  // other stage and bn; the DMA writes must have landed before the barrier
  // that opens the next round
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int st = (int)(kt & 1);
#pragma unroll
    for (int v = 0; v < S; ++v)
#pragma unroll
      for (int j = 0; j < NJ; ++j) bc[v][j] = bn[v][j];
    if (kt + 1 < nk) {
      stage_a(kt + 1, st ^ 1);
      load_b(kt + 1);
    }
    // A fragments of slice u + 1 are read while the products of slice u
    // run (issued after its first two products)
    const unsigned char* a_frag = lds + st * STAGE + (wm * 4) * 1024 + lane * 16;
    i4 afr[2][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) afr[0][i] = *reinterpret_cast<const i4*>(a_frag + i * 1024);
#pragma unroll
    for (int u = 0; u < S; ++u) {
#pragma unroll
      for (int q = 0; q < (S - u) * 4 * NJ; ++q) {
        if (q == 2 && u + 1 < S) {
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int i = 0; i < 4; ++i)
            afr[(u + 1) & 1][i] =
                *reinterpret_cast<const i4*>(a_frag + (u + 1) * A_BLK + i * 1024);
          __builtin_amdgcn_sched_barrier(0);
        }
        const int v = q / (4 * NJ), i = (q / NJ) % 4, j = q % NJ;
        // slice u = 0 opens every diagonal of the round: start from zero
        acc[u + v][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8, afr[u & 1][i]), __builtin_bit_cast(bf8, bc[v][j]),
            u == 0 ? zero : acc[u + v][i][j], 0, 0, 0);
      }
      // diagonal u (digit pairs u' + v' = u, 0-based) got its last pair,
      // (u, 0), above: its exact round sum goes into binary64 with weight
      // 2^-8(u+2) while the later slices' products run on the matrix cores
      const double w = pow2_neg8(u + 2);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) sum[i][j][v] = fma((double)acc[u][i][j][v], w, sum[i][j][v]);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  // epilogue: scale by 2^(e_i + f_j); 16 x 16 output layout
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t col = col0 + (wn * NJ + j) * 16 + lr;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + wm * 64 + i * 16 + lg * 4 + v;
        if (row < g.m && col < g.n) {
          const int er = g.e[row], fc = g.f[col];
          const double r = (er == OZAKI_NONFINITE || fc == OZAKI_NONFINITE)
                               ? __builtin_nan("")
                               : ldexp(sum[i][j][v], er + fc);
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
hipError_t launch_ob(const ObArgs& g, hipStream_t s) {
  const int64_t items = g.tiles_m * g.tiles_n * g.splits;
  if (items <= 0) return hipSuccess;
  if (items > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ozaki_bf16_gemm_kernel<S>, dim3((unsigned)items), dim3(ob_waves<S>() * 64),
                     0, s, g);
  return hipGetLastError();
}

}  // namespace

int run_ozaki_bf16(const cosma_plan_info& plan, double alpha, const void* A, int64_t lda,
                   const void* B, int64_t ldb, double beta, void* C, int64_t ldc, void* workspace,
                   hipStream_t stream) {
  const int64_t m = plan.m, n = plan.n, k = plan.k;
  const int s = plan.slices;
  if (s < 1 || s > 8 || plan.tile_m != OB_BM || plan.tile_n != OB_BN || plan.tile_k != OB_BK)
    return COSMA_ERR_INVALID_ARG;
  if (m > INT_MAX / 4 || n > INT_MAX / 4) return COSMA_ERR_UNSUPPORTED;
  const int64_t kp = ceil_div(k, OB_BK) * OB_BK;
  const int64_t a_rows = ceil_div(m, OB_BM) * OB_BM, b_cols = ceil_div(n, OB_BN) * OB_BN;
  // the slice kernels' grids: one block per (row tile, round) for A, one
  // thread per (column, 8 k) for B
  if ((a_rows / OB_BM) * (kp / OB_BK) > 0x7fffffffLL || b_cols * (kp / 8) / 256 > 0x7fffffffLL)
    return COSMA_ERR_UNSUPPORTED;
  // workspace layout (matches workspace_bytes): partials | A planes, B planes | e, f
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  char* w = static_cast<char*>(workspace);
  const size_t part = plan.p_k > 1 ? up((size_t)plan.p_k * m * n * sizeof(double)) : 0;
  unsigned char* a_planes = reinterpret_cast<unsigned char*>(w + part);
  unsigned char* b_planes = a_planes + (size_t)s * a_rows * kp * 2;
  int* e = reinterpret_cast<int*>(w + part + up((size_t)s * kp * 2 * (a_rows + b_cols)));
  int* f = e + m;
  hipError_t err;

  if ((err = launch_ozaki_exponents(static_cast<const double*>(A), m, k, lda,
                                    static_cast<const double*>(B), n, ldb, e, f, stream)) !=
      hipSuccess)
    return COSMA_ERR_HIP;
  hipLaunchKernelGGL(slice_a_bf16_kernel, dim3((unsigned)((a_rows / OB_BM) * (kp / OB_BK))),
                     dim3(256), 0, stream, static_cast<const double*>(A), m, k, lda, e, s,
                     a_planes, a_rows, kp);
  hipLaunchKernelGGL(slice_b_bf16_kernel, dim3(blocks_for(b_cols * (kp / 8))), dim3(256), 0,
                     stream, static_cast<const double*>(B), k, n, ldb, f, s, b_planes, b_cols,
                     kp);
  if ((err = hipGetLastError()) != hipSuccess) return COSMA_ERR_HIP;

  ObArgs g;
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
    case 1: err = launch_ob<1>(g, stream); break;
    case 2: err = launch_ob<2>(g, stream); break;
    case 3: err = launch_ob<3>(g, stream); break;
    case 4: err = launch_ob<4>(g, stream); break;
    case 5: err = launch_ob<5>(g, stream); break;
    case 6: err = launch_ob<6>(g, stream); break;
    case 7: err = launch_ob<7>(g, stream); break;
    default: err = launch_ob<8>(g, stream); break;
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
