// FP32-class GEMMs on the CDNA4 matrix cores.
//
//   gemm_f32_kernel     native FP32: v_mfma_f32_16x16x4f32 on 16x16 blocks
//                       or v_mfma_f32_32x32x2f32 on 32x32 blocks (the
//                       widest tile, whose 64x64 wave blocks keep four
//                       independent accumulator chains per wave)
//   gemm_bf16x3_kernel  FP32-accurate product from bf16 pieces: every FP32
//                       operand x is split as x_hi = bf16_rn(x),
//                       x_lo = bf16_rn(x - x_hi) and
//                       A*B ~ A_lo*B_hi + A_hi*B_lo + A_hi*B_hi
//                       (the dropped A_lo*B_lo and split residues are
//                       below 2^-16 relative), with v_mfma_f32_16x16x32_bf16
//                       and FP32 accumulation.
//
// Both keep the work item's block of C resident in accumulators and stream
// k in LDS-staged rounds (the loop of Algorithm 1, section 5's resident
// block), double-buffered as in section 7.3.  For BF16x3 a split pass
// first writes A and B once as bf16 hi / lo planes in the order the GEMM
// stages them (32-wide k blocks of padded rows, zero padding), so the GEMM
// moves contiguous 16-byte chunks straight into LDS, already in the
// matrix-core operand order, with no conversion arithmetic and no bounds
// checks in its main loop.
//
// Matrix-core layouts (lane l, r = l % 16, g = l / 16, c = l % 32, q = l / 32):
//   f32 16x16x4:  a = A[r][g], b = B[g][r], acc[v] = D[4g + v][r]
//   f32 32x32x2:  a = A[c][q], b = B[q][c],
//                 acc[v] = D[8 (v / 4) + 4q + v % 4][c] (v < 16)
//   bf16 16x16x32: a[i] = A[r][8g + i], b[i] = B[8g + i][r] (i < 8),
//                  acc[v] = D[4g + v][r]
#include <hip/hip_runtime.h>

#include "batch_device.hpp"
#include "kernels.hpp"
#include "tiles.hpp"

namespace cosma {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------- native FP32
// BLK: edge of the matrix-core output block, 16 (16x16x4) or 32 (32x32x2).
template <int BM, int BN, int BK, int WM, int WN, int BLK = 16>
struct F32Tile {
  static constexpr int NT = WM * WN * 64;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int MI = WTM / BLK, NI = WTN / BLK;  // output blocks per wave
  static constexpr int LDA_S = BK + 4;   // As[row][k] (floats), 16-byte rows
  static constexpr int LDB_S = BN + 4;   // Bs[k][col]
  static constexpr int A_CHUNKS = BM * BK / 4 / NT;  // float4 per thread
  static constexpr int B_CHUNKS = BK * BN / 4 / NT;
  static constexpr int A_STAGE = BM * LDA_S, B_STAGE = BK * LDB_S;
  static_assert(BLK == 16 || BLK == 32, "matrix-core form");
  static_assert(WTM % BLK == 0 && WTN % BLK == 0, "wave blocks");
  static_assert(BK % 16 == 0 && (BM * BK / 4) % NT == 0 && (BK * BN / 4) % NT == 0, "tiling");
  static_assert(2 * (A_STAGE + B_STAGE) * 4 <= 160 * 1024, "LDS budget");
};

// Operand loads of one round, per operand in one of three modes:
// LOAD_VEC: 16-byte loads (base and row pitch 16-byte aligned, round in
// bounds); LOAD_SCALAR: four 4-byte loads, no checks (in bounds, pitch not a
// multiple of 16 bytes, e.g. an odd k or n); LOAD_CHECKED: element-wise with
// zero fill (edge tiles and the last partial round).
enum LoadMode { LOAD_VEC = 0, LOAD_SCALAR = 1, LOAD_CHECKED = 2 };

template <class TL, int BM, int BN, int BK, int MODE>
__device__ __forceinline__ void f32_load_a(const GemmArgs& g, int64_t row0, int64_t k0,
                                           int64_t kend, f4 (&ra)[TL::A_CHUNKS]) {
  const float* __restrict__ A = static_cast<const float*>(g.A);
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < TL::A_CHUNKS; ++i) {
    const int c = t + TL::NT * i;
    const int r = c / (BK / 4), kk = (c % (BK / 4)) * 4;
    const int64_t gr = row0 + r, gk = k0 + kk;
    const float* p = A + gr * g.lda + gk;
    if (MODE == LOAD_VEC) {
      ra[i] = *reinterpret_cast<const f4*>(p);
    } else if (MODE == LOAD_SCALAR) {
#pragma unroll
      for (int e = 0; e < 4; ++e) ra[i][e] = p[e];
    } else {
      const bool rin = gr < g.m;
#pragma unroll
      for (int e = 0; e < 4; ++e) ra[i][e] = (rin && gk + e < kend) ? p[e] : 0.0f;
    }
  }
}

template <class TL, int BM, int BN, int BK, int MODE>
__device__ __forceinline__ void f32_load_b(const GemmArgs& g, int64_t col0, int64_t k0,
                                           int64_t kend, f4 (&rb)[TL::B_CHUNKS]) {
  const float* __restrict__ B = static_cast<const float*>(g.B);
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < TL::B_CHUNKS; ++i) {
    const int c = t + TL::NT * i;
    const int r = c / (BN / 4), nn = (c % (BN / 4)) * 4;
    const int64_t gk = k0 + r, gc = col0 + nn;
    const float* p = B + gk * g.ldb + gc;
    if (MODE == LOAD_VEC) {
      rb[i] = *reinterpret_cast<const f4*>(p);
    } else if (MODE == LOAD_SCALAR) {
#pragma unroll
      for (int e = 0; e < 4; ++e) rb[i][e] = p[e];
    } else {
      const bool kin = gk < kend;
#pragma unroll
      for (int e = 0; e < 4; ++e) rb[i][e] = (kin && gc + e < g.n) ? p[e] : 0.0f;
    }
  }
}

// One round's A and B panels.  FAST (a full tile with both operands 16-byte
// aligned, decided once per work item): vector loads, element-wise only in
// a partial last round; the common case keeps this short loop body.
// Otherwise each operand takes its own mode; a_in / b_in say whether the
// tile's rows of A / columns of B all lie inside the matrix.
template <class TL, int BM, int BN, int BK, bool FAST>
__device__ __forceinline__ void f32_load(const GemmArgs& g, int64_t row0, int64_t col0, int64_t k0,
                                         int64_t kend, bool a_in, bool b_in,
                                         f4 (&ra)[TL::A_CHUNKS], f4 (&rb)[TL::B_CHUNKS]) {
  const bool k_in = k0 + BK <= kend;
  if (FAST) {
    if (k_in) {
      f32_load_a<TL, BM, BN, BK, LOAD_VEC>(g, row0, k0, kend, ra);
      f32_load_b<TL, BM, BN, BK, LOAD_VEC>(g, col0, k0, kend, rb);
    } else {
      f32_load_a<TL, BM, BN, BK, LOAD_CHECKED>(g, row0, k0, kend, ra);
      f32_load_b<TL, BM, BN, BK, LOAD_CHECKED>(g, col0, k0, kend, rb);
    }
    return;
  }
  if (a_in && k_in) {
    if (g.vec_a)
      f32_load_a<TL, BM, BN, BK, LOAD_VEC>(g, row0, k0, kend, ra);
    else
      f32_load_a<TL, BM, BN, BK, LOAD_SCALAR>(g, row0, k0, kend, ra);
  } else {
    f32_load_a<TL, BM, BN, BK, LOAD_CHECKED>(g, row0, k0, kend, ra);
  }
  if (b_in && k_in) {
    if (g.vec_b)
      f32_load_b<TL, BM, BN, BK, LOAD_VEC>(g, col0, k0, kend, rb);
    else
      f32_load_b<TL, BM, BN, BK, LOAD_SCALAR>(g, col0, k0, kend, rb);
  } else {
    f32_load_b<TL, BM, BN, BK, LOAD_CHECKED>(g, col0, k0, kend, rb);
  }
}

template <class TL, int BM, int BN, int BK>
__device__ __forceinline__ void f32_store(float* As, float* Bs, const f4 (&ra)[TL::A_CHUNKS],
                                          const f4 (&rb)[TL::B_CHUNKS]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < TL::A_CHUNKS; ++i) {
    const int c = t + TL::NT * i;
    const int r = c / (BK / 4), kk = (c % (BK / 4)) * 4;
    *reinterpret_cast<f4*>(As + r * TL::LDA_S + kk) = ra[i];
  }
#pragma unroll
  for (int i = 0; i < TL::B_CHUNKS; ++i) {
    const int c = t + TL::NT * i;
    const int r = c / (BN / 4), nn = (c % (BN / 4)) * 4;
    *reinterpret_cast<f4*>(Bs + r * TL::LDB_S + nn) = rb[i];
  }
}

// Epilogue shared by the FP32-class kernels.  Accumulator v of lane l in
// the BLK x BLK output block holds row 8 (v / 4) + 4 (l / BLK) + v % 4,
// column l % BLK (for BLK = 16, v < 4, this is the 16x16 layout above).
template <int BLK, int MI, int NI, int WTM, int WTN, class V>
__device__ __forceinline__ void f32_epilogue(const GemmArgs& g, const ItemCoord& ic, int64_t row0,
                                             int64_t col0, int wm, int wn, int lane,
                                             const V (&acc)[MI][NI]) {
  constexpr int NV = BLK * BLK / 64;
  const int lcol = lane % BLK, lrow = 4 * (lane / BLK);
  const bool direct = g.splits == 1;
  float* __restrict__ C = static_cast<float*>(g.C);
  float* __restrict__ P = direct ? nullptr : static_cast<float*>(g.P) + ic.split * g.split_stride;
  const float alpha = (float)g.alpha, beta = (float)g.beta;
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int64_t col = col0 + wn * WTN + j * BLK + lcol;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int64_t row = row0 + wm * WTM + i * BLK + 8 * (v / 4) + lrow + v % 4;
        if (row < g.m && col < g.n) {
          if (direct) {
            float* p = C + row * g.ldc + col;
            const float r = alpha * acc[i][j][v];
            *p = beta != 0.0f ? r + beta * *p : r;
          } else {
            P[row * g.ldp + col] = acc[i][j][v];
          }
        }
      }
    }
}

// One work item: the BM x BN block (ic.tile_row, ic.tile_col) over the
// reduction range of split ic.split.  As / Bs: two LDS stages each.  Each
// 16-k group of a round is split among the lanes so that every lane reads
// contiguous k of its A row (one or two 16-byte LDS reads per block) and
// every LDS element is read once per wave: in the 16x16x4 form lane group
// g takes k = 4g + s (s < 4), in the 32x32x2 form lane half q takes
// k = 8q + s (s < 8), instruction s pairing the two halves.
template <int BM, int BN, int BK, int WM, int WN, int BLK, bool FAST>
__device__ __forceinline__ void f32_tile_body(const GemmArgs& g, const ItemCoord& ic,
                                              float (*As)[F32Tile<BM, BN, BK, WM, WN>::A_STAGE],
                                              float (*Bs)[F32Tile<BM, BN, BK, WM, WN>::B_STAGE]) {
  using TL = F32Tile<BM, BN, BK, WM, WN, BLK>;
  typedef float acc_t __attribute__((ext_vector_type(BLK * BLK / 64)));
  const int64_t row0 = ic.tile_row * BM, col0 = ic.tile_col * BN;
  const int64_t kbeg = ic.split * g.k_split;
  const int64_t kend = min64(g.k, kbeg + g.k_split);
  const int64_t nk = ceil_div(kend - kbeg, BK);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int lr = lane % BLK, lg = lane / BLK;  // block row / column, k group
  constexpr int KS = BLK / 4;                  // k per lane group and 16-k group
  static_assert(KS % 4 == 0 && KS * (64 / BLK) == 16, "k split of a 16-k group");
  const bool a_in = row0 + BM <= g.m, b_in = col0 + BN <= g.n;
  // On an edge tile a wave whose rows or columns all lie outside C skips
  // its LDS reads and products (it still loads, stores and meets every
  // barrier), leaving the matrix cores of its SIMD to the other waves.
  const bool live = FAST || __builtin_amdgcn_readfirstlane(
                                (int)(row0 + wm * TL::WTM < g.m && col0 + wn * TL::WTN < g.n));

  acc_t acc[TL::MI][TL::NI];
#pragma unroll
  for (int i = 0; i < TL::MI; ++i)
#pragma unroll
    for (int j = 0; j < TL::NI; ++j)
#pragma unroll
      for (int v = 0; v < BLK * BLK / 64; ++v) acc[i][j][v] = 0.f;

  f4 ra[TL::A_CHUNKS], rb[TL::B_CHUNKS];
  if (nk > 0) {
    f32_load<TL, BM, BN, BK, FAST>(g, row0, col0, kbeg, kend, a_in, b_in, ra, rb);
    f32_store<TL, BM, BN, BK>(As[0], Bs[0], ra, rb);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    const bool more = kt + 1 < nk;
    if (more)
      f32_load<TL, BM, BN, BK, FAST>(g, row0, col0, kbeg + (kt + 1) * BK, kend, a_in, b_in, ra,
                                     rb);
    const float* as = As[cur];
    const float* bs = Bs[cur];
#pragma unroll
    for (int h = 0; h < (live ? BK / 16 : 0); ++h) {
      f4 af[TL::MI][KS / 4];
      float bf[TL::NI][KS];
#pragma unroll
      for (int i = 0; i < TL::MI; ++i)
#pragma unroll
        for (int c = 0; c < KS / 4; ++c)
          af[i][c] = *reinterpret_cast<const f4*>(as + (wm * TL::WTM + i * BLK + lr) * TL::LDA_S +
                                                  h * 16 + lg * KS + c * 4);
#pragma unroll
      for (int j = 0; j < TL::NI; ++j)
#pragma unroll
        for (int s = 0; s < KS; ++s)
          bf[j][s] = bs[(h * 16 + lg * KS + s) * TL::LDB_S + wn * TL::WTN + j * BLK + lr];
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int i = 0; i < TL::MI; ++i)
#pragma unroll
          for (int j = 0; j < TL::NI; ++j) {
            if constexpr (BLK == 16)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][s / 4][s % 4], bf[j][s],
                                                               acc[i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][s / 4][s % 4], bf[j][s],
                                                               acc[i][j], 0, 0, 0);
          }
    }
    if (more) f32_store<TL, BM, BN, BK>(As[cur ^ 1], Bs[cur ^ 1], ra, rb);
    __syncthreads();
  }
  f32_epilogue<BLK, TL::MI, TL::NI, TL::WTM, TL::WTN>(g, ic, row0, col0, wm, wn, lane, acc);
}

// The two loop bodies are compiled apart and chosen once per work item.
template <int BM, int BN, int BK, int WM, int WN, int BLK>
__device__ __forceinline__ void f32_tile(const GemmArgs& g, const ItemCoord& ic,
                                         float (*As)[F32Tile<BM, BN, BK, WM, WN>::A_STAGE],
                                         float (*Bs)[F32Tile<BM, BN, BK, WM, WN>::B_STAGE]) {
  const bool fast = (ic.tile_row + 1) * BM <= g.m && (ic.tile_col + 1) * BN <= g.n && g.vec_a &&
                    g.vec_b;
  if (fast)
    f32_tile_body<BM, BN, BK, WM, WN, BLK, true>(g, ic, As, Bs);
  else
    f32_tile_body<BM, BN, BK, WM, WN, BLK, false>(g, ic, As, Bs);
}

// WPE: waves per SIMD the register allocation must allow (the tile menu's
// blocks per CU times WM * WN / 4).  BLK: matrix-core form (16 or 32).
template <int BM, int BN, int BK, int WM, int WN, int WPE, int BLK>
__global__ __launch_bounds__(WM* WN * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void gemm_f32_kernel(
    GemmArgs g) {
  using TL = F32Tile<BM, BN, BK, WM, WN>;
  __shared__ __attribute__((aligned(16))) float As[2][TL::A_STAGE];
  __shared__ __attribute__((aligned(16))) float Bs[2][TL::B_STAGE];
  const int64_t l = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x, g.num_xcds);
  const ItemCoord ic = item_coord(l, g.tiles_m, g.tiles_n, g.group_m);
  f32_tile<BM, BN, BK, WM, WN, BLK>(g, ic, As, Bs);
}

// Persistent batched form: every workgroup takes (problem, split, tile)
// items from the device counters until every chunk is drained; each item is
// computed exactly as by gemm_f32_kernel under the problem's split.
template <int BM, int BN, int BK, int WM, int WN, int WPE, int BLK>
__global__ __launch_bounds__(WM* WN * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void gemm_f32_batched_kernel(
    BatchArgs b) {
  using TL = F32Tile<BM, BN, BK, WM, WN>;
  __shared__ __attribute__((aligned(16))) float As[2][TL::A_STAGE];
  __shared__ __attribute__((aligned(16))) float Bs[2][TL::B_STAGE];
  __shared__ int64_t next;
  int step = 0;
  for (;;) {
    if (threadIdx.x == 0) next = batch_take(b, step);
    __syncthreads();
    const int64_t it = uniform_i64(next);
    __syncthreads();
    if (it < 0) return;
    GemmArgs g;
    ItemCoord ic;
    batch_item(b, (unsigned)it, g, ic);
    f32_tile<BM, BN, BK, WM, WN, BLK>(g, ic, As, Bs);
  }
}

// ------------------------------------------------------------- BF16x3
// LDS holds four planes per stage: A_hi, A_lo by rows and B_hi, B_lo by
// columns, each round's 32 k of 16 rows (columns) as one 1 KiB group in
// matrix-core operand order (the 16 bytes of k 8g .. 8g + 7 of row r at
// position 16 g + r), so every MFMA operand is one 16-byte read per lane and
// a wave's read of an operand is one 1 KiB group in lane order.
template <int BM, int BN, int BK, int WM, int WN>
struct X3Tile {
  static constexpr int NT = WM * WN * 64;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int MI = WTM / 16, NI = WTN / 16;
  static constexpr int LD = BK;                            // bf16 per LDS row
  static constexpr int A_CHUNKS = BM * BK / 8 / NT;        // 8-element pieces per thread
  static constexpr int B_CHUNKS = BK * BN / 8 / NT;
  static constexpr int A_PLANE = BM * LD, B_PLANE = BN * LD;
  static constexpr int STAGE = 2 * A_PLANE + 2 * B_PLANE;  // bf16 elements
  static_assert(BK == 32, "the operand order assumes 32 k per round");
  static_assert((BM * BK / 8) % NT == 0 && (BK * BN / 8) % NT == 0, "tiling");
  static_assert(2 * STAGE * 2 <= 160 * 1024, "LDS budget");
};

// Offset (in bf16) of 16-byte chunk `chunk` (k % 32 in [8 chunk,
// 8 chunk + 8)) of row `row` inside a round's block of a plane: rows come in
// groups of 16 (512 bf16 = 1 KiB each), and within a group the chunk-th 16
// bytes of row r sit at position 16 chunk + r.  That is the operand order of
// v_mfma_f32_16x16x32_bf16 (lane 16 g + r takes k 8g .. 8g + 7 of row r), so
// a wave's read of one 16-row operand is the 1 KiB group in lane order.
__device__ __forceinline__ int64_t x3_pos(int64_t row, int chunk) {
  return (row & ~(int64_t)15) * 32 + chunk * 128 + (row & 15) * 8;
}

// Round-to-nearest-even split of 8 floats into bf16 hi and lo pieces.
__device__ __forceinline__ void split8(const float (&x)[8], us8& hi, us8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)x[e];
    const float r = x[e] - (float)h;
    const __bf16 q = (__bf16)r;
    hi[e] = __builtin_bit_cast(unsigned short, h);
    lo[e] = __builtin_bit_cast(unsigned short, q);
  }
}

// Split pass: FP32 operands -> bf16 hi / lo planes in the GEMM's staging
// order.  A plane: element (row, k) at
//   (k / 32) * rows_p * 32 + x3_pos(row, (k % 32) / 8) + k % 8
// (rows_p = rows padded to 256, the tallest tile); B planes are stored
// transposed, (col, k) likewise with cols_p (columns padded to 256).  Padding
// rows, columns and k hold zeros, so a tile's round of any tile shape is one
// contiguous block, already in the operand order the GEMM's LDS uses, and
// the GEMM copies it with no bounds checks.
constexpr int X3_K = 32;

// A: one block per 16 rows x 256 k (8 rounds).  The FP32 values are read as
// 1 KiB row segments (one wave instruction per row) into LDS, then every
// round's 16 rows x 32 k are split and written as 1 KiB contiguous runs of
// each plane.  LDS rows are padded to 260 floats so that the second phase's
// 16-byte reads (8 lanes = 2 rows x 4 chunks) touch distinct bank quads.
constexpr int XA_ROWS = 16, XA_K = 256, XA_LD = XA_K + 4;

__global__ __launch_bounds__(256) void x3_split_a_kernel(const float* __restrict__ A, int64_t m,
                                                         int64_t k, int64_t lda, int vec,
                                                         int64_t rows_p, int64_t kp,
                                                         unsigned short* __restrict__ hi,
                                                         unsigned short* __restrict__ lo) {
  __shared__ __attribute__((aligned(16))) float tile[XA_ROWS * XA_LD];
  const int64_t kblocks = ceil_div(kp, (int64_t)XA_K);
  const int64_t row0 = ((int64_t)blockIdx.x / kblocks) * XA_ROWS;
  const int64_t k0 = ((int64_t)blockIdx.x % kblocks) * XA_K;
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = t + 256 * i;  // float4 index: row q / 64, k 4 (q % 64)
    const int r = q >> 6, c = (q & 63) * 4;
    const int64_t row = row0 + r, kk = k0 + c;
    f4 x = f4{0.f, 0.f, 0.f, 0.f};
    if (row < m) {
      const float* src = A + row * lda + kk;
      if (vec && kk + 4 <= k) {
        x = *reinterpret_cast<const f4*>(src);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (kk + e < k) x[e] = src[e];
      }
    }
    *reinterpret_cast<f4*>(tile + r * XA_LD + c) = x;
  }
  __syncthreads();
  const int64_t rounds = kp / X3_K;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = t + 256 * h;  // 8-value chunk: round c / 64, row (c % 64) / 4, k chunk c % 4
    const int rr = c >> 6, r = (c & 63) >> 2, kc = c & 3;
    const int64_t round = k0 / X3_K + rr;
    if (round < rounds) {
      const float* src = tile + r * XA_LD + rr * X3_K + kc * 8;
      const f4 x0 = *reinterpret_cast<const f4*>(src);
      const f4 x1 = *reinterpret_cast<const f4*>(src + 4);
      const float x[8] = {x0[0], x0[1], x0[2], x0[3], x1[0], x1[1], x1[2], x1[3]};
      us8 hv, lv;
      split8(x, hv, lv);
      const int64_t row = row0 + r;
      const int64_t off = round * rows_p * X3_K + x3_pos(row, kc);
      *reinterpret_cast<us8*>(hi + off) = hv;
      *reinterpret_cast<us8*>(lo + off) = lv;
    }
  }
}

// B: one block per round (32 k) x 128 columns.  The 32 rows are read as
// 512-byte segments into LDS, then every column's 32 k are split and written
// (16 columns x 64 bytes = 1 KiB contiguous per wave and plane).  LDS rows
// are 130 floats apart, so the column reads of a wave (16 columns x 4 k
// chunks) fall into 64 distinct banks.
constexpr int XB_COLS = 128, XB_LD = XB_COLS + 2;

__global__ __launch_bounds__(256) void x3_split_b_kernel(const float* __restrict__ B, int64_t k,
                                                         int64_t n, int64_t ldb, int vec,
                                                         int64_t cols_p, int64_t kp,
                                                         unsigned short* __restrict__ hi,
                                                         unsigned short* __restrict__ lo) {
  __shared__ __attribute__((aligned(16))) float tile[X3_K * XB_LD];
  const int64_t cblocks = cols_p / XB_COLS;
  const int64_t round = (int64_t)blockIdx.x / cblocks;
  const int64_t col0 = ((int64_t)blockIdx.x % cblocks) * XB_COLS;
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = t + 256 * i;  // float4 index: k row q / 32, columns 4 (q % 32)
    const int r = q >> 5, c = (q & 31) * 4;
    const int64_t kk = round * X3_K + r, col = col0 + c;
    f4 x = f4{0.f, 0.f, 0.f, 0.f};
    if (kk < k) {
      const float* src = B + kk * ldb + col;
      if (vec && col + 4 <= n) {
        x = *reinterpret_cast<const f4*>(src);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (col + e < n) x[e] = src[e];
      }
    }
    float* dst = tile + r * XB_LD + c;  // 8-byte aligned (XB_LD is even)
    *reinterpret_cast<float2*>(dst) = float2{x[0], x[1]};
    *reinterpret_cast<float2*>(dst + 2) = float2{x[2], x[3]};
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = t + 256 * h;  // 8-value chunk: column c / 4, k chunk c % 4
    const int cc = c >> 2, kc = c & 3;
    float x[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = tile[(kc * 8 + e) * XB_LD + cc];
    us8 hv, lv;
    split8(x, hv, lv);
    const int64_t col = col0 + cc;
    const int64_t off = round * cols_p * X3_K + x3_pos(col, kc);
    *reinterpret_cast<us8*>(hi + off) = hv;
    *reinterpret_cast<us8*>(lo + off) = lv;
  }
}

// GEMM on the split planes.  A round's A_hi, A_lo (BM rows x 64 bytes each)
// and B_hi, B_lo (BN columns x 64 bytes) blocks are contiguous and already
// in operand order, so staging is a copy of 1 KiB pieces by 16-byte global-to-LDS
// DMA (no registers, no LDS write instructions).  NS LDS stages form a ring:
// the DMA of round r + NS - 1 is issued at the start of round r.
typedef __attribute__((address_space(3))) void* lds_ptr;

template <int BM, int BN, int BK, int WM, int WN, int NS>
__global__ __launch_bounds__(WM* WN * 64) void gemm_bf16x3_kernel(X3Args g) {
  using TL = X3Tile<BM, BN, BK, WM, WN>;
  constexpr int NW = WM * WN;
  constexpr int A_CH = BM * 64 / 1024, B_CH = BN * 64 / 1024;  // 1 KiB pieces per plane
  static_assert(A_CH % NW == 0 && B_CH % NW == 0, "every wave moves whole pieces of each plane");
  constexpr int A_PW = A_CH / NW, B_PW = B_CH / NW;
  constexpr int DMA_PW = 2 * (A_PW + B_PW);  // DMA instructions per wave and round
  static_assert(NS * TL::STAGE * 2 <= 160 * 1024, "LDS budget");
  __shared__ __attribute__((aligned(1024))) unsigned short lds[NS * TL::STAGE];

  const int64_t l = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x, g.num_xcds);
  const ItemCoord ic = item_coord(l, g.tiles_m, g.tiles_n, g.group_m);
  const int64_t row0 = ic.tile_row * BM, col0 = ic.tile_col * BN;
  const int64_t kbeg = ic.split * g.k_split;
  const int64_t kend = min64(g.kp, kbeg + g.k_split);
  const int64_t nk = ceil_div(kend - kbeg, BK);
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int lr = lane & 15, lg = lane >> 4;

  f4 acc[TL::MI][TL::NI];
#pragma unroll
  for (int i = 0; i < TL::MI; ++i)
#pragma unroll
    for (int j = 0; j < TL::NI; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // this lane's 16 bytes of piece 0 of round 0 of the item, per plane (bf16 units)
  const int64_t a_step = g.rows_p * X3_K, b_step = g.cols_p * X3_K;  // one round further
  const int64_t a0 = (kbeg / X3_K) * a_step + row0 * X3_K + lane * 8;
  const int64_t b0 = (kbeg / X3_K) * b_step + col0 * X3_K + lane * 8;
  const unsigned short* a_hi_src = g.a_hi + a0;
  const unsigned short* a_lo_src = g.a_lo + a0;
  const unsigned short* b_hi_src = g.b_hi + b0;
  const unsigned short* b_lo_src = g.b_lo + b0;
  // wave w moves pieces w, w + NW, ... of every plane
  auto stage_in = [&](int64_t round, int st) {
    unsigned short* base = lds + st * TL::STAGE;
#pragma unroll
    for (int h = 0; h < A_PW; ++h) {
      const int c = (wave + NW * h) * 512;
      __builtin_amdgcn_global_load_lds((const void*)(a_hi_src + round * a_step + c),
                                       (lds_ptr)(base + c), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(a_lo_src + round * a_step + c),
                                       (lds_ptr)(base + TL::A_PLANE + c), 16, 0, 0);
    }
#pragma unroll
    for (int h = 0; h < B_PW; ++h) {
      const int c = (wave + NW * h) * 512;
      __builtin_amdgcn_global_load_lds((const void*)(b_hi_src + round * b_step + c),
                                       (lds_ptr)(base + 2 * TL::A_PLANE + c), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(b_lo_src + round * b_step + c),
                                       (lds_ptr)(base + 2 * TL::A_PLANE + TL::B_PLANE + c), 16, 0,
                                       0);
    }
  };
  const int frag = lane * 8;  // operand order: lane l reads the l-th 16 bytes of a group
  auto compute = [&](const unsigned short* st) {
    const unsigned short* a_hi = st;
    const unsigned short* a_lo = st + TL::A_PLANE;
    const unsigned short* b_hi = st + 2 * TL::A_PLANE;
    const unsigned short* b_lo = st + 2 * TL::A_PLANE + TL::B_PLANE;
    bf8 ah[TL::MI], al[TL::MI], bh[TL::NI], bl[TL::NI];
#pragma unroll
    for (int i = 0; i < TL::MI; ++i) {
      const int off = (wm * TL::WTM + i * 16) * TL::LD + frag;
      ah[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const us8*>(a_hi + off));
      al[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const us8*>(a_lo + off));
    }
#pragma unroll
    for (int j = 0; j < TL::NI; ++j) {
      const int off = (wn * TL::WTN + j * 16) * TL::LD + frag;
      bh[j] = __builtin_bit_cast(bf8, *reinterpret_cast<const us8*>(b_hi + off));
      bl[j] = __builtin_bit_cast(bf8, *reinterpret_cast<const us8*>(b_lo + off));
    }
    // small terms first
#pragma unroll
    for (int i = 0; i < TL::MI; ++i)
#pragma unroll
      for (int j = 0; j < TL::NI; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
  };
  // round kt computes from stage kt % NS while the DMA of round kt + NS - 1
  // fills the stage that round kt - 1 used; before the barrier that opens
  // round kt + 1, that round's pieces (issued NS - 2 rounds earlier) must
  // have landed, which leaves this round's DMA_PW instructions in flight
  for (int r = 0; r < NS - 1; ++r)
    if (r < nk) stage_in(r, r);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const bool issue = kt + NS - 1 < nk;
    if (issue) stage_in(kt + NS - 1, (int)((kt + NS - 1) % NS));
    compute(lds + (int)(kt % NS) * TL::STAGE);
    if (NS > 2 && issue) {
      static_assert(DMA_PW <= 15, "vmcnt immediate");
      // vmcnt(DMA_PW): bits 3:0, expcnt and lgkmcnt left at their maximum
      __builtin_amdgcn_s_waitcnt((NS > 2 ? DMA_PW : 0) | 0x0F70);
    } else {
      __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
  }
  GemmArgs e;
  e.C = g.C;
  e.P = g.P;
  e.ldc = g.ldc;
  e.m = g.m;
  e.n = g.n;
  e.splits = g.splits;
  e.ldp = g.ldp;
  e.split_stride = g.split_stride;
  e.alpha = g.alpha;
  e.beta = g.beta;
  f32_epilogue<16, TL::MI, TL::NI, TL::WTM, TL::WTN>(e, ic, row0, col0, wm, wn, lane, acc);
}

template <class K>
hipError_t launch_items(K kernel, int threads, const GemmArgs& g, hipStream_t s) {
  const int64_t items = g.tiles_m * g.tiles_n * g.splits;
  if (items <= 0) return hipSuccess;
  if (items > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kernel, dim3((unsigned)items), dim3(threads), 0, s, g);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_f32(int tile_id, const GemmArgs& g, hipStream_t s) {
  switch (tile_id) {
    case 0: return launch_items(gemm_f32_kernel<128, 128, 32, 4, 2, 4, 16>, 512, g, s);
    case 1: return launch_items(gemm_f32_kernel<64, 64, 32, 2, 2, 4, 16>, 256, g, s);
    case 2: return launch_items(gemm_f32_kernel<256, 128, 32, 4, 4, 4, 16>, 1024, g, s);
    case 3: return launch_items(gemm_f32_kernel<256, 256, 32, 4, 4, 4, 32>, 1024, g, s);
    default: return hipErrorInvalidValue;
  }
}

template <class K>
hipError_t launch_persistent(K kernel, int threads, const BatchArgs& b, int grid, hipStream_t s) {
  if (b.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(threads), 0, s, b);
  return hipGetLastError();
}

// Tiles with a persistent batched form: all but the 256 x 256 tile, whose
// 64 accumulators per lane leave no room for the item loop's state.
bool batched_form_f32(int tile_id) { return tile_id >= 0 && tile_id <= 2; }

hipError_t launch_batched_f32(int tile_id, const BatchArgs& b, int grid, hipStream_t s) {
  switch (tile_id) {
    case 0: return launch_persistent(gemm_f32_batched_kernel<128, 128, 32, 4, 2, 4, 16>, 512, b, grid, s);
    case 1: return launch_persistent(gemm_f32_batched_kernel<64, 64, 32, 2, 2, 4, 16>, 256, b, grid, s);
    case 2: return launch_persistent(gemm_f32_batched_kernel<256, 128, 32, 4, 4, 4, 16>, 1024, b, grid, s);
    default: return hipErrorInvalidValue;
  }
}

template <class K>
int occupancy_of(K kernel, int threads) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess) return 1;
  return n < 1 ? 1 : n;
}

int batched_occupancy_f32(int tile_id) {
  switch (tile_id) {
    case 0: return occupancy_of(gemm_f32_batched_kernel<128, 128, 32, 4, 2, 4, 16>, 512);
    case 1: return occupancy_of(gemm_f32_batched_kernel<64, 64, 32, 2, 2, 4, 16>, 256);
    case 2: return occupancy_of(gemm_f32_batched_kernel<256, 128, 32, 4, 4, 4, 16>, 1024);
    default: return 1;
  }
}

template <class K>
hipError_t launch_x3(K kernel, int threads, const X3Args& g, hipStream_t s) {
  const int64_t items = g.tiles_m * g.tiles_n * g.splits;
  if (items <= 0) return hipSuccess;
  if (items > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kernel, dim3((unsigned)items), dim3(threads), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_bf16x3_split(const float* A, int64_t m, int64_t k, int64_t lda, const float* B,
                               int64_t n, int64_t ldb, const X3Args& g, hipStream_t s) {
  if (g.rows_p % XA_ROWS || g.cols_p % XB_COLS || g.kp % X3_K) return hipErrorInvalidValue;
  const int64_t ba = (g.rows_p / XA_ROWS) * ceil_div(g.kp, (int64_t)XA_K);
  const int64_t bb = (g.kp / X3_K) * (g.cols_p / XB_COLS);
  if (ba > 0x7fffffffLL || bb > 0x7fffffffLL) return hipErrorInvalidValue;
  const int vec_a = (reinterpret_cast<uintptr_t>(A) % 16 == 0 && lda % 4 == 0) ? 1 : 0;
  const int vec_b = (reinterpret_cast<uintptr_t>(B) % 16 == 0 && ldb % 4 == 0) ? 1 : 0;
  if (ba > 0)
    hipLaunchKernelGGL(x3_split_a_kernel, dim3((unsigned)ba), dim3(256), 0, s, A, m, k, lda, vec_a,
                       g.rows_p, g.kp, const_cast<unsigned short*>(g.a_hi),
                       const_cast<unsigned short*>(g.a_lo));
  if (bb > 0)
    hipLaunchKernelGGL(x3_split_b_kernel, dim3((unsigned)bb), dim3(256), 0, s, B, k, n, ldb, vec_b,
                       g.cols_p, g.kp, const_cast<unsigned short*>(g.b_hi),
                       const_cast<unsigned short*>(g.b_lo));
  return hipGetLastError();
}

hipError_t launch_gemm_bf16x3(int tile_id, const X3Args& g, hipStream_t s) {
  switch (tile_id) {
    case 0: return launch_x3(gemm_bf16x3_kernel<128, 128, 32, 2, 2, 2>, 256, g, s);
    case 1: return launch_x3(gemm_bf16x3_kernel<64, 64, 32, 2, 2, 2>, 256, g, s);
    case 2: return launch_x3(gemm_bf16x3_kernel<256, 128, 32, 4, 2, 2>, 512, g, s);
    case 3: return launch_x3(gemm_bf16x3_kernel<256, 256, 32, 4, 4, 2>, 1024, g, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cosma
