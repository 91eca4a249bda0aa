// FP64-accurate GEMM from modular int8 products (Ozaki scheme II: Ozaki,
// Uchino & Imamura, "Ozaki Scheme II: A GEMM-oriented emulation of
// floating-point matrix multiplication using an integer modular technique",
// 2025).  The digit-slice path needs s(s+1)/2 int8 products for about 7s
// bits; this one needs one int8 product per modulus.
//
//   1. Exponents e_i, f_j of the row maxima of A and column maxima of B
//      (max < 2^e), shared with the digit path.
//   2. Integer operands A'_it = rint(A_it 2^(beta - e_i)) and
//      B'_tj = rint(B_tj 2^(beta - f_j)), |A'|, |B'| <= 2^beta (exact in
//      binary64).  beta is chosen on the host so that every
//      |sum_t A'_it B'_tj| <= k 2^(2 beta) <= M / 4, M = prod p_l.
//   3. Residues a_l = A' mod p_l, b_l = B' mod p_l, represented in
//      [-128, 127] (int8, p_l <= 256), one plane per modulus, stored as MFMA
//      operand fragments like the digit planes.
//   4. Products: (a_l b_l)_ij exact in int32 (v_mfma_i32_16x16x64_i8, at
//      most 65536 k per work item), reduced to y_l = (a_l b_l)_ij mod p_l
//      and stored as one byte per modulus and k split, in the order the
//      accumulators hold them.
//   5. Reconstruction (Chinese remainder theorem): r_l = sum_splits y_l,
//      X = sum_l r_l T_l with T_l = (M/p_l) ((M/p_l)^-1 mod p_l) mod M
//      (exact in binary64 limbs of 30 bits), C'_ij = X - M rint(X / M),
//      which equals sum_t A'_it B'_tj because |C'_ij| <= M / 4; then
//      C_ij = C'_ij 2^(e_i + f_j - 2 beta), rounded to binary64.
//
// The GEMM keeps a 256 x 128 block of C resident per work item and streams
// k in LDS-staged rounds like the other kernels (Algorithm 1 / section 5):
// binary64 is used only for the exponents, the scaling and residues, and
// the reconstruction.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstring>

#include "crt.hpp"
#include "kernels.hpp"
#include "ozaki.hpp"
#include "planner.hpp"
#include "runtime.hpp"
#include "tiles.hpp"
#include "uniform.hpp"

namespace cosma {
namespace {

typedef int i4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void* lds_ptr;

// Plane geometry.  For modulus l, row tile T (O2_BM rows of A, or O2_BN
// columns of B) and k round R (O2_BK values) there is one contiguous block
// of 1 KiB operand fragments of v_mfma_i32_16x16x64_i8: fragment f covers
// 16 rows (columns of B) and the round's 64 k; lane q = 16 g + r of the
// instruction reads bytes [16 q, 16 q + 16) = the residues of row 16 f + r
// at k = 64 R + 16 g .. + 15:
//   A: l * plane_a + T * crt_tile_stride(O2_BM, kp) + R * O2_BM * O2_BK
//        + ((row % O2_BM) / 16) * 1024 + (16 g + row % 16) * 16 + k % 16
//   B: likewise with col for row and O2_BN for O2_BM;
// plane_a = crt_plane_bytes(a_rows, O2_BM, kp), plane_b likewise.  Rows of
// padded tiles and k beyond the matrix hold zero residues.
constexpr int O2_BM = 256, O2_BN = 128, O2_BK = 64;
constexpr int64_t O2_MAX_K_ITEM = 65536;  // |sum| <= 65536 * 128^2 = 2^30

__device__ __forceinline__ int frag_off(int rr, int g) {
  return (rr >> 4) * 1024 + (g * 16 + (rr & 15)) * 16;
}

// A residue of an integer-valued x (|x| <= 2^50) modulo p that fits int8:
// r = x - p rint(x * pinv) is exact (one fused rounding of a small integer),
// and since x * pinv misses x / p by less than 2^-51 |x| / p, |x / p - q| <
// 1/2 + 1/(2p), so |r| < p / 2 + 1/2 <= 128 for odd p <= 255.  For p = 256
// the quotient is exact and r in [-128, 128]; its low byte is the
// two's-complement residue either way.  Any representative in [-128, 127]
// serves the int8 products (only r = x mod p matters), so no correction
// step is needed.
__device__ __forceinline__ unsigned residue_byte(double x, double p, double pinv) {
  return (unsigned)(int)fma(-p, rint(x * pinv), x) & 0xffu;
}

// 16 integer-valued doubles -> one 16-byte group of residues per modulus.
__device__ __forceinline__ void residues16(const double (&x)[16], const CrtParams& cp,
                                           int8_t* __restrict__ out, int64_t plane_stride) {
  for (int l = 0; l < cp.nmod; ++l) {
    const double p = (double)cp.p[l], pinv = cp.pinv[l];
    unsigned w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      unsigned v = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) v |= residue_byte(x[4 * q + b], p, pinv) << (8 * b);
      w[q] = v;
    }
    *reinterpret_cast<i4*>(out + l * plane_stride) = i4{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
  }
}

// A: one workgroup per 64 rows and one k round.  The block is read row by
// row (512 contiguous bytes per wave instruction), scaled to integers into
// LDS, and each wave then produces one 16-row fragment per modulus (a
// contiguous 1 KiB store per plane).
__global__ __launch_bounds__(256) void residue_a_kernel(const double* __restrict__ A, int64_t m,
                                                        int64_t k, int64_t lda,
                                                        const int* __restrict__ e, CrtParams cp,
                                                        int8_t* __restrict__ planes, int64_t rows_p,
                                                        int64_t kp) {
  __shared__ double tile[64][O2_BK + 1];
  const int64_t rounds = kp / O2_BK;
  const int64_t rb = blockIdx.x / rounds, R = blockIdx.x % rounds;
  const int t = threadIdx.x;
  // Wave w reads rows w, w + 4, ..., w + 60 of the block, lane kk its k:
  // 512 contiguous bytes per load, all 16 loads in flight at once (rows
  // and k beyond the matrix read a valid entry and are replaced by zero).
  {
    const int kk = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t kt = R * O2_BK + kk;
    double a[16];
    int ex[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int64_t row = rb * 64 + w + 4 * j;
      const bool ok = row < m && kt < k;
      a[j] = A[ok ? row * lda + kt : 0];
      ex[j] = e[row < m ? row : 0];
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int64_t row = rb * 64 + w + 4 * j;
      // A row marked non-finite has e = OZAKI_NONFINITE: the shift then
      // takes its finite entries to zero and leaves NaN / infinity, which
      // the magnitude test zeroes (finite rows stay below 2^50).
      double x = rint(ldexp(a[j], cp.beta - ex[j]));
      x = fabs(x) <= 0x1p60 ? x : 0.0;
      tile[w + 4 * j][kk] = row < m && kt < k ? x : 0.0;
    }
  }
  __syncthreads();
  const int lane = t & 63, w = t >> 6, g = lane >> 4, rr = lane & 15;
  const int r = 16 * w + rr;
  double x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = tile[r][16 * g + i];
  const int64_t row = rb * 64 + r;
  residues16(x, cp,
             planes + (row / O2_BM) * crt_tile_stride(O2_BM, kp) + R * (O2_BM * O2_BK) +
                 frag_off((int)(row % O2_BM), g),
             crt_plane_bytes(rows_p, O2_BM, kp));
}

// B: one workgroup per 64 columns and one k round; rows of B are read
// along n (512 contiguous bytes per wave instruction) and each wave emits
// one 16-column fragment per modulus.
__global__ __launch_bounds__(256) void residue_b_kernel(const double* __restrict__ B, int64_t k,
                                                        int64_t n, int64_t ldb,
                                                        const int* __restrict__ f, CrtParams cp,
                                                        int8_t* __restrict__ planes, int64_t cols_p,
                                                        int64_t kp) {
  __shared__ double tile[O2_BK][64 + 1];
  const int64_t rounds = kp / O2_BK;
  const int64_t cb = blockIdx.x / rounds, R = blockIdx.x % rounds;
  const int t = threadIdx.x;
  // Wave w reads k rows w, w + 4, ..., w + 60 of the round, lane cc its
  // column: 512 contiguous bytes per load, all 16 in flight at once.
  {
    const int cc = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t col = cb * 64 + cc;
    const int fc = f[col < n ? col : 0];
    double b[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int64_t kt = R * O2_BK + w + 4 * j;
      b[j] = B[col < n && kt < k ? kt * ldb + col : 0];
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int64_t kt = R * O2_BK + w + 4 * j;
      double x = rint(ldexp(b[j], cp.beta - fc));  // non-finite columns: as for A
      x = fabs(x) <= 0x1p60 ? x : 0.0;
      tile[w + 4 * j][cc] = col < n && kt < k ? x : 0.0;
    }
  }
  __syncthreads();
  const int lane = t & 63, w = t >> 6, g = lane >> 4, rr = lane & 15;
  const int cc = 16 * w + rr;
  double x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = tile[16 * g + i][cc];
  const int64_t col = cb * 64 + cc;
  residues16(x, cp,
             planes + (col / O2_BN) * crt_tile_stride(O2_BN, kp) + R * (O2_BN * O2_BK) +
                 frag_off((int)(col % O2_BN), g),
             crt_plane_bytes(cols_p, O2_BN, kp));
}

// ---------------------------------------------------------------- GEMM
// Work item: (outer = split * nmod + l, tile); a 256 x 128 block of C for
// modulus l over the split's k range.  8 waves (4 along m, 2 along n) of
// 64 x 64, 16 blocks of 16 x 16 on v_mfma_i32_16x16x64_i8 per wave: lane
// q = 16 g + r supplies A[r][16g .. 16g+15] and B[16g .. 16g+15][r] and holds
// D[4g + v][r] in element v.  One round = 64 k.
//
// A round's 24 fragments (16 of A, 8 of B) go global -> LDS by 16-byte DMA
// (the planes are already fragments: each wave instruction moves one 1 KiB
// fragment) into one of three stages, two rounds ahead of the MFMAs; LDS per
// block 72 KiB, so two blocks share a CU.
constexpr int O2_STAGES = 3;
constexpr int O2_A_BLK = O2_BM * O2_BK, O2_B_BLK = O2_BN * O2_BK;
constexpr int O2_STAGE = O2_A_BLK + O2_B_BLK;
constexpr int O2_FRAGS = O2_STAGE / 1024;  // 24
constexpr int O2_WAVES = 8;
static_assert(O2_FRAGS % O2_WAVES == 0, "fragments per wave");

struct Oz2Args {
  const int8_t* a_planes;
  const int8_t* b_planes;
  uint8_t* y;               // residues [outer][tile][wave][block][lane][4 rows]
  int64_t m, n, kp;
  int64_t a_rows, b_cols;   // padded plane extents
  int64_t k_split;          // multiple of O2_BK
  int64_t tiles_m, tiles_n;
  int nmod, group_m, num_xcds;
  int32_t p[CRT_MAX_MODULI];
  double pinv[CRT_MAX_MODULI];
};

// Workgroup barrier that keeps the compiler from moving memory accesses
// across it but adds no wait of its own.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// s_waitcnt immediate for gfx9: vmcnt = v (low 4 bits at [3:0], high 2 at
// [15:14]), expcnt and lgkmcnt left at their maxima (no wait).
constexpr int waitcnt_vm(int v) { return (v & 15) | ((v >> 4) << 14) | (7 << 4) | (15 << 8); }

__global__ __launch_bounds__(O2_WAVES * 64) void ozaki2_gemm_kernel(Oz2Args g) {
  __shared__ __attribute__((aligned(1024))) int8_t lds[O2_STAGES * O2_STAGE];

  const int64_t li = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x, g.num_xcds);
  const ItemCoord ic = item_coord(li, g.tiles_m, g.tiles_n, g.group_m);
  const int mod = (int)(ic.split % g.nmod);
  const int64_t split = ic.split / g.nmod;
  const int64_t row0 = ic.tile_row * O2_BM, col0 = ic.tile_col * O2_BN;
  const int64_t kbeg = split * g.k_split;
  const int64_t kend = min64(g.kp, kbeg + g.k_split);
  const int64_t nk = kend > kbeg ? (kend - kbeg) / O2_BK : 0;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;  // rows 64 wm .., columns 64 wn ..
  const int lr = lane & 15, lg = lane >> 4;

  const int64_t rounds = g.kp / O2_BK;
  const int64_t rbeg = kbeg / O2_BK;
  const int8_t* a_src = g.a_planes + (int64_t)mod * crt_plane_bytes(g.a_rows, O2_BM, g.kp) +
                        ic.tile_row * crt_tile_stride(O2_BM, g.kp) + rbeg * O2_A_BLK + lane * 16;
  const int8_t* b_src = g.b_planes + (int64_t)mod * crt_plane_bytes(g.b_cols, O2_BN, g.kp) +
                        ic.tile_col * crt_tile_stride(O2_BN, g.kp) + rbeg * O2_B_BLK + lane * 16;

  i4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = i4{0, 0, 0, 0};

  // wave w moves fragments w, w + 8, w + 16 of a stage: 0..15 of A, 16..23 of B
  auto stage = [&](int64_t kt, int st) {
#pragma unroll
    for (int h = 0; h < O2_FRAGS / O2_WAVES; ++h) {
      const int q = wave + O2_WAVES * h;
      const int8_t* src = q < 16 ? a_src + kt * O2_A_BLK + q * 1024
                                 : b_src + kt * O2_B_BLK + (q - 16) * 1024;
      __builtin_amdgcn_global_load_lds((const void*)src, (lds_ptr)(lds + st * O2_STAGE + q * 1024),
                                       16, 0, 0);
    }
  };

  if (nk > 0) stage(0, 0);
  if (nk > 1) stage(1, 1);
  // round 0's fragments have landed when at most round 1's are in flight
  if (nk > 1)
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(O2_FRAGS / O2_WAVES));
  else
    __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int st = 0;
  for (int64_t kt = 0; kt < nk; ++kt) {
    // stage (kt + 2) % 3 was last read in round kt - 1, which every wave
    // finished before the barrier that closed it
    if (kt + 2 < nk) stage(kt + 2, st == 0 ? 2 : st - 1);
    const int8_t* base = lds + st * O2_STAGE + lane * 16;
    i4 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const i4*>(base + (wm * 4 + i) * 1024);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      b[j] = *reinterpret_cast<const i4*>(base + (16 + wn * 4 + j) * 1024);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i][j], 0, 0, 0);
    // round kt + 1 must have landed; round kt + 2's DMA may stay in flight.
    // A plain barrier (no release fence, which would wait for every DMA):
    // this wave's LDS reads are complete (the MFMAs consumed them) and its
    // own DMA for round kt + 1 is complete by the wait above.
    if (kt + 2 < nk)
      __builtin_amdgcn_s_waitcnt(waitcnt_vm(O2_FRAGS / O2_WAVES));
    else
      __builtin_amdgcn_s_waitcnt(0);
    lds_barrier();
    st = st == 2 ? 0 : st + 1;
  }

  // epilogue: y = acc mod p (exact: |acc| < 2^31, so floor(acc * pinv) is
  // within one of the quotient), stored in the accumulator layout: per
  // 16 x 16 block one dword per lane (its four rows), 256 contiguous bytes
  // per wave instruction
  const double p = (double)g.p[mod], pinv = g.pinv[mod];
  unsigned* yb = reinterpret_cast<unsigned*>(
      g.y + ic.split * g.a_rows * g.b_cols +
      (ic.tile_row * g.tiles_n + ic.tile_col) * (int64_t)(O2_BM * O2_BN) + wave * 4096);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      unsigned wv = 0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double x = (double)acc[i][j][v];
        double r = fma(-p, floor(x * pinv), x);
        r = r < 0.0 ? r + p : r;
        r = r >= p ? r - p : r;
        wv |= (unsigned)(int)r << (8 * v);
      }
      yb[(i * 4 + j) * 64 + lane] = wv;
    }
}

// ---------------------------------------------------------------- CRT
// Residue layout (written by the GEMM, read here): for outer index
// o = split * nmod + l, tile (T, U) of 256 x 128, wave w = 2 wm + wn, block
// (i, j) of 16 x 16 and lane q = 16 g + r, the dword at
//   o * a_rows * b_cols + (T * tiles_n + U) * 32768 + w * 4096
//     + (4 i + j) * 256 + 4 q
// holds the residues of rows 256 T + 64 wm + 16 i + 4 g + v (byte v) of
// column 128 U + 64 wn + 16 j + r.
struct CrtArgs {
  const uint8_t* y;
  const int* e;
  const int* f;
  double* C;
  int64_t ldc, m, n;
  int64_t tiles_n;          // 128-column tiles
  int64_t plane;            // a_rows * b_cols: bytes per outer index
  int64_t splits;
  double alpha, beta;
  CrtParams cp;
};

// Thread per residue dword: four rows of one column.  With T_l as in
// CrtParams, X = sum_l r_l T_l (r_l: the residue summed over the splits,
// not reduced) is congruent to C' modulo M; in 30-bit limbs every limb sum
// stays below 16 * 256 * splits * 2^30 < 2^53 (splits <= 1024), so X is
// exact, q = rint(X / M) < 2^22 and X - q M = C' is exact limb by limb.
template <int NM, int L, bool SPLIT>
__global__ __launch_bounds__(256) void crt_kernel(CrtArgs a) {
  // A tile's residues are 8192 dwords per outer index, 32 workgroups of 256
  // threads; the tile and its base address are the same for the whole
  // workgroup, so each load takes a scalar base and a 32-bit lane offset.
  const int64_t tile = blockIdx.x >> 5;
  const int dl = (int)(blockIdx.x & 31) * 256 + (int)threadIdx.x;  // dword in the tile
  if (tile * 32768 + (int64_t)dl * 4 >= a.plane) return;
  const int w = dl >> 10, blk = (dl >> 6) & 15, q = dl & 63;
  const int64_t row0 = (tile / a.tiles_n) * 256 + (w >> 1) * 64 + (blk >> 2) * 16 + (q >> 4) * 4;
  const int64_t col = (tile % a.tiles_n) * 128 + (w & 1) * 64 + (blk & 3) * 16 + (q & 15);
  if (row0 >= a.m || col >= a.n) return;
  const CrtParams& cp = a.cp;
  const int off = dl * 4;
  // dword of this thread for outer index o: a buffer load over the tile's
  // 32 KiB of that index (base in scalar registers, read through the first
  // lane) at the lane's 32-bit offset, so no lane computes a 64-bit address.
  // Descriptor: stride 0 (raw bytes), 32768 bytes in range, and the third
  // word's 32-bit data format that gfx9-family buffer loads expect.
  auto res = [&](int64_t o) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        (void*)uniform_ptr(a.y + tile * 32768 + o * a.plane), 0, 32768, 0x00020000);
    return (unsigned)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
  };
  double acc[4][L];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < L; ++i) acc[v][i] = 0.0;
  // acc[v] += r_l(v) T_l for every modulus.  The L limbs of T_l come from
  // the kernel arguments through scalar registers, which cannot hold all
  // NM * L of them at once: the products run modulus by modulus over all
  // four rows; empty asm statements on the residues before and the
  // accumulators after each modulus keep the compiler from regrouping the
  // products row by row (which would keep every limb live to the end) or
  // converting every residue up front.
  auto accumulate = [&](auto residue) {
#pragma unroll
    for (int l = 0; l < NM; ++l) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        unsigned rv = residue(l, v);
        asm volatile("" : "+v"(rv));  // converted here, not all up front
        const double r = (double)rv;
#pragma unroll
        for (int i = 0; i < L; ++i) acc[v][i] = fma(r, cp.t[l][i], acc[v][i]);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int i = 0; i < L; ++i) asm volatile("" : "+v"(acc[v][i]));
    }
  };
  if (!SPLIT) {  // one split: the launch's register count is that of this path alone
    // one dword per modulus, its bytes taken as the products need them
    unsigned x[NM];
#pragma unroll
    for (int l = 0; l < NM; ++l) x[l] = res(l);
    accumulate([&](int l, int v) { return (x[l] >> (8 * v)) & 0xffu; });
  } else {
    // residues of the four rows, summed over the splits
    unsigned sum[NM][4];
#pragma unroll
    for (int l = 0; l < NM; ++l) sum[l][0] = sum[l][1] = sum[l][2] = sum[l][3] = 0;
    for (int64_t s = 0; s < a.splits; ++s) {
#pragma unroll
      for (int l = 0; l < NM; ++l) {
        const unsigned x = res(s * NM + l);
#pragma unroll
        for (int v = 0; v < 4; ++v) sum[l][v] += (x >> (8 * v)) & 0xffu;
      }
    }
    accumulate([&](int l, int v) { return sum[l][v]; });
  }
  const int fj = a.f[col];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t row = row0 + v;
    if (row >= a.m) break;
    double X = acc[v][L - 1];
#pragma unroll
    for (int i = L - 2; i >= 0; --i) X = fma(X, 0x1p30, acc[v][i]);
    const double qm = rint(X * cp.m_inv);
    double u[L];
#pragma unroll
    for (int i = 0; i < L; ++i) u[i] = fma(-qm, cp.mlimb[i], acc[v][i]);
    // carries: limbs below the top one into [0, 2^30)
#pragma unroll
    for (int i = 0; i < L - 1; ++i) {
      const double c = floor(u[i] * 0x1p-30);
      u[i] = fma(-c, 0x1p30, u[i]);
      u[i + 1] += c;
    }
    // C' top-down: each step is floor(C' / 2^(30 i)), exact whenever that
    // fits in 53 bits, else rounded once
    double cpv = u[L - 1];
#pragma unroll
    for (int i = L - 2; i >= 0; --i) cpv = fma(cpv, 0x1p30, u[i]);
    const int er = a.e[row];
    const double r = (er == OZAKI_NONFINITE || fj == OZAKI_NONFINITE)
                         ? __builtin_nan("")
                         : ldexp(cpv, er + fj - 2 * cp.beta);
    double* out = a.C + row * a.ldc + col;
    const double yv = a.alpha * r;
    *out = a.beta != 0.0 ? yv + a.beta * *out : yv;
  }
}

template <int NM>
hipError_t launch_crt_nm(const CrtArgs& c, unsigned grid, hipStream_t s) {
  const bool split = c.splits > 1;
  if (c.cp.limbs <= 4) {
    if (split)
      hipLaunchKernelGGL((crt_kernel<NM, 4, true>), dim3(grid), dim3(256), 0, s, c);
    else
      hipLaunchKernelGGL((crt_kernel<NM, 4, false>), dim3(grid), dim3(256), 0, s, c);
  } else {
    if (split)
      hipLaunchKernelGGL((crt_kernel<NM, 5, true>), dim3(grid), dim3(256), 0, s, c);
    else
      hipLaunchKernelGGL((crt_kernel<NM, 5, false>), dim3(grid), dim3(256), 0, s, c);
  }
  return hipGetLastError();
}

hipError_t launch_crt(const CrtArgs& c, unsigned grid, hipStream_t s) {
  switch (c.cp.nmod) {
    case 2: return launch_crt_nm<2>(c, grid, s);
    case 3: return launch_crt_nm<3>(c, grid, s);
    case 4: return launch_crt_nm<4>(c, grid, s);
    case 5: return launch_crt_nm<5>(c, grid, s);
    case 6: return launch_crt_nm<6>(c, grid, s);
    case 7: return launch_crt_nm<7>(c, grid, s);
    case 8: return launch_crt_nm<8>(c, grid, s);
    case 9: return launch_crt_nm<9>(c, grid, s);
    case 10: return launch_crt_nm<10>(c, grid, s);
    case 11: return launch_crt_nm<11>(c, grid, s);
    case 12: return launch_crt_nm<12>(c, grid, s);
    case 13: return launch_crt_nm<13>(c, grid, s);
    case 14: return launch_crt_nm<14>(c, grid, s);
    case 15: return launch_crt_nm<15>(c, grid, s);
    case 16: return launch_crt_nm<16>(c, grid, s);
    default: return hipErrorInvalidValue;
  }
}

unsigned grid_for(int64_t threads) {
  int64_t b = (threads + 255) / 256;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

int run_ozaki2(const cosma_plan_info& plan, double alpha, const void* A, int64_t lda,
               const void* B, int64_t ldb, double beta, void* C, int64_t ldc, void* workspace,
               hipStream_t stream) {
  const int64_t m = plan.m, n = plan.n, k = plan.k;
  CrtParams cp;
  if (!crt_params(k, plan.slices, &cp)) return COSMA_ERR_UNSUPPORTED;
  if (plan.tile_m != O2_BM || plan.tile_n != O2_BN || plan.tile_k != O2_BK ||
      plan.k_split > O2_MAX_K_ITEM || plan.k_split % O2_BK)
    return COSMA_ERR_INVALID_ARG;
  if (plan.p_k > 1024) return COSMA_ERR_UNSUPPORTED;  // exact limb sums (see crt_kernel)
  const int64_t kp = ceil_div(k, O2_BK) * O2_BK;
  const int64_t a_rows = ceil_div(m, O2_BM) * O2_BM, b_cols = ceil_div(n, O2_BN) * O2_BN;
  const int64_t outer = (int64_t)plan.p_k * cp.nmod;
  const int64_t items = (int64_t)plan.p_m * plan.p_n * outer;
  if (a_rows / 64 * (kp / O2_BK) > 0x7fffffffLL || b_cols / 64 * (kp / O2_BK) > 0x7fffffffLL ||
      items > 0x7fffffffLL || ceil_div(a_rows * b_cols / 4, 256) > 0x7fffffffLL)
    return COSMA_ERR_UNSUPPORTED;
  // workspace layout (matches workspace_bytes): A planes | B planes | y | e, f
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  char* w = static_cast<char*>(workspace);
  int8_t* a_planes = reinterpret_cast<int8_t*>(w);
  const size_t plane_a = (size_t)crt_plane_bytes(a_rows, O2_BM, kp);
  const size_t plane_b = (size_t)crt_plane_bytes(b_cols, O2_BN, kp);
  int8_t* b_planes = a_planes + (size_t)cp.nmod * plane_a;
  const size_t planes = up((size_t)cp.nmod * (plane_a + plane_b));
  uint8_t* y = reinterpret_cast<uint8_t*>(w + planes);
  int* e = reinterpret_cast<int*>(w + planes + up((size_t)outer * a_rows * b_cols));
  int* f = e + m;

  hipError_t err = launch_ozaki_exponents(static_cast<const double*>(A), m, k, lda,
                                          static_cast<const double*>(B), n, ldb, e, f, stream);
  if (err != hipSuccess) return COSMA_ERR_HIP;
  hipLaunchKernelGGL(residue_a_kernel, dim3((unsigned)(a_rows / 64 * (kp / O2_BK))), dim3(256), 0,
                     stream, static_cast<const double*>(A), m, k, lda, e, cp, a_planes, a_rows, kp);
  hipLaunchKernelGGL(residue_b_kernel, dim3((unsigned)(b_cols / 64 * (kp / O2_BK))), dim3(256), 0,
                     stream, static_cast<const double*>(B), k, n, ldb, f, cp, b_planes, b_cols, kp);
  if ((err = hipGetLastError()) != hipSuccess) return COSMA_ERR_HIP;

  Oz2Args g;
  std::memset(&g, 0, sizeof(g));
  g.a_planes = a_planes;
  g.b_planes = b_planes;
  g.y = y;
  g.m = m;
  g.n = n;
  g.kp = kp;
  g.a_rows = a_rows;
  g.b_cols = b_cols;
  g.k_split = plan.k_split;
  g.tiles_m = plan.p_m;
  g.tiles_n = plan.p_n;
  g.nmod = cp.nmod;
  g.group_m = plan.group_m > 0 ? plan.group_m : 1;
  int st = COSMA_OK;
  g.num_xcds = device_facts(&st).num_xcds;
  for (int l = 0; l < cp.nmod; ++l) {
    g.p[l] = cp.p[l];
    g.pinv[l] = cp.pinv[l];
  }
  hipLaunchKernelGGL(ozaki2_gemm_kernel, dim3((unsigned)items), dim3(O2_WAVES * 64), 0, stream, g);
  if ((err = hipGetLastError()) != hipSuccess) return COSMA_ERR_HIP;

  CrtArgs c;
  c.y = y;
  c.e = e;
  c.f = f;
  c.C = static_cast<double*>(C);
  c.ldc = ldc;
  c.m = m;
  c.n = n;
  c.tiles_n = b_cols / O2_BN;
  c.plane = a_rows * b_cols;
  c.splits = plan.p_k;
  c.alpha = alpha;
  c.beta = beta;
  c.cp = cp;
  if ((err = launch_crt(c, grid_for(a_rows * b_cols / 4), stream)) != hipSuccess)
    return COSMA_ERR_HIP;
  return COSMA_OK;
}

}  // namespace cosma
