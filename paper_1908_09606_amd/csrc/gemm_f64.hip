// FP64 GEMM on the CDNA4 matrix cores, the split-K reduction and the beta
// scaling used by the BLAS quick returns.
//
// Structure (Algorithm 1 / section 5 of the paper, one work item per
// workgroup): the workgroup keeps a BM x BN block of C resident in the
// waves' accumulator registers for its whole reduction range and streams k
// in rounds of BK.  Each round stages the BM x BK panel of A and the BK x BN
// panel of B in LDS (the DistrData step of Algorithm 1 moved one level down
// the memory hierarchy) while the matrix cores consume the previous round
// (double buffering, the overlap of section 7.3).  When k is split the item
// stores its partial block and splitk_reduce adds the partials (Reduce).
//
// Matrix-core operation: v_mfma_f64_16x16x4f64, D(16x16) += A(16x4) B(4x16).
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[4 * v + l / 16][l % 16] in accumulator element v (rows interleaved across
// the four lane groups; this differs from the FP32 form of the instruction,
// where element v of lane l is row 4 * (l / 16) + v).  The four k slots of
// one instruction are a sum, so their assignment to real k indices is free:
// lane group g = l / 16 takes k = 16 h + 4 g + s at step s of 16-wide chunk
// h, which lets a lane read its four A values of a chunk as one contiguous
// 32-byte run.
#include <hip/hip_runtime.h>

#include "batch_device.hpp"
#include "kernels.hpp"
#include "tiles.hpp"

namespace cosma {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

template <int BM, int BN, int BK, int WM, int WN>
struct F64Tile {
  static constexpr int NT = WM * WN * 64;       // threads
  static constexpr int WTM = BM / WM;           // wave tile rows
  static constexpr int WTN = BN / WN;           // wave tile cols
  static constexpr int MI = WTM / 16;           // MFMA blocks per wave (rows)
  static constexpr int NI = WTN / 16;           // MFMA blocks per wave (cols)
  static constexpr int LDA_S = BK + 2;          // As[row][k], padded
  static constexpr int LDB_S = BN + 2;          // Bs[k][col], padded
  static constexpr int A_CHUNKS = BM * BK / 2 / NT;  // double2 per thread
  static constexpr int B_CHUNKS = BK * BN / 2 / NT;
  static constexpr int A_STAGE = BM * LDA_S;
  static constexpr int B_STAGE = BK * LDB_S;
  static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "wave tiling");
  static_assert(BK % 16 == 0, "BK must be a multiple of 16");
  static_assert((BM * BK / 2) % NT == 0 && (BK * BN / 2) % NT == 0, "load tiling");
  static_assert(2 * (A_STAGE + B_STAGE) * 8 <= 160 * 1024, "LDS budget");
};

// Operand loads of one round, per operand in one of three modes:
// LOAD_VEC: 16-byte loads (base and row pitch 16-byte aligned, round in
// bounds); LOAD_SCALAR: two 8-byte loads, no checks (in bounds, pitch an odd
// number of elements); LOAD_CHECKED: element-wise with zero fill (edge tiles
// and the last partial round).
enum LoadMode { LOAD_VEC = 0, LOAD_SCALAR = 1, LOAD_CHECKED = 2 };

// Per-thread operand pointers of a work item at k = 0: chunk i of A is
// row c / (BK / 2), columns 2 (c % (BK / 2)) + {0, 1} of the panel, with
// c = t + NT i, i.e. pa + i (NT / (BK / 2)) lda; chunk i of B is row
// c / (BN / 2), i.e. pb + i (NT / (BN / 2)) ldb.  A round then adds one
// scalar offset per chunk.
template <class TL, int BM, int BN, int BK>
__device__ __forceinline__ void operand_bases(const GemmArgs& g, int64_t row0, int64_t col0,
                                              const double*& pa, const double*& pb) {
  static_assert(TL::NT % (BK / 2) == 0 && TL::NT % (BN / 2) == 0, "chunk rows");
  const int t = threadIdx.x;
  pa = static_cast<const double*>(g.A) + (row0 + t / (BK / 2)) * g.lda + (t % (BK / 2)) * 2;
  pb = static_cast<const double*>(g.B) + (int64_t)(t / (BN / 2)) * g.ldb + col0 +
       (t % (BN / 2)) * 2;
}

template <class TL, int BM, int BN, int BK, int MODE>
__device__ __forceinline__ void load_a(const GemmArgs& g, int64_t row0, int64_t k0, int64_t kend,
                                       const double* pa, d2 (&ra)[TL::A_CHUNKS]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < TL::A_CHUNKS; ++i) {
    const double* p = pa + (int64_t)i * (TL::NT / (BK / 2)) * g.lda + k0;
    if (MODE == LOAD_VEC) {
      ra[i] = *reinterpret_cast<const d2*>(p);
    } else if (MODE == LOAD_SCALAR) {
      ra[i].x = p[0];
      ra[i].y = p[1];
    } else {
      const int c = t + TL::NT * i;
      const int64_t gr = row0 + c / (BK / 2), gk = k0 + (c % (BK / 2)) * 2;
      const bool rin = gr < g.m;
      ra[i].x = (rin && gk < kend) ? p[0] : 0.0;
      ra[i].y = (rin && gk + 1 < kend) ? p[1] : 0.0;
    }
  }
}

template <class TL, int BM, int BN, int BK, int MODE>
__device__ __forceinline__ void load_b(const GemmArgs& g, int64_t col0, int64_t k0, int64_t kend,
                                       const double* pb, d2 (&rb)[TL::B_CHUNKS]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < TL::B_CHUNKS; ++i) {
    const double* p = pb + (k0 + (int64_t)i * (TL::NT / (BN / 2))) * g.ldb;
    if (MODE == LOAD_VEC) {
      rb[i] = *reinterpret_cast<const d2*>(p);
    } else if (MODE == LOAD_SCALAR) {
      rb[i].x = p[0];
      rb[i].y = p[1];
    } else {
      const int c = t + TL::NT * i;
      const int64_t gk = k0 + c / (BN / 2), gc = col0 + (c % (BN / 2)) * 2;
      const bool kin = gk < kend;
      rb[i].x = (kin && gc < g.n) ? p[0] : 0.0;
      rb[i].y = (kin && gc + 1 < g.n) ? p[1] : 0.0;
    }
  }
}

// One round's A and B panels into registers.  FAST (a full tile with both
// operands 16-byte aligned, decided once per work item): vector loads,
// element-wise only in a partial last round; the common case keeps this
// short loop body.  Otherwise each operand takes its own mode; a_in / b_in
// say whether the tile's rows of A / columns of B all lie inside the matrix.
template <class TL, int BM, int BN, int BK, bool FAST>
__device__ __forceinline__ void load_round(const GemmArgs& g, int64_t row0, int64_t col0,
                                           int64_t k0, int64_t kend, bool a_in, bool b_in,
                                           const double* pa, const double* pb,
                                           d2 (&ra)[TL::A_CHUNKS], d2 (&rb)[TL::B_CHUNKS]) {
  const bool k_in = k0 + BK <= kend;
  if (FAST) {
    if (k_in) {
      load_a<TL, BM, BN, BK, LOAD_VEC>(g, row0, k0, kend, pa, ra);
      load_b<TL, BM, BN, BK, LOAD_VEC>(g, col0, k0, kend, pb, rb);
    } else {
      load_a<TL, BM, BN, BK, LOAD_CHECKED>(g, row0, k0, kend, pa, ra);
      load_b<TL, BM, BN, BK, LOAD_CHECKED>(g, col0, k0, kend, pb, rb);
    }
    return;
  }
  if (a_in && k_in) {
    if (g.vec_a)
      load_a<TL, BM, BN, BK, LOAD_VEC>(g, row0, k0, kend, pa, ra);
    else
      load_a<TL, BM, BN, BK, LOAD_SCALAR>(g, row0, k0, kend, pa, ra);
  } else {
    load_a<TL, BM, BN, BK, LOAD_CHECKED>(g, row0, k0, kend, pa, ra);
  }
  if (b_in && k_in) {
    if (g.vec_b)
      load_b<TL, BM, BN, BK, LOAD_VEC>(g, col0, k0, kend, pb, rb);
    else
      load_b<TL, BM, BN, BK, LOAD_SCALAR>(g, col0, k0, kend, pb, rb);
  } else {
    load_b<TL, BM, BN, BK, LOAD_CHECKED>(g, col0, k0, kend, pb, rb);
  }
}

template <class TL, int BM, int BN, int BK>
__device__ __forceinline__ void store_round(double* __restrict__ As, double* __restrict__ Bs,
                                            const d2 (&ra)[TL::A_CHUNKS],
                                            const d2 (&rb)[TL::B_CHUNKS]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < TL::A_CHUNKS; ++i) {
    const int c = t + TL::NT * i;
    const int r = c / (BK / 2);
    const int kk = (c % (BK / 2)) * 2;
    *reinterpret_cast<d2*>(As + r * TL::LDA_S + kk) = ra[i];
  }
#pragma unroll
  for (int i = 0; i < TL::B_CHUNKS; ++i) {
    const int c = t + TL::NT * i;
    const int r = c / (BN / 2);
    const int nn = (c % (BN / 2)) * 2;
    *reinterpret_cast<d2*>(Bs + r * TL::LDB_S + nn) = rb[i];
  }
}

// One work item: the BM x BN block (ic.tile_row, ic.tile_col) over the
// reduction range of split ic.split.  As / Bs: two LDS stages each.
template <int BM, int BN, int BK, int WM, int WN, bool FAST>
__device__ __forceinline__ void f64_tile_body(const GemmArgs& g, const ItemCoord& ic,
                                              double (*As)[F64Tile<BM, BN, BK, WM, WN>::A_STAGE],
                                              double (*Bs)[F64Tile<BM, BN, BK, WM, WN>::B_STAGE]) {
  using TL = F64Tile<BM, BN, BK, WM, WN>;
  const int64_t row0 = ic.tile_row * BM, col0 = ic.tile_col * BN;
  const int64_t kbeg = ic.split * g.k_split;
  const int64_t kend = min64(g.k, kbeg + g.k_split);
  const int64_t nk = ceil_div(kend - kbeg, BK);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int lr = lane & 15, lg = lane >> 4;

  const bool a_in = row0 + BM <= g.m, b_in = col0 + BN <= g.n;

  d4 acc[TL::MI][TL::NI];
#pragma unroll
  for (int i = 0; i < TL::MI; ++i)
#pragma unroll
    for (int j = 0; j < TL::NI; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const double* pa;
  const double* pb;
  operand_bases<TL, BM, BN, BK>(g, row0, col0, pa, pb);
  d2 ra[TL::A_CHUNKS], rb[TL::B_CHUNKS];
  if (nk > 0) {
    load_round<TL, BM, BN, BK, FAST>(g, row0, col0, kbeg, kend, a_in, b_in, pa, pb, ra, rb);
    store_round<TL, BM, BN, BK>(As[0], Bs[0], ra, rb);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    const bool more = kt + 1 < nk;
    if (more)
      load_round<TL, BM, BN, BK, FAST>(g, row0, col0, kbeg + (kt + 1) * BK, kend, a_in, b_in, pa,
                                       pb, ra, rb);
    const double* __restrict__ as = As[cur];
    const double* __restrict__ bs = Bs[cur];
    // waves in their product phase issue first: a wave that has reached the
    // LDS store and barrier of the round waits for the others anyway (about
    // 1 % on the large FP64 products; the FP32 and BF16x3 loops got slower
    // with it)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int h = 0; h < BK / 16; ++h) {
      d4 af[TL::MI];
      double bf[TL::NI][4];
#pragma unroll
      for (int i = 0; i < TL::MI; ++i) {
        const double* p = as + (wm * TL::WTM + i * 16 + lr) * TL::LDA_S + h * 16 + lg * 4;
        const d2 lo = *reinterpret_cast<const d2*>(p);
        const d2 hi = *reinterpret_cast<const d2*>(p + 2);
        af[i] = d4{lo.x, lo.y, hi.x, hi.y};
      }
#pragma unroll
      for (int j = 0; j < TL::NI; ++j)
#pragma unroll
        for (int s = 0; s < 4; ++s)
          bf[j][s] = bs[(h * 16 + lg * 4 + s) * TL::LDB_S + wn * TL::WTN + j * 16 + lr];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < TL::MI; ++i)
#pragma unroll
          for (int j = 0; j < TL::NI; ++j)
            acc[i][j] =
                __builtin_amdgcn_mfma_f64_16x16x4f64(af[i][s], bf[j][s], acc[i][j], 0, 0, 0);
    }
    __builtin_amdgcn_s_setprio(0);
    if (more) store_round<TL, BM, BN, BK>(As[cur ^ 1], Bs[cur ^ 1], ra, rb);
    __syncthreads();
  }

  // Epilogue: lane holds rows 4*v + lg of column lr of each 16x16 block.
  if (g.splits == 1) {
    double* __restrict__ C = static_cast<double*>(g.C);
    const double alpha = g.alpha, beta = g.beta;
#pragma unroll
    for (int i = 0; i < TL::MI; ++i)
#pragma unroll
      for (int j = 0; j < TL::NI; ++j) {
        const int64_t col = col0 + wn * TL::WTN + j * 16 + lr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = row0 + wm * TL::WTM + i * 16 + v * 4 + lg;
          if (row < g.m && col < g.n) {
            double* p = C + row * g.ldc + col;
            const double r = alpha * acc[i][j][v];
            *p = beta != 0.0 ? r + beta * *p : r;
          }
        }
      }
  } else {
    double* __restrict__ P = static_cast<double*>(g.P) + ic.split * g.split_stride;
#pragma unroll
    for (int i = 0; i < TL::MI; ++i)
#pragma unroll
      for (int j = 0; j < TL::NI; ++j) {
        const int64_t col = col0 + wn * TL::WTN + j * 16 + lr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = row0 + wm * TL::WTM + i * 16 + v * 4 + lg;
          if (row < g.m && col < g.n) P[row * g.ldp + col] = acc[i][j][v];
        }
      }
  }
}

// The two loop bodies are compiled apart and chosen once per work item.
template <int BM, int BN, int BK, int WM, int WN>
__device__ __forceinline__ void f64_tile(const GemmArgs& g, const ItemCoord& ic,
                                         double (*As)[F64Tile<BM, BN, BK, WM, WN>::A_STAGE],
                                         double (*Bs)[F64Tile<BM, BN, BK, WM, WN>::B_STAGE]) {
  const bool fast = (ic.tile_row + 1) * BM <= g.m && (ic.tile_col + 1) * BN <= g.n && g.vec_a &&
                    g.vec_b;
  if (fast)
    f64_tile_body<BM, BN, BK, WM, WN, true>(g, ic, As, Bs);
  else
    f64_tile_body<BM, BN, BK, WM, WN, false>(g, ic, As, Bs);
}

// ------------------------------------------------- DMA-staged form
// For launches of full tiles whose rows start 16-byte aligned and whose
// k ranges are whole rounds (BK = 16): the operands go from global memory
// straight into LDS (16-byte global-to-LDS loads, no staging registers, no
// LDS store instructions) into NS stages, NS - 1 rounds ahead of the
// products, so the latency of the slowest load of a round hides behind
// NS - 1 rounds of products instead of one.
//
// LDS per stage: A as BM rows of 16 doubles (128 bytes, no padding); the
// eight 16-byte chunks of row r sit at chunk positions c ^ ((r >> 1) & 7),
// so the 16 rows one MFMA operand read touches cover all banks.  B as 16
// rows of BN doubles with a row pitch of BN + 4 doubles.  One wave
// instruction moves 1 KiB: 8 rows of A, or one row of B (BN = 128).
template <int BM, int BN, int WM, int WN, int NS>
struct F64Dma {
  static constexpr int BK = 16;
  static constexpr int NW = WM * WN;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int MI = WTM / 16, NI = WTN / 16;
  static constexpr int LDB = BN + 4;               // doubles
  static constexpr int A_STAGE = BM * BK;          // doubles
  static constexpr int B_STAGE = BK * LDB;
  static constexpr int STAGE = A_STAGE + B_STAGE;
  static constexpr int A_PW = BM / 8 / NW;         // A instructions per wave and round
  static constexpr int B_PW = BK / NW;             // B instructions per wave and round
  static constexpr int PW = A_PW + B_PW;
  static_assert(BN == 128, "one B row per wave instruction");
  static_assert(A_PW * NW * 8 == BM && B_PW * NW == BK, "instruction split");
  static_assert(NS >= 2 && (NS - 2) * PW <= 15, "vmcnt immediate");
  static_assert(NS * STAGE * 8 <= 160 * 1024, "LDS budget");
};

typedef __attribute__((address_space(3))) void* lds_ptr;

__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// s_waitcnt immediate: vmcnt = v, expcnt and lgkmcnt at their maxima.
constexpr int vm_wait(int v) { return (v & 15) | ((v >> 4) << 14) | (7 << 4) | (15 << 8); }

template <int BM, int BN, int WM, int WN, int NS, int WPE>
__global__ __launch_bounds__(WM* WN * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void gemm_f64_dma_kernel(
    GemmArgs g) {
  using TL = F64Dma<BM, BN, WM, WN, NS>;
  constexpr int BK = TL::BK;
  __shared__ __attribute__((aligned(1024))) double lds[NS * TL::STAGE];
  const int64_t l = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x, g.num_xcds);
  const ItemCoord ic = item_coord(l, g.tiles_m, g.tiles_n, g.group_m);
  const int64_t row0 = ic.tile_row * BM, col0 = ic.tile_col * BN;
  const int64_t kbeg = ic.split * g.k_split;
  const int64_t kend = min64(g.k, kbeg + g.k_split);
  const int64_t nk = (kend - kbeg) / BK;  // whole rounds (checked by the launcher)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int lr = lane & 15, lg = lane >> 4;
  const double* A = static_cast<const double*>(g.A);
  const double* B = static_cast<const double*>(g.B);

  // this lane's source of each of the wave's DMA instructions at round 0
  const double* pa[TL::A_PW];
#pragma unroll
  for (int h = 0; h < TL::A_PW; ++h) {
    const int grp = wave + TL::NW * h;  // rows 8 grp .. 8 grp + 7
    const int r = 8 * grp + (lane >> 3);
    const int c = (lane & 7) ^ ((r >> 1) & 7);
    pa[h] = A + (row0 + r) * g.lda + kbeg + 2 * c;
  }
  const double* pb[TL::B_PW];
#pragma unroll
  for (int h = 0; h < TL::B_PW; ++h) {
    const int kr = wave + TL::NW * h;
    pb[h] = B + (kbeg + kr) * g.ldb + col0 + 2 * lane;
  }
  auto issue = [&](int64_t kt, int st) {
    double* sa = lds + st * TL::STAGE;
    double* sb = sa + TL::A_STAGE;
#pragma unroll
    for (int h = 0; h < TL::A_PW; ++h)
      __builtin_amdgcn_global_load_lds((const void*)(pa[h] + kt * BK),
                                       (lds_ptr)(sa + (wave + TL::NW * h) * 128), 16, 0, 0);
#pragma unroll
    for (int h = 0; h < TL::B_PW; ++h)
      __builtin_amdgcn_global_load_lds((const void*)(pb[h] + kt * BK * g.ldb),
                                       (lds_ptr)(sb + (wave + TL::NW * h) * TL::LDB), 16, 0, 0);
  };

  d4 acc[TL::MI][TL::NI];
#pragma unroll
  for (int i = 0; i < TL::MI; ++i)
#pragma unroll
    for (int j = 0; j < TL::NI; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // rounds 0 .. NS - 2 in flight; round 0 landed when at most the later
  // ones are outstanding (loads complete in issue order)
  for (int r = 0; r < NS - 1; ++r)
    if (r < nk) issue(r, r);
  if (nk >= NS - 1)
    __builtin_amdgcn_s_waitcnt(vm_wait((NS - 2) * TL::PW));
  else
    __builtin_amdgcn_s_waitcnt(0);
  lds_barrier();
  int st = 0;
  for (int64_t kt = 0; kt < nk; ++kt) {
    // the stage round kt + NS - 1 fills was read in round kt - 1, which
    // every wave finished before the barrier that closed it
    const bool ahead = kt + NS - 1 < nk;
    if (ahead) issue(kt + NS - 1, st == 0 ? NS - 1 : st - 1);
    const double* as = lds + st * TL::STAGE;
    const double* bs = as + TL::A_STAGE;
    __builtin_amdgcn_s_setprio(1);
    d4 af[TL::MI];
    double bf[TL::NI][4];
#pragma unroll
    for (int i = 0; i < TL::MI; ++i) {
      const int r = wm * TL::WTM + i * 16 + lr;
      const int sw = (r >> 1) & 7;
      const d2 lo = *reinterpret_cast<const d2*>(as + r * 16 + ((2 * lg) ^ sw) * 2);
      const d2 hi = *reinterpret_cast<const d2*>(as + r * 16 + ((2 * lg + 1) ^ sw) * 2);
      af[i] = d4{lo.x, lo.y, hi.x, hi.y};
    }
#pragma unroll
    for (int j = 0; j < TL::NI; ++j)
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
        bf[j][s4] = bs[(lg * 4 + s4) * TL::LDB + wn * TL::WTN + j * 16 + lr];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
      for (int i = 0; i < TL::MI; ++i)
#pragma unroll
        for (int j = 0; j < TL::NI; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i][s4], bf[j][s4], acc[i][j], 0, 0, 0);
    __builtin_amdgcn_s_setprio(0);
    // round kt + 1 must have landed before the barrier that opens it
    if (ahead)
      __builtin_amdgcn_s_waitcnt(vm_wait((NS - 2) * TL::PW));
    else
      __builtin_amdgcn_s_waitcnt(0);
    lds_barrier();
    st = st == NS - 1 ? 0 : st + 1;
  }

  // epilogue as gemm_f64_kernel's (full tile: no bounds checks needed, kept
  // for the split case's shared form)
  if (g.splits == 1) {
    double* __restrict__ C = static_cast<double*>(g.C);
    const double alpha = g.alpha, beta = g.beta;
#pragma unroll
    for (int i = 0; i < TL::MI; ++i)
#pragma unroll
      for (int j = 0; j < TL::NI; ++j) {
        const int64_t col = col0 + wn * TL::WTN + j * 16 + lr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = row0 + wm * TL::WTM + i * 16 + v * 4 + lg;
          double* p = C + row * g.ldc + col;
          const double r = alpha * acc[i][j][v];
          *p = beta != 0.0 ? r + beta * *p : r;
        }
      }
  } else {
    double* __restrict__ P = static_cast<double*>(g.P) + ic.split * g.split_stride;
#pragma unroll
    for (int i = 0; i < TL::MI; ++i)
#pragma unroll
      for (int j = 0; j < TL::NI; ++j) {
        const int64_t col = col0 + wn * TL::WTN + j * 16 + lr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = row0 + wm * TL::WTM + i * 16 + v * 4 + lg;
          P[row * g.ldp + col] = acc[i][j][v];
        }
      }
  }
}

// WPE: waves per SIMD the register allocation must allow (the tile menu's
// blocks per CU times WM * WN / 4).
template <int BM, int BN, int BK, int WM, int WN, int WPE>
__global__ __launch_bounds__(WM* WN * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void gemm_f64_kernel(
    GemmArgs g) {
  using TL = F64Tile<BM, BN, BK, WM, WN>;
  __shared__ __attribute__((aligned(16))) double As[2][TL::A_STAGE];
  __shared__ __attribute__((aligned(16))) double Bs[2][TL::B_STAGE];
  const int64_t l = xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x, g.num_xcds);
  const ItemCoord ic = item_coord(l, g.tiles_m, g.tiles_n, g.group_m);
  f64_tile<BM, BN, BK, WM, WN>(g, ic, As, Bs);
}

// Persistent batched form: workgroups take (problem, split, tile) items from
// the device counters until every chunk is drained; every item is computed as
// by gemm_f64_kernel under the problem's split (partials to its planes).
template <int BM, int BN, int BK, int WM, int WN, int WPE>
__global__ __launch_bounds__(WM* WN * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void gemm_f64_batched_kernel(
    BatchArgs b) {
  using TL = F64Tile<BM, BN, BK, WM, WN>;
  __shared__ __attribute__((aligned(16))) double As[2][TL::A_STAGE];
  __shared__ __attribute__((aligned(16))) double Bs[2][TL::B_STAGE];
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
    f64_tile<BM, BN, BK, WM, WN>(g, ic, As, Bs);
  }
}

__global__ void reset_counters_kernel(unsigned* __restrict__ c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0u;
}

template <typename T>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const T* __restrict__ P,
                                                            int64_t split_stride, int64_t ldp,
                                                            int64_t splits, T* __restrict__ C,
                                                            int64_t ldc, int64_t m, int64_t n,
                                                            T alpha, T beta) {
  const int64_t total = m * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t row = e / n, col = e - row * n;
    const T* p = P + row * ldp + col;
    T s = p[0];
    for (int64_t q = 1; q < splits; ++q) s += p[q * split_stride];
    T* c = C + row * ldc + col;
    const T r = alpha * s;
    *c = beta != T(0) ? r + beta * *c : r;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void scale_kernel(T* __restrict__ C, int64_t ldc, int64_t m,
                                                    int64_t n, T beta) {
  const int64_t total = m * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t row = e / n, col = e - row * n;
    T* c = C + row * ldc + col;
    *c = beta != T(0) ? beta * *c : T(0);
  }
}

unsigned elementwise_blocks(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// The DMA-staged form applies to full tiles with 16-byte aligned rows and
// whole 16-k rounds in every split (NS = 0: no such form for the tile).
template <int BM, int BN, int BK, int WM, int WN, int WPE, int NS>
hipError_t launch_f64(const GemmArgs& g, hipStream_t s) {
  const int64_t items = g.tiles_m * g.tiles_n * g.splits;
  if (items <= 0) return hipSuccess;
  if (items > 0x7fffffffLL) return hipErrorInvalidValue;
  if constexpr (NS > 0) {
    if (g.m % BM == 0 && g.n % BN == 0 && g.vec_a && g.vec_b && g.k % BK == 0 &&
        g.k_split % BK == 0 && g.k > 0) {
      hipLaunchKernelGGL((gemm_f64_dma_kernel<BM, BN, WM, WN, NS, WPE>), dim3((unsigned)items),
                         dim3(WM * WN * 64), 0, s, g);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, WPE>), dim3((unsigned)items),
                     dim3(WM * WN * 64), 0, s, g);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_f64(int tile_id, const GemmArgs& g, hipStream_t s) {
  switch (tile_id) {
    case 0: return launch_f64<128, 128, 16, 4, 2, 4, 2>(g, s);
    case 1: return launch_f64<64, 64, 16, 2, 2, 4, 0>(g, s);
    case 2: return launch_f64<256, 128, 16, 4, 4, 4, 3>(g, s);
    default: return hipErrorInvalidValue;
  }
}

namespace {

template <class K>
hipError_t launch_persistent(K kernel, int threads, const BatchArgs& b, int grid, hipStream_t s) {
  if (b.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(threads), 0, s, b);
  return hipGetLastError();
}

template <class K>
int occupancy_of(K kernel, int threads) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess) return 1;
  return n < 1 ? 1 : n;
}

}  // namespace

hipError_t launch_batched_f64(int tile_id, const BatchArgs& b, int grid, hipStream_t s) {
  switch (tile_id) {
    case 0: return launch_persistent(gemm_f64_batched_kernel<128, 128, 16, 4, 2, 4>, 512, b, grid, s);
    case 1: return launch_persistent(gemm_f64_batched_kernel<64, 64, 16, 2, 2, 4>, 256, b, grid, s);
    case 2: return launch_persistent(gemm_f64_batched_kernel<256, 128, 16, 4, 4, 4>, 1024, b, grid, s);
    default: return hipErrorInvalidValue;
  }
}

int batched_occupancy_f64(int tile_id) {
  switch (tile_id) {
    case 0: return occupancy_of(gemm_f64_batched_kernel<128, 128, 16, 4, 2, 4>, 512);
    case 1: return occupancy_of(gemm_f64_batched_kernel<64, 64, 16, 2, 2, 4>, 256);
    case 2: return occupancy_of(gemm_f64_batched_kernel<256, 128, 16, 4, 4, 4>, 1024);
    default: return 1;
  }
}

hipError_t launch_reset_counters(unsigned* counter, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(1024), 0, s, counter, n);
  return hipGetLastError();
}

hipError_t launch_splitk_reduce_f64(const double* P, int64_t split_stride, int64_t ldp,
                                    int64_t splits, double* C, int64_t ldc, int64_t m, int64_t n,
                                    double alpha, double beta, hipStream_t s) {
  hipLaunchKernelGGL(splitk_reduce_kernel<double>, dim3(elementwise_blocks(m * n)), dim3(256), 0,
                     s, P, split_stride, ldp, splits, C, ldc, m, n, alpha, beta);
  return hipGetLastError();
}

hipError_t launch_splitk_reduce_f32(const float* P, int64_t split_stride, int64_t ldp,
                                    int64_t splits, float* C, int64_t ldc, int64_t m, int64_t n,
                                    float alpha, float beta, hipStream_t s) {
  hipLaunchKernelGGL(splitk_reduce_kernel<float>, dim3(elementwise_blocks(m * n)), dim3(256), 0,
                     s, P, split_stride, ldp, splits, C, ldc, m, n, alpha, beta);
  return hipGetLastError();
}

hipError_t launch_scale_f64(double* C, int64_t ldc, int64_t m, int64_t n, double beta,
                            hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel<double>, dim3(elementwise_blocks(m * n)), dim3(256), 0, s, C,
                     ldc, m, n, beta);
  return hipGetLastError();
}

hipError_t launch_scale_f32(float* C, int64_t ldc, int64_t m, int64_t n, float beta,
                            hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel<float>, dim3(elementwise_blocks(m * n)), dim3(256), 0, s, C,
                     ldc, m, n, beta);
  return hipGetLastError();
}

}  // namespace cosma
