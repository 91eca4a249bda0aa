// Kernel launch interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cosma {

// One GEMM launch: items = tiles_m * tiles_n * splits work items, each a
// tile_m x tile_n block of C over the reduction range
// [split * k_split, min(k, (split + 1) * k_split)).
struct GemmArgs {
  const void* A;
  const void* B;
  void* C;           // result (splits == 1)
  void* P;           // partial blocks (splits > 1): P[split][row][col]
  int64_t lda, ldb, ldc;
  int64_t m, n, k;
  int64_t k_split;
  int64_t tiles_m, tiles_n, splits;
  int64_t ldp;           // row stride of a partial plane
  int64_t split_stride;  // elements between partial planes
  double alpha, beta;
  int group_m;
  int num_xcds;
  int vec_a, vec_b;      // operand rows may be read 16 bytes at a time
};

// Batches: problem descriptors in device memory, one persistent launch per
// tile variant.  Work items are numbered batch-wide, problem by problem
// (problem p owns items [first, first + tiles_m * tiles_n * splits), the
// problems of one launch contiguous); an item map in device memory names
// the problem of every item, and within a problem item i is split
// i / (tiles_m * tiles_n), tile i % (tiles_m * tiles_n) in row-major order.
struct BatchProblem {
  const void* A;
  const void* B;
  void* C;
  void* P;                 // partial planes P[split][row][col] (splits > 1)
  int64_t lda, ldb, ldc;
  int64_t m, n, k;
  int64_t k_split;         // reduction length per split (multiple of the tile's k)
  double alpha, beta;
  int64_t first;           // first work item of the problem in its launch
  int32_t tiles_m, tiles_n, splits;
  int32_t vec_a, vec_b;
  int32_t pad_;
};

// A launch's items are cut into contiguous chunks, one per XCD, each a run
// of whole problems: the workgroups of XCD x (blocks b with b % chunks == x)
// take items of chunk x first, so a problem's panels are fetched into one
// L2, and then help drain the other chunks in turn.
constexpr int kBatchChunks = 8;
struct BatchArgs {
  const BatchProblem* probs;  // every problem of the batch
  const int32_t* map;         // problem index of every item of the batch
  int64_t base;               // batch-wide number of this launch's first item
  int64_t count;              // items in this launch
  unsigned* counter;          // per chunk: next item to hand out (reset before the launch)
  int32_t chunks;             // chunks in use, 1..kBatchChunks
  int32_t pad_;
  int64_t chunk[kBatchChunks + 1];  // chunk x = launch items [chunk[x], chunk[x + 1])
};

// Problems travel to device memory inside kernel arguments (no host copy,
// so the enqueue needs no staging memory and can be captured into a graph).
constexpr int kStageProblems = 24;
struct BatchStage {
  BatchProblem* dst;
  int32_t count;
  BatchProblem p[kStageProblems];
};
hipError_t launch_batch_stage(const BatchStage& st, hipStream_t s);
// map[probs[p].first + i] = p for every item i of every problem p < nprobs.
hipError_t launch_batch_expand(const BatchProblem* probs, int64_t nprobs, int32_t* map,
                               hipStream_t s);
// Split-K reduction of the listed problems of a batch: C = alpha * sum_s P_s
// + beta * C, summed in ascending s (as splitk_reduce).
constexpr int kReduceList = 900;
struct BatchReduceArgs {
  const BatchProblem* probs;
  int32_t count;
  int32_t idx[kReduceList];
};
hipError_t launch_batch_reduce(int dtype, const BatchReduceArgs& r, int64_t max_elems,
                               hipStream_t s);

// FP64 MFMA GEMM (tile menu kTilesF64).
hipError_t launch_gemm_f64(int tile_id, const GemmArgs& g, hipStream_t s);
// FP32 MFMA GEMM (tile menu kTilesF32).
hipError_t launch_gemm_f32(int tile_id, const GemmArgs& g, hipStream_t s);
// BF16x3: operands pre-split into bf16 hi / lo planes in staging order
// (element (row, k) of A at ((k / 32) * rows_p + row) * 32 + k % 32; B
// transposed likewise with cols_p); rows_p, cols_p multiples of 256 / 128,
// kp of 32, padding zero.
struct X3Args {
  const unsigned short* a_hi;
  const unsigned short* a_lo;
  const unsigned short* b_hi;
  const unsigned short* b_lo;
  void* C;
  void* P;
  int64_t ldc;
  int64_t m, n, kp;          // kp: padded k
  int64_t rows_p, cols_p;    // padded plane extents
  int64_t k_split;           // multiple of 32
  int64_t tiles_m, tiles_n, splits;
  int64_t ldp, split_stride;
  double alpha, beta;
  int group_m, num_xcds;
};
// Split pass (writes the four planes) and the GEMM on them (tile menu
// kTilesBf16x3).
hipError_t launch_bf16x3_split(const float* A, int64_t m, int64_t k, int64_t lda, const float* B,
                               int64_t n, int64_t ldb, const X3Args& g, hipStream_t s);
hipError_t launch_gemm_bf16x3(int tile_id, const X3Args& g, hipStream_t s);

// Persistent batched launches (grid = resident workgroups) for a tile variant.
hipError_t launch_batched_f64(int tile_id, const BatchArgs& b, int grid, hipStream_t s);
hipError_t launch_batched_f32(int tile_id, const BatchArgs& b, int grid, hipStream_t s);
// counter[0..n) = 0 with a kernel (graph-capture safe).
hipError_t launch_reset_counters(unsigned* counter, int n, hipStream_t s);
// Resident workgroups per CU of a tile variant (from the compiled kernel).
int batched_occupancy(int dtype, int tile_id);

// C = alpha * sum_{s < splits} P[s] + beta * C, summed in ascending s.
hipError_t launch_splitk_reduce_f64(const double* P, int64_t split_stride, int64_t ldp,
                                    int64_t splits, double* C, int64_t ldc, int64_t m, int64_t n,
                                    double alpha, double beta, hipStream_t s);
hipError_t launch_splitk_reduce_f32(const float* P, int64_t split_stride, int64_t ldp,
                                    int64_t splits, float* C, int64_t ldc, int64_t m, int64_t n,
                                    float alpha, float beta, hipStream_t s);
// C = beta * C (beta == 0 writes zeros without reading C).
hipError_t launch_scale_f64(double* C, int64_t ldc, int64_t m, int64_t n, double beta,
                            hipStream_t s);
hipError_t launch_scale_f32(float* C, int64_t ldc, int64_t m, int64_t n, float beta,
                            hipStream_t s);

}  // namespace cosma
