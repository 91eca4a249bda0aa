// Device side of the persistent batched launches: the item a workgroup
// takes and its problem's launch arguments, held in scalar registers (the
// whole workgroup works on one item, so every such value is the same in all
// lanes).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "tiles.hpp"
#include "uniform.hpp"

namespace cosma {

// The next item of a launch for the calling thread's workgroup (called by
// one thread): the workgroup's own chunk first, then the following chunks
// in turn; -1 once every chunk is drained.  `step` (initially 0) counts the
// chunks the workgroup has found drained.  A counter keeps counting past
// its chunk's end, at most once per workgroup, so every chunk is left after
// finitely many tries.
__device__ __forceinline__ int64_t batch_take(const BatchArgs& b, int& step) {
  const int x0 = (int)(blockIdx.x % (unsigned)b.chunks);
  while (step < b.chunks) {
    int x = x0 + step;
    if (x >= b.chunks) x -= b.chunks;
    const int64_t lo = b.chunk[x], size = b.chunk[x + 1] - lo;
    if (size > 0) {
      const unsigned got = atomicAdd(b.counter + x, 1u);
      if ((int64_t)got < size) return lo + (int64_t)got;
    }
    ++step;
  }
  return -1;
}

// Launch arguments and coordinates of batch item `it` (batch-wide number
// b.base + it), as gemm_{f32,f64}_kernel would see them for the problem's
// own launch under its tile and split.
__device__ __forceinline__ void batch_item(const BatchArgs& b, unsigned it, GemmArgs& g,
                                           ItemCoord& ic) {
  const int64_t gi = b.base + (int64_t)it;
  const int pi = __builtin_amdgcn_readfirstlane(b.map[gi]);
  const BatchProblem& p = b.probs[pi];
  g.A = uniform_ptr(p.A);
  g.B = uniform_ptr(p.B);
  g.C = uniform_ptr(p.C);
  g.P = uniform_ptr(p.P);
  g.lda = uniform_i64(p.lda);
  g.ldb = uniform_i64(p.ldb);
  g.ldc = uniform_i64(p.ldc);
  g.m = uniform_i64(p.m);
  g.n = uniform_i64(p.n);
  g.k = uniform_i64(p.k);
  g.k_split = uniform_i64(p.k_split);
  const int tiles_m = __builtin_amdgcn_readfirstlane(p.tiles_m);
  const int tiles_n = __builtin_amdgcn_readfirstlane(p.tiles_n);
  g.tiles_m = tiles_m;
  g.tiles_n = tiles_n;
  g.splits = __builtin_amdgcn_readfirstlane(p.splits);
  g.ldp = g.n;
  g.split_stride = g.m * g.n;
  g.alpha = uniform_f64(p.alpha);
  g.beta = uniform_f64(p.beta);
  g.group_m = 1;
  g.num_xcds = 1;
  g.vec_a = __builtin_amdgcn_readfirstlane(p.vec_a);
  g.vec_b = __builtin_amdgcn_readfirstlane(p.vec_b);
  const int64_t tiles = (int64_t)tiles_m * tiles_n;
  const int64_t local = gi - uniform_i64(p.first);
  ic.split = local / tiles;
  const int64_t t = local - ic.split * tiles;
  ic.tile_row = t / tiles_n;
  ic.tile_col = t - ic.tile_row * tiles_n;
}

}  // namespace cosma
