// Kernel tile menus and the work-item raster.  Shared by the host planner and
// the device kernels so that the planner's I/O model walks exactly the order
// the kernels run in.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define COSMA_HD __host__ __device__
#else
#define COSMA_HD
#endif

namespace cosma {

enum Dtype : int {
  F64 = 0,
  F32 = 1,
  F32_BF16X3 = 2,
  F64_OZAKI_I8 = 3,
  F64_OZAKI2_I8 = 4,
  F64_OZAKI_BF16 = 5,
  NUM_DTYPES = 6
};

// One compiled kernel variant: a tile_m x tile_n block of C per work item,
// k streamed in rounds of tile_k (one LDS stage per round, double-buffered).
struct TileDesc {
  int tm, tn, tk;
  int threads;     // workgroup size
  int wg_per_cu;   // resident workgroups per CU (LDS / register limited)
  double eff;      // planner's expectation of sustained MFMA issue fraction
};

// Menus, one per dtype; index = tile_id.  Order does not matter to the planner.
constexpr TileDesc kTilesF64[] = {
    {128, 128, 16, 512, 2, 0.87},
    {64, 64, 16, 256, 4, 0.75},
    {256, 128, 16, 1024, 1, 0.855},
};
constexpr TileDesc kTilesF32[] = {
    {128, 128, 32, 512, 2, 0.86},
    {64, 64, 32, 256, 4, 0.70},
    {256, 128, 32, 1024, 1, 0.865},
    {256, 256, 32, 1024, 1, 0.895},
};
constexpr TileDesc kTilesBf16x3[] = {
    {128, 128, 32, 256, 2, 0.48},
    {64, 64, 32, 256, 4, 0.35},
    {256, 128, 32, 512, 1, 0.45},
    {256, 256, 32, 1024, 1, 0.57},
};
constexpr TileDesc kTilesOzaki[] = {
    {128, 64, 64, 256, 1, 0.60},
};
constexpr TileDesc kTilesOzaki2[] = {
    {256, 128, 64, 512, 2, 0.45},
};
constexpr TileDesc kTilesOzakiBf16[] = {
    {128, 64, 32, 512, 1, 0.46},
};

COSMA_HD inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
COSMA_HD inline int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

// Workgroups are handed to the XCDs round-robin (block b runs on XCD b % X).
// Give each XCD a contiguous chunk of logical item ids, so that items that
// share A row-panels and B column-panels meet in the same L2.  Bijective on
// [0, G).
COSMA_HD inline int64_t xcd_remap(int64_t b, int64_t G, int X) {
  if (X <= 1) return b;
  const int64_t q = G / X, r = G % X;
  const int64_t x = b % X, local = b / X;
  return x * q + (x < r ? x : r) + local;
}

struct ItemCoord {
  int64_t tile_row, tile_col, split;
};

// Logical item id -> (tile row, tile column, k split).  Splits are outermost
// (items of one split share panels); within a split, tiles run in groups of
// group_m tile rows, column by column inside a group.
COSMA_HD inline ItemCoord item_coord(int64_t l, int64_t tiles_m, int64_t tiles_n, int group_m) {
  ItemCoord c;
  const int64_t T = tiles_m * tiles_n;
  c.split = l / T;
  const int64_t t = l - c.split * T;
  const int64_t per_group = (int64_t)group_m * tiles_n;
  const int64_t g = t / per_group;
  const int64_t first = g * group_m;
  const int64_t gm = min64(tiles_m - first, group_m);
  const int64_t in = t - g * per_group;
  c.tile_row = first + in % gm;
  c.tile_col = in / gm;
  return c;
}

}  // namespace cosma
