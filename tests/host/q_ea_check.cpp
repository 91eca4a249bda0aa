// Host-only check of the planner's L2 <-> memory traffic model: compares
// q_ea_bytes with a direct walk that visits every work item of every wave in
// the launch order (xcd_remap chunks, item_coord raster), collects the
// distinct A row-panels and B column-panels each wave touches and adds their
// bytes.  Built with g++ by tests/test_host_sanitizers.py; exits non-zero on
// the first mismatch.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_1908_09606_amd/csrc/planner.hpp"
#include "../../paper_1908_09606_amd/csrc/tiles.hpp"

using namespace cosma;

static double walk(int64_t m, int64_t n, int64_t k, int64_t k_split, int64_t splits, int tm,
                   int tn, int group_m, int64_t slots_per_xcd, int num_xcds, double w) {
  const int64_t tiles_m = ceil_div(m, tm), tiles_n = ceil_div(n, tn);
  const int64_t items = tiles_m * tiles_n * splits;
  const int X = std::max(1, num_xcds);
  const int64_t q = items / X, r = items % X;
  double bytes = 0.0;
  for (int x = 0; x < X; ++x) {
    const int64_t begin = x * q + std::min<int64_t>(x, r);
    const int64_t count = q + (x < r ? 1 : 0);
    for (int64_t w0 = 0; w0 < count; w0 += slots_per_xcd) {
      const int64_t w1 = std::min(count, w0 + slots_per_xcd);
      std::vector<int64_t> rows, cols;
      for (int64_t l = begin + w0; l < begin + w1; ++l) {
        const ItemCoord c = item_coord(l, tiles_m, tiles_n, group_m);
        rows.push_back(c.split * tiles_m + c.tile_row);
        cols.push_back(c.split * tiles_n + c.tile_col);
      }
      std::sort(rows.begin(), rows.end());
      rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
      std::sort(cols.begin(), cols.end());
      cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
      for (int64_t key : rows) {
        const int64_t tr = key % tiles_m, sp = key / tiles_m;
        const int64_t klen = std::min<int64_t>(k_split, k - sp * k_split);
        bytes += (double)std::min<int64_t>(tm, m - tr * tm) * (double)klen * w;
      }
      for (int64_t key : cols) {
        const int64_t tc = key % tiles_n, sp = key / tiles_n;
        const int64_t klen = std::min<int64_t>(k_split, k - sp * k_split);
        bytes += (double)std::min<int64_t>(tn, n - tc * tn) * (double)klen * w;
      }
    }
  }
  return bytes;
}

int main() {
  unsigned long long s = 0x243F6A8885A308D3ull;
  auto rnd = [&](int64_t lo, int64_t hi) {  // uniform in [lo, hi]
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return lo + (int64_t)((s >> 33) % (unsigned long long)(hi - lo + 1));
  };
  const int tms[] = {64, 128, 256};
  int checked = 0;
  for (int it = 0; it < 20000; ++it) {
    const int tm = tms[rnd(0, 2)], tn = tms[rnd(0, 2)];
    // sizes from a few tiles up to ~60 tiles per side, often ragged
    const int64_t m = rnd(1, 60) * tm - (rnd(0, 1) ? rnd(0, tm - 1) : 0);
    const int64_t n = rnd(1, 60) * tn - (rnd(0, 1) ? rnd(0, tn - 1) : 0);
    const int64_t kc = 16;
    const int64_t k = rnd(1, 4096);
    const int64_t req = rnd(1, 8);
    const int64_t k_split = ceil_div(ceil_div(k, kc), req) * kc;
    const int64_t splits = ceil_div(k, k_split);
    const int group_m = (int)std::min<int64_t>(rnd(1, 16), ceil_div(m, tm) + rnd(0, 2));
    const int64_t slots = rnd(1, 130);
    const int X = (int)rnd(1, 8);
    const double w = (double)rnd(1, 16);
    if (m <= 0 || n <= 0) continue;
    const double a = q_ea_bytes(m, n, k, k_split, splits, tm, tn, group_m, slots, X, w);
    const double b = walk(m, n, k, k_split, splits, tm, tn, group_m, slots, X, w);
    if (a != b) {
      std::fprintf(stderr,
                   "mismatch m=%lld n=%lld k=%lld k_split=%lld splits=%lld tm=%d tn=%d g=%d "
                   "slots=%lld X=%d w=%g: %.17g vs walk %.17g\n",
                   (long long)m, (long long)n, (long long)k, (long long)k_split,
                   (long long)splits, tm, tn, group_m, (long long)slots, X, w, a, b);
      return 1;
    }
    ++checked;
  }
  // the benchmark's square FP64 launch: 256x128 tiles, group_m 2, 32 slots per XCD
  const double sq = q_ea_bytes(16384, 16384, 16384, 16384, 1, 256, 128, 2, 32, 8, 8.0);
  const double sqw = walk(16384, 16384, 16384, 16384, 1, 256, 128, 2, 32, 8, 8.0);
  if (sq != sqw) {
    std::fprintf(stderr, "square mismatch %.17g vs %.17g\n", sq, sqw);
    return 1;
  }
  std::printf("q_ea check ok: %d random launches, square %.6g bytes\n", checked, sq);
  return 0;
}
