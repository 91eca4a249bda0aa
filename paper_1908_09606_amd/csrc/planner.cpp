// Host schedule planner.  See planner.hpp.
#include "planner.hpp"

#include "crt.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <utility>
#include <vector>

namespace cosma {

cosma_device_facts mi355x_defaults() {
  cosma_device_facts f;
  f.num_cus = 256;
  f.num_xcds = 8;
  f.lds_bytes_per_cu = 160 * 1024;
  f.vgpr_bytes_per_cu = 512 * 1024;
  f.l2_bytes_per_xcd = 4 * 1024 * 1024;
  f.clock_ghz = 2.4;
  f.hbm_gbps = 8000.0;
  return f;
}

const TileDesc* tile_menu(int dtype, int* count) {
  switch (dtype) {
    case F64: *count = (int)(sizeof(kTilesF64) / sizeof(TileDesc)); return kTilesF64;
    case F32: *count = (int)(sizeof(kTilesF32) / sizeof(TileDesc)); return kTilesF32;
    case F32_BF16X3: *count = (int)(sizeof(kTilesBf16x3) / sizeof(TileDesc)); return kTilesBf16x3;
    case F64_OZAKI_I8: *count = (int)(sizeof(kTilesOzaki) / sizeof(TileDesc)); return kTilesOzaki;
    case F64_OZAKI2_I8:
      *count = (int)(sizeof(kTilesOzaki2) / sizeof(TileDesc));
      return kTilesOzaki2;
    case F64_OZAKI_BF16:
      *count = (int)(sizeof(kTilesOzakiBf16) / sizeof(TileDesc));
      return kTilesOzakiBf16;
    default: *count = 0; return nullptr;
  }
}

int word_bytes(int dtype) {
  return (dtype == F64 || dtype == F64_OZAKI_I8 || dtype == F64_OZAKI2_I8 ||
          dtype == F64_OZAKI_BF16)
             ? 8
             : 4;
}
int partial_bytes(int dtype) { return word_bytes(dtype); }

namespace {

// Slice (or moduli) count forced through the environment, or -1.
int env_count(const char* name, int lo, int hi) {
  const char* e = std::getenv(name);
  if (!e || !*e) return -1;
  const int v = std::atoi(e);
  return v < lo ? lo : (v > hi ? hi : v);
}

std::atomic<double> g_spread{-1.0};

}  // namespace

int ozaki_slices() {
  static int s = env_count("COSMA_OZAKI_SLICES", 1, 8);
  return s;
}

int ozaki_bf16_slices() {
  static int s = env_count("COSMA_OZAKI_BF16_SLICES", 1, 8);
  return s;
}

int ozaki2_moduli() {
  static int s = env_count("COSMA_OZAKI2_MODULI", CRT_MIN_MODULI, CRT_MAX_MODULI);
  return s;
}

double ozaki_target_spread() {
  double v = g_spread.load();
  if (v >= 1.0) return v;
  const char* e = std::getenv("COSMA_OZAKI_SPREAD");
  v = e ? std::atof(e) : 0.0;
  if (!(v >= 1.0 && v < 1e300)) v = kDefaultOzakiSpread;
  g_spread.store(v);
  return v;
}

bool set_ozaki_target_spread(double v) {
  if (!(v >= 1.0 && v < 1e300)) return false;
  g_spread.store(v);
  return true;
}

// The error contract of the Ozaki paths.  Let e_i, f_j be the row / column
// exponents (max_t |A_it| < 2^e_i, max_t |B_tj| < 2^f_j), D_ij the sum
// |alpha| sum_t |A_it||B_tj| + |beta||C0_ij| and C_ij the exact result.
// Each path computes, up to binary64 rounding, the exact product of
// approximations of the scaled operands, and
//     |C^_ij - C_ij| <= |alpha| scaled * k 2^(e_i + f_j) + rounding * D_ij,
// with (unit roundoff u = 2^-53, gamma_n <= 1.01 n u):
//  - int8 digits, truncated (x = A 2^-e in (-1, 1), x = X + R with
//    X = sum_(u<=s) X_u, |X_u| <= 127 2^-7u, |R| < 2^-7s, |X| <= |x|):
//    xy - sum_(u+v<=s+1) X_u Y_v = sum_(u+v>=s+2) X_u Y_v + X R_y + R_x y,
//    at most (127/128)^2 (s-1) 2^-7s / (1 - 2^-7) + 2 2^-7s <= (s+1) 2^-7s
//    per term; the digits of x share its sign, so the s diagonal values
//    of a work item sum to at most sum_t |x_t||y_t| in magnitude, and the
//    binary64 steps (s - 1 additions, p_k - 1 split additions, alpha,
//    beta) give rounding = gamma_(s + p_k + 1).
//  - modular (Ozaki scheme II): A~ = 2^(e - beta) rint(A 2^(beta - e)) with
//    |A - A~| <= 2^(e - beta - 1), |A~| <= 2^e, so per term
//    |AB - A~B~| <= |A - A~||B~| + |A||B - B~| <= 2^(e + f - beta); the
//    integer product is exact, and the reconstruction rounds at most once
//    per 30-bit limb below the top one, then alpha and beta:
//    rounding = gamma_(limbs + 2) (1 + 2^-50).
//  - bf16 digits, rounded to nearest (|R| <= 2^-8s-1, |X_1| <= 1,
//    |X_u| <= 2^(7 - 8u) for u >= 2): dropped pairs have u, v >= 2, so the
//    per-term error is at most (s - 1) 2^(-8s-2) (1 - 2^-8)^-1 + 2^-8s-1
//    (1 + 2^-8s-1) + 2^-8s-1 <= (0.251 s + 0.751) 2^-8s.  From the first
//    non-zero digit of x on, sum_u |X_u| < 3.004 |x|; every 32-long round
//    adds s diagonal values to one binary64 accumulator, so
//    rounding = 9.03 gamma_(s ceil(k_item / 32) + p_k + 2).
// A binary64 reference product is itself within gamma_k D_ij of C_ij, so
// the normalised error against it stays within 4k 2^-53 wherever the
// spread rho_ij = k 2^(e_i + f_j) |alpha| / D_ij satisfies
//     scaled * rho_ij + rounding <= 3k 2^-53,
// i.e. rho_ij <= spread_limit.  (The scaled results must stay inside the
// normal binary64 range.)
OzakiBound ozaki_bound(int dtype, int slices, int64_t k, int64_t k_split, int64_t p_k) {
  OzakiBound b{0.0, 0.0, 0.0};
  if (k < 1 || slices < 1 || p_k < 1) return b;
  const double u = 0x1p-53;
  auto gamma = [&](double n) { return 1.01 * n * u; };
  const double s = (double)slices;
  if (k_split < 1 || k_split > k) k_split = k;
  switch (dtype) {
    case F64_OZAKI_I8:
      b.scaled = (s + 1.0) * std::ldexp(1.0, -7 * slices);
      b.rounding = gamma(s + (double)p_k + 1.0);
      break;
    case F64_OZAKI_BF16:
      b.scaled = (0.251 * s + 0.751) * std::ldexp(1.0, -8 * slices);
      b.rounding = 9.03 * gamma(s * (double)ceil_div(k_split, 32) + (double)p_k + 2.0);
      break;
    case F64_OZAKI2_I8: {
      CrtParams cp;
      if (!crt_params(k, slices, &cp)) return b;
      b.scaled = std::ldexp(1.0, -cp.beta) * (1.0 + 0x1p-50);
      b.rounding = gamma((double)cp.limbs + 2.0) * (1.0 + 0x1p-50);
      break;
    }
    default: return b;
  }
  const double room = 3.0 * (double)k * u - b.rounding;
  b.spread_limit = room > 0.0 ? room / b.scaled : 0.0;
  return b;
}

int ozaki_choose_slices(int dtype, int64_t k, double target) {
  int lo = 1, hi = 8;
  if (dtype == F64_OZAKI2_I8) {
    lo = CRT_MIN_MODULI;
    hi = CRT_MAX_MODULI;
  } else if (dtype != F64_OZAKI_I8 && dtype != F64_OZAKI_BF16) {
    return 0;
  }
  // the int8 digit path cuts k into items of at most 8192 (int32 sums)
  const int64_t item = dtype == F64_OZAKI_I8 ? std::min<int64_t>(k, 8192) : k;
  const int64_t pk = ceil_div(std::max<int64_t>(k, 1), std::max<int64_t>(item, 1));
  int best = hi;
  double best_scaled = INFINITY;
  for (int s = lo; s <= hi; ++s) {
    const OzakiBound b = ozaki_bound(dtype, s, std::max<int64_t>(k, 1), item, pk);
    if (b.spread_limit >= target) return s;
    if (b.scaled > 0.0 && b.scaled < best_scaled * (1.0 - 1e-12)) {
      best_scaled = b.scaled;
      best = s;
    }
  }
  return best;  // the most accurate emulation
}

double useful_flops_per_clk_per_cu(int dtype, int slices) {
  switch (dtype) {
    case F64: return 128.0;               // FP64 MFMA
    case F32: return 256.0;               // FP32 MFMA
    case F32_BF16X3: return 4096.0 / 3;   // three bf16 products per useful one
    case F64_OZAKI_I8: {                  // s(s+1)/2 int8 products per useful one
      const double pairs = slices * (slices + 1) / 2.0;
      return 8192.0 / (pairs > 0 ? pairs : 1.0);
    }
    case F64_OZAKI2_I8:                   // one int8 product per modulus
      return 8192.0 / (slices > 0 ? slices : 1);
    case F64_OZAKI_BF16: {                // s(s+1)/2 bf16 products per useful one
      const double pairs = slices * (slices + 1) / 2.0;
      return 4096.0 / (pairs > 0 ? pairs : 1.0);
    }
    default: return 1.0;
  }
}

// ---- the paper's schedule functions ------------------------------------

// Theorem 1: at least 2mnk/sqrt(S) + mn I/O operations.
double thm1_bound(double m, double n, double k, double S) {
  return 2.0 * m * n * k / std::sqrt(S) + m * n;
}

// Section 5: the optimal greedy step loads a elements of A and b of B while
// an a x b block of C stays resident; maximise ab/(a+b) under
// ab + a + 1 <= S.  For fixed a the best b is the largest feasible one, so a
// scan over a finds the integer optimum (the printed floors of eq. aopt /
// eq. bopt are close to, but not always equal to, this optimum).
void seq_schedule(int64_t S, int64_t* a_out, int64_t* b_out) {
  int64_t best_a = 0, best_b = 0;
  double best = -1.0;
  for (int64_t a = 1; a < S; ++a) {
    const int64_t b = (S - 1 - a) / a;
    if (b < 1) break;
    const double rho = (double)a * (double)b / (double)(a + b);
    if (rho > best * (1.0 + 1e-15)) {
      best = rho;
      best_a = a;
      best_b = b;
    }
  }
  *a_out = best_a;
  *b_out = best_b;
}

// eq. optTileShape: the local domain is a x a x b with a = min{sqrt S, V^(1/3)},
// b = max{V/S, V^(1/3)}, V = mnk/p.
void par_schedule(double m, double n, double k, double p, double S, double* a, double* b) {
  const double V = m * n * k / p;
  const double cube = std::cbrt(V);
  *a = std::min(std::sqrt(S), cube);
  *b = std::max(V / S, cube);
}

// Theorem 2 (per processor): min{2mnk/(p sqrt S) + S, 3 (mnk/p)^(2/3)}.
double thm2_bound(double m, double n, double k, double p, double S) {
  const double V = m * n * k / p;
  return std::min(2.0 * V / std::sqrt(S) + S, 3.0 * std::cbrt(V) * std::cbrt(V));
}

// Section 7.1: allow up to a fraction delta of the processors to idle when
// that gives a grid with less communication.  The local domain of grid
// (pm, pn, pk) is (m/pm) x (n/pn) x (k/pk); its surface -- the inputs and
// output it touches -- is the communication per processor.  Scan the used
// counts from p down and every factorisation; strict improvement only, so
// ties keep the larger used count.
bool fit_ranks(int64_t m, int64_t n, int64_t k, int64_t p, double delta, int64_t grid[3],
               int64_t* used) {
  if (m < 1 || n < 1 || k < 1 || p < 1 || delta < 0 || delta >= 1) return false;
  const int64_t lo = std::max<int64_t>(1, (int64_t)std::ceil((1.0 - delta) * (double)p - 1e-9));
  double best = INFINITY;
  for (int64_t q = p; q >= lo; --q) {
    for (int64_t pm = 1; pm <= q; ++pm) {
      if (q % pm) continue;
      const int64_t rest = q / pm;
      for (int64_t pn = 1; pn <= rest; ++pn) {
        if (rest % pn) continue;
        const int64_t pk = rest / pn;
        const double dm = (double)m / pm, dn = (double)n / pn, dk = (double)k / pk;
        const double surface = dm * dk + dn * dk + dm * dn;
        if (surface < best * (1.0 - 1e-12)) {
          best = surface;
          grid[0] = pm;
          grid[1] = pn;
          grid[2] = pk;
          *used = q;
        }
      }
    }
  }
  return true;
}

// Words moved by the tiled schedule.  Each work item keeps its block of C
// resident and reads, over its k range, every element of its A row-panel
// and B column-panel once: summed over items that is
// k * (m * ceil(n/tn) + n * ceil(m/tm)), independent of kc and of p_k.
// The output adds mn stores (Theorem 1's "+ mn"); with k split in p_k
// parts every item also stores its partial block and the reduction reloads
// all p_k partials before storing C; beta != 0 adds one load of C per entry.
double io_count(int64_t m, int64_t n, int64_t k, int64_t tm, int64_t tn, int64_t kc, int64_t pk,
                bool beta_nonzero) {
  if (m <= 0 || n <= 0 || tm <= 0 || tn <= 0 || kc <= 0 || pk <= 0 || k < 0) return 0.0;
  const double mn = (double)m * (double)n;
  const double operands =
      (double)k * ((double)m * (double)ceil_div(n, tn) + (double)n * (double)ceil_div(m, tm));
  double out = mn * (beta_nonzero ? 2.0 : 1.0);
  if (pk > 1) out += 2.0 * (double)pk * mn;
  return operands + out;
}

namespace {

// Elements covered by the tiles [t0, t1) of an extent `total` cut into
// `tiles` tiles of `t` (only the last tile can be partial).
double span_elems(int64_t t0, int64_t t1, int64_t tiles, int64_t t, int64_t total) {
  if (t1 <= t0) return 0.0;
  double e = (double)(t1 - t0) * (double)t;
  if (t1 == tiles) e -= (double)(tiles * t - total);
  return e;
}

}  // namespace

// Each wave of an XCD (slots_per_xcd consecutive items of its chunk) reads
// every distinct A row-panel and B column-panel its items touch once.  The
// distinct panels follow from the raster without visiting items: inside one
// split, a run of items of one raster group touches a cyclic run of the
// group's rows (all of them once the run is as long as the group is tall)
// and one contiguous range of columns; groups have disjoint rows, and their
// column ranges are merged.  The cost is one step per group a wave touches.
double q_ea_bytes(int64_t m, int64_t n, int64_t k, int64_t k_split, int64_t splits, int tm,
                  int tn, int group_m, int64_t slots_per_xcd, int num_xcds, double w_bytes) {
  const int64_t tiles_m = ceil_div(m, tm), tiles_n = ceil_div(n, tn);
  const int64_t T = tiles_m * tiles_n;
  const int64_t items = T * splits;
  if (items <= 0) return 0.0;
  const int X = std::max(1, num_xcds);
  const int64_t slots = std::max<int64_t>(1, slots_per_xcd);
  const int64_t gsz = std::max(1, group_m);
  const int64_t per_group = gsz * tiles_n;
  const int64_t q = items / X, r = items % X;
  double bytes = 0.0;
  std::vector<std::pair<int64_t, int64_t>> cols;
  for (int x = 0; x < X; ++x) {
    const int64_t begin = x * q + std::min<int64_t>(x, r);
    const int64_t count = q + (x < r ? 1 : 0);
    for (int64_t w0 = 0; w0 < count; w0 += slots) {
      const int64_t a = begin + w0, b = begin + std::min(count, w0 + slots);
      for (int64_t sp = a / T; sp * T < b; ++sp) {
        const int64_t ta = std::max(a, sp * T) - sp * T, tb = std::min(b, (sp + 1) * T) - sp * T;
        const int64_t klen = std::min<int64_t>(k_split, k - sp * k_split);
        double row_elems = 0.0;
        cols.clear();
        for (int64_t g = ta / per_group; g * per_group < tb; ++g) {
          const int64_t first = g * gsz, gm = std::min(tiles_m - first, gsz);
          const int64_t g0 = g * per_group;
          const int64_t ia = std::max(ta, g0) - g0, ib = std::min(tb, g0 + gm * tiles_n) - g0;
          if (ib <= ia) continue;
          // rows: item `in` of the group has row first + in % gm
          if (ib - ia >= gm) {
            row_elems += span_elems(first, first + gm, tiles_m, tm, m);
          } else {
            const int64_t r0 = ia % gm, r1 = r0 + (ib - ia);
            if (r1 <= gm) {
              row_elems += span_elems(first + r0, first + r1, tiles_m, tm, m);
            } else {
              row_elems += span_elems(first + r0, first + gm, tiles_m, tm, m);
              row_elems += span_elems(first, first + r1 - gm, tiles_m, tm, m);
            }
          }
          // columns: item `in` of the group has column in / gm
          cols.emplace_back(ia / gm, (ib - 1) / gm + 1);
        }
        std::sort(cols.begin(), cols.end());
        double col_elems = 0.0;
        int64_t c0 = -1, c1 = -1;
        for (const auto& c : cols) {
          if (c.first > c1) {
            col_elems += span_elems(c0, c1, tiles_n, tn, n);
            c0 = c.first;
            c1 = c.second;
          } else {
            c1 = std::max(c1, c.second);
          }
        }
        col_elems += span_elems(c0, c1, tiles_n, tn, n);
        bytes += (row_elems + col_elems) * (double)klen * w_bytes;
      }
    }
  }
  return bytes;
}

// Cost of one problem inside a persistent batch, where items of many
// problems share the machine and per-problem wave quantisation does not
// matter: the padded work of the tile at its expected issue rate against the
// tile's CU-level I/O (section 5's counted loads) at the memory rate.
double batch_item_cost(int64_t m, int64_t n, int64_t k, int dtype, int tile_id,
                       const cosma_device_facts& f) {
  int cnt = 0;
  const TileDesc* menu = tile_menu(dtype, &cnt);
  if (!menu || tile_id < 0 || tile_id >= cnt) return INFINITY;
  const TileDesc& T = menu[tile_id];
  const double padded = 2.0 * (double)(ceil_div(m, T.tm) * T.tm) *
                        (double)(ceil_div(n, T.tn) * T.tn) * (double)k;
  const double rate = useful_flops_per_clk_per_cu(dtype, ozaki_slices()) * f.clock_ghz * 1e9 *
                      (double)f.num_cus;
  const double t_compute = padded / (rate * T.eff);
  const double t_io = io_count(m, n, k, T.tm, T.tn, T.tk, 1, false) * word_bytes(dtype) /
                      (f.hbm_gbps * 1e9);
  return std::max(t_compute, t_io);
}

size_t workspace_bytes(const cosma_plan_info& p) {
  if (p.m <= 0 || p.n <= 0 || p.k <= 0) return 0;
  if (p.dtype == F64_OZAKI2_I8) {
    // residue planes of A (rows padded to 256) and of B (columns padded to
    // 128), k padded to 64; one residue byte per modulus, split and entry
    // of the padded C; then per-row / per-column exponents
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t kp = (size_t)ceil_div(p.k, 64) * 64;
    const size_t rows = (size_t)ceil_div(p.m, 256) * 256, cols = (size_t)ceil_div(p.n, 128) * 128;
    const size_t nm = (size_t)(p.slices > 0 ? p.slices : 0);
    const size_t planes = (size_t)crt_plane_bytes((int64_t)rows, 256, (int64_t)kp) +
                          (size_t)crt_plane_bytes((int64_t)cols, 128, (int64_t)kp);
    return up(nm * planes) + up((size_t)p.p_k * nm * rows * cols) +
           up(((size_t)p.m + (size_t)p.n) * sizeof(int32_t));
  }
  size_t ws = 0;
  if (p.p_k > 1) ws += (size_t)p.p_k * (size_t)p.m * (size_t)p.n * (size_t)partial_bytes(p.dtype);
  ws = (ws + 255) / 256 * 256;
  if (p.dtype == F32_BF16X3) {
    // bf16 hi and lo planes of A (rows padded to 256) and B (columns padded
    // to 256, transposed), k padded to 32
    const size_t kp = (size_t)ceil_div(p.k, 32) * 32;
    const size_t rows = (size_t)ceil_div(p.m, 256) * 256, cols = (size_t)ceil_div(p.n, 256) * 256;
    ws += (2 * 2 * kp * (rows + cols) + 255) / 256 * 256;
  }
  if (p.dtype == F64_OZAKI_BF16) {
    // bf16 digit planes of A (rows padded to 128) and of B (columns padded
    // to 64), k padded to 32, then per-row / per-column exponents
    const size_t kp = (size_t)ceil_div(p.k, 32) * 32;
    const size_t rows = (size_t)ceil_div(p.m, 128) * 128, cols = (size_t)ceil_div(p.n, 64) * 64;
    ws += (2 * (size_t)p.slices * kp * (rows + cols) + 255) / 256 * 256;
    ws += (((size_t)p.m + (size_t)p.n) * sizeof(int32_t) + 255) / 256 * 256;
  }
  if (p.dtype == F64_OZAKI_I8) {
    // digit planes of A (rows padded to 128) and of B (columns padded to 64),
    // k padded to 64, then per-row / per-column exponents
    const size_t kp = (size_t)ceil_div(p.k, 64) * 64;
    const size_t rows = (size_t)ceil_div(p.m, 128) * 128, cols = (size_t)ceil_div(p.n, 64) * 64;
    ws += ((size_t)p.slices * kp * (rows + cols) + 255) / 256 * 256;
    ws += (((size_t)p.m + (size_t)p.n) * sizeof(int32_t) + 255) / 256 * 256;
  }
  return ws;
}

namespace {

struct Candidate {
  int tile_id;
  int p_k;            // actual number of splits
  int64_t k_split;
  int group_m;
  int64_t items, waves;
  double q_cu, q_ea, t;
};

double launch_overhead_s() { return 4e-6; }

}  // namespace

bool conflicting_pitch(int64_t a_pitch_bytes) {
  return a_pitch_bytes > 0 && a_pitch_bytes % 4096 == 0;
}

int make_plan(int64_t m, int64_t n, int64_t k, int dtype, const cosma_device_facts& f,
              double delta, int tile_id, int p_k, cosma_plan_info* out, int64_t a_pitch_bytes) {
  if (!out || m < 0 || n < 0 || k < 0) return COSMA_ERR_INVALID_ARG;
  int ntiles = 0;
  const TileDesc* menu = tile_menu(dtype, &ntiles);
  if (!menu) return COSMA_ERR_INVALID_ARG;
  if (tile_id >= ntiles) return COSMA_ERR_INVALID_ARG;
  if (f.num_cus < 1 || f.num_xcds < 1 || f.clock_ghz <= 0 || f.hbm_gbps <= 0 ||
      f.lds_bytes_per_cu < 0 || f.vgpr_bytes_per_cu < 0)
    return COSMA_ERR_INVALID_ARG;
  if (!(delta >= 0.0 && delta < 1.0)) return COSMA_ERR_INVALID_ARG;

  std::memset(out, 0, sizeof(*out));
  out->m = m;
  out->n = n;
  out->k = k;
  out->dtype = dtype;
  const bool oz2 = dtype == F64_OZAKI2_I8;
  const bool ozb = dtype == F64_OZAKI_BF16;
  // Ozaki paths: the smallest slice (moduli) count whose error contract
  // covers the target spread at this k, unless forced through the
  // environment.
  const int forced = dtype == F64_OZAKI_I8 ? ozaki_slices()
                     : oz2                 ? ozaki2_moduli()
                     : ozb                 ? ozaki_bf16_slices()
                                           : 0;
  const bool ozaki = dtype == F64_OZAKI_I8 || oz2 || ozb;
  const int slices =
      !ozaki ? 0 : (forced > 0 ? forced : ozaki_choose_slices(dtype, k, ozaki_target_spread()));
  out->slices = slices;

  // Fast memory of one CU in words of the stored operand (an Ozaki word is
  // the s digit bytes of one element, two per digit on bf16, a modular word
  // its residue bytes).
  const double w = (dtype == F64_OZAKI_I8 || oz2) ? (double)slices
                   : ozb                          ? 2.0 * slices
                                                  : (double)word_bytes(dtype);
  const double S = std::max(3.0, (double)(f.lds_bytes_per_cu + f.vgpr_bytes_per_cu) / w);
  out->S_words = S;
  const double P = (double)f.num_cus;
  out->p1 = (double)m * (double)n / S;
  out->regime = P > out->p1 ? 1 : 0;
  int64_t a_seq = 0, b_seq = 0;
  seq_schedule((int64_t)S, &a_seq, &b_seq);
  out->a_seq = a_seq;
  out->b_seq = b_seq;
  if (m > 0 && n > 0 && k > 0) {
    par_schedule((double)m, (double)n, (double)k, P, S, &out->a_par, &out->b_par);
    out->thm1_words = thm1_bound((double)m, (double)n, (double)k, S);
    out->thm2_words = thm2_bound((double)m, (double)n, (double)k, P, S);
  }

  if (m == 0 || n == 0 || k == 0) {
    // BLAS quick returns: no products to schedule.
    const int id = tile_id >= 0 ? tile_id : 0;
    out->tile_id = id;
    out->tile_m = menu[id].tm;
    out->tile_n = menu[id].tn;
    out->tile_k = menu[id].tk;
    out->p_m = out->p_n = 0;
    out->p_k = 1;
    out->group_m = 1;
    out->wg_per_cu = menu[id].wg_per_cu;
    return COSMA_OK;
  }

  const double per_cu_rate = useful_flops_per_clk_per_cu(dtype, slices) * f.clock_ghz * 1e9;
  const double hbm = f.hbm_gbps * 1e9;
  const double pb = (double)partial_bytes(dtype);
  const double wb = (double)word_bytes(dtype);
  const double mn = (double)m * (double)n;
  const int cus_per_xcd = std::max(1, f.num_cus / f.num_xcds);

  // Rows of A whose pitch is a multiple of 4 KiB put the lines of one k
  // offset into the same L2 sets; sharing an A panel across the tiles of an
  // XCD then only works while the XCD's block holds few A rows (measured on
  // the square FP64 product: 1.04x / 1.15x / 1.8x / 2.2x the sharing model
  // with 256 / 512 / 1024 / 2048 rows).  Such pitches restrict the raster
  // groups to at most 512 A rows.
  if (a_pitch_bytes <= 0) a_pitch_bytes = k * (int64_t)word_bytes(dtype);
  const bool pow2_pitch =
      dtype != F64_OZAKI_I8 && !oz2 && !ozb && conflicting_pitch(a_pitch_bytes);
  // The modular path runs one GEMM per modulus in the same launch.
  const int64_t per_tile = oz2 ? slices : 1;
  static const int kSplits[] = {1,  2,  3,  4,  5,  6,   8,   10,  12,  16,  20,
                                24, 32, 48, 64, 96, 128, 192, 256, 384, 512};
  static const int kGroups[] = {1, 2, 4, 8, 16};
  std::vector<Candidate> cands;
  for (int id = 0; id < ntiles; ++id) {
    if (tile_id >= 0 && id != tile_id) continue;
    const TileDesc& T = menu[id];
    const int64_t panels = ceil_div(k, T.tk);
    const int64_t tiles = ceil_div(m, T.tm) * ceil_div(n, T.tn);
    // the planner searches its split menu; a forced split may be any count
    std::vector<int> reqs(kSplits, kSplits + sizeof(kSplits) / sizeof(kSplits[0]));
    if (p_k > 0) reqs.assign(1, p_k);
    for (int req : reqs) {
      if (p_k <= 0 && req > 1 && (double)k / req < 256.0) continue;  // keep rounds long
      const int64_t k_split = ceil_div(panels, req) * T.tk;
      const int64_t splits = ceil_div(k, k_split);
      // Ozaki: a work item's int32 diagonal sums stay exact for <= 8192 k
      if (dtype == F64_OZAKI_I8 && k_split > 8192) continue;
      // modular path: int32 sums of residue products stay exact
      if (oz2 && k_split > OZAKI2_MAX_K_ITEM) continue;
      if (p_k <= 0 && splits != req) continue;  // duplicate of a smaller request
      const int64_t items = tiles * splits * per_tile;
      const int64_t slots = (int64_t)f.num_cus * T.wg_per_cu;
      const int64_t waves = ceil_div(items, slots);
      const double item_flops = 2.0 * T.tm * T.tn * (double)k_split / (double)per_tile;
      const double t_compute = (double)waves * item_flops / (per_cu_rate / T.wg_per_cu) / T.eff;
      double best_q = INFINITY;
      int best_g = 1;
      for (int g : kGroups) {
        if (g > 1 && g > ceil_div(m, T.tm)) break;
        if (g > 1 && pow2_pitch && g * T.tm > 512) break;
        // modular path: per modulus a GEMM on one byte per element
        const double q = q_ea_bytes(m, n, k, k_split, splits, T.tm, T.tn, g,
                                    (int64_t)cus_per_xcd * T.wg_per_cu, f.num_xcds,
                                    oz2 ? 1.0 : w) *
                         (double)per_tile;
        if (q < best_q * (1.0 - 1e-12)) {
          best_q = q;
          best_g = g;
        }
      }
      // GEMM launch: operand panels + either C or the partial blocks (the
      // modular path: one residue byte per modulus, split and entry).
      const double out_bytes = oz2 ? (double)splits * slices * (double)(ceil_div(m, T.tm) * T.tm) *
                                         (double)(ceil_div(n, T.tn) * T.tn)
                                   : (splits > 1 ? (double)splits * mn * pb : mn * wb);
      const double gemm_bytes = best_q + out_bytes;
      // Reduce launch: reload the partials, store C (the modular path
      // always reconstructs from its residues).
      const double reduce_bytes =
          oz2 ? out_bytes + mn * wb : (splits > 1 ? (double)splits * mn * pb + mn * wb : 0.0);
      // Ozaki prologue: read A and B once, write their digit planes (the
      // modular path reads them twice: exponents, then residues).
      const double pre_bytes =
          dtype == F64_OZAKI_I8 ? ((double)m * k + (double)k * n) * (8.0 + slices)
          : ozb                 ? ((double)m * k + (double)k * n) * (8.0 + 2.0 * slices)
          : oz2                 ? ((double)m * k + (double)k * n) * (16.0 + slices)
                                : 0.0;
      const double q_ea = gemm_bytes + reduce_bytes + pre_bytes;
      const double t_mem = gemm_bytes / hbm;
      const double t_reduce =
          (splits > 1 || oz2) ? reduce_bytes / hbm + launch_overhead_s() : 0.0;
      // A tile that runs one block per CU exposes its epilogue: the C block
      // (or partial) leaves at the CU's share of the memory bandwidth while
      // nothing else computes on that CU.  With two or more blocks per CU
      // the others' rounds hide it.
      const double item_out_bytes =
          (double)T.tm * T.tn * (oz2 ? (double)slices : (splits > 1 ? pb : wb));
      const double t_epi =
          T.wg_per_cu == 1 ? (double)waves * item_out_bytes / (hbm / (double)f.num_cus) : 0.0;
      const double t_pre = pre_bytes > 0 ? pre_bytes / hbm + 2 * launch_overhead_s() : 0.0;
      Candidate c;
      c.tile_id = id;
      c.p_k = (int)splits;
      c.k_split = k_split;
      c.group_m = best_g;
      c.items = items;
      c.waves = waves;
      c.q_cu = io_count(m, n, k, T.tm, T.tn, T.tk, splits, false);
      c.q_ea = q_ea;
      c.t = std::max(t_compute, t_mem) + t_epi + t_reduce + t_pre + launch_overhead_s();
      cands.push_back(c);
    }
  }
  if (cands.empty()) return COSMA_ERR_INVALID_ARG;
  double t_best = INFINITY;
  for (const Candidate& c : cands) t_best = std::min(t_best, c.t);
  // Section 7.1's trade: accept up to a fraction delta more (modelled)
  // compute time for a schedule that moves less data.
  const Candidate* pick = nullptr;
  for (const Candidate& c : cands) {
    if (c.t > t_best * (1.0 + delta) + 1e-12) continue;
    if (!pick || c.q_cu < pick->q_cu * (1.0 - 1e-12) ||
        (c.q_cu <= pick->q_cu * (1.0 + 1e-12) && c.t < pick->t))
      pick = &c;
  }
  const TileDesc& T = menu[pick->tile_id];
  out->tile_id = pick->tile_id;
  out->tile_m = T.tm;
  out->tile_n = T.tn;
  out->tile_k = T.tk;
  out->p_m = (int32_t)ceil_div(m, T.tm);
  out->p_n = (int32_t)ceil_div(n, T.tn);
  out->p_k = pick->p_k;
  out->group_m = pick->group_m;
  out->wg_per_cu = T.wg_per_cu;
  out->k_split = pick->k_split;
  out->items = pick->items;
  out->waves = pick->waves;
  out->q_cu_words = pick->q_cu;
  out->q_ea_bytes = pick->q_ea;
  out->predicted_ms = pick->t * 1e3;
  const size_t ws = workspace_bytes(*out);
  out->workspace_bytes = ws;
  set_error_contract(out);
  return COSMA_OK;
}

void set_error_contract(cosma_plan_info* p) {
  p->err_scaled = p->err_rounding = p->spread_limit = 0.0;
  if (p->k < 1 || p->p_k < 1) return;
  const OzakiBound b = ozaki_bound(p->dtype, p->slices, p->k, p->k_split, p->p_k);
  p->err_scaled = b.scaled;
  p->err_rounding = b.rounding;
  p->spread_limit = b.spread_limit;
}

}  // namespace cosma
