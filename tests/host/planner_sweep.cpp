// Host-only driver for the sanitizer test: sweeps the planner and the
// modular-path parameter code over many shapes, dtypes, devices and forced
// tiles / splits, and checks the invariants every plan must satisfy.  Built
// with g++ -fsanitize=address,undefined by tests/test_host_sanitizers.py;
// exits non-zero on the first violated invariant.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <initializer_list>

#include "../../paper_1908_09606_amd/csrc/crt.hpp"
#include "../../paper_1908_09606_amd/csrc/planner.hpp"

using namespace cosma;

static int fails = 0;
#define CHECK(cond, ...)                      \
  do {                                        \
    if (!(cond)) {                            \
      std::fprintf(stderr, "FAIL %s: ", #cond); \
      std::fprintf(stderr, __VA_ARGS__);      \
      std::fprintf(stderr, "\n");             \
      if (++fails > 20) std::exit(1);         \
    }                                         \
  } while (0)

// real: the device's fast memory holds the menu's tiles, so Theorem 1 applies
// (the degenerate devices of the sweep have far less than one tile's worth)
static void check_plan(const cosma_plan_info& p, int64_t m, int64_t n, int64_t k, int dtype,
                       bool real) {
  int cnt = 0;
  const TileDesc* menu = tile_menu(dtype, &cnt);
  CHECK(p.tile_id >= 0 && p.tile_id < cnt, "tile %d", p.tile_id);
  if (m == 0 || n == 0 || k == 0) return;
  const TileDesc& T = menu[p.tile_id];
  CHECK(p.tile_m == T.tm && p.tile_n == T.tn && p.tile_k == T.tk, "tile shape");
  CHECK(p.p_m == (m + T.tm - 1) / T.tm && p.p_n == (n + T.tn - 1) / T.tn, "grid");
  CHECK(p.p_k >= 1 && p.k_split >= T.tk && p.k_split % T.tk == 0, "split %d %lld", p.p_k,
        (long long)p.k_split);
  CHECK((int64_t)p.p_k * p.k_split >= k && (int64_t)(p.p_k - 1) * p.k_split < k,
        "splits cover k exactly once: %d x %lld vs %lld", p.p_k, (long long)p.k_split,
        (long long)k);
  CHECK(p.group_m >= 1, "group");
  if (real)
    CHECK(p.q_cu_words >= p.thm1_words * (1 - 1e-9), "Theorem 1: %g < %g", p.q_cu_words,
          p.thm1_words);
  CHECK(std::isfinite(p.predicted_ms) && p.predicted_ms > 0, "time %g", p.predicted_ms);
  CHECK(p.workspace_bytes == workspace_bytes(p), "workspace");
  if (dtype == F64_OZAKI2_I8) CHECK(p.k_split <= OZAKI2_MAX_K_ITEM, "oz2 split");
  if (dtype == F64_OZAKI_I8) CHECK(p.k_split <= 8192, "oz split");
}

int main() {
  const int64_t dims[] = {0, 1, 17, 64, 65, 257, 1000, 4096};
  const int64_t ks[] = {0, 1, 65, 1000, 70000};
  cosma_device_facts devs[3];
  devs[0] = mi355x_defaults();
  devs[1] = mi355x_defaults();
  devs[1].num_cus = 1;
  devs[1].num_xcds = 1;
  devs[1].lds_bytes_per_cu = 64;
  devs[1].vgpr_bytes_per_cu = 64;
  devs[2] = mi355x_defaults();
  devs[2].num_cus = 7;
  devs[2].num_xcds = 3;
  for (int dv = 0; dv < 3; ++dv)
    for (int dtype = 0; dtype < NUM_DTYPES; ++dtype)
      for (int64_t m : dims)
        for (int64_t n : {(int64_t)1, (int64_t)257, (int64_t)4096})
          for (int64_t k : ks) {
            cosma_plan_info p;
            const cosma_device_facts& f = devs[dv];
            const int rc = make_plan(m, n, k, dtype, f, 0.03, -1, -1, &p);
            CHECK(rc == COSMA_OK, "make_plan %lld %lld %lld dtype %d rc %d", (long long)m,
                  (long long)n, (long long)k, dtype, rc);
            if (rc == COSMA_OK) check_plan(p, m, n, k, dtype, dv == 0);
            if (dv != 0 || m > 1000) continue;
            int cnt = 0;
            tile_menu(dtype, &cnt);
            for (int t = 0; t < cnt; ++t)
              for (int pk : {1, 3, 16}) {
                cosma_plan_info q;
                if (make_plan(m, n, k, dtype, f, 0.0, t, pk, &q, 4096 * 8) == COSMA_OK)
                  check_plan(q, m, n, k, dtype, true);
              }
          }
  // grid fitting and the I/O counter
  for (int64_t p = 1; p <= 300; p += 7) {
    int64_t grid[3], used = 0;
    CHECK(fit_ranks(1000, 2000, 3000, p, 0.03, grid, &used), "fit_ranks %lld", (long long)p);
    CHECK(grid[0] * grid[1] * grid[2] == used && used <= p, "grid product");
  }
  CHECK(io_count(100, 200, 300, 64, 64, 16, 2, true) > 0, "io_count");
  // modular parameters: M / 4 holds k 2^(2 beta)
  for (int nm = CRT_MIN_MODULI; nm <= CRT_MAX_MODULI; ++nm)
    for (int64_t k : {1LL, 2LL, 1000LL, 65536LL, 1LL << 30}) {
      CrtParams cp;
      if (!crt_params(k, nm, &cp)) continue;
      unsigned __int128 M = 1;
      for (int l = 0; l < nm; ++l) M *= (unsigned __int128)cp.p[l];
      const unsigned __int128 need = ((unsigned __int128)k << (2 * cp.beta)) * 4;
      CHECK(2 * cp.beta + 66 < 128 || need <= M, "beta bound");
      CHECK(cp.beta >= 1 && cp.beta <= CRT_MAX_BETA, "beta range %d", cp.beta);
      for (int l = 0; l < nm; ++l) {
        // T_l = 1 mod p_l and 0 mod the other moduli, from its limbs
        for (int j = 0; j < nm; ++j) {
          long double r = 0;
          unsigned __int128 t = 0;
          for (int i = cp.limbs - 1; i >= 0; --i) t = (t << 30) + (unsigned __int128)cp.t[l][i];
          r = (long double)(t % (unsigned __int128)cp.p[j]);
          CHECK(r == (l == j ? 1.0L : 0.0L), "T_%d mod p_%d = %Lg", l, j, r);
        }
      }
    }
  if (fails) return 1;
  std::puts("planner sweep ok");
  return 0;
}
