"""Pins of the oracle's I/O model against the paper (CPU only)."""
import math

import pytest

from oracle import schedule as sch


def test_xs_schedule_gap_at_ten_million_words():
    # Abstract / section 5 Corollary: the X = S schedule is within 0.03 % of
    # the lower bound for a fast memory of 10^7 words.
    f = sch.xs_factor(1e7)
    assert round((f - 1.0) * 100, 2) == 0.03
    assert f - 1.0 < 0.0004  # conclusion: "< 0.04 %"
    m, n, k, S = 1000, 2000, 3000, 1e7
    assert math.isclose(sch.xs_schedule_io(m, n, k, S) - m * n,
                        f * (sch.thm1_bound(m, n, k, S) - m * n), rel_tol=1e-12)


def test_sequential_optimum_square_block():
    # eq. seqSolution: a = b = sqrt(S), rho = sqrt(S)/2, and Q = |V|/rho + mn
    # equals Theorem 1.
    S = 10000
    rho = sch.rho_seq(100, 100)
    assert rho == math.sqrt(S) / 2
    m, n, k = 300, 500, 700
    assert math.isclose(m * n * k / rho + m * n, sch.thm1_bound(m, n, k, S), rel_tol=1e-15)
    assert math.isclose(sch.seq_greedy_io(m, n, k, 100, 100), sch.thm1_bound(m, n, k, S),
                        rel_tol=1e-15)


@pytest.mark.parametrize("S", [20480, 65536, 86016, 100000, 172032, 10 ** 6, 10 ** 7])
def test_aopt_bopt_closed_forms_vs_integer_search(S):
    a, b, rho = sch.seq_tile_search(S)
    assert a * b + a + 1 <= S
    ac, bc = sch.seq_tile_closed(S)
    assert ac * bc + ac + 1 <= S             # the printed floors are feasible
    assert ac < math.sqrt(S) and bc < math.sqrt(S)
    assert sch.rho_seq(ac, bc) >= (1 - 2e-3) * rho   # and near-optimal
    assert ac == math.floor(math.sqrt(S + 1) - 1)    # a_opt ~ sqrt(S+1) - 1
    # brute-force the integer optimum on a coarse grid
    best = max(sch.rho_seq(x, (S - 1 - x) // x) for x in range(1, int(2 * math.sqrt(S)))
               if (S - 1 - x) // x >= 1)
    assert math.isclose(best, rho, rel_tol=1e-15)


def test_opt_tile_shape_regimes():
    m = n = k = 4096
    S = 86016
    V = m * n * k
    p_switch = V / S ** 1.5          # a^2 <= S binds for p <= mnk / S^(3/2)
    a, b = sch.opt_tile_shape(m, n, k, int(p_switch // 2), S)
    assert a == math.sqrt(S) and math.isclose(a * a * b, V / int(p_switch // 2), rel_tol=1e-12)
    a, b = sch.opt_tile_shape(m, n, k, int(p_switch * 4), S)
    assert math.isclose(a, b) and a < math.sqrt(S)


@pytest.mark.parametrize("p", [1, 8, 64, 256, 4096, 10 ** 6])
def test_thm2_vs_schedule_cost(p):
    m, n, k, S = 8192, 8192, 8192, 86016
    cost = sch.par_schedule_cost(m, n, k, p, S)
    bound = sch.thm2_bound(m, n, k, p, S)
    a, _ = sch.opt_tile_shape(m, n, k, p, S)
    cubic = (m * n * k / p) ** (1 / 3)
    assert cost >= bound * (1 - 1e-12)
    if a < math.sqrt(S):
        assert math.isclose(cost, bound, rel_tol=1e-12)
    else:
        assert math.isclose(cost, 2 * m * n * k / (p * math.sqrt(S)) + S, rel_tol=1e-12)


def test_ij_regime_per_processor_io():
    m, n, k, S = 16384, 16384, 16384, 86016
    p = 256
    assert sch.p1(m, n, S) > p
    assert math.isclose(sch.ij_per_proc_io(m, n, k, p, S) * p, sch.thm1_bound(m, n, k, S), rel_tol=1e-12)
    assert sch.p1(2048, 2048, S) < 256   # the large-k shape cuts k on 256 CUs


def test_algorithm1_step_and_latency():
    S, a = 86016, 200
    s = sch.step_size(S, a)
    assert a * a + 2 * a * s <= S < a * a + 2 * a * (s + 1)
    b = 5000
    t = math.ceil(b / s)
    L = sch.latency_rounds(a, b, S)
    assert L <= t <= L + 1


def test_fit_ranks_fig5_example():
    # Section 7.1, Fig. 5: 65 processors, square matrices: a 4x4x4 grid with
    # one idle processor computes 1.5 % more per processor and communicates
    # 36 % less than the 1x5x13 grid that uses all 65.
    n = 16384
    g, used = sch.fit_ranks(n, n, n, 65, 0.03)
    assert sorted(g) == [4, 4, 4] and used == 64
    g_all, used_all = sch.fit_ranks(n, n, n, 65, 0.0)
    assert sorted(g_all) == [1, 5, 13] and used_all == 65
    comm = sch.grid_surface(n, n, n, g) / sch.grid_surface(n, n, n, g_all) - 1
    assert round(comm * 100) == -36
    assert round((65 / 64 - 1) * 100, 1) == 1.6  # printed as 1.5 %: 1/64 = 1.5625 %


def test_fit_ranks_2198_and_9216_9217():
    n = 16384
    g, used = sch.fit_ranks(n, n, n, 2198, 0.03)
    assert g == (13, 13, 13) and used == 2197
    g1, u1 = sch.fit_ranks(n, n, n, 9216, 0.03)
    g2, u2 = sch.fit_ranks(n, n, n, 9217, 0.03)
    assert (g1, u1) == (g2, u2)


def test_fit_ranks_idle_budget_and_monotone():
    n = 16384
    for p in range(2, 300):
        g, used = sch.fit_ranks(n, n, n, p, 0.03)
        assert g[0] * g[1] * g[2] == used and p - used <= 0.03 * p + 1e-9
        g2, used2 = sch.fit_ranks(n, n, n, p + 1, 0.03)
        if used >= math.ceil(0.97 * (p + 1) - 1e-9):   # p's grid is a candidate for p + 1
            assert sch.grid_surface(n, n, n, g2) <= sch.grid_surface(n, n, n, g) * (1 + 1e-12)


def test_pebble_simulator_listing1_count():
    # X = S schedule of Listing 1 (a x a block, one outer product per round):
    # loads 2mnk/a plus mn stores, with a^2 + 2a red pebbles.
    m, n, k, a = 8, 12, 5, 4
    io = sch.simulate_tiled(m, n, k, a, a, 1, 1, S=a * a + 2 * a)
    assert io == sch.seq_greedy_io(m, n, k, a, a)
    with pytest.raises(sch.PebbleError):
        sch.simulate_tiled(m, n, k, a, a, 1, 1, S=a * a + 2 * a - 1)


def test_pebble_counts_respect_theorem1():
    # Theorem 1 holds for every schedule the simulator can play.
    for (m, n, k) in [(6, 7, 5), (9, 4, 11), (12, 12, 12)]:
        for S in (16, 30, 64):
            for tm in range(1, 9):
                for tn in range(1, 9):
                    for kc in (1, 2, 3):
                        if tm * tn + kc * (tm + tn) > S:
                            continue
                        for pk in (1, 2):
                            io = sch.simulate_tiled(m, n, k, tm, tn, kc, pk, S)
                            assert io >= sch.thm1_bound(m, n, k, S) - 1e-9
