"""The product planner (host logic behind the C ABI) against the oracle's
I/O model, the pebble simulator and the paper's numbers.  CPU only."""
import math
import os
import re

import pytest

import paper_1908_09606_amd as cm
from oracle import schedule as sch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "cosma_mi355.h")) as f:
        names = set(re.findall(r"COSMA_API\s+[\w\s\*]+?\b(cosma_\w+)\s*\(", f.read()))
    assert len(names) >= 20
    L = cm.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(cm.EXPORTED) == names
    assert "gfx950" in cm.cosma_version()


def test_status_strings():
    for st in (0, -1, -2, -3, -4, -5):
        assert cm.cosma_status_string(st).startswith("COSMA_")


def test_thm1_and_seq_schedule_match_oracle():
    for S in (3, 16, 64, 20480, 86016, 172032, 10 ** 6):
        rc, a, b = cm.cosma_seq_schedule(S)
        assert rc == 0
        oa, ob, _ = sch.seq_tile_search(S)
        assert (a, b) == (oa, ob)
    assert cm.cosma_thm1_bound(100, 200, 300, 86016) == pytest.approx(
        sch.thm1_bound(100, 200, 300, 86016), rel=1e-15)
    rc, a, b = cm.cosma_par_schedule(16384, 16384, 16384, 256, 86016)
    oa, ob = sch.opt_tile_shape(16384, 16384, 16384, 256, 86016)
    assert rc == 0 and a == pytest.approx(oa) and b == pytest.approx(ob)


def test_fit_ranks_paper_examples():
    n = 16384
    rc, g, used = cm.cosma_fit_ranks(n, n, n, 65, 0.03)
    assert rc == 0 and sorted(g) == [4, 4, 4] and used == 64
    rc, g, used = cm.cosma_fit_ranks(n, n, n, 2198, 0.03)
    assert g == (13, 13, 13) and used == 2197
    r1 = cm.cosma_fit_ranks(n, n, n, 9216, 0.03)
    r2 = cm.cosma_fit_ranks(n, n, n, 9217, 0.03)
    assert r1 == r2
    for p in (7, 64, 100, 255, 256, 1000):
        for shape in ((n, n, n), (2048, 2048, 1 << 20), (32768, 32768, 256)):
            rc, g, used = cm.cosma_fit_ranks(*shape, p, 0.03)
            og, oused = sch.fit_ranks(*shape, p, 0.03)
            assert (g, used) == (og, oused)


def test_io_count_equals_pebble_simulator():
    for (m, n, k) in [(5, 7, 9), (8, 8, 8), (13, 6, 11), (1, 9, 4)]:
        for tm, tn, kc in [(1, 1, 1), (2, 3, 2), (4, 4, 3), (3, 5, 1)]:
            for pk in (1, 2, 3):
                for beta in (False, True):
                    S = max(tm * tn + kc * (tm + tn), pk) + (1 if beta else 0)
                    io = sch.simulate_tiled(m, n, k, tm, tn, kc, pk, S, beta)
                    assert cm.cosma_io_count(m, n, k, tm, tn, kc, pk, beta) == io


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16x3", "ozaki", "ozaki_bf16"])
@pytest.mark.parametrize("shape", [(512, 512, 512), (16384, 16384, 16384), (2048, 2048, 1 << 20),
                                   (32768, 32768, 256), (4096, 4096, 1 << 18), (8192, 8192, 8192),
                                   (1, 1, 1), (65, 3, 1000), (3000, 17, 5)])
def test_every_plan_respects_theorem1_and_is_consistent(dtype, shape):
    m, n, k = shape
    rc, p = cm.cosma_plan_query(m, n, k, dtype)
    assert rc == 0
    assert p.tile_m > 0 and p.tile_n > 0 and p.tile_k > 0
    assert p.p_m == math.ceil(m / p.tile_m) and p.p_n == math.ceil(n / p.tile_n)
    assert p.p_k >= 1 and p.k_split % p.tile_k == 0 and math.ceil(k / p.k_split) == p.p_k
    assert p.items == p.p_m * p.p_n * p.p_k
    # counted I/O sits on or above Theorem 1's bound for the CU's fast memory
    assert p.q_cu_words >= p.thm1_words * (1 - 1e-12)
    assert p.q_cu_words == cm.cosma_io_count(m, n, k, p.tile_m, p.tile_n, p.tile_k, p.p_k, False)
    assert p.regime == (1 if 256 > m * n / p.S_words else 0)
    # predicted memory traffic covers at least the compulsory traffic
    w = 8 if dtype in ("f64", "ozaki", "ozaki_bf16") else 4
    assert p.q_ea_bytes >= (m * k + k * n + m * n) * w * (1 - 1e-12) or dtype.startswith("ozaki")
    rc, ws = cm.cosma_workspace_size(m, n, k, dtype)
    assert rc == 0 and ws == p.workspace_bytes
    if p.p_k > 1:
        assert ws >= p.p_k * m * n * (8 if dtype in ("f64", "ozaki", "ozaki_bf16") else 4)


def test_planner_regimes_on_paper_shapes():
    # square and flat: p <= p1, no split; large-k: p > p1, k is cut
    rc, sq = cm.cosma_plan_query(16384, 16384, 16384, "f64")
    assert sq.regime == 0 and sq.p_k == 1
    rc, fl = cm.cosma_plan_query(32768, 32768, 256, "f64")
    assert fl.regime == 0 and fl.p_k == 1
    rc, lk = cm.cosma_plan_query(2048, 2048, 1 << 20, "f64")
    assert lk.regime == 1 and lk.p_k > 1
    # the S of one CU: (LDS + VGPR bytes) / 8 for FP64
    assert sq.S_words == (160 * 1024 + 512 * 1024) / 8
    rc, a, b = cm.cosma_seq_schedule(int(sq.S_words))
    assert (sq.a_seq, sq.b_seq) == (a, b)


def test_plan_make_forced_and_invalid():
    rc, p = cm.cosma_plan_make(1000, 1000, 4096, "f64", 0, 4)
    assert rc == 0 and p.p_k == 4 and p.tile_id == 0
    assert cm.cosma_plan_make(1000, 1000, 4096, "f64", 99, 1)[0] == cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_plan_make(1000, 1000, 16, "f64", 0, 4)[0] == cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_plan_query(-1, 4, 4, "f64")[0] == cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_plan_query(4, 4, 4, 7)[0] == cm.COSMA_ERR_INVALID_ARG


def test_degenerate_devices_still_plan():
    f = cm.cosma_device_facts(num_cus=1, num_xcds=1, lds_bytes_per_cu=1024,
                              vgpr_bytes_per_cu=1024, l2_bytes_per_xcd=1 << 16,
                              clock_ghz=1.0, hbm_gbps=100.0)
    for shape in ((1, 1, 1), (100, 100, 100), (4096, 64, 70000)):
        rc, p = cm.cosma_plan_query_facts(*shape, "f64", f, 0.03)
        assert rc == 0 and p.items == p.p_m * p.p_n * p.p_k
        assert p.waves == math.ceil(p.items / p.wg_per_cu)
    bad = cm.cosma_device_facts(num_cus=0, num_xcds=1, lds_bytes_per_cu=1, vgpr_bytes_per_cu=1,
                                l2_bytes_per_xcd=1, clock_ghz=1.0, hbm_gbps=1.0)
    assert cm.cosma_plan_query_facts(8, 8, 8, "f64", bad, 0.03)[0] == cm.COSMA_ERR_INVALID_ARG


def test_gpu_entry_points_reject_bad_arguments_without_launching():
    # Argument errors are detected before any device work, so these run on a
    # machine without a GPU too.
    assert cm.cosma_gemm(-1, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4, 0, 0) == cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_gemm(4, 4, 4, 1.0, 8, 3, 8, 4, 0.0, 8, 4, 0, 0) == cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_gemm(4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, None, 4, 0, 0) == cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_gemm(4, 4, 4, 1.0, None, 4, 8, 4, 0.0, 8, 4, 0, 0) == cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_gemm(4, 4, 4, 1.0, 8, 4, 8, 4, 0.0, 8, 4, 9, 0) == cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_gemm(4, 4, 4, 1.0, 12, 4, 8, 4, 0.0, 8, 4, 0, 0) == cm.COSMA_ERR_INVALID_ARG  # misaligned
    assert cm.cosma_gemm(0, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 0, 0) == cm.COSMA_OK


def test_raster_groups_respect_conflicting_pitch():
    """A row pitch that is a multiple of 4 KiB puts the A-panel lines of one k
    offset into the same L2 sets: the planner keeps at most 512 A rows per
    raster group then; other pitches may use taller groups."""
    for dtype in ("f64", "f32", "bf16x3"):
        rc, p = cm.cosma_plan_query(16384, 16384, 16384, dtype)   # pitch 2^16 or 2^17 bytes
        assert rc == 0 and (p.group_m == 1 or p.group_m * p.tile_m <= 512)
    rc, p = cm.cosma_plan_query(16000, 16000, 16000, "f64")        # pitch 128000 bytes
    assert rc == 0 and p.group_m * p.tile_m > 512


def test_ozaki_bf16_plan_and_workspace():
    """bf16 digit path: one 128 x 64 tile with 32-k rounds, slices chosen by
    the error contract (tests/test_ozaki_contract.py), 1..8 accepted;
    workspace = split partials, then 2 s bytes per padded element of each
    operand's planes, then the exponents."""
    up = lambda x: (x + 255) // 256 * 256
    for (m, n, k, pk) in [(300, 200, 1000, 1), (129, 65, 33, 1), (200, 190, 3000, 3),
                          (8192, 8192, 8192, 1)]:
        rc, p = cm.cosma_plan_make(m, n, k, "ozaki_bf16", 0, pk)
        assert rc == 0
        assert (p.tile_m, p.tile_n, p.tile_k) == (128, 64, 32) and 1 <= p.slices <= 8
        s = p.slices
        kp = -(-k // 32) * 32
        rows, cols = -(-m // 128) * 128, -(-n // 64) * 64
        part = up(pk * m * n * 8) if pk > 1 else 0
        assert p.workspace_bytes == part + up(2 * s * kp * (rows + cols)) + up((m + n) * 4)
        assert cm.cosma_plan_set_slices(p, 8) == 0
        assert p.workspace_bytes == part + up(2 * 8 * kp * (rows + cols)) + up((m + n) * 4)
        assert cm.cosma_plan_set_slices(p, 0) == cm.COSMA_ERR_INVALID_ARG
        assert cm.cosma_plan_set_slices(p, 9) == cm.COSMA_ERR_INVALID_ARG
    # a work item's reduction length is not limited (binary64 accumulation
    # after every round): the square product runs without a split
    rc, p = cm.cosma_plan_query(2048, 2048, 1 << 20, "ozaki_bf16")
    assert rc == 0 and p.k_split > 65536
    # the modelled rate is the bf16 rate over s(s+1)/2 products
    rc, q = cm.cosma_plan_query(8192, 8192, 8192, "ozaki")
    rc, b = cm.cosma_plan_query(8192, 8192, 8192, "ozaki_bf16")
    assert b.predicted_ms > q.predicted_ms


def test_f32_menu_and_wide_tile_choice():
    """The FP32 menu's fourth tile is 256 x 256 (32x32x2 instructions); the
    planner takes it for large squares and long reductions, and keeps the
    smaller tiles where 256 x 256 blocks would leave CUs idle."""
    assert cm.cosma_tile_count("f32") == 4
    assert cm.cosma_tile_shape("f32", 3) == (0, (256, 256, 32))
    for shape in [(16384, 16384, 16384), (8192, 8192, 8192), (4096, 4096, 1 << 18)]:
        rc, p = cm.cosma_plan_query(*shape, "f32")
        assert rc == 0 and (p.tile_m, p.tile_n) == (256, 256), shape
    for shape in [(1000, 1000, 1000), (4097, 4095, 4093), (300, 257, 1000)]:
        rc, p = cm.cosma_plan_query(*shape, "f32")
        assert rc == 0 and (p.tile_m, p.tile_n) != (256, 256), shape


def test_plan_cache_under_concurrent_queries():
    """The plan cache is shared and mutex-guarded: eight threads querying
    overlapping and distinct shapes (enough distinct ones to force the
    cache's clearing) get exactly the plans a serial pass produces."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    rng = np.random.default_rng(11)
    # more distinct (shape, dtype) keys than the cache's 4096 entries
    shapes = [tuple(int(x) for x in rng.integers(1, 3000, size=3)) for _ in range(4200)]
    shapes += [(16384, 16384, 16384), (2048, 2048, 1 << 20), (300, 257, 1000)] * 50
    dtypes = ["f64", "f32", "bf16x3", "ozaki2"]
    fields = [f for f, _ in cm.cosma_plan_info._fields_]

    def plan(i):
        rc, p = cm.cosma_plan_query(*shapes[i], dtypes[i % len(dtypes)])
        assert rc == 0
        return tuple(getattr(p, f) for f in fields)

    serial = [plan(i) for i in range(len(shapes))]
    order = list(range(len(shapes))) * 2
    rng.shuffle(order)
    with ThreadPoolExecutor(max_workers=8) as ex:
        got = list(ex.map(plan, order))
    for i, g in zip(order, got):
        assert g == serial[i], shapes[i]


def test_memory_scaling_scenarios_follow_the_regime():
    """The paper's limited / extra-memory shapes (section 8) for p = 256 CUs
    of S_CU words: the recipe meets its definition (p S / I = 1 and
    p^(2/3) S / I = 1, I = mn + mk + nk); eq. optTileShape's a is sqrt(S) on
    the limited-memory squares and (mnk / p)^(1/3) < sqrt(S) on the
    extra-memory ones and below the switch; every shape has mn / S < p, so
    the plans sit in the k-cut regime of section 6.2, and the shapes whose
    unsplit tiles would fill under a quarter of the machine cut k (the flat
    rank-256 updates keep k whole: rounds stay at least 256 long)."""
    import math
    import synth
    for dtype, S in (("f64", 86016.0), ("f32", 172032.0)):
        scen = dict(synth.memory_scenarios(S, 256))
        for name, (m, n, k) in scen.items():
            I = m * n + m * k + n * k
            if "limited" in name:
                assert abs(I / (256 * S) - 1) < 0.02, (name, I)
            elif "extra" in name:
                assert abs(I / (256 ** (2 / 3) * S) - 1) < 0.02, (name, I)
            rc, p = cm.cosma_plan_query(m, n, k, dtype)
            assert rc == 0 and p.S_words == S
            cube = (m * n * k / 256) ** (1 / 3)
            assert p.a_par == pytest.approx(min(math.sqrt(S), cube), rel=1e-12)
            assert p.regime == 1 and p.p1 < 256
            assert p.q_cu_words >= p.thm1_words * (1 - 1e-12)
            tiles = -(-m // p.tile_m) * -(-n // p.tile_n)
            if k >= 2048 and 4 * tiles <= 256 * p.wg_per_cu:
                assert p.p_k > 1, (dtype, name, p.p_k)
            if name.startswith("flat"):
                assert p.p_k == 1
        assert scen["square limited"][0] > 0
        rc, p = cm.cosma_plan_query(*scen["square limited"], dtype)
        assert p.a_par == pytest.approx(math.sqrt(S))
        for nm in ("square extra", "optTileShape switch x0.75"):
            rc, p = cm.cosma_plan_query(*scen[nm], dtype)
            assert p.a_par < math.sqrt(S) * 0.9, nm
