"""FP64 across the planner's regimes (section 6.2: k is cut while mn / S is
below the processor count, i and j alone are parallelised above it), at
equal work 2 mnk = 2^35, plus large-M and flat shapes, and one shape under
every tile of the menu; each result is checked on sampled entries against
the oracle, and the plan's regime against p1 = mn / S."""
import numpy as np
import pytest

import oracle
import synth
import paper_1908_09606_amd as cm
from gpu_util import device_matrix, log, sampled_check, sample_indices

pytestmark = pytest.mark.gpu

SHAPES = [(256, 256, 1 << 18), (512, 512, 1 << 16), (1024, 1024, 1 << 14), (2048, 2048, 1 << 12),
          (1 << 18, 256, 256), (8192, 8192, 256), (300, 200, 100000)]


def _run_and_check(m, n, k, plan, seed, nsamp=24):
    import torch
    _, A = device_matrix(m, k, seed, synth.STREAM_A, synth.UNIFORM_F64)
    _, B = device_matrix(k, n, seed, synth.STREAM_B, synth.UNIFORM_F64)
    C = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    cm.ensure_workspace(plan.workspace_bytes)
    cm.gemm(A, B, C, dtype="f64", plan=plan)
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed)
    rows = sample_indices(m, nsamp, rng, plan.tile_m)
    cols = sample_indices(n, nsamp, rng, plan.tile_n)
    err = sampled_check(C, m, n, k, seed, synth.UNIFORM_F64, rows=rows, cols=cols,
                        bound=oracle.fp64_bound(k))
    assert not torch.isnan(C).any().item()
    del A, B, C
    torch.cuda.empty_cache()
    return err


@pytest.mark.parametrize("shape", SHAPES)
def test_regime_shapes(gpu, shape):
    m, n, k = shape
    rc, plan = cm.cosma_plan_query(m, n, k, "f64")
    assert rc == 0
    log(f"f64 regime {m}x{n}x{k}: p1 {plan.p1:.1f} regime {plan.regime} tile "
        f"{plan.tile_m}x{plan.tile_n} p_k {plan.p_k} items {plan.items}")
    # the paper's classification: k is cut exactly when mn / S < p
    assert plan.regime == (1 if plan.p1 < 256 else 0)
    # a schedule that would leave most CUs without an ij domain must cut k
    tiles = -(-m // plan.tile_m) * -(-n // plan.tile_n)
    if 4 * tiles <= 256:
        assert plan.p_k > 1
    err = _run_and_check(m, n, k, plan, seed=m % 97 + k % 89)
    log(f"  sampled err={err:.3e} bound={oracle.fp64_bound(k):.3e}")


@pytest.mark.parametrize("tile", range(3))
def test_every_tile_on_one_shape(gpu, tile):
    m, n, k = 1536, 1280, 2304
    rc, plan = cm.cosma_plan_make(m, n, k, "f64", tile, 1)
    assert rc == 0
    log(f"f64 {m}x{n}x{k} tile {plan.tile_m}x{plan.tile_n}")
    err = _run_and_check(m, n, k, plan, seed=7 + tile)
    log(f"  sampled err={err:.3e}")


def _scenarios():
    out = []
    for dtype, S in (("f64", 86016), ("f32", 172032)):
        for name, shape in synth.memory_scenarios(S, 256):
            out.append((dtype, name, shape))
    return out


@pytest.mark.parametrize("case", _scenarios(), ids=lambda c: f"{c[0]}-{c[1].replace(' ', '_')}")
def test_memory_scaling_scenarios(gpu, case):
    """The paper's limited- and extra-memory shapes for p = 256 CUs of S_CU
    words (square, largeK, largeM, flat) and the sizes around the switch of
    eq. optTileShape, FP64 and FP32, under the planner's own plan: the plan
    follows the regime (checked on the host in test_planner.py) and every
    result matches the oracle on 65,536 sampled entries plus the edge tiles."""
    import torch
    from gpu_util import fullsize_check
    dtype, name, (m, n, k) = case
    rc, plan = cm.cosma_plan_query(m, n, k, dtype)
    assert rc == 0
    log(f"{dtype} {name} {m}x{n}x{k}: a {plan.a_par:.0f} (sqrt S {plan.S_words ** 0.5:.0f}) "
        f"p1 {plan.p1:.1f} tile {plan.tile_m}x{plan.tile_n} p_k {plan.p_k}")
    f32 = dtype == "f32"
    dist = synth.UNIFORM_F32 if f32 else synth.UNIFORM_F64
    seed = 60 + m % 31
    _, A = device_matrix(m, k, seed, synth.STREAM_A, dist)
    _, B = device_matrix(k, n, seed, synth.STREAM_B, dist)
    C = torch.full((m, n), float("nan"), dtype=A.dtype, device="cuda")
    cm.gemm(A, B, C, dtype=dtype)
    torch.cuda.synchronize()
    fullsize_check(C, m, n, k, seed, dist, plan,
                   oracle.fp32_bound(k) if f32 else oracle.fp64_bound(k))
    del A, B, C
    torch.cuda.empty_cache()


def test_device_facts_come_from_the_runtime(gpu):
    """The planner's machine model reads the processor count and each CU's
    fast memory (LDS + register file), the per-XCD L2 and the XCD count from
    the runtime; on MI355X they equal the published figures."""
    import torch
    rc, f = cm.cosma_device_query()
    assert rc == 0
    props = torch.cuda.get_device_properties(0)
    assert f.num_cus == props.multi_processor_count
    log(f"device facts: {f.num_cus} CUs, {f.num_xcds} XCDs, LDS {f.lds_bytes_per_cu}, "
        f"VGPR {f.vgpr_bytes_per_cu}, L2/XCD {f.l2_bytes_per_xcd}, {f.clock_ghz} GHz")
    assert (f.num_cus, f.num_xcds) == (256, 8)
    assert f.lds_bytes_per_cu == 160 * 1024 and f.vgpr_bytes_per_cu == 512 * 1024
    assert f.l2_bytes_per_xcd == 4 * 1024 * 1024
    rc, p = cm.cosma_plan_query(4096, 4096, 4096, "f64")
    assert p.S_words == (f.lds_bytes_per_cu + f.vgpr_bytes_per_cu) / 8
