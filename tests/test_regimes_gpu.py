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
