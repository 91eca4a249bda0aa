"""FP64 at the full benchmark sizes, in the planner's launch configuration,
checked on sampled entries (random rows/columns plus edge tiles)."""
import numpy as np
import pytest

import oracle
import synth
import paper_1908_09606_amd as cm
from gpu_util import device_matrix, log, sampled_check, sample_indices

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,nsamp", [((16384, 16384, 16384), 48), ((32768, 32768, 256), 64),
                                         ((2048, 2048, 1 << 20), 12)])
def test_fullsize_sampled(gpu, shape, nsamp):
    import torch
    m, n, k = shape
    log(f"f64 full size {m}x{n}x{k}")
    _, A = device_matrix(m, k, 1, synth.STREAM_A, synth.UNIFORM_F64)
    _, B = device_matrix(k, n, 1, synth.STREAM_B, synth.UNIFORM_F64)
    C = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    cm.gemm(A, B, C, dtype="f64")
    torch.cuda.synchronize()
    rc, plan = cm.cosma_plan_query(m, n, k, "f64")
    log(f"  plan tile {plan.tile_m}x{plan.tile_n} p_k {plan.p_k}")
    rng = np.random.default_rng(m + n + k)
    rows = sample_indices(m, nsamp, rng, plan.tile_m)
    cols = sample_indices(n, nsamp, rng, plan.tile_n)
    err = sampled_check(C, m, n, k, 1, synth.UNIFORM_F64, rows=rows, cols=cols,
                        bound=oracle.fp64_bound(k))
    log(f"  sampled err={err:.3e} bound={oracle.fp64_bound(k):.3e}")
    assert not torch.isnan(C).any().item()
    del A, B, C
    torch.cuda.empty_cache()
