"""FP64 at the full benchmark sizes, in the planner's launch configuration,
checked on 65,536 sampled entries plus the edge tiles (see fullsize_check)."""
import numpy as np
import pytest

import oracle
import synth
import paper_1908_09606_amd as cm
from gpu_util import device_matrix, fullsize_check, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(16384, 16384, 16384), (32768, 32768, 256),
                                   (2048, 2048, 1 << 20)])
def test_fullsize_sampled(gpu, shape):
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
    fullsize_check(C, m, n, k, 1, synth.UNIFORM_F64, plan, oracle.fp64_bound(k))
    assert not torch.isnan(C).any().item()
    del A, B, C
    torch.cuda.empty_cache()
