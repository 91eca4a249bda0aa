"""FP32-class paths at the full benchmark sizes (BF16x3 workload), sampled."""
import numpy as np
import pytest

import oracle
import synth
import paper_1908_09606_amd as cm
from gpu_util import device_matrix, fullsize_check, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f32", "bf16x3"])
@pytest.mark.parametrize("shape", [(16384, 16384, 16384), (4096, 4096, 1 << 18)])
def test_fullsize_sampled(gpu, dtype, shape):
    import torch
    m, n, k = shape
    log(f"{dtype} full size {m}x{n}x{k}")
    _, A = device_matrix(m, k, 1, synth.STREAM_A, synth.UNIFORM_F32)
    _, B = device_matrix(k, n, 1, synth.STREAM_B, synth.UNIFORM_F32)
    C = torch.full((m, n), float("nan"), dtype=torch.float32, device="cuda")
    cm.gemm(A, B, C, dtype=dtype)
    torch.cuda.synchronize()
    rc, plan = cm.cosma_plan_query(m, n, k, dtype)
    log(f"  plan tile {plan.tile_m}x{plan.tile_n} p_k {plan.p_k}")
    fullsize_check(C, m, n, k, 1, synth.UNIFORM_F32, plan, oracle.fp32_bound(k))
    assert not torch.isnan(C).any().item()
    del A, B, C
    torch.cuda.empty_cache()
