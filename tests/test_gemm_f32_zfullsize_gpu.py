"""FP32-class paths at the full benchmark sizes (BF16x3 workload), sampled."""
import numpy as np
import pytest

import oracle
import synth
import paper_1908_09606_amd as cm
from gpu_util import device_matrix, log, sampled_check, sample_indices

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f32", "bf16x3"])
@pytest.mark.parametrize("shape,nsamp", [((16384, 16384, 16384), 40), ((4096, 4096, 1 << 18), 16)])
def test_fullsize_sampled(gpu, dtype, shape, nsamp):
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
    rng = np.random.default_rng(m + k)
    rows = sample_indices(m, nsamp, rng, plan.tile_m)
    cols = sample_indices(n, nsamp, rng, plan.tile_n)
    err = sampled_check(C, m, n, k, 1, synth.UNIFORM_F32, rows=rows, cols=cols,
                        bound=oracle.fp32_bound(k))
    log(f"  sampled err={err:.3e} bound={oracle.fp32_bound(k):.3e}")
    assert not torch.isnan(C).any().item()
    del A, B, C
    torch.cuda.empty_cache()
