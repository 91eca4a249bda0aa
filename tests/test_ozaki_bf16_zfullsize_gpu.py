"""Ozaki bf16-slice path at the full benchmark size 8192^3 on the
wide-exponent distribution, sampled rows/columns against the oracle."""
import numpy as np
import pytest

import oracle
import synth
import paper_1908_09606_amd as cm
from gpu_util import device_matrix, fullsize_check, log

pytestmark = pytest.mark.gpu


def test_fullsize_sampled(gpu):
    import torch
    m = n = k = 8192
    log("ozaki_bf16 full size 8192^3 wide exponents")
    _, A = device_matrix(m, k, 1, synth.STREAM_A, synth.WIDE_F64)
    _, B = device_matrix(k, n, 1, synth.STREAM_B, synth.WIDE_F64)
    C = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    cm.gemm(A, B, C, dtype="ozaki_bf16")
    torch.cuda.synchronize()
    rc, plan = cm.cosma_plan_query(m, n, k, "ozaki_bf16")
    err, _ = fullsize_check(C, m, n, k, 1, synth.WIDE_F64, plan, oracle.fp64_bound(k))
    log(f"  slices {plan.slices} sampled err={err:.3e} bound={oracle.fp64_bound(k):.3e}")
    del A, B, C
    torch.cuda.empty_cache()
