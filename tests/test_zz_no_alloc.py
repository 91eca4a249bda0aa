"""cosma_gemm_noalloc through the C ABI: the schedule's workspace is the
library's static device array, so the call needs no registered workspace
and allocates nothing.  Its results must equal cosma_gemm's (same plan, same
kernels) bit for bit, on two calls in a row where the second is smaller, and
a plan that needs more than the array holds must be refused with nothing
launched."""
import pytest

import synth
import paper_1908_09606_amd as cm
from gpu_util import device_matrix, log

pytestmark = pytest.mark.gpu

# (dtype, first shape, second smaller shape): split-K partials filling the
# whole array, BF16x3 planes, Ozaki digit and residue planes
CASES = [("f64", (256, 256, 65536), (200, 180, 9000)),
         ("f32", (1024, 1024, 1 << 15), (300, 257, 1000)),
         ("bf16x3", (513, 300, 700), (130, 140, 300)),
         ("ozaki", (300, 257, 1000), (100, 90, 500)),
         ("ozaki2", (300, 257, 1000), (100, 90, 500)),
         ("ozaki_bf16", (300, 257, 1000), (100, 90, 500))]


def operands(dtype, m, n, k, seed):
    f32 = dtype in ("f32", "bf16x3")
    dist = synth.UNIFORM_F32 if f32 else synth.UNIFORM_F64
    _, A = device_matrix(m, k, seed, synth.STREAM_A, dist)
    _, B = device_matrix(k, n, seed, synth.STREAM_B, dist)
    _, C0 = device_matrix(m, n, seed, synth.STREAM_C, dist)
    return A, B, C0


def reference(dtype, A, B, C0, alpha, beta):
    """cosma_gemm with a registered workspace."""
    import torch
    m, k = A.shape
    n = B.shape[1]
    rc, ws = cm.cosma_workspace_size(m, n, k, dtype)
    assert rc == 0
    buf = torch.empty(max(ws, 256), dtype=torch.uint8, device="cuda")
    assert cm.cosma_set_workspace(buf, buf.numel()) == 0
    C = C0.clone()
    assert cm.cosma_gemm(m, n, k, alpha, A, k, B, n, beta, C, n, dtype) == 0
    torch.cuda.synchronize()
    assert cm.cosma_set_workspace(None, 0) == 0
    return C


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_cosma_gemm_twice(gpu, case):
    import torch
    dtype, first, second = case
    d = cm.DTYPES[dtype]
    saved = cm._workspace.get(torch.cuda.current_device())
    try:
        for call, (m, n, k) in enumerate((first, second)):
            log(f"noalloc {dtype} call {call} {m}x{n}x{k}")
            rc, plan = cm.cosma_plan_query(m, n, k, d)
            assert rc == 0 and 0 < plan.workspace_bytes <= cm.NOALLOC_SCRATCH_BYTES
            A, B, C0 = operands(dtype, m, n, k, 40 + call)
            alpha, beta = 1.25, -0.5
            want = reference(d, A, B, C0, alpha, beta)
            # no workspace registered: only the static array can serve
            C = C0.clone()
            rc = cm.cosma_gemm_noalloc(m, n, k, alpha, A, k, B, n, beta, C, n, d)
            torch.cuda.synchronize()
            assert rc == 0
            assert torch.equal(C, want), (dtype, call)
    finally:
        if saved is not None:
            assert cm.cosma_set_workspace(saved, saved.numel()) == 0


def test_noalloc_refuses_plans_beyond_the_array(gpu):
    import torch
    m = n = k = 4096
    rc, plan = cm.cosma_plan_query(m, n, k, cm.COSMA_F32_BF16X3)
    assert rc == 0 and plan.workspace_bytes > cm.NOALLOC_SCRATCH_BYTES
    A, B, _ = operands("bf16x3", m, n, k, 50)
    C = torch.full((m, n), float("nan"), dtype=torch.float32, device="cuda")
    rc = cm.cosma_gemm_noalloc(m, n, k, 1.0, A, k, B, n, 0.0, C, n, cm.COSMA_F32_BF16X3)
    torch.cuda.synchronize()
    assert rc == cm.COSMA_ERR_WORKSPACE
    assert torch.isnan(C).all().item()          # nothing was launched
    # argument errors as cosma_gemm
    assert cm.cosma_gemm_noalloc(10, 10, 10, 1.0, A, 5, B, n, 0.0, C, n, 0) == \
        cm.COSMA_ERR_INVALID_ARG
