"""cosma_gemm under HIP graph capture: the single-product path launches only
kernels on the caller's stream (no allocation, no memset), so it can be
recorded into a graph.  Each dtype's multi-kernel sequence (split pass,
exponent / residue prologues, split-K reduction, reconstruction) is captured
once and replayed several times, with eager work on the same buffers between
the replays; every replay must equal the eager result bit for bit."""
import pytest

import synth
import paper_1908_09606_amd as cm
from gpu_util import device_matrix, log

pytestmark = pytest.mark.gpu

CASES = [("f64", (300, 257, 1000), 1), ("f64", (256, 128, 5000), 3), ("f32", (300, 257, 1000), 2),
         ("f32", (600, 520, 900), 2, 3),
         ("bf16x3", (513, 300, 700), 1), ("ozaki", (300, 257, 1000), 1),
         ("ozaki2", (513, 300, 700), 1), ("ozaki2", (130, 140, 70000), 2),
         ("ozaki_bf16", (300, 257, 1000), 1), ("ozaki_bf16", (130, 140, 5000), 2)]


@pytest.mark.parametrize("case", CASES)
def test_replays_equal_eager(gpu, case):
    import torch
    dtype, (m, n, k), p_k = case[:3]
    tile = case[3] if len(case) > 3 else 0
    f32 = dtype in ("f32", "bf16x3")
    dist = synth.UNIFORM_F32 if f32 else synth.UNIFORM_F64
    tdt = torch.float32 if f32 else torch.float64
    log(f"graph capture {dtype} {m}x{n}x{k} p_k={p_k}")
    _, A = device_matrix(m, k, 21, synth.STREAM_A, dist)
    _, B = device_matrix(k, n, 21, synth.STREAM_B, dist)
    _, C0 = device_matrix(m, n, 21, synth.STREAM_C, dist)
    rc, plan = cm.cosma_plan_make(m, n, k, dtype, tile, p_k)
    assert rc == 0 and plan.p_k == p_k
    cm.ensure_workspace(plan.workspace_bytes)   # before capture: no allocation inside
    alpha, beta = 1.25, -0.5
    C = C0.clone()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        cm.gemm(A, B, C, alpha=alpha, beta=beta, dtype=dtype, plan=plan, stream=stream)
    stream.synchronize()
    eager = C.clone()

    Cg = C0.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        cm.gemm(A, B, Cg, alpha=alpha, beta=beta, dtype=dtype, plan=plan, stream=stream)
    for r in range(3):
        Cg.copy_(C0)                            # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(Cg, eager), (dtype, r)
        # eager launches on the same workspace between replays
        scratch = C0.clone()
        cm.gemm(A, B, scratch, alpha=alpha, beta=beta, dtype=dtype, plan=plan)
        torch.cuda.synchronize()
        assert torch.equal(scratch, eager)
    assert A.dtype == tdt
    del graph
