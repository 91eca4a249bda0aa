"""FP64 path on the GPU against the oracle (element by element)."""
import numpy as np
import pytest

import oracle
import synth
import paper_1908_09606_amd as cm
from gpu_util import device_matrix, log, sampled_check, sample_indices

pytestmark = pytest.mark.gpu

F64 = cm.COSMA_F64


def run(m, n, k, A, lda, B, ldb, C, ldc, alpha=1.0, beta=0.0, plan=None, dtype=F64):
    import torch
    if plan is None:
        rc, ws = cm.cosma_workspace_size(m, n, k, dtype)
        assert rc == 0
    else:
        ws = plan.workspace_bytes
    if ws:
        cm.ensure_workspace(ws)
    if plan is None:
        rc = cm.cosma_gemm(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype)
    else:
        rc = cm.cosma_gemm_planned(plan, alpha, A, lda, B, ldb, beta, C, ldc)
    torch.cuda.synchronize()
    return rc


def test_device_fill_matches_host_generator(gpu):
    for dist, param in [(synth.UNIFORM_F64, 0), (synth.UNIFORM_F32, 0), (synth.WIDE_F64, 0),
                        (synth.INT_F64, 8), (synth.INT_F32, 100)]:
        buf, v = device_matrix(37, 53, 11, synth.STREAM_B, dist, param, ld=60)
        host = synth.gen(37, 53, 11, synth.STREAM_B, dist, param)
        assert np.array_equal(v.cpu().numpy(), host), dist


def test_config_512_cube_full_oracle(gpu):
    m = n = k = 512
    log("f64 512^3 seed 0")
    _, A = device_matrix(m, k, 0, synth.STREAM_A, synth.UNIFORM_F64)
    _, B = device_matrix(k, n, 0, synth.STREAM_B, synth.UNIFORM_F64)
    _, C = device_matrix(m, n, 0, synth.STREAM_C, synth.UNIFORM_F64)
    C.fill_(float("nan"))
    assert run(m, n, k, A, k, B, n, C, n) == 0
    Ah = synth.gen(m, k, 0, synth.STREAM_A, synth.UNIFORM_F64)
    Bh = synth.gen(k, n, 0, synth.STREAM_B, synth.UNIFORM_F64)
    ref, D = oracle.gemm(Ah, Bh)
    err = oracle.normalised_err(C.cpu().numpy(), ref, D)
    log(f"  err={err:.3e} bound={oracle.fp64_bound(k):.3e}")
    assert err <= oracle.fp64_bound(k)


SHAPES = [(1, 1, 1), (1, 7, 3), (17, 33, 5), (64, 64, 16), (65, 63, 17), (130, 129, 131),
          (257, 300, 97), (300, 257, 1000), (129, 1, 64), (1, 300, 45)]


@pytest.mark.parametrize("tile", range(3))
def test_integer_exact_all_tiles_ragged(gpu, tile):
    """Integer entries in [-8, 8]: every partial sum is an exact integer, so
    the result must equal the exact product bit for bit, for every tile and
    every ragged shape."""
    for (m, n, k) in SHAPES:
        log(f"f64 int tile {tile} {m}x{n}x{k}")
        lda, ldb, ldc = k + 3, n + 1, n + 2
        _, A = device_matrix(m, k, 5, synth.STREAM_A, synth.INT_F64, 8, ld=lda)
        _, B = device_matrix(k, n, 5, synth.STREAM_B, synth.INT_F64, 8, ld=ldb)
        _, C = device_matrix(m, n, 5, synth.STREAM_C, synth.INT_F64, 8, ld=ldc)
        rc, plan = cm.cosma_plan_make(m, n, k, F64, tile, 1)
        assert rc == 0
        assert run(m, n, k, A, lda, B, ldb, C, ldc, plan=plan) == 0
        Ah = synth.gen(m, k, 5, synth.STREAM_A, synth.INT_F64, 8).astype(np.int64)
        Bh = synth.gen(k, n, 5, synth.STREAM_B, synth.INT_F64, 8).astype(np.int64)
        assert np.array_equal(C.cpu().numpy(), (Ah @ Bh).astype(np.float64)), (m, n, k)


def test_split_k_bit_identical_on_integers(gpu):
    m, n, k = 300, 200, 3000
    Ah = synth.gen(m, k, 9, synth.STREAM_A, synth.INT_F64, 8).astype(np.int64)
    Bh = synth.gen(k, n, 9, synth.STREAM_B, synth.INT_F64, 8).astype(np.int64)
    exact = (Ah @ Bh).astype(np.float64)
    _, A = device_matrix(m, k, 9, synth.STREAM_A, synth.INT_F64, 8)
    _, B = device_matrix(k, n, 9, synth.STREAM_B, synth.INT_F64, 8)
    for tile in range(3):
        for pk in (1, 2, 3, 5, 8):
            log(f"f64 split-k tile {tile} pk {pk}")
            _, C = device_matrix(m, n, 1, synth.STREAM_C, synth.UNIFORM_F64)
            rc, plan = cm.cosma_plan_make(m, n, k, F64, tile, pk)
            assert rc == 0 and plan.p_k == pk
            assert run(m, n, k, A, k, B, n, C, n, plan=plan) == 0
            assert np.array_equal(C.cpu().numpy(), exact), (tile, pk)


@pytest.mark.parametrize("pk", [1, 4])
def test_alpha_beta_random_within_bound(gpu, pk):
    m, n, k = 250, 190, 700
    log(f"f64 alpha/beta pk {pk}")
    _, A = device_matrix(m, k, 3, synth.STREAM_A, synth.UNIFORM_F64)
    _, B = device_matrix(k, n, 3, synth.STREAM_B, synth.UNIFORM_F64)
    _, C = device_matrix(m, n, 3, synth.STREAM_C, synth.UNIFORM_F64)
    C0 = synth.gen(m, n, 3, synth.STREAM_C, synth.UNIFORM_F64)
    alpha, beta = -1.25, 0.6
    rc, plan = cm.cosma_plan_make(m, n, k, F64, 0, pk)
    assert run(m, n, k, A, k, B, n, C, n, alpha, beta, plan=plan) == 0
    ref, D = oracle.gemm(synth.gen(m, k, 3, synth.STREAM_A, synth.UNIFORM_F64),
                         synth.gen(k, n, 3, synth.STREAM_B, synth.UNIFORM_F64), alpha, beta, C0)
    err = oracle.normalised_err(C.cpu().numpy(), ref, D)
    assert err <= oracle.fp64_bound(k), err


def test_blas_quick_returns(gpu):
    import torch
    m, n, k = 70, 90, 33
    _, A = device_matrix(m, k, 4, synth.STREAM_A, synth.UNIFORM_F64)
    _, B = device_matrix(k, n, 4, synth.STREAM_B, synth.UNIFORM_F64)
    _, C = device_matrix(m, n, 4, synth.STREAM_C, synth.UNIFORM_F64)
    C0 = C.clone()
    # alpha == 0: A and B not read (NaN operands), C = beta*C
    An = A.clone().fill_(float("nan"))
    assert run(m, n, k, An, k, B, n, C, n, 0.0, 0.5) == 0
    assert torch.equal(C, 0.5 * C0)
    # k == 0: C = beta * C
    C.copy_(C0)
    assert run(m, n, 0, A, 1, B, n, C, n, 1.0, -2.0) == 0
    assert torch.equal(C, -2.0 * C0)
    # beta == 0 with NaN C and alpha == 0: exact zeros
    C.fill_(float("nan"))
    assert run(m, n, k, A, k, B, n, C, n, 0.0, 0.0) == 0
    assert torch.count_nonzero(C).item() == 0
    # m == 0 and n == 0: nothing is touched
    C.copy_(C0)
    assert run(0, n, k, A, k, B, n, C, n) == 0 and run(m, 0, k, A, k, B, 1, C, 1) == 0
    assert torch.equal(C, C0)


def test_identity_and_rank1_closed_forms(gpu):
    import torch
    m = 200
    _, B = device_matrix(m, 150, 6, synth.STREAM_B, synth.UNIFORM_F64)
    I = torch.eye(m, dtype=torch.float64, device="cuda")
    C = torch.empty((m, 150), dtype=torch.float64, device="cuda")
    assert run(m, 150, m, I, m, B, 150, C, 150) == 0
    assert torch.equal(C, B)
    x = torch.arange(-50, 50, dtype=torch.float64, device="cuda")[:, None].repeat(1, 333)
    y = torch.arange(-30, 40, dtype=torch.float64, device="cuda")[None, :].repeat(333, 1)
    C = torch.empty((100, 70), dtype=torch.float64, device="cuda")
    assert run(100, 70, 333, x.contiguous(), 333, y.contiguous(), 70, C, 70) == 0
    want = 333.0 * torch.outer(torch.arange(-50, 50, dtype=torch.float64),
                                torch.arange(-30, 40, dtype=torch.float64))
    assert torch.equal(C.cpu(), want)


def test_errors_do_not_launch(gpu):
    import torch
    _, A = device_matrix(8, 8, 1, synth.STREAM_A, synth.UNIFORM_F64)
    _, C = device_matrix(8, 8, 1, synth.STREAM_C, synth.UNIFORM_F64)
    C0 = C.clone()
    assert run(8, 8, 8, A, 7, A, 8, C, 8) == cm.COSMA_ERR_INVALID_ARG
    assert run(8, 8, 8, A, 8, A, 8, C, 7) == cm.COSMA_ERR_INVALID_ARG
    assert torch.equal(C, C0)
    # a split plan with no registered workspace fails cleanly
    rc, plan = cm.cosma_plan_make(300, 300, 4096, F64, 0, 4)
    assert cm.cosma_set_workspace(None, 0) == 0
    cm._workspace.clear()
    _, A2 = device_matrix(300, 4096, 1, synth.STREAM_A, synth.UNIFORM_F64)
    _, B2 = device_matrix(4096, 300, 1, synth.STREAM_B, synth.UNIFORM_F64)
    _, C2 = device_matrix(300, 300, 1, synth.STREAM_C, synth.UNIFORM_F64)
    C20 = C2.clone()
    rc = cm.cosma_gemm_planned(plan, 1.0, A2, 4096, B2, 300, 0.0, C2, 300)
    torch.cuda.synchronize()
    assert rc == cm.COSMA_ERR_WORKSPACE and torch.equal(C2, C20)
    # a caller-edited plan cannot shrink the workspace requirement
    plan.workspace_bytes = 0
    assert cm.cosma_gemm_planned(plan, 1.0, A2, 4096, B2, 300, 0.0, C2, 300) == cm.COSMA_ERR_WORKSPACE
    # inconsistent plans are rejected
    plan.p_k = 3
    assert cm.cosma_gemm_planned(plan, 1.0, A2, 4096, B2, 300, 0.0, C2, 300) == cm.COSMA_ERR_INVALID_ARG


# Full tiles with 16-byte aligned rows and whole 16-k rounds run the
# DMA-staged kernel form (tiles 0 and 2); a product one row taller runs the
# register-staged form on every tile.  Both take each entry's k sum in the
# same order, so the shared rows must agree bit for bit, and the aligned
# product must meet the oracle's bound.
@pytest.mark.parametrize("tile,pk", [(0, 1), (0, 3), (2, 1), (2, 2)])
def test_dma_form_bit_equal_to_register_form(gpu, tile, pk):
    import torch
    rc, (bm, bn, _) = cm.cosma_tile_shape(F64, tile)
    assert rc == 0
    m, n, k = 2 * bm, 2 * bn, 16 * 37
    log(f"f64 dma vs register form tile {tile} p_k {pk} {m}x{n}x{k}")
    _, Ap = device_matrix(m + 1, k, 7, synth.STREAM_A, synth.UNIFORM_F64)
    _, B = device_matrix(k, n, 7, synth.STREAM_B, synth.UNIFORM_F64)
    C1 = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    C2 = torch.full((m + 1, n), float("nan"), dtype=torch.float64, device="cuda")
    rc, plan = cm.cosma_plan_make(m, n, k, F64, tile, pk)
    assert rc == 0 and plan.p_k == pk
    assert run(m, n, k, Ap, k, B, n, C1, n, alpha=0.75, plan=plan) == 0
    rc, plan2 = cm.cosma_plan_make(m + 1, n, k, F64, tile, pk)
    assert rc == 0 and plan2.k_split == plan.k_split
    assert run(m + 1, n, k, Ap, k, B, n, C2, n, alpha=0.75, plan=plan2) == 0
    assert torch.equal(C1, C2[:m]), "DMA and register forms differ"
    Ah = synth.gen(m + 1, k, 7, synth.STREAM_A, synth.UNIFORM_F64)[:m]
    Bh = synth.gen(k, n, 7, synth.STREAM_B, synth.UNIFORM_F64)
    ref, D = oracle.gemm(Ah, Bh, alpha=0.75)
    err = oracle.normalised_err(C1.cpu().numpy(), ref, D)
    log(f"  err={err:.3e} bound={oracle.fp64_bound(k):.3e}")
    assert err <= oracle.fp64_bound(k)
