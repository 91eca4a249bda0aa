"""cosma_gemm_ex on the GPU: every layout and transpose combination against
the oracle, exact on integer data, within the bound on uniform data."""
import numpy as np
import pytest

import oracle
import synth
import paper_1908_09606_amd as cm
from gpu_util import log

pytestmark = pytest.mark.gpu

R, Cm, N, T = cm.COSMA_ROW_MAJOR, cm.COSMA_COL_MAJOR, cm.COSMA_NO_TRANS, cm.COSMA_TRANS


def stored(X, layout, trans, pad, torch_dtype):
    """Device buffer holding the matrix op^-1(X) in the given layout, with
    `pad` extra elements per leading dimension; returns (tensor, ld)."""
    import torch
    S = X.T if trans == T else X            # the matrix as stored
    if layout == Cm:
        S = S.T                             # column-major = row-major of the transpose
    rows, cols = S.shape
    buf = torch.full((max(rows, 1), cols + pad), float("nan"), dtype=torch_dtype, device="cuda")
    buf[:rows, :cols] = torch.as_tensor(np.ascontiguousarray(S), dtype=torch_dtype)
    return buf, cols + pad


def run_ex(layout, ta, tb, Ah, Bh, Ch, alpha, beta, dtype, torch_dtype):
    import torch
    m, k = Ah.shape
    n = Bh.shape[1]
    A, lda = stored(Ah, layout, ta, 3, torch_dtype)
    B, ldb = stored(Bh, layout, tb, 1, torch_dtype)
    C, ldc = stored(Ch, layout, N, 2, torch_dtype)
    rc, ws = cm.cosma_workspace_size_ex(layout, ta, tb, m, n, k, dtype)
    assert rc == 0
    cm.ensure_workspace(max(ws, 1))
    rc = cm.cosma_gemm_ex(layout, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype)
    assert rc == 0, cm.cosma_status_string(rc)
    torch.cuda.synchronize()
    out = C.double().cpu().numpy()
    out = out[:n, :m].T if layout == Cm else out[:m, :n]
    return out


COMBOS = [(lay, ta, tb) for lay in (R, Cm) for ta in (N, T) for tb in (N, T)]
SHAPES = [(1, 1, 1), (70, 45, 33), (257, 130, 300), (64, 200, 129)]


@pytest.mark.parametrize("combo", COMBOS)
@pytest.mark.parametrize("dtype", [cm.COSMA_F64, cm.COSMA_F32, cm.COSMA_F64_OZAKI2_I8,
                                   cm.COSMA_F64_OZAKI_BF16])
def test_integer_exact(gpu, combo, dtype):
    import torch
    layout, ta, tb = combo
    tdt = torch.float32 if dtype == cm.COSMA_F32 else torch.float64
    for (m, n, k) in SHAPES:
        Ah = synth.gen(m, k, 11, synth.STREAM_A, synth.INT_F64, 15)
        Bh = synth.gen(k, n, 11, synth.STREAM_B, synth.INT_F64, 15)
        Ch = synth.gen(m, n, 11, synth.STREAM_C, synth.INT_F64, 15)
        got = run_ex(layout, ta, tb, Ah, Bh, Ch, 2.0, -1.0, dtype, tdt)
        exact = 2.0 * (Ah.astype(np.int64) @ Bh.astype(np.int64)) - Ch.astype(np.int64)
        assert np.array_equal(got, exact.astype(np.float64)), (combo, m, n, k)


@pytest.mark.parametrize("combo", COMBOS)
def test_uniform_f64_within_bound(gpu, combo):
    import torch
    layout, ta, tb = combo
    m, n, k = 300, 257, 700
    Ah = synth.gen(m, k, 12, synth.STREAM_A, synth.UNIFORM_F64)
    Bh = synth.gen(k, n, 12, synth.STREAM_B, synth.UNIFORM_F64)
    Ch = synth.gen(m, n, 12, synth.STREAM_C, synth.UNIFORM_F64)
    got = run_ex(layout, ta, tb, Ah, Bh, Ch, 0.5, 2.0, cm.COSMA_F64, torch.float64)
    ref, D = oracle.gemm(Ah, Bh, 0.5, 2.0, Ch)
    err = oracle.normalised_err(got, ref, D)
    log(f"gemm_ex {combo} err={err:.3e}")
    assert err <= oracle.fp64_bound(k)


def test_quick_returns_and_nan_c(gpu):
    """alpha = 0 scales C without reading A or B (NaN operands); beta = 0
    never reads C (NaN C), also with transposed operands."""
    import torch
    m, n, k = 40, 30, 20
    Ah = synth.gen(m, k, 13, synth.STREAM_A, synth.INT_F64, 9)
    Bh = synth.gen(k, n, 13, synth.STREAM_B, synth.INT_F64, 9)
    Ch = synth.gen(m, n, 13, synth.STREAM_C, synth.INT_F64, 9)
    nanA = np.full_like(Ah, np.nan)
    got = run_ex(Cm, T, T, nanA, Bh * np.nan, Ch, 0.0, 3.0, cm.COSMA_F64, torch.float64)
    assert np.array_equal(got, 3.0 * Ch)
    got = run_ex(R, T, N, Ah, Bh, np.full_like(Ch, np.nan), 1.0, 0.0, cm.COSMA_F64, torch.float64)
    assert np.array_equal(got, (Ah.astype(np.int64) @ Bh.astype(np.int64)).astype(np.float64))
