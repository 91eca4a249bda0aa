"""CBLAS-style entry point cosma_gemm_ex: argument rules and workspace sizes
on the host (no GPU)."""
import pytest

import paper_1908_09606_amd as cm

R, Cm, N, T = cm.COSMA_ROW_MAJOR, cm.COSMA_COL_MAJOR, cm.COSMA_NO_TRANS, cm.COSMA_TRANS


def ld_min(layout, trans, rows, cols):
    """Smallest legal leading dimension of an operand whose op() is rows x cols."""
    stored_rows, stored_cols = (cols, rows) if trans == T else (rows, cols)
    return max(1, stored_cols if layout == R else stored_rows)


@pytest.mark.parametrize("layout", [R, Cm])
@pytest.mark.parametrize("ta", [N, T])
@pytest.mark.parametrize("tb", [N, T])
def test_leading_dimension_rules(layout, ta, tb):
    m, n, k = 7, 5, 3
    lda, ldb = ld_min(layout, ta, m, k), ld_min(layout, tb, k, n)
    ldc = max(1, n if layout == R else m)
    # one below the minimum is rejected before anything touches a device
    # (stream 0: the default stream, never used here)
    assert cm.cosma_gemm_ex(layout, ta, tb, m, n, k, 1.0, 0, lda - 1, 0, ldb, 0.0, 0, ldc,
                            cm.COSMA_F64, 0) == cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_gemm_ex(layout, ta, tb, m, n, k, 1.0, 0, lda, 0, ldb - 1, 0.0, 0, ldc,
                            cm.COSMA_F64, 0) == cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_gemm_ex(layout, ta, tb, m, n, k, 1.0, 0, lda, 0, ldb, 0.0, 0, ldc - 1,
                            cm.COSMA_F64, 0) == cm.COSMA_ERR_INVALID_ARG


def test_unknown_flags_and_dtype():
    for bad in [(2, N, N), (R, 2, N), (R, N, -1)]:
        assert cm.cosma_gemm_ex(*bad, 4, 4, 4, 1.0, 0, 4, 0, 4, 0.0, 0, 4,
                                cm.COSMA_F64, 0) == cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_gemm_ex(R, N, N, 4, 4, 4, 1.0, 0, 4, 0, 4, 0.0, 0, 4, 9, 0) == \
        cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_gemm_ex(R, N, N, -1, 4, 4, 1.0, 0, 4, 0, 4, 0.0, 0, 4, 0, 0) == \
        cm.COSMA_ERR_INVALID_ARG


@pytest.mark.parametrize("dtype", [cm.COSMA_F64, cm.COSMA_F32, cm.COSMA_F32_BF16X3,
                                   cm.COSMA_F64_OZAKI_I8, cm.COSMA_F64_OZAKI2_I8,
                                   cm.COSMA_F64_OZAKI_BF16])
def test_workspace_sizes(dtype):
    m, n, k = 300, 200, 1000
    w = 8 if dtype in (cm.COSMA_F64, cm.COSMA_F64_OZAKI_I8, cm.COSMA_F64_OZAKI2_I8,
                       cm.COSMA_F64_OZAKI_BF16) else 4
    up = lambda x: (x + 255) // 256 * 256
    rc, base = cm.cosma_workspace_size(m, n, k, dtype)
    assert rc == 0
    # no transposes: the plan's own workspace
    assert cm.cosma_workspace_size_ex(R, N, N, m, n, k, dtype) == (0, base)
    # transposed A (m x k copy) and / or B (k x n copy) after the plan's part
    assert cm.cosma_workspace_size_ex(R, T, N, m, n, k, dtype) == (0, up(base) + up(m * k * w))
    assert cm.cosma_workspace_size_ex(R, N, T, m, n, k, dtype) == (0, up(base) + up(k * n * w))
    assert cm.cosma_workspace_size_ex(R, T, T, m, n, k, dtype) == \
        (0, up(base) + up(m * k * w) + up(k * n * w))
    # column-major runs the swapped row-major product (n x m) with the flags swapped
    rc, base_t = cm.cosma_workspace_size(n, m, k, dtype)
    assert cm.cosma_workspace_size_ex(Cm, N, N, m, n, k, dtype) == (0, base_t)
    assert cm.cosma_workspace_size_ex(Cm, T, N, m, n, k, dtype) == (0, up(base_t) + up(k * m * w))
    assert cm.cosma_workspace_size_ex(Cm, N, T, m, n, k, dtype) == (0, up(base_t) + up(n * k * w))
