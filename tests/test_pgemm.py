"""ScaLAPACK-style entry point cosma_pgemm: descriptor and submatrix rules on
the host (no GPU; every call here is rejected before anything touches a
device, stream 0 is never used)."""
import pytest

import paper_1908_09606_amd as cm

N, T = cm.COSMA_NO_TRANS, cm.COSMA_TRANS
F64 = cm.COSMA_F64


def call(desca, descb, descc, ia=1, ja=1, ib=1, jb=1, ic=1, jc=1, m=4, n=3, k=2, ta=N, tb=N,
         dtype=F64):
    return cm.cosma_pgemm(ta, tb, m, n, k, 1.0, 0, ia, ja, desca, 0, ib, jb, descb, 0.0, 0, ic, jc,
                          descc, dtype, 0)


def good():
    # A 10 x 8, B 8 x 9, C 10 x 9, column-major, padded leading dimensions
    return cm.descinit(10, 8, 4, 4, 12), cm.descinit(8, 9, 2, 3, 8), cm.descinit(10, 9, 5, 5, 11)


def test_descinit_fields():
    assert cm.descinit(7, 5, 2, 3, 9) == [1, 0, 7, 5, 2, 3, 0, 0, 9]


@pytest.mark.parametrize("which", [0, 1, 2])
@pytest.mark.parametrize("field,value", [(0, 2), (2, -1), (3, -1), (4, 0), (5, 0), (6, 1), (7, 1),
                                         (8, 0)])
def test_bad_descriptor_field(which, field, value):
    """DTYPE_ other than dense, negative sizes, empty blocks, a first block
    off process (0, 0) of the 1 x 1 grid, LLD_ below M_."""
    d = list(good())
    bad = list(d[which])
    bad[field] = value
    if field == 8:
        bad[8] = bad[2] - 1
    d[which] = bad
    assert call(*d) == cm.COSMA_ERR_INVALID_ARG


@pytest.mark.parametrize("which", [0, 1, 2])
def test_null_descriptor(which):
    d = list(good())
    d[which] = None
    assert call(*d) == cm.COSMA_ERR_INVALID_ARG


@pytest.mark.parametrize("kw", [dict(ia=0), dict(ja=0), dict(ib=0), dict(jb=0), dict(ic=0),
                                dict(jc=0)])
def test_offsets_are_one_based(kw):
    assert call(*good(), **kw) == cm.COSMA_ERR_INVALID_ARG


@pytest.mark.parametrize("ta", [N, T])
@pytest.mark.parametrize("tb", [N, T])
def test_submatrix_must_fit(ta, tb):
    """op(sub(A)) is m x k: stored k x m when transposed, and the block from
    (ia, ja) must stay inside M_ x N_ (likewise B and C)."""
    m, n, k = 4, 3, 2
    a_rows, a_cols = (k, m) if ta == T else (m, k)
    b_rows, b_cols = (n, k) if tb == T else (k, n)
    da = cm.descinit(6, 6, 2, 2, 6)
    db = cm.descinit(6, 6, 2, 2, 6)
    dc = cm.descinit(6, 6, 2, 2, 6)
    args = dict(m=m, n=n, k=k, ta=ta, tb=tb)
    # the last legal positions pass the descriptor checks only if they fit:
    # one step further is rejected
    assert call(da, db, dc, ia=6 - a_rows + 2, **args) == cm.COSMA_ERR_INVALID_ARG
    assert call(da, db, dc, ja=6 - a_cols + 2, **args) == cm.COSMA_ERR_INVALID_ARG
    assert call(da, db, dc, ib=6 - b_rows + 2, **args) == cm.COSMA_ERR_INVALID_ARG
    assert call(da, db, dc, jb=6 - b_cols + 2, **args) == cm.COSMA_ERR_INVALID_ARG
    assert call(da, db, dc, ic=6 - m + 2, **args) == cm.COSMA_ERR_INVALID_ARG
    assert call(da, db, dc, jc=6 - n + 2, **args) == cm.COSMA_ERR_INVALID_ARG


def test_flags_sizes_dtype():
    assert call(*good(), ta=2) == cm.COSMA_ERR_INVALID_ARG
    assert call(*good(), tb=-1) == cm.COSMA_ERR_INVALID_ARG
    assert call(*good(), m=-1) == cm.COSMA_ERR_INVALID_ARG
    assert call(*good(), dtype=9) == cm.COSMA_ERR_INVALID_ARG


def test_argument_errors_of_the_column_major_product_pass_through():
    """Descriptors that pass but leave a null operand for a product that
    reads it: cosma_gemm_ex's own check rejects it."""
    assert call(*good()) == cm.COSMA_ERR_INVALID_ARG
