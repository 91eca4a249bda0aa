"""Ozaki INT8-slice path (FP64-accurate) on the GPU against the oracle."""
import numpy as np
import pytest

import oracle
import synth
import paper_1908_09606_amd as cm
from gpu_util import contract_check, device_matrix, log, run_gemm, sampled_check, sample_indices

pytestmark = pytest.mark.gpu

OZ = cm.COSMA_F64_OZAKI_I8
SHAPES = [(1, 1, 1), (1, 7, 3), (17, 33, 5), (64, 64, 64), (65, 63, 65), (130, 129, 131),
          (257, 300, 97), (300, 257, 1000), (129, 1, 64), (1, 300, 45)]


def oz_plan(m, n, k, slices, p_k=1):
    rc, plan = cm.cosma_plan_make(m, n, k, OZ, 0, p_k)
    assert rc == 0
    assert cm.cosma_plan_set_slices(plan, slices) == 0
    return plan


@pytest.mark.parametrize("slices", [1, 2, 7])
def test_integer_single_digit_exact(gpu, slices):
    """|x| <= 127 integers need one digit after row/column scaling, so the
    slice products are the exact integer product for every s."""
    for (m, n, k) in SHAPES:
        log(f"ozaki s={slices} int {m}x{n}x{k}")
        lda, ldb, ldc = k + 3, n + 1, n + 2
        _, A = device_matrix(m, k, 5, synth.STREAM_A, synth.INT_F64, 127, ld=lda)
        _, B = device_matrix(k, n, 5, synth.STREAM_B, synth.INT_F64, 127, ld=ldb)
        _, C = device_matrix(m, n, 5, synth.STREAM_C, synth.INT_F64, 127, ld=ldc)
        plan = oz_plan(m, n, k, slices)
        assert run_gemm(cm, m, n, k, A, lda, B, ldb, C, ldc, plan=plan) == 0
        Ah = synth.gen(m, k, 5, synth.STREAM_A, synth.INT_F64, 127).astype(np.int64)
        Bh = synth.gen(k, n, 5, synth.STREAM_B, synth.INT_F64, 127).astype(np.int64)
        assert np.array_equal(C.cpu().numpy(), (Ah @ Bh).astype(np.float64)), (m, n, k)


def test_two_digit_times_one_digit_exact_with_two_slices(gpu):
    """A with 14-bit integers needs two digits, B with 7-bit integers one: with
    s = 2 the triangular truncation (u + v <= 3) drops only zero products, so
    the result is exact (error-free transformation)."""
    m, n, k = 190, 150, 700
    _, A = device_matrix(m, k, 8, synth.STREAM_A, synth.INT_F64, 16383)
    _, B = device_matrix(k, n, 8, synth.STREAM_B, synth.INT_F64, 127)
    _, C = device_matrix(m, n, 8, synth.STREAM_C, synth.UNIFORM_F64)
    plan = oz_plan(m, n, k, 2)
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, plan=plan) == 0
    Ah = synth.gen(m, k, 8, synth.STREAM_A, synth.INT_F64, 16383).astype(np.int64)
    Bh = synth.gen(k, n, 8, synth.STREAM_B, synth.INT_F64, 127).astype(np.int64)
    assert np.array_equal(C.cpu().numpy(), (Ah @ Bh).astype(np.float64))
    # with one slice the second digit of A is dropped: the result must differ
    plan1 = oz_plan(m, n, k, 1)
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, plan=plan1) == 0
    assert not np.array_equal(C.cpu().numpy(), (Ah @ Bh).astype(np.float64))


def test_split_k_bit_identical_on_integers(gpu):
    m, n, k = 200, 190, 3000
    Ah = synth.gen(m, k, 9, synth.STREAM_A, synth.INT_F64, 127).astype(np.int64)
    Bh = synth.gen(k, n, 9, synth.STREAM_B, synth.INT_F64, 127).astype(np.int64)
    exact = (Ah @ Bh).astype(np.float64)
    _, A = device_matrix(m, k, 9, synth.STREAM_A, synth.INT_F64, 127)
    _, B = device_matrix(k, n, 9, synth.STREAM_B, synth.INT_F64, 127)
    for pk in (1, 2, 3, 5):
        _, C = device_matrix(m, n, 1, synth.STREAM_C, synth.UNIFORM_F64)
        plan = oz_plan(m, n, k, 3, pk)
        assert plan.p_k == pk
        assert run_gemm(cm, m, n, k, A, k, B, n, C, n, plan=plan) == 0
        assert np.array_equal(C.cpu().numpy(), exact), pk


@pytest.mark.parametrize("slices", [6, 7, 8])
def test_wide_exponent_data_error(gpu, slices):
    """Entries sign * U[1,2) * 2^e, e in [-20, 20]: every s keeps the plan's
    error contract; s = 7 and 8 also meet 4k * 2^-53 on every entry here
    (s = 7 beyond its guaranteed spread_limit), s = 6 does not."""
    m, n, k = 300, 280, 2048
    _, A = device_matrix(m, k, 4, synth.STREAM_A, synth.WIDE_F64)
    _, B = device_matrix(k, n, 4, synth.STREAM_B, synth.WIDE_F64)
    _, C = device_matrix(m, n, 4, synth.STREAM_C, synth.UNIFORM_F64)
    C0 = synth.gen(m, n, 4, synth.STREAM_C, synth.UNIFORM_F64)
    alpha, beta = 1.5, -0.25
    plan = oz_plan(m, n, k, slices)
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, alpha, beta, plan=plan) == 0
    ref, D = oracle.gemm(synth.gen(m, k, 4, synth.STREAM_A, synth.WIDE_F64),
                         synth.gen(k, n, 4, synth.STREAM_B, synth.WIDE_F64), alpha, beta, C0)
    err = oracle.normalised_err(C.cpu().numpy(), ref, D)
    ratio, cov, _ = contract_check(C.cpu().numpy(), synth.gen(m, k, 4, synth.STREAM_A, synth.WIDE_F64),
                                   synth.gen(k, n, 4, synth.STREAM_B, synth.WIDE_F64), plan, alpha,
                                   beta, C0)
    log(f"  ozaki s={slices} err={err:.3e} bound={oracle.fp64_bound(k):.3e} "
        f"contract {ratio:.3g}, covered {cov:.3f}")
    if slices >= 7:
        assert err <= oracle.fp64_bound(k)
    else:
        assert err < 1e-9


def test_zero_rows_and_columns(gpu):
    """An all-zero row of A / column of B gets exponent 0 and zero digits:
    its row / column of C is exactly zero and the rest stays exact."""
    import torch
    m, n, k = 70, 80, 90
    _, A = device_matrix(m, k, 3, synth.STREAM_A, synth.INT_F64, 127)
    _, B = device_matrix(k, n, 3, synth.STREAM_B, synth.INT_F64, 127)
    A[5].zero_()
    B[:, 7].zero_()
    C = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, dtype=OZ) == 0
    Ah, Bh = A.cpu().numpy().astype(np.int64), B.cpu().numpy().astype(np.int64)
    Ch = C.cpu().numpy()
    assert np.all(Ch[5] == 0.0) and np.all(Ch[:, 7] == 0.0)
    assert np.array_equal(Ch, (Ah @ Bh).astype(np.float64))


def test_small_k_wide_exponents_within_contract(gpu):
    """With 41 binades of exponent spread and few terms, D_ij can lie far
    below 2^(e_i + f_j): at k = 90 the spread of some entries exceeds every
    plan's spread_limit, so 4k * 2^-53 is not promised there.  Every entry
    keeps the absolute bound, the covered entries meet 4k * 2^-53, and the
    error shrinks by about 2^-7 per extra slice."""
    m, n, k = 70, 80, 90
    _, A = device_matrix(m, k, 3, synth.STREAM_A, synth.WIDE_F64)
    _, B = device_matrix(k, n, 3, synth.STREAM_B, synth.WIDE_F64)
    Ah = synth.gen(m, k, 3, synth.STREAM_A, synth.WIDE_F64)
    Bh = synth.gen(k, n, 3, synth.STREAM_B, synth.WIDE_F64)
    ref, D = oracle.gemm(Ah, Bh)
    errs = {}
    for s in (6, 7, 8):
        _, C = device_matrix(m, n, 3, synth.STREAM_C, synth.UNIFORM_F64)
        plan = oz_plan(m, n, k, s)
        assert run_gemm(cm, m, n, k, A, k, B, n, C, n, plan=plan) == 0
        errs[s] = oracle.normalised_err(C.cpu().numpy(), ref, D)
        contract_check(C.cpu().numpy(), Ah, Bh, plan, 1.0, 0.0, None)
    log(f"  k=90 wide exponents: errors by slices {errs}, 4k*2^-53 = {oracle.fp64_bound(k):.2e}")
    assert errs[8] < errs[7] < errs[6] < 1e-6
    assert errs[7] / errs[8] > 16 and errs[6] / errs[7] > 16


def test_blas_quick_returns(gpu):
    import torch
    m, n, k = 70, 90, 33
    _, A = device_matrix(m, k, 4, synth.STREAM_A, synth.UNIFORM_F64)
    _, B = device_matrix(k, n, 4, synth.STREAM_B, synth.UNIFORM_F64)
    _, C = device_matrix(m, n, 4, synth.STREAM_C, synth.UNIFORM_F64)
    C0 = C.clone()
    An = A.clone().fill_(float("nan"))
    assert run_gemm(cm, m, n, k, An, k, B, n, C, n, 0.0, 0.5, dtype=OZ) == 0
    assert torch.equal(C, 0.5 * C0)
    C.copy_(C0)
    assert run_gemm(cm, m, n, 0, A, 1, B, n, C, n, 1.0, 2.0, dtype=OZ) == 0
    assert torch.equal(C, 2.0 * C0)


@pytest.mark.parametrize("slices", [3, 7])
def test_equals_exact_truncated_digit_sum(gpu, slices):
    """With one split the digit path computes, exactly up to its final
    binary64 additions, 2^(e_i + f_j) sum_{u+v <= s+1} 2^-7(u+v) (A_u B_v)_ij:
    digits from the recurrence d_u = trunc(2^7 r_(u-1)), r_u = 2^7 r_(u-1) -
    d_u of A 2^-e (exact in binary64), integer products summed exactly here.
    The kernel adds its s diagonal sums in binary64, so the result lies
    within s ulps of the correctly rounded value."""
    import math
    m, n, k = 37, 29, 300
    Ah = synth.gen(m, k, 33, synth.STREAM_A, synth.WIDE_F64)
    Bh = synth.gen(k, n, 33, synth.STREAM_B, synth.WIDE_F64)
    _, A = device_matrix(m, k, 33, synth.STREAM_A, synth.WIDE_F64)
    _, B = device_matrix(k, n, 33, synth.STREAM_B, synth.WIDE_F64)
    import torch
    C = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    plan = oz_plan(m, n, k, slices)
    assert plan.p_k == 1
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, plan=plan) == 0
    got = C.cpu().numpy()
    e = np.array([math.frexp(float(np.max(np.abs(Ah[i]))))[1] for i in range(m)])
    f = np.array([math.frexp(float(np.max(np.abs(Bh[:, j]))))[1] for j in range(n)])

    def digits(X):  # rows of X already scaled into (-1, 1)
        out = []
        for _ in range(slices):
            y = X * 128.0
            d = np.trunc(y)
            X = y - d
            out.append(d.astype(np.int64))
        return out

    Ad = digits(np.ldexp(Ah, -e[:, None]))
    Bd = digits(np.ldexp(Bh, -f[None, :]))
    worst = 0.0
    P = {(u, v): Ad[u] @ Bd[v] for u in range(slices) for v in range(slices) if u + v <= slices - 1}
    for i in range(m):
        for j in range(n):
            # sum over pairs with weight 2^(7 (2s - (u+1) - (v+1))), exact integers
            S = sum(int(p[i, j]) << (7 * (2 * slices - u - v - 2)) for (u, v), p in P.items())
            sh = int(e[i] + f[j]) - 14 * slices
            ref = S * 2 ** sh if sh >= 0 else S / 2 ** (-sh)
            ulps = abs(got[i, j] - ref) / math.ulp(ref) if ref != 0.0 else abs(got[i, j])
            worst = max(worst, ulps)
    log(f"  ozaki s={slices}: worst {worst:.2f} ulp from the rounded exact truncated sum")
    assert worst <= slices
