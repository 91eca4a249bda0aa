"""Modular (Ozaki scheme II) FP64-accurate path on the GPU against the oracle.

The reconstruction is exact: for integer inputs (any number of moduli whose
beta covers the inputs' bits) the result is the exact integer product, and
splitting k changes nothing in the result bit for bit, whatever the data."""
import numpy as np
import pytest

import oracle
import synth
import paper_1908_09606_amd as cm
from gpu_util import contract_check, device_matrix, log, run_gemm

pytestmark = pytest.mark.gpu

OZ2 = cm.COSMA_F64_OZAKI2_I8
SHAPES = [(1, 1, 1), (1, 7, 3), (17, 33, 5), (64, 64, 64), (65, 63, 65), (257, 129, 131),
          (300, 257, 1000), (513, 300, 97), (129, 1, 64), (1, 300, 45)]


def oz2_plan(m, n, k, nmod, p_k=1):
    rc, plan = cm.cosma_plan_make(m, n, k, OZ2, 0, p_k)
    assert rc == 0
    assert cm.cosma_plan_set_slices(plan, nmod) == 0
    return plan


@pytest.mark.parametrize("nmod", [4, 8, 14, 16])
def test_integer_exact(gpu, nmod):
    """|x| <= 127 integers are exact after scaling (beta >= 8 for every k
    here), so the modular products give the exact integer product."""
    for (m, n, k) in SHAPES:
        log(f"ozaki2 N={nmod} int {m}x{n}x{k}")
        lda, ldb, ldc = k + 3, n + 1, n + 2
        _, A = device_matrix(m, k, 5, synth.STREAM_A, synth.INT_F64, 127, ld=lda)
        _, B = device_matrix(k, n, 5, synth.STREAM_B, synth.INT_F64, 127, ld=ldb)
        _, C = device_matrix(m, n, 5, synth.STREAM_C, synth.INT_F64, 127, ld=ldc)
        rc, beta, _ = cm.cosma_ozaki2_params(k, nmod)
        assert rc == 0 and beta >= 8
        assert run_gemm(cm, m, n, k, A, lda, B, ldb, C, ldc, plan=oz2_plan(m, n, k, nmod)) == 0
        Ah = synth.gen(m, k, 5, synth.STREAM_A, synth.INT_F64, 127).astype(np.int64)
        Bh = synth.gen(k, n, 5, synth.STREAM_B, synth.INT_F64, 127).astype(np.int64)
        assert np.array_equal(C.cpu().numpy(), (Ah @ Bh).astype(np.float64)), (m, n, k)


@pytest.mark.parametrize("sign", [1.0, -1.0])
@pytest.mark.parametrize("k", [1000, 65536, 70000])
def test_top_of_range_exact(gpu, sign, k):
    """Every entry 1 - 2^-20 (B negated for sign -1): the scaled operands sit
    just below 2^beta, so sum_t A'B' = k (2^beta - 2^(beta-20))^2 is close to
    the largest value the moduli must hold (k 2^(2 beta) <= M / 4).  The
    product k (1 - 2^-20)^2 has 40 + log2 k significant bits: exact."""
    import torch
    m, n = 70, 90
    v = 1.0 - 2.0 ** -20
    A = torch.full((m, k), v, dtype=torch.float64, device="cuda")
    B = torch.full((k, n), sign * v, dtype=torch.float64, device="cuda")
    C = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    for nmod in (6, 14):
        rc, beta, _ = cm.cosma_ozaki2_params(k, nmod)
        assert rc == 0
        if beta < 20:
            continue  # 1 - 2^-20 would not be exact after scaling
        log(f"ozaki2 N={nmod} top of range k={k} sign={sign} beta={beta}")
        C.fill_(float("nan"))
        assert run_gemm(cm, m, n, k, A, k, B, n, C, n, dtype=OZ2,
                        plan=oz2_plan(m, n, k, nmod, -(-k // 65536))) == 0
        exact = sign * k * (1.0 - 2.0 ** -19 + 2.0 ** -40)
        assert torch.all(C == exact).item(), (C[0, 0].item(), exact)


def test_split_k_bit_identical_any_data(gpu):
    """Residues of the split sums add up modulo each p_l before the
    reconstruction: the result does not depend on p_k, bit for bit, also on
    data that is not integer."""
    import torch
    m, n, k = 300, 190, 3000
    _, A = device_matrix(m, k, 9, synth.STREAM_A, synth.WIDE_F64)
    _, B = device_matrix(k, n, 9, synth.STREAM_B, synth.UNIFORM_F64)
    ref = None
    for pk in (1, 2, 3, 5, 8):
        _, C = device_matrix(m, n, 1, synth.STREAM_C, synth.UNIFORM_F64)
        plan = oz2_plan(m, n, k, 14, pk)
        assert plan.p_k == pk
        assert run_gemm(cm, m, n, k, A, k, B, n, C, n, plan=plan) == 0
        if ref is None:
            ref = C.clone()
        else:
            assert torch.equal(C, ref), pk
    Ah = synth.gen(m, k, 9, synth.STREAM_A, synth.WIDE_F64)
    Bh = synth.gen(k, n, 9, synth.STREAM_B, synth.UNIFORM_F64)
    r, D = oracle.gemm(Ah, Bh)
    err = oracle.normalised_err(ref.cpu().numpy(), r, D)
    log(f"  split-invariant result err={err:.3e}")
    assert err <= oracle.fp64_bound(k)


@pytest.mark.parametrize("nmod", [12, 13, 14, 15, 16])
def test_wide_exponent_data_error(gpu, nmod):
    """Entries sign * U[1,2) * 2^e, e in [-20, 20] (41 binades), alpha and
    beta != 0: every N keeps the plan's error contract; N >= 14 also meets
    4k * 2^-53 on every entry here (beyond the guaranteed spread_limit);
    the error grows about 2^4 per modulus dropped."""
    m, n, k = 300, 280, 2048
    _, A = device_matrix(m, k, 4, synth.STREAM_A, synth.WIDE_F64)
    _, B = device_matrix(k, n, 4, synth.STREAM_B, synth.WIDE_F64)
    _, C = device_matrix(m, n, 4, synth.STREAM_C, synth.UNIFORM_F64)
    C0 = synth.gen(m, n, 4, synth.STREAM_C, synth.UNIFORM_F64)
    alpha, beta = 1.5, -0.25
    plan = oz2_plan(m, n, k, nmod)
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, alpha, beta, plan=plan) == 0
    Ah = synth.gen(m, k, 4, synth.STREAM_A, synth.WIDE_F64)
    Bh = synth.gen(k, n, 4, synth.STREAM_B, synth.WIDE_F64)
    ref, D = oracle.gemm(Ah, Bh, alpha, beta, C0)
    err = oracle.normalised_err(C.cpu().numpy(), ref, D)
    contract_check(C.cpu().numpy(), Ah, Bh, plan, alpha, beta, C0)
    log(f"  ozaki2 N={nmod} beta={cm.cosma_ozaki2_params(k, nmod)[1]} err={err:.3e} "
        f"bound={oracle.fp64_bound(k):.3e}")
    if nmod >= 14:
        assert err <= oracle.fp64_bound(k)
    else:
        assert err < 1e-6


def test_uniform_data_default_plan(gpu):
    """Uniform [-1, 1) data through cosma_gemm's own plan (N from the error
    contract)."""
    for (m, n, k) in [(513, 300, 97), (1000, 1100, 1500), (64, 64, 70000)]:
        _, A = device_matrix(m, k, 6, synth.STREAM_A, synth.UNIFORM_F64)
        _, B = device_matrix(k, n, 6, synth.STREAM_B, synth.UNIFORM_F64)
        _, C = device_matrix(m, n, 6, synth.STREAM_C, synth.UNIFORM_F64)
        assert run_gemm(cm, m, n, k, A, k, B, n, C, n, dtype=OZ2) == 0
        ref, D = oracle.gemm(synth.gen(m, k, 6, synth.STREAM_A, synth.UNIFORM_F64),
                             synth.gen(k, n, 6, synth.STREAM_B, synth.UNIFORM_F64))
        err = oracle.normalised_err(C.cpu().numpy(), ref, D)
        log(f"  ozaki2 uniform {m}x{n}x{k} err={err:.3e}")
        assert err <= oracle.fp64_bound(k)


def test_zero_rows_and_columns(gpu):
    import torch
    m, n, k = 70, 80, 90
    _, A = device_matrix(m, k, 3, synth.STREAM_A, synth.INT_F64, 127)
    _, B = device_matrix(k, n, 3, synth.STREAM_B, synth.INT_F64, 127)
    A[5].zero_()
    B[:, 7].zero_()
    C = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, dtype=OZ2) == 0
    Ah, Bh = A.cpu().numpy().astype(np.int64), B.cpu().numpy().astype(np.int64)
    Ch = C.cpu().numpy()
    assert np.all(Ch[5] == 0.0) and np.all(Ch[:, 7] == 0.0)
    assert np.array_equal(Ch, (Ah @ Bh).astype(np.float64))


def test_blas_quick_returns(gpu):
    import torch
    m, n, k = 70, 90, 33
    _, A = device_matrix(m, k, 4, synth.STREAM_A, synth.UNIFORM_F64)
    _, B = device_matrix(k, n, 4, synth.STREAM_B, synth.UNIFORM_F64)
    _, C = device_matrix(m, n, 4, synth.STREAM_C, synth.UNIFORM_F64)
    C0 = C.clone()
    An = A.clone().fill_(float("nan"))
    assert run_gemm(cm, m, n, k, An, k, B, n, C, n, 0.0, 0.5, dtype=OZ2) == 0
    assert torch.equal(C, 0.5 * C0)
    C.copy_(C0)
    assert run_gemm(cm, m, n, 0, A, 1, B, n, C, n, 1.0, 2.0, dtype=OZ2) == 0
    assert torch.equal(C, 2.0 * C0)


@pytest.mark.parametrize("dtype", ["ozaki", "ozaki2", "ozaki_bf16"])
def test_nonfinite_rows_and_columns_give_nan(gpu, dtype):
    """Every Ozaki form scales whole rows of A and columns of B, so a NaN or an
    infinity there makes that row / column of C NaN (with beta != 0 too);
    every other entry stays the exact integer product."""
    import torch
    m, n, k = 140, 150, 300
    _, A = device_matrix(m, k, 7, synth.STREAM_A, synth.INT_F64, 127)
    _, B = device_matrix(k, n, 7, synth.STREAM_B, synth.INT_F64, 127)
    Ah, Bh = A.cpu().numpy().astype(np.int64), B.cpu().numpy().astype(np.int64)
    A[3, 5] = float("nan")
    A[100, 0] = float("inf")
    B[7, 2] = float("-inf")
    B[299, 149] = float("nan")
    C = torch.ones((m, n), dtype=torch.float64, device="cuda")
    d = cm.DTYPES[dtype]
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, 1.0, 2.0, dtype=d) == 0
    Ch = C.cpu().numpy()
    bad_r, bad_c = [3, 100], [2, 149]
    assert np.isnan(Ch[bad_r, :]).all() and np.isnan(Ch[:, bad_c]).all()
    keep_r = np.setdiff1d(np.arange(m), bad_r)
    keep_c = np.setdiff1d(np.arange(n), bad_c)
    exact = (Ah @ Bh).astype(np.float64) + 2.0
    assert np.array_equal(Ch[np.ix_(keep_r, keep_c)], exact[np.ix_(keep_r, keep_c)])


@pytest.mark.parametrize("nmod,k", [(14, 300), (9, 1000), (16, 64)])
def test_equals_exact_scaled_integer_product(gpu, nmod, k):
    """The modular path computes the scaled integer product exactly: with
    e_i, f_j the exponents of the row / column maxima (max < 2^e) and beta
    from cosma_ozaki2_params, A'_it = rint(A_it 2^(beta - e_i)) and
    B'_tj = rint(B_tj 2^(beta - f_j)) are integers, C'_ij = sum_t A'_it B'_tj
    is recovered exactly by the reconstruction, and C_ij is C'_ij 2^(e_i + f_j
    - 2 beta) rounded to binary64 (the limb-by-limb conversion rounds up to
    twice: within 2 ulps of the correctly rounded value).  Checked on
    wide-exponent, non-integer data against big-integer arithmetic written
    out here, far inside the 4k 2^-53 bound."""
    import math
    m, n = 37, 29
    Ah = synth.gen(m, k, 31, synth.STREAM_A, synth.WIDE_F64)
    Bh = synth.gen(k, n, 31, synth.STREAM_B, synth.WIDE_F64)
    _, A = device_matrix(m, k, 31, synth.STREAM_A, synth.WIDE_F64)
    _, B = device_matrix(k, n, 31, synth.STREAM_B, synth.WIDE_F64)
    import torch
    C = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, plan=oz2_plan(m, n, k, nmod)) == 0
    got = C.cpu().numpy()
    rc, beta, _ = cm.cosma_ozaki2_params(k, nmod)
    assert rc == 0
    e = [math.frexp(float(np.max(np.abs(Ah[i]))))[1] for i in range(m)]
    f = [math.frexp(float(np.max(np.abs(Bh[:, j]))))[1] for j in range(n)]
    # scaling by a power of two is exact; rint of the scaled value is exact
    Ai = [[int(np.rint(math.ldexp(float(Ah[i, t]), beta - e[i]))) for t in range(k)] for i in range(m)]
    Bi = [[int(np.rint(math.ldexp(float(Bh[t, j]), beta - f[j]))) for t in range(k)] for j in range(n)]
    worst = 0.0
    for i in range(m):
        for j in range(n):
            exact = sum(a * b for a, b in zip(Ai[i], Bi[j]))
            sh = e[i] + f[j] - 2 * beta
            ref = math.ldexp(float(exact), sh) if abs(exact) < 2 ** 53 else \
                float(exact * 2 ** sh) if sh >= 0 else exact / 2 ** (-sh)
            ulps = abs(got[i, j] - ref) / math.ulp(ref) if ref != 0.0 else abs(got[i, j])
            worst = max(worst, ulps)
    log(f"  ozaki2 N={nmod} k={k} beta={beta}: worst {worst:.2f} ulp from the rounded exact product")
    assert worst <= 2.0
