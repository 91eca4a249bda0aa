"""Ozaki digit path on bf16 slices (FP64-accurate) on the GPU against the
oracle and against its exact arithmetic written out here."""
import math

import numpy as np
import pytest

import oracle
import synth
import paper_1908_09606_amd as cm
from gpu_util import contract_check, device_matrix, log, run_gemm

pytestmark = pytest.mark.gpu

OB = cm.COSMA_F64_OZAKI_BF16
SHAPES = [(1, 1, 1), (1, 7, 3), (17, 33, 5), (64, 64, 64), (65, 63, 65), (130, 129, 131),
          (257, 300, 97), (300, 257, 1000), (129, 1, 64), (1, 300, 45)]


def ob_plan(m, n, k, slices, p_k=1):
    rc, plan = cm.cosma_plan_make(m, n, k, OB, 0, p_k)
    assert rc == 0
    assert cm.cosma_plan_set_slices(plan, slices) == 0
    return plan


@pytest.mark.parametrize("slices", [1, 2, 6, 7, 8])
def test_integer_single_digit_exact(gpu, slices):
    """|x| <= 255 integers are one digit after row / column scaling, so
    the slice products are the exact integer product for every s (this
    covers both kernel layouts: 8 waves up to s = 6, 4 waves above)."""
    for (m, n, k) in SHAPES:
        log(f"ozaki_bf16 s={slices} int {m}x{n}x{k}")
        lda, ldb, ldc = k + 3, n + 1, n + 2
        _, A = device_matrix(m, k, 5, synth.STREAM_A, synth.INT_F64, 255, ld=lda)
        _, B = device_matrix(k, n, 5, synth.STREAM_B, synth.INT_F64, 255, ld=ldb)
        _, C = device_matrix(m, n, 5, synth.STREAM_C, synth.INT_F64, 255, ld=ldc)
        plan = ob_plan(m, n, k, slices)
        assert run_gemm(cm, m, n, k, A, lda, B, ldb, C, ldc, plan=plan) == 0
        Ah = synth.gen(m, k, 5, synth.STREAM_A, synth.INT_F64, 255).astype(np.int64)
        Bh = synth.gen(k, n, 5, synth.STREAM_B, synth.INT_F64, 255).astype(np.int64)
        assert np.array_equal(C.cpu().numpy(), (Ah @ Bh).astype(np.float64)), (m, n, k)


def test_two_digit_times_one_digit_exact_with_two_slices(gpu):
    """A with 16-bit integers needs two 8-bit digits, B with 8-bit integers
    one: with s = 2 the truncation (u + v <= 3) drops only zero products, so
    the result is exact; with s = 1 the second digit of A is lost."""
    m, n, k = 190, 150, 700
    _, A = device_matrix(m, k, 8, synth.STREAM_A, synth.INT_F64, 65535)
    _, B = device_matrix(k, n, 8, synth.STREAM_B, synth.INT_F64, 255)
    _, C = device_matrix(m, n, 8, synth.STREAM_C, synth.UNIFORM_F64)
    Ah = synth.gen(m, k, 8, synth.STREAM_A, synth.INT_F64, 65535).astype(np.int64)
    Bh = synth.gen(k, n, 8, synth.STREAM_B, synth.INT_F64, 255).astype(np.int64)
    exact = (Ah @ Bh).astype(np.float64)
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, plan=ob_plan(m, n, k, 2)) == 0
    assert np.array_equal(C.cpu().numpy(), exact)
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, plan=ob_plan(m, n, k, 1)) == 0
    assert not np.array_equal(C.cpu().numpy(), exact)


def test_split_k_bit_identical_on_integers(gpu):
    m, n, k = 200, 190, 3000
    Ah = synth.gen(m, k, 9, synth.STREAM_A, synth.INT_F64, 255).astype(np.int64)
    Bh = synth.gen(k, n, 9, synth.STREAM_B, synth.INT_F64, 255).astype(np.int64)
    exact = (Ah @ Bh).astype(np.float64)
    _, A = device_matrix(m, k, 9, synth.STREAM_A, synth.INT_F64, 255)
    _, B = device_matrix(k, n, 9, synth.STREAM_B, synth.INT_F64, 255)
    for pk in (1, 2, 3, 5):
        _, C = device_matrix(m, n, 1, synth.STREAM_C, synth.UNIFORM_F64)
        plan = ob_plan(m, n, k, 3, pk)
        assert plan.p_k == pk
        assert run_gemm(cm, m, n, k, A, k, B, n, C, n, plan=plan) == 0
        assert np.array_equal(C.cpu().numpy(), exact), pk


@pytest.mark.parametrize("slices", [5, 6, 7, 8])
def test_wide_exponent_data_error(gpu, slices):
    """Entries sign * U[1,2) * 2^e, e in [-20, 20]: every s keeps the plan's
    error contract; s >= 6 (48 bits) also meets 4k * 2^-53 on every entry
    here (s = 6 beyond its guaranteed spread_limit), s = 5 does not."""
    m, n, k = 300, 280, 2048
    _, A = device_matrix(m, k, 4, synth.STREAM_A, synth.WIDE_F64)
    _, B = device_matrix(k, n, 4, synth.STREAM_B, synth.WIDE_F64)
    _, C = device_matrix(m, n, 4, synth.STREAM_C, synth.UNIFORM_F64)
    C0 = synth.gen(m, n, 4, synth.STREAM_C, synth.UNIFORM_F64)
    alpha, beta = 1.5, -0.25
    plan = ob_plan(m, n, k, slices)
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, alpha, beta, plan=plan) == 0
    Ah = synth.gen(m, k, 4, synth.STREAM_A, synth.WIDE_F64)
    Bh = synth.gen(k, n, 4, synth.STREAM_B, synth.WIDE_F64)
    ref, D = oracle.gemm(Ah, Bh, alpha, beta, C0)
    err = oracle.normalised_err(C.cpu().numpy(), ref, D)
    ratio, cov, _ = contract_check(C.cpu().numpy(), Ah, Bh, plan, alpha, beta, C0)
    log(f"  ozaki_bf16 s={slices} err={err:.3e} bound={oracle.fp64_bound(k):.3e} "
        f"contract {ratio:.3g}, covered {cov:.3f}")
    if slices >= 6:
        assert err <= oracle.fp64_bound(k)
    else:
        assert err < 1e-9


def test_uniform_data_within_bound(gpu):
    m, n, k = 257, 190, 5000
    _, A = device_matrix(m, k, 6, synth.STREAM_A, synth.UNIFORM_F64)
    _, B = device_matrix(k, n, 6, synth.STREAM_B, synth.UNIFORM_F64)
    _, C = device_matrix(m, n, 6, synth.STREAM_C, synth.UNIFORM_F64)
    C0 = synth.gen(m, n, 6, synth.STREAM_C, synth.UNIFORM_F64)
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, -1.0, 0.5, dtype=OB) == 0
    ref, D = oracle.gemm(synth.gen(m, k, 6, synth.STREAM_A, synth.UNIFORM_F64),
                         synth.gen(k, n, 6, synth.STREAM_B, synth.UNIFORM_F64), -1.0, 0.5, C0)
    err = oracle.normalised_err(C.cpu().numpy(), ref, D)
    log(f"  ozaki_bf16 uniform err={err:.3e} bound={oracle.fp64_bound(k):.3e}")
    assert err <= oracle.fp64_bound(k)


def test_small_k_wide_exponents_within_contract(gpu):
    """At k = 90 on 41-binade data D_ij can lie far below 2^(e_i + f_j): every
    entry keeps the plan's absolute bound, the entries within spread_limit
    meet 4k * 2^-53, and the error shrinks by about 2^-8 per extra slice."""
    m, n, k = 70, 80, 90
    _, A = device_matrix(m, k, 3, synth.STREAM_A, synth.WIDE_F64)
    _, B = device_matrix(k, n, 3, synth.STREAM_B, synth.WIDE_F64)
    Ah = synth.gen(m, k, 3, synth.STREAM_A, synth.WIDE_F64)
    Bh = synth.gen(k, n, 3, synth.STREAM_B, synth.WIDE_F64)
    ref, D = oracle.gemm(Ah, Bh)
    errs = {}
    for s in (5, 6, 7):
        _, C = device_matrix(m, n, 3, synth.STREAM_C, synth.UNIFORM_F64)
        plan = ob_plan(m, n, k, s)
        assert run_gemm(cm, m, n, k, A, k, B, n, C, n, plan=plan) == 0
        errs[s] = oracle.normalised_err(C.cpu().numpy(), ref, D)
        contract_check(C.cpu().numpy(), Ah, Bh, plan, 1.0, 0.0, None)
    log(f"  k=90 wide exponents: errors by slices {errs}, 4k*2^-53 = {oracle.fp64_bound(k):.2e}")
    assert errs[7] < errs[6] < errs[5] < 1e-6
    assert errs[5] / errs[6] > 32 and errs[6] / errs[7] > 32


def test_zero_rows_and_columns(gpu):
    import torch
    m, n, k = 70, 80, 90
    _, A = device_matrix(m, k, 3, synth.STREAM_A, synth.INT_F64, 255)
    _, B = device_matrix(k, n, 3, synth.STREAM_B, synth.INT_F64, 255)
    A[5].zero_()
    B[:, 7].zero_()
    C = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, dtype=OB) == 0
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
    assert run_gemm(cm, m, n, k, An, k, B, n, C, n, 0.0, 0.5, dtype=OB) == 0
    assert torch.equal(C, 0.5 * C0)
    C.copy_(C0)
    assert run_gemm(cm, m, n, 0, A, 1, B, n, C, n, 1.0, 2.0, dtype=OB) == 0
    assert torch.equal(C, 2.0 * C0)


@pytest.mark.parametrize("slices", [3, 6])
def test_equals_exact_truncated_digit_sum(gpu, slices):
    """With one split the path computes 2^(e_i + f_j) sum_{u+v <= s+1}
    2^-8(u+v) (A_u B_v)_ij exactly up to its binary64 additions: digits
    d_u = rint(2^8 r_(u-1)), r_u = 2^8 r_(u-1) - d_u of A 2^-e (exact in
    binary64; |d_1| <= 256, |d_u| <= 128 after), integer products summed
    exactly here.  Per 32-k round the
    kernel adds each of its s exact diagonal sums, scaled, to a running
    binary64 sum, so the distance to the exact value is at most
    (s rounds + 1) 2^-53 times the sum of the rounds' absolute diagonal
    contributions, plus half an ulp of the result."""
    import torch
    m, n, k = 37, 29, 300
    Ah = synth.gen(m, k, 33, synth.STREAM_A, synth.WIDE_F64)
    Bh = synth.gen(k, n, 33, synth.STREAM_B, synth.WIDE_F64)
    _, A = device_matrix(m, k, 33, synth.STREAM_A, synth.WIDE_F64)
    _, B = device_matrix(k, n, 33, synth.STREAM_B, synth.WIDE_F64)
    C = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    plan = ob_plan(m, n, k, slices)
    assert plan.p_k == 1
    assert run_gemm(cm, m, n, k, A, k, B, n, C, n, plan=plan) == 0
    got = C.cpu().numpy()
    e = np.array([math.frexp(float(np.max(np.abs(Ah[i]))))[1] for i in range(m)])
    f = np.array([math.frexp(float(np.max(np.abs(Bh[:, j]))))[1] for j in range(n)])

    def digits(X):  # entries already scaled into (-1, 1)
        out = []
        for _ in range(slices):
            y = X * 256.0
            d = np.rint(y)
            X = y - d
            assert np.all(np.abs(d) <= (256 if not out else 128))
            out.append(d.astype(np.int64))
        return out

    Ad = digits(np.ldexp(Ah, -e[:, None]))
    Bd = digits(np.ldexp(Bh, -f[None, :]))
    pairs = [(u, v) for u in range(slices) for v in range(slices) if u + v <= slices - 1]
    rounds = -(-k // 32)
    P = {uv: np.zeros((m, n), dtype=np.int64) for uv in pairs}
    mag = np.zeros((m, n))
    for r in range(rounds):
        ks = slice(32 * r, min(k, 32 * r + 32))
        diag = np.zeros((slices, m, n), dtype=np.int64)
        for (u, v) in pairs:
            p = Ad[u][:, ks] @ Bd[v][ks, :]
            P[(u, v)] += p
            diag[u + v] += p
        assert np.all(np.abs(diag) < 2 ** 24)   # the fp32 sums of a round are exact
        for d in range(slices):
            mag += np.abs(diag[d]) * 2.0 ** (-8 * (d + 2))
    worst = 0.0
    for i in range(m):
        for j in range(n):
            S = sum(int(p[i, j]) << (8 * (2 * slices - u - v - 2)) for (u, v), p in P.items())
            sh = int(e[i] + f[j]) - 16 * slices
            ref = S * 2 ** sh if sh >= 0 else S / 2 ** (-sh)
            tol = (slices * rounds + 1) * 2.0 ** -53 * math.ldexp(mag[i, j], int(e[i] + f[j]))
            tol += 0.5 * math.ulp(ref)
            assert abs(got[i, j] - ref) <= tol, (i, j, got[i, j], ref, tol)
            if ref != 0.0:
                worst = max(worst, abs(got[i, j] - ref) / math.ulp(ref))
    log(f"  ozaki_bf16 s={slices}: worst {worst:.2f} ulp from the rounded exact truncated sum")
