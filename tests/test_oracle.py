"""Pins of the oracle against exact arithmetic and closed forms (CPU only)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import exact

U = 2.0 ** -53
HERE = os.path.dirname(os.path.abspath(__file__))


def _dyadic(rng, shape, scale=8, span=64):
    return rng.integers(-span, span + 1, size=shape).astype(np.float64) / scale


def test_fraction_brute_force_exact_dyadic():
    """All m, n, k in [1, 6]: dyadic inputs keep every sum exact in binary64,
    so the oracle must equal the rational product exactly (pins indices,
    operand order/transposition, alpha and beta)."""
    rng = np.random.default_rng(1)
    for m in range(1, 7):
        for n in range(1, 7):
            for k in range(1, 7):
                A = _dyadic(rng, (m, k))
                B = _dyadic(rng, (k, n))
                C0 = _dyadic(rng, (m, n))
                alpha, beta = 0.75, -1.5
                C, D = oracle.gemm(A, B, alpha, beta, C0, threads=1)
                ref = exact.gemm(A.tolist(), B.tolist(), alpha, beta, C0.tolist())
                for i in range(m):
                    for j in range(n):
                        assert Fraction(C[i, j]) == ref[i][j], (m, n, k, i, j)
                        mag = (abs(Fraction(alpha)) * sum(abs(Fraction(A[i, t]) * Fraction(B[t, j]))
                                                          for t in range(k))
                               + abs(Fraction(beta)) * abs(Fraction(C0[i, j])))
                        assert Fraction(D[i, j]) == mag


def test_fraction_brute_force_rounding_bound():
    """Random binary64 inputs: |C - C_exact| <= gamma_{k+2} * D (standard
    floating-point dot-product bound), checked against exact rationals."""
    rng = np.random.default_rng(2)
    for m, n, k in [(3, 5, 6), (6, 1, 4), (1, 6, 5), (5, 5, 6)]:
        A = rng.uniform(-1, 1, (m, k))
        B = rng.uniform(-1, 1, (k, n))
        C0 = rng.uniform(-1, 1, (m, n))
        alpha, beta = 1.1, 0.3
        C, D = oracle.gemm(A, B, alpha, beta, C0, threads=1)
        ref = exact.gemm(A.tolist(), B.tolist(), alpha, beta, C0.tolist())
        g = (k + 2) * U / (1 - (k + 2) * U)
        for i in range(m):
            for j in range(n):
                assert abs(Fraction(C[i, j]) - ref[i][j]) <= Fraction(g) * Fraction(D[i, j]) * Fraction(1.01)


def test_integer_exact_against_int64():
    rng = np.random.default_rng(3)
    m, n, k = 37, 29, 513
    A = rng.integers(-8, 9, (m, k))
    B = rng.integers(-8, 9, (k, n))
    C, _ = oracle.gemm(A, B, threads=4)
    assert np.array_equal(C, (A @ B).astype(np.float64))


def test_identity_closed_form():
    rng = np.random.default_rng(4)
    m = 33
    B = rng.uniform(-1, 1, (m, 17))
    C0 = rng.uniform(-1, 1, (m, 17))
    alpha, beta = 1.7, -0.9
    C, _ = oracle.gemm(np.eye(m), B, alpha, beta, C0)
    assert np.array_equal(C, alpha * B + beta * C0)


def test_rank1_closed_form():
    rng = np.random.default_rng(5)
    m, n, k = 19, 23, 300
    x = rng.integers(-9, 10, m).astype(np.float64)
    y = rng.integers(-9, 10, n).astype(np.float64)
    A = np.repeat(x[:, None], k, axis=1)
    B = np.repeat(y[None, :], k, axis=0)
    C, _ = oracle.gemm(A, B)
    assert np.array_equal(C, k * np.outer(x, y))


def test_blas_special_cases():
    rng = np.random.default_rng(6)
    m, n, k = 5, 7, 3
    A = rng.uniform(-1, 1, (m, k))
    B = rng.uniform(-1, 1, (k, n))
    C0 = rng.uniform(-1, 1, (m, n))
    # k == 0: C = beta * C0
    C, D = oracle.gemm(np.zeros((m, 0)), np.zeros((0, n)), 2.0, 0.5, C0)
    assert np.array_equal(C, 0.5 * C0) and np.array_equal(D, 0.5 * np.abs(C0))
    # alpha == 0: A and B are not read (NaNs do not propagate)
    An = A.copy(); An[0, 0] = np.nan
    C, _ = oracle.gemm(An, B, 0.0, -2.0, C0)
    assert np.array_equal(C, -2.0 * C0)
    # beta == 0: C0 is not read
    C0n = C0.copy(); C0n[:] = np.nan
    C, _ = oracle.gemm(A, B, 1.0, 0.0, C0n)
    assert np.all(np.isfinite(C))
    # alpha == beta == 0: exact zeros
    C, _ = oracle.gemm(An, B, 0.0, 0.0, C0n)
    assert np.array_equal(C, np.zeros((m, n)))


def test_thread_count_independent():
    rng = np.random.default_rng(7)
    A = rng.uniform(-1, 1, (61, 127))
    B = rng.uniform(-1, 1, (127, 45))
    C1, D1 = oracle.gemm(A, B, threads=1)
    C8, D8 = oracle.gemm(A, B, threads=8)
    assert np.array_equal(C1, C8) and np.array_equal(D1, D8)


def test_sub_block_equals_full():
    """An entry computed from the gathered row of A and column of B equals the
    full product's entry bit for bit (the sampled-verification path)."""
    rng = np.random.default_rng(8)
    A = rng.uniform(-1, 1, (40, 300))
    B = rng.uniform(-1, 1, (300, 50))
    C, D = oracle.gemm(A, B)
    ri, cj = np.array([0, 7, 39]), np.array([3, 49])
    Cs, Ds = oracle.gemm(A[ri], B[:, cj])
    assert np.array_equal(Cs, C[np.ix_(ri, cj)]) and np.array_equal(Ds, D[np.ix_(ri, cj)])


def test_error_metric_injections():
    rng = np.random.default_rng(9)
    A = rng.uniform(-1, 1, (8, 64))
    B = rng.uniform(-1, 1, (64, 8))
    C, D = oracle.gemm(A, B)
    assert oracle.normalised_err(C, C, D) == 0.0
    for rel in (2.0 ** -40, 1e-7, 0.5):
        P = C.copy()
        P[3, 5] += rel * D[3, 5]
        got = oracle.normalised_err(P, C, D)
        assert got == abs(P[3, 5] - C[3, 5]) / D[3, 5]
        assert math.isclose(got, rel, rel_tol=1e-4)
    P = C.copy(); P[0, 0] = np.nan
    assert oracle.normalised_err(P, C, D) == math.inf
    Z = np.zeros((2, 2))
    assert oracle.normalised_err(Z, Z, Z) == 0.0
    assert oracle.normalised_err(Z + 1e-300, Z, Z) == math.inf
    assert oracle.fp64_bound(1024) == 4 * 1024 * 2.0 ** -53
    assert oracle.fp32_bound(1024) == 8 * 1024 * 2.0 ** -24


# ------------------------------------------------------------------ generator
def test_splitmix64_published_vector():
    with open(os.path.join(HERE, "golden", "splitmix64_seed1234567.txt")) as f:
        want = [int(x) for x in f if x.strip() and not x.startswith("#")]
    got = [synth.mix_int(1234567 + i * synth.GAMMA) for i in range(1, 6)]
    assert got == want


def test_generator_vectorised_matches_scalar():
    idx = np.array([0, 1, 2, 12345, 2 ** 40 + 7], dtype=np.uint64)
    h = synth.hashes(42, 1, idx)
    assert [int(x) for x in h] == [synth.hash_int(42, 1, int(i)) for i in idx]


def test_generator_distributions_exact_and_in_range():
    a = synth.gen(64, 96, seed=0, stream=synth.STREAM_A, dist=synth.UNIFORM_F64)
    assert a.dtype == np.float64 and a.min() >= -1.0 and a.max() < 1.0
    assert np.all(((a + 1.0) * 2.0 ** 52) == np.floor((a + 1.0) * 2.0 ** 52))
    f = synth.gen(64, 96, seed=0, stream=synth.STREAM_B, dist=synth.UNIFORM_F32)
    assert f.dtype == np.float32 and f.min() >= -1.0 and f.max() < 1.0
    w = synth.gen(64, 96, seed=3, stream=synth.STREAM_A, dist=synth.WIDE_F64)
    e = np.frexp(np.abs(w))[1] - 1
    assert e.min() >= -20 and e.max() <= 20 and (e.max() - e.min()) > 30
    assert np.any(w < 0) and np.any(w > 0)
    i = synth.gen(50, 50, seed=1, stream=0, dist=synth.INT_F64, param=8)
    assert np.all(i == np.round(i)) and i.min() >= -8 and i.max() <= 8
    sub = synth.gen(64, 96, 0, synth.STREAM_A, synth.UNIFORM_F64, row_idx=[5, 63], col_idx=[0, 95])
    assert np.array_equal(sub, a[np.ix_([5, 63], [0, 95])])


def test_batch_dims_log_uniform():
    d = synth.batch_dims(512, seed=0)
    assert d.shape == (512, 3) and d.min() >= 64 and d.max() <= 4096
    lg = np.log2(d / 64.0)
    assert 2.5 < lg.mean() < 3.5  # log-uniform on [0, 6] has mean 3
