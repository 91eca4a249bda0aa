"""BF16x3 split on the host: what the GPU tests' thresholds can see.

BF16x3 writes each FP32 operand as x = hi + lo + r with hi = bf16_rn(x),
lo = bf16_rn(x - hi) and sums lo*hi + hi*lo + hi*hi in FP32.  Here the split
and the three products are emulated exactly in binary64 (bf16 products are
exact there) on the GPU tests' data, to show that the GPU tests' threshold
2^-18 on the normalised error passes the three-product sum with margin and
fails a product that drops any one of lo*hi, hi*lo or hi*hi, and that the
exact hi + lo data of the GPU test make every product term visible."""
import numpy as np
import pytest

import oracle
import synth

THRESH = 2.0 ** -16


def bf16_rn(x):
    """Round binary32 values to bf16 (nearest, ties to even), as binary32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def split(x):
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_rn(x)
    lo = bf16_rn(x - hi)  # x - hi is exact in binary32
    return hi.astype(np.float64), lo.astype(np.float64)


def test_bf16_rounding_pins():
    assert bf16_rn(np.float32(1.0)) == 1.0
    assert bf16_rn(np.float32(1 + 2.0 ** -8)) == 1.0          # tie to even
    assert bf16_rn(np.float32(1 + 3 * 2.0 ** -8)) == 1 + 2.0 ** -6
    assert bf16_rn(np.float32(1 + 2.0 ** -8 + 2.0 ** -20)) == 1 + 2.0 ** -7


@pytest.mark.parametrize("k", [512, 1024, 3000])
def test_threshold_separates_three_products_from_two(k):
    m, n = 48, 40
    A = synth.gen(m, k, 2, synth.STREAM_A, synth.UNIFORM_F32)
    B = synth.gen(k, n, 2, synth.STREAM_B, synth.UNIFORM_F32)
    ref, D = oracle.gemm(A, B)
    ah, al = split(A)
    bh, bl = split(B)
    terms = {"lo*hi": al @ bh, "hi*lo": ah @ bl, "hi*hi": ah @ bh}
    full = sum(terms.values())
    err_full = oracle.normalised_err(full, ref, D)
    assert err_full < THRESH / 8                      # dropped lo*lo and residues
    assert err_full + 8 * k * 2.0 ** -24 > THRESH   # the 8k 2^-24 gate alone would not see it
    for name, t in terms.items():
        err = oracle.normalised_err(full - t, ref, D)
        assert err > 4 * THRESH, (name, err)


def exact_split_data(rows, cols, seed, stream):
    """Binary32 entries hi + lo with hi = +-(9 + h), h in [0, 6], and
    lo = j 2^-10, |j| <= 31: |hi + lo| stays in [8, 16), where half an ulp
    of bf16 is 2^-5 > |lo|, so the split gives exactly (hi, lo); returned as
    (x, hi, j) with x = hi + j/1024."""
    a = synth.gen(rows, cols, seed, stream, synth.INT_F32, 15).astype(np.int64)
    hi = np.where(a < 0, -1, 1) * (9 + np.abs(a) % 7)
    j = synth.gen(rows, cols, seed + 1000, stream, synth.INT_F32, 31).astype(np.int64)
    x = (hi.astype(np.float64) + j / 1024.0).astype(np.float32)
    return x, hi, j


def exact_three_product(hA, jA, hB, jB):
    """lo*hi + hi*lo + hi*hi in integers (units of 2^-20); lo*lo is dropped."""
    return ((hA @ hB) << 20) + ((hA @ jB) << 10) + ((jA @ hB) << 10)


def test_exact_split_data_is_split_exactly_and_sees_every_term():
    m, n, k = 40, 30, 64
    x, hi, j = exact_split_data(m, k, 3, synth.STREAM_A)
    h, l = split(x)
    assert np.array_equal(h, hi.astype(np.float64)) and np.array_equal(l, j / 1024.0)
    xb, hB, jB = exact_split_data(k, n, 3, synth.STREAM_B)
    want = exact_three_product(hi, j, hB, jB)
    # every partial sum is a multiple of 2^-10 below 2^14: exact in FP32
    bound = np.abs(hi) @ np.abs(hB) * 2 ** 20 + (np.abs(hi) @ np.abs(jB) + np.abs(j) @ np.abs(hB)) * 2 ** 10
    assert bound.max() < 2 ** 34
    # dropping any one product, or keeping lo*lo, changes many entries
    for drop in (((hi @ hB) << 20), ((hi @ jB) << 10), ((j @ hB) << 10), -(j @ jB)):
        assert np.mean(drop != 0) > 0.9
