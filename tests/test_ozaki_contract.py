"""Error contract of the Ozaki dtypes (host only).

The planner reports, per plan, err_scaled (E: bound per unit
k 2^(e_i + f_j) from the finite number of slices or moduli), err_rounding
(G: bound per unit D_ij from binary64 rounding) and spread_limit.  The
constants are pinned here against brute force on the scalar expansions the
methods define (Ozaki et al. 2012 digit splitting; Ozaki scheme II integer
scaling), written out independently of the library with exact rational
arithmetic: every per-term error found must stay within E, and the
adversarial inputs must come close to it, so that a wrong or vacuous
constant fails."""
import math
from fractions import Fraction

import numpy as np
import pytest

import paper_1908_09606_amd as cm

OZ, OZ2, OZB = cm.COSMA_F64_OZAKI_I8, cm.COSMA_F64_OZAKI2_I8, cm.COSMA_F64_OZAKI_BF16


def plan_for(dtype, k, slices):
    item = {OZ: 8192, OZ2: 65536}.get(dtype, k)  # longest reduction per work item
    rc, p = cm.cosma_plan_make(64, 64, k, dtype, 0, -(-k // item))
    assert rc == 0
    assert cm.cosma_plan_set_slices(p, slices) == 0
    return p


def trunc_digits(x, s):
    """x in (-1, 1): d_u = trunc(2^7 r), r <- 2^7 r - d_u (exact rationals)."""
    r, out = Fraction(x), []
    for _ in range(s):
        y = r * 128
        d = math.trunc(y)
        out.append(Fraction(d, 128 ** (len(out) + 1)))
        r = y - d
    return out


def round_digits(x, s):
    """x in (-1, 1): d_u = rint(2^8 r) (ties to even), r <- 2^8 r - d_u."""
    r, out = Fraction(x), []
    for _ in range(s):
        y = r * 256
        d = round(y)  # Python rounds half to even, as rint does
        out.append(Fraction(d, 256 ** (len(out) + 1)))
        r = y - d
    return out


def triangular(X, Y, s):
    return sum(X[u] * Y[v] for u in range(s) for v in range(s) if (u + 1) + (v + 1) <= s + 1)


def samples(rng, count):
    xs = list(rng.uniform(-1, 1, count))
    xs += [1 - 2.0 ** -52, -(1 - 2.0 ** -52), 0.5, 2.0 ** -30, -(2.0 ** -9) * 1.0000001]
    xs += [float(v) for v in rng.uniform(0.5, 1, 8) * 2.0 ** -rng.integers(0, 40, 8)]
    return xs


@pytest.mark.parametrize("s", [1, 2, 3, 5, 7, 8])
def test_int8_digit_term_error_within_err_scaled(s):
    E = plan_for(OZ, 1000, s).err_scaled
    assert E == pytest.approx((s + 1) * 2.0 ** (-7 * s), rel=1e-12)
    rng = np.random.default_rng(s)
    xs = samples(rng, 40)
    worst = Fraction(0)
    for x in xs:
        X = trunc_digits(x, s)
        # truncation digits share the sign of x and never exceed it in sum
        assert sum(abs(v) for v in X) <= abs(Fraction(x))
        for y in xs[:20] + xs[40:]:
            err = abs(Fraction(x) * Fraction(y) - triangular(X, trunc_digits(y, s), s))
            worst = max(worst, err)
    assert float(worst) <= E
    # all-127 digits make every dropped product and residual add up (while
    # the 7s digit bits fit in a binary64 significand)
    if 7 * s <= 52:
        assert float(worst) >= 0.7 * E


@pytest.mark.parametrize("s", [1, 2, 4, 6, 7, 8])
def test_bf16_digit_term_error_within_err_scaled(s):
    E = plan_for(OZB, 1000, s).err_scaled
    assert E == pytest.approx((0.251 * s + 0.751) * 2.0 ** (-8 * s), rel=1e-12)
    rng = np.random.default_rng(100 + s)
    xs = samples(rng, 40)
    # digits just below a rounding tie push every residual to 1/2
    half = sum(Fraction(1, 2) * Fraction(1, 256 ** u) for u in range(1, s + 2))
    xs += [float(half - Fraction(1, 2 ** 60)), -float(half - Fraction(1, 2 ** 60))]
    worst = Fraction(0)
    for x in xs:
        X = round_digits(x, s)
        assert sum(abs(v) for v in X) <= Fraction(3004, 1000) * abs(Fraction(x))
        for y in xs[:20] + xs[40:]:
            err = abs(Fraction(x) * Fraction(y) - triangular(X, round_digits(y, s), s))
            worst = max(worst, err)
    assert float(worst) <= E
    if 8 * s <= 52:
        assert float(worst) >= 0.3 * E


@pytest.mark.parametrize("k,nmod", [(64, 8), (2048, 14), (8192, 15), (1 << 20, 16)])
def test_modular_operand_rounding_within_err_scaled(k, nmod):
    rc, beta, _ = cm.cosma_ozaki2_params(k, nmod)
    assert rc == 0
    E = plan_for(OZ2, k, nmod).err_scaled
    assert E == pytest.approx(2.0 ** -beta, rel=1e-12)
    rng = np.random.default_rng(k)
    # scaled operands in (-1, 1): a~ = rint(a 2^beta) 2^-beta
    vals = list(rng.uniform(-1, 1, 60)) + [1 - 2.0 ** -52, (0.5 + 2.0 ** -beta) - 2.0 ** -53]
    vals += [(2 * j + 1) * 2.0 ** (-beta - 1) for j in range(3)]  # ties
    worst = Fraction(0)
    for a in vals:
        at = Fraction(round(Fraction(a) * 2 ** beta), 2 ** beta)
        assert abs(at) <= 1
        for b in vals[:20] + vals[60:]:
            bt = Fraction(round(Fraction(b) * 2 ** beta), 2 ** beta)
            worst = max(worst, abs(Fraction(a) * Fraction(b) - at * bt))
    assert float(worst) <= E
    assert float(worst) >= 0.5 * E


def test_spread_limit_definition():
    for dtype, s in ((OZ, 7), (OZ2, 14), (OZB, 6)):
        for k in (100, 2048, 8192):
            p = plan_for(dtype, k, s)
            lim = (3 * k * 2.0 ** -53 - p.err_rounding) / p.err_scaled
            assert p.spread_limit == pytest.approx(max(lim, 0.0), rel=1e-12)
            assert p.err_rounding < 0.05 * 3 * k * 2.0 ** -53 or dtype == OZB


def test_planner_picks_smallest_count_meeting_the_target():
    rc, target = cm.cosma_get_ozaki_spread()
    assert rc == 0 and target == 2048.0
    for dtype, lo, hi in ((OZ, 1, 8), (OZ2, 2, 16), (OZB, 1, 8)):
        for k in (64, 512, 2048, 8192, 65536, 1 << 20):
            rc, p = cm.cosma_plan_query(1024, 1024, k, dtype)
            assert rc == 0
            s = p.slices
            qs = [q for q in range(lo, hi + 1)
                  if dtype != OZ2 or cm.cosma_ozaki2_params(k, q)[0] == 0]
            ok = [q for q in qs if plan_for(dtype, k, q).spread_limit >= target]
            if ok:
                assert s == ok[0], (dtype, k, s, ok)
                assert p.spread_limit >= target
            else:
                Es = {q: plan_for(dtype, k, q).err_scaled for q in qs}
                assert Es[s] == min(Es.values()) and s == min(q for q in Es if Es[q] == Es[s])


def test_more_slices_only_tighten_the_bound():
    for dtype, lo, hi in ((OZ, 1, 8), (OZB, 1, 8)):
        E = [plan_for(dtype, 4096, s).err_scaled for s in range(lo, hi + 1)]
        assert all(a > b for a, b in zip(E, E[1:]))
    valid = [s for s in range(2, 17) if cm.cosma_ozaki2_params(4096, s)[0] == 0]
    assert valid == list(range(valid[0], 17)) and valid[0] > 2
    rc, p = cm.cosma_plan_make(64, 64, 4096, OZ2, 0, 1)
    assert cm.cosma_plan_set_slices(p, valid[0] - 1) == cm.COSMA_ERR_INVALID_ARG
    E2 = [plan_for(OZ2, 4096, s).err_scaled for s in valid]
    assert all(a >= b for a, b in zip(E2, E2[1:]))


def test_set_spread_changes_the_choice_and_is_validated():
    rc, p0 = cm.cosma_plan_query(2048, 2048, 8192, OZ)
    assert rc == 0
    try:
        assert cm.cosma_set_ozaki_spread(100.0) == 0
        rc, p1 = cm.cosma_plan_query(2048, 2048, 8192, OZ)
        assert rc == 0 and p1.slices < p0.slices and p1.spread_limit >= 100.0
        assert cm.cosma_set_ozaki_spread(0.5) == cm.COSMA_ERR_INVALID_ARG
        assert cm.cosma_set_ozaki_spread(float("nan")) == cm.COSMA_ERR_INVALID_ARG
        assert cm.cosma_get_ozaki_spread() == (0, 100.0)
    finally:
        assert cm.cosma_set_ozaki_spread(2048.0) == 0
    rc, p2 = cm.cosma_plan_query(2048, 2048, 8192, OZ)
    assert p2.slices == p0.slices


def test_native_dtypes_carry_no_contract_fields():
    for dtype in (cm.COSMA_F64, cm.COSMA_F32, cm.COSMA_F32_BF16X3):
        rc, p = cm.cosma_plan_query(512, 512, 512, dtype)
        assert rc == 0 and p.err_scaled == 0 and p.err_rounding == 0 and p.spread_limit == 0


def _golden_spread():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "wide_spread_8192.txt")
    with open(path) as fh:
        for line in fh:
            if line.startswith("max_spread"):
                return float(line.split()[1])
    raise AssertionError("no max_spread line")


def test_benchmark_ozaki_plans_cover_their_data():
    """The 8192^3 wide-exponent benchmark product: every Ozaki plan's
    spread_limit covers the largest spread of that data (written by
    tests/golden/make_wide_spread.py from the oracle's D)."""
    worst = _golden_spread()
    assert 1000 < worst < 1e5
    for dtype in (OZ, OZ2, OZB):
        rc, p = cm.cosma_plan_query(8192, 8192, 8192, dtype)
        assert rc == 0
        assert p.spread_limit >= worst, (dtype, p.slices, p.spread_limit, worst)
