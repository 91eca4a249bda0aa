"""Modular (Ozaki scheme II) path on the host: the moduli, the operand scale
beta and the planner's schedule, checked against exact integer arithmetic
written out here (no GPU)."""
from math import gcd, prod

import pytest

import paper_1908_09606_amd as cm

OZ2 = cm.COSMA_F64_OZAKI2_I8


def greedy_coprime(count):
    """Pairwise coprime integers taken greedily from 256 downwards."""
    out = []
    x = 256
    while len(out) < count:
        if all(gcd(x, y) == 1 for y in out):
            out.append(x)
        x -= 1
    return out


@pytest.mark.parametrize("nmod", [2, 4, 8, 13, 14, 15, 16])
@pytest.mark.parametrize("k", [1, 2, 63, 64, 65, 1000, 8192, 65536, 1 << 20])
def test_moduli_and_beta(nmod, k):
    rc, beta, mods = cm.cosma_ozaki2_params(k, nmod)
    M = prod(greedy_coprime(nmod))
    if rc != 0:
        # only when the moduli leave no room for a 1-bit operand
        assert 4 * k * 4 > M
        return
    assert mods == greedy_coprime(nmod)
    assert all(2 <= p <= 256 for p in mods)
    assert all(gcd(a, b) == 1 for i, a in enumerate(mods) for b in mods[:i])
    # residues within one half of the modulus fit int8
    assert all(-(p // 2) >= -128 and (p - 1) // 2 <= 127 for p in mods)
    # every |sum_t A'B'| <= k 2^(2 beta) stays within a quarter of M, so the
    # reconstruction's rint(X / M) cannot be off by one
    assert 1 <= beta <= 50
    assert 4 * k * 4 ** beta <= M
    # and beta is not wasteful: at most 2 bits below the largest such value
    # (or at the 50-bit cap under which residues need no correction step)
    assert beta == 50 or 4 * k * 4 ** (beta + 3) > M


def test_invalid_params():
    assert cm.cosma_ozaki2_params(100, 1)[0] == cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_ozaki2_params(100, 17)[0] == cm.COSMA_ERR_INVALID_ARG
    assert cm.cosma_ozaki2_params(0, 14)[0] == cm.COSMA_ERR_INVALID_ARG
    # two moduli (M = 65280) cannot hold k = 2^20 products of 1-bit operands
    assert cm.cosma_ozaki2_params(1 << 20, 2)[0] == cm.COSMA_ERR_INVALID_ARG


def test_beta_grows_with_moduli():
    """Each modulus adds about 8 bits to M, so about 4 bits to beta."""
    betas = [cm.cosma_ozaki2_params(8192, n)[1] for n in range(8, 15)]
    gains = [b - a for a, b in zip(betas, betas[1:])]
    assert all(3 <= g <= 5 for g in gains), betas


@pytest.mark.parametrize("shape", [(8192, 8192, 8192), (300, 257, 1000), (64, 64, 200000),
                                   (2048, 2048, 1 << 20), (1, 1, 1)])
def test_planner_modular(shape):
    m, n, k = shape
    rc, p = cm.cosma_plan_query(m, n, k, OZ2)
    assert rc == 0
    assert (p.tile_m, p.tile_n, p.tile_k) == (256, 128, 64)
    nm = p.slices  # the error contract's choice (tests/test_ozaki_contract.py)
    assert 2 <= nm <= 16 and cm.cosma_ozaki2_params(k, nm)[0] == 0
    assert p.k_split <= 65536 and p.k_split % 64 == 0
    assert p.p_k == -(-k // p.k_split)
    tiles = -(-m // 256) * -(-n // 128)
    assert p.items == tiles * p.p_k * p.slices
    # the schedule's counted I/O respects Theorem 1 for its word (N bytes)
    assert p.q_cu_words >= p.thm1_words * (1 - 1e-12)
    # workspace: residue planes of A and B, one byte per modulus, split and
    # entry of the padded C, then the exponents
    up = lambda x: (x + 255) // 256 * 256
    kp = -(-k // 64) * 64
    rows, cols = -(-m // 256) * 256, -(-n // 128) * 128
    # each row tile's blocks are followed by 1 KiB of padding
    planes = rows // 256 * (kp * 256 + 1024) + cols // 128 * (kp * 128 + 1024)
    ws = up(nm * planes) + up(p.p_k * nm * rows * cols) + up((m + n) * 4)
    assert p.workspace_bytes == ws
    rc, b = cm.cosma_workspace_size(m, n, k, OZ2)
    assert rc == 0 and b == ws


def test_set_moduli_on_plan():
    rc, p = cm.cosma_plan_make(1000, 900, 5000, OZ2, 0, 2)
    assert rc == 0 and p.p_k == 2
    assert cm.cosma_plan_set_slices(p, 14) == 0
    items14 = p.items
    assert cm.cosma_plan_set_slices(p, 16) == 0
    assert p.slices == 16 and p.items == items14 // 14 * 16
    for bad in (1, 17, 0):
        assert cm.cosma_plan_set_slices(p, bad) == cm.COSMA_ERR_INVALID_ARG
    # a split longer than 65536 cannot be forced
    rc, _ = cm.cosma_plan_make(64, 64, 200000, OZ2, 0, 1)
    assert rc == cm.COSMA_ERR_INVALID_ARG
