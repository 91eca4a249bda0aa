"""Exact rational brute force for tiny products.  TEST INFRASTRUCTURE ONLY.

C[i][j] = alpha * sum_t A[i][t] * B[t][j] + beta * C0[i][j] over the
rationals (Python ``fractions.Fraction``), the plain definition of the
product of section 2.4 with no rounding at all.  It pins the binary64
oracle: on dyadic inputs whose sums stay within 53 bits the two agree
exactly, and otherwise their difference stays within gamma_k * D.
"""
from __future__ import annotations

from fractions import Fraction


def to_frac_matrix(M):
    return [[Fraction(float(x)) for x in row] for row in M]


def gemm(A, B, alpha=Fraction(1), beta=Fraction(0), C0=None):
    """Exact product of nested lists (or arrays) of floats / Fractions."""
    Af = [[x if isinstance(x, Fraction) else Fraction(float(x)) for x in row] for row in A]
    Bf = [[x if isinstance(x, Fraction) else Fraction(float(x)) for x in row] for row in B]
    m = len(Af)
    k = len(Bf)
    n = len(Bf[0]) if k else (len(C0[0]) if C0 is not None and len(C0) else 0)
    alpha = alpha if isinstance(alpha, Fraction) else Fraction(float(alpha))
    beta = beta if isinstance(beta, Fraction) else Fraction(float(beta))
    out = []
    for i in range(m):
        if k and len(Af[i]) != k:
            raise ValueError("inner dimension mismatch")
        row = []
        for j in range(n):
            s = Fraction(0)
            for t in range(k):
                s += Af[i][t] * Bf[t][j]
            c = alpha * s
            if beta != 0:
                c += beta * Fraction(float(C0[i][j]))
            row.append(c)
        out.append(row)
    return out
