"""Write wide_spread_8192.txt: the largest spread of the 8192^3 product of
wide-exponent inputs (sign * U[1,2) * 2^e, e uniform in [-20, 20], seed 1,
the benchmark's Ozaki workload).

The spread of entry (i, j) is rho_ij = k 2^(e_i + f_j) / D_ij, with e_i the
frexp exponent of the largest |A_it| of row i (max < 2^e_i), f_j that of
column j of B, and D_ij = sum_t |A_it| |B_tj| from the oracle.  Inputs come
from synth, D only from the oracle.  Run: python tests/golden/make_wide_spread.py
(about a minute on 8 cores).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

M = N = K = 8192
SEED = 1
ROWS = 512


def main():
    B = synth.gen(K, N, SEED, synth.STREAM_B, synth.WIDE_F64)
    _, f = np.frexp(np.abs(B).max(axis=0))
    worst, where = 0.0, None
    for r0 in range(0, M, ROWS):
        A = synth.gen(M, K, SEED, synth.STREAM_A, synth.WIDE_F64, row_idx=np.arange(r0, r0 + ROWS))
        _, e = np.frexp(np.abs(A).max(axis=1))
        _, D = oracle.gemm(A, B)
        rho = np.ldexp(np.full(D.shape, float(K)), e[:, None] + f[None, :]) / D
        i, j = np.unravel_index(int(np.argmax(rho)), rho.shape)
        if rho[i, j] > worst:
            worst, where = float(rho[i, j]), (r0 + int(i), int(j))
        print(f"rows {r0}..{r0 + ROWS}: max so far {worst:.6g} at {where}", flush=True)
    with open(os.path.join(HERE, "wide_spread_8192.txt"), "w") as fh:
        fh.write("# largest spread rho_ij = k 2^(e_i+f_j) / D_ij of the 8192^3 product of\n"
                 "# synth WIDE_F64 inputs, seed 1 (A stream 0, B stream 1); D from the oracle.\n"
                 "# Written by tests/golden/make_wide_spread.py.\n")
        fh.write(f"max_spread {worst!r}\nrow {where[0]}\ncol {where[1]}\n")


if __name__ == "__main__":
    main()
