"""Writes separated_8192_seed0_samples.txt: sampled entries of the CPU oracle's solution of the
separated-spectra workload at m = n = 8192 (seed 0; diagonals U[1,10], 20% 2x2 blocks, strict
upper N(0,1)/sqrt(order), C ~ N(0,1)).  Alg. 4 by the oracle (tile 64, OpenMP over independent
tile updates); no scaling happens on this input (e = 0), so the samples are entries of the unique
solution X of eq. (2).  Only the oracle and the seeded generators are used.

Format: header lines starting with '#', then one line per sample 'i j x' with x as a hexadecimal
float (exact).  The sample: 4096 seeded uniform (i, j) pairs plus the 8 x 8 top-right corner,
the last block the back substitution reaches.

Usage: python tests/golden/make_separated_8192.py [threads]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle                     # noqa: E402
import trsyl_workloads as W       # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "separated_8192_seed0_samples.txt")


def sample_positions(m, n, count=4096, seed=20261203):
    rng = np.random.default_rng(seed)
    ij = [(int(i), int(j)) for i, j in zip(rng.integers(0, m, count), rng.integers(0, n, count))]
    ij += [(i, j) for i in range(8) for j in range(n - 8, n)]
    return ij


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    m = n = 8192
    oracle.build(force=False)
    A, B, C = W.config_separated(0, m, n)
    t0 = time.time()
    Y, e, rc = oracle.drsylv(A, B, C, 64, threads=threads)
    dt = time.time() - t0
    assert e == 0 and rc == 0 and np.isfinite(Y).all()
    with open(OUT, "w") as fh:
        fh.write(f"# oracle Alg. 4 (tile 64, {threads} threads, {dt:.0f} s) on config_separated(0, 8192, 8192)\n")
        fh.write(f"# e = {e}, max|Y| = {float(np.abs(Y).max()).hex()}, ||Y||_F = {float(np.linalg.norm(Y)).hex()}\n")
        for i, j in sample_positions(m, n):
            fh.write(f"{i} {j} {float(Y[i, j]).hex()}\n")
    print(f"wrote {OUT} ({dt:.0f} s)")


if __name__ == "__main__":
    main()
