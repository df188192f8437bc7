"""Writes lowrank_planted_n65536_r32.txt: the best rank-k error Delta_k of the
planted low-rank sparse workload (n = 65536, rank-32 factors, about 10 million
nonzeros, trial 0), k = 32, from the oracle alone.

Run from the repository root:  python tests/golden/make_lowrank_golden.py
"""

import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    k = 32
    A = W.planted_lowrank_sparse()
    t0 = time.time()
    dk = oracle.best_rank_k_error(A, k)
    fro = float(np.sqrt(np.sum(A.val.astype(np.float64) ** 2)))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lowrank_planted_n65536_r32.txt")
    with open(out, "w") as f:
        f.write("# Best rank-k Frobenius error of the planted low-rank sparse workload\n")
        f.write("# (workloads.planted_lowrank_sparse(): n = 65536, rank-32 factors of density 0.0085,\n")
        f.write("# N(0, 0.01^2) noise on the pattern, float32 values, trial 0), from\n")
        f.write("# oracle.best_rank_k_error (||A||_F^2 minus the top-k squared singular values).\n")
        f.write("# Written by tests/golden/make_lowrank_golden.py.\n")
        f.write(f"n: {A.n}\nnnz: {A.nnz}\nk: {k}\n")
        f.write(f"fro_norm: {fro!r}\ndelta_k: {dk!r}\n")
    print(f"delta_k {dk!r} fro {fro!r} ({time.time() - t0:.1f} s)")


if __name__ == "__main__":
    main()
