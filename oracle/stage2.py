"""Oracle: the second sketch stage ``Pi1 = F S`` (Section 6).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the library never does.

Section 6 replaces the subspace embedding of the leverage-score algorithm by
the product of the sparse embedding ``S`` (``t`` rows) with a dense
Johnson-Lindenstrauss map ``F`` (``m`` rows), and factors ``F S A`` instead of
``S A``; the composition facts of Section 8 say such a product keeps the
embedding property (each factor's distortion multiplies).  The paper takes
``F`` from a fast transform; this project uses a matrix of random signs
scaled by ``1 / sqrt(m)`` (a Johnson-Lindenstrauss map with the same
guarantee), drawn from SplitMix64 like the rest of the randomness:

* entry ``(i, r)`` is ``-1 / sqrt(m)`` when bit ``b(r mod 64)`` of output
  ``i * W + floor(r / 64)`` (``W = ceil(t / 64)``) of the stream
  ``seed ^ 0x7374616765327369`` is set, else ``+1 / sqrt(m)``, with
  ``b(c) = 32 floor(c / 32) + 16 (c mod 2) + 15 - floor((c mod 32) / 2)``
  (a fixed permutation of the word's 64 bits, so every sign is still a fair
  independent bit).

Precision (a convention of this project, not the paper's): ``S A`` enters the
product rounded to float32 and then to bfloat16, each to nearest with ties
to even; ``S b`` enters as given.  Everything else here is float64.
"""

from __future__ import annotations

import numpy as np

from .hashing import splitmix64
from .linalg import apply_qt, check_rank, householder_qr, solve_upper
from .operator import MatrixOp
from .solve import lsqr, sketch_matrix
from .sketch import sketch_dense

STAGE_SALT = 0x7374616765327369


def round_bf16(x) -> np.ndarray:
    """``x`` rounded to float32, then to bfloat16 (nearest, ties to even),
    returned as float64.  Finite inputs only."""
    u = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32)).view(np.uint32).astype(np.uint64)
    # add half an ulp of bfloat16 (0x7FFF) plus the parity bit of the kept part,
    # then truncate the low 16 bits
    r = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bit_of_offset(c):
    """``b(c)``: the bit of a sign word that holds the sign of row offset ``c``
    (0..63) within its 64-row block."""
    c = np.asarray(c)
    return 32 * (c // 32) + 16 * (c % 2) + 15 - (c % 32) // 2


def sign_rows(seed: int, rows, t: int) -> np.ndarray:
    """Rows ``rows`` of ``sqrt(m) F``: entries +1 / -1 (int8), shape
    ``[len(rows), t]``."""
    rows = np.asarray(rows, np.uint64).reshape(-1)
    W = (t + 63) // 64
    idx = rows[:, None] * np.uint64(W) + np.arange(W, dtype=np.uint64)[None, :]
    z = splitmix64(seed ^ STAGE_SALT, idx)
    pos = bit_of_offset(np.arange(64)).astype(np.uint64)
    bits = (z[:, :, None] >> pos[None, None, :]) & np.uint64(1)
    bits = bits.reshape(len(rows), W * 64)[:, :t]
    return np.where(bits == np.uint64(1), -1, 1).astype(np.int8)


def stage_matrix(seed: int, m: int, t: int) -> np.ndarray:
    """``F`` (float64, ``m x t``)."""
    return sign_rows(seed, np.arange(m), t).astype(np.float64) / np.sqrt(m)


def second_stage(SA: np.ndarray, Sb, seed: int, m: int, rows=None):
    """``(F SA, F Sb)`` with ``SA`` rounded as the header says; ``rows``
    restricts the result to those rows of ``F`` (``Sb`` may be None)."""
    SA = np.asarray(SA)
    t = SA.shape[0]
    rows = np.arange(m) if rows is None else np.asarray(rows)
    F = sign_rows(seed, rows, t).astype(np.float64) / np.sqrt(m)
    FSA = F @ round_bf16(SA)
    FSb = None if Sb is None else F @ np.asarray(Sb, np.float64)
    return FSA, FSb


def sketch_and_solve(A, b, seed: int, t: int, m: int):
    """``(x~, R)`` for ``min ||F S A x - F S b||`` (Pi1 = F S), by a Householder
    QR of ``F S A``."""
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    SA = sketch_matrix(op, seed, t)
    Sb = sketch_dense(np.asarray(b, np.float64), seed, t)
    FSA, FSb = second_stage(SA, Sb, seed, m)
    Vs, R = householder_qr(FSA)
    check_rank(R)
    c = apply_qt(Vs, FSb)[: op.d]
    return solve_upper(R, c), R


def lstsq(A, b, seed: int, t: int, m: int, delta: float, sigma_lb: float = 0.5, max_iter: int = 200):
    """Sketch-and-solve through ``Pi1 = F S``, then LSQR preconditioned by the
    R of ``F S A`` to ``ratio <= 1 + delta``.  Returns ``(x, x~, R,
    iterations, converged)``."""
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    xs, R = sketch_and_solve(op, b, seed, t, m)
    x, it, ok, _ = lsqr(op, b, xs, R, delta, sigma_lb, max_iter)
    return x, xs, R, it, ok
