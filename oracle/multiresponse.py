"""Oracle: multiple-response regression ``min_Y ||A Y - B||_F`` by
leverage-score sampling (Section 7, theorem on the generalized-regression
algorithm).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the proof's order:

1. Estimate the leverage scores of ``A`` to constant relative error with the
   algorithm of the Section 6 theorem: ``R`` from a QR of a sparse-embedding
   sketch ``S1 A`` (``t`` rows, stream ``seed``), then the squared row norms of
   ``A R^{-1} Pi2`` with ``Pi2`` the ``d x k_G`` sign matrix of
   :func:`oracle.lowrank.sign_projection`.
2. A leverage-score sampling matrix ``S``: ``t_S`` draws with replacement,
   probabilities proportional to the scores, each drawn row scaled by
   ``1/sqrt(t_S p)`` (:func:`oracle.lowrank.sample_rows`).  The drawn rows and
   their weights are the coreset.
3. ``Y~ = argmin ||S (A Y - B)||_F`` from a QR factorisation ``S A = Q R``:
   ``Y~ = R^{-1} Q^T S B`` (Householder).
"""

from __future__ import annotations

import numpy as np
from .leverage import leverage_approx, sketch_r
from .linalg import apply_qt, check_rank, householder_qr, solve_upper
from .lowrank import sample_rows, sampling_matrix, sign_projection
from .operator import MatrixOp


def multi_response_lstsq(A, B, seed: int, t: int, t_s: int, k_g: int = 32, S=None) -> dict:
    """Returns ``Y`` (``d x d'``) and the scores, draws and counts.  ``S``
    (``t_S x n``) replaces the sampling when given."""
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    n, d = op.n, op.d
    scores = rows = counts = None
    if S is None:
        R1 = sketch_r(op, seed, t)
        scores = leverage_approx(op, seed, t, sign_projection(seed, d, k_g), R=R1)
        rows, counts = sample_rows(scores, t_s, seed)
        S = sampling_matrix(rows, scores, n)
    Ad = op.dense()
    SA = np.asarray(S @ Ad)
    SB = np.asarray(S @ B)
    Vs, R = householder_qr(SA)
    check_rank(R)
    QtSB = np.stack([apply_qt(Vs, SB[:, c])[:d] for c in range(SB.shape[1])], axis=1)
    Y = solve_upper(R, QtSB)
    return {"Y": Y, "scores": scores, "rows": rows, "counts": counts, "R": R}


def residual_fro(A, Y: np.ndarray, B: np.ndarray) -> float:
    """``||A Y - B||_F`` in float64."""
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    return float(np.linalg.norm(op.matmat(np.asarray(Y, np.float64).reshape(op.d, -1)) - B))
