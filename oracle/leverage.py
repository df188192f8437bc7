"""Oracle: leverage scores (Introduction and Section 3 definitions; the
approximation theorem of Section 6).

* Exact: ``u_i = ||U[i, :]||^2`` for ``U`` an orthonormal basis of the column
  space of ``A`` (here the thin ``Q`` of a Householder QR of ``A``).
* Approximate: sketch ``A`` with ``S``, compute ``R`` with ``S A R^{-1}``
  orthonormal (QR of the sketch), draw a ``d x k`` Gaussian ``Pi2``, form
  ``T = R^{-1} Pi2`` and return the squared row norms of ``A T``.  The paper
  gives no scaling for ``Pi2``; entries N(0, 1/k) make ``E ||z^T Pi2||^2 =
  ||z||^2``.  ``Pi2`` is an input (drawn by the caller).
"""

from __future__ import annotations

import numpy as np

from .linalg import check_rank, householder_qr, solve_upper, thin_q
from .operator import MatrixOp
from .solve import sketch_matrix


def leverage_exact(A) -> np.ndarray:
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    Ad = op.dense()
    Vs, R = householder_qr(Ad)
    check_rank(R)
    Q = thin_q(Vs, op.n)
    return (Q * Q).sum(axis=1)


def sketch_r(A, seed: int, t: int) -> np.ndarray:
    """Upper-triangular ``R`` of a QR factorisation of ``S A``."""
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    _, R = householder_qr(sketch_matrix(op, seed, t))
    check_rank(R)
    return R


def leverage_approx(A, seed: int, t: int, Pi2: np.ndarray, R: np.ndarray | None = None) -> np.ndarray:
    """Squared row norms of ``A R^{-1} Pi2``."""
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    if R is None:
        R = sketch_r(op, seed, t)
    T = solve_upper(R, np.asarray(Pi2, np.float64))
    AT = op.matmat(T)
    return (AT * AT).sum(axis=1)
