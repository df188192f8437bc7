"""Oracle: small dense linear algebra in float64, written out plainly.

* Householder QR (the paper leaves the QR variant open; the regression
  theorem of Section 7.4 solves the sketched problem through a QR
  factorisation of the sketch and ``R^{-1} Q^T S B``).  The ``R`` returned has
  a non-negative diagonal.
* Triangular solves by substitution.
* Exact least squares ``x* = A^- b`` (Introduction; for full column rank the
  minimiser of ``||A x - b||``), via Householder QR of the whole ``A``.
* The residual ratio ``||A x - b|| / ||A x* - b||`` computed through the
  Pythagorean identity of the normal equations (the Pythagorean theorem and
  normal-equations facts of Section 7.2):
  ``||A x - b||^2 = ||A (x - x*)||^2 + ||A x* - b||^2``.
"""

from __future__ import annotations

import numpy as np


class RankDeficient(ValueError):
    """The factor has a diagonal entry too small relative to the largest."""


def householder_qr(M: np.ndarray):
    """Householder QR of an ``m x d`` matrix, ``m >= d``.

    Returns ``(V, R)``: ``V`` the list of unit Householder vectors (``V[k]``
    acts on rows ``k..m-1``) and ``R`` the ``d x d`` upper-triangular factor
    with ``R[k,k] >= 0``; ``Q^T = D H_{d-1} ... H_0`` with ``H_k = I - 2 v v^T``
    and ``D`` the diagonal of signs that makes ``R``'s diagonal non-negative.
    """
    W = np.array(M, dtype=np.float64, copy=True)
    m, d = W.shape
    if m < d:
        raise ValueError("need at least as many rows as columns")
    V = []
    for k in range(d):
        x = W[k:, k]
        normx = np.sqrt(np.dot(x, x))
        if normx == 0.0:
            V.append(None)
            continue
        alpha = -normx if x[0] >= 0 else normx
        v = x.copy()
        v[0] -= alpha
        v /= np.sqrt(np.dot(v, v))
        W[k:, k:] -= 2.0 * np.outer(v, v @ W[k:, k:])
        V.append(v)
    R = np.triu(W[:d, :d])
    signs = np.where(np.diag(R) < 0, -1.0, 1.0)
    return (V, signs), signs[:, None] * R


def apply_qt(Vs, y: np.ndarray) -> np.ndarray:
    """``Q^T y`` (first ``d`` entries are the coordinates in ``Q``'s columns)."""
    V, signs = Vs
    z = np.array(y, dtype=np.float64, copy=True)
    for k, v in enumerate(V):
        if v is not None:
            z[k:] -= 2.0 * v * np.dot(v, z[k:])
    z[: len(signs)] *= signs if z.ndim == 1 else signs[:, None]
    return z


def thin_q(Vs, m: int) -> np.ndarray:
    """The ``m x d`` matrix ``Q`` with orthonormal columns."""
    V, signs = Vs
    d = len(signs)
    Q = np.zeros((m, d))
    Q[np.arange(d), np.arange(d)] = signs
    for k in range(d - 1, -1, -1):
        v = V[k]
        if v is not None:
            Q[k:, :] -= 2.0 * np.outer(v, v @ Q[k:, :])
    return Q


def check_rank(R: np.ndarray, rtol: float | None = None) -> None:
    """Raise :class:`RankDeficient` if ``|R_kk| <= rtol * max |R_jj|``
    (default ``rtol = d * 2^-52``)."""
    diag = np.abs(np.diag(R))
    d = len(diag)
    tol = (d * np.finfo(np.float64).eps if rtol is None else rtol) * (diag.max() if d else 0.0)
    if d == 0 or diag.min() <= tol:
        raise RankDeficient("triangular factor is numerically singular")


def solve_upper(R: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Back substitution for ``R x = y``, ``R`` upper triangular."""
    d = R.shape[0]
    x = np.array(y, dtype=np.float64, copy=True)
    for k in range(d - 1, -1, -1):
        x[k] = (x[k] - np.dot(R[k, k + 1:], x[k + 1:])) / R[k, k]
    return x


def solve_upper_t(R: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Forward substitution for ``R^T x = y``, ``R`` upper triangular."""
    d = R.shape[0]
    x = np.array(y, dtype=np.float64, copy=True)
    for k in range(d):
        x[k] = (x[k] - np.dot(R[:k, k], x[:k])) / R[k, k]
    return x


def lstsq_exact(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """``x* = argmin ||A x - b||`` for dense full-column-rank ``A``."""
    A = np.asarray(A, dtype=np.float64)
    Vs, R = householder_qr(A)
    check_rank(R)
    c = apply_qt(Vs, b)[: A.shape[1]]
    return solve_upper(R, c)


def residual_ratio(A: np.ndarray, b: np.ndarray, x: np.ndarray, xstar: np.ndarray) -> float:
    """``||A x - b|| / ||A x* - b||`` via the Pythagorean identity (no
    cancellation between two nearly equal norms)."""
    A = np.asarray(A, dtype=np.float64)
    e = A @ (np.asarray(x, np.float64) - xstar)
    rstar = A @ xstar - b
    return float(np.sqrt(1.0 + np.dot(e, e) / np.dot(rstar, rstar)))
