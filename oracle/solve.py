"""Oracle: sketch-and-solve regression and R-preconditioned iterations.

* :func:`sketch_and_solve` follows the regression theorem of Section 7: sketch
  ``A`` adjoined with ``b`` by ``Phi D``, then minimise ``||Phi D A x - Phi D b||``
  by a QR factorisation of the sketch and ``x~ = R^{-1} Q^T (S b)`` (the
  solve described in the proof of the regression theorem of Section 7.4).
* :func:`lsqr` is the conjugate-gradient type method of Section 7.7
  preconditioned by the triangular factor: the Krylov method runs on ``M = A R^{-1}``, whose
  condition number is at most ``((1+e0)/(1-e0))^2`` when the sketch is an
  ``e0``-embedding, started from an iterate with bounded relative error.
  The Krylov method used is LSQR (Paige and Saunders, ACM TOMS 8(1), 1982),
  written from its published recurrences.
* :func:`richardson` is the simple iterative improvement scheme of Section
  7.6: ``y <- y + R^{-T} A^T (b - A R^{-1} y)`` in the notation where ``R`` is
  the QR factor (the paper's ``R`` denotes its inverse).

Stopping rule (the paper gives none): with ``r = b - A x`` and
``g = R^{-T} A^T r = M^T r``, the error obeys ``||A (x - x*)|| <= ||g|| /
sigma_min(M)`` because ``M^T (b - A x*) = 0``.  Given a lower bound
``sigma_lb`` on ``sigma_min(M)``, ``||g|| <= sigma_lb * sqrt(D / (1 + D)) ||r||``
with ``D = (1 + delta)^2 - 1`` certifies ``||A x - b|| <= (1 + delta)
||A x* - b||`` through the Pythagorean identity.  The oracle evaluates ``r``
and ``g`` explicitly at every iterate rather than from recurrences.
"""

from __future__ import annotations

import math

import numpy as np

from .linalg import apply_qt, check_rank, householder_qr, solve_upper, solve_upper_t
from .operator import MatrixOp
from .sketch import sketch_csr, sketch_dense


def sketch_matrix(op: MatrixOp, seed: int, t: int, w=None) -> np.ndarray:
    """``S A`` for the operator's matrix (float64)."""
    if op.kind == "csr":
        return sketch_csr(op.n, op.d, op.row_ptr, op.col_idx, op.val, seed, t, w)
    return sketch_dense(op.A, seed, t, w)


def sketch_and_solve(A, b, seed: int, t: int, w=None):
    """Returns ``(x~, R, SA, Sb)`` for ``min ||S A x - S b||``."""
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    SA = sketch_matrix(op, seed, t, w)
    Sb = sketch_dense(np.asarray(b, np.float64), seed, t, w)
    Vs, R = householder_qr(SA)
    check_rank(R)
    c = apply_qt(Vs, Sb)[: op.d]
    return solve_upper(R, c), R, SA, Sb


def certificate_threshold(delta: float, sigma_lb: float) -> float:
    D = (1.0 + delta) ** 2 - 1.0
    return sigma_lb * math.sqrt(D / (1.0 + D))


def _certify(op, R, b, x, thr):
    r = b - op.matvec(x)
    g = solve_upper_t(R, op.rmatvec(r))
    rn, gn = float(np.linalg.norm(r)), float(np.linalg.norm(g))
    return gn <= thr * rn, rn, gn


def lsqr(A, b, x0, R, delta: float, sigma_lb: float = 0.5, max_iter: int = 200):
    """Preconditioned LSQR on ``M = A R^{-1}`` started at ``x0``.

    Returns ``(x, iterations, converged, history)`` where ``history`` lists
    ``(||r||, ||M^T r||)`` evaluated explicitly at each iterate."""
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    b = np.asarray(b, np.float64)
    thr = certificate_threshold(delta, sigma_lb)
    x0 = np.asarray(x0, np.float64)
    hist = []
    ok, rn, gn = _certify(op, R, b, x0, thr)
    hist.append((rn, gn))
    if ok:
        return x0.copy(), 0, True, hist
    u = b - op.matvec(x0)
    beta = np.linalg.norm(u)
    u /= beta
    v = solve_upper_t(R, op.rmatvec(u))
    alpha = np.linalg.norm(v)
    v /= alpha
    w = v.copy()
    y = np.zeros(op.d)
    phibar, rhobar = beta, alpha
    for it in range(1, max_iter + 1):
        u = op.matvec(solve_upper(R, v)) - alpha * u
        beta = np.linalg.norm(u)
        if beta > 0:
            u /= beta
        v = solve_upper_t(R, op.rmatvec(u)) - beta * v
        alpha = np.linalg.norm(v)
        if alpha > 0:
            v /= alpha
        rho = math.hypot(rhobar, beta)
        c, s = rhobar / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        y += (phi / rho) * w
        w = v - (theta / rho) * w
        x = x0 + solve_upper(R, y)
        ok, rn, gn = _certify(op, R, b, x, thr)
        hist.append((rn, gn))
        if ok:
            return x, it, True, hist
    return x, max_iter, False, hist


def richardson(A, b, x0, R, delta: float, sigma_lb: float = 0.5, max_iter: int = 500):
    """Simple iterative improvement on ``M = A R^{-1}`` (Section 7.7).

    Returns ``(x, iterations, converged, history)``.  It converges when every
    singular value of ``M`` lies in ``(0, sqrt 2)``; the contraction factor
    per step is ``max_i |1 - sigma_i(M)^2|``."""
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    b = np.asarray(b, np.float64)
    thr = certificate_threshold(delta, sigma_lb)
    x = np.asarray(x0, np.float64).copy()
    hist = []
    for it in range(max_iter + 1):
        r = b - op.matvec(x)
        g = solve_upper_t(R, op.rmatvec(r))
        rn, gn = float(np.linalg.norm(r)), float(np.linalg.norm(g))
        hist.append((rn, gn))
        if gn <= thr * rn:
            return x, it, True, hist
        if it == max_iter:
            break
        x = x + solve_upper(R, g)
    return x, max_iter, False, hist


def lstsq(A, b, seed: int, t: int, delta: float, sigma_lb: float = 0.5, max_iter: int = 200):
    """Sketch-and-solve start, then preconditioned LSQR to ``ratio <= 1+delta``.

    Returns ``(x, x_sketch, R, iterations, converged)``."""
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    xs, R, _, _ = sketch_and_solve(op, b, seed, t)
    x, it, ok, _ = lsqr(op, b, xs, R, delta, sigma_lb, max_iter)
    return x, xs, R, it, ok
