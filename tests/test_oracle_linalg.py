"""Pins for the oracle's dense linear algebra: Householder QR, substitution,
exact least squares (normal equations, Section 7.2) and the residual ratio
(Pythagorean identity, Section 7.2)."""

from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def _rng(s):
    return np.random.default_rng(s)


@pytest.mark.parametrize("m,d", [(5, 5), (40, 7), (300, 20)])
def test_householder_qr_factorises(m, d):
    A = _rng(m).standard_normal((m, d))
    Vs, R = O.householder_qr(A)
    Q = O.thin_q(Vs, m)
    assert np.allclose(Q @ R, A, atol=1e-12)
    assert np.allclose(Q.T @ Q, np.eye(d), atol=1e-12)
    assert np.allclose(R, np.triu(R))
    assert np.all(np.diag(R) >= 0)
    # same R as LAPACK's Householder QR after fixing the signs of the diagonal
    R2 = np.linalg.qr(A, mode="r")
    R2 = np.sign(np.diag(R2))[:, None] * R2
    assert np.allclose(R, R2, atol=1e-11)
    # Q^T applied to a vector matches the explicit Q
    y = _rng(m + 1).standard_normal(m)
    assert np.allclose(O.apply_qt(Vs, y)[:d], Q.T @ y, atol=1e-12)


def test_triangular_solves():
    R = np.triu(_rng(1).standard_normal((9, 9))) + 4 * np.eye(9)
    y = _rng(2).standard_normal(9)
    assert np.allclose(R @ O.solve_upper(R, y), y, atol=1e-12)
    assert np.allclose(R.T @ O.solve_upper_t(R, y), y, atol=1e-12)
    Y = _rng(3).standard_normal((9, 4))
    assert np.allclose(R @ O.solve_upper(R, Y), Y, atol=1e-12)


def _exact_normal_equations(A_int, b_int):
    """Solve A^T A x = A^T b in exact rationals (Gauss-Jordan)."""
    n, d = A_int.shape
    AtA = [[Fraction(int(sum(A_int[k, i] * A_int[k, j] for k in range(n)))) for j in range(d)] for i in range(d)]
    Atb = [Fraction(int(sum(A_int[k, i] * b_int[k] for k in range(n)))) for i in range(d)]
    M = [row + [rhs] for row, rhs in zip(AtA, Atb)]
    for c in range(d):
        p = next(r for r in range(c, d) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for r in range(d):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [M[i][d] for i in range(d)]


@pytest.mark.parametrize("seed,n,d", [(0, 6, 2), (1, 9, 3), (2, 12, 4)])
def test_lstsq_against_exact_rationals(seed, n, d):
    g = _rng(seed)
    A = g.integers(-4, 5, size=(n, d))
    b = g.integers(-6, 7, size=n)
    x_exact = np.array([float(v) for v in _exact_normal_equations(A, b)])
    x = O.lstsq_exact(A.astype(float), b.astype(float))
    assert np.allclose(x, x_exact, rtol=1e-12, atol=1e-12)


def test_lstsq_against_lapack_and_normal_equations():
    A = _rng(5).standard_normal((500, 12))
    b = _rng(6).standard_normal(500)
    x = O.lstsq_exact(A, b)
    x2, *_ = np.linalg.lstsq(A, b, rcond=None)
    assert np.allclose(x, x2, rtol=1e-11, atol=1e-12)
    r = A @ x - b
    # normal equations: A^T (A x* - b) = 0 up to rounding
    assert np.linalg.norm(A.T @ r) <= 1e-12 * np.linalg.norm(A) * np.linalg.norm(r) * 100


def test_residual_ratio_pythagoras():
    A = _rng(7).standard_normal((200, 5))
    b = _rng(8).standard_normal(200)
    xs = O.lstsq_exact(A, b)
    x = xs + 0.1 * _rng(9).standard_normal(5)
    rho = O.residual_ratio(A, b, x, xs)
    direct = np.linalg.norm(A @ x - b) / np.linalg.norm(A @ xs - b)
    assert rho >= 1.0
    assert abs(rho - direct) < 1e-12
    assert O.residual_ratio(A, b, xs, xs) == 1.0


def test_rank_deficiency_detected():
    A = _rng(10).standard_normal((50, 4))
    A[:, 3] = A[:, 0] - 2 * A[:, 1]
    with pytest.raises(O.RankDeficient):
        O.lstsq_exact(A, np.ones(50))
    A[:, 3] = 0.0
    with pytest.raises(O.RankDeficient):
        O.lstsq_exact(A, np.ones(50))
