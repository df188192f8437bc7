"""Pins for the oracle's sketch-and-solve (Section 7 regression theorem) and
its preconditioned iterations (Section 7.7)."""

import numpy as np
import pytest

import oracle as O
import workloads as W

from test_oracle_sketch import injective_seed


def _rng(s):
    return np.random.default_rng(s)


def _tall(seed, n, d, heavy=False):
    g = _rng(seed)
    A = g.standard_normal((n, d))
    if heavy:
        A *= (1.0 + g.pareto(1.5, size=n))[:, None]
    b = A @ g.standard_normal(d) + 0.1 * g.standard_normal(n)
    return A, b


def test_sketch_and_solve_is_lstsq_of_sketch():
    A, b = _tall(0, 2000, 6)
    x, R, SA, Sb = O.sketch_and_solve(A, b, 77, 200)
    x2, *_ = np.linalg.lstsq(SA, Sb, rcond=None)
    assert np.allclose(x, x2, rtol=1e-10, atol=1e-12)
    assert np.allclose(R.T @ R, SA.T @ SA, rtol=1e-10, atol=1e-9)


def test_perfect_hashing_gives_exact_solution():
    n, d = 10, 3
    A, b = _tall(1, n, d)
    seed = injective_seed(n, 512)
    x, *_ = O.sketch_and_solve(A, b, seed, 512)
    xs = O.lstsq_exact(A, b)
    assert np.allclose(x, xs, rtol=1e-12, atol=1e-12)
    assert O.residual_ratio(A, b, x, xs) == pytest.approx(1.0, abs=1e-14)


def test_small_workload_sketch_and_solve_ratio():
    A, b, _ = W.lstsq_small()
    op = O.MatrixOp(A)
    x, *_ = O.sketch_and_solve(op, b, W.sketch_seed(0), 4000)
    xs = O.lstsq_exact(op.dense(), b)
    rho = O.residual_ratio(op.dense(), b, x, xs)
    assert 1.0 <= rho < 1.05


def _svals(A, R):
    M = A @ np.linalg.inv(R)
    return np.linalg.svd(M, compute_uv=False)


def test_lsqr_converges_to_exact_and_meets_cg_bound():
    A, b = _tall(2, 3000, 10, heavy=True)
    xs = O.lstsq_exact(A, b)
    x0, R, _, _ = O.sketch_and_solve(A, b, 5, 400)
    sv = _svals(A, R)
    assert sv.min() > 0.5  # the certificate's default lower bound holds here
    x, it, ok, hist = O.lsqr(A, b, x0, R, delta=1e-12, max_iter=100)
    assert ok
    rho = O.residual_ratio(A, b, x, xs)
    assert rho - 1.0 <= 1e-12
    # Krylov rate on M = A R^{-1}: ||A(x_m - x*)|| <= 2 q^m ||A(x_0 - x*)||,
    # q = (k - 1)/(k + 1), k = sigma_max/sigma_min (textbook CG/CGLS bound)
    kappa = sv.max() / sv.min()
    q = (kappa - 1) / (kappa + 1)
    rstar2 = np.sum((A @ xs - b) ** 2)
    e = [np.sqrt(max(rn * rn - rstar2, 0.0)) for rn, _ in hist]
    for m in range(1, len(e)):
        if e[m] > 1e-9 * np.sqrt(rstar2):  # above rounding level
            assert e[m] <= 2 * q ** m * e[0] * (1 + 1e-6)


def test_lsqr_and_richardson_agree():
    A, b = _tall(3, 2500, 8)
    xs = O.lstsq_exact(A, b)
    x0, R, _, _ = O.sketch_and_solve(A, b, 9, 600)
    sv = _svals(A, R)
    assert np.max(np.abs(1 - sv ** 2)) < 1.0  # Richardson contracts
    x1, _, ok1, _ = O.lsqr(A, b, x0, R, delta=1e-12)
    x2, _, ok2, _ = O.richardson(A, b, x0, R, delta=1e-12)
    assert ok1 and ok2
    assert np.allclose(x1, xs, rtol=1e-6, atol=1e-9)
    assert np.allclose(x2, xs, rtol=1e-6, atol=1e-9)


def test_richardson_contraction_factor():
    # one step of oracle.richardson contracts the error in y = R x by exactly
    # |1 - sigma^2| along the singular direction of M = A R^-1 with value
    # sigma (Section 7.7; the factor exceeds 1 once some singular value of M
    # passes sqrt(2)).  M = U diag(sig) is built with known singular values
    # and A = M R for an arbitrary well-conditioned upper-triangular R, so a
    # step through R^-T where R^-1 is meant (or the reverse) fails.
    n, d = 40, 3
    U, _ = np.linalg.qr(_rng(4).standard_normal((n, d)))
    sig = np.array([0.9, 1.0, 1.2])
    M = U * sig
    R = np.triu(_rng(8).standard_normal((d, d))) + 3.0 * np.eye(d)
    A = M @ R
    b = _rng(5).standard_normal(n)
    xs = O.lstsq_exact(A, b)
    for j, s in enumerate(sig):
        x = xs + np.linalg.solve(R, np.eye(d)[j])  # error e_j in y = R x
        x1, it, ok, _ = O.richardson(A, b, x, R, delta=1e-300, max_iter=1)
        assert it == 1 and not ok
        ratio = np.linalg.norm(A @ (x1 - xs)) / np.linalg.norm(A @ (x - xs))
        assert ratio == pytest.approx(abs(1 - s ** 2), rel=1e-9)
        x2, _, _, _ = O.richardson(A, b, x, R, delta=1e-300, max_iter=2)
        ratio2 = np.linalg.norm(A @ (x2 - xs)) / np.linalg.norm(A @ (x - xs))
        assert ratio2 == pytest.approx((1 - s ** 2) ** 2, rel=1e-8)


def test_zero_iterations_when_preconditioner_is_exact():
    n, d = 12, 3
    A, b = _tall(6, n, d)
    seed = injective_seed(n, 1024)
    x0, R, _, _ = O.sketch_and_solve(A, b, seed, 1024)
    x, it, ok, _ = O.lsqr(A, b, x0, R, delta=1e-8)
    assert ok and it == 0


def test_lstsq_driver_on_sparse_input():
    A = W.csr_uniform_rows(12, 5000, 15, 4, dtype=np.float64)
    g = _rng(7)
    b = A.matvec64(g.standard_normal(15)) + 0.01 * g.standard_normal(5000)
    op = O.MatrixOp(A)
    x, xs_sk, R, it, ok = O.lstsq(op, b, 3, 900, delta=1e-10)
    assert ok
    xs = O.lstsq_exact(op.dense(), b)
    assert O.residual_ratio(op.dense(), b, x, xs) - 1 <= 1e-10


@pytest.mark.parametrize("delta", [1e-1, 1e-3, 1e-6])
def test_certificate_is_tight_at_the_smallest_singular_value(delta):
    # The stopping rule certifies ratio <= 1 + delta whenever sigma_min(M) >=
    # sigma_lb (M = A R^-1).  With sigma_min(M) = sigma_lb exactly and the
    # error of x along that singular direction, ||M^T r|| / ||r|| equals the
    # threshold exactly when the ratio equals 1 + delta (Pythagorean identity
    # of the regression residual), so a point just inside is certified and a
    # point just outside is not.
    n, d, slb = 30, 3, 0.5
    U, _ = np.linalg.qr(_rng(21).standard_normal((n, d + 1)))
    sig = np.array([slb, 1.0, 1.3])
    M = U[:, :d] * sig
    R = np.triu(_rng(22).standard_normal((d, d))) + 2.0 * np.eye(d)
    A = M @ R
    rstar = 0.7 * U[:, d]                    # orthogonal to the range of A
    c = _rng(23).standard_normal(d)
    b = U[:, :d] @ c + rstar
    xs = np.linalg.solve(R, c / sig)         # A xs = U c
    for rel, want in ((1 - 1e-7, True), (1 + 1e-7, False)):
        rho = (1 + delta) * rel
        eps = np.linalg.norm(rstar) * np.sqrt(rho ** 2 - 1) / slb
        x0 = xs + np.linalg.solve(R, eps * np.eye(d)[0])
        assert O.residual_ratio(A, b, x0, xs) == pytest.approx(rho, rel=1e-12)
        _, it, ok, _ = O.richardson(A, b, x0, R, delta=delta, sigma_lb=slb, max_iter=0)
        assert it == 0 and ok is want
