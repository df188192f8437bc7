"""Pins for the oracle's leverage scores (Section 6) and the learned-value
distortion loss and gradient (extension; closed-form expectation)."""

import numpy as np
import pytest

import oracle as O

from test_oracle_sketch import injective_seed


def _rng(s):
    return np.random.default_rng(s)


def test_exact_leverage_properties():
    g = _rng(0)
    A = g.standard_normal((300, 6)) * (1 + g.pareto(1.5, size=300))[:, None]
    u = O.leverage_exact(A)
    assert np.all(u >= -1e-15) and np.all(u <= 1 + 1e-12)
    assert u.sum() == pytest.approx(6.0, abs=1e-10)  # trace of the projection = rank
    P = A @ np.linalg.pinv(A)  # projection onto the column space (library)
    assert np.allclose(u, np.diag(P), atol=1e-12)


def test_identity_projection_gives_row_norms_of_A_Rinv():
    A = _rng(1).standard_normal((500, 5))
    R = O.sketch_r(A, 3, 100)
    u1 = O.leverage_approx(A, 3, 100, np.eye(5), R=R)
    M = A @ np.linalg.inv(R)
    assert np.allclose(u1, (M * M).sum(axis=1), rtol=1e-10)


def test_leverage_sandwich():
    # A R^{-1} = U Sigma V^T with U a basis of C(A): u'_i / u_i lies in
    # [sigma_min^2, sigma_max^2] (the constant-factor guarantee of Section 6)
    g = _rng(2)
    A = g.standard_normal((800, 6)) * (1 + g.pareto(1.5, size=800))[:, None]
    R = O.sketch_r(A, 7, 200)
    u = O.leverage_exact(A)
    u1 = O.leverage_approx(A, 7, 200, np.eye(6), R=R)
    sv = np.linalg.svd(A @ np.linalg.inv(R), compute_uv=False)
    ratio = u1 / u
    assert ratio.min() >= sv.min() ** 2 * (1 - 1e-10)
    assert ratio.max() <= sv.max() ** 2 * (1 + 1e-10)


def test_perfect_hashing_gives_exact_leverage():
    n = 10
    A = _rng(3).standard_normal((n, 3))
    seed = injective_seed(n, 2048)
    u1 = O.leverage_approx(A, seed, 2048, np.eye(3))
    assert np.allclose(u1, O.leverage_exact(A), atol=1e-12)


def test_gaussian_projection_is_unbiased():
    A = _rng(4).standard_normal((200, 8))
    R = O.sketch_r(A, 1, 64)
    k, K = 4, 600
    est = np.mean([O.leverage_approx(A, 1, 64, _rng(100 + j).standard_normal((8, k)) / np.sqrt(k), R=R)
                   for j in range(K)], axis=0)
    ref = O.leverage_approx(A, 1, 64, np.eye(8), R=R)
    assert np.allclose(est, ref, rtol=0.15)


# ------------------------------------------------------------ learned values
def test_gradient_matches_finite_differences():
    n, d, t = 8, 3, 4
    A = _rng(5).standard_normal((n, d))
    w = _rng(6).standard_normal(n)
    L, g = O.distortion_grad(A, 2, t, w)
    assert L == pytest.approx(O.distortion_loss(A, 2, t, w), rel=1e-12)
    h = 1e-5
    fd = np.array([(O.distortion_loss(A, 2, t, w + h * e) - O.distortion_loss(A, 2, t, w - h * e)) / (2 * h)
                   for e in np.eye(n)])
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_gradient_symmetries():
    A = _rng(7).standard_normal((40, 4))
    w = _rng(8).standard_normal(40)
    L1, g1 = O.distortion_grad(A, 3, 6, w)
    L2, g2 = O.distortion_grad(A, 3, 6, -w)
    assert L1 == pytest.approx(L2, rel=1e-13)
    assert np.allclose(g1, -g2, rtol=1e-12)
    # directional derivative along w: 4 <Y^T Y, Y^T Y - A^T A>
    Y = O.sketch_dense(A, 3, 6, w)
    P = Y.T @ Y
    assert g1 @ w == pytest.approx(4 * np.sum(P * (P - A.T @ A)), rel=1e-11)


def test_perfect_hashing_with_signs_has_zero_distortion():
    n = 9
    A = _rng(9).standard_normal((n, 3))
    seed = injective_seed(n, 4096)
    _, s = O.bucket_and_sign(seed, n, 4096)
    L, g = O.distortion_grad(A, seed, 4096, s.astype(float))
    assert L == pytest.approx(0.0, abs=1e-24)
    assert np.allclose(g, 0.0, atol=1e-12)


def test_expected_plain_distortion_closed_form():
    A = _rng(10).standard_normal((30, 3))
    t, K = 5, 4000
    vals = []
    for seed in range(K):
        _, s = O.bucket_and_sign(seed, 30, t)
        vals.append(O.distortion_loss(A, seed, t, s.astype(float)))
    vals = np.array(vals)
    se = vals.std(ddof=1) / np.sqrt(K)
    assert abs(vals.mean() - O.expected_plain_distortion(A, t)) < 5 * se


def test_adam_first_step_is_lr_times_sign():
    opt = O.Adam(5, lr=0.01)
    g = np.array([3.0, -2.0, 0.5, -1e-3, 7.0])
    w = opt.step(np.zeros(5), g)
    assert np.allclose(w, -0.01 * np.sign(g), rtol=1e-4)
