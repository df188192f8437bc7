"""Pins of the l_p regression oracle (Section 9) against facts that do not
depend on it: the written-out block-diagonal embedding, expectations of the
embedding and of the sampling, brute force over the vertices of the l_1
problem, least squares for p = 2, first-order optimality, the subspace
embedding property, and the (1 + eps) guarantee on small problems."""

import itertools

import numpy as np
import pytest

import oracle.lp as LP
import workloads as W
from oracle.lowrank import SAMPLE_SALT
from oracle.sketch import generalized_S


def _small_csr(n=300, d=6, k=3, seed=4):
    return W.csr_uniform_rows(seed, n, d, k, dtype=np.float64)


def test_block_embedding_matches_written_out_F():
    # F = blockdiag(S, ..., S) with the same S on every block; a short last
    # block takes the first columns of S
    A = _small_csr(n=250)
    Ad = A.to_dense().astype(np.float64)
    seed, q, v, a, w = 0xABC, 3, 4, 2, 100
    S = generalized_S(seed, w, q, v, a)  # t x w
    t = a * q * v
    F = np.zeros((3 * t, 250))
    F[:t, :100] = S
    F[t:2 * t, 100:200] = S
    F[2 * t:, 200:] = S[:, :50]
    assert np.allclose(LP.block_embedding(A, seed, q, v, a, w), F @ Ad, rtol=1e-13, atol=1e-13)
    # one block (w = 0 or w >= n) is the generalized embedding itself
    S1 = generalized_S(seed, 250, q, v, a)
    assert np.allclose(LP.block_embedding(Ad, seed, q, v, a, 0), S1 @ Ad, rtol=1e-13, atol=1e-13)
    assert np.allclose(LP.block_embedding(Ad, seed, q, v, a, 400), S1 @ Ad, rtol=1e-13, atol=1e-13)


def test_block_embedding_preserves_norms_in_expectation():
    # E ||F A x||^2 = ||A x||^2 over the hash seed (every block of F is an
    # embedding with E S^T S = I)
    g = np.random.default_rng(1)
    A = g.standard_normal((120, 4))
    x = g.standard_normal(4)
    ref = np.sum((A @ x) ** 2)
    vals = [np.sum((LP.block_embedding(A, s, 4, 2, 1, 50) @ x) ** 2) for s in range(3000)]
    se = np.std(vals) / np.sqrt(len(vals))
    assert abs(np.mean(vals) - ref) < 4 * se


def test_uniform_streams_are_uniform_and_distinct():
    from scipy.stats import kstest

    u = LP.stream_uniforms(7, SAMPLE_SALT, 20000)
    u2 = LP.stream_uniforms(7, LP.STAGE2_SALT, 20000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert kstest(u, "uniform").pvalue > 1e-3 and kstest(u2, "uniform").pvalue > 1e-3
    assert abs(np.corrcoef(u, u2)[0, 1]) < 0.05


@pytest.mark.parametrize("p", [1.0, 1.5, 3.0])
def test_sampling_is_unbiased_for_the_lp_norm(p):
    # sum over kept rows of w_i^p |y_i|^p has expectation ||y||_p^p, and the
    # expected number of kept rows is sum(prob)
    g = np.random.default_rng(2)
    y = g.standard_normal(400) * np.exp(g.standard_normal(400))
    prob = np.minimum(1.0, 60 * np.abs(y) / np.sum(np.abs(y)))
    ref = np.sum(np.abs(y) ** p)
    est, cnt = [], []
    for s in range(3000):
        rows, wts = LP.bernoulli_sample(prob, p, LP.stream_uniforms(s, SAMPLE_SALT, y.size))
        est.append(np.sum(wts ** p * np.abs(y[rows]) ** p))
        cnt.append(rows.size)
    assert abs(np.mean(est) - ref) < 4 * np.std(est) / np.sqrt(len(est))
    assert abs(np.mean(cnt) - prob.sum()) < 4 * np.std(cnt) / np.sqrt(len(cnt)) + 1e-9
    # rows with probability one are always kept, with weight one
    sure = np.nonzero(prob == 1.0)[0]
    rows, wts = LP.bernoulli_sample(prob, p, LP.stream_uniforms(0, SAMPLE_SALT, y.size))
    assert np.all(np.isin(sure, rows)) and np.all(wts[np.isin(rows, sure)] == 1.0)


def test_l1_solver_matches_vertex_brute_force():
    # an l_1 fit has an optimal vertex: d residuals are zero, so the optimum
    # is the best of the solutions of all nonsingular d x d row subsystems
    g = np.random.default_rng(3)
    for _ in range(5):
        M = g.standard_normal((9, 2))
        y = g.standard_normal(9) + 3 * (g.random(9) < 0.2)
        best = np.inf
        for idx in itertools.combinations(range(9), 2):
            sub = M[list(idx)]
            if abs(np.linalg.det(sub)) < 1e-12:
                continue
            best = min(best, np.sum(np.abs(M @ np.linalg.solve(sub, y[list(idx)]) - y)))
        x = LP.solve_weighted(M, y, np.ones(9), 1.0)
        assert LP.lp_objective(M, y, x, 1.0) == pytest.approx(best, rel=1e-9)


def test_l1_solver_on_a_fit_where_the_default_method_stops_short():
    # the stage-1 fit of a dense n = 12000, d = 150 input with s1 = 1500 (about
    # 1500 x 150), on which HiGHS's default method stops with an unknown
    # status at the oracle's 1e-10 tolerances: the returned x is an optimal
    # vertex (at least d residuals vanish) that no small perturbation improves
    A, b, _ = W.lp_dense(n=12000, d=150)
    seed = 0x3150 + 10
    R = LP.condition(A, seed, 1200, 8, 1)
    lam = np.sqrt(LP.row_norm_estimates(A, R, seed, 32))
    rows, w = LP.bernoulli_sample(np.minimum(1.0, 1500.0 * lam / lam.sum()), 1.0,
                                  LP.stream_uniforms(seed, SAMPLE_SALT, A.shape[0]))
    M, y = A[rows] * w[:, None], b[rows] * w
    x = LP.solve_weighted(M, y, np.ones(rows.size), 1.0)
    r = M @ x - y
    assert np.count_nonzero(np.abs(r) <= 1e-9 * np.max(np.abs(y))) >= M.shape[1]
    f = LP.lp_objective(M, y, x, 1.0)
    g = np.random.default_rng(8)
    for _ in range(20):
        dx = g.standard_normal(x.size) * 1e-6 * np.max(np.abs(x))
        assert LP.lp_objective(M, y, x + dx, 1.0) >= f * (1 - 1e-12)


def test_l2_solver_is_weighted_least_squares():
    g = np.random.default_rng(4)
    M, y, w = g.standard_normal((50, 5)), g.standard_normal(50), g.random(50) + 0.5
    x = LP.solve_weighted(M, y, w, 2.0)
    ref = np.linalg.lstsq(M * w[:, None], y * w, rcond=None)[0]
    assert np.allclose(x, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("p", [1.25, 1.5, 3.0, 4.0])
def test_general_p_solver_is_stationary_and_minimal(p):
    g = np.random.default_rng(5)
    M, y = g.standard_normal((200, 6)), g.standard_normal(200) + g.laplace(size=200)
    w = np.exp(0.3 * g.standard_normal(200))
    x = LP.solve_weighted(M, y, w, p)
    r = w * (M @ x - y)
    grad = (M * w[:, None]).T @ (np.sign(r) * np.abs(r) ** (p - 1))
    scale = np.abs(M * w[:, None]).T @ np.abs(r) ** (p - 1)
    assert np.max(np.abs(grad) / scale) < 1e-8
    f = np.sum(np.abs(r) ** p)
    for _ in range(20):
        xp = x + 1e-3 * g.standard_normal(6)
        assert np.sum(np.abs(w * (M @ xp - y)) ** p) >= f * (1 - 1e-13)


def test_conditioned_basis_is_an_l2_embedding():
    # U = R^{-1} from a subspace embedding F A makes A U nearly orthonormal
    # (Section 5 theorem); a transposed R or a wrong block hash breaks this
    A, _, _ = W.lp_dense(n=3000, d=8)
    for w in (0, 1000):
        R = LP.condition(A, 11, 64, 8, 2, w)
        sv = np.linalg.svd(A @ np.linalg.inv(R), compute_uv=False)
        assert 0.6 < sv.min() <= sv.max() < 1.4


@pytest.mark.parametrize("p", [1.0, 1.5, 2.0, 3.0])
def test_keeping_every_row_gives_the_exact_fit(p):
    A, b, _ = W.lp_dense(n=600, d=5)
    out = LP.lp_regression(A, b, p, 3, 16, 4, 1, s1=1e30, s2=1e30)
    assert out["rows1"].size == 600 and out["rows2"].size == 600
    assert np.all(out["w2"] == 1.0)
    fx = LP.lp_objective(A, b, out["x"], p)
    fe = LP.lp_objective(A, b, LP.lp_exact(A, b, p), p)
    assert fx == pytest.approx(fe, rel=1e-9)
    if p == 2.0:
        assert np.allclose(out["x"], np.linalg.lstsq(A, b, rcond=None)[0], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("p", [1.0, 1.5, 3.0])
def test_sampled_fit_is_within_one_plus_eps(p):
    A, b, _ = W.lp_dense(n=20000, d=8)
    out = LP.lp_regression(A, b, p, 0x5EED, 64, 8, 1, s1=800, s2=800)
    assert 8 <= out["rows2"].size < 2000
    ratio = LP.lp_objective(A, b, out["x"], p) / LP.lp_objective(A, b, LP.lp_exact(A, b, p), p)
    assert 1 - 1e-12 <= ratio < 1.1 ** p
    # the stage-2 probabilities dominate the stage-1 share of every row
    share = out["pi"] / 800
    assert np.all(out["q"] >= np.minimum(1.0, 800 * share) * (1 - 1e-12))


@pytest.mark.parametrize("p", [1.0, 1.5, 3.0])
def test_consistent_system_is_solved_exactly(p):
    A, _, x0 = W.lp_dense(n=2500, d=7)
    b = A @ x0
    out = LP.lp_regression(A, b, p, 4, 64, 4, 1, 300.0, 300.0)
    assert np.allclose(out["x"], x0, rtol=0, atol=1e-9 * np.max(np.abs(x0)))
    assert np.allclose(out["x_c"], x0, rtol=0, atol=1e-9 * np.max(np.abs(x0)))


def test_rank_deficient_input_is_rejected():
    A, b, _ = W.lp_dense(n=500, d=4)
    A[:, 2] = 0.0
    with pytest.raises(ValueError):
        LP.lp_regression(A, b, 1.0, 1, 16, 4, 1, s1=100, s2=100)
    with pytest.raises(ValueError):
        LP.lp_regression(A, b, 0.5, 1, 16, 4, 1, s1=100, s2=100)


def _exact_r(Ad):
    # R of A's own QR by LAPACK (non-negative diagonal): A R^-1 is then an
    # orthonormal basis Q of the column space of A
    R = np.linalg.qr(Ad, mode="r")
    return R * np.sign(np.diag(R))[:, None]


def test_row_norm_estimates_sum_to_the_squared_frobenius_norm_of_pi2():
    # with the exact R, A R^-1 = Q has orthonormal columns, so the squared
    # row norms of Q Pi2 sum to ||Q Pi2||_F^2 = ||Pi2||_F^2 = d for a sign
    # matrix with entries +-1/sqrt(k) (Section 9 row-norm estimates through
    # Section 6's Pi2).  R^-T in place of R^-1, unsquared norms, or A in
    # place of A R^-1 all break the identity.
    rng = np.random.default_rng(11)
    n, d = 400, 7
    Ad = rng.standard_normal((n, d)) * np.exp(rng.standard_normal(n))[:, None]
    Ad[:, 3] *= 50.0
    R = _exact_r(Ad)
    for seed, k in [(1, 8), (2, 32), (3, 5)]:
        lev = LP.row_norm_estimates(Ad, R, seed, k)
        assert lev.shape == (n,)
        assert np.all(lev >= 0)
        assert lev.sum() == pytest.approx(d, rel=1e-12)


def test_row_norm_estimates_are_unbiased_for_the_leverage_scores():
    # E over the signs of ||e_i^T Q Pi2||^2 = ||Q_i||^2 = u_i (LAPACK Q),
    # with variance 2 (||z||^4 - ||z||_4^4) / k for z = Q_i (independent
    # +-1/sqrt(k) entries); the mean over many seeds lies within 5 standard
    # errors for every row
    rng = np.random.default_rng(12)
    n, d, k, reps = 60, 5, 4, 3000
    Ad = rng.standard_normal((n, d)) * np.exp(rng.standard_normal(n))[:, None]
    R = _exact_r(Ad)
    Q = np.linalg.qr(Ad)[0]
    u = (Q * Q).sum(axis=1)
    var = 2.0 * (u ** 2 - (Q ** 4).sum(axis=1)) / k
    acc = np.zeros(n)
    for s in range(reps):
        acc += LP.row_norm_estimates(Ad, R, 1000 + s, k)
    mean = acc / reps
    se = np.sqrt(var / reps) + 1e-15
    assert np.all(np.abs(mean - u) <= 5 * se)


def test_row_norm_estimates_on_csr_match_a_dense_evaluation():
    # A R^-1 Pi2 evaluated by LAPACK's inverse and a dense product, for a
    # sketched R and the sign matrix drawn from the same stream
    from oracle.lowrank import sign_projection

    A = _small_csr(n=500, d=9, k=4, seed=13)
    Ad = A.to_dense().astype(np.float64)
    R = LP.condition(A, 77, 16, 4, 1)
    Z = Ad @ np.linalg.inv(R) @ sign_projection(5, 9, 16)
    assert np.allclose(LP.row_norm_estimates(A, R, 5, 16), (Z * Z).sum(axis=1), rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("p", [1.0, 1.5, 3.0])
def test_stage1_probabilities_follow_the_p_th_power_of_the_l2_estimates(p):
    # Section 9: the l_p norm of row i of A U is estimated by the l_2 norm of
    # row i of A U Pi2, so stage 1 keeps row i with probability
    # min(1, s1 * e_i^p / sum_j e_j^p), e_i = ||(A R^-1 Pi2)_i||_2 (here
    # evaluated with LAPACK's inverse, independently of the oracle's solves)
    from oracle.lowrank import sign_projection

    rng = np.random.default_rng(14)
    n, d = 800, 6
    Ad = rng.standard_normal((n, d)) * np.exp(rng.standard_normal(n))[:, None]
    b = Ad @ rng.standard_normal(d) + rng.laplace(0, 0.1, n)
    seed, s1 = 0x1234, 200.0
    out = LP.lp_regression(Ad, b, p, seed, 16, 4, 1, s1, s1)
    e = np.linalg.norm(Ad @ np.linalg.inv(out["R"]) @ sign_projection(seed, d, 32), axis=1)
    want = np.minimum(1.0, s1 * e ** p / np.sum(e ** p))
    assert np.allclose(out["pi"], want, rtol=1e-9, atol=1e-15)
