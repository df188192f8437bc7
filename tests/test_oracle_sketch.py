"""Pins for the oracle's sketch ``S A`` (Section 2 definition; moments used in
Section 7: unbiasedness of ``||S A||_F^2`` and of ``(S A)^T (S B)``)."""

import numpy as np

import oracle as O
import workloads as W


def _rng(s):
    return np.random.default_rng(s)


def injective_seed(n, t, start=1):
    for seed in range(start, start + 100000):
        h, _ = O.bucket_and_sign(seed, n, t)
        if len(np.unique(h)) == n:
            return seed
    raise AssertionError("no injective seed found")


def test_explicit_S_structure():
    # exactly one nonzero, of value +-1, in every column of Phi D
    S = O.explicit_S(11, 200, 17)
    nz = (S != 0).sum(axis=0)
    assert np.all(nz == 1)
    assert set(np.unique(S[S != 0])) <= {-1.0, 1.0}


def test_sketch_matches_explicit_product():
    A = _rng(0).standard_normal((300, 7))
    S = O.explicit_S(5, 300, 40)
    assert np.allclose(O.sketch_dense(A, 5, 40), S @ A, rtol=0, atol=1e-12)
    b = _rng(1).standard_normal(300)
    assert np.allclose(O.sketch_dense(b, 5, 40), S @ b, rtol=0, atol=1e-12)


def test_csr_and_dense_agree():
    A = W.csr_uniform_rows(3, 500, 30, 5, dtype=np.float64)
    Y1 = O.sketch_csr(A.n, A.d, A.row_ptr, A.col_idx, A.val, 9, 64)
    Y2 = O.sketch_dense(A.to_dense(), 9, 64)
    assert np.allclose(Y1, Y2, rtol=0, atol=1e-12)
    S = O.explicit_S(9, 500, 64)
    assert np.allclose(Y1, S @ A.to_dense(), rtol=0, atol=1e-12)


def test_integer_values_are_exact():
    A = W.csr_uniform_rows(4, 2000, 16, 4, dtype=np.float32, values="int")
    Y = O.sketch_csr(A.n, A.d, A.row_ptr, A.col_idx, A.val, 1, 32)
    S = O.explicit_S(1, 2000, 32).astype(np.int64)
    exact = S @ A.to_dense().astype(np.int64)
    assert np.array_equal(Y, exact.astype(np.float64))


def test_t_equal_one_is_signed_sum():
    A = _rng(2).standard_normal((50, 4))
    _, s = O.bucket_and_sign(8, 50, 1)
    assert np.allclose(O.sketch_dense(A, 8, 1)[0], s @ A, atol=1e-12)


def test_perfect_hashing_is_isometry():
    # If h is injective on the rows, S A only permutes and re-signs rows, so
    # (SA)^T SA = A^T A exactly (birthday/perfect-hashing step of Section 3).
    n, t = 8, 256
    seed = injective_seed(n, t)
    A = _rng(3).integers(-5, 6, size=(n, 3)).astype(np.float64)
    Y = O.sketch_dense(A, seed, t)
    assert np.array_equal(Y.T @ Y, A.T @ A)


def test_row_shards_sum_to_whole():
    # Linearity of Phi D with global row indices: sum_g S A_g = S A.
    A = _rng(4).standard_normal((1000, 6))
    full = O.sketch_dense(A, 21, 33)
    parts = sum(O.sketch_dense(A[a:b], 21, 33, start=a) for a, b in [(0, 250), (250, 700), (700, 1000)])
    assert np.allclose(parts, full, atol=1e-12)


def _moments(vals):
    vals = np.asarray(vals)
    return vals.mean(), vals.std(ddof=1) / np.sqrt(len(vals))


def test_norm_unbiased_with_exact_variance():
    # E ||S y||^2 = ||y||^2 and Var = (2/t)(||y||_2^4 - ||y||_4^4)
    y = _rng(5).standard_normal(40)
    t, K = 6, 4000
    vals = np.array([np.sum(O.sketch_dense(y, s, t) ** 2) for s in range(K)])
    m, se = _moments(vals)
    ny2 = np.sum(y * y)
    assert abs(m - ny2) < 5 * se
    var_exact = 2.0 / t * (ny2 ** 2 - np.sum(y ** 4))
    var_mc = vals.var(ddof=1)
    assert abs(var_mc / var_exact - 1) < 0.15


def test_frobenius_unbiased_and_variance_bound():
    # E ||S A||_F^2 = ||A||_F^2; Var = (2/t) sum_{i != j} <a_i, a_j>^2 <= (6/t) ||A||_F^4
    A = _rng(6).standard_normal((30, 3))
    t, K = 5, 4000
    vals = np.array([np.sum(O.sketch_dense(A, s, t) ** 2) for s in range(K)])
    m, se = _moments(vals)
    F2 = np.sum(A * A)
    assert abs(m - F2) < 5 * se
    G = A @ A.T
    var_exact = 2.0 / t * (np.sum(G * G) - np.sum(np.diag(G) ** 2))
    assert abs(vals.var(ddof=1) / var_exact - 1) < 0.15
    assert var_exact <= 6.0 / t * F2 ** 2


def test_product_unbiased():
    # E[(S A)^T (S B)] = A^T B (approximate matrix multiplication lemma)
    A = _rng(7).standard_normal((25, 2))
    B = _rng(8).standard_normal((25, 2))
    t, K = 4, 4000
    P = np.array([(O.sketch_dense(A, s, t).T @ O.sketch_dense(B, s, t)) for s in range(K)])
    mean = P.mean(axis=0)
    se = P.std(axis=0, ddof=1) / np.sqrt(K)
    assert np.all(np.abs(mean - A.T @ B) < 5 * se)


def test_bucket_rows_sampler():
    A = _rng(9).standard_normal((400, 5))
    full = O.sketch_dense(A, 13, 20)
    rows = O.sketch_bucket_rows(lambda idx: A[idx], 13, 400, 20, [0, 7, 19])
    assert np.allclose(rows, full[[0, 7, 19]], atol=1e-12)


def test_learned_values_replace_signs():
    A = _rng(10).standard_normal((60, 3))
    _, s = O.bucket_and_sign(4, 60, 9)
    assert np.allclose(O.sketch_dense(A, 4, 9, w=s.astype(float)), O.sketch_dense(A, 4, 9), atol=1e-12)
    w = _rng(11).standard_normal(60)
    assert np.allclose(O.sketch_dense(A, 4, 9, w=w), O.explicit_S(4, 60, 9, w=w) @ A, atol=1e-12)
