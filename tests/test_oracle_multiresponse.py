"""Pins for the oracle's multiple-response regression by leverage-score
sampling (Section 7, generalized-regression algorithm)."""

import numpy as np
import pytest

import oracle as O
import workloads as W


def _problem(seed=0, dp=4, noise=0.01):
    A, _, _ = W.lstsq_small()
    g = np.random.default_rng(seed)
    Y0 = g.standard_normal((A.d, dp))
    B = O.MatrixOp(A).matmat(Y0) + noise * g.standard_normal((A.n, dp))
    return A, B, Y0


def test_identity_sampling_gives_exact_least_squares():
    g = np.random.default_rng(1)
    A = g.standard_normal((300, 12))
    B = g.standard_normal((300, 5))
    r = O.multi_response_lstsq(A, B, 0, 0, 0, S=np.eye(300))
    ref = np.linalg.lstsq(A, B, rcond=None)[0]
    assert np.allclose(r["Y"], ref, rtol=1e-10, atol=1e-12)


def test_columns_are_solved_independently():
    A, B, _ = _problem()
    r = O.multi_response_lstsq(A, B, 5, 4000, 1500)
    for c in range(B.shape[1]):
        rc = O.multi_response_lstsq(A, B[:, c], 5, 4000, 1500)
        assert np.array_equal(rc["counts"], r["counts"])
        assert np.allclose(rc["Y"][:, 0], r["Y"][:, c], rtol=1e-13, atol=1e-15)


def test_consistent_system_is_solved_exactly():
    A, B, Y0 = _problem(noise=0.0)
    r = O.multi_response_lstsq(A, B, 9, 4000, 800)
    assert np.allclose(r["Y"], Y0, rtol=1e-10, atol=1e-11)


def test_residual_ratio_at_least_one_and_small():
    A, B, _ = _problem(seed=3)
    opt = O.residual_fro(A, np.linalg.lstsq(A.to_dense(), B, rcond=None)[0], B)
    for seed in range(4):
        r = O.multi_response_lstsq(A, B, 100 + seed, 4000, 2000)
        ratio = O.residual_fro(A, r["Y"], B) / opt
        assert 1 - 1e-12 <= ratio <= 1.05
