"""Pins for the oracle's generalized sparse embedding (Section 5, the
construction: S = blockdiag(B^(1), ..., B^(q)) P)."""

import numpy as np
import pytest

import oracle.sketch as SK
from oracle.hashing import bucket_and_sign


def test_columns_have_one_scaled_sign_per_copy():
    n, q, v, a, seed = 300, 5, 8, 3, 17
    S = SK.generalized_S(seed, n, q, v, a)
    assert S.shape == (a * q * v, n)
    nz = S != 0
    assert np.all(nz.sum(axis=0) == a)
    assert np.allclose(np.abs(S[nz]), 1 / np.sqrt(a))
    for j in range(a):  # one entry in each copy's rows
        assert np.all(nz[j * q * v:(j + 1) * q * v].sum(axis=0) == 1)


def test_outer_group_is_shared_by_the_copies():
    n, q, v, a, seed = 200, 7, 4, 4, 3
    S = SK.generalized_S(seed, n, q, v, a)
    h, _ = bucket_and_sign(seed, n, q)
    for i in range(n):
        rows = np.nonzero(S[:, i])[0]
        groups = (rows % (q * v)) // v
        assert np.all(groups == h[i])


def test_block_order_is_block_diagonal_after_grouping_columns():
    n, q, v, a, seed = 150, 4, 5, 2, 8
    Sb = SK.generalized_S(seed, n, q, v, a, order="block")
    h, _ = bucket_and_sign(seed, n, q)
    perm = np.argsort(h, kind="stable")
    B = Sb[:, perm]
    counts = np.bincount(h, minlength=q)
    c0 = 0
    for g in range(q):
        blk = np.zeros_like(B, dtype=bool)
        blk[g * a * v:(g + 1) * a * v, c0:c0 + counts[g]] = True
        c0 += counts[g]
        assert np.all(B[:, np.any(blk, axis=0)][~np.any(blk, axis=1)] == 0)
    # the copy order is a row permutation of the block order
    Sc = SK.generalized_S(seed, n, q, v, a)
    assert sorted(map(tuple, Sb.round(12))) == sorted(map(tuple, Sc.round(12)))


def test_row_scatter_matches_the_written_out_matrix():
    g = np.random.default_rng(1)
    A = g.standard_normal((120, 7))
    for q, v, a in ((3, 4, 2), (1, 16, 1), (6, 2, 5)):
        S = SK.generalized_S(99, 120, q, v, a)
        assert np.allclose(SK.sketch_generalized(A, 99, q, v, a), S @ A, atol=1e-13)


def test_one_group_one_copy_is_the_plain_sketch():
    A = np.random.default_rng(2).standard_normal((500, 9))
    seed, v = 12345, 64
    got = SK.sketch_generalized(A, seed, 1, v, 1)
    ref = SK.sketch_dense(A, SK.copy_seed(seed, 0), v)
    assert np.array_equal(got, ref)


def test_norm_is_unbiased_with_the_exact_variance():
    # ||S y||^2 averages a independent sketches of composite bucket h(i) v + h_j(i):
    # mean ||y||^2, variance (1/a) (2 / (q v)) (||y||^4 - ||y||_4^4)
    g = np.random.default_rng(3)
    y = g.standard_normal(60)
    q, v, a = 3, 4, 3
    vals = np.array([np.sum(SK.sketch_generalized(y[:, None], s, q, v, a) ** 2) for s in range(4000)])
    n2, n4 = np.sum(y ** 2), np.sum(y ** 4)
    var = (2.0 / (a * q * v)) * (n2 ** 2 - n4)
    assert abs(vals.mean() - n2) < 5 * np.sqrt(var / vals.size)
    assert vals.var() == pytest.approx(var, rel=0.15)
