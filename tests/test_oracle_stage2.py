"""Pins for the oracle's second sketch stage Pi1 = F S (Section 6; the
composition facts of Section 8).

* bfloat16 rounding against torch's own float32 -> bfloat16 conversion,
  including exact ties (a library routine);
* F is a Johnson-Lindenstrauss map: every column has unit norm exactly,
  ``E ||F y||^2 = ||y||^2`` over seeds, distinct rows are uncorrelated, and
  on a d-dimensional subspace its singular values lie within the
  random-matrix range ``1 +- sqrt(d / m)`` (up to a small margin);
* composition: on a consistent system whose sketch is exact in bfloat16,
  sketch-and-solve through ``F S`` returns the solution exactly (any
  full-rank Pi1 does), and a wrong F on one side (transposed, another seed)
  does not;
* the iteration with the R of ``F S A`` reaches the exact least-squares
  optimum within the certified ratio.
"""

import numpy as np
import pytest
import torch

import oracle as O
import oracle.stage2 as S2


def test_round_bf16_matches_torch_including_ties():
    g = np.random.default_rng(5)
    x = np.concatenate([g.standard_normal(4000) * 10.0 ** g.integers(-8, 8, 4000),
                        [0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-40]])
    # exact ties: low 16 bits 0x8000 above even and odd kept parts
    ties = (np.array([0x3F808000, 0x3F818000, 0xBF808000, 0xBF818000, 0x40490000 | 0x8000], np.uint32)
            .view(np.float32).astype(np.float64))
    x = np.concatenate([x, ties])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = S2.round_bf16(x)
    assert np.array_equal(got, ref)
    # float64 inputs are rounded to float32 first (two roundings)
    y = np.array([1.0 + 2.0 ** -8 + 2.0 ** -30])  # just above a bfloat16 tie only in float64
    assert S2.round_bf16(y)[0] == 1.0  # float32 rounding lands on the tie, which goes to even


def test_stage_matrix_entries_and_unit_columns():
    m, t = 96, 1000
    F = S2.stage_matrix(123, m, t)
    assert F.shape == (m, t)
    assert np.all(np.abs(F) == 1.0 / np.sqrt(m))
    assert np.allclose((F * F).sum(axis=0), 1.0, rtol=0, atol=1e-14)
    # both signs occur in about equal numbers (binomial, 6 sigma)
    neg = np.count_nonzero(F < 0)
    assert abs(neg - m * t / 2) <= 6 * np.sqrt(m * t / 4)


def test_stage_rows_are_the_rows_of_the_matrix():
    m, t = 40, 333
    F = S2.stage_matrix(9, m, t)
    rows = np.array([0, 7, 39])
    assert np.array_equal(S2.sign_rows(9, rows, t).astype(np.float64) / np.sqrt(m), F[rows])


def test_norm_preserved_in_expectation():
    # E ||F y||^2 = ||y||^2 for entries of mean 0 and variance 1/m
    m, t = 32, 500
    y = np.random.default_rng(1).standard_normal(t)
    vals = [np.sum((S2.stage_matrix(s, m, t) @ y) ** 2) for s in range(400)]
    # each value has variance ~ 2 ||y||^4 / m; the mean of 400 is within 6 sigma
    assert abs(np.mean(vals) / np.dot(y, y) - 1.0) <= 6 * np.sqrt(2.0 / m / 400)


def test_rows_uncorrelated():
    m, t = 64, 8192
    F = S2.stage_matrix(77, m, t)
    G = F @ F.T  # diagonal t / m exactly; off-diagonal mean 0, sd sqrt(t) / m
    assert np.allclose(np.diag(G), t / m, rtol=1e-14)
    off = G[~np.eye(m, dtype=bool)]
    assert np.max(np.abs(off)) <= 6 * np.sqrt(t) / m
    # rows shifted against each other by one word are uncorrelated too (an
    # index map that reused words across rows would show here)
    S = np.sqrt(m) * F
    for shift in (64, 128):
        c = np.mean(S[1:, shift:] * S[:-1, :-shift])
        assert abs(c) <= 6 / np.sqrt((m - 1) * (t - shift))


def test_subspace_singular_values_in_random_matrix_range():
    m, t, d = 512, 4096, 64
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((t, d)))
    sv = np.linalg.svd(S2.stage_matrix(4, m, t) @ Q, compute_uv=False)
    r = np.sqrt(d / m)
    assert sv.max() <= 1 + r + 0.1 and sv.min() >= 1 - r - 0.1


def _integer_system(seed, n, d):
    g = np.random.default_rng(seed)
    A = g.integers(-2, 3, size=(n, d)).astype(np.float64)
    x0 = g.integers(-4, 5, size=d).astype(np.float64)
    return A, x0


def test_composition_exact_on_consistent_integer_system():
    # S A is integer with |entries| < 256, hence exact in bfloat16, and
    # b = A x0: any full-rank Pi1 gives x~ = x0
    n, d, t, m = 3000, 12, 400, 60
    A, x0 = _integer_system(0, n, d)
    SA = O.sketch_dense(A, 31, t)
    assert np.max(np.abs(SA)) < 256 and np.array_equal(S2.round_bf16(SA), SA)
    x, R = S2.sketch_and_solve(A, A @ x0, 31, t, m)
    assert np.allclose(x, x0, rtol=0, atol=1e-10)
    FSA, _ = S2.second_stage(SA, None, 31, m)
    assert np.allclose(R.T @ R, FSA.T @ FSA, rtol=1e-12, atol=1e-9)


def test_composition_detects_mismatched_second_stage():
    # F S b formed with another F (other seed, or F applied from the other
    # side) does not reproduce x0
    n, d, t, m = 3000, 12, 400, 60
    A, x0 = _integer_system(1, n, d)
    SA = O.sketch_dense(A, 32, t)
    Sb = O.sketch_dense(A @ x0, 32, t)
    FSA, FSb = S2.second_stage(SA, Sb, 32, m)
    x_ok = np.linalg.lstsq(FSA, FSb, rcond=None)[0]
    assert np.allclose(x_ok, x0, atol=1e-10)
    _, FSb_other = S2.second_stage(SA, Sb, 33, m)
    assert not np.allclose(np.linalg.lstsq(FSA, FSb_other, rcond=None)[0], x0, atol=1e-3)


def test_two_stage_lstsq_reaches_certified_ratio():
    g = np.random.default_rng(8)
    n, d, t, m = 6000, 16, 1500, 128
    A = g.standard_normal((n, d)) * (1.0 + g.pareto(1.5, size=n))[:, None]
    b = A @ g.standard_normal(d) + 0.1 * g.standard_normal(n)
    xs = O.lstsq_exact(A, b)
    x, x_t, R, it, ok = S2.lstsq(A, b, 17, t, m, delta=1e-10)
    assert ok
    assert O.residual_ratio(A, b, x, xs) <= 1 + 1e-10
    # A R^{-1} is well conditioned: singular values within the composed range
    sv = np.linalg.svd(A @ np.linalg.inv(R), compute_uv=False)
    assert sv.min() >= 0.5 and sv.max() <= 1 / (1 - np.sqrt(d / m)) / 0.8
    # the sketch-and-solve start is already close
    assert O.residual_ratio(A, b, x_t, xs) <= 1.5


def test_bit_order_is_a_permutation():
    b = S2.bit_of_offset(np.arange(64))
    assert sorted(b.tolist()) == list(range(64))
    # neighbouring rows 2j, 2j + 1 sit 16 bits apart in the same 32-bit half
    assert np.all(b[1::2] - b[0::2] == 16)
