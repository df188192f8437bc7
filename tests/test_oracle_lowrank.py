"""Pins for the oracle's rank-k approximation (Section 8 theorem on low-rank
approximation, simplified as in the Section 10 experiments)."""

import os

import numpy as np
import pytest
import scipy.sparse as sps

import oracle.lowrank as LR
import workloads as W


def _golden(golden_dir):
    out = []
    with open(os.path.join(golden_dir, "splitmix64_seed0.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                i, v = line.split()
                out.append((int(i), int(v, 16)))
    return out


def _planted(n=600, m=400, k=6, noise=1e-3, seed=0):
    g = np.random.default_rng(seed)
    P = g.standard_normal((n, k)) * np.linspace(3.0, 1.0, k)
    Q = g.standard_normal((m, k))
    return P @ Q.T + noise * g.standard_normal((n, m))


def test_sampling_uniforms_and_signs_follow_published_generator(golden_dir):
    # with the salt cancelled, stream outputs are the published SplitMix64 ones
    gold = _golden(golden_dir)
    u = LR.uniforms(LR.SAMPLE_SALT, len(gold))
    for i, v in gold:
        assert u[i] == (v >> 11) * 2.0**-53
    s = LR.sign_projection(LR.PI2_SALT, 1, len(gold))[0] * np.sqrt(len(gold))
    for i, v in gold:
        assert s[i] == (-1.0 if v & 1 else 1.0)
    assert np.all((u >= 0) & (u < 1))


def test_column_embedding_one_signed_entry_per_column():
    R = LR.column_embedding(7, 500, 37).toarray()
    assert R.shape == (37, 500)
    assert np.all(np.count_nonzero(R, axis=0) == 1)
    assert set(np.unique(R[R != 0])) <= {-1.0, 1.0}


def test_identity_embedding_and_sampling_give_truncated_svd():
    # R^ = I and S = I: U spans C(A), S U = U, and the result is [A]_k itself
    A = np.random.default_rng(3).standard_normal((70, 45))
    k = 6
    r = LR.low_rank(A, k, 0, 0, 0, Rhat=np.eye(45), S=np.eye(70))
    Us, s, Vt = np.linalg.svd(A, full_matrices=False)
    Ak = (Us[:, :k] * s[:k]) @ Vt[:k]
    assert np.allclose(r["D"], s[:k], rtol=1e-12)
    assert np.max(np.abs((r["L"] * r["D"]) @ r["W"].T - Ak)) <= 1e-11 * s[0]
    assert LR.frobenius_error(A, r["L"], r["D"], r["W"]) == pytest.approx(LR.best_rank_k_error(A, k), rel=1e-12)


@pytest.mark.parametrize("csr", [False, True])
def test_exact_rank_k_is_recovered(csr):
    # rank(A) = k = t_R: C(A R^T) = C(A), so U X~ = U U^T A = A
    g = np.random.default_rng(5)
    k = 5
    A = g.standard_normal((300, k)) @ g.standard_normal((k, 180))
    inp = A
    if csr:
        P = g.standard_normal((300, k))
        P[g.random(P.shape) < 0.6] = 0.0  # all-zero rows of P give empty rows of A
        A = P @ g.standard_normal((k, 180))
        S = sps.csr_matrix(A)
        inp = W.CSR(300, 180, S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data)
    r = LR.low_rank(inp, k, 11, k, 120)
    approx = (r["L"] * r["D"]) @ r["W"].T
    assert np.linalg.norm(approx - A) <= 1e-10 * np.linalg.norm(A)


def test_error_ratio_never_below_one_and_near_one_for_planted():
    A = _planted()
    k = 6
    dk = LR.best_rank_k_error(A, k)
    ratios = []
    for seed in range(4):
        r = LR.low_rank(A, k, seed, 48, 600)
        e = LR.frobenius_error(A, r["L"], r["D"], r["W"])
        ratios.append(e / dk)
    ratios = np.array(ratios)
    assert np.all(ratios >= 1 - 1e-12)
    assert np.all(ratios <= 1.2)


def test_factors_orthonormal_and_values_sorted():
    A = _planted(seed=2)
    r = LR.low_rank(A, 6, 9, 40, 500)
    assert np.allclose(r["L"].T @ r["L"], np.eye(6), atol=1e-12)
    assert np.allclose(r["W"].T @ r["W"], np.eye(6), atol=1e-12)
    assert np.all(np.diff(r["D"]) <= 0) and np.all(r["D"] >= 0)


def test_sampling_frequencies_match_probabilities():
    g = np.random.default_rng(8)
    scores = g.random(40) ** 2
    scores[[3, 17, 39]] = 0.0  # rows with no leverage are never drawn
    t_s = 400000
    rows, counts = LR.sample_rows(scores, t_s, 123)
    assert counts.sum() == t_s and rows.size == t_s
    assert np.all(counts[[3, 17, 39]] == 0)
    p = scores / scores.sum()
    keep = p > 0
    chi2 = np.sum((counts[keep] - t_s * p[keep]) ** 2 / (t_s * p[keep]))
    dof = keep.sum() - 1
    assert chi2 < dof + 6 * np.sqrt(2 * dof)


def test_sampling_is_unbiased_for_the_identity():
    # E[S^T S] = sum_i (E count_i) / (t_S p_i) e_i e_i^T = I on rows with p_i > 0
    g = np.random.default_rng(4)
    scores = g.random(12) + 0.05
    p = scores / scores.sum()
    t_s = 50
    reps = 3000
    acc = np.zeros((reps, 12))
    for s in range(reps):
        _, c = LR.sample_rows(scores, t_s, 1000 + s)
        acc[s] = c / (t_s * p)
    mean = acc.mean(axis=0)
    se = acc.std(axis=0) / np.sqrt(reps)
    assert np.all(np.abs(mean - 1.0) < 5 * se)


def test_step_four_is_the_best_rank_k_solution():
    # lemma used in the theorem's proof: [U~^T SA]_k minimises ||U~ X - SA||_F
    # over rank-k X; compare with perturbed rank-k factorisations
    g = np.random.default_rng(6)
    Ut, _ = np.linalg.qr(g.standard_normal((90, 20)))
    SA = g.standard_normal((90, 35))
    k = 4
    Uk, sk, Vkt = np.linalg.svd(Ut.T @ SA, full_matrices=False)
    F, G = Uk[:, :k] * sk[:k], Vkt[:k]
    best = np.linalg.norm(Ut @ (F @ G) - SA)
    for _ in range(200):
        Fp = F + 1e-3 * g.standard_normal(F.shape)
        Gp = G + 1e-3 * g.standard_normal(G.shape)
        assert np.linalg.norm(Ut @ (Fp @ Gp) - SA) >= best - 1e-12
    for _ in range(50):
        X = g.standard_normal((20, k)) @ g.standard_normal((k, 35))
        assert np.linalg.norm(Ut @ X - SA) >= best


def test_sparse_and_dense_best_rank_k_error_agree():
    A = W.planted_lowrank_sparse(n=600, rank=5, density=0.08)
    dense = A.to_dense()
    assert LR.best_rank_k_error(A, 5) == pytest.approx(LR.best_rank_k_error(dense, 5), rel=1e-9)


def test_csr_and_dense_inputs_agree():
    A = W.planted_lowrank_sparse(n=500, rank=4, density=0.1)
    r1 = LR.low_rank(A, 4, 21, 24, 300)
    r2 = LR.low_rank(A.to_dense(), 4, 21, 24, 300)
    assert np.array_equal(r1["counts"], r2["counts"])
    assert np.allclose(r1["D"], r2["D"], rtol=1e-10)
