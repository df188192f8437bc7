"""GPU parity: rank-k approximation A ~ L D W^T (Section 8 theorem in the
simplified form of the Section 10 experiments) against the oracle.

The GPU evaluates the theorem's steps through equivalent QR-based
factorisations and finds the best rank-k part by subspace iteration, so the
comparison is on what is unique: the drawn rows (integer counts, decided in
float64 on both sides), the values D, the rank-k matrix L D W^T, and the
Frobenius error; L and W are checked for orthonormal columns.
"""

import numpy as np
import pytest
import torch

import oracle.lowrank as LR
import workloads as W
from gpu_util import dev, up, up_bf16, up_csr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_1207_6365_amd as sk

    return sk


def _check(got, ref, A_dense, tol=1e-9):
    L, D, Wm, info = got
    L, D, Wm = L.cpu().numpy(), D.cpu().numpy(), Wm.cpu().numpy()
    k = D.size
    assert np.allclose(L.T @ L, np.eye(k), atol=1e-10)
    assert np.allclose(Wm.T @ Wm, np.eye(k), atol=1e-10)
    assert np.all(np.diff(D) <= 1e-12 * D[0]) and np.all(D >= 0)
    assert np.allclose(D, ref["D"], rtol=tol, atol=tol * ref["D"][0])
    Xg = (L * D) @ Wm.T
    Xo = (ref["L"] * ref["D"]) @ ref["W"].T
    assert np.max(np.abs(Xg - Xo)) <= tol * ref["D"][0]
    err = np.linalg.norm(A_dense - Xg)
    assert info["resid_fro"] == pytest.approx(err, rel=1e-7, abs=1e-9 * np.linalg.norm(A_dense))
    assert info["fro_norm"] == pytest.approx(np.linalg.norm(A_dense), rel=1e-12)
    return err


@pytest.mark.parametrize("row64", [False, True])
def test_planted_sparse_matches_oracle(sk, row64):
    A = W.planted_lowrank_sparse(n=3000, rank=8, density=0.04)
    k, seed, t_r, t_s = 8, 0x1234, 64, 2048
    ref = LR.low_rank(A, k, seed, t_r, t_s)
    got = sk.low_rank(up_csr(A, row64=row64), k, seed, t_r=t_r, t_s=t_s)
    info = got[3]
    assert info["rows_sampled"] == int(np.count_nonzero(ref["counts"]))
    assert info["converged"] == 1
    err = _check(got, ref, A.to_dense())
    dk = LR.best_rank_k_error(A.to_dense(), k)
    assert err >= dk * (1 - 1e-9)


def test_empty_rows_and_columns_match_oracle(sk):
    # the planted input with every ninth row and every seventh column emptied
    A0 = W.planted_lowrank_sparse(n=3000, rank=8, density=0.04)
    rows = np.repeat(np.arange(A0.n), np.diff(A0.row_ptr))
    keep = (rows % 9 != 4) & (A0.col_idx % 7 != 2)
    lens = np.bincount(rows[keep], minlength=A0.n)
    A = W.CSR(A0.n, A0.d, np.concatenate([[0], np.cumsum(lens)]).astype(np.int64), A0.col_idx[keep], A0.val[keep])
    Ad = A.to_dense()
    assert not np.any(Ad[4::9]) and not np.any(Ad[:, 2::7])
    k, seed, t_r, t_s = 8, 0x4321, 64, 2048
    ref = LR.low_rank(A, k, seed, t_r, t_s)
    got = sk.low_rank(up_csr(A), k, seed, t_r=t_r, t_s=t_s)
    assert got[3]["rows_sampled"] == int(np.count_nonzero(ref["counts"]))
    assert not np.any(ref["counts"][4::9])
    _check(got, ref, Ad)
    L, Wm = got[0].cpu().numpy(), got[2].cpu().numpy()
    assert np.max(np.abs(L[4::9])) <= 1e-12 and np.max(np.abs(Wm[2::7])) <= 1e-12


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_dense_matches_oracle(sk, storage):
    g = np.random.default_rng(11)
    n, m, k = 1500, 700, 6
    A = (g.standard_normal((n, k)) * np.linspace(4, 1, k)) @ g.standard_normal((k, m)) \
        + 0.01 * g.standard_normal((n, m))
    if storage == "bf16":
        bits = W.bf16_round(A.astype(np.float32))
        Ad, Ag = W.bf16_to_f32(bits).astype(np.float64), up_bf16(bits)
    elif storage == "f32":
        Ad = A.astype(np.float32).astype(np.float64)
        Ag = up(A.astype(np.float32))
    else:
        Ad, Ag = A, up(A)
    ref = LR.low_rank(Ad, k, 77, 40, 1200)
    got = sk.low_rank(Ag, k, 77, t_r=40, t_s=1200)
    _check(got, ref, Ad)


def test_exact_rank_k_is_recovered(sk):
    # rank(A) = k = t_R: the approximation is A itself
    g = np.random.default_rng(5)
    k = 5
    A = g.standard_normal((800, k)) @ g.standard_normal((k, 300))
    L, D, Wm, info = sk.low_rank(up(A), k, 3, t_r=k, t_s=600)
    X = (L.cpu().numpy() * D.cpu().numpy()) @ Wm.cpu().numpy().T
    assert np.linalg.norm(X - A) <= 1e-10 * np.linalg.norm(A)
    assert info["resid_fro"] <= 1e-6 * info["fro_norm"]


def test_ragged_sizes_and_small_k(sk):
    # sizes that are not multiples of any tile, k = 1, t_r < k + oversample
    A = W.planted_lowrank_sparse(n=1111, rank=3, density=0.09)
    for k, t_r, t_s in ((1, 7, 300), (3, 13, 517)):
        ref = LR.low_rank(A, k, 5, t_r, t_s)
        got = sk.low_rank(up_csr(A), k, 5, t_r=t_r, t_s=t_s)
        _check(got, ref, A.to_dense())


def test_eps_sets_the_default_sketch_size(sk):
    A = W.planted_lowrank_sparse(n=2000, rank=4, density=0.05)
    _, _, _, info = sk.low_rank(up_csr(A), 4, 9, eps=0.125)
    assert info["t_r"] == 32 and info["t_s"] == 64 * 32  # max(ceil(4 / 0.125), 4 + 16)


def test_rank_deficient_sketch_is_reported(sk):
    # rank(A) = 2 < t_r: Y = A R^T cannot have full column rank
    g = np.random.default_rng(2)
    A = g.standard_normal((500, 2)) @ g.standard_normal((2, 200))
    with pytest.raises(sk.SklsError):
        sk.low_rank(up(A), 2, 1, t_r=16, t_s=400)
    # as many draws as columns of S U: repeated rows leave it rank deficient
    B = g.standard_normal((500, 200))
    with pytest.raises(ValueError):
        LR.low_rank(B, 2, 1, 64, 64)
    with pytest.raises(sk.SklsError):
        sk.low_rank(up(B), 2, 1, t_r=64, t_s=64)


def test_planted_full_size_properties(sk, golden_dir):
    # n = 65536, ~10M nonzeros, k = 32, t_r = 512: properties that hold at any
    # size, and the error against the stored best rank-k error
    import os

    vals = {}
    with open(os.path.join(golden_dir, "lowrank_planted_n65536_r32.txt")) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                key, v = line.split(":", 1)
                vals[key.strip()] = float(v)
    A = W.planted_lowrank_sparse()
    L, D, Wm, info = sk.low_rank(up_csr(A), 32, 0x5EED0000, t_r=512)
    assert info["converged"] == 1
    assert info["fro_norm"] == pytest.approx(vals["fro_norm"], rel=1e-12)
    ratio = info["resid_fro"] / vals["delta_k"]
    assert 1 - 1e-9 <= ratio <= 1.05
    print(f"error ratio {ratio:.6f}, iterations {info['iterations']}, rows {info['rows_sampled']}")
    k = 32
    G = (L.T @ L).cpu().numpy()
    H = (Wm.T @ Wm).cpu().numpy()
    assert np.allclose(G, np.eye(k), atol=1e-10) and np.allclose(H, np.eye(k), atol=1e-10)
    # spot entries of L D W^T against the rank-k reconstruction from the oracle's
    # view of A: |(L D W^T)_ij - A_ij| summed over the stored nonzeros is at most
    # the Frobenius error
    Dn = D.cpu().numpy()
    rows = torch.from_numpy(A.row_ids()).to(dev())
    cols = torch.from_numpy(A.col_idx.astype(np.int64)).to(dev())
    vals_g = ((L[rows] * D) * Wm[cols]).sum(dim=1).cpu().numpy()
    res_nz = np.linalg.norm(vals_g - A.val.astype(np.float64))
    assert res_nz <= info["resid_fro"] * (1 + 1e-9)
    assert Dn[0] >= Dn[-1] > 0
