"""Oracle: rank-k approximation ``A ~ L D W^T`` (Section 8, theorem on low-rank
approximation), in the simplified form run in the Section 10 experiments: a
sparse embedding ``R^`` on the columns, no randomized Hadamard transform, and
leverage-score sampling for ``S``.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the theorem's order:

1. ``Y = A R^T`` for ``R^`` a ``t_R x m`` sparse embedding of the columns of
   ``A`` (the construction of Section 2 with the ``m`` columns as the
   coordinates); ``U`` an orthonormal basis of the column space of ``Y``
   (thin ``Q`` of a Householder QR).
2. ``S``: ``t_S`` rows drawn independently with replacement, row ``i`` with
   probability ``p_i`` proportional to its leverage score, each drawn row
   scaled by ``1 / sqrt(t_S p_i)``; then ``S U`` and ``S A``.  The scores are
   those of Section 6 for ``Y``: squared row norms of ``Y R_Y^{-1} Pi2`` with
   ``R_Y`` the triangular factor of ``Y`` and ``Pi2`` a ``t_R x k_G`` sign
   matrix scaled by ``1 / sqrt(k_G)``.
3. SVD ``S U = U~ Sigma~ V~^T``.
4. ``[U~^T S A]_k`` (best rank-``k`` approximation by a truncated SVD), then
   the SVD ``U^ D W^T`` of ``V~ Sigma~^{-1} [U~^T S A]_k`` truncated at ``k``.
5. ``L = U U^``.

Randomness (all from the one seed; SplitMix64 as in :mod:`.hashing`):
``R^`` uses the stream ``seed``; the signs of ``Pi2`` are bit 0 of outputs
``r * k_G + c`` of the stream ``seed ^ PI2_SALT``; draw ``j`` of the sampling
takes ``u_j = (z_j >> 11) * 2^-53`` from output ``j`` of the stream
``seed ^ SAMPLE_SALT`` and picks the first row whose running score sum
exceeds ``u_j`` times the total (the last row with a positive score if
rounding would run past it).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sps

from .hashing import bucket_and_sign, splitmix64
from .leverage import leverage_approx
from .linalg import check_rank, householder_qr, thin_q

PI2_SALT = 0x6C65766572616765     # "leverage"
SAMPLE_SALT = 0x73616D706C696E67  # "sampling"


def column_embedding(seed: int, m: int, t_r: int) -> sps.csr_matrix:
    """``R^`` (``t_R x m``): column ``j`` holds ``sigma(j)`` in row ``h(j)``."""
    h, s = bucket_and_sign(seed, m, t_r)
    return sps.csr_matrix((s.astype(np.float64), (h, np.arange(m))), shape=(t_r, m))


def sign_projection(seed: int, rows: int, k_g: int) -> np.ndarray:
    """``Pi2``: entries ``+-1 / sqrt(k_G)``, sign from bit 0 of SplitMix64."""
    z = splitmix64(seed ^ PI2_SALT, np.arange(rows * k_g, dtype=np.uint64))
    s = np.where((z & np.uint64(1)) == np.uint64(1), -1.0, 1.0)
    return s.reshape(rows, k_g) / np.sqrt(k_g)


def uniforms(seed: int, count: int) -> np.ndarray:
    """``u_j`` in ``[0, 1)`` with 53 random bits, ``j = 0 .. count - 1``."""
    z = splitmix64(seed ^ SAMPLE_SALT, np.arange(count, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0**-53


def sample_rows(scores: np.ndarray, t_s: int, seed: int):
    """Draws of the leverage-score sampling: ``(rows, counts)`` where
    ``rows[j]`` is the row of draw ``j`` and ``counts[i]`` how often row ``i``
    was drawn."""
    cum = np.cumsum(np.asarray(scores, dtype=np.float64))
    pos = np.nonzero(scores > 0)[0]
    if pos.size == 0:
        raise ValueError("all leverage scores are zero")
    x = uniforms(seed, t_s) * cum[-1]
    rows = np.searchsorted(cum, x, side="right")
    rows = np.minimum(rows, pos[-1])
    counts = np.bincount(rows, minlength=scores.size)
    return rows, counts


def sampling_matrix(rows: np.ndarray, scores: np.ndarray, n: int) -> sps.csr_matrix:
    """``S`` (``t_S x n``): draw ``j`` is row ``rows[j]`` of the identity
    scaled by ``1 / sqrt(t_S p)``, ``p`` the probability of that row."""
    t_s = rows.size
    p = np.asarray(scores, dtype=np.float64) / np.sum(scores)
    vals = 1.0 / np.sqrt(t_s * p[rows])
    return sps.csr_matrix((vals, (np.arange(t_s), rows)), shape=(t_s, n))


def _as_matrix(A):
    """Float64 dense array or scipy CSR of the input."""
    if isinstance(A, np.ndarray):
        return np.asarray(A, dtype=np.float64)
    return sps.csr_matrix((np.asarray(A.val, dtype=np.float64), np.asarray(A.col_idx), np.asarray(A.row_ptr)),
                          shape=(int(A.n), int(A.d)))


def _rank_k_svd(M: np.ndarray, k: int):
    Uk, sk, Vkt = np.linalg.svd(M, full_matrices=False)
    return Uk[:, :k], sk[:k], Vkt[:k, :]


def low_rank(A, k: int, seed: int, t_r: int, t_s: int, k_g: int = 32, Rhat=None, S=None) -> dict:
    """Rank-``k`` approximation by the steps above.  ``Rhat`` (``t_R x m``)
    and ``S`` (``t_S x n``) replace the random embedding and the sampling when
    given.  Returns ``L`` (``n x k``), ``D`` (``k``), ``W`` (``m x k``) and the
    intermediate quantities."""
    M = _as_matrix(A)
    n, m = M.shape
    if not 1 <= k <= min(n, m):
        raise ValueError("need 1 <= k <= min(n, m)")
    # step 1: Y = A R^T and an orthonormal basis U of its column space
    if Rhat is None:
        Rhat = column_embedding(seed, m, t_r)
    Rd = Rhat.toarray() if sps.issparse(Rhat) else np.asarray(Rhat, dtype=np.float64)
    Y = np.asarray(M @ Rd.T, dtype=np.float64)
    t_r = Y.shape[1]
    Vs, R_Y = householder_qr(Y)
    check_rank(R_Y)
    U = thin_q(Vs, n)
    # step 2: leverage-score sampling (Section 6 scores of Y)
    scores = None
    rows = counts = None
    if S is None:
        scores = leverage_approx(Y, 0, 1, sign_projection(seed, t_r, k_g), R=R_Y)
        rows, counts = sample_rows(scores, t_s, seed)
        S = sampling_matrix(rows, scores, n)
    SU = np.asarray(S @ U)
    SA = S @ M
    SA = SA.toarray() if sps.issparse(SA) else np.asarray(SA)
    # step 3: SVD of S U
    Ut, st, Vtt = np.linalg.svd(SU, full_matrices=False)
    if st[-1] <= st[0] * SU.shape[1] * np.finfo(np.float64).eps:
        raise ValueError("S U is rank deficient")
    # step 4: best rank-k approximation of U~^T S A, then the SVD of
    # V~ Sigma~^{-1} [U~^T S A]_k
    Pk, sk, Qkt = _rank_k_svd(Ut.T @ SA, k)
    X = (Vtt.T / st) @ (Pk * sk) @ Qkt
    Uh, D, Wt = _rank_k_svd(X, k)
    # step 5
    L = U @ Uh
    return {"L": L, "D": D, "W": Wt.T, "Y": Y, "R_Y": R_Y, "U": U, "scores": scores, "rows": rows,
            "counts": counts, "cond_SU": st[0] / st[-1]}


def frobenius_error(A, L: np.ndarray, D: np.ndarray, W: np.ndarray) -> float:
    """``||A - L diag(D) W^T||_F`` formed explicitly."""
    M = _as_matrix(A)
    M = M.toarray() if sps.issparse(M) else M
    return float(np.linalg.norm(M - (L * D) @ W.T))


def best_rank_k_error(A, k: int) -> float:
    """``Delta_k = ||A - [A]_k||_F`` (Section 8 definition): from all singular
    values of a dense input, or ``||A||_F^2`` minus the top ``k`` squared
    singular values (ARPACK) of a sparse one."""
    M = _as_matrix(A)
    if not sps.issparse(M):
        s = np.linalg.svd(M, compute_uv=False)
        return float(np.sqrt(np.sum(s[k:] ** 2)))
    from scipy.sparse.linalg import svds

    sk = svds(M, k=k, return_singular_vectors=False, tol=0, maxiter=10000,
              v0=np.ones(M.shape[1]) / np.sqrt(M.shape[1]))
    tot = float(np.sum(M.data ** 2))
    return float(np.sqrt(max(tot - np.sum(sk ** 2), 0.0)))
