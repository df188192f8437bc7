"""Oracle: applying the sparse embedding ``S = Phi D`` (Section 2) to a matrix.

``Phi`` is the ``t x n`` 0/1 matrix with ``Phi[h(i), i] = 1`` and ``D`` the
diagonal of random signs, so ``(S A)[b, :] = sum over i with h(i) = b of
sigma(i) * A[i, :]``; this is the ``O(nnz(A))`` product of the main theorem
(Section 3) and of the regression theorem in Section 7, which sketches ``A``
adjoined with ``b``.  Everything is accumulated in float64, rows in increasing
order.

The learned-value form replaces ``sigma(i)`` by a real weight ``w_i`` and
keeps ``h`` from the seed.
"""

from __future__ import annotations

import numpy as np

from .hashing import bucket_and_sign


def explicit_S(seed: int, n: int, t: int, w=None) -> np.ndarray:
    """The ``t x n`` matrix ``Phi D`` written out (small ``n`` only)."""
    h, sigma = bucket_and_sign(seed, n, t)
    S = np.zeros((t, n))
    S[h, np.arange(n)] = sigma if w is None else np.asarray(w, np.float64)
    return S


def _row_values(seed: int, n: int, t: int, w, start: int = 0):
    h, sigma = bucket_and_sign(seed, n, t, start=start)
    if w is None:
        return h, sigma.astype(np.float64)
    w = np.asarray(w, dtype=np.float64)
    if w.shape != (n,):
        raise ValueError("w must have one value per row")
    return h, w


def sketch_dense(A: np.ndarray, seed: int, t: int, w=None, start: int = 0) -> np.ndarray:
    """``S A`` for a dense ``n x d`` (or length-``n``) array, float64.

    ``start`` is the global index of the first row (row shards)."""
    A = np.asarray(A)
    vec = A.ndim == 1
    A2 = A.reshape(A.shape[0], -1).astype(np.float64)
    n, d = A2.shape
    h, s = _row_values(seed, n, t, w, start)
    Y = np.zeros((t, d))
    np.add.at(Y, h, s[:, None] * A2)  # unbuffered: rows accumulate in order
    return Y[:, 0] if vec else Y


def sketch_csr(n: int, d: int, row_ptr, col_idx, val, seed: int, t: int, w=None,
               start: int = 0) -> np.ndarray:
    """``S A`` for CSR ``A`` (0-based), float64, nonzeros in storage order."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    v = np.asarray(val).astype(np.float64)
    h, s = _row_values(seed, n, t, w, start)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    flat = h[rows] * d + col_idx
    Y = np.bincount(flat, weights=s[rows] * v, minlength=t * d)
    return Y.reshape(t, d)


def sketch_bucket_rows(A_rows_of, seed: int, n: int, t: int, buckets, w=None):
    """Selected rows of ``S A`` computed one bucket at a time.

    ``A_rows_of(idx)`` returns the float64 rows ``idx`` of ``A`` as a dense
    array; used to check sampled outputs at sizes where the full sketch would
    be slow to compare."""
    h, s = _row_values(seed, n, t, w)
    out = []
    for b in np.atleast_1d(buckets):
        idx = np.nonzero(h == b)[0]
        rows = A_rows_of(idx)
        out.append((s[idx][:, None] * rows).sum(axis=0) if idx.size else np.zeros(rows.shape[1]))
    return np.stack(out)
