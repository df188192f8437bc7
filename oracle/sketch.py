"""Oracle: applying the sparse embedding ``S = Phi D`` (Section 2) to a matrix.

``Phi`` is the ``t x n`` 0/1 matrix with ``Phi[h(i), i] = 1`` and ``D`` the
diagonal of random signs, so ``(S A)[b, :] = sum over i with h(i) = b of
sigma(i) * A[i, :]``; this is the ``O(nnz(A))`` product of the main theorem
(Section 3) and of the regression theorem in Section 7, which sketches ``A``
adjoined with ``b``.  Everything is accumulated in float64, rows in increasing
order.

The learned-value form replaces ``sigma(i)`` by a real weight ``w_i`` and
keeps ``h`` from the seed.  The generalized sparse embedding of Section 5
(a hash to groups, then a stack of independent sparse embeddings per group)
is at the end.
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


# ---------------------------------------------------------------- Section 5
COPY_STEP = 0xD1B54A32D192ED03  # stream of copy j: seed + (j + 1) * COPY_STEP (mod 2^64)


def copy_seed(seed: int, j: int) -> int:
    return (seed + (j + 1) * COPY_STEP) & 0xFFFFFFFFFFFFFFFF


def generalized_S(seed: int, n: int, q: int, v: int, a: int, order: str = "copy") -> np.ndarray:
    """Generalized sparse embedding (Section 5, the construction), written out.

    ``h`` sends row ``i`` to group ``h(i)`` (``a_g`` rows in group ``g``); ``P``
    lists the rows group by group; ``B^(g)`` stacks ``a`` copies
    ``sqrt(1/a) Phi_j D_j`` of sparse embeddings of the group's rows onto ``v``
    rows; ``S = blockdiag(B^(1), ..., B^(q)) P``.  Copy ``j`` hashes row ``i``
    with the stream ``copy_seed(seed, j)``.  ``order="block"`` keeps the rows
    of ``S`` in that block-diagonal order (group, copy, bucket);
    ``order="copy"`` lists them copy by copy (copy, group, bucket), the order
    of the GPU output.
    """
    h, _ = bucket_and_sign(seed, n, q)
    perm = np.argsort(h, kind="stable")  # P: rows grouped by h, in row order
    counts = np.bincount(h, minlength=q)
    P = np.zeros((n, n))
    P[np.arange(n), perm] = 1.0
    blocks = []
    start = 0
    for g in range(q):
        rows_g = perm[start:start + counts[g]]
        start += counts[g]
        Bg = np.zeros((a * v, counts[g]))
        for j in range(a):
            hj, sj = bucket_and_sign(copy_seed(seed, j), n, v)
            Bg[j * v + hj[rows_g], np.arange(counts[g])] = sj[rows_g] / np.sqrt(a)
        blocks.append(Bg)
    Bd = np.zeros((a * v * q, n))
    c0 = 0
    for g, Bg in enumerate(blocks):
        Bd[g * a * v:(g + 1) * a * v, c0:c0 + Bg.shape[1]] = Bg
        c0 += Bg.shape[1]
    S = Bd @ P
    if order == "block":
        return S
    # row (g, j, u) of the block order is row (j, g, u) of the copy order
    idx = np.arange(a * q * v)
    g_, rem = np.divmod(idx, a * v)
    j_, u_ = np.divmod(rem, v)
    out = np.zeros_like(S)
    out[j_ * q * v + g_ * v + u_] = S
    return out


def sketch_generalized(A, seed: int, q: int, v: int, a: int, signs: bool = True) -> np.ndarray:
    """``S A`` for the generalized sparse embedding, copy-major rows, as a sum
    over copies of signed, scaled row scatters (float64, rows in order).
    ``signs=False`` uses ``|S|`` (the scale of a sum's rounding error)."""
    from .operator import MatrixOp

    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    h, _ = bucket_and_sign(seed, op.n, q)
    out = np.zeros((a * q * v, op.d))
    for j in range(a):
        hj, sj = bucket_and_sign(copy_seed(seed, j), op.n, v)
        rows = j * q * v + h * v + hj
        w = (sj.astype(np.float64) if signs else np.ones(op.n)) / np.sqrt(a)
        if op.kind == "csr":
            nz_rows = op.rows_of_nz
            np.add.at(out, (rows[nz_rows], op.col_idx), w[nz_rows] * op.val)
        else:
            for r0, r1, B in op._blocks():
                np.add.at(out, rows[r0:r1], w[r0:r1, None] * B)
    return out
