"""Oracle: float64 access to the input matrix ``A`` (dense or CSR)."""

from __future__ import annotations

import numpy as np


class MatrixOp:
    """Float64 products with a dense ``n x d`` array or a CSR container.

    A CSR container is any object with attributes ``n, d, row_ptr, col_idx,
    val`` (0-based).  Dense inputs of any float type are widened to float64
    block by block; row blocks never change a single row's dot product.
    """

    def __init__(self, A, block: int = 1 << 16):
        self.block = block
        if isinstance(A, np.ndarray):
            if A.ndim != 2:
                raise ValueError("dense A must be 2-D")
            self.kind = "dense"
            self.A = A
            self.n, self.d = A.shape
        else:
            self.kind = "csr"
            self.n, self.d = int(A.n), int(A.d)
            self.row_ptr = np.asarray(A.row_ptr, dtype=np.int64)
            self.col_idx = np.asarray(A.col_idx, dtype=np.int64)
            self.val = np.asarray(A.val).astype(np.float64)
            self.rows_of_nz = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))

    def _blocks(self):
        for r0 in range(0, self.n, self.block):
            r1 = min(self.n, r0 + self.block)
            yield r0, r1, self.A[r0:r1].astype(np.float64)

    def matvec(self, x) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        if self.kind == "csr":
            return np.bincount(self.rows_of_nz, weights=self.val * x[self.col_idx], minlength=self.n)
        out = np.empty(self.n)
        for r0, r1, B in self._blocks():
            out[r0:r1] = B @ x
        return out

    def rmatvec(self, y) -> np.ndarray:
        y = np.asarray(y, dtype=np.float64)
        if self.kind == "csr":
            return np.bincount(self.col_idx, weights=self.val * y[self.rows_of_nz], minlength=self.d)
        out = np.zeros(self.d)
        for r0, r1, B in self._blocks():
            out += B.T @ y[r0:r1]
        return out

    def matmat(self, X) -> np.ndarray:
        X = np.asarray(X, dtype=np.float64)
        if self.kind == "csr":
            return np.stack([self.matvec(X[:, j]) for j in range(X.shape[1])], axis=1)
        out = np.empty((self.n, X.shape[1]))
        for r0, r1, B in self._blocks():
            out[r0:r1] = B @ X
        return out

    def dense(self) -> np.ndarray:
        if self.kind == "csr":
            out = np.zeros((self.n, self.d))
            out[self.rows_of_nz, self.col_idx] = self.val
            return out
        return self.A.astype(np.float64)

    def rows(self, idx) -> np.ndarray:
        idx = np.asarray(idx, dtype=np.int64)
        if self.kind == "dense":
            return self.A[idx].astype(np.float64)
        out = np.zeros((idx.size, self.d))
        for k, i in enumerate(idx):
            a, b = self.row_ptr[i], self.row_ptr[i + 1]
            out[k, self.col_idx[a:b]] = self.val[a:b]
        return out
