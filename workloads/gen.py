"""Seeded input generators (NumPy PCG64).

Every workload is synthetic.  Shapes, value distributions and sparsity follow
the workloads the sketch-and-solve method is meant for: tall ``n x d`` inputs
(the paper assumes ``n > d`` throughout), sparse rows with a fixed number of
nonzeros at uniform columns, dense rows whose norms follow a heavy-tailed
Pareto law (so that a few rows carry most of the leverage, the "heavy"
coordinates of the analysis in Section 4), and families of related matrices
for training per-row sketch values.

Inputs are rounded to their storage type here; the rounded values define the
matrix for both the oracle and the GPU path.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SKETCH_SEED_BASE = 0x5EED0000


def data_seed(config: int, trial: int = 0) -> int:
    """Seed for the data of workload ``config`` (1-based), trial ``trial``."""
    return 1000 * config + trial


def sketch_seed(trial: int = 0) -> int:
    """64-bit seed of the hash/sign generator for trial ``trial``."""
    return SKETCH_SEED_BASE + trial


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- bfloat16
def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even).

    Returns the raw 16-bit patterns as ``uint16`` (NumPy has no bfloat16).
    NaN/Inf do not occur in these workloads.
    """
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    lsb = (u >> np.uint32(16)) & np.uint32(1)
    r = (u + np.uint32(0x7FFF) + lsb) >> np.uint32(16)
    return r.astype(np.uint16)


def bf16_to_f32(bits: np.ndarray) -> np.ndarray:
    """Widen bfloat16 bit patterns to float32 (exact)."""
    return (bits.astype(np.uint32) << np.uint32(16)).view(np.float32)


# ---------------------------------------------------------------- CSR
@dataclass
class CSR:
    """Compressed sparse rows, 0-based, columns sorted and distinct per row."""

    n: int
    d: int
    row_ptr: np.ndarray  # int64[n+1]
    col_idx: np.ndarray  # int32[nnz]
    val: np.ndarray      # float64 / float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_ptr32(self) -> np.ndarray:
        if self.nnz >= 2**31:
            raise ValueError("nnz does not fit int32 row pointers")
        return self.row_ptr.astype(np.int32)

    def to_dense(self, dtype=np.float64) -> np.ndarray:
        out = np.zeros((self.n, self.d), dtype=dtype)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        out[rows, self.col_idx] = self.val
        return out

    def row_ids(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))

    def matvec64(self, x: np.ndarray) -> np.ndarray:
        """``A @ x`` in float64 (used to build right-hand sides)."""
        prod = self.val.astype(np.float64) * np.asarray(x, np.float64)[self.col_idx]
        return np.bincount(self.row_ids(), weights=prod, minlength=self.n)


def _distinct_sorted_cols(g: np.random.Generator, n: int, d: int, k: int) -> np.ndarray:
    """``n x k`` matrix of column indices, distinct and sorted within each row,
    uniform over the k-subsets of ``[0, d)`` (rejection of rows with repeats)."""
    if k > d:
        raise ValueError("more nonzeros per row than columns")
    cols = g.integers(0, d, size=(n, k), dtype=np.int32)
    cols.sort(axis=1)
    bad = np.nonzero((cols[:, 1:] == cols[:, :-1]).any(axis=1))[0] if k > 1 else np.zeros(0, np.int64)
    while bad.size:
        new = g.integers(0, d, size=(bad.size, k), dtype=np.int32)
        new.sort(axis=1)
        cols[bad] = new
        bad = bad[(new[:, 1:] == new[:, :-1]).any(axis=1)]
    return cols


def csr_uniform_rows(seed: int, n: int, d: int, k: int, dtype=np.float32,
                     values: str = "normal") -> CSR:
    """CSR matrix with exactly ``k`` distinct uniform columns in every row.

    ``values``: ``"normal"`` for N(0,1), ``"int"`` for integers drawn
    uniformly from {-8..-1, 1..8} (exact in any float format and in any
    summation order while partial sums stay small).
    """
    g = _rng(seed)
    cols = _distinct_sorted_cols(g, n, d, k)
    if values == "normal":
        val = g.standard_normal(n * k, dtype=np.float64 if dtype == np.float64 else np.float32)
    elif values == "int":
        mag = g.integers(1, 9, size=n * k, dtype=np.int32)
        sgn = g.integers(0, 2, size=n * k, dtype=np.int32) * 2 - 1
        val = (mag * sgn).astype(dtype)
    else:
        raise ValueError(values)
    row_ptr = np.arange(n + 1, dtype=np.int64) * k
    return CSR(n=n, d=d, row_ptr=row_ptr, col_idx=cols.reshape(-1), val=val.astype(dtype, copy=False))


def dense_gaussian(seed: int, n: int, d: int, dtype=np.float32) -> np.ndarray:
    g = _rng(seed)
    return g.standard_normal((n, d), dtype=np.float32 if dtype != np.float64 else np.float64).astype(dtype, copy=False)


def gaussian_matrix(seed: int, rows: int, cols: int, scale: float = 1.0) -> np.ndarray:
    """Float64 Gaussian ``rows x cols`` with entries N(0, scale^2)."""
    return _rng(seed).standard_normal((rows, cols)) * scale


# ---------------------------------------------------------------- workloads
def lstsq_small(trial: int = 0, n: int = 20000, d: int = 20, k: int = 4):
    """Small sketch-and-solve regression: CSR ``n x d`` with ``k`` N(0,1)
    float64 nonzeros per row at distinct uniform columns; ``x0 ~ N(0,I)``;
    ``b = A x0 + 0.01 N(0,1)``.  Returns ``(A, b, x0)``."""
    seed = data_seed(1, trial)
    A = csr_uniform_rows(seed, n, d, k, dtype=np.float64)
    g = _rng(seed + 500)
    x0 = g.standard_normal(d)
    b = A.matvec64(x0) + 0.01 * g.standard_normal(n)
    return A, b, x0


def sketch_csr(trial: int = 0, n: int = 2**22, d: int = 256, k: int = 16):
    """Sketch-apply workload, sparse: CSR with ``k`` float32 N(0,1) nonzeros
    per row at distinct uniform columns, plus ``b ~ N(0,1)`` float32."""
    seed = data_seed(2, trial)
    A = csr_uniform_rows(seed, n, d, k, dtype=np.float32)
    b = _rng(seed + 500).standard_normal(n, dtype=np.float32)
    return A, b


def sketch_csr_int(trial: int = 0, n: int = 2**22, d: int = 256, k: int = 16):
    """Integer-valued variant of :func:`sketch_csr` (values in {-8..8}\\{0},
    stored float32) for bit-exact comparison."""
    seed = data_seed(2, trial) + 100
    A = csr_uniform_rows(seed, n, d, k, dtype=np.float32, values="int")
    g = _rng(seed + 500)
    b = (g.integers(1, 9, size=n) * (2 * g.integers(0, 2, size=n) - 1)).astype(np.float32)
    return A, b


def sketch_dense(trial: int = 0, n: int = 2**20, d: int = 256):
    """Dense row-major float32 N(0,1) variant of the sketch-apply workload."""
    seed = data_seed(2, trial) + 200
    A = dense_gaussian(seed, n, d, np.float32)
    b = _rng(seed + 500).standard_normal(n, dtype=np.float32)
    return A, b


def pareto_rows(trial: int = 0, n: int = 2**21, d: int = 512, storage: str = "f32",
                alpha: float = 1.5, noise: float = 1e-3, chunk: int = 1 << 16):
    """Dense regression with heavy-tailed row norms.

    Row ``i`` is ``s_i * g_i / ||g_i||`` with ``g_i ~ N(0, I_d)`` and
    ``s_i ~ Pareto(alpha, x_m = 1)``, so a few rows carry leverage close
    to one.  ``x0 ~ N(0, I)`` and ``b = A x0 + noise * N(0,1)`` in float64,
    computed from the stored (rounded) ``A``.

    ``storage``: ``"f32"`` returns float32 ``A``; ``"bf16"`` returns the
    bfloat16 bit patterns (``uint16``).  Returns ``(A, b, x0)``.
    """
    seed = data_seed(3, trial)
    g = _rng(seed)
    s = 1.0 + g.pareto(alpha, size=n)
    gx = _rng(seed + 500)
    x0 = gx.standard_normal(d)
    A = np.empty((n, d), dtype=np.uint16 if storage == "bf16" else np.float32)
    b = np.empty(n)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        G = g.standard_normal((r1 - r0, d))
        G *= (s[r0:r1] / np.linalg.norm(G, axis=1))[:, None]
        G32 = G.astype(np.float32)
        if storage == "bf16":
            bits = bf16_round(G32)
            A[r0:r1] = bits
            Af = bf16_to_f32(bits).astype(np.float64)
        elif storage == "f32":
            A[r0:r1] = G32
            Af = G32.astype(np.float64)
        else:
            raise ValueError(storage)
        b[r0:r1] = Af @ x0
    b += noise * gx.standard_normal(n)
    return A, b, x0


def learned_family(num: int = 256, n: int = 32768, d: int = 64, rank: int = 16,
                   alpha: float = 1.5, noise: float = 0.05, seed: int | None = None):
    """Generator of related matrices for training per-row sketch values.

    ``A_m = diag(s) B0 Q_m + E_m`` where ``B0`` (``n x rank``, N(0,1)) and the
    Pareto(alpha) row scales ``s`` are shared by the whole family, ``Q_m`` is
    ``rank`` rows of a Haar-random orthogonal ``d x d`` matrix drawn per
    matrix, and ``E_m`` has i.i.d. N(0, noise^2) entries.  Returns a callable
    ``make(m) -> float32 (n, d)`` plus the shared scale vector.
    """
    base = data_seed(5, 0) if seed is None else seed
    g = _rng(base)
    s = 1.0 + g.pareto(alpha, size=n)
    B0 = g.standard_normal((n, rank))
    SB = s[:, None] * B0

    def make(m: int) -> np.ndarray:
        if not 0 <= m < num:
            raise IndexError(m)
        gm = _rng(base + 1 + m)
        Z = gm.standard_normal((d, d))
        Q, Rz = np.linalg.qr(Z)
        Q = Q * np.sign(np.diag(Rz))[None, :]  # Haar measure
        A = SB @ Q[:rank, :] + noise * gm.standard_normal((n, d))
        return A.astype(np.float32)

    return make, s


def learned_rhs(A: np.ndarray, m: int, noise: float = 0.01, seed: int | None = None) -> np.ndarray:
    """Right-hand side ``b = A x0 + noise N(0,1)`` (float64, from the stored
    ``A``) for matrix ``m`` of the learned-values family, ``x0 ~ N(0,1)``."""
    base = data_seed(5, 0) if seed is None else seed
    g = _rng(base + 100000 + m)
    x0 = g.standard_normal(A.shape[1])
    return A.astype(np.float64) @ x0 + noise * g.standard_normal(A.shape[0])


def planted_lowrank_sparse(trial: int = 0, n: int = 65536, rank: int = 32, density: float = 0.0085,
                           noise: float = 0.01, dtype=np.float32) -> CSR:
    """Sparse ``n x n`` matrix ``P Q^T + E``: ``P`` and ``Q`` are ``n x rank``
    with each entry nonzero with probability ``density`` (values N(0,1)), and
    ``E`` carries N(0, noise^2) values on the nonzero pattern of ``P Q^T``.

    The default density 0.0085 gives about 10 million nonzeros at
    ``n = 65536`` (the pattern of ``P Q^T`` is nonzero with probability
    ``1 - (1 - density^2)^rank``).  Columns are sorted within each row.
    """
    import scipy.sparse as sp

    g = _rng(data_seed(4, trial))

    def factor():
        mask = g.random((n, rank)) < density
        r, c = np.nonzero(mask)
        return sp.csr_matrix((g.standard_normal(r.size), (r, c)), shape=(n, rank))

    P = factor()
    Q = factor()
    M = (P @ Q.T).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    val = M.data + noise * g.standard_normal(M.data.size)
    return CSR(n, n, M.indptr.astype(np.int64), M.indices.astype(np.int32), val.astype(dtype))


def lp_sparse(trial: int = 0, n: int = 2**22, d: int = 256, k: int = 16, scale: float = 0.1,
              outliers: float = 0.01):
    """l_p regression workload: the CSR matrix of :func:`sketch_csr`'s shape
    (``k`` float32 N(0,1) nonzeros per row at distinct uniform columns),
    ``x0 ~ N(0, I)`` and ``b = A x0 + e`` in float64 with Laplace(``scale``)
    noise plus, on a fraction ``outliers`` of the rows, a gross error of
    100 ``scale`` times a standard Cauchy draw.  Returns ``(A, b, x0)``."""
    seed = data_seed(6, trial)
    A = csr_uniform_rows(seed, n, d, k, dtype=np.float32)
    g = _rng(seed + 500)
    x0 = g.standard_normal(d)
    e = g.laplace(scale=scale, size=n)
    bad = g.random(n) < outliers
    e[bad] += 100.0 * scale * g.standard_cauchy(int(bad.sum()))
    return A, A.matvec64(x0) + e, x0


def lp_dense(trial: int = 0, n: int = 4096, d: int = 16, scale: float = 0.1, outliers: float = 0.01):
    """Small dense l_p regression: float64 rows ``s_i g_i`` with ``g_i ~ N(0, I)``
    and ``s_i = exp(N(0, 1))`` (uneven row norms), ``b`` as in
    :func:`lp_sparse`.  Returns ``(A, b, x0)``."""
    g = _rng(data_seed(6, trial) + 300)
    A = g.standard_normal((n, d)) * np.exp(g.standard_normal((n, 1)))
    x0 = g.standard_normal(d)
    e = g.laplace(scale=scale, size=n)
    bad = g.random(n) < outliers
    e[bad] += 100.0 * scale * g.standard_cauchy(int(bad.sum()))
    return A, A @ x0 + e, x0
