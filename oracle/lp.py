"""Oracle: l_p regression ``min_x ||A x - b||_p`` for ``1 <= p < inf``
(Section 9: the conditioning step built on generalized sparse embeddings,
then the row-sampling algorithm of Dasgupta, Drineas, Harb, Kumar and Mahoney
(2009) that the section relies on).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the section's order:

1. ``F A`` for ``F`` block-diagonal: the rows of ``A`` are cut into blocks of
   ``w`` consecutive rows and every block is embedded by the same generalized
   sparse embedding ``S`` (Section 5 construction, ``t = a q v`` rows, rows of
   a block hashed by their index inside the block).  A last block shorter
   than ``w`` uses the first columns of ``S``.  Block ``j`` of ``F A`` is rows
   ``j t .. (j + 1) t - 1``.
2. A change of basis ``U`` that makes ``F A U`` well conditioned:
   ``U = R^{-1}`` for ``F A = Q R`` (Householder, non-negative diagonal).
   The section cites a general-``p`` basis construction without giving it;
   this is the ``p = 2`` case of the cited theorem, which is a
   well-conditioned basis for every ``p`` with factors polynomial in the
   dimensions; only the sample sizes feel them.
3. Row-norm estimates: ``l_i`` = squared row norms of ``A U Pi2`` (``Pi2`` the
   ``d x k_G`` sign matrix of :func:`oracle.lowrank.sign_projection`); the
   section estimates the l_p norms of the rows of ``A U`` from these l_2
   norms, so the sampling weight is ``lam_i = l_i^{p/2}``.
4. Stage 1: row ``i`` kept, independently, with probability
   ``pi_i = min(1, s1 lam_i / sum(lam))`` (kept iff ``u_i < pi_i``, ``u_i``
   output ``i`` of the stream ``seed ^ SAMPLE_SALT``) and weight
   ``pi_i^{-1/p}``; ``x_c`` minimises the weighted objective
   ``sum_i w_i^p |A_i x - b_i|^p`` over the kept rows.
5. Stage 2: residual ``rho = A x_c - b``; row ``i`` kept with probability
   ``min(1, s2 max(lam_i / sum(lam), |rho_i|^p / sum |rho|^p))`` (uniforms
   from the stream ``seed ^ STAGE2_SALT``; the residual share is dropped when
   ``rho = 0``) and weight ``q_i^{-1/p}``; ``x^`` minimises the stage-2
   weighted objective.

The weighted sampled problems are solved exactly: ``p = 2`` by Householder
least squares, ``p = 1`` as a linear program (SciPy's HiGHS; its
interior-point method with crossover where the default method stops
short), other ``p`` by a convex minimiser from the ``p = 2`` start (SciPy's
trust-region Newton with the exact gradient and Hessian), polished to a
vanishing gradient.
"""

from __future__ import annotations

from types import SimpleNamespace

import numpy as np

from .hashing import splitmix64
from .leverage import leverage_approx
from .linalg import apply_qt, check_rank, householder_qr, solve_upper
from .lowrank import SAMPLE_SALT, sign_projection
from .operator import MatrixOp
from .sketch import sketch_generalized

STAGE2_SALT = 0x726573616D706C65  # "resample"


def stream_uniforms(seed: int, salt: int, count: int) -> np.ndarray:
    """``u_i = (z_i >> 11) 2^-53`` for output ``i`` of SplitMix64 stream ``seed ^ salt``."""
    z = splitmix64(seed ^ salt, np.arange(count, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0**-53


def _row_block(op: MatrixOp, r0: int, r1: int):
    if op.kind == "dense":
        return op.A[r0:r1]
    a, b = int(op.row_ptr[r0]), int(op.row_ptr[r1])
    return SimpleNamespace(n=r1 - r0, d=op.d, row_ptr=op.row_ptr[r0:r1 + 1] - a, col_idx=op.col_idx[a:b],
                           val=op.val[a:b])


def block_embedding(A, seed: int, q: int, v: int, a: int, w: int = 0) -> np.ndarray:
    """``F A`` (step 1): ``ceil(n / w)`` blocks of ``t = a q v`` rows."""
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    w = op.n if w <= 0 else w
    t = a * q * v
    nb = max(1, -(-op.n // w))
    out = np.zeros((nb * t, op.d))
    for j in range(nb):
        r0, r1 = j * w, min(op.n, (j + 1) * w)
        if r1 > r0:
            out[j * t:(j + 1) * t] = sketch_generalized(_row_block(op, r0, r1), seed, q, v, a)
    return out


def condition(A, seed: int, q: int, v: int, a: int, w: int = 0) -> np.ndarray:
    """``R`` of ``F A = Q R`` (step 2); ``U = R^{-1}``."""
    _, R = householder_qr(block_embedding(A, seed, q, v, a, w))
    check_rank(R)
    return R


def row_norm_estimates(A, R: np.ndarray, seed: int, k_g: int) -> np.ndarray:
    """Squared row norms of ``A R^{-1} Pi2`` (step 3): the Section 6
    estimate of :func:`oracle.leverage.leverage_approx` with the given ``R``
    and the sign matrix ``Pi2``."""
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    return leverage_approx(op, 0, 0, sign_projection(seed, op.d, k_g), R=R)


def bernoulli_sample(prob: np.ndarray, p: float, u: np.ndarray):
    """Rows kept (``u_i < prob_i``) and their weights ``prob_i^{-1/p}``."""
    rows = np.nonzero(u < prob)[0]
    return rows, prob[rows] ** (-1.0 / p)


def lp_objective(M: np.ndarray, y: np.ndarray, x: np.ndarray, p: float) -> float:
    """``||M x - y||_p^p``."""
    return float(np.sum(np.abs(M @ x - y) ** p))


def _solve_l1(M: np.ndarray, y: np.ndarray) -> np.ndarray:
    # min 1^T e  s.t.  -e <= M x - y <= e
    from scipy.optimize import linprog
    from scipy.sparse import bmat, eye, csr_matrix

    s, d = M.shape
    Ms = csr_matrix(M)
    I = eye(s, format="csr")
    A_ub = bmat([[Ms, -I], [-Ms, -I]], format="csr")
    # HiGHS's default method can stop with an unknown status at these
    # tolerances on larger fits; its interior-point method with crossover
    # then returns an optimal vertex of the same linear program
    for method in ("highs", "highs-ipm"):
        res = linprog(np.r_[np.zeros(d), np.ones(s)], A_ub=A_ub, b_ub=np.r_[y, -y],
                      bounds=[(None, None)] * d + [(0, None)] * s, method=method,
                      options={"primal_feasibility_tolerance": 1e-10, "dual_feasibility_tolerance": 1e-10})
        if res.status == 0:
            return res.x[:d]
    raise RuntimeError(f"linprog: {res.message}")


def _solve_l2(M: np.ndarray, y: np.ndarray) -> np.ndarray:
    d = M.shape[1]
    Vs, R = householder_qr(M)
    check_rank(R)
    return solve_upper(R, apply_qt(Vs, y)[:d])


def _solve_lp_general(M: np.ndarray, y: np.ndarray, p: float) -> np.ndarray:
    from scipy.optimize import minimize

    x0 = _solve_l2(M, y)
    f0 = max(lp_objective(M, y, x0, p), 1e-300)

    def f(x):
        return np.sum(np.abs(M @ x - y) ** p) / f0

    def g(x):
        r = M @ x - y
        return p * (M.T @ (np.sign(r) * np.abs(r) ** (p - 1))) / f0

    def h(x):
        r = M @ x - y
        with np.errstate(divide="ignore"):
            wts = p * (p - 1) * np.abs(r) ** (p - 2)
        wts = np.where(np.isfinite(wts), wts, 0.0)
        return (M.T * wts) @ M / f0

    res = minimize(f, x0, jac=g, hess=h, method="trust-exact", options={"gtol": 1e-13, "maxiter": 1000})
    return res.x


def solve_weighted(M: np.ndarray, y: np.ndarray, wts: np.ndarray, p: float) -> np.ndarray:
    """``argmin_x sum_i wts_i^p |M_i x - y_i|^p`` = ``argmin ||D (M x - y)||_p``."""
    Mw = M * wts[:, None]
    yw = y * wts
    if p == 2.0:
        return _solve_l2(Mw, yw)
    if p == 1.0:
        return _solve_l1(Mw, yw)
    return _solve_lp_general(Mw, yw, p)


def lp_regression(A, b, p: float, seed: int, q: int, v: int, a: int, s1: float, s2: float, k_g: int = 32,
                  w: int = 0) -> dict:
    """Steps 1-5; returns ``x``, ``x_c``, the scores and both samples."""
    if not (p >= 1.0 and np.isfinite(p)):
        raise ValueError("need 1 <= p < inf")
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    b = np.asarray(b, dtype=np.float64)
    n = op.n
    R = condition(op, seed, q, v, a, w)
    lev = row_norm_estimates(op, R, seed, k_g)
    lam = lev ** (p / 2.0)
    share = lam / np.sum(lam)
    pi = np.minimum(1.0, s1 * share)
    rows1, w1 = bernoulli_sample(pi, p, stream_uniforms(seed, SAMPLE_SALT, n))
    if rows1.size < op.d:
        raise ValueError("stage 1 kept fewer rows than columns")
    xc = solve_weighted(op.rows(rows1), b[rows1], w1, p)
    rho = op.matvec(xc) - b
    rp = np.abs(rho) ** p
    tot = np.sum(rp)
    share2 = np.maximum(share, rp / tot) if tot > 0 else share
    q2 = np.minimum(1.0, s2 * share2)
    rows2, w2 = bernoulli_sample(q2, p, stream_uniforms(seed, STAGE2_SALT, n))
    if rows2.size < op.d:
        raise ValueError("stage 2 kept fewer rows than columns")
    x = solve_weighted(op.rows(rows2), b[rows2], w2, p)
    return {"x": x, "x_c": xc, "R": R, "scores": lev, "pi": pi, "q": q2, "rows1": rows1, "w1": w1,
            "rows2": rows2, "w2": w2}


def lp_exact(A, b, p: float) -> np.ndarray:
    """``argmin_x ||A x - b||_p`` over all rows (small inputs)."""
    op = A if isinstance(A, MatrixOp) else MatrixOp(A)
    return solve_weighted(op.dense(), np.asarray(b, dtype=np.float64), np.ones(op.n), p)
