"""Oracle: learned per-row sketch values.

This form is not in the paper.  It keeps the random bucket map ``h`` of the
sparse embedding (Section 2) and replaces each random sign ``sigma(i)`` by a
real value ``w_i``, so ``S_w[h(i), i] = w_i``; ``w = sigma`` is the plain
sketch.  The values are trained to reduce the embedding distortion

    L(w) = || (S_w A)^T (S_w A) - A^T A ||_F^2,

the quantity whose smallness makes ``S_w`` approximate the products of the
approximate-matrix-multiplication lemma (Section 7.2).

With ``Y = S_w A`` and ``M = Y^T Y - A^T A``: ``dL/dY = 4 Y M`` and, since
row ``i`` of ``A`` enters only bucket ``h(i)`` with weight ``w_i``,
``dL/dw_i = < (4 Y M)[h(i), :], A[i, :] >``.

For random signs the expected distortion has the closed form
``E L(sigma) = (1/t) * sum_{i != j} (||a_i||^2 ||a_j||^2 + <a_i, a_j>^2)``
(the pair ``(i, j)`` contributes when the two rows share a bucket, which
happens with probability ``1/t``, and only the terms pairing ``(i,j)`` with
itself or with ``(j,i)`` survive the expectation over signs).
"""

from __future__ import annotations

import numpy as np

from .hashing import bucket_and_sign
from .sketch import sketch_dense


def distortion_loss(A: np.ndarray, seed: int, t: int, w) -> float:
    A = np.asarray(A, np.float64)
    Y = sketch_dense(A, seed, t, w)
    M = Y.T @ Y - A.T @ A
    return float((M * M).sum())


def distortion_grad(A: np.ndarray, seed: int, t: int, w):
    """``(L(w), dL/dw)``."""
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    h, _ = bucket_and_sign(seed, n, t)
    Y = sketch_dense(A, seed, t, w)
    M = Y.T @ Y - A.T @ A
    G = 4.0 * (Y @ M)
    grad = (G[h] * A).sum(axis=1)
    return float((M * M).sum()), grad


def expected_plain_distortion(A: np.ndarray, t: int) -> float:
    """Closed form of ``E L(sigma)`` over ``h`` and the signs."""
    A = np.asarray(A, np.float64)
    sq = (A * A).sum(axis=1)
    C = A.T @ A
    s4 = float((sq * sq).sum())
    return (float(sq.sum()) ** 2 - s4 + float((C * C).sum()) - s4) / t


class Adam:
    """Adam (Kingma and Ba, ICLR 2015) with bias correction, float64."""

    def __init__(self, n: int, lr: float = 1e-2, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.k = 0

    def step(self, w: np.ndarray, g: np.ndarray) -> np.ndarray:
        self.k += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mhat = self.m / (1 - self.b1 ** self.k)
        vhat = self.v / (1 - self.b2 ** self.k)
        return w - self.lr * mhat / (np.sqrt(vhat) + self.eps)
