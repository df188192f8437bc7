"""Helpers shared by the GPU parity tests: upload seeded inputs and compare
against the oracle."""

from __future__ import annotations

import numpy as np
import torch

import oracle as O
import workloads as W


def dev():
    return torch.device("cuda:0")


def up(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev())


def up_csr(A: W.CSR, row64: bool = False, dtype=None):
    import paper_1207_6365_amd as sk

    rp = A.row_ptr if row64 else A.row_ptr32()
    val = torch.from_numpy(np.ascontiguousarray(A.val))
    if dtype is not None:
        val = val.to(dtype)
    return sk.Csr(A.n, A.d, up(rp), up(A.col_idx.astype(np.int32)), val.to(dev()))


def up_bf16(bits: np.ndarray) -> torch.Tensor:
    """bfloat16 tensor on the GPU holding the given bit patterns."""
    return torch.from_numpy(bits.view(np.int16)).to(dev()).view(torch.bfloat16)


def sketch_abs_scale(op: O.MatrixOp, seed: int, t: int) -> np.ndarray:
    """Per-entry sums of |A_ij| over each bucket: the scale of the rounding
    error of any summation order of that bucket."""
    n = op.n
    ones = np.ones(n)
    if op.kind == "csr":
        return O.sketch_csr(n, op.d, op.row_ptr, op.col_idx, np.abs(op.val), seed, t, w=ones)
    return O.sketch_dense(np.abs(op.A.astype(np.float64)), seed, t, w=ones)


def assert_sum_close(got: np.ndarray, ref: np.ndarray, scale: np.ndarray, unit: float, factor: float = 64.0):
    """|got - ref| <= factor * unit * scale elementwise (scale = sum of |terms|)."""
    err = np.abs(np.asarray(got, np.float64) - ref)
    bound = factor * unit * scale + 1e-300
    bad = err > bound
    if bad.any():
        i = np.argmax(err / bound)
        raise AssertionError(f"{bad.sum()} entries off; worst {err.flat[i]:.3e} vs bound {bound.flat[i]:.3e}")
