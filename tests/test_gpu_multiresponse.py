"""GPU parity: multiple-response regression by leverage-score sampling
(Section 7, generalized-regression algorithm) against the oracle.  The draws
are decided in float64 on both sides and compared exactly; Y and the residual
within float64 rounding of the normal-equations solve."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import up, up_bf16, up_csr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_1207_6365_amd as sk

    return sk


def _rhs(A, dp, seed, noise=0.01):
    g = np.random.default_rng(seed)
    op = O.MatrixOp(A)
    return op.matmat(g.standard_normal((op.d, dp))) + noise * g.standard_normal((op.n, dp))


def _check(sk, Ag, A, B, t, t_s, seed, tol=1e-9):
    Y, info, (rows, wts) = sk.multi_lstsq(Ag, up(B), t, t_s, seed, coreset=True)
    ref = O.multi_response_lstsq(A, B, seed, t, t_s)
    ref_rows = np.nonzero(ref["counts"])[0]
    assert np.array_equal(rows.cpu().numpy(), ref_rows)
    p = ref["scores"] / ref["scores"].sum()
    ref_w = np.sqrt(ref["counts"][ref_rows] / (t_s * p[ref_rows]))
    assert np.allclose(wts.cpu().numpy(), ref_w, rtol=1e-9)
    Yg = Y.cpu().numpy()
    assert np.max(np.abs(Yg - ref["Y"])) <= tol * np.max(np.abs(ref["Y"]))
    assert info["resid_fro"] == pytest.approx(O.residual_fro(A, Yg, B), rel=1e-9)
    assert info["b_fro"] == pytest.approx(np.linalg.norm(B), rel=1e-12)
    return Yg, info


@pytest.mark.parametrize("row64", [False, True])
def test_sparse_small_workload(sk, row64):
    A, _, _ = W.lstsq_small()
    B = _rhs(A, 6, 1)
    _check(sk, up_csr(A, row64=row64), A, B, 4000, 2500, W.sketch_seed(0))


def test_sparse_with_empty_rows(sk):
    # every eleventh row empty: zero score, never drawn
    A0, _, _ = W.lstsq_small()
    lens = np.diff(A0.row_ptr)
    lens[5::11] = 0
    keep = np.repeat(lens > 0, np.diff(A0.row_ptr))
    A = W.CSR(A0.n, A0.d, np.concatenate([[0], np.cumsum(lens)]).astype(np.int64), A0.col_idx[keep], A0.val[keep])
    B = _rhs(A, 6, 3)
    _, info = _check(sk, up_csr(A), A, B, 4000, 2500, W.sketch_seed(0))
    ref = O.multi_response_lstsq(A, B, W.sketch_seed(0), 4000, 2500)
    assert not np.any(ref["counts"][5::11])


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_dense_heavy_rows(sk, storage):
    A, _, _ = W.pareto_rows(n=1 << 14, d=48, storage="f32" if storage != "bf16" else "bf16")
    if storage == "bf16":
        Ad, Ag = W.bf16_to_f32(A).astype(np.float64), up_bf16(A)
    elif storage == "f64":
        Ad = A.astype(np.float64)
        Ag = up(Ad)
    else:
        Ad, Ag = A.astype(np.float64), up(A)
    B = _rhs(Ad, 33, 2)
    _check(sk, Ag, Ad, B, 4096, 3000, 77)


@pytest.mark.parametrize("d,dp", [(68, 16), (70, 16), (36, 32)])
def test_dense_product_shapes(sk, d, dp):
    # A T (32 columns) and A Y (d' columns) on the slab kernel with a padded
    # last slab (d = 68, 36), and on the tiled GEMM when d is not a multiple
    # of 4 (d = 70); n is not a multiple of 16 rows per wavefront
    A, _, _ = W.pareto_rows(n=5003, d=d, storage="f32")
    Ad = A.astype(np.float64)
    B = _rhs(Ad, dp, 3)
    _check(sk, up(A), Ad, B, 2048, 2000, 91)


def test_consistent_system_is_solved_exactly(sk):
    A, _, _ = W.lstsq_small()
    B = _rhs(A, 4, 3, noise=0.0)
    Yg, info = _check(sk, up_csr(A), A, B, 4000, 800, 5)
    assert info["resid_fro"] <= 1e-10 * info["b_fro"]


def test_single_response_and_ragged_sizes(sk):
    A = W.csr_uniform_rows(17, 7777, 13, 3, dtype=np.float64)
    B = _rhs(A, 1, 4)
    _check(sk, up_csr(A), A, B, 1000, 999, 2**64 - 5)


def test_too_few_draws_is_reported(sk):
    A, _, _ = W.lstsq_small()
    B = _rhs(A, 2, 5)
    with pytest.raises(sk.SklsError):
        sk.multi_lstsq(up_csr(A), up(B), 4000, 10, 1)
