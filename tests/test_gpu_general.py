"""GPU parity: the generalized sparse embedding (Section 5) against the
oracle.  Integer inputs with a = 4 (scale 1/2) match bit for bit; floating
inputs within the rounding bound of a sum in the output precision."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import assert_sum_close, up, up_csr

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U64 = 2.0 ** -53
VARIANTS = ["atomic", "sorted", "binned"]


@pytest.fixture(scope="module")
def sk():
    import paper_1207_6365_amd as sk

    return sk


@pytest.mark.parametrize("variant", VARIANTS)
def test_csr_integer_bit_exact(sk, variant):
    A, b = W.sketch_csr_int(n=50000, d=64, k=8)
    seed, q, v, a = 0x5EED0003, 256, 16, 4
    SA, Sb = sk.sketch_general(up_csr(A), q, v, a, seed, b=up(b), variant=variant)
    ref = O.sketch_generalized(A, seed, q, v, a)
    assert np.array_equal(SA.cpu().numpy().astype(np.float64), ref)
    refb = O.sketch_generalized(b[:, None].astype(np.float64), seed, q, v, a)[:, 0]
    assert np.array_equal(Sb.cpu().numpy().astype(np.float64), refb)


@pytest.mark.parametrize("variant", VARIANTS)
def test_csr_integer_ragged_and_empty_rows_bit_exact(sk, variant):
    # row lengths 0..12 (every fifth row empty) over d = 37 columns, integer
    # values: every copy's additions are exact, so the result is bit-exact
    A0, b = W.sketch_csr_int(n=30011, d=37, k=12)
    g = np.random.default_rng(5)
    lens0 = np.diff(A0.row_ptr)
    lens = np.minimum(lens0, g.integers(0, 13, A0.n))
    lens[::5] = 0
    pos = np.arange(A0.nnz) - np.repeat(A0.row_ptr[:-1], lens0)
    keep = pos < np.repeat(lens, lens0)
    A = W.CSR(A0.n, A0.d, np.concatenate([[0], np.cumsum(lens)]).astype(np.int64), A0.col_idx[keep], A0.val[keep])
    seed, q, v, a = 0x5EED0007, 97, 8, 4
    SA, Sb = sk.sketch_general(up_csr(A), q, v, a, seed, b=up(b), variant=variant)
    assert np.array_equal(SA.cpu().numpy().astype(np.float64), O.sketch_generalized(A, seed, q, v, a))
    refb = O.sketch_generalized(b[:, None].astype(np.float64), seed, q, v, a)[:, 0]
    assert np.array_equal(Sb.cpu().numpy().astype(np.float64), refb)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("out", [torch.float64, torch.float32])
def test_csr_float_within_sum_bound(sk, variant, out):
    A = W.csr_uniform_rows(41, 30011, 96, 12)
    seed, q, v, a = 7, 128, 8, 3
    SA = sk.sketch_general(up_csr(A), q, v, a, seed, variant=variant, out_dtype=out)
    ref = O.sketch_generalized(A, seed, q, v, a)
    scale = O.sketch_generalized(W.CSR(A.n, A.d, A.row_ptr, A.col_idx, np.abs(A.val)), seed, q, v, a, signs=False)
    assert_sum_close(SA.cpu().numpy(), ref, scale, U64 if out == torch.float64 else U32)


@pytest.mark.parametrize("variant", VARIANTS)
def test_dense_float_within_sum_bound(sk, variant):
    g = np.random.default_rng(5)
    A = g.standard_normal((20000, 48)).astype(np.float32)
    seed, q, v, a = 2**63 + 11, 64, 32, 2
    SA = sk.sketch_general(up(A), q, v, a, seed, variant=variant)
    ref = O.sketch_generalized(A, seed, q, v, a)
    scale = O.sketch_generalized(np.abs(A), seed, q, v, a, signs=False)
    assert_sum_close(SA.cpu().numpy(), ref, scale, U32)


def test_one_group_one_copy_is_the_plain_sketch(sk):
    A = W.csr_uniform_rows(3, 10000, 32, 5)
    seed, v = 4242, 512
    got = sk.sketch_general(up_csr(A), 1, v, 1, seed, out_dtype=torch.float64).cpu().numpy()
    ref = sk.sketch(up_csr(A), v, O.copy_seed(seed, 0), out_dtype=torch.float64).cpu().numpy()
    assert np.array_equal(got, ref)


def test_headline_sized_input_sampled_rows(sk):
    # n = 2^22, d = 256, 16 nnz/row, q v = 16384 per copy, a = 4: full output
    # checked on sampled rows of S A against the oracle's row formula
    A, _ = W.sketch_csr()
    seed, q, v, a = W.sketch_seed(0), 1024, 16, 4
    SA = sk.sketch_general(up_csr(A), q, v, a, seed).cpu().numpy()
    n = A.n
    h, _ = O.bucket_and_sign(seed, n, q)
    rng = np.random.default_rng(0)
    for j in range(a):
        hj, sj = O.bucket_and_sign(O.copy_seed(seed, j), n, v)
        tgt = j * q * v + h * v + hj
        for r in rng.choice(q * v, size=8, replace=False):
            row = j * q * v + r
            members = np.nonzero(tgt == row)[0]
            ref = np.zeros(A.d)
            sc = np.zeros(A.d)
            for i in members:
                cols = A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]
                vals = A.val[A.row_ptr[i]:A.row_ptr[i + 1]].astype(np.float64)
                ref[cols] += sj[i] * vals / np.sqrt(a)
                sc[cols] += np.abs(vals) / np.sqrt(a)
            assert np.all(np.abs(SA[row] - ref) <= 64 * U32 * sc + 1e-30)
