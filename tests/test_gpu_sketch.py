"""GPU parity: hash/sign (bit-exact) and the sketch S A, S b against the
oracle (Section 2).  Integer-valued inputs must match bit for bit; floating
inputs within the rounding bound of a sum in the output precision."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import assert_sum_close, dev, sketch_abs_scale, up, up_bf16, up_csr

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def sk():
    import paper_1207_6365_amd as sk

    return sk


@pytest.mark.parametrize("n,t,seed,start", [
    (100000, 4000, W.sketch_seed(0), 0),
    (70001, 65536, 123, 5),
    (5000, 1, 7, 0),
    (5000, 2**31 - 1, 2**64 - 1, 1000),
    (1, 3, 0, 2**40),
    (0, 5, 1, 0),
])
def test_hash_bit_exact(sk, n, t, seed, start):
    b, s = sk.hash_rows(n, t, seed, start=start)
    h_o, s_o = O.bucket_and_sign(seed, n, t, start=start)
    assert np.array_equal(b.cpu().numpy().astype(np.int64), h_o)
    assert np.array_equal(s.cpu().numpy(), s_o)


VARIANTS = ["atomic", "sorted", "binned"]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("out", [torch.float64, torch.float32])
def test_csr_f64_small_workload(sk, variant, out):
    A, b, _ = W.lstsq_small()
    seed, t = W.sketch_seed(0), 4000
    SA, Sb = sk.sketch(up_csr(A), t, seed, b=up(b), variant=variant, out_dtype=out)
    op = O.MatrixOp(A)
    ref = O.sketch_matrix(op, seed, t)
    unit = U64 if out == torch.float64 else U32
    assert_sum_close(SA.cpu().numpy(), ref, sketch_abs_scale(op, seed, t), unit)
    refb = O.sketch_dense(b, seed, t)
    scb = O.sketch_dense(np.abs(b), seed, t, w=np.ones(len(b)))
    assert_sum_close(Sb.cpu().numpy(), refb, scb, unit)


@pytest.mark.parametrize("variant", VARIANTS)
def test_csr_integer_bit_exact(sk, variant):
    A, b = W.sketch_csr_int(n=50000, d=64, k=8)
    seed, t = 99, 2048
    SA, Sb = sk.sketch(up_csr(A), t, seed, b=up(b), variant=variant)
    ref = O.sketch_csr(A.n, A.d, A.row_ptr, A.col_idx, A.val, seed, t)
    assert np.array_equal(SA.cpu().numpy().astype(np.float64), ref)
    assert np.array_equal(Sb.cpu().numpy().astype(np.float64), O.sketch_dense(b, seed, t))


@pytest.mark.parametrize("variant", VARIANTS)
def test_csr_f32_tolerance_and_ragged_rows(sk, variant):
    # variable row lengths (0..40 nonzeros, some empty rows), int64 row pointers
    g = np.random.default_rng(5)
    n, d = 30000, 100
    lens = g.integers(0, 41, size=n)
    lens[::97] = 0
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cols = np.concatenate([np.sort(g.choice(d, size=k, replace=False)) for k in lens]).astype(np.int32)
    val = g.standard_normal(row_ptr[-1]).astype(np.float32)
    A = W.CSR(n=n, d=d, row_ptr=row_ptr, col_idx=cols, val=val)
    seed, t = 4242, 777
    SA = sk.sketch(up_csr(A, row64=True), t, seed, variant=variant)
    op = O.MatrixOp(A)
    ref = O.sketch_matrix(op, seed, t)
    got = SA.cpu().numpy()
    assert_sum_close(got, ref, sketch_abs_scale(op, seed, t), U32)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("storage,d,ld", [("f32", 40, 40), ("f32", 37, 37), ("f32", 64, 70), ("bf16", 64, 64),
                                          ("bf16", 30, 30), ("f64", 24, 24), ("f32", 4, 4), ("f32", 100, 100),
                                          ("f32", 128, 128)])
def test_dense_storage_types(sk, variant, storage, d, ld):
    n, t, seed = 20000, 900, 31337
    g = np.random.default_rng(d)
    X = g.standard_normal((n, ld)).astype(np.float32)
    if storage == "bf16":
        bits = W.bf16_round(X)
        Ag = up_bf16(bits)[:, :d]
        Ad = W.bf16_to_f32(bits)[:, :d]
    elif storage == "f64":
        Xd = g.standard_normal((n, ld))
        Ad = Xd[:, :d]
        Ag = up(Xd)[:, :d]
    else:
        Ad = X[:, :d]
        Ag = up(X)[:, :d]
    b = g.standard_normal(n)
    out = torch.float64 if storage == "f64" else torch.float32
    SA, Sb = sk.sketch(Ag, t, seed, b=up(b), variant=variant, out_dtype=out)
    op = O.MatrixOp(np.ascontiguousarray(Ad))
    ref = O.sketch_matrix(op, seed, t)
    unit = U64 if out == torch.float64 else U32
    assert_sum_close(SA.cpu().numpy(), ref, sketch_abs_scale(op, seed, t), unit)
    assert_sum_close(Sb.cpu().numpy(), O.sketch_dense(b, seed, t), O.sketch_dense(np.abs(b), seed, t, w=np.ones(n)),
                     unit)


@pytest.mark.parametrize("variant", VARIANTS)
def test_learned_values_replace_signs(sk, variant):
    n, d, t, seed = 10000, 32, 300, 5
    g = np.random.default_rng(1)
    A = g.standard_normal((n, d)).astype(np.float32)
    w = g.standard_normal(n).astype(np.float32)
    SA = sk.sketch(up(A), t, seed, w=up(w), variant=variant)
    ref = O.sketch_dense(A, seed, t, w=w.astype(np.float64))
    scale = O.sketch_dense(np.abs(A).astype(np.float64), seed, t, w=np.abs(w).astype(np.float64))
    assert_sum_close(SA.cpu().numpy(), ref, scale, U32)


@pytest.mark.parametrize("variant", VARIANTS)
def test_edge_cases(sk, variant):
    # empty input: every row of S A is written as zero
    E = torch.zeros((0, 8), dtype=torch.float32, device=dev())
    SA = sk.sketch(E, 16, 1, variant=variant)
    assert torch.count_nonzero(SA).item() == 0
    # t = 1: signed sum of all rows
    A = np.random.default_rng(2).integers(-3, 4, size=(5000, 16)).astype(np.float32)
    SA = sk.sketch(up(A), 1, 77, variant=variant)
    _, s = O.bucket_and_sign(77, 5000, 1)
    assert np.array_equal(SA.cpu().numpy()[0].astype(np.float64), s.astype(np.float64) @ A.astype(np.float64))
    # buckets far larger than the in-LDS sort capacity
    A = np.random.default_rng(3).integers(-8, 9, size=(40000, 12)).astype(np.float32)
    SA = sk.sketch(up(A), 7, 11, variant=variant)
    assert np.array_equal(SA.cpu().numpy().astype(np.float64), O.sketch_dense(A, 11, 7))


def _int_csr(g, n, d, lens):
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cols = np.concatenate([np.sort(g.choice(d, size=k, replace=False)) for k in lens]).astype(np.int32)
    val = g.integers(-8, 9, size=row_ptr[-1]).astype(np.float32)
    val[val == 0] = 1
    return W.CSR(n=n, d=d, row_ptr=row_ptr, col_idx=cols, val=val)


def _shifted_csr(A: W.CSR, row64: bool):
    """The same matrix with column and value arrays starting 4 bytes into
    their allocations (no 16-byte groups of nonzeros)."""
    import paper_1207_6365_amd as sk

    rp = A.row_ptr if row64 else A.row_ptr32()
    col = torch.zeros(A.col_idx.size + 1, dtype=torch.int32, device=dev())
    val = torch.zeros(A.val.size + 1, dtype=torch.float32, device=dev())
    col[1:] = up(A.col_idx.astype(np.int32))
    val[1:] = up(A.val)
    return sk.Csr(A.n, A.d, up(rp), col[1:], val[1:])


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("shift", [False, True])
def test_csr_gather_paths_bit_exact(sk, variant, shift):
    """Integer-valued CSR through every gather path: rows whose lengths are
    multiples of four (grouped loads when aligned), long rows that overflow
    the position table (binary search), crowded buckets (binned: several
    blocks per bin; sorted: buckets past the in-LDS sort) and an empty
    input."""
    g = np.random.default_rng(11)
    n, d = 6000, 512
    lens = 4 * g.integers(0, 101, size=n)  # 0..400 nonzeros, multiples of 4
    lens[::13] = 0
    A = _int_csr(g, n, d, lens)
    for row64 in (False, True):
        Ag = _shifted_csr(A, row64) if shift else up_csr(A, row64=row64)
        for t, seed in ((501, 3), (3, 8)):
            SA = sk.sketch(Ag, t, seed, variant=variant)
            ref = O.sketch_csr(A.n, A.d, A.row_ptr, A.col_idx, A.val, seed, t)
            assert np.array_equal(SA.cpu().numpy().astype(np.float64), ref), (row64, t)
    # ragged lengths, many rows per bucket, b folded into the plan
    lens = g.integers(0, 23, size=200000)
    B = _int_csr(g, 200000, 40, lens)
    b = g.integers(-5, 6, size=200000).astype(np.float64)
    Bg = _shifted_csr(B, False) if shift else up_csr(B)
    SA, Sb = sk.sketch(Bg, 5, 21, b=up(b), variant=variant)
    assert np.array_equal(SA.cpu().numpy().astype(np.float64),
                          O.sketch_csr(B.n, B.d, B.row_ptr, B.col_idx, B.val, 21, 5))
    assert np.array_equal(Sb.cpu().numpy().astype(np.float64), O.sketch_dense(b, 21, 5))
    # empty CSR: S A is all zeros
    E = W.CSR(n=0, d=16, row_ptr=np.zeros(1, np.int64), col_idx=np.zeros(0, np.int32),
              val=np.zeros(0, np.float32))
    SA = sk.sketch(up_csr(E), 40, 1, variant=variant)
    assert SA.shape == (40, 16) and torch.count_nonzero(SA).item() == 0


def test_sorted_variant_is_deterministic(sk):
    A, b = W.sketch_csr(n=200000, d=64, k=8)
    Ag = up_csr(A)
    r1 = sk.sketch(Ag, 5000, 3, variant="sorted")
    r2 = sk.sketch(Ag, 5000, 3, variant="sorted")
    assert torch.equal(r1, r2)
    D = up(np.random.default_rng(4).standard_normal((100000, 48)).astype(np.float32))
    assert torch.equal(sk.sketch(D, 3000, 9, variant="sorted"), sk.sketch(D, 3000, 9, variant="sorted"))


def test_argument_errors(sk):
    A = up(np.ones((10, 4), np.float32))
    with pytest.raises(sk.SklsError):
        sk.sketch(A, 0, 1)
    with pytest.raises(sk.SklsError):
        sk.sketch(A, 2**31, 1)


# ----------------------------------------------------------- full-size workloads
@pytest.mark.parametrize("variant", VARIANTS)
def test_full_size_integer_csr_bit_exact(sk, variant):
    A, b = W.sketch_csr_int()
    seed, t = W.sketch_seed(0), 65536
    SA, Sb = sk.sketch(up_csr(A), t, seed, b=up(b), variant=variant)
    ref = O.sketch_csr(A.n, A.d, A.row_ptr, A.col_idx, A.val, seed, t)
    assert np.array_equal(SA.cpu().numpy().astype(np.float64), ref)
    assert np.array_equal(Sb.cpu().numpy().astype(np.float64), O.sketch_dense(b.astype(np.float64), seed, t))


@pytest.mark.parametrize("variant", ["binned", "sorted"])
def test_full_size_f32_csr(sk, variant):
    A, b = W.sketch_csr()
    seed, t = W.sketch_seed(0), 65536
    SA = sk.sketch(up_csr(A), t, seed, variant=variant).cpu().numpy()
    op = O.MatrixOp(A)
    ref = O.sketch_matrix(op, seed, t)
    assert np.linalg.norm(SA - ref) <= 1e-5 * np.linalg.norm(ref)
    assert_sum_close(SA, ref, sketch_abs_scale(op, seed, t), U32)


def test_full_size_dense_sampled_buckets(sk):
    A, b = W.sketch_dense()
    seed, t = W.sketch_seed(0), 65536
    SA = sk.sketch(up(A), t, seed).cpu().numpy()
    buckets = np.random.default_rng(0).choice(t, size=64, replace=False)
    ref = O.sketch_bucket_rows(lambda idx: A[idx].astype(np.float64), seed, A.shape[0], t, buckets)
    scale = O.sketch_bucket_rows(lambda idx: np.abs(A[idx]).astype(np.float64), seed, A.shape[0], t, buckets,
                                 w=np.ones(A.shape[0]))
    assert_sum_close(SA[buckets], ref, scale, U32)


def test_int64_row_pointers_past_2p31_entries(sk):
    # 2^31 + 80 stored entries (16 per row, n = 2^27 + 5 rows, d = 64): the
    # entry offsets only fit 64-bit row pointers.  Integer values keep every
    # bucket sum exact in float32, so sampled rows of S A are compared bit for
    # bit with the oracle's per-bucket sums.  The entries are drawn on the GPU
    # from a seeded generator (17 GB; drawing them on the host would take
    # minutes).
    n, d, k, t = (1 << 27) + 5, 64, 16, 4096
    nnz = n * k
    assert nnz > 2**31
    g = torch.Generator(device=dev())
    g.manual_seed(12345)
    col = torch.randint(0, d, (nnz,), dtype=torch.int32, device=dev(), generator=g)
    mag = torch.randint(1, 9, (nnz,), dtype=torch.int8, device=dev(), generator=g)
    sgn = torch.randint(0, 2, (nnz,), dtype=torch.int8, device=dev(), generator=g)
    val = (mag * (2 * sgn - 1)).to(torch.float32)
    del mag, sgn
    row_ptr = torch.arange(0, nnz + 1, k, dtype=torch.int64, device=dev())
    seed = W.sketch_seed(3)
    SA = sk.sketch(sk.Csr(n, d, row_ptr, col, val), t, seed).cpu().numpy().astype(np.float64)

    def rows_of(idx):
        if len(idx) == 0:
            return np.zeros((0, d))
        it = torch.from_numpy(np.asarray(idx, dtype=np.int64)).to(dev())
        ent = (it[:, None] * k + torch.arange(k, device=dev())[None, :]).reshape(-1)
        c = col[ent].cpu().numpy()
        v = val[ent].cpu().numpy().astype(np.float64)
        out = np.zeros((len(idx), d))
        np.add.at(out, (np.repeat(np.arange(len(idx)), k), c), v)
        return out

    buckets = np.array([0, 1234, t - 1])
    ref = O.sketch_bucket_rows(rows_of, seed, n, t, buckets)
    assert np.array_equal(SA[buckets], ref)
    del col, val, row_ptr
    torch.cuda.empty_cache()
