"""GPU parity: sketches of row blocks with global row offsets (S A = sum of
S A_g over row blocks, the linearity of Phi D in Section 2) and reusable
bucket plans (h depends only on the seed, the row index and t), against the
oracle and against the one-call sketch.  Integer-valued inputs make every
comparison exact, whatever the order of the additions."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import up, up_csr

pytestmark = pytest.mark.gpu

VARIANTS = ["atomic", "sorted", "binned"]


@pytest.fixture(scope="module")
def sk():
    import paper_1207_6365_amd as sk

    return sk


def _int_csr(g, n, d, lens):
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cols = np.concatenate([np.sort(g.choice(d, size=k, replace=False)) for k in lens]).astype(np.int32)
    val = g.integers(-8, 9, size=row_ptr[-1]).astype(np.float32)
    val[val == 0] = 1
    return W.CSR(n=n, d=d, row_ptr=row_ptr, col_idx=cols, val=val)


def _rows(A: W.CSR, r0: int, r1: int) -> W.CSR:
    p0, p1 = A.row_ptr[r0], A.row_ptr[r1]
    return W.CSR(n=r1 - r0, d=A.d, row_ptr=A.row_ptr[r0:r1 + 1] - p0, col_idx=A.col_idx[p0:p1], val=A.val[p0:p1])


@pytest.mark.parametrize("variant", VARIANTS)
def test_row_shards_sum_to_the_whole_csr(sk, variant):
    g = np.random.default_rng(5)
    n, d, t, seed = 90001, 64, 3001, W.sketch_seed(2)
    A = _int_csr(g, n, d, g.integers(0, 17, size=n))
    b = g.integers(-6, 7, size=n).astype(np.float64)
    whole, whole_b = sk.sketch(up_csr(A), t, seed, b=up(b), variant=variant, out_dtype=torch.float64)
    cuts = [0, 20000, 20001, 90001]  # a one-row shard in the middle
    total = torch.zeros_like(whole)
    total_b = torch.zeros_like(whole_b)
    for r0, r1 in zip(cuts[:-1], cuts[1:]):
        part, part_b = sk.sketch(up_csr(_rows(A, r0, r1)), t, seed, b=up(b[r0:r1]), variant=variant,
                                 out_dtype=torch.float64, row_start=r0)
        ref = O.sketch_csr(r1 - r0, d, _rows(A, r0, r1).row_ptr, _rows(A, r0, r1).col_idx, _rows(A, r0, r1).val,
                           seed, t, start=r0)
        assert np.array_equal(part.cpu().numpy(), ref)
        assert np.array_equal(part_b.cpu().numpy(), O.sketch_dense(b[r0:r1], seed, t, start=r0))
        total += part
        total_b += part_b
    assert torch.equal(total, whole)
    assert torch.equal(total_b, whole_b)
    assert np.array_equal(whole.cpu().numpy(), O.sketch_csr(n, d, A.row_ptr, A.col_idx, A.val, seed, t))


@pytest.mark.parametrize("variant", VARIANTS)
def test_row_shards_sum_to_the_whole_dense(sk, variant):
    g = np.random.default_rng(6)
    n, d, t, seed = 50000, 40, 777, 99
    A = g.integers(-8, 9, size=(n, d)).astype(np.float32)
    whole = sk.sketch(up(A), t, seed, variant=variant)
    total = torch.zeros_like(whole)
    for r0, r1 in ((0, 12345), (12345, 40000), (40000, n)):
        part = sk.sketch(up(A[r0:r1]), t, seed, variant=variant, row_start=r0)
        assert np.array_equal(part.cpu().numpy().astype(np.float64), O.sketch_dense(A[r0:r1], seed, t, start=r0))
        total += part
    assert torch.equal(total, whole)


@pytest.mark.parametrize("variant", VARIANTS)
def test_plan_reused_across_csr_values(sk, variant):
    # one plan for the row pointers; two matrices with those rows, new
    # columns and values; with b (gathered during the reduce) and learned w
    g = np.random.default_rng(7)
    n, d, t, seed = 120000, 96, 5003, W.sketch_seed(3)
    lens = g.integers(0, 21, size=n)
    lens[::17] = 0
    A1 = _int_csr(g, n, d, lens)
    A2 = _int_csr(g, n, d, lens)
    assert np.array_equal(A1.row_ptr, A2.row_ptr)
    for out in (torch.float32, torch.float64):
        plan = sk.sketch_plan(up_csr(A1), t, seed, variant=variant, out_dtype=out, row_start=10)
        assert plan.desc.variant in (1, 2, 3) and plan.desc.row_start == 10
        for A in (A1, A2):
            Ag = up_csr(A)
            b = g.integers(-5, 6, size=n).astype(np.float64)
            w = g.integers(-3, 4, size=n).astype(np.float32)
            SA, Sb = sk.sketch_planned(plan, Ag, b=up(b))
            ref = O.sketch_csr(n, d, A.row_ptr, A.col_idx, A.val, seed, t, start=10)
            assert np.array_equal(SA.cpu().numpy().astype(np.float64), ref)
            assert np.array_equal(Sb.cpu().numpy().astype(np.float64), O.sketch_dense(b, seed, t, start=10))
            SW = sk.sketch_planned(plan, Ag, w=up(w))
            assert np.array_equal(SW.cpu().numpy().astype(np.float64),
                                  O.sketch_csr(n, d, A.row_ptr, A.col_idx, A.val, seed, t, w=w, start=10))
            one = sk.sketch(Ag, t, seed, variant=variant, out_dtype=out, row_start=10)
            assert torch.equal(one, SA)


@pytest.mark.parametrize("variant", VARIANTS)
def test_plan_reused_across_dense_matrices(sk, variant):
    g = np.random.default_rng(8)
    n, d, t, seed = 60000, 48, 2048, 5
    plan = sk.sketch_plan(up(np.zeros((n, d), np.float32)), t, seed, variant=variant)
    for _ in range(2):
        A = g.integers(-8, 9, size=(n, d)).astype(np.float32)
        b = g.integers(-5, 6, size=n).astype(np.float32)
        SA, Sb = sk.sketch_planned(plan, up(A), b=up(b))
        assert np.array_equal(SA.cpu().numpy().astype(np.float64), O.sketch_dense(A, seed, t))
        assert np.array_equal(Sb.cpu().numpy().astype(np.float64), O.sketch_dense(b.astype(np.float64), seed, t))


def test_plan_of_the_benchmark_dense_shape_is_bit_identical(sk):
    # float inputs: the sorted schedule is reproducible, so the planned
    # reduce equals the one-call sketch bit for bit
    D, _ = W.sketch_dense(n=1 << 18)
    Dg = up(D)
    plan = sk.sketch_plan(Dg, 65536, W.sketch_seed(0), variant="sorted")
    assert torch.equal(sk.sketch_planned(plan, Dg), sk.sketch(Dg, 65536, W.sketch_seed(0), variant="sorted"))


def test_plan_mismatch_is_rejected(sk):
    g = np.random.default_rng(9)
    A = _int_csr(g, 1000, 16, g.integers(1, 5, size=1000))
    plan = sk.sketch_plan(up_csr(A), 64, 1)
    B = _int_csr(g, 999, 16, g.integers(1, 5, size=999))
    with pytest.raises(sk.SklsError) as e:
        sk.sketch_planned(plan, up_csr(B))
    assert e.value.status == 2
    with pytest.raises(sk.SklsError):
        sk.sketch(up_csr(A), 64, 1, row_start=-1)


def test_learned_grad_with_a_shared_plan(sk):
    # one plan for a family of matrices of one shape: loss and gradient equal
    # those of the call that builds its own plan (the sorted schedule is
    # reproducible), for two matrices and two value vectors
    make, _ = W.learned_family(num=4, n=8192, d=32)
    t, seed = 512, W.sketch_seed(4)
    mats = [up(make(m)) for m in range(2)]
    plan = sk.sketch_plan(mats[0], t, seed, variant="sorted")
    g = np.random.default_rng(10)
    for A in mats:
        C = sk.gram(A)
        for w in (up(np.sign(g.standard_normal(8192)).astype(np.float32)),
                  up(g.standard_normal(8192).astype(np.float32))):
            l1, g1 = sk.learned_grad(A, C, t, seed, w)
            l2, g2 = sk.learned_grad(A, C, t, seed, w, plan=plan)
            assert torch.equal(l1, l2) and torch.equal(g1, g2)
