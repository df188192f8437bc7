"""GPU parity: l_p regression (Section 9) against the oracle.

Compared on what is unique: the rows kept by each stage (integer decisions
taken in float64 on both sides; a stage-2 row may differ only where its
uniform lies within 1e-6 relative of its probability, because the stage-2
probabilities depend on the stage-1 fit), the weights, the objective values of
the weighted fits (the GPU's iterative fits against the oracle's exact ones,
to the tolerance of their stopping rules), the solutions where the fit is
unique (p > 1), and the reported objectives against float64 evaluations."""

import numpy as np
import pytest

import oracle.lp as LP
import workloads as W
from gpu_util import up, up_bf16, up_csr
from oracle.lowrank import SAMPLE_SALT
from oracle.operator import MatrixOp

pytestmark = pytest.mark.gpu

# relative tolerance of a weighted fit's objective against the exact optimum:
# the IPM stops at a duality gap of 1e-12 of the objective and the oracle's LP
# solver at feasibility 1e-10; IRLS stops once the objective moves by 1e-12
FIT_TOL = {1.0: 1e-8, 1.2: 1e-9, 1.5: 1e-9, 2.0: 1e-12, 3.0: 1e-9}


@pytest.fixture(scope="module")
def sk():
    import paper_1207_6365_amd as sk

    return sk


def _cpu(t):
    return t.cpu().numpy()


def _coreset_obj(op, b, rows, wts, x, p):
    return float(np.sum(wts ** p * np.abs(op.rows(rows) @ x - b[rows]) ** p))


def _check(got, ref, op, b, p, seed, x_unique=True):
    x, info, sm = got
    x, xc = _cpu(x), _cpu(sm["x_c"])
    r1, w1, r2, w2 = (_cpu(sm[k]) for k in ("rows1", "w1", "rows2", "w2"))
    tol = FIT_TOL[p]
    # stage 1: identical draws
    assert np.array_equal(r1, ref["rows1"])
    assert np.allclose(w1, ref["w1"], rtol=1e-12, atol=0)
    fg = _coreset_obj(op, b, r1, w1, xc, p)
    fo = _coreset_obj(op, b, ref["rows1"], ref["w1"], ref["x_c"], p)
    assert abs(fg - fo) <= tol * fo, (fg, fo)
    if x_unique:
        assert np.allclose(xc, ref["x_c"], rtol=0, atol=1e-5 * np.max(np.abs(ref["x_c"])))
    full1 = float(np.sum(np.abs(op.matvec(xc) - b) ** p))
    assert info["obj_stage1"] == pytest.approx(full1, rel=1e-10)
    # stage 2: identical up to rows whose uniform sits on their probability
    u2 = LP.stream_uniforms(seed, LP.STAGE2_SALT, op.n)
    diff = np.setxor1d(r2, ref["rows2"])
    q = ref["q"]
    assert np.all(np.abs(u2[diff] - q[diff]) <= 1e-6 * q[diff]), diff
    if diff.size == 0:
        # stage-2 weights move with the residuals at x_c: exact fits (p = 1
        # at a vertex, p = 2) agree to rounding, IRLS ones to the square root
        # of its objective tolerance
        assert np.allclose(w2, ref["w2"], rtol=1e-9 if p in (1.0, 2.0) else 1e-5, atol=0)
        fg2 = _coreset_obj(op, b, r2, w2, x, p)
        fo2 = _coreset_obj(op, b, ref["rows2"], ref["w2"], ref["x"], p)
        assert abs(fg2 - fo2) <= tol * fo2, (fg2, fo2)
        assert info["coreset_obj"] == pytest.approx(fg2, rel=1e-10)
        if x_unique:
            assert np.allclose(x, ref["x"], rtol=0, atol=1e-5 * np.max(np.abs(ref["x"])))
    full = float(np.sum(np.abs(op.matvec(x) - b) ** p))
    assert info["obj"] == pytest.approx(full, rel=1e-10)
    assert info["converged"] == 1
    return full


@pytest.mark.parametrize("p", [1.0, 1.2, 1.5, 2.0, 3.0])
def test_dense_matches_oracle(sk, p):
    A, b, _ = W.lp_dense(n=4000, d=8)
    seed, kw = 0x1234 + int(10 * p), dict(q=64, v=8, a=2, s1=400.0, s2=400.0)
    ref = LP.lp_regression(A, b, p, seed, kw["q"], kw["v"], kw["a"], kw["s1"], kw["s2"])
    got = sk.lp_regression(up(A), up(b), p, seed, samples=True, **kw)
    full = _check(got, ref, MatrixOp(A), b, p, seed, x_unique=p > 1.0)
    # the sampled fit against the exact fit over all rows
    fe = LP.lp_objective(A, b, LP.lp_exact(A, b, p), p)
    assert fe * (1 - 1e-9) <= full <= fe * 1.1 ** p


@pytest.mark.parametrize("p", [1.0, 1.5])
def test_several_factor_blocks_match_oracle(sk, p):
    # d = 130: the weighted normal systems factor in 64-column blocks with a
    # two-column last block (64 + 64 + 2), solved block by block
    A, b, _ = W.lp_dense(n=10000, d=130)
    seed, kw = 0x3150 + int(10 * p), dict(q=1000, v=8, a=1, s1=1000.0, s2=1000.0)
    ref = LP.lp_regression(A, b, p, seed, kw["q"], kw["v"], kw["a"], kw["s1"], kw["s2"])
    got = sk.lp_regression(up(A), up(b), p, seed, samples=True, **kw)
    _check(got, ref, MatrixOp(A), b, p, seed, x_unique=p > 1.0)


def test_wide_l1_fit_matches_oracle(sk):
    # d = 150 (factor blocks 64 + 64 + 22) with s1 = s2 = 1500: the oracle's
    # stage-1 fit is one where HiGHS's default method stops short and its
    # interior-point method with crossover supplies the optimal vertex
    A, b, _ = W.lp_dense(n=12000, d=150)
    seed, p, kw = 0x3150 + 10, 1.0, dict(q=1200, v=8, a=1, s1=1500.0, s2=1500.0)
    ref = LP.lp_regression(A, b, p, seed, kw["q"], kw["v"], kw["a"], kw["s1"], kw["s2"])
    got = sk.lp_regression(up(A), up(b), p, seed, samples=True, **kw)
    _check(got, ref, MatrixOp(A), b, p, seed, x_unique=False)


@pytest.mark.parametrize("row64", [False, True])
def test_csr_blocks_match_oracle(sk, row64):
    # several blocks of F with a short last block; sizes not multiples of any tile
    A, b, _ = W.lp_sparse(n=21111, d=13, k=4)
    seed, p = 0x77, 1.0
    kw = dict(q=97, v=4, a=3, w=6000, s1=500.0, s2=700.0)
    ref = LP.lp_regression(A, b, p, seed, kw["q"], kw["v"], kw["a"], kw["s1"], kw["s2"], w=kw["w"])
    got = sk.lp_regression(up_csr(A, row64=row64), up(b), p, seed, samples=True, **kw)
    _check(got, ref, MatrixOp(A), b, p, seed, x_unique=False)


@pytest.mark.parametrize("p", [1.0, 1.5])
def test_csr_with_empty_rows_matches_oracle(sk, p):
    # every seventh row empty: its score is zero, so stage 1 never draws it,
    # while stage 2 may through its residual share (the residual is -b_i)
    A0, b, _ = W.lp_sparse(n=20000, d=13, k=4)
    lens = np.diff(A0.row_ptr)
    lens[3::7] = 0
    keep = np.repeat(lens > 0, np.diff(A0.row_ptr))
    A = W.CSR(A0.n, A0.d, np.concatenate([[0], np.cumsum(lens)]).astype(np.int64), A0.col_idx[keep], A0.val[keep])
    seed = 0xE0 + int(10 * p)
    kw = dict(q=97, v=4, a=2, s1=500.0, s2=600.0)
    ref = LP.lp_regression(A, b, p, seed, kw["q"], kw["v"], kw["a"], kw["s1"], kw["s2"])
    assert not np.any(ref["rows1"] % 7 == 3)
    got = sk.lp_regression(up_csr(A), up(b), p, seed, samples=True, **kw)
    _check(got, ref, MatrixOp(A), b, p, seed, x_unique=p > 1.0)


def _check_stage2_valid(got, ref, op, b, p, seed, s2):
    """Checks for inputs whose stage-1 fit is not unique (a flat set of l_1
    minimisers): stage 1 as in _check; stage 2 must be the draw that the
    section's rule gives at the GPU's own x_c, and the final fit optimal on
    the GPU's coreset."""
    x, info, sm = got
    x, xc = _cpu(x), _cpu(sm["x_c"])
    r1, w1, r2, w2 = (_cpu(sm[k]) for k in ("rows1", "w1", "rows2", "w2"))
    tol = FIT_TOL[p]
    assert np.array_equal(r1, ref["rows1"])
    assert np.allclose(w1, ref["w1"], rtol=1e-12, atol=0)
    fg = _coreset_obj(op, b, r1, w1, xc, p)
    fo = _coreset_obj(op, b, ref["rows1"], ref["w1"], ref["x_c"], p)
    assert abs(fg - fo) <= tol * fo, (fg, fo)
    lam = ref["scores"] ** (p / 2.0)
    rp = np.abs(op.matvec(xc) - b) ** p
    q = np.minimum(1.0, s2 * np.maximum(lam / lam.sum(), rp / rp.sum()))
    u2 = LP.stream_uniforms(seed, LP.STAGE2_SALT, op.n)
    diff = np.setxor1d(r2, np.nonzero(u2 < q)[0])
    assert np.all(np.abs(u2[diff] - q[diff]) <= 1e-6 * q[diff]), diff
    if diff.size == 0:
        assert np.allclose(w2, q[r2] ** (-1.0 / p), rtol=1e-9, atol=0)
    xo = LP.solve_weighted(op.rows(r2), b[r2], w2, p)
    fg2 = _coreset_obj(op, b, r2, w2, x, p)
    fo2 = _coreset_obj(op, b, r2, w2, xo, p)
    assert abs(fg2 - fo2) <= tol * fo2, (fg2, fo2)
    assert info["coreset_obj"] == pytest.approx(fg2, rel=1e-10)
    assert info["obj"] == pytest.approx(float(np.sum(np.abs(op.matvec(x) - b) ** p)), rel=1e-10)
    assert info["converged"] == 1


@pytest.mark.parametrize("p", [1.0, 1.5])
def test_one_column_matches_oracle(sk, p):
    # d = 1: R is 1 x 1 and the fits are weighted medians (p = 1) or their
    # l_p analogues.  A weighted median can be any point of an interval, so
    # at p = 1 the stage-2 draw is checked against the GPU's own x_c
    A, b, _ = W.lp_sparse(n=6000, d=1, k=1)
    seed, kw = 0xD1 + int(10 * p), dict(q=64, v=4, a=1, s1=200.0, s2=200.0)
    ref = LP.lp_regression(A, b, p, seed, kw["q"], kw["v"], kw["a"], kw["s1"], kw["s2"])
    got = sk.lp_regression(up_csr(A), up(b), p, seed, samples=True, **kw)
    if p == 1.0:
        _check_stage2_valid(got, ref, MatrixOp(A), b, p, seed, kw["s2"])
    else:
        _check(got, ref, MatrixOp(A), b, p, seed)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_narrow_storage_matches_oracle(sk, storage):
    A, b, _ = W.lp_dense(n=3000, d=16)
    if storage == "bf16":
        bits = W.bf16_round(A.astype(np.float32))
        Ad, Ag = W.bf16_to_f32(bits).astype(np.float64), up_bf16(bits)
    else:
        Ad = A.astype(np.float32).astype(np.float64)
        Ag = up(A.astype(np.float32))
    seed, p = 5, 1.5
    kw = dict(q=128, v=4, a=1, s1=600.0, s2=600.0, k_g=16)
    ref = LP.lp_regression(Ad, b, p, seed, kw["q"], kw["v"], kw["a"], kw["s1"], kw["s2"], k_g=16)
    got = sk.lp_regression(Ag, up(b), p, seed, samples=True, **kw)
    _check(got, ref, MatrixOp(Ad), b, p, seed)


@pytest.mark.parametrize("p", [1.0, 2.5])
def test_keeping_every_row_gives_the_exact_fit(sk, p):
    A, b, _ = W.lp_dense(n=700, d=6)
    x, info = sk.lp_regression(up(A), up(b), p, 9, q=32, v=4, s1=1e30, s2=1e30)
    assert info["rows_stage1"] == 700 and info["rows_stage2"] == 700
    fe = LP.lp_objective(A, b, LP.lp_exact(A, b, p), p)
    assert info["obj"] == pytest.approx(fe, rel=FIT_TOL.get(p, 1e-9))


@pytest.mark.parametrize("p", [1.0, 1.5, 3.0])
def test_consistent_system_is_solved_exactly(sk, p):
    # b = A x0: the least-squares start already fits every row, the residual
    # share of stage 2 is empty, and x = x0
    A, _, x0 = W.lp_dense(n=2500, d=7)
    b = A @ x0
    x, info = sk.lp_regression(up(A), up(b), p, 4, q=64, v=4, s1=300.0, s2=300.0)
    assert np.allclose(x.cpu().numpy(), x0, rtol=0, atol=1e-9 * np.max(np.abs(x0)))
    assert info["converged"] == 1 and info["iters_stage1"] == 1 and info["iters_stage2"] == 1
    assert info["obj"] <= (1e-12 * np.sum(np.abs(b))) ** p * b.size
    ref = LP.lp_regression(A, b, p, 4, 64, 4, 1, 300.0, 300.0)
    assert np.allclose(ref["x"], x0, rtol=0, atol=1e-9 * np.max(np.abs(x0)))


def test_errors(sk):
    A, b, _ = W.lp_dense(n=500, d=4)
    with pytest.raises(sk.SklsError):
        sk.lp_regression(up(A), up(b), 0.9, 1)
    with pytest.raises(sk.SklsError):  # stage 1 keeps fewer rows than columns
        sk.lp_regression(up(A), up(b), 1.0, 1, q=16, v=4, s1=1.0, s2=100.0)
    A0 = A.copy()
    A0[:, 1] = 0.0
    with pytest.raises(sk.SklsError):  # F A rank deficient
        sk.lp_regression(up(A0), up(b), 1.0, 1, q=16, v=4)


def test_full_size_properties(sk):
    # the benchmark workload: CSR n = 2^22, d = 256, 16 nonzeros per row,
    # Laplace noise with 1% gross outliers, p = 1, default sizes
    A, b, x0 = W.lp_sparse()
    Ag, bg = up_csr(A), up(b)
    x, info, sm = sk.lp_regression(Ag, bg, 1.0, 0x5EED0006, samples=True)
    s1 = 32.0 * 256
    assert info["converged"] == 1
    assert 256 <= info["rows_stage1"] <= s1 + 5 * np.sqrt(s1)
    assert 256 <= info["rows_stage2"] <= 2 * s1 + 5 * np.sqrt(2 * s1)
    xg = _cpu(x)
    full = float(np.sum(np.abs(A.matvec64(xg) - b)))
    assert info["obj"] == pytest.approx(full, rel=1e-10)
    planted = float(np.sum(np.abs(A.matvec64(x0) - b)))
    print(f"l1 objective / planted {full / planted:.6f}, rows {info['rows_stage1']} + {info['rows_stage2']}")
    assert full <= 1.05 * planted
    # the kept rows carry the weights of their probabilities: at most one
    # for rows kept surely, and stage-1 uniforms below the implied probability
    w1, r1 = _cpu(sm["w1"]), _cpu(sm["rows1"])
    u1 = LP.stream_uniforms(0x5EED0006, SAMPLE_SALT, A.n)
    assert np.all(w1 >= 1.0) and np.all(u1[r1] < 1.0 / w1)
    assert np.all(np.diff(r1) > 0)


def test_l1_past_2p31_entries(sk):
    # CSR with 2^31 + 80 entries (64-bit row pointers, n = 2^27 + 5, d = 64,
    # 16 N(0,1) float32 values per row), b = A x0 + Laplace(0.1) noise, all
    # drawn on the GPU from a seeded generator and formed with torch ops.
    # Properties: the fits converge, the reported objective matches a torch
    # evaluation, and the fit is within 5% of the planted x0's objective.
    import torch

    n, d, k = (1 << 27) + 5, 64, 16
    nnz = n * k
    g = torch.Generator(device="cuda:0")
    g.manual_seed(2024)
    col = torch.randint(0, d, (nnz,), dtype=torch.int32, device="cuda:0", generator=g)
    val = torch.randn(nnz, dtype=torch.float32, device="cuda:0", generator=g)
    row_ptr = torch.arange(0, nnz + 1, k, dtype=torch.int64, device="cuda:0")
    x0 = torch.randn(d, dtype=torch.float64, device="cuda:0", generator=g)

    def times(x):
        out = torch.empty(n, dtype=torch.float64, device="cuda:0")
        for r0 in range(0, n, 1 << 24):
            r1 = min(n, r0 + (1 << 24))
            c = col[r0 * k:r1 * k].long()
            out[r0:r1] = (val[r0 * k:r1 * k].double() * x[c]).view(-1, k).sum(dim=1)
        return out

    u = torch.rand(n, dtype=torch.float64, device="cuda:0", generator=g) - 0.5
    noise = -0.1 * torch.sign(u) * torch.log1p(-2.0 * torch.abs(u))  # Laplace(0.1)
    b = times(x0) + noise
    x, info = sk.lp_regression(sk.Csr(n, d, row_ptr, col, val), b, 1.0, 0x5EED, s1=4096.0, s2=4096.0)
    assert info["converged"] == 1
    obj = float(torch.abs(times(x) - b).sum())
    assert info["obj"] == pytest.approx(obj, rel=1e-9)
    planted = float(torch.abs(noise).sum())
    assert obj <= 1.05 * planted
    del col, val, row_ptr, b, noise, u
    torch.cuda.empty_cache()
