"""GPU parity of the second sketch stage Pi1 = F S (Section 6) and of least
squares through it, against the oracle.

Bound for F (S A): the library rounds S A to bfloat16 (as the oracle does)
and sums the products with the +-1 signs in float32 within splits of at most
t rows, then adds the splits in float64.  Each float32 sum of k terms is off
by at most gamma_k = k u / (1 - k u), u = 2^-24, times the sum of the terms'
magnitudes, so every entry obeys
``|FSA_gpu - FSA_oracle| <= gamma_t * sum_r |bf16(SA)[r, j]| / sqrt(m)``
(plus float64 rounding).  F (S b) is summed in float64 on both sides.
On integer-valued S A below 2^8 in magnitude every partial sum is an integer
below 2^24, so the float32 sums are exact and the results must agree
exactly.
"""

import numpy as np
import pytest
import torch

import oracle as O
import oracle.stage2 as S2
import workloads as W
from gpu_util import up

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_1207_6365_amd as sk

    return sk


def _bound(SA, t, m):
    u = 2.0 ** -24
    gam = t * u / (1 - t * u)
    return gam * np.abs(S2.round_bf16(SA)).sum(axis=0)[None, :] / np.sqrt(m) + 1e-300


def _sa(seed, t, d, dtype):
    g = np.random.default_rng(seed)
    SA = g.standard_normal((t, d)) * 10.0 ** g.uniform(-3, 3, size=(1, d))
    Sb = g.standard_normal(t)
    return SA.astype(dtype), Sb.astype(dtype)


# ragged tails in every direction, exact tiles, a single column and row, t
# below one 64-row step, and t spanning many splits
SHAPES = [(3000, 200, 300), (1000, 7, 20), (4096, 128, 256), (777, 1, 1), (50, 3, 3), (70000, 65, 513)]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("t,d,m", SHAPES)
def test_second_stage_matches_oracle(sk, t, d, m, dtype):
    seed = 0xABCD + t
    SA, Sb = _sa(t + d, t, d, dtype)
    FSA, FSb = sk.second_stage(up(SA), up(Sb), m, seed)
    FSA, FSb = FSA.cpu().numpy(), FSb.cpu().numpy()
    ref, ref_b = S2.second_stage(SA, Sb, seed, m)
    assert FSA.shape == (m, d) and FSb.shape == (m,)
    assert np.all(np.abs(FSA - ref) <= _bound(SA, t, m))
    sb = np.abs(Sb.astype(np.float64)).sum() / np.sqrt(m)
    assert np.all(np.abs(FSb - ref_b) <= 1e-13 * sb)


def test_second_stage_exact_on_integer_sketch(sk):
    # every partial sum is an integer below 2^24: exact in float32
    t, d, m = 5000, 96, 260
    g = np.random.default_rng(4)
    SA = g.integers(-255, 256, size=(t, d)).astype(np.float32)
    seed = 91
    FSA, _ = sk.second_stage(up(SA), None, m, seed)
    got = np.rint(FSA.cpu().numpy() * np.sqrt(m)).astype(np.int64)
    Fi = S2.sign_rows(seed, np.arange(m), t).astype(np.int64)
    assert np.array_equal(got, Fi @ SA.astype(np.int64))
    assert np.allclose(FSA.cpu().numpy() * np.sqrt(m), got, rtol=1e-15, atol=0)


def test_second_stage_benchmark_shape_sampled_rows(sk):
    # the size the least-squares benchmark runs (t = 2^18 rows of a float32
    # sketch, d = 512, m = 4 d), checked on sampled rows of F
    t, d, m = 1 << 18, 512, 2048
    g = np.random.default_rng(12)
    SA = g.standard_normal((t, d), dtype=np.float32)
    Sb = g.standard_normal(t, dtype=np.float32)
    FSA, FSb = sk.second_stage(up(SA), up(Sb), m, 5)
    rows = np.array([0, 1, 255, 256, 1023, 2047])
    ref, ref_b = S2.second_stage(SA, Sb, 5, m, rows=rows)
    got = FSA.cpu().numpy()[rows]
    assert np.all(np.abs(got - ref) <= _bound(SA, t, m))
    assert np.allclose(FSb.cpu().numpy()[rows], ref_b, rtol=0, atol=1e-12 * np.abs(Sb).sum() / np.sqrt(m))


def test_second_stage_argument_errors(sk):
    SA = up(np.zeros((100, 4)))
    with pytest.raises(sk.SklsError):
        sk.second_stage(SA, None, 0, 1)
    with pytest.raises(sk.SklsError):
        sk.second_stage(SA, None, 70000, 1)


def _resid(Ad, b, x):
    r = Ad @ np.asarray(x, np.float64) - b
    return float(np.sqrt(np.dot(r, r)))


@pytest.mark.parametrize("precision", ["plain", "mixed"])
def test_lstsq_second_stage_small(sk, precision):
    A, b, _ = W.lstsq_small()
    Ad = O.MatrixOp(A).dense()
    seed, t, m = W.sketch_seed(0), 4000, 80
    x_o, xt_o, R_o, _, ok = S2.lstsq(Ad, b, seed, t, m, delta=1e-11)
    assert ok
    x_g, info = sk.lstsq(up(Ad), up(b), t, seed, delta=1e-11, precision=precision, second_stage=m)
    assert info["certified"] == 1
    r_g, r_o = _resid(Ad, b, x_g.cpu().numpy()), _resid(Ad, b, x_o)
    assert abs(r_g / r_o - 1.0) <= 1e-10
    # sketch-and-solve start: F S A agrees to float32 summation, so x~ agrees
    # to that times the conditioning of F S A
    xs_g, _ = sk.lstsq(up(Ad), up(b), t, seed, sketch_only=True, precision="plain", second_stage=m)
    kappa = np.linalg.cond(R_o)
    assert np.max(np.abs(xs_g.cpu().numpy() - xt_o)) <= 1e-6 * kappa * np.max(np.abs(xt_o))


def test_lstsq_second_stage_heavy_rows_d512(sk):
    # the benchmark's d = 512 with m = 4 d on a row sample of the heavy-row
    # workload: parity through the certified residual, and the assumption
    # sigma_min(A R^-1) >= 0.5 checked for the oracle's R
    N, D, T, M = 1 << 15, 512, 8192, 2048
    A, b, _ = W.pareto_rows(n=N, d=D, storage="f32")
    Ad = A.astype(np.float64)
    seed = W.sketch_seed(0)
    x_o, _, R_o, _, ok = S2.lstsq(Ad, b, seed, T, M, delta=1e-11)
    assert ok
    x_g, info = sk.lstsq(up(A), up(b), T, seed, delta=1e-11, precision="mixed", second_stage=M)
    assert info["certified"] == 1
    r_g, r_o = _resid(Ad, b, x_g.cpu().numpy()), _resid(Ad, b, x_o)
    assert abs(r_g / r_o - 1.0) <= 1e-10
    assert np.linalg.svd(Ad @ np.linalg.inv(R_o), compute_uv=False).min() >= 0.5


def test_lstsq_second_stage_rejects_bad_m(sk):
    A, b, _ = W.lstsq_small()
    Ad = O.MatrixOp(A).dense()
    with pytest.raises(sk.SklsError):
        sk.lstsq(up(Ad), up(b), 4000, 1, second_stage=10)  # below d = 20
    with pytest.raises(sk.SklsError):
        sk.lstsq(up(Ad), up(b), 4000, 1, second_stage=4001)  # above t
