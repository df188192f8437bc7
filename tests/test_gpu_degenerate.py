"""GPU: the one-column case (d = 1) of least squares and leverage scores on
CSR input, where R is 1 x 1 and every block loop runs once.  Least squares
is checked against its closed form x* = <a, b> / <a, a>, leverage scores
against the oracle."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import up, up_csr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_1207_6365_amd as sk

    return sk


def _one_column(n, seed):
    # about 90% of the rows hold one N(0,1) entry, the rest are empty
    g = np.random.default_rng(seed)
    full = g.random(n) < 0.9
    a = np.where(full, g.standard_normal(n), 0.0)
    lens = full.astype(np.int64)
    A = W.CSR(n, 1, np.concatenate([[0], np.cumsum(lens)]), np.zeros(int(lens.sum()), dtype=np.int32),
              a[full].astype(np.float32))
    return A, a.astype(np.float32).astype(np.float64), g


@pytest.mark.parametrize("precision", ["plain", "mixed"])
def test_lstsq_one_column(sk, precision):
    A, a, g = _one_column(5000, 11)
    b = 2.5 * a + 0.1 * g.standard_normal(A.n)
    xs = float(a @ b / (a @ a))
    x, info = sk.lstsq(up_csr(A), up(b), 64, W.sketch_seed(0), delta=1e-11, precision=precision)
    assert info["certified"] == 1
    assert float(x.cpu().numpy()[0]) == pytest.approx(xs, rel=1e-9)
    assert info["resid_norm"] == pytest.approx(float(np.linalg.norm(a * xs - b)), rel=1e-9)


def test_leverage_one_column(sk):
    A, a, _ = _one_column(5000, 12)
    seed, t, k = W.sketch_seed(0), 64, 32
    Pi2 = W.gaussian_matrix(7, 1, k, scale=1 / np.sqrt(k))
    got = sk.leverage_scores(up_csr(A), t, seed, up(Pi2)).cpu().numpy()
    ref = O.leverage_approx(O.MatrixOp(A), seed, t, Pi2)
    empty = a == 0.0
    assert np.all(got[empty] == 0.0) and np.all(ref[empty] == 0.0)
    assert np.max(np.abs(got[~empty] - ref[~empty]) / ref[~empty]) <= 1e-5
    # with one column the scores are proportional to a_i^2
    ratio = got[~empty] / a[~empty] ** 2
    assert np.max(ratio) / np.min(ratio) - 1.0 <= 1e-5
