"""GPU check of the allocation-free sketch entry point against skls_sketch:
two calls in a row (the second on a smaller input, so stale scratch contents
from the first would show), through the C ABI, plus the size limit."""

import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import up, up_csr

pytestmark = pytest.mark.gpu


def _int_csr(g, n, d, lens):
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cols = np.concatenate([np.sort(g.choice(d, size=k, replace=False)) for k in lens]).astype(np.int32)
    val = g.integers(-8, 9, size=row_ptr[-1]).astype(np.float32)
    val[val == 0] = 1
    return W.CSR(n=n, d=d, row_ptr=row_ptr, col_idx=cols, val=val)


def _noalloc(sk, Ag, t, seed, variant, b=None):
    m, dev = sk.api._matrix(Ag)
    SA = torch.full((t, m.d), float("nan"), dtype=torch.float32, device=dev)
    Sb = torch.full((t,), float("nan"), dtype=torch.float32, device=dev) if b is not None else None
    st = sk.lib().skls_sketch_noalloc(ctypes.byref(m), None if b is None else b.data_ptr(), 0, t, seed, None,
                                      sk.api._VARIANT[variant], SA.data_ptr(),
                                      None if Sb is None else Sb.data_ptr(), 1,
                                      torch.cuda.current_stream(dev).cuda_stream)
    return st, SA, Sb


@pytest.mark.parametrize("variant", ["auto", "sorted", "binned", "atomic"])
def test_noalloc_matches_sketch_twice(sk, variant):
    g = np.random.default_rng(21)
    for n, d, t in ((300000, 64, 4096), (70001, 24, 1500)):
        A = _int_csr(g, n, d, g.integers(0, 25, size=n))
        b = up(g.integers(-5, 6, size=n).astype(np.float64))
        Ag = up_csr(A)
        st, SA, Sb = _noalloc(sk, Ag, t, 77, variant, b)
        assert st == 0, sk.lib().skls_last_error()
        ref, ref_b = sk.sketch(Ag, t, 77, b=b, variant=variant)
        torch.cuda.synchronize()
        assert torch.equal(SA, ref) and torch.equal(Sb, ref_b)
        D = up(g.integers(-8, 9, size=(n // 4, d)).astype(np.float32))
        st, SD, _ = _noalloc(sk, D, t, 78, variant)
        assert st == 0
        assert torch.equal(SD, sk.sketch(D, t, 78, variant=variant))


def test_noalloc_rejects_inputs_past_its_scratch(sk):
    n = 1 << 22  # the binned plan of 2^22 rows needs about 68 MB
    A, _ = W.sketch_csr(n=n, d=16, k=2)
    st, _, _ = _noalloc(sk, up_csr(A), 65536, 1, "auto")
    assert st == 6  # SKLS_ERR_WORKSPACE
    assert b"scratch" in sk.lib().skls_last_error()


@pytest.fixture(scope="module")
def sk():
    import paper_1207_6365_amd as sk

    return sk
