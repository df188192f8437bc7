"""Entry points reject a workspace smaller than their query with
SKLS_ERR_WORKSPACE before launching anything (C ABI, real device pointers)."""

import ctypes

import pytest
import torch

import workloads as W
from gpu_util import dev, up

pytestmark = pytest.mark.gpu

WORKSPACE = 6  # SKLS_ERR_WORKSPACE


@pytest.fixture(scope="module")
def env():
    import paper_1207_6365_amd as sk
    from paper_1207_6365_amd import _lib as L
    from paper_1207_6365_amd import api

    A, b, _ = W.lp_dense(n=3000, d=8)
    Ag, bg = up(A), up(b)
    m, _ = api._matrix(Ag)
    small = torch.empty(16, dtype=torch.uint8, device=dev())
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev()).cuda_stream)
    return sk, L, m, Ag, bg, small, stream


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def test_lstsq(env):
    sk, L, m, Ag, bg, small, stream = env
    o = L.SklsLstsqOpts()
    o.t, o.seed = 256, 1
    x = torch.empty(8, dtype=torch.float64, device=dev())
    info = L.SklsLstsqInfo()
    st = sk.lib().skls_lstsq(ctypes.byref(m), _ptr(bg), ctypes.byref(o), _ptr(x), ctypes.byref(info), _ptr(small),
                             16, stream)
    assert st == WORKSPACE and b"workspace" in sk.lib().skls_last_error()


def test_multi_lstsq(env):
    sk, L, m, Ag, bg, small, stream = env
    o = L.SklsMultiOpts()
    o.t, o.t_s, o.seed = 256, 200, 1
    B = bg.reshape(-1, 1).contiguous()
    Y = torch.empty((8, 1), dtype=torch.float64, device=dev())
    info = L.SklsMultiInfo()
    st = sk.lib().skls_multi_lstsq(ctypes.byref(m), _ptr(B), 1, ctypes.byref(o), _ptr(Y), None, None,
                                   ctypes.byref(info), _ptr(small), 16, stream)
    assert st == WORKSPACE


def test_lp_regression(env):
    sk, L, m, Ag, bg, small, stream = env
    o = L.SklsLpOpts()
    o.p, o.seed, o.q, o.v = 1.0, 1, 32, 4
    x = torch.empty(8, dtype=torch.float64, device=dev())
    info = L.SklsLpInfo()
    st = sk.lib().skls_lp_regression(ctypes.byref(m), _ptr(bg), ctypes.byref(o), _ptr(x), None, None, None, None,
                                     None, ctypes.byref(info), _ptr(small), 16, stream)
    assert st == WORKSPACE


def test_low_rank(env):
    sk, L, m, Ag, bg, small, stream = env
    o = L.SklsLowRankOpts()
    o.k, o.t_r, o.seed = 2, 6, 1
    Lm = torch.empty((3000, 2), dtype=torch.float64, device=dev())
    D = torch.empty(2, dtype=torch.float64, device=dev())
    Wm = torch.empty((8, 2), dtype=torch.float64, device=dev())
    info = L.SklsLowRankInfo()
    st = sk.lib().skls_low_rank(ctypes.byref(m), ctypes.byref(o), _ptr(Lm), _ptr(D), _ptr(Wm), ctypes.byref(info),
                                _ptr(small), 16, stream)
    assert st == WORKSPACE
