"""The C ABI library loads and exports every entry point the header declares
(no GPU needed: only validation paths that return before any HIP call)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "skls.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"SKLS_API\s+[\w\s\*]+?\b(skls_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1207_6365_amd import _lib

    return _lib.load()


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("skls_hash", "skls_sketch", "skls_lstsq", "skls_leverage_scores", "skls_low_rank",
                 "skls_learned_grad", "skls_qr_r", "skls_sketch_general", "skls_multi_lstsq",
                 "skls_lp_regression"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1207_6365_amd import _lib

    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, name


def test_status_strings(lib):
    assert lib.skls_status_str(0) == b"SKLS_OK"
    assert lib.skls_status_str(4) == b"SKLS_ERR_RANK"
    assert lib.skls_status_str(99) == b"SKLS_ERR_UNKNOWN"


def _mat(layout=0, dtype=1, n=100, d=4, ld=4, nnz=0):
    from paper_1207_6365_amd import _lib

    m = _lib.SklsMatrix()
    m.layout, m.dtype, m.n, m.d, m.ld, m.nnz = layout, dtype, n, d, ld, nnz
    m.val = 0x1000  # never dereferenced by the workspace queries
    m.row_ptr = 0x1000
    m.col_idx = 0x1000
    return m


def test_validation_errors(lib):
    sz = ctypes.c_size_t(0)
    assert lib.skls_sketch_workspace(ctypes.byref(_mat()), 0, 0, ctypes.byref(sz)) == 2
    assert b"t=0" in lib.skls_last_error()
    assert lib.skls_sketch_workspace(ctypes.byref(_mat(dtype=7)), 8, 0, ctypes.byref(sz)) == 3
    assert lib.skls_sketch_workspace(ctypes.byref(_mat(ld=2)), 8, 0, ctypes.byref(sz)) == 2
    assert lib.skls_sketch_workspace(ctypes.byref(_mat(layout=5)), 8, 0, ctypes.byref(sz)) == 1
    assert lib.skls_sketch_workspace(ctypes.byref(_mat()), 8, 9, ctypes.byref(sz)) == 1
    assert lib.skls_sketch_workspace(None, 8, 0, ctypes.byref(sz)) == 1
    assert lib.skls_sketch_workspace(ctypes.byref(_mat()), 2**31, 0, ctypes.byref(sz)) == 2


def test_workspace_sizes(lib):
    sz = ctypes.c_size_t(0)
    # atomic variant needs no workspace; sorted needs the bucket plan
    assert lib.skls_sketch_workspace(ctypes.byref(_mat(n=1000)), 64, 1, ctypes.byref(sz)) == 0
    assert sz.value == 0
    assert lib.skls_sketch_workspace(ctypes.byref(_mat(n=1000)), 64, 2, ctypes.byref(sz)) == 0
    assert sz.value >= 4 * (2 * 1000 + 2 * 64)
    from paper_1207_6365_amd import _lib

    o = _lib.SklsLstsqOpts()
    o.t = 2  # t < d
    assert lib.skls_lstsq_workspace(ctypes.byref(_mat(n=1000)), ctypes.byref(o), ctypes.byref(sz)) == 2
    o.t = 64
    assert lib.skls_lstsq_workspace(ctypes.byref(_mat(n=1000)), ctypes.byref(o), ctypes.byref(sz)) == 0
    assert sz.value > 64 * 4 * 8
    o.precision = 3
    assert lib.skls_lstsq_workspace(ctypes.byref(_mat(n=1000)), ctypes.byref(o), ctypes.byref(sz)) == 1
    assert lib.skls_qr_r_workspace(10, 20, ctypes.byref(sz)) == 2


def test_learned_batch_workspace_and_argument_checks(lib):
    # every check below fails before any device call
    from paper_1207_6365_amd import _lib as L

    sz = ctypes.c_size_t(0)
    A = _mat(n=32768, d=64, ld=64)
    assert lib.skls_learned_batch_workspace(ctypes.byref(A), 1024, ctypes.byref(sz)) == 0
    # four lanes, each with Y = S_w A (t x d floats), plus four gradient slots
    assert sz.value >= 4 * 1024 * 64 * 4 + 4 * 32768 * 4
    assert lib.skls_learned_batch_workspace(ctypes.byref(A), 0, ctypes.byref(sz)) == 2
    desc = L.SklsSketchPlanDesc()
    desc.n, desc.d, desc.t, desc.layout, desc.out_dtype = 32768, 64, 1024, 0, 1
    mats = (L.SklsMatrix * 2)(A, A)
    cps = (ctypes.c_void_p * 2)(0x1000, 0x1000)
    args = (ctypes.byref(desc), 0x1000, 1 << 20, 0x1000, 0, 0x1000, 0x1000, 0x1000, 1 << 30, None)
    assert lib.skls_learned_grad_batch(0, mats, cps, None, *args) == 1  # count 0
    assert lib.skls_learned_grad_batch(2, mats, None, None, *args) == 1  # no targets
    desc.n = 1000  # the plan is for another shape
    assert lib.skls_learned_grad_batch(2, mats, cps, None, *args) == 2
    assert b"plan" in lib.skls_last_error()
    desc.n = 32768
    bf = (L.SklsMatrix * 1)(_mat(n=32768, d=64, ld=64, dtype=2))  # bfloat16 A
    assert lib.skls_learned_grad_batch(1, bf, cps, None, *args) == 3


def test_learned_batch_binding_checks_lists():
    import paper_1207_6365_amd.api as api

    with pytest.raises(ValueError):
        api.learned_grad_batch([], [], None, None, None)
    with pytest.raises(ValueError):
        api.learned_grad_batch([object()], [], None, None, None)


def test_low_rank_workspace_checks_options(lib):
    from paper_1207_6365_amd import _lib as L

    sz = ctypes.c_size_t(0)
    A = _mat(n=5000, d=300, ld=300)
    o = L.SklsLowRankOpts()
    o.k, o.t_r, o.seed = 4, 32, 1
    assert lib.skls_low_rank_workspace(ctypes.byref(A), ctypes.byref(o), ctypes.byref(sz)) == 0
    assert sz.value > 5000 * 32 * 8
    o.k = 0
    assert lib.skls_low_rank_workspace(ctypes.byref(A), ctypes.byref(o), ctypes.byref(sz)) == 1
    o.k, o.t_r, o.eps = 4, 0, 0.0  # neither t_r nor eps
    assert lib.skls_low_rank_workspace(ctypes.byref(A), ctypes.byref(o), ctypes.byref(sz)) == 1
    o.eps = 0.25  # t_r = max(ceil(k / eps), k + 16), capped by min(n, m)
    assert lib.skls_low_rank_workspace(ctypes.byref(A), ctypes.byref(o), ctypes.byref(sz)) == 0
    o.t_r, o.t_s = 32, 16  # fewer draws than t_r
    assert lib.skls_low_rank_workspace(ctypes.byref(A), ctypes.byref(o), ctypes.byref(sz)) == 1
    o.t_s, o.k = 0, 60
    assert lib.skls_low_rank_workspace(ctypes.byref(A), ctypes.byref(o), ctypes.byref(sz)) == 1


def test_lp_workspace_checks_options(lib):
    from paper_1207_6365_amd import _lib as L

    sz = ctypes.c_size_t(0)
    A = _mat(n=5000, d=16, ld=16)
    o = L.SklsLpOpts()
    o.p, o.seed = 1.0, 3
    assert lib.skls_lp_regression_workspace(ctypes.byref(A), ctypes.byref(o), ctypes.byref(sz)) == 0
    # F A (2 d^2 rows by default) and the coreset of capacity 2 s2 + 8 sqrt(2 s2) + 64
    assert sz.value > 512 * 16 * 8 + 1024 * 16 * 8 * 2
    for bad_p in (0.5, float("inf"), float("nan")):
        o.p = bad_p
        assert lib.skls_lp_regression_workspace(ctypes.byref(A), ctypes.byref(o), ctypes.byref(sz)) == 1
    o.p, o.k_g = 1.5, 65
    assert lib.skls_lp_regression_workspace(ctypes.byref(A), ctypes.byref(o), ctypes.byref(sz)) == 1
    o.k_g, o.w, o.q, o.v = 0, 100, 2, 4  # 50 blocks of 8 rows
    assert lib.skls_lp_regression_workspace(ctypes.byref(A), ctypes.byref(o), ctypes.byref(sz)) == 0
    o.w = 5000  # one block of 8 rows cannot hold d = 16
    assert lib.skls_lp_regression_workspace(ctypes.byref(A), ctypes.byref(o), ctypes.byref(sz)) == 2
    assert lib.skls_lp_regression_workspace(ctypes.byref(_mat(n=10, d=16, ld=16)), ctypes.byref(o),
                                            ctypes.byref(sz)) == 2


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1207_6365_amd import _lib

    with pytest.raises(ImportError):
        _lib._lib_saved = _lib._lib
        try:
            _lib._lib = None
            _lib.load(str(tmp_path / "missing.so"))
        finally:
            _lib._lib = _lib._lib_saved
