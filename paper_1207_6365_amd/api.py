"""Python binding of libskls: argument marshalling only.

Every function turns torch tensors (device memory owned by the caller) into
plain pointers and sizes, asks the library for its workspace size, allocates
the workspace as a torch byte tensor and calls the C entry point on the
current HIP stream.  All arithmetic runs in the library's HIP kernels.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L

_DTYPE = {torch.float64: L.F64, torch.float32: L.F32, torch.bfloat16: L.BF16}
_VARIANT = {"auto": L.SKETCH_AUTO, "atomic": L.SKETCH_ATOMIC, "sorted": L.SKETCH_SORTED,
            "binned": L.SKETCH_BINNED}


@dataclass
class Csr:
    """CSR matrix on the GPU: ``row_ptr`` int32/int64 ``[n+1]``, ``col_idx``
    int32 ``[nnz]``, ``val`` float64/float32/bfloat16 ``[nnz]``."""

    n: int
    d: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    val: torch.Tensor

    @property
    def device(self):
        return self.val.device


def _ptr(t: torch.Tensor | None) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors passed to skls must live on the GPU")
    return t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _matrix(A) -> tuple[L.SklsMatrix, torch.device]:
    m = L.SklsMatrix()
    if isinstance(A, Csr):
        if A.row_ptr.dtype not in (torch.int32, torch.int64) or A.col_idx.dtype != torch.int32:
            raise TypeError("CSR row_ptr must be int32/int64 and col_idx int32")
        if A.val.dtype not in _DTYPE:
            raise TypeError(f"unsupported value dtype {A.val.dtype}")
        for t in (A.row_ptr, A.col_idx, A.val):
            if not t.is_contiguous():
                raise ValueError("CSR arrays must be contiguous")
        m.layout = L.CSR
        m.dtype = _DTYPE[A.val.dtype]
        m.n, m.d, m.ld = A.n, A.d, A.d
        m.nnz = A.col_idx.numel()
        m.row_ptr = _ptr(A.row_ptr)
        m.row_ptr_64 = 1 if A.row_ptr.dtype == torch.int64 else 0
        m.col_idx = _ptr(A.col_idx)
        m.val = _ptr(A.val)
        return m, A.val.device
    if not isinstance(A, torch.Tensor) or A.dim() != 2:
        raise TypeError("A must be a 2-D torch tensor or a Csr")
    if A.dtype not in _DTYPE:
        raise TypeError(f"unsupported dtype {A.dtype}")
    if A.stride(1) != 1:
        raise ValueError("dense A must be row-major (unit column stride)")
    m.layout = L.DENSE
    m.dtype = _DTYPE[A.dtype]
    m.n, m.d = A.shape
    m.ld = A.stride(0) if A.shape[0] > 1 else A.shape[1]
    m.val = _ptr(A)
    return m, A.device


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _size(fn, *args) -> int:
    out = ctypes.c_size_t(0)
    L.check(fn(*args, ctypes.byref(out)))
    return out.value


def lib():
    return L.load()


def version() -> str:
    return lib().skls_version().decode()


# ------------------------------------------------------------------ a1
def hash_rows(n: int, t: int, seed: int, start: int = 0, device="cuda"):
    """Bucket ``h(i)`` (int32) and sign (int8, +-1) for rows ``start..start+n-1``."""
    device = torch.device(device)
    bucket = torch.empty(n, dtype=torch.int32, device=device)
    sign = torch.empty(n, dtype=torch.int8, device=device)
    L.check(lib().skls_hash(n, t, seed & 0xFFFFFFFFFFFFFFFF, start, _ptr(bucket), _ptr(sign), _stream(device)))
    return bucket, sign


# ------------------------------------------------------------------ a2
def _sketch_inputs(m, b, w):
    if b is not None and (b.dtype not in (torch.float64, torch.float32) or not b.is_contiguous()):
        raise TypeError("b must be a contiguous float64/float32 vector")
    if b is not None and b.numel() != m.n:
        raise ValueError("b must have n entries")
    if w is not None and (w.dtype != torch.float32 or not w.is_contiguous() or w.numel() != m.n):
        raise TypeError("w must be a contiguous float32 vector of n entries")


def sketch(A, t: int, seed: int, b: torch.Tensor | None = None, w: torch.Tensor | None = None,
           variant: str = "auto", out_dtype=torch.float32, row_start: int = 0):
    """``S A`` (and ``S b`` when ``b`` is given); ``w`` replaces the signs.
    ``row_start``: global index of ``A``'s first row (a block of a taller
    matrix), by which its rows are hashed."""
    m, device = _matrix(A)
    if out_dtype not in (torch.float64, torch.float32):
        raise TypeError("out_dtype must be float64 or float32")
    _sketch_inputs(m, b, w)
    v = _VARIANT[variant]
    ws = _workspace(_size(lib().skls_sketch_workspace, ctypes.byref(m), t, v), device)
    SA = torch.empty((t, m.d), dtype=out_dtype, device=device)
    Sb = torch.empty(t, dtype=out_dtype, device=device) if b is not None else None
    L.check(lib().skls_sketch_rows(ctypes.byref(m), row_start, _ptr(b), _DTYPE[b.dtype] if b is not None else L.F64,
                                   t, seed & 0xFFFFFFFFFFFFFFFF, _ptr(w), v, _ptr(SA), _ptr(Sb), _DTYPE[out_dtype],
                                   _ptr(ws), ws.numel(), _stream(device)))
    return (SA, Sb) if b is not None else SA


@dataclass
class SketchPlan:
    """A reusable bucket plan: the device buffer and its descriptor."""

    buf: torch.Tensor
    desc: L.SklsSketchPlanDesc


def sketch_plan(A, t: int, seed: int, variant: str = "auto", out_dtype=torch.float32,
                row_start: int = 0) -> SketchPlan:
    """Build the bucket plan of ``A``'s rows (row pointers for CSR) once."""
    m, device = _matrix(A)
    if out_dtype not in (torch.float64, torch.float32):
        raise TypeError("out_dtype must be float64 or float32")
    v = _VARIANT[variant]
    od = _DTYPE[out_dtype]
    buf = _workspace(_size(lib().skls_sketch_plan_workspace, ctypes.byref(m), t, v, od), device)
    desc = L.SklsSketchPlanDesc()
    L.check(lib().skls_sketch_plan(ctypes.byref(m), row_start, t, seed & 0xFFFFFFFFFFFFFFFF, v, od, _ptr(buf),
                                   buf.numel(), ctypes.byref(desc), _stream(device)))
    return SketchPlan(buf, desc)


def sketch_planned(plan: SketchPlan, A, b: torch.Tensor | None = None, w: torch.Tensor | None = None,
                   SA: torch.Tensor | None = None, Sb: torch.Tensor | None = None):
    """``S A`` (and ``S b``) with a plan from :func:`sketch_plan`."""
    m, device = _matrix(A)
    _sketch_inputs(m, b, w)
    od = torch.float64 if plan.desc.out_dtype == L.F64 else torch.float32
    if SA is None:
        SA = torch.empty((plan.desc.t, m.d), dtype=od, device=device)
    if b is not None and Sb is None:
        Sb = torch.empty(plan.desc.t, dtype=od, device=device)
    L.check(lib().skls_sketch_planned(ctypes.byref(m), _ptr(b), _DTYPE[b.dtype] if b is not None else L.F64, _ptr(w),
                                      _ptr(SA), _ptr(Sb), ctypes.byref(plan.desc), _ptr(plan.buf), plan.buf.numel(),
                                      _stream(device)))
    return (SA, Sb) if b is not None else SA


def sketch_general(A, q: int, v: int, a: int, seed: int, b: torch.Tensor | None = None, variant: str = "auto",
                   out_dtype=torch.float32):
    """Generalized sparse embedding (Section 5): ``S A`` with ``a q v`` rows,
    copy-major (row ``j q v + h(i) v + h_j(i)``), and ``S b`` when ``b`` is given."""
    m, device = _matrix(A)
    if out_dtype not in (torch.float64, torch.float32):
        raise TypeError("out_dtype must be float64 or float32")
    if b is not None and (b.dtype not in (torch.float64, torch.float32) or not b.is_contiguous()
                          or b.numel() != m.n):
        raise TypeError("b must be a contiguous float64/float32 vector of n entries")
    vv = _VARIANT[variant]
    ws = _workspace(_size(lib().skls_sketch_general_workspace, ctypes.byref(m), q, v, vv), device)
    t = a * q * v
    SA = torch.empty((t, m.d), dtype=out_dtype, device=device)
    Sb = torch.empty(t, dtype=out_dtype, device=device) if b is not None else None
    L.check(lib().skls_sketch_general(ctypes.byref(m), _ptr(b), _DTYPE[b.dtype] if b is not None else L.F64, q, v, a,
                                      seed & 0xFFFFFFFFFFFFFFFF, vv, _ptr(SA), _ptr(Sb), _DTYPE[out_dtype],
                                      _ptr(ws), ws.numel(), _stream(device)))
    return (SA, Sb) if b is not None else SA


# ------------------------------------------------------------------ a3
def qr_r(M: torch.Tensor, inverse: bool = True):
    """``R`` (and ``R^{-1}``) of a QR factorisation of a tall ``m x d`` matrix."""
    if M.dim() != 2 or M.dtype not in (torch.float64, torch.float32) or not M.is_contiguous():
        raise TypeError("M must be a contiguous 2-D float64/float32 tensor")
    mm, d = M.shape
    ws = _workspace(_size(lib().skls_qr_r_workspace, mm, d), M.device)
    R = torch.empty((d, d), dtype=torch.float64, device=M.device)
    Rinv = torch.empty((d, d), dtype=torch.float64, device=M.device) if inverse else None
    L.check(lib().skls_qr_r(_ptr(M), _DTYPE[M.dtype], mm, d, _ptr(R), _ptr(Rinv), _ptr(ws), ws.numel(),
                            _stream(M.device)))
    return (R, Rinv) if inverse else R


# ------------------------------------------------------------------ a3 + a4
def lstsq(A, b: torch.Tensor, t: int, seed: int, delta: float = 1e-6, precision: str = "plain",
          sigma_lb: float = 0.5, max_iter: int = 100, sketch_only: bool = False, variant: str = "auto",
          w: torch.Tensor | None = None, raise_noconv: bool = True, x0: torch.Tensor | None = None,
          max_retries: int = 0, second_stage: int = 0):
    """Least squares ``min ||A x - b||``: sketch-and-solve, then R-preconditioned
    LSQR to a certified residual ratio ``<= 1 + delta``.  ``x0``: start of the
    iteration in place of the sketch-and-solve solution; ``max_retries``:
    extra attempts with a new sketch after a failed one; ``second_stage = m``:
    take R from ``F (S A)`` (m rows, see :func:`second_stage`) instead of
    ``S A``.  Returns ``(x, info)``."""
    m, device = _matrix(A)
    if b.dtype != torch.float64 or not b.is_contiguous() or b.numel() != m.n:
        raise TypeError("b must be a contiguous float64 vector with n entries")
    if x0 is not None and (x0.dtype != torch.float64 or not x0.is_contiguous() or x0.numel() != m.d):
        raise TypeError("x0 must be a contiguous float64 vector with d entries")
    o = L.SklsLstsqOpts()
    o.t, o.seed, o.delta, o.sigma_lb, o.max_iter = t, seed & 0xFFFFFFFFFFFFFFFF, delta, sigma_lb, max_iter
    o.precision = {"plain": 0, "mixed": 1}[precision]
    o.sketch_only = 1 if sketch_only else 0
    o.variant = _VARIANT[variant]
    o.w = _ptr(w)
    o.x0 = _ptr(x0)
    o.max_retries = max_retries
    o.second_stage = second_stage
    ws = _workspace(_size(lib().skls_lstsq_workspace, ctypes.byref(m), ctypes.byref(o)), device)
    x = torch.empty(m.d, dtype=torch.float64, device=device)
    info = L.SklsLstsqInfo()
    st = lib().skls_lstsq(ctypes.byref(m), _ptr(b), ctypes.byref(o), _ptr(x), ctypes.byref(info), _ptr(ws),
                          ws.numel(), _stream(device))
    out = {f: getattr(info, f) for f, _ in L.SklsLstsqInfo._fields_ if f != "reserved"}
    out["status"] = L.STATUS.get(st, st)
    if st != 0 and not (st == 5 and not raise_noconv):
        L.check(st)
    return x, out


def second_stage(SA: torch.Tensor, Sb: torch.Tensor | None, m: int, seed: int):
    """``(F SA, F Sb)`` for the m x t sign matrix F of the second sketch
    stage (float64 results; ``Sb`` may be None, then the second is None).
    ``SA``: contiguous float64/float32 ``[t, d]``; ``Sb`` the same dtype ``[t]``."""
    if SA.dim() != 2 or SA.dtype not in (torch.float64, torch.float32) or not SA.is_contiguous():
        raise TypeError("SA must be a contiguous float64/float32 matrix")
    t, d = SA.shape
    if Sb is not None and (Sb.dtype != SA.dtype or not Sb.is_contiguous() or Sb.numel() != t):
        raise TypeError("Sb must be a contiguous vector of SA's dtype with t entries")
    ws = _workspace(_size(lib().skls_second_stage_workspace, t, d, m), SA.device)
    FSA = torch.empty(m, d, dtype=torch.float64, device=SA.device)
    FSb = torch.empty(m, dtype=torch.float64, device=SA.device) if Sb is not None else None
    L.check(lib().skls_second_stage(_ptr(SA), _ptr(Sb), _DTYPE[SA.dtype], t, d, m, seed & 0xFFFFFFFFFFFFFFFF,
                                    _ptr(FSA), _ptr(FSb), _ptr(ws), ws.numel(), _stream(SA.device)))
    return FSA, FSb


def multi_lstsq(A, B: torch.Tensor, t: int, t_s: int, seed: int, k_g: int = 0, coreset: bool = False):
    """Multiple-response regression ``min_Y ||A Y - B||_F`` by leverage-score
    sampling (Section 7, generalized-regression algorithm).  Returns ``(Y,
    info)``, plus the coreset ``(rows, weights)`` when ``coreset``."""
    m, device = _matrix(A)
    if B.dtype != torch.float64 or not B.is_contiguous() or B.dim() != 2 or B.shape[0] != m.n:
        raise TypeError("B must be a contiguous float64 n x d' tensor")
    dp = B.shape[1]
    o = L.SklsMultiOpts()
    o.t, o.t_s, o.seed, o.k_g = t, t_s, seed & 0xFFFFFFFFFFFFFFFF, k_g
    ws = _workspace(_size(lib().skls_multi_lstsq_workspace, ctypes.byref(m), dp, ctypes.byref(o)), device)
    Y = torch.empty((m.d, dp), dtype=torch.float64, device=device)
    cap = min(m.n, t_s)
    rows = torch.empty(cap, dtype=torch.int32, device=device) if coreset else None
    wts = torch.empty(cap, dtype=torch.float64, device=device) if coreset else None
    info = L.SklsMultiInfo()
    L.check(lib().skls_multi_lstsq(ctypes.byref(m), _ptr(B), dp, ctypes.byref(o), _ptr(Y), _ptr(rows), _ptr(wts),
                                   ctypes.byref(info), _ptr(ws), ws.numel(), _stream(device)))
    out = {f: getattr(info, f) for f, _ in L.SklsMultiInfo._fields_ if f != "reserved"}
    if coreset:
        k = out["rows_sampled"]
        return Y, out, (rows[:k], wts[:k])
    return Y, out


def lp_regression(A, b: torch.Tensor, p: float, seed: int, q: int = 0, v: int = 0, a: int = 0, w: int = 0,
                  s1: float = 0.0, s2: float = 0.0, k_g: int = 0, max_iter: int = 0, tol: float = 0.0,
                  samples: bool = False):
    """``l_p`` regression ``min_x ||A x - b||_p`` (Section 9: conditioning by a
    block-diagonal generalized sparse embedding, then two-stage row sampling
    and weighted ``l_p`` fits of the samples).  Returns ``(x, info)``, plus a
    dict with ``x_c`` and the rows and weights of both stages when
    ``samples``."""
    m, device = _matrix(A)
    if b.dtype != torch.float64 or not b.is_contiguous() or b.dim() != 1 or b.shape[0] != m.n:
        raise TypeError("b must be a contiguous float64 vector of length n")
    o = L.SklsLpOpts()
    o.p, o.q, o.v, o.a, o.k_g, o.w = float(p), q, v, a, k_g, w
    o.s1, o.s2, o.seed, o.max_iter, o.tol = float(s1), float(s2), seed & 0xFFFFFFFFFFFFFFFF, max_iter, float(tol)
    ws = _workspace(_size(lib().skls_lp_regression_workspace, ctypes.byref(m), ctypes.byref(o)), device)
    x = torch.empty(m.d, dtype=torch.float64, device=device)
    extra = None
    if samples:
        extra = {"x_c": torch.empty(m.d, dtype=torch.float64, device=device),
                 "rows1": torch.empty(m.n, dtype=torch.int32, device=device),
                 "w1": torch.empty(m.n, dtype=torch.float64, device=device),
                 "rows2": torch.empty(m.n, dtype=torch.int32, device=device),
                 "w2": torch.empty(m.n, dtype=torch.float64, device=device)}
    g = (lambda k: _ptr(extra[k])) if samples else (lambda k: None)
    info = L.SklsLpInfo()
    L.check(lib().skls_lp_regression(ctypes.byref(m), _ptr(b), ctypes.byref(o), _ptr(x), g("x_c"), g("rows1"),
                                     g("w1"), g("rows2"), g("w2"), ctypes.byref(info), _ptr(ws), ws.numel(),
                                     _stream(device)))
    out = {f: getattr(info, f) for f, _ in L.SklsLpInfo._fields_ if not f.startswith("reserved")}
    if samples:
        k1, k2 = out["rows_stage1"], out["rows_stage2"]
        for key, k in (("rows1", k1), ("w1", k1), ("rows2", k2), ("w2", k2)):
            extra[key] = extra[key][:k]
        return x, out, extra
    return x, out


# ------------------------------------------------------------------ a5
def leverage_scores(A, t: int, seed: int, Pi2: torch.Tensor | None = None, k: int = 32,
                    R: torch.Tensor | None = None):
    """Squared row norms of ``A R^{-1} Pi2`` (Section 6).  ``Pi2``: ``d x k``
    float64, or None for the seeded ``d x k`` sign matrix of the library.
    ``R``: a ``d x d`` float64 upper-triangular factor to use instead of the
    one of ``S A`` (``t`` is then unused)."""
    m, device = _matrix(A)
    if Pi2 is not None:
        if Pi2.dtype != torch.float64 or not Pi2.is_contiguous() or Pi2.dim() != 2 or Pi2.shape[0] != m.d:
            raise TypeError("Pi2 must be a contiguous float64 d x k tensor")
        k = Pi2.shape[1]
    scores = torch.empty(m.n, dtype=torch.float32, device=device)
    sd = seed & 0xFFFFFFFFFFFFFFFF
    if R is not None:
        if R.dtype != torch.float64 or not R.is_contiguous() or tuple(R.shape) != (m.d, m.d):
            raise TypeError("R must be a contiguous float64 d x d tensor")
        ws = _workspace(_size(lib().skls_leverage_from_r_workspace, ctypes.byref(m), k), device)
        L.check(lib().skls_leverage_scores_from_r(ctypes.byref(m), _ptr(R), k, _ptr(Pi2), sd, _ptr(scores),
                                                  _ptr(ws), ws.numel(), _stream(device)))
        return scores
    ws = _workspace(_size(lib().skls_leverage_workspace, ctypes.byref(m), t, k), device)
    L.check(lib().skls_leverage_scores(ctypes.byref(m), t, sd, k, _ptr(Pi2), _ptr(scores),
                                       _ptr(ws), ws.numel(), _stream(device)))
    return scores


# ------------------------------------------------------------------ a6
def gram(A: torch.Tensor) -> torch.Tensor:
    """``A^T A`` (float32 result) of a dense matrix."""
    m, device = _matrix(A)
    ws = _workspace(_size(lib().skls_gram_workspace, ctypes.byref(m)), device)
    C = torch.empty((m.d, m.d), dtype=torch.float32, device=device)
    L.check(lib().skls_gram(ctypes.byref(m), _ptr(C), _ptr(ws), ws.numel(), _stream(device)))
    return C


class LearnedWorkspace:
    """Reusable workspace for :func:`learned_grad` at one ``(n, d, t)``."""

    def __init__(self, A: torch.Tensor, t: int):
        m, device = _matrix(A)
        self.key = (m.n, m.d, t)
        self.buf = _workspace(_size(lib().skls_learned_workspace, ctypes.byref(m), t), device)


def learned_grad(A: torch.Tensor, C: torch.Tensor, t: int, seed: int, w: torch.Tensor,
                 ws: LearnedWorkspace | None = None, loss: torch.Tensor | None = None,
                 grad: torch.Tensor | None = None, grad_scale: float = 1.0, accumulate: bool = False,
                 want_grad: bool = True, plan: SketchPlan | None = None):
    """Distortion loss ``||(S_w A)^T S_w A - C||_F^2`` and ``grad_scale`` times its
    gradient in ``w`` (added into ``grad`` when ``accumulate``).  ``plan``: a
    reusable plan of :func:`sketch_plan` for ``A``'s shape, ``t`` and
    ``seed`` (float32 output), so that the forward sketch runs without
    rebuilding it."""
    m, device = _matrix(A)
    if ws is None or ws.key != (m.n, m.d, t):
        ws = LearnedWorkspace(A, t)
    loss = torch.empty(1, dtype=torch.float32, device=device) if loss is None else loss
    if want_grad and grad is None:
        grad = torch.empty(m.n, dtype=torch.float32, device=device)
    if accumulate and grad is None:
        raise ValueError("accumulate needs a grad buffer")
    if plan is not None:
        if plan.desc.t != t or plan.desc.seed != seed & 0xFFFFFFFFFFFFFFFF:
            raise ValueError("the plan was built for another t or seed")
        L.check(lib().skls_learned_grad_planned(ctypes.byref(m), _ptr(C), ctypes.byref(plan.desc), _ptr(plan.buf),
                                                plan.buf.numel(), _ptr(w), grad_scale, 1 if accumulate else 0,
                                                _ptr(loss), _ptr(grad) if want_grad else None, _ptr(ws.buf),
                                                ws.buf.numel(), _stream(device)))
        return loss, (grad if want_grad else None)
    L.check(lib().skls_learned_grad(ctypes.byref(m), _ptr(C), t, seed & 0xFFFFFFFFFFFFFFFF, _ptr(w), grad_scale,
                                    1 if accumulate else 0, _ptr(loss), _ptr(grad) if want_grad else None,
                                    _ptr(ws.buf), ws.buf.numel(), _stream(device)))
    return loss, (grad if want_grad else None)


class LearnedBatchWorkspace:
    """Reusable workspace for :func:`learned_grad_batch` at one ``(n, d, t)``."""

    def __init__(self, A: torch.Tensor, t: int):
        m, device = _matrix(A)
        self.key = (m.n, m.d, t)
        self.buf = _workspace(_size(lib().skls_learned_batch_workspace, ctypes.byref(m), t), device)


def learned_grad_batch(mats, grams, plan: SketchPlan, w: torch.Tensor, grad: torch.Tensor | None,
                       scale=None, ws: LearnedBatchWorkspace | None = None, loss: torch.Tensor | None = None,
                       accumulate: bool = False):
    """Losses of the matrices ``mats`` (one shape, float32) against their Gram
    targets ``grams`` and the sum of their gradients in ``w`` weighted by
    ``scale`` (one float per matrix; default 1), written to ``grad`` (added
    when ``accumulate``; ``None``: the losses only).  The forward sketches run from the reusable
    ``plan``; the matrices' chains run on several streams at once.  Returns
    ``(loss, grad)`` with ``loss`` a float32 device vector of the raw loss of
    each matrix."""
    if len(mats) != len(grams) or not mats:
        raise ValueError("need one Gram target per matrix and at least one matrix")
    count = len(mats)
    if scale is not None and len(scale) != count:
        raise ValueError("need one weight per matrix")
    descs = [_matrix(A) for A in mats]
    device = descs[0][1]
    m0 = descs[0][0]
    if not isinstance(ws, LearnedBatchWorkspace) or ws.key != (m0.n, m0.d, plan.desc.t):
        ws = LearnedBatchWorkspace(mats[0], plan.desc.t)
    loss = torch.empty(count, dtype=torch.float32, device=device) if loss is None else loss
    if loss.numel() < count or loss.dtype != torch.float32:
        raise ValueError("loss must be a float32 vector with one entry per matrix")
    arr = (L.SklsMatrix * count)(*[m for m, _ in descs])
    cps = (ctypes.c_void_p * count)(*[_ptr(C) for C in grams])
    sc = None if scale is None else (ctypes.c_float * count)(*[float(x) for x in scale])
    L.check(lib().skls_learned_grad_batch(count, arr, cps, sc, ctypes.byref(plan.desc), _ptr(plan.buf),
                                          plan.buf.numel(), _ptr(w), 1 if accumulate else 0, _ptr(loss),
                                          _ptr(grad), _ptr(ws.buf), ws.buf.numel(), _stream(device)))
    return loss, grad


def adam_step(w: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float = 1e-2,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    """In-place Adam update of ``w`` (float32 device vectors)."""
    for t in (w, g, m, v):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != w.numel():
            raise TypeError("Adam buffers must be contiguous float32 vectors of equal length")
    L.check(lib().skls_adam_step(w.numel(), _ptr(w), _ptr(g), _ptr(m), _ptr(v), step, lr, beta1, beta2, eps,
                                 _stream(w.device)))


def low_rank_opts(k: int, seed: int, eps: float = 0.0, t_r: int = 0, t_s: int = 0, k_g: int = 0,
                  oversample: int = 0, max_iter: int = 0, tol: float = 0.0) -> L.SklsLowRankOpts:
    o = L.SklsLowRankOpts()
    o.k, o.t_r, o.t_s, o.seed, o.eps = k, t_r, t_s, seed & 0xFFFFFFFFFFFFFFFF, eps
    o.k_g, o.oversample, o.max_iter, o.tol = k_g, oversample, max_iter, tol
    return o


def low_rank(A, k: int, seed: int, eps: float = 0.0, t_r: int = 0, t_s: int = 0, k_g: int = 0,
             oversample: int = 0, max_iter: int = 0, tol: float = 0.0):
    """Rank-``k`` approximation ``A ~ L diag(D) W^T`` (Section 8 theorem,
    simplified as in the Section 10 experiments).  Returns ``(L, D, W, info)``
    with float64 device tensors ``L`` (n x k), ``D`` (k), ``W`` (m x k)."""
    m, device = _matrix(A)
    o = low_rank_opts(k, seed, eps, t_r, t_s, k_g, oversample, max_iter, tol)
    ws = _workspace(_size(lib().skls_low_rank_workspace, ctypes.byref(m), ctypes.byref(o)), device)
    Lm = torch.empty((m.n, k), dtype=torch.float64, device=device)
    D = torch.empty(k, dtype=torch.float64, device=device)
    Wm = torch.empty((m.d, k), dtype=torch.float64, device=device)
    info = L.SklsLowRankInfo()
    L.check(lib().skls_low_rank(ctypes.byref(m), ctypes.byref(o), _ptr(Lm), _ptr(D), _ptr(Wm), ctypes.byref(info),
                                _ptr(ws), ws.numel(), _stream(device)))
    out = {f: getattr(info, f) for f, _ in L.SklsLowRankInfo._fields_ if f != "reserved"}
    return Lm, D, Wm, out
