"""skls: input-sparsity-time sketching and least squares on AMD MI355X.

The sparse embedding ``S = Phi D`` of Clarkson & Woodruff (arXiv:1207.6365,
Section 2) applied in ``O(nnz(A))``, sketch-and-solve regression (Section 7),
R-preconditioned LSQR (Section 7.7), approximate leverage scores (Section 6)
and learned per-row sketch values, all in hand-written HIP kernels for gfx950
behind the C ABI of ``include/skls.h``.  This package only marshals torch
tensors into that ABI; importing it does not load the library, the first call
does (and raises if ``libskls.so`` has not been built).
"""

from ._lib import SklsError  # noqa: F401
from .api import (  # noqa: F401
    Csr,
    LearnedBatchWorkspace,
    LearnedWorkspace,
    adam_step,
    gram,
    hash_rows,
    learned_grad,
    learned_grad_batch,
    leverage_scores,
    lib,
    low_rank,
    lstsq,
    multi_lstsq,
    lp_regression,
    qr_r,
    second_stage,
    SketchPlan,
    sketch,
    sketch_general,
    sketch_plan,
    sketch_planned,
    version,
)
