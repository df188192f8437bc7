"""CPU float64 oracle for the sparse-embedding sketch-and-solve path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path (the
HIP library and its Python binding) never does, and shares no code with it.

Plain, slow, obviously correct implementations, each citing the part of
Clarkson & Woodruff, "Low Rank Approximation and Regression in Input Sparsity
Time" (arXiv:1207.6365) it follows:

* :mod:`.hashing`  -- ``h`` and ``D`` of the sparse embedding (Section 2)
* :mod:`.sketch`   -- ``S A = Phi D A`` (Section 2; Section 3 main theorem) and
  the generalized sparse embedding (Section 5)
* :mod:`.linalg`   -- Householder QR, substitution, exact least squares,
  residual ratio via the Pythagorean identity (Section 7.2 facts)
* :mod:`.solve`    -- sketch-and-solve (Section 7 regression theorem),
  preconditioned LSQR and Richardson iteration (Section 7.7)
* :mod:`.stage2`   -- the second sketch stage ``Pi1 = F S`` with a dense sign
  matrix ``F`` (Section 6; composition facts of Section 8)
* :mod:`.leverage` -- exact and approximate leverage scores (Section 6)
* :mod:`.multiresponse` -- multiple-response regression by leverage-score
  sampling (Section 7, generalized-regression algorithm)
* :mod:`.lowrank`  -- rank-k approximation ``L D W^T`` (Section 8 theorem in
  the simplified form of the Section 10 experiments)
* :mod:`.lp`       -- l_p regression: block-diagonal generalized embedding,
  conditioning, two-stage row sampling, exact weighted l_p fits (Section 9)
* :mod:`.learned`  -- distortion loss and gradient of learned sketch values
  (an extension; closed-form expectation for the plain sketch)

Every function is pinned by the CPU tests against facts fixed by the paper or
by mathematics (published generator outputs, exact moments, special cases,
brute force on tiny inputs, library routines); see the tests for each pin.
"""

from .hashing import bucket_and_sign, splitmix64  # noqa: F401
from .learned import Adam, distortion_grad, distortion_loss, expected_plain_distortion  # noqa: F401
from .leverage import leverage_approx, leverage_exact, sketch_r  # noqa: F401
from .lowrank import best_rank_k_error, frobenius_error, low_rank  # noqa: F401
from .lp import block_embedding, lp_exact, lp_objective, lp_regression  # noqa: F401
from .multiresponse import multi_response_lstsq, residual_fro  # noqa: F401
from .linalg import (  # noqa: F401
    RankDeficient,
    apply_qt,
    check_rank,
    householder_qr,
    lstsq_exact,
    residual_ratio,
    solve_upper,
    solve_upper_t,
    thin_q,
)
from .operator import MatrixOp  # noqa: F401
from .sketch import (  # noqa: F401
    copy_seed,
    explicit_S,
    generalized_S,
    sketch_bucket_rows,
    sketch_csr,
    sketch_dense,
    sketch_generalized,
)
from .solve import (  # noqa: F401
    certificate_threshold,
    lsqr,
    lstsq,
    richardson,
    sketch_and_solve,
    sketch_matrix,
)
