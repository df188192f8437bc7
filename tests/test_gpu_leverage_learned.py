"""GPU parity: approximate leverage scores (Section 6) and the learned sketch
values (distortion loss, gradient, Adam, training) against the oracle."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import dev, up, up_bf16, up_csr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sk():
    import paper_1207_6365_amd as sk

    return sk


def test_leverage_small_workload_csr(sk):
    A, b, _ = W.lstsq_small()
    seed, t, k = W.sketch_seed(0), 4000, 32
    Pi2 = W.gaussian_matrix(7, A.d, k, scale=1 / np.sqrt(k))
    got = sk.leverage_scores(up_csr(A), t, seed, up(Pi2)).cpu().numpy()
    ref = O.leverage_approx(O.MatrixOp(A), seed, t, Pi2)
    assert np.max(np.abs(got - ref) / ref) <= 1e-5


def test_leverage_csr_with_empty_rows(sk):
    # every eleventh row empty: its score is exactly zero on both sides
    A0, _, _ = W.lstsq_small()
    lens = np.diff(A0.row_ptr)
    lens[5::11] = 0
    keep = np.repeat(lens > 0, np.diff(A0.row_ptr))
    A = W.CSR(A0.n, A0.d, np.concatenate([[0], np.cumsum(lens)]).astype(np.int64), A0.col_idx[keep], A0.val[keep])
    seed, t, k = W.sketch_seed(0), 4000, 32
    Pi2 = W.gaussian_matrix(7, A.d, k, scale=1 / np.sqrt(k))
    got = sk.leverage_scores(up_csr(A), t, seed, up(Pi2)).cpu().numpy()
    ref = O.leverage_approx(O.MatrixOp(A), seed, t, Pi2)
    empty = lens == 0
    assert np.all(got[empty] == 0.0) and np.all(ref[empty] == 0.0)
    assert np.max(np.abs(got[~empty] - ref[~empty]) / ref[~empty]) <= 1e-5


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_leverage_dense_pareto_rows(sk, storage):
    n, d, t, k = 1 << 14, 64, 4096, 32
    A, b, _ = W.pareto_rows(n=n, d=d, storage=storage)
    Af = (W.bf16_to_f32(A) if storage == "bf16" else A).astype(np.float64)
    Ag = up_bf16(A) if storage == "bf16" else up(A)
    seed = W.sketch_seed(1)
    Pi2 = W.gaussian_matrix(8, d, k, scale=1 / np.sqrt(k))
    got = sk.leverage_scores(Ag, t, seed, up(Pi2)).cpu().numpy()
    ref = O.leverage_approx(Af, seed, t, Pi2)
    # float32 sketch and float32 accumulation of the d-term products
    assert np.max(np.abs(got - ref) / ref) <= 1e-4


def test_leverage_identity_projection_sandwich(sk):
    # Pi2 = I: scores are the row norms of A R^{-1}; their ratio to the exact
    # leverage lies in [sigma_min^2, sigma_max^2] of A R^{-1}
    n, d, t = 20000, 16, 2000
    g = np.random.default_rng(3)
    A = g.standard_normal((n, d)) * (1 + g.pareto(1.5, size=n))[:, None]
    seed = 12
    got = sk.leverage_scores(up(A), t, seed, up(np.eye(d))).cpu().numpy().astype(np.float64)
    exact = O.leverage_exact(A)
    R = O.sketch_r(A, seed, t)
    sv = np.linalg.svd(A @ np.linalg.inv(R), compute_uv=False)
    ratio = got / exact
    assert ratio.min() >= sv.min() ** 2 * (1 - 1e-5)
    assert ratio.max() <= sv.max() ** 2 * (1 + 1e-5)
    assert abs(got.sum() - d) <= 0.5 * d


def test_gram_matches_numpy(sk):
    g = np.random.default_rng(4)
    for n, d in [(32768, 64), (1000, 5), (4099, 130)]:
        A = g.standard_normal((n, d)).astype(np.float32)
        C = sk.gram(up(A)).cpu().numpy()
        ref = A.astype(np.float64).T @ A.astype(np.float64)
        assert np.max(np.abs(C - ref)) <= 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,d,ld", [(1, 1, 1), (63, 3, 3), (64, 64, 64), (65, 61, 61), (1000, 64, 72),
                                    (16385, 32, 32), (70001, 64, 64), (5000, 65, 65)])
def test_gram_narrow_integer_exact(sk, storage, n, d, ld):
    # small integers: every partial sum is an integer below 2^24, so the
    # float32 Gram equals the exact one bit for bit whatever the split of the
    # rows and the order of the sums (d <= 64 takes the small-Gram kernel,
    # d = 65 the tiled one)
    g = np.random.default_rng(n + d)
    X = g.integers(-7, 8, size=(n, ld))
    if storage == "bf16":
        Ag = up_bf16(W.bf16_round(X.astype(np.float32)))[:, :d]
    else:
        Ag = up(X.astype(np.float64 if storage == "f64" else np.float32))[:, :d]
    A = X[:, :d].astype(np.int64)
    C = sk.gram(Ag).cpu().numpy()
    assert np.array_equal(C.astype(np.int64), A.T @ A)


@pytest.mark.parametrize("n,d,t", [(4096, 16, 128), (32768, 64, 1024), (5000, 70, 333), (3000, 13, 37),
                                   (3000, 24, 37)])
def test_learned_loss_and_gradient(sk, n, d, t):
    # both the call that builds its own plan and the call with a shared plan
    # (at d <= 64 the product 4 Y E and the gather then run as one kernel
    # over the plan's bucket order), each against the oracle
    make, _ = W.learned_family(num=4, n=n, d=d, rank=min(16, d))
    A = make(1)
    seed = W.sketch_seed(0)
    w = np.random.default_rng(5).standard_normal(n).astype(np.float32)
    Ag = up(A)
    C = sk.gram(Ag)
    L_o, g_o = O.distortion_grad(A.astype(np.float64), seed, t, w.astype(np.float64))
    plan = sk.sketch_plan(Ag, t, seed, variant="sorted", out_dtype=torch.float32)
    for pl in (plan, None):
        loss, grad = sk.learned_grad(Ag, C, t, seed, up(w), plan=pl)
        assert abs(loss.item() - L_o) <= 1e-4 * L_o
        gg = grad.cpu().numpy()
        assert np.linalg.norm(gg - g_o) <= 1e-4 * np.linalg.norm(g_o)
    # scaled accumulation: grad2 = grad + 0.5 grad
    g2 = grad.clone()
    sk.learned_grad(Ag, C, t, seed, up(w), loss=loss, grad=g2, grad_scale=0.5, accumulate=True)
    assert torch.allclose(g2, 1.5 * grad, rtol=1e-5, atol=1e-6 * float(grad.abs().max()))


@pytest.mark.parametrize("n,d,t,count", [(5000, 70, 333, 3), (32768, 64, 1024, 6), (4096, 16, 128, 1),
                                         (4096, 16, 128, 18), (3000, 13, 37, 3), (500, 1, 1, 2), (2000, 8, 5, 17)])
def test_learned_batch_matches_single_calls(sk, n, d, t, count):
    # the batched gradient against one planned call per matrix.  d = 70 runs
    # the per-matrix kernels on several streams (the losses then equal the
    # single calls' bit for bit); d <= 64 runs every step as one launch over
    # up to 16 matrices (18: two groups; d = 13: element-wise loads), whose
    # losses agree to float32 rounding.  The weighted gradient sums agree to
    # float32 rounding of the different order.
    make, _ = W.learned_family(num=count, n=n, d=d, rank=min(16, d))
    seed = W.sketch_seed(1)
    mats = [up(make(i)) for i in range(count)]
    grams = [sk.gram(A) for A in mats]
    w = up(np.random.default_rng(8).standard_normal(n).astype(np.float32))
    plan = sk.sketch_plan(mats[0], t, seed, variant="sorted", out_dtype=torch.float32)
    scale = [0.5 + 0.25 * i for i in range(count)]
    ref_loss, ref = [], torch.zeros(n, dtype=torch.float32, device=dev())
    for i, (A, C) in enumerate(zip(mats, grams)):
        loss, g = sk.learned_grad(A, C, t, seed, w, plan=plan)
        ref_loss.append(loss.item())
        ref += scale[i] * g
    loss, grad = sk.learned_grad_batch(mats, grams, plan, w, torch.empty(n, device=dev()), scale=scale)
    if d > 64:
        assert np.array_equal(loss.cpu().numpy(), np.array(ref_loss, dtype=np.float32))
    else:
        assert np.allclose(loss.cpu().numpy(), np.array(ref_loss, dtype=np.float32), rtol=1e-5, atol=0)
    tol = 1e-5 * float(ref.abs().max())
    assert torch.allclose(grad, ref, rtol=1e-5, atol=tol)
    # the same call again gives the same bits; accumulate adds; NULL grad
    # gives the losses alone
    _, again = sk.learned_grad_batch(mats, grams, plan, w, torch.empty(n, device=dev()), scale=scale)
    assert torch.equal(again, grad)
    acc = grad.clone()
    sk.learned_grad_batch(mats, grams, plan, w, acc, scale=scale, accumulate=True)
    assert torch.allclose(acc, 2 * grad, rtol=1e-6, atol=1e-6 * float(grad.abs().max()))
    only, none = sk.learned_grad_batch(mats, grams, plan, w, None)
    assert none is None and torch.equal(only, loss)


def test_learned_plain_signs_match_closed_form_expectation(sk):
    # mean distortion of random-sign sketches over seeds vs the closed form
    n, d, t = 2048, 8, 64
    A = np.random.default_rng(6).standard_normal((n, d)).astype(np.float32)
    Ag = up(A)
    C = sk.gram(Ag)
    vals = []
    for seed in range(200):
        _, s = sk.hash_rows(n, t, seed)
        loss, _ = sk.learned_grad(Ag, C, t, seed, s.to(torch.float32), want_grad=False)
        vals.append(loss.item())
    vals = np.array(vals)
    ref = O.expected_plain_distortion(A.astype(np.float64), t)
    assert abs(vals.mean() - ref) <= 5 * vals.std(ddof=1) / np.sqrt(len(vals))


def test_adam_matches_oracle(sk):
    n = 1000
    g = np.random.default_rng(7)
    w0 = g.standard_normal(n).astype(np.float32)
    opt = O.Adam(n, lr=0.01)
    w_o = w0.astype(np.float64)
    wt, m, v = up(w0), torch.zeros(n, device=dev()), torch.zeros(n, device=dev())
    for step in range(1, 6):
        gr = g.standard_normal(n).astype(np.float32)
        w_o = opt.step(w_o, gr.astype(np.float64))
        sk.adam_step(wt, up(gr), m, v, step, lr=0.01)
    assert np.allclose(wt.cpu().numpy(), w_o, rtol=1e-5, atol=1e-6)


def test_training_lowers_distortion_on_held_out_matrices(sk):
    from paper_1207_6365_amd import train

    n, d, t = 8192, 32, 256
    make, _ = W.learned_family(num=40, n=n, d=d, seed=777)
    mats = [up(make(m)) for m in range(40)]
    seed = W.sketch_seed(0)
    res = train.train(mats[:24], mats[24:32], t, seed, steps=150, lr=2e-2, batch=8)
    grams, norms, ws = train.prepare(mats[32:], t, seed)
    plain = train.distortions(mats[32:], grams, norms, t, seed, train.signs(n, t, seed, dev()), ws)
    learned = train.distortions(mats[32:], grams, norms, t, seed, res.learned, ws)
    # the learned values must do better on average than the random signs on
    # matrices never seen in training (and the fallback must pick them)
    assert learned.mean() < plain.mean()
    assert res.used_learned
    print(f"test distortion plain {plain.mean():.4f} learned {learned.mean():.4f}")


def test_leverage_past_2p31_entries(sk):
    # CSR with 2^31 + 80 entries (64-bit row pointers, n = 2^27 + 5, d = 64),
    # drawn on the GPU from a seeded generator.  With R from a 2^16-row sketch,
    # A R^{-1} is close to orthonormal, so the scores (unbiased for the squared
    # row norms with the scaled Gaussian Pi2) sum to about d; every score is
    # finite and non-negative.
    import numpy as np
    import torch

    n, d, k = (1 << 27) + 5, 64, 16
    nnz = n * k
    g = torch.Generator(device="cuda:0")
    g.manual_seed(4321)
    col = torch.randint(0, d, (nnz,), dtype=torch.int32, device="cuda:0", generator=g)
    val = torch.randn(nnz, dtype=torch.float32, device="cuda:0", generator=g)
    row_ptr = torch.arange(0, nnz + 1, k, dtype=torch.int64, device="cuda:0")
    Pi2 = torch.from_numpy(np.random.default_rng(1).standard_normal((d, 32)) / np.sqrt(32.0)).to("cuda:0")
    scores = sk.leverage_scores(sk.Csr(n, d, row_ptr, col, val), 1 << 16, 99, Pi2)
    assert scores.numel() == n
    assert bool(torch.isfinite(scores).all()) and float(scores.min()) >= 0.0
    total = float(scores.double().sum())
    assert 0.7 * d < total < 1.3 * d
    del col, val, row_ptr, scores
    torch.cuda.empty_cache()
