"""Training of learned per-row sketch values on the GPU.

The values ``w`` start at the random signs of ``D`` (the plain sparse
embedding of Section 2) and follow Adam on the mean normalised distortion
``||(S_w A)^T S_w A - A^T A||_F^2 / ||A^T A||_F^2`` over minibatches of
training matrices; ``h`` stays hashed.  Loss, gradient (forward sketch,
Gram, ``4 Y E`` and the gather backward) and the Adam update all run in the
library's kernels; this module only orders the calls.  When the trained
values do not lower the mean distortion on held-out matrices, the plain
signs are kept.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import api


@dataclass
class TrainResult:
    w: torch.Tensor                 # values to use (learned, or the signs on fallback)
    learned: torch.Tensor           # trained values
    used_learned: bool
    val_plain: float                # mean normalised distortion on the validation set
    val_learned: float
    history: list = field(default_factory=list)


def signs(n: int, t: int, seed: int, device) -> torch.Tensor:
    _, s = api.hash_rows(n, t, seed, device=device)
    return s.to(torch.float32)


def shared_plan(A: torch.Tensor, t: int, seed: int) -> api.SketchPlan:
    """The bucket plan of the forward sketch: it depends only on (seed, n, t),
    so one plan serves every matrix of the family."""
    return api.sketch_plan(A, t, seed, variant="sorted", out_dtype=torch.float32)


def prepare(mats: list[torch.Tensor], t: int, seed: int, plan: api.SketchPlan | None = None):
    """Gram matrices, normalisers ``||A^T A||_F^2`` (the loss at ``w = 0``)
    and a workspace for batched calls at this shape."""
    n = mats[0].shape[0]
    dev = mats[0].device
    ws = api.LearnedBatchWorkspace(mats[0], t)
    plan = shared_plan(mats[0], t, seed) if plan is None else plan
    zero = torch.zeros(n, dtype=torch.float32, device=dev)
    grams = [api.gram(A) for A in mats]
    loss, _ = api.learned_grad_batch(mats, grams, plan, zero, None, ws=ws)
    norms = [float(x) for x in loss.cpu().numpy()]
    return grams, norms, ws


def distortions(mats, grams, norms, t: int, seed: int, w: torch.Tensor, ws=None,
                plan: api.SketchPlan | None = None) -> np.ndarray:
    """Normalised distortion of each matrix for values ``w``."""
    plan = shared_plan(mats[0], t, seed) if plan is None else plan
    loss, _ = api.learned_grad_batch(mats, grams, plan, w, None, ws=ws)
    return loss.cpu().numpy().astype(np.float64) / np.asarray(norms, dtype=np.float64)


def train(train_mats, val_mats, t: int, seed: int, steps: int = 300, lr: float = 1e-2, batch: int = 16,
          rng_seed: int = 0, log_every: int = 0) -> TrainResult:
    n = train_mats[0].shape[0]
    dev = train_mats[0].device
    plan = shared_plan(train_mats[0], t, seed)
    grams, norms, bws = prepare(train_mats, t, seed, plan)
    vgrams, vnorms, _ = prepare(val_mats, t, seed, plan)
    w = signs(n, t, seed, dev)
    w_plain = w.clone()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    g = torch.empty_like(w)
    rng = np.random.default_rng(rng_seed)
    hist = []
    bsz = min(batch, len(train_mats))
    bloss = torch.empty(bsz, dtype=torch.float32, device=dev)
    for step in range(1, steps + 1):
        idx = rng.choice(len(train_mats), size=bsz, replace=False)
        api.learned_grad_batch([train_mats[i] for i in idx], [grams[i] for i in idx], plan, w, g,
                               scale=[1.0 / (bsz * norms[i]) for i in idx], ws=bws, loss=bloss)
        api.adam_step(w, g, m, v, step, lr)
        if log_every and (step % log_every == 0 or step == steps):
            hist.append((step, float(distortions(val_mats, vgrams, vnorms, t, seed, w, bws, plan).mean())))
    d_plain = float(distortions(val_mats, vgrams, vnorms, t, seed, w_plain, bws, plan).mean())
    d_learned = float(distortions(val_mats, vgrams, vnorms, t, seed, w, bws, plan).mean())
    use = d_learned < d_plain
    return TrainResult(w=w if use else w_plain, learned=w, used_learned=use, val_plain=d_plain,
                       val_learned=d_learned, history=hist)
