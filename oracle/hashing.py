"""Oracle: the random map ``h`` and the random signs ``D`` of the sparse
embedding matrix ``S = Phi D`` (Section 2, "Sparse Embedding Matrices").

The paper asks for ``h(i)`` uniform on ``[t]`` and independent fair signs on
the diagonal of ``D``; it does not say how the randomness is produced.  Both
sides of this project draw it from one counter-based generator, SplitMix64
(Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014), implemented independently on each side from its published
definition:

* output ``i`` (0-based) of the stream with seed ``s`` is the SplitMix64
  finaliser applied to ``s + (i + 1) * 0x9E3779B97F4A7C15`` (mod 2^64);
* the bucket is the multiply-high range reduction of the upper 32 bits,
  ``h(i) = ((z >> 32) * t) >> 32`` (Lemire 2019), exactly uniform when ``t``
  is a power of two and within relative bias ``t / 2^32`` otherwise;
* the sign is ``-1`` when bit 0 of ``z`` is set, else ``+1``.

Only 64-bit integer operations are used, so the result is bit-exact.
"""

from __future__ import annotations

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, index) -> np.ndarray:
    """SplitMix64 outputs number ``index`` (0-based, array) of stream ``seed``."""
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (idx + np.uint64(1)) * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
        z = z ^ (z >> np.uint64(31))
    return z


def bucket_and_sign(seed: int, n: int, t: int, start: int = 0):
    """``h(i)`` in ``[0, t)`` (int64) and ``sigma(i)`` in {+1, -1} (int8) for
    global rows ``i = start .. start + n - 1``."""
    if not 1 <= t < 2**31:
        raise ValueError("t must lie in [1, 2^31)")
    z = splitmix64(seed, np.arange(start, start + n, dtype=np.uint64))
    h = ((z >> np.uint64(32)) * np.uint64(t)) >> np.uint64(32)
    sigma = np.where((z & np.uint64(1)) == np.uint64(1), -1, 1).astype(np.int8)
    return h.astype(np.int64), sigma
