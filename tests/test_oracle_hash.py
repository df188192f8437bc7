"""Pins for the oracle's hash/sign generator (Section 2: ``h`` uniform on
``[t]``, ``D`` independent fair signs)."""

import os

import numpy as np
import pytest

import oracle as O


def _golden(golden_dir):
    out = []
    with open(os.path.join(golden_dir, "splitmix64_seed0.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            i, v = line.split()
            out.append((int(i), int(v, 16)))
    return out


def test_splitmix64_published_outputs(golden_dir):
    for i, v in _golden(golden_dir):
        assert int(O.splitmix64(0, np.array([i], np.uint64))[0]) == v


def test_bucket_range_and_signs():
    for t in (1, 3, 4000, 65536, 2**31 - 1):
        h, s = O.bucket_and_sign(7, 5000, t)
        assert h.min() >= 0 and h.max() < t
        assert set(np.unique(s)) <= {-1, 1}


def test_power_of_two_bucket_is_top_bits():
    # For t = 2^k the multiply-high reduction keeps the top k bits of z.
    n, k = 4096, 12
    z = O.splitmix64(99, np.arange(n, dtype=np.uint64))
    h, _ = O.bucket_and_sign(99, n, 2**k)
    assert np.array_equal(h, (z >> np.uint64(64 - k)).astype(np.int64))
    _, s = O.bucket_and_sign(99, n, 2**k)
    assert np.array_equal(s == -1, (z & np.uint64(1)) == np.uint64(1))


def test_start_offset_is_a_slice():
    h, s = O.bucket_and_sign(5, 1000, 77)
    h2, s2 = O.bucket_and_sign(5, 300, 77, start=400)
    assert np.array_equal(h[400:700], h2) and np.array_equal(s[400:700], s2)


def test_uniform_buckets_chi_square():
    n, t = 1 << 20, 64
    h, s = O.bucket_and_sign(0x5EED0000, n, t)
    counts = np.bincount(h, minlength=t)
    e = n / t
    chi2 = ((counts - e) ** 2 / e).sum()
    # chi-square with 63 dof: 99.99% quantile is about 116
    assert chi2 < 116
    # fair signs: 5 standard errors
    assert abs(s.mean()) < 5 / np.sqrt(n)


def test_pair_collision_rate():
    # P[h(i) = h(j)] = 1/t for i != j (used in the birthday argument of Section 3)
    n, t = 3000, 50
    h, _ = O.bucket_and_sign(3, n, t)
    c = np.bincount(h, minlength=t)
    pairs = (c * (c - 1) // 2).sum()
    total = n * (n - 1) // 2
    rate = pairs / total
    assert abs(rate - 1 / t) < 0.1 / t


def test_rejects_bad_t():
    with pytest.raises(ValueError):
        O.bucket_and_sign(0, 10, 0)
    with pytest.raises(ValueError):
        O.bucket_and_sign(0, 10, 2**31)
