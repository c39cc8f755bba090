"""Pins for the oracle's Philox4x64-10 stream and Box-Muller normals.

Philox is checked against numpy's independent implementation (numpy's bit
generator advances its 256-bit counter before each block, so its first block
is our counter + 1).  The known-answer vector for a zero key and counter is in
tests/golden/philox4x64_10_kat.txt.
"""
import os

import numpy as np
import pytest
from scipy import stats

from oracle.philox import philox4x64_10, normal_stream

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def test_philox_matches_numpy():
    rng = np.random.default_rng(123)
    for _ in range(20):
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64)
        ctr = rng.integers(0, 2**63, size=4, dtype=np.uint64)
        bg = np.random.Philox(key=key, counter=ctr)
        ref = bg.random_raw(4 * 3)
        for blk in range(3):
            c0 = ctr[0] + np.uint64(blk + 1)
            out = philox4x64_10(np.array([c0]), ctr[1], ctr[2], ctr[3], key[0], key[1])
            got = np.array([o[0] for o in out], dtype=np.uint64)
            np.testing.assert_array_equal(got, ref[4 * blk: 4 * blk + 4])


def test_philox_known_answer():
    with open(GOLDEN) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    for r in rows:
        vals = [int(x, 16) for x in r]
        ctr, key, exp = vals[0:4], vals[4:6], vals[6:10]
        out = philox4x64_10(np.array([ctr[0]], dtype=np.uint64), ctr[1], ctr[2], ctr[3], key[0], key[1])
        assert [int(o[0]) for o in out] == exp


def test_normals_are_standard():
    x = normal_stream(400_000, seed=7, index=3, instance=0, purpose=0)
    assert abs(x.mean()) < 5 / np.sqrt(x.size)
    assert abs(x.var() - 1.0) < 0.02
    assert stats.kstest(x, "norm").pvalue > 1e-4


def test_streams_differ_and_are_reproducible():
    a = normal_stream(1000, 7, 1, 0, 0)
    b = normal_stream(1000, 7, 2, 0, 0)
    c = normal_stream(1000, 7, 1, 1, 0)
    d = normal_stream(1000, 7, 1, 0, 1)
    np.testing.assert_array_equal(a, normal_stream(1000, 7, 1, 0, 0))
    for other in (b, c, d):
        assert abs(np.corrcoef(a, other)[0, 1]) < 0.15
    # prefix property: a longer draw starts with the shorter one
    np.testing.assert_array_equal(normal_stream(1003, 7, 1, 0, 0)[:1000], a)
