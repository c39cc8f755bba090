"""Philox4x64-10 counter-based generator and Box-Muller normals (oracle side).

Written from the published definition: J. K. Salmon, M. A. Moraes,
R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11, Section 3 (Philox-4x64, R = 10 rounds).  Pinned against numpy's
independent Philox bit generator (tests/test_oracle_rng.py).

The paper draws `randn` for the Lanczos start vector (alg:rand-lanczos) and
for the test matrix Omega (alg:nystrom-sketch).  Both sides of the parity
check derive those draws from this counter-based stream so that no draw has
to be shipped between them:

    key     = (seed, 0)
    counter = (block, index, instance, purpose)
    purpose = 0: Lanczos start vector of iteration `index` (1-based t)
    purpose = 1: column `index` of Omega
    block j yields normals 4j .. 4j+3 of that vector.

Normals come from the Box-Muller transform: for a 64-bit pair (a, b),
u1 = ((a >> 11) + 1) 2^-53 in (0, 1], u2 = (b >> 11) 2^-53 in [0, 1),
r = sqrt(-2 log u1), theta = 2 pi u2, giving r cos(theta), r sin(theta).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a: np.uint64, x: np.ndarray):
    """Full 64x64 -> 128-bit product of a scalar and a vector, as (hi, lo)."""
    a_lo, a_hi = a & _MASK32, a >> _S32
    x_lo, x_hi = x & _MASK32, x >> _S32
    ll = a_lo * x_lo
    lh = a_lo * x_hi
    hl = a_hi * x_lo
    hh = a_hi * x_hi
    mid = (ll >> _S32) + (lh & _MASK32) + (hl & _MASK32)
    lo = (ll & _MASK32) | ((mid & _MASK32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x64-10 over arrays of counters; returns 4 uint64 arrays."""
    with np.errstate(over="ignore"):
        x0 = np.asarray(c0, dtype=np.uint64).copy()
        x1 = np.broadcast_to(np.asarray(c1, dtype=np.uint64), x0.shape).copy()
        x2 = np.broadcast_to(np.asarray(c2, dtype=np.uint64), x0.shape).copy()
        x3 = np.broadcast_to(np.asarray(c3, dtype=np.uint64), x0.shape).copy()
        k0 = np.uint64(k0)
        k1 = np.uint64(k1)
        for rnd in range(10):
            hi0, lo0 = _mulhilo64(M0, x0)
            hi1, lo1 = _mulhilo64(M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            if rnd < 9:
                k0 = k0 + W0
                k1 = k1 + W1
    return x0, x1, x2, x3


def uniform_pair(a: np.ndarray, b: np.ndarray):
    """53-bit uniforms: u1 in (0, 1], u2 in [0, 1)."""
    s = np.uint64(11)
    u1 = ((a >> s).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (b >> s).astype(np.float64) * 2.0 ** -53
    return u1, u2


def normal_stream(n: int, seed: int, index: int, instance: int, purpose: int) -> np.ndarray:
    """n standard normals of the stream (seed; index, instance, purpose)."""
    nb = (n + 3) // 4
    blk = np.arange(nb, dtype=np.uint64)
    x0, x1, x2, x3 = philox4x64_10(blk, index, instance, purpose, seed, 0)
    out = np.empty(4 * nb, dtype=np.float64)
    for k, (a, b) in enumerate(((x0, x1), (x2, x3))):
        u1, u2 = uniform_pair(a, b)
        r = np.sqrt(-2.0 * np.log(u1))
        th = (2.0 * np.pi) * u2
        out[2 * k::4] = r * np.cos(th)
        out[2 * k + 1::4] = r * np.sin(th)
    return out[:n]
