"""Instance lists for the batched-engine tests (not a test module).

All are seeded: Erdos-Renyi graphs of average degree 8 with uneven sizes (the
shape of the batched workload, scaled down), plus degenerate members: a
9-cycle (Lanczos breaks down before q steps) and a star whose hub row holds
most of the instance's nonzeros.
"""
from __future__ import annotations

import numpy as np

import synth

SEED4 = synth.CONFIG_SEEDS[4]


def _star(n: int, seed: int, weights: str) -> synth.MaxCutInstance:
    rng = np.random.default_rng(seed)
    er = synth.erdos_renyi(n, 2 * n, seed)
    src = np.concatenate([np.zeros(n - 1, dtype=np.int64), er.src])
    dst = np.concatenate([np.arange(1, n, dtype=np.int64), er.dst])
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    key = np.unique(lo * n + hi)
    key = key[(key // n) != (key % n)]
    if weights == "unit":
        w = np.ones(key.size)
    else:
        w = rng.uniform(0.5, 1.5, key.size)
    return synth.laplacian_instance(synth.Graph(n, key // n, key % n, w))


def _signed(g: synth.Graph, seed: int) -> synth.Graph:
    rng = np.random.default_rng(seed)
    return synth.Graph(g.n, g.src, g.dst, np.where(rng.random(g.src.size) < 0.5, -1.0, 1.0))


def traj_batch() -> list:
    """Unit weights (columns-only storage): uneven Erdos-Renyi graphs and a 9-cycle."""
    return synth.batched_erdos_renyi(6, 200, 1500, 8) + [synth.laplacian_instance(synth.cycle(9))]


def small_batch() -> list:
    """traj_batch plus a star, whose hub row holds most of the nonzeros.

    The star's trajectory is rounding-sensitive (its top eigenvector converges
    in two Lanczos steps, after which the recurrence is driven by rounding), so
    it is compared one iteration at a time from a common state."""
    return traj_batch() + [_star(2500, 77, "unit")]


def signed_batch() -> list:
    """Weights +-1 (columns with a sign bit)."""
    rng = np.random.default_rng(SEED4)
    sizes = rng.integers(200, 1500, size=5)
    return [synth.laplacian_instance(_signed(synth.erdos_renyi(int(n), 4 * int(n), SEED4 + 10 + k), SEED4 + k))
            for k, n in enumerate(sizes)]


def _uniform(g: synth.Graph, seed: int) -> synth.Graph:
    rng = np.random.default_rng(seed)
    return synth.Graph(g.n, g.src, g.dst, rng.uniform(0.5, 1.5, g.src.size))


def valued_traj_batch() -> list:
    """Weights uniform in [0.5, 1.5] (values stored)."""
    rng = np.random.default_rng(SEED4 + 1)
    sizes = rng.integers(300, 900, size=4)
    return [synth.laplacian_instance(_uniform(synth.erdos_renyi(int(n), 4 * int(n), SEED4 + 100 + k), SEED4 + 200 + k))
            for k, n in enumerate(sizes)]


def valued_batch() -> list:
    """valued_traj_batch plus a weighted star (rounding-sensitive, see small_batch)."""
    return [_star(1200, 78, "uniform")] + valued_traj_batch()
