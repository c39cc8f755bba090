"""Seeded synthetic MaxCut instances.

This module is the only code shared by the FP64 oracle and the HIP path.  It
draws graphs and assembles the problem data (C, b) of the MaxCut SDP
(Section 1.1, eqns comb-laplacian and maxcut-sdp): C = -L/4 with L the
weighted combinatorial Laplacian, b = 1, so that -<C, X> is the SDP value in
cut-weight units.  It holds none of the solver's arithmetic.

The paper's MaxCut inputs are the public Gset and DIMACS10 collections
(Section 7.2.3).  They are not used here: the generators below are stand-ins
with the same kinds of structure (uniform random, grid plus long-range,
power-law, random geometric) and the sizes of the workloads this library is
measured on.  Nothing from those collections is reproduced.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

__all__ = [
    "Graph", "MaxCutInstance", "laplacian_instance", "erdos_renyi", "torus_longrange",
    "chung_lu", "random_geometric", "cycle", "complete", "complete_bipartite",
    "batched_erdos_renyi", "config_instance", "CONFIG_SEEDS",
]

# Seed of workload k is 0x5C6A1000 + k; batched instance j uses 0x5C6A4000 + j.
CONFIG_SEEDS = {k: 0x5C6A1000 + k for k in range(1, 6)}


@dataclasses.dataclass
class Graph:
    n: int
    src: np.ndarray      # int64[m], src < dst
    dst: np.ndarray      # int64[m]
    w: np.ndarray        # float64[m] edge weights

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


@dataclasses.dataclass
class MaxCutInstance:
    """Problem data (C, b) in CSR form, C symmetric including its diagonal."""
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[nnz], sorted within each row
    val: np.ndarray      # float64[nnz]
    b: np.ndarray        # float64[n]
    graph: Graph | None = None

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def laplacian_instance(g: Graph) -> MaxCutInstance:
    """C = -L/4 as CSR, with L = sum_e w_e (e_i - e_j)(e_i - e_j)^T; b = ones."""
    n = g.n
    deg = np.bincount(g.src, weights=g.w, minlength=n) + np.bincount(g.dst, weights=g.w, minlength=n)
    diag = np.arange(n, dtype=np.int64)
    rows = np.concatenate([g.src, g.dst, diag])
    cols = np.concatenate([g.dst, g.src, diag])
    vals = np.concatenate([0.25 * g.w, 0.25 * g.w, -0.25 * deg])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return MaxCutInstance(
        n=n,
        row_ptr=A.indptr.astype(np.int64),
        col=A.indices.astype(np.int32),
        val=A.data.astype(np.float64),
        b=np.ones(n, dtype=np.float64),
        graph=g,
    )


def _unrank_pairs(idx: np.ndarray, n: int):
    """Map pair ranks 0..n(n-1)/2-1 to (i, j), i < j, row-major over i."""
    idx = idx.astype(np.int64)
    # row i starts at rank i*n - i*(i+1)/2; invert the quadratic, then correct.
    nf = float(n)
    i = np.floor((2 * nf - 1 - np.sqrt((2 * nf - 1) ** 2 - 8.0 * idx)) / 2).astype(np.int64)
    i = np.clip(i, 0, n - 2)
    start = i * n - i * (i + 1) // 2
    over = idx < start
    while np.any(over):
        i[over] -= 1
        start = i * n - i * (i + 1) // 2
        over = idx < start
    nxt = (i + 1) * n - (i + 1) * (i + 2) // 2
    under = idx >= nxt
    while np.any(under):
        i[under] += 1
        nxt = (i + 1) * n - (i + 1) * (i + 2) // 2
        under = idx >= nxt
    start = i * n - i * (i + 1) // 2
    j = idx - start + i + 1
    return i, j


def erdos_renyi(n: int, m: int, seed: int, weights: str = "unit") -> Graph:
    """G(n, m): m distinct pairs drawn uniformly without replacement."""
    rng = np.random.default_rng(seed)
    total = n * (n - 1) // 2
    if m > total:
        raise ValueError("m exceeds the number of vertex pairs")
    idx = np.sort(rng.choice(total, size=m, replace=False))
    i, j = _unrank_pairs(idx, n)
    w = _weights(rng, m, weights)
    return Graph(n, i, j, w)


def _weights(rng, m, kind):
    if kind == "unit":
        return np.ones(m, dtype=np.float64)
    if kind == "pm1":
        return np.where(rng.random(m) < 0.5, -1.0, 1.0)
    if kind == "uniform":
        return rng.uniform(0.5, 1.5, size=m)
    raise ValueError(kind)


def _dedupe(i, j, n):
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    keep = lo != hi
    key = np.unique(lo[keep] * np.int64(n) + hi[keep])
    return key // n, key % n


def torus_longrange(side: int, seed: int, extra_factor: int = 2) -> Graph:
    """side x side torus (4-neighbour) plus extra_factor*n random pairs, weights +-1.

    Vertex (r, c) is numbered side*r + c.  Random pairs that are self-loops or
    duplicate an existing edge are rejected and redrawn.
    """
    rng = np.random.default_rng(seed)
    n = side * side
    v = np.arange(n, dtype=np.int64)
    r, c = v // side, v % side
    right = r * side + (c + 1) % side
    down = ((r + 1) % side) * side + c
    ei = np.concatenate([v, v])
    ej = np.concatenate([right, down])
    lo, hi = np.minimum(ei, ej), np.maximum(ei, ej)
    keys = np.unique(lo * n + hi)
    need = extra_factor * n
    extra = np.empty(0, dtype=np.int64)
    while extra.size < need:
        k = need - extra.size
        a = rng.integers(0, n, size=2 * k + 16, dtype=np.int64)
        b = rng.integers(0, n, size=2 * k + 16, dtype=np.int64)
        ok = a != b
        a, b = a[ok], b[ok]
        cand = np.minimum(a, b) * n + np.maximum(a, b)
        cand = cand[~np.isin(cand, keys)]
        cand = cand[~np.isin(cand, extra)]
        _, first = np.unique(cand, return_index=True)
        cand = cand[np.sort(first)]
        extra = np.concatenate([extra, cand[:k]])
    allk = np.concatenate([keys, extra])
    order = np.argsort(allk, kind="stable")
    allk = allk[order]
    src, dst = allk // n, allk % n
    w = _weights(rng, allk.size, "pm1")
    return Graph(n, src, dst, w)


def chung_lu(n: int, m_draw: int, exponent: float, seed: int) -> Graph:
    """Chung-Lu power-law graph, unit weights.

    Expected-degree weights w_i ~ (i + 1)^(-1/(exponent-1)), scaled to mean
    degree 2*m_draw/n and capped at sqrt(sum w).  m_draw endpoint pairs are
    drawn with probability proportional to w; self-loops are dropped and
    duplicates merged.  Vertex ids are randomly permuted.
    """
    rng = np.random.default_rng(seed)
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (exponent - 1.0))
    target = 2.0 * m_draw
    for _ in range(8):
        w *= target / w.sum()
        cap = math.sqrt(w.sum())
        w = np.minimum(w, cap)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    chunk = 1 << 24
    keys = []
    for s in range(0, m_draw, chunk):
        k = min(chunk, m_draw - s)
        a = np.searchsorted(cdf, rng.random(k), side="right")
        b = np.searchsorted(cdf, rng.random(k), side="right")
        a = np.minimum(a, n - 1)
        b = np.minimum(b, n - 1)
        ok = a != b
        lo, hi = np.minimum(a[ok], b[ok]), np.maximum(a[ok], b[ok])
        keys.append(lo.astype(np.int64) * n + hi)
    key = np.unique(np.concatenate(keys))
    perm = rng.permutation(n).astype(np.int64)
    i, j = perm[key // n], perm[key % n]
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    key = np.sort(lo * n + hi)
    return Graph(n, key // n, key % n, np.ones(key.size, dtype=np.float64))


def random_geometric(n: int, mean_degree: float, seed: int) -> Graph:
    """Random geometric graph on [0,1)^2 with weights U[0.5, 1.5].

    Pairs closer than r = sqrt(mean_degree / (pi n)) are joined.  Vertices are
    numbered in grid-cell order (row-major cells of side >= r, then point), a
    road-network-like locality.
    """
    rng = np.random.default_rng(seed)
    r = math.sqrt(mean_degree / (math.pi * n))
    G = max(1, int(math.floor(1.0 / r)))
    pts = rng.random((n, 2))
    cx = np.minimum((pts[:, 0] * G).astype(np.int64), G - 1)
    cy = np.minimum((pts[:, 1] * G).astype(np.int64), G - 1)
    cell = cy * G + cx
    order = np.argsort(cell, kind="stable")
    pts = pts[order]
    cell = cell[order]
    cx, cy = cx[order], cy[order]
    counts = np.bincount(cell, minlength=G * G)
    start = np.concatenate([[0], np.cumsum(counts)[:-1]])
    maxc = int(counts.max())
    r2 = r * r
    src_l, dst_l = [], []
    p = np.arange(n, dtype=np.int64)
    for dy, dx in ((0, 0), (0, 1), (1, -1), (1, 0), (1, 1)):
        ny, nx = cy + dy, cx + dx
        valid = (ny < G) & (nx >= 0) & (nx < G)
        pv = p[valid]
        ncell = ny[valid] * G + nx[valid]
        st, ct = start[ncell], counts[ncell]
        for s in range(maxc):
            has = ct > s
            a = pv[has]
            q = st[has] + s
            if dy == 0 and dx == 0:
                keep = q > a
                a, q = a[keep], q[keep]
            d = pts[a] - pts[q]
            close = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) < r2
            src_l.append(a[close])
            dst_l.append(q[close])
    src = np.concatenate(src_l)
    dst = np.concatenate(dst_l)
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    key = np.sort(lo * n + hi)
    w = rng.uniform(0.5, 1.5, size=key.size)
    return Graph(n, key // n, key % n, w)


def cycle(n: int) -> Graph:
    i = np.arange(n, dtype=np.int64)
    j = (i + 1) % n
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    return Graph(n, lo, hi, np.ones(n))


def complete(n: int) -> Graph:
    i, j = np.triu_indices(n, 1)
    return Graph(n, i.astype(np.int64), j.astype(np.int64), np.ones(i.size))


def complete_bipartite(a: int, b: int) -> Graph:
    i, j = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    i, j = i.ravel().astype(np.int64), j.ravel().astype(np.int64)
    return Graph(a + b, i, j, np.ones(i.size))


def batched_erdos_renyi(count: int, n_lo: int, n_hi: int, degree: float, seed_base: int = 0x5C6A4000):
    """`count` independent G(n_k, degree*n_k/2) instances, n_k ~ U{n_lo..n_hi}."""
    rng = np.random.default_rng(seed_base - 1)
    sizes = rng.integers(n_lo, n_hi + 1, size=count)
    out = []
    for k, nk in enumerate(sizes):
        m = int(round(degree * nk / 2))
        out.append(laplacian_instance(erdos_renyi(int(nk), m, seed_base + k)))
    return out


def config_instance(k: int) -> MaxCutInstance:
    """The five measured workloads (k = 1..5); k = 4 returns the first batched instance list."""
    s = CONFIG_SEEDS[k]
    if k == 1:
        return laplacian_instance(erdos_renyi(800, 19176, s))
    if k == 2:
        return laplacian_instance(torus_longrange(1024, s))
    if k == 3:
        return laplacian_instance(chung_lu(1 << 22, 34_000_000, 2.5, s))
    if k == 5:
        return laplacian_instance(random_geometric(1 << 23, 4.77, s))
    raise ValueError("workload 4 is batched: use batched_erdos_renyi(256, 200, 20000, 8)")
