"""Pins of the MaxCut rounding (Section 7.2, sec:maxcut-rounding) in the oracle.

The cut weight is checked against a direct count over the edge list (not the
quadratic form), the heaviest of R rounded cuts against brute-force MaxCut on
small graphs, and the whole pipeline (solve, reconstruct, round) against
graphs whose maximum cut is known in closed form.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import OracleParams, sketchy_cgal, cut_indicators, cut_weight, round_maxcut
from oracle.sketchycgal import reconstruct_result


def _edge_count(g: synth.Graph, chi) -> float:
    return float(sum(w for i, j, w in zip(g.src, g.dst, g.w) if chi[i] != chi[j]))


def _brute_max_cut(g: synth.Graph) -> float:
    best = 0.0
    for bits in itertools.product((-1, 1), repeat=g.n - 1):
        chi = (1,) + bits
        best = max(best, _edge_count(g, chi))
    return best


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_cut_weight_is_the_weight_of_cut_edges(seed):
    rng = np.random.default_rng(seed)
    g = synth.erdos_renyi(30, 90, seed)
    g = synth.Graph(g.n, g.src, g.dst, rng.uniform(0.5, 2.0, g.src.size))
    inst = synth.laplacian_instance(g)
    for _ in range(5):
        chi = rng.choice([-1, 1], size=g.n)
        assert abs(cut_weight(inst.to_scipy(), chi) - _edge_count(g, chi)) < 1e-12 * max(1.0, g.w.sum())


def test_signs_put_zero_on_the_plus_side():
    U = np.array([[0.0, -0.0], [-1e-300, 2.0], [3.0, -4.0]])
    assert cut_indicators(U).tolist() == [[1, 1], [-1, 1], [1, -1]]


def test_best_of_r_cuts_is_the_heaviest_and_at_most_the_max_cut():
    g = synth.erdos_renyi(12, 30, 7)
    inst = synth.laplacian_instance(g)
    rng = np.random.default_rng(0)
    U = rng.standard_normal((12, 5))
    w, best, chi = round_maxcut(U, inst.to_scipy())
    assert w.shape == (5,) and best == int(np.argmax(w))
    for j in range(5):
        assert abs(w[j] - _edge_count(g, cut_indicators(U)[:, j])) < 1e-12
    assert w[best] <= _brute_max_cut(g) + 1e-12
    assert chi.tolist() == cut_indicators(U)[:, best].tolist()


@pytest.mark.parametrize("graph,opt", [(synth.complete_bipartite(3, 4), 12.0), (synth.cycle(8), 8.0),
                                       (synth.cycle(7), 6.0)])
def test_solve_reconstruct_round_finds_the_max_cut(graph, opt):
    """Bipartite graphs (even cycles, K_{3,4}) have every edge cut at the optimum;
    the 7-cycle's maximum cut is 6."""
    inst = synth.laplacian_instance(graph)
    res = sketchy_cgal(inst.to_scipy(), inst.b, OracleParams(R=4, T=2000, seed=1))
    rec = reconstruct_result(res)
    w, best, _ = round_maxcut(rec["U"], inst.to_scipy())
    assert w[best] == pytest.approx(opt, abs=1e-12)
    assert w[best] == pytest.approx(_brute_max_cut(graph), abs=1e-12)
