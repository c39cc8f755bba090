"""End-to-end pins of the oracle on MaxCut SDPs with known values.

The SDP  max (1/4) tr(L X)  s.t. diag X = 1, X psd  (Section 1.1, eqn
maxcut-sdp, in cut-weight units) has closed-form values for:
  * odd cycles C_n: (n/2)(1 + cos(pi/n))  (Delorme and Poljak);
  * bipartite graphs: the total edge weight m (the cut of all edges);
  * complete graphs K_n: n^2/4 (X = (n I - 11^T)/(n-1) attains the bound
    lambda_max(L) tr X / 4).
For small random graphs, brute-force MaxCut <= SDP <= MaxCut / 0.87856
(Goemans-Williamson), and weak duality bounds the SDP value from above by the
dual function at the final dual iterate (Appendix E).
The paper reports O(1/t) objective error in practice (Section 7.2.5); the
tests require the error to shrink with T.
"""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import OracleParams, sketchy_cgal, maxcut_dual_bound


def _cut_value(inst, T, seed=1, R=4, **kw):
    res = sketchy_cgal(inst.to_scipy(), inst.b, OracleParams(R=R, T=T, seed=seed, **kw))
    return -res.objective, res


@pytest.mark.parametrize("n", [5, 7, 9])
def test_odd_cycle_closed_form(n):
    inst = synth.laplacian_instance(synth.cycle(n))
    ref = n / 2 * (1 + math.cos(math.pi / n))
    v_short, _ = _cut_value(inst, 200)
    v_long, res = _cut_value(inst, 2000)
    err_short = abs(v_short - ref) / ref
    err_long = abs(v_long - ref) / ref
    assert err_long < 2e-3
    assert err_long < err_short / 3
    assert res.infeasibility / math.sqrt(n) < 5e-3


@pytest.mark.parametrize("graph,ref", [
    (synth.cycle(8), 8.0),
    (synth.complete_bipartite(3, 4), 12.0),
    (synth.complete(6), 9.0),
    (synth.complete(7), 12.25),
])
def test_closed_form_values(graph, ref):
    inst = synth.laplacian_instance(graph)
    val, _ = _cut_value(inst, 2000)
    assert abs(val - ref) / ref < 2e-3


def _brute_maxcut(g):
    n = g.n
    best = 0.0
    signs = np.array(list(itertools.product((-1.0, 1.0), repeat=n - 1)))
    chi = np.hstack([np.ones((signs.shape[0], 1)), signs])
    cut = ((chi[:, g.src] != chi[:, g.dst]) * g.w).sum(axis=1)
    return float(cut.max())


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_and_duality_sandwich(seed):
    g = synth.erdos_renyi(12, 30, seed=seed)
    inst = synth.laplacian_instance(g)
    mc = _brute_maxcut(g)
    val, res = _cut_value(inst, 3000)
    assert mc <= val * (1 + 3e-3)
    assert val <= mc / 0.87856 * (1 + 3e-3)
    # weak duality in scaled units: phi(y) <= min <C_s, X>, so the SDP cut value
    # is at most -c_F * alpha * phi(y_T)
    Cs = inst.to_scipy().toarray() / res.c_F
    upper = -res.c_F * res.alpha * maxcut_dual_bound(Cs, res.b_s, res.y, res.alpha_s)
    assert mc <= upper + 1e-9
    assert val <= upper * (1 + 3e-3)


def test_unscaled_run_reaches_same_value():
    inst = synth.laplacian_instance(synth.cycle(7))
    ref = 3.5 * (1 + math.cos(math.pi / 7))
    val, _ = _cut_value(inst, 3000, scale=False)
    assert abs(val - ref) / ref < 2e-2


def test_stopping_quantities_shrink():
    inst = synth.config_instance(1)
    res = sketchy_cgal(inst.to_scipy(), inst.b, OracleParams(R=10, T=200, seed=synth.CONFIG_SEEDS[1]))
    so, sf = res.log["stop_obj"], res.log["stop_feas"]
    assert sf[-1] < sf[9] / 5
    assert abs(so[-1]) < abs(so[9])
