"""Pins of the oracle's general template (Appendix D, alg:full-sketchy-cgal-supp)
with A = diag: constraint set K = {lo <= diag X <= hi}, trace set tr X = alpha or
tr X <= alpha.

* K = {b} written as the box [b, b] must run the equality model exactly.
* With C positive definite and tr X <= alpha the linear minimisation always
  returns H = 0, so X stays 0 (the minimiser) and every iterate is exact.
* Relaxing diag X = 1 to diag X <= 1 (or to diag X >= 1 with tr X <= n) does not
  move the MaxCut SDP optimum for a Laplacian objective: X + D with D >= 0
  diagonal is still psd and <L, D> >= 0.  Odd cycles then have the closed form
  (n/2)(1 + cos(pi/n)).
* The surrogate gap <D_t, X_t - H_t> is nonnegative when the eigenvector is exact
  (H_t minimises <D_t, .> over the trace set, which holds X_t).
* The l2 ball {||diag X - b|| <= r}: radius 0 runs the equality model bit for
  bit, the reported distance equals the closed form max(0, ||z - b|| - r), and
  a larger ball does not lower the cut value (a larger feasible set).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import OracleParams, sketchy_cgal
from oracle.sketchycgal import reconstruct_result


def _run(inst, lo=None, hi=None, C=None, radius=None, **kw):
    prm = OracleParams(**kw)
    return sketchy_cgal(inst.to_scipy() if C is None else C, inst.b, prm, lo=lo, hi=hi, radius=radius)


def test_box_with_equal_bounds_runs_the_equality_model():
    inst = synth.laplacian_instance(synth.erdos_renyi(60, 200, seed=4))
    kw = dict(R=5, T=40, seed=7, q_mode=1, q_fixed=10)
    a = _run(inst, **kw)
    b = _run(inst, lo=inst.b, hi=inst.b, **kw)
    for key in ("p", "xi", "cv", "gamma", "gap", "k"):
        np.testing.assert_array_equal(a.log[key], b.log[key], err_msg=key)
    np.testing.assert_allclose(a.log["infeas"], b.log["infeas"], rtol=1e-15, atol=0)
    np.testing.assert_array_equal(a.z, b.z)
    np.testing.assert_array_equal(a.y, b.y)
    np.testing.assert_array_equal(a.S, b.S)
    assert np.all(np.isnan(b.log["stop_obj"])) and not np.any(np.isnan(a.log["stop_obj"]))


def test_trace_bounded_positive_definite_objective_stays_at_zero():
    g = synth.erdos_renyi(40, 120, seed=2)
    inst = synth.laplacian_instance(g)
    C = -inst.to_scipy() + 0.25 * sp.identity(inst.n, format="csr")   # L/4 + I/4, smallest eigenvalue 1/4
    res = _run(inst, C=C, hi=np.ones(inst.n), R=4, T=30, seed=3, trace_mode=1)
    # xi is in scaled units (C / ||C||_F): lambda_min = 1/4 / ||C||_F
    assert np.all(res.log["xi"] > 0.9 * 0.25 / res.c_F)
    assert res.p == 0.0 and not res.z.any() and not res.S.any() and res.tau == 0.0
    assert np.all(res.log["gap"] == 0.0)
    assert np.all(res.log["infeas"] == 0.0)   # z = 0 lies in K = {u <= 1}


@pytest.mark.parametrize("template", ["upper", "lower"])
@pytest.mark.parametrize("n", [7, 9])
def test_relaxed_templates_reach_the_odd_cycle_value(n, template):
    inst = synth.laplacian_instance(synth.cycle(n))
    ref = n / 2 * (1 + math.cos(math.pi / n))
    ones = np.ones(n)
    if template == "upper":
        res = _run(inst, hi=ones, R=4, T=3000, seed=1, trace_mode=1)
    else:
        res = _run(inst, lo=ones, R=4, T=3000, seed=1, trace_mode=1)
    val = -res.objective
    assert abs(val - ref) / ref < 5e-3, (val, ref)
    assert res.infeasibility / math.sqrt(n) < 1e-2


def test_surrogate_gap_is_nonnegative_with_exact_eigenvectors():
    rng = np.random.default_rng(5)
    g = synth.erdos_renyi(30, 90, seed=9)
    inst = synth.laplacian_instance(g)
    lo = rng.uniform(0.5, 1.0, inst.n)
    hi = lo + rng.uniform(0.0, 1.0, inst.n)
    for tm in (0, 1):
        res = _run(inst, lo=lo, hi=hi, R=4, T=60, seed=2, q_mode=1, q_fixed=inst.n - 1, trace_mode=tm, reorth=2)
        scale = 1.0 + np.abs(res.log["p"])
        assert np.all(res.log["gap"] >= -1e-10 * scale), tm


def test_trace_bounded_reconstruction_targets_the_tracked_trace():
    inst = synth.laplacian_instance(synth.cycle(9))
    res = _run(inst, hi=np.ones(9), R=4, T=200, seed=1, trace_mode=1)
    rec = reconstruct_result(res)
    assert abs(rec["lam"].sum() - res.tau) < 1e-12
    assert res.tau <= res.alpha_s + 1e-12


def test_ball_of_radius_zero_runs_the_equality_model():
    inst = synth.laplacian_instance(synth.erdos_renyi(60, 200, seed=4))
    kw = dict(R=5, T=40, seed=7, q_mode=1, q_fixed=10)
    a = _run(inst, **kw)
    b = _run(inst, radius=0.0, **kw)
    for key in ("p", "xi", "cv", "gamma", "gap", "k"):
        np.testing.assert_array_equal(a.log[key], b.log[key], err_msg=key)
    np.testing.assert_array_equal(a.z, b.z)
    np.testing.assert_array_equal(a.y, b.y)


def test_ball_distance_and_growing_radius():
    # dist_K(z) of a ball is max(0, ||z - b|| - r) (closed form, checked on the
    # final state); a larger ball only lowers the optimum of the minimisation
    inst = synth.laplacian_instance(synth.cycle(9))
    ref = 4.5 * (1 + math.cos(math.pi / 9))
    vals = []
    for r in (0.0, 0.5, 1.5):
        res = _run(inst, radius=r, R=4, T=3000, seed=1, trace_mode=1)
        d_closed = max(0.0, float(np.linalg.norm(res.z - res.b_s)) - r / res.alpha)
        assert abs(res.dist_K - d_closed) < 1e-15
        vals.append(-res.objective)
    assert abs(vals[0] - ref) / ref < 5e-3
    assert vals[0] <= vals[1] * (1 + 2e-3) and vals[1] <= vals[2] * (1 + 2e-3)


def test_ball_surrogate_gap_is_nonnegative_with_exact_eigenvectors():
    g = synth.erdos_renyi(30, 90, seed=9)
    inst = synth.laplacian_instance(g)
    for tm in (0, 1):
        res = _run(inst, radius=2.0, R=4, T=60, seed=2, q_mode=1, q_fixed=inst.n - 1, trace_mode=tm, reorth=2)
        assert np.all(res.log["gap"] >= -1e-10 * (1.0 + np.abs(res.log["p"]))), tm
