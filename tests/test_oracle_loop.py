"""Pins for the oracle's SketchyCGAL state updates via the loop invariants of
Section 6.2 (eqn loop-invariant): run dense CGAL (alg:cgal, X stored as an
n x n matrix) on the same eigenvectors v_t and check h = A H, z = A X,
S = X Omega, tau = tr X, p = <C, X>, and that each v_t satisfies the
approximate-LMO condition (eqn cgal-lmo-approx) for the dense gradient D_t.
"""
import math

import numpy as np
import pytest

import synth
from oracle import OracleParams, sketchy_cgal
from oracle.sketchycgal import scale_problem, dual_step_size


def _largest_gamma(r2, t, alpha, beta0):
    """Largest gamma in [0, beta0] with gamma*r2 <= 4 alpha^2 beta0 / (t+1)^1.5, by bisection."""
    bound = 4.0 * alpha * alpha * beta0 / (t + 1.0) ** 1.5
    if beta0 * r2 <= bound:
        return beta0
    lo, hi = 0.0, beta0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid * r2 <= bound:
            lo = mid
        else:
            hi = mid
    return lo


@pytest.mark.parametrize("scale,K,reorth", [(True, math.inf, 0), (False, math.inf, 0), (True, 0.5, 0),
                                            (True, math.inf, 2)])
def test_dense_cgal_on_same_vectors(scale, K, reorth):
    g = synth.erdos_renyi(40, 150, seed=2)
    inst = synth.laplacian_instance(g)
    C = inst.to_scipy()
    prm = OracleParams(R=5, T=60, seed=4, scale=scale, K=K, reorth=reorth)
    res = sketchy_cgal(C, inst.b, prm, record_v=True)
    Cs, bs, alpha, _ = scale_problem(C, inst.b, float(inst.n), scale)
    Cd = Cs.toarray()
    n = inst.n
    X = np.zeros((n, n))
    y = np.zeros(n)
    for t in range(1, prm.T + 1):
        beta = math.sqrt(t + 1.0)
        eta = 2.0 / (t + 1.0)
        D = Cd + np.diag(y + beta * (np.diag(X) - bs))
        v = res.vs[t - 1]
        ev = np.linalg.eigvalsh(D)
        normD = np.abs(ev).max()
        # v is an approximate minimum eigenvector of the dense gradient
        assert v @ D @ v <= ev[0] + normD / math.sqrt(t + 1.0) + 1e-12
        assert res.log["xi"][t - 1] >= ev[0] - 1e-12 * normD
        H = alpha * np.outer(v, v)
        X = (1 - eta) * X + eta * H
        np.testing.assert_allclose(res.log["p"][t - 1], np.sum(Cd * X), rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(res.log["infeas"][t - 1], np.linalg.norm(np.diag(X) - bs), rtol=1e-10)
        gamma = _largest_gamma(float(np.sum((np.diag(X) - bs) ** 2)), t, alpha, 1.0)
        y_new = y + gamma * (np.diag(X) - bs)
        if np.linalg.norm(y_new) <= K:
            y = y_new
            assert abs(res.log["gamma"][t - 1] - gamma) <= 1e-12 * max(gamma, 1e-300) + 1e-15
        else:
            assert res.log["gamma"][t - 1] == 0.0
    np.testing.assert_allclose(res.z, np.diag(X), rtol=0, atol=1e-13 * alpha)
    np.testing.assert_allclose(res.y, y, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(res.S, X @ res.Omega, rtol=0, atol=1e-12 * np.abs(res.S).max())
    assert abs(res.tau - np.trace(X)) < 1e-13


def test_trace_and_diagonal_invariants():
    inst = synth.config_instance(1)
    prm = OracleParams(R=10, T=30, seed=synth.CONFIG_SEEDS[1], q_mode=1, q_fixed=36)
    res = sketchy_cgal(inst.to_scipy(), inst.b, prm)
    # X_{t+1} lies in alpha*Delta_n: tr X = alpha, diag X >= 0  (X_1 = 0; eta_1 = 1)
    assert abs(res.z.sum() - res.alpha_s) < 1e-12
    assert res.z.min() >= 0.0
    assert abs(res.tau - res.alpha_s) < 1e-12
    assert np.all(res.log["k"] == 36)


def test_dual_step_is_largest_feasible():
    for r2 in (0.0, 1e-8, 0.3, 5.0):
        for t in (1, 7, 100):
            for beta0 in (0.5, 1.0, 3.0):
                g = dual_step_size(r2, t, 1.0, beta0)
                ref = _largest_gamma(r2, t, 1.0, beta0)
                assert abs(g - ref) <= 1e-12 * beta0
