"""Pins for the oracle's Nystrom sketch (Section 5, Appendix B).

* exact recovery when rank X <= R (Appendix B, "statistical properties": the
  approximation is exact for low-rank inputs);
* agreement with the pseudo-inverse definition (eqn nystrom-supp);
* the exact error identity err_r = ||X - [[X_hat]]_r||_* (eqn sketch-err-supp);
* X_hat <= X in the psd order; trace correction gives trace alpha and at most
  doubles the error (eqn trace-correct-supp).
"""
import numpy as np
import pytest

import synth
from oracle import OracleParams, sketchy_cgal
from oracle.sketchycgal import nystrom_reconstruct, NystromSketch, gaussian_test_matrix


def _psd(n, rng, decay):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = decay ** np.arange(n)
    return (Q * ev) @ Q.T


def _nuc(A):
    return np.abs(np.linalg.eigvalsh(0.5 * (A + A.T))).sum()


def test_exact_for_low_rank():
    rng = np.random.default_rng(0)
    n, R, r = 50, 6, 3
    G = rng.standard_normal((n, r))
    X = G @ G.T
    Om = rng.standard_normal((n, R))
    out = nystrom_reconstruct(X @ Om, Om, np.trace(X))
    Xh = (out["U"] * out["lam_raw"]) @ out["U"].T
    assert np.abs(Xh - X).max() < 1e-8 * np.abs(X).max()
    assert np.abs(out["U"].T @ out["U"] - np.eye(R)).max() < 1e-10
    assert out["err"][r - 1] < 1e-8 * np.trace(X)
    # the shift sigma is removed: the R - r trailing values of the shifted
    # sketch's approximation are sigma (up to rounding), so Lambda there is ~0
    assert out["sigma"] > 0
    assert np.all(out["lam_raw"][r:] < 0.5 * out["sigma"])


def test_matches_pseudoinverse_definition():
    rng = np.random.default_rng(1)
    n, R = 60, 8
    X = _psd(n, rng, 0.7)
    Om = rng.standard_normal((n, R))
    S = X @ Om
    out = nystrom_reconstruct(S, Om, np.trace(X))
    Xh = (out["U"] * out["lam_raw"]) @ out["U"].T
    ref = S @ np.linalg.pinv(Om.T @ S) @ S.T
    assert np.abs(Xh - ref).max() < 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("decay", [0.9, 0.6])
def test_error_identity_and_order(decay):
    rng = np.random.default_rng(2)
    n, R = 60, 10
    X = _psd(n, rng, decay)
    Om = rng.standard_normal((n, R))
    out = nystrom_reconstruct(X @ Om, Om, np.trace(X), alpha=np.trace(X))
    U, lam = out["U"], out["lam_raw"]
    assert np.all(np.diff(lam) <= 1e-15)
    for r in range(1, R + 1):
        Xr = (U[:, :r] * lam[:r]) @ U[:, :r].T
        assert abs(out["err"][r - 1] - _nuc(X - Xr)) < 1e-9 * np.trace(X)
    Xh = (U * lam) @ U.T
    assert np.linalg.eigvalsh(X - Xh).min() > -1e-10
    Xt = (U * out["lam"]) @ U.T
    assert abs(np.trace(Xt) - np.trace(X)) < 1e-12 * np.trace(X)
    assert _nuc(X - Xt) <= 2 * _nuc(X - Xh) + 1e-12


def test_sketch_of_sketchycgal_run_recovers_implicit_iterate():
    """After t-1 <= R iterations X_t has rank <= R, so the sketch recovers it."""
    inst = synth.laplacian_instance(synth.erdos_renyi(30, 90, seed=5))
    prm = OracleParams(R=8, T=6, seed=3)
    res = sketchy_cgal(inst.to_scipy(), inst.b, prm, record_v=True)
    X = np.zeros((30, 30))
    for t, v in enumerate(res.vs, start=1):
        eta = 2.0 / (t + 1)
        X = (1 - eta) * X + eta * res.alpha_s * np.outer(v, v)
    out = nystrom_reconstruct(res.S, res.Omega, res.tau)
    Xh = (out["U"] * out["lam_raw"]) @ out["U"].T
    assert np.abs(Xh - X).max() < 1e-9 * np.abs(X).max()


def test_rank_one_update_matches_definition():
    rng = np.random.default_rng(4)
    Om = rng.standard_normal((20, 4))
    sk = NystromSketch(Om)
    X = np.zeros((20, 20))
    for eta in (1.0, 0.5, 0.25):
        v = rng.standard_normal(20)
        sk.rank_one_update(v, eta)
        X = (1 - eta) * X + eta * np.outer(v, v)
        assert np.abs(sk.S - X @ Om).max() < 1e-12
        assert abs(sk.tau - np.trace(X)) < 1e-12


def test_test_matrix_columns_are_independent_normals():
    Om = gaussian_test_matrix(20000, 5, seed=9)
    assert Om.shape == (20000, 5)
    C = np.corrcoef(Om.T)
    assert np.abs(C - np.eye(5)).max() < 0.05
    assert abs(Om.var() - 1) < 0.03
