"""Pins for the oracle's randomized Lanczos (alg:rand-lanczos, Fact rand-lanczos).

* The tridiagonal T_k must equal Q^T M Q for an orthonormal basis Q of the
  Krylov space K_k(M, g), built here by QR of explicit Krylov vectors.
* Ritz values interlace: xi >= lambda_min(M).
* Accuracy after the iteration count of the Fact (probabilistic bound).
* Exact answer at breakdown when M has few distinct eigenvalues.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle.sketchycgal import approx_min_evec, approx_min_evec_regenerated, tridiag_min_eigpair


def _sym(n, rng, spread=1.0):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.sort(rng.uniform(-spread, spread, n))
    return (Q * ev) @ Q.T, ev


def _lanczos_coeffs(M, g, q, reorth=0):
    xi, v, info = approx_min_evec(lambda x: M @ x, g, q, reorth)
    return xi, v, info


@pytest.mark.parametrize("reorth", [0, 1, 2])
@pytest.mark.parametrize("k", [2, 3, 5, 6])
def test_tridiagonal_is_projection_on_krylov_space(k, reorth):
    rng = np.random.default_rng(k)
    n = 40
    M, _ = _sym(n, rng)
    g = rng.standard_normal(n)
    # k Lanczos steps produce omega_1..k and rho_1..k-1 (any reorthogonalisation
    # leaves them unchanged in exact arithmetic)
    _, _, info = _lanczos_coeffs(M, g, k, reorth)
    K = np.empty((n, k))
    x = g / np.linalg.norm(g)
    for j in range(k):
        K[:, j] = x
        x = M @ x
        x = x / np.linalg.norm(x)
    Q, _ = np.linalg.qr(K)
    T = Q.T @ M @ Q
    np.testing.assert_allclose(info["omega"], np.diag(T), rtol=0, atol=1e-11)
    np.testing.assert_allclose(info["rho"], np.abs(np.diag(T, 1)), rtol=0, atol=1e-11)
    # T is tridiagonal in that basis
    assert np.abs(np.triu(T, 2)).max() < 1e-10


@pytest.mark.parametrize("reorth", [0, 1, 2])
def test_ritz_value_interlaces_and_converges(reorth):
    rng = np.random.default_rng(11)
    n = 120
    M, ev = _sym(n, rng)
    g = rng.standard_normal(n)
    prev = np.inf
    for q in (2, 5, 10, 20, 40, n - 1):
        xi, v, info = _lanczos_coeffs(M, g, q, reorth)
        assert xi >= ev[0] - 1e-12
        assert abs(np.linalg.norm(v) - 1.0) < 1e-13
        # Ritz values of nested Krylov spaces decrease monotonically
        assert xi <= prev + 1e-12
        prev = xi
    assert abs(xi - ev[0]) < 1e-9
    resid = np.linalg.norm(M @ v - xi * v)
    assert resid < 1e-6


def test_fact_rand_lanczos_bound():
    """u^T M u <= lambda_min + eps/8 ||M|| after q >= 1/2 + eps^(-1/2) log(n/delta^2)."""
    rng = np.random.default_rng(5)
    n, eps, delta = 200, 0.05, 0.1
    q = int(math.ceil(0.5 + eps ** -0.5 * math.log(n / delta ** 2)))
    fails = 0
    for trial in range(20):
        M, ev = _sym(n, rng)
        g = rng.standard_normal(n)
        _, v, _ = _lanczos_coeffs(M, g, q)
        normM = np.abs(ev).max()
        if v @ M @ v > ev[0] + eps / 8 * normM:
            fails += 1
    # failure probability is at most 2 delta per trial
    assert fails <= 4


@pytest.mark.parametrize("regenerated", [False, True])
def test_breakdown_returns_exact_minimum(regenerated):
    rng = np.random.default_rng(3)
    n = 30
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.repeat([-2.0, 0.5, 3.0], 10)
    M = (Q * ev) @ Q.T
    g = rng.standard_normal(n)
    if regenerated:
        xi, v, info = approx_min_evec_regenerated(lambda x: M @ x, g, n - 1)
    else:
        xi, v, info = _lanczos_coeffs(M, g, n - 1)
    assert info["broke"] and info["k"] == 3
    assert abs(xi + 2.0) < 1e-12
    assert np.linalg.norm(M @ v + 2.0 * v) < 1e-10


@pytest.mark.parametrize("q", [1, 2, 7, 30, 59])
def test_regenerated_basis_gives_the_stored_basis_result(q):
    # Section 4.2: the second sweep rebuilds the same vectors, so the Ritz pair is
    # the stored-basis one; checked also against the Krylov-space Rayleigh-Ritz
    # solution built from scratch (dense eigh of Q^T M Q).
    rng = np.random.default_rng(100 + q)
    n = 60
    M, ev = _sym(n, rng)
    g = rng.standard_normal(n)
    xs, vs, infos = approx_min_evec(lambda x: M @ x, g, q)
    xr, vr, infor = approx_min_evec_regenerated(lambda x: M @ x, g, q)
    assert infor["k"] == infos["k"] == q and not infor["broke"]
    assert xr == xs
    np.testing.assert_array_equal(infor["omega"], infos["omega"])
    np.testing.assert_allclose(vr, vs, rtol=0, atol=1e-14)
    K = np.empty((n, q))
    x = g / np.linalg.norm(g)
    for j in range(q):
        K[:, j] = x
        x = M @ x
        x = x / np.linalg.norm(x)
    Qk, _ = np.linalg.qr(K)
    w, Y = np.linalg.eigh(Qk.T @ M @ Qk)
    u = Qk @ Y[:, 0]
    assert abs(xr - w[0]) < 1e-9 * max(1.0, abs(w[0]))
    if q < 30:   # explicit Krylov vectors lose rank beyond that
        assert abs(abs(u @ vr) - 1.0) < 1e-8


def test_tridiagonal_solver_against_dense():
    rng = np.random.default_rng(9)
    for k in (1, 2, 7, 40):
        d = rng.standard_normal(k)
        e = rng.uniform(0.1, 1.0, max(k - 1, 0))
        xi, u = tridiag_min_eigpair(d, e)
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        w, V = np.linalg.eigh(T)
        assert abs(xi - w[0]) < 1e-13
        assert abs(abs(u @ V[:, 0]) - 1.0) < 1e-10


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_local_reorthogonalisation(seed):
    # reorth = 1 keeps each new vector orthogonal to the two before it to about
    # one ulp, where the plain recurrence (or a pass against the last vector
    # only) drifts to 1e-15..1e-13 once the Ritz values converge; the
    # regenerated form reproduces the stored one
    rng = np.random.default_rng(seed)
    n, q = 80, 60
    M, ev = _sym(n, rng)
    ev = ev.copy()
    Q = np.linalg.eigh(M)[1]
    ev[0], ev[1] = -3.0, -2.5          # a separated minimum: fast convergence
    M = (Q * ev) @ Q.T
    g = rng.standard_normal(n)

    def local_orth(reorth):
        B = []
        out = approx_min_evec(lambda x: (B.append(x.copy()), M @ x)[1], g, q, reorth)
        m1 = max(abs(B[i] @ B[i - 1]) for i in range(1, len(B)))
        m2 = max(abs(B[i] @ B[i - 2]) for i in range(2, len(B)))
        return out, max(m1, m2)

    (xi_s, v_s, info_s), o1 = local_orth(1)
    _, o0 = local_orth(0)
    assert o1 < 3e-16 < 1e-15 < o0
    xi_r, v_r, info_r = approx_min_evec_regenerated(lambda x: M @ x, g, q, 1)
    assert xi_r == xi_s
    np.testing.assert_array_equal(info_r["omega"], info_s["omega"])
    np.testing.assert_allclose(v_r, v_s, rtol=0, atol=1e-14)
    assert abs(xi_s + 3.0) < 1e-12
    with pytest.raises(ValueError):
        approx_min_evec_regenerated(lambda x: M @ x, g, q, 2)
