"""Pins of the phase retrieval oracle against what the paper and the mathematics fix.

* The measurement operator (Section 7.3.1, Appendix F.1) against measurement
  vectors a_{j,l} built explicitly from their definition (dense DFT rows
  times the waveform), and against the generator's measurements.
* The adjoint against the dense matrix sum_i w_i a_i a_i^*.
* The closed form of ||A|| (reading P1) against the largest eigenvalue of the
  explicit Gram matrix <A_i, A_k> = |a_i^* a_k|^2, for the paper's waveforms
  and for complex Gaussian ones; the scaled operator has ||A|| = 1 and equal
  ||A_i||_F (eqn problem-scaling).
* Complex randomized Lanczos run to a full Krylov space against a dense
  Hermitian eigensolver.
* The implicit state of the loop (z = A(X), S = X Omega, p = <C, X>,
  tau = tr X) against a dense run that keeps X itself and forms D_t as an
  explicit matrix.
* The complex Nystrom reconstruction is exact on a sketch of a matrix of rank
  at most R.
* The relative error's closed form against a search over the global phase.
* A small instance is solved to the paper's success criterion (relative error
  below 1e-2, Section 7.3.4).
"""
import math

import numpy as np
import pytest

from synth.phase import coded_diffraction
from oracle.phase_retrieval import (CDPOperator, PhaseParams, approx_min_evec_complex, complex_start_vector,
                                    complex_test_matrix, nystrom_reconstruct_complex, operator_norm,
                                    relative_error, round_phase, scale_phase, sketchy_cgal_phase)
from oracle.sketchycgal import lanczos_q


def explicit_vectors(psi):
    """a_{j,l} with a^* x = sum_m exp(-2 pi i l m / n) conj(psi_j(m)) x_m, as rows of an (L n) x n array."""
    L, n = psi.shape
    l = np.arange(n)[:, None]
    m = np.arange(n)[None, :]
    W = np.exp(-2j * np.pi * l * m / n)              # DFT matrix, entry (l, m)
    rows = []
    for j in range(L):
        rows.append(np.conj(W * np.conj(psi[j])[None, :]))   # a = conj(row of W diag(conj psi))
    return np.concatenate(rows, axis=0)


@pytest.mark.parametrize("n,L", [(6, 3), (7, 2), (12, 4)])
def test_forward_matches_explicit_vectors_and_generator(n, L):
    inst = coded_diffraction(n, 11, L=L)
    A = explicit_vectors(inst.psi)
    b_explicit = np.abs(A.conj() @ inst.chi) ** 2
    op = CDPOperator(inst.psi)
    assert np.allclose(op.forward(inst.chi).reshape(-1), b_explicit, rtol=1e-12, atol=1e-12)
    assert np.allclose(inst.b.reshape(-1), b_explicit, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("masks", ["cdp", "gaussian"])
def test_adjoint_matches_dense_sum(masks):
    n, L = 10, 3
    inst = coded_diffraction(n, 5, L=L, masks=masks)
    rng = np.random.default_rng(3)
    s = rng.uniform(0.5, 2.0, L)
    w = rng.standard_normal((L, n))
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    A = explicit_vectors(inst.psi)
    wt = (s[:, None] * w).reshape(-1)
    D = (A.T * wt) @ A.conj()                        # sum_i wt_i a_i a_i^*
    assert np.allclose(D, D.conj().T)
    op = CDPOperator(inst.psi, s)
    assert np.allclose(op.adjoint_apply(w, v), D @ v, rtol=1e-12, atol=1e-11)


def test_adjoint_identity_at_size():
    n, L = 1000, 12
    inst = coded_diffraction(n, 9, L=L)
    rng = np.random.default_rng(1)
    w = rng.standard_normal((L, n))
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    op = CDPOperator(inst.psi)
    lhs = float(np.sum(op.forward(v) * w))           # <A(v v^*), w>
    rhs = complex(np.vdot(v, op.adjoint_apply(w, v)))  # <v v^*, A^*(w)> = v^* A^*(w) v
    assert abs(rhs.imag) < 1e-9 * abs(rhs.real)
    assert abs(lhs - rhs.real) < 1e-12 * abs(lhs) * n


def explicit_gram_norm(psi, s):
    A = explicit_vectors(psi)
    wt = np.repeat(s, psi.shape[1])
    G = np.abs(A.conj() @ A.T) ** 2 * np.outer(wt, wt)   # <A_i, A_k> = |a_i^* a_k|^2
    return math.sqrt(float(np.linalg.eigvalsh(G)[-1]))


@pytest.mark.parametrize("masks,n,L", [("cdp", 8, 4), ("cdp", 9, 12), ("gaussian", 8, 3), ("gaussian", 5, 6)])
def test_operator_norm_closed_form_matches_gram(masks, n, L):
    inst = coded_diffraction(n, 21, L=L, masks=masks)
    rng = np.random.default_rng(n)
    s = rng.uniform(0.3, 3.0, L)
    assert abs(operator_norm(inst.psi, s) - explicit_gram_norm(inst.psi, s)) < 1e-12 * explicit_gram_norm(inst.psi, s)


def test_scaling_gives_unit_norm_equal_frobenius_norms():
    n, L = 9, 5
    inst = coded_diffraction(n, 4, L=L)
    alpha = 3.0 * n
    s, bs, alpha_s, c_F = scale_phase(inst.psi, inst.b, alpha)
    assert alpha_s == 1.0 and c_F == math.sqrt(n)
    A = explicit_vectors(inst.psi)
    fro = np.repeat(s, n) * np.sum(np.abs(A) ** 2, axis=1)   # ||s a a^*||_F = s ||a||^2
    assert np.ptp(fro) < 1e-13 * fro.max()
    assert abs(explicit_gram_norm(inst.psi, s) - 1.0) < 1e-12
    # b_s is the scaled operator applied to X = chi chi^* / alpha
    assert np.allclose(bs, CDPOperator(inst.psi, s).forward(inst.chi) / alpha, rtol=1e-12, atol=0)


def test_complex_lanczos_full_krylov_space_is_exact():
    n = 12
    rng = np.random.default_rng(8)
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    D = 0.5 * (M + M.conj().T)
    g = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    xi, v, info = approx_min_evec_complex(lambda x: D @ x, g, n)
    lam = np.linalg.eigvalsh(D)
    assert abs(xi - lam[0]) < 1e-12 * np.abs(lam).max()
    assert np.linalg.norm(D @ v - xi * v) < 1e-10 * np.abs(lam).max()
    assert abs(np.linalg.norm(v) - 1.0) < 1e-14


def dense_phase_cgal(psi, b, prm, T):
    """The same iteration keeping X (n x n) itself and D_t as an explicit matrix."""
    L, n = psi.shape
    alpha0 = 3.0 * n
    s, bs, alpha, c_F = scale_phase(psi, b, alpha0)
    A = explicit_vectors(psi)
    wt_s = np.repeat(s, n)
    Omega = complex_test_matrix(n, prm.R, prm.seed)
    X = np.zeros((n, n), dtype=complex)
    y = np.zeros(L * n)
    bsv = bs.reshape(-1)

    def measure(X):
        return wt_s * np.real(np.einsum("ij,jk,ik->i", A.conj(), X, A))

    out = []
    for t in range(1, T + 1):
        beta = prm.beta0 * math.sqrt(t + 1.0)
        eta = 2.0 / (t + 1.0)
        z = measure(X)
        w = y + beta * (z - bsv)
        D = np.eye(n) / c_F + (A.T * (wt_s * w)) @ A.conj()
        q = lanczos_q(t, n)
        xi, v, _ = approx_min_evec_complex(lambda x: D @ x, complex_start_vector(n, prm.seed, t), q)
        H = alpha * np.outer(v, v.conj()) if xi < 0 else np.zeros((n, n))
        gap = float(np.trace(D @ (X - H)).real)      # surrogate gap <D_t, X_t - H_t>
        X = (1 - eta) * X + eta * H
        zb = measure(X) - bsv
        r2 = float(zb @ zb)
        gamma = min(prm.beta0, 4 * alpha ** 2 * prm.beta0 / ((t + 1.0) ** 1.5 * r2)) if r2 > 0 else prm.beta0
        y = y + gamma * zb
        out.append(dict(z=measure(X), y=y.copy(), S=X @ Omega, p=float(np.trace(X).real) / c_F,
                        tau=float(np.trace(X).real), gap=gap))
    return out


def test_implicit_state_matches_dense_iteration():
    n, L, T = 8, 3, 25
    inst = coded_diffraction(n, 17, L=L)
    prm = PhaseParams(R=3, T=T, seed=5)
    dense = dense_phase_cgal(inst.psi, inst.b, prm, T)
    st = None
    for t in range(1, T + 1):
        res = sketchy_cgal_phase(inst.psi, inst.b, prm, state0=st, t_stop=t)
        st = dict(t=t + 1, z=res.z, y=res.y, p=res.p, S=res.S, tau=res.tau)
        d = dense[t - 1]
        scale = max(1.0, np.abs(d["z"]).max())
        assert np.abs(res.z.reshape(-1) - d["z"]).max() < 1e-10 * scale, t
        assert np.abs(res.y.reshape(-1) - d["y"]).max() < 1e-10 * max(1.0, np.abs(d["y"]).max()), t
        assert np.abs(res.S - d["S"]).max() < 1e-10 * max(1.0, np.abs(d["S"]).max()), t
        assert abs(res.p - d["p"]) < 1e-12 and abs(res.tau - d["tau"]) < 1e-12, t
        assert abs(res.log["gap"][-1] - d["gap"]) < 1e-10 * max(1.0, abs(d["gap"])), t
    assert (res.log["xi"] < 0).any()                 # the run reached the H != 0 branch


def test_nystrom_complex_exact_for_low_rank():
    n, R, r = 40, 5, 3
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r)))
    lam = np.array([3.0, 1.0, 0.25])
    X = (Q * lam) @ Q.conj().T
    Omega = complex_test_matrix(n, R, 9)
    rec = nystrom_reconstruct_complex(X @ Omega, Omega, float(np.trace(X).real))
    Xh = (rec["U"] * rec["lam_raw"]) @ rec["U"].conj().T
    assert np.abs(Xh - X).max() < 1e-12
    assert np.abs(rec["U"].conj().T @ rec["U"] - np.eye(R)).max() < 1e-12
    assert np.allclose(rec["lam_raw"][:3], lam, atol=1e-12) and np.all(rec["lam_raw"][3:] < 1e-12)
    # trace correction to a target adds (target - sum) / R to every eigenvalue
    rec2 = nystrom_reconstruct_complex(X @ Omega, Omega, 5.0, alpha=5.0)
    assert np.allclose(rec2["lam"], rec2["lam_raw"] + (5.0 - rec2["lam_raw"].sum()) / R)


def test_relative_error_closed_form_matches_phase_search():
    rng = np.random.default_rng(6)
    chi_nat = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    chi = 0.9 * np.exp(1.3j) * chi_nat + 0.2 * (rng.standard_normal(30) + 1j * rng.standard_normal(30))
    phis = np.linspace(0.0, 2 * np.pi, 200001)
    errs = [np.linalg.norm(np.exp(1j * ph) * chi - chi_nat) for ph in phis[::1000]]
    i = int(np.argmin(errs))
    fine = phis[max(0, i * 1000 - 1000): i * 1000 + 1001]
    best = min(np.linalg.norm(np.exp(1j * ph) * chi - chi_nat) for ph in fine) / np.linalg.norm(chi_nat)
    assert abs(relative_error(chi, chi_nat) - best) < 1e-9
    assert relative_error(np.exp(-0.7j) * chi_nat, chi_nat) < 1e-7
    # rounding of an exact rank-one reconstruction returns the signal up to phase
    U = (chi_nat / np.linalg.norm(chi_nat))[:, None]
    lam = np.array([float(np.vdot(chi_nat, chi_nat).real)])
    assert relative_error(round_phase(U, lam), chi_nat) < 1e-7


def test_small_instance_recovers_the_signal():
    inst = coded_diffraction(64, 123)
    prm = PhaseParams(R=5, T=1000, seed=7)
    res = sketchy_cgal_phase(inst.psi, inst.b, prm)
    rec = nystrom_reconstruct_complex(res.S, res.Omega, res.tau, alpha=res.tau)
    chi = round_phase(rec["U"], rec["lam"], res.alpha)
    assert relative_error(chi, inst.chi) < 1e-2
    # the objective tr X approaches the signal energy, the tracked trace equals p sqrt(n)
    energy = float(np.vdot(inst.chi, inst.chi).real)
    assert abs(res.objective / energy - 1.0) < 1e-2
    assert abs(res.tau - res.p * math.sqrt(64)) < 1e-12
