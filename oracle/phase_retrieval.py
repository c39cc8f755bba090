"""Plain FP64 SketchyCGAL for the phase retrieval SDP (oracle; test infrastructure only).

The problem (Section 7.3.1, eqn numerics-phase-retrieval-sdp): minimise tr X
over complex Hermitian psd X subject to A X = b and tr X <= alpha, where
(A X)_i = a_i^* X a_i = <a_i a_i^*, X> (eqn phase-retrieval-meas-linear).  The
measurement vectors come from coded diffraction patterns (Appendix F.1):
measurement (j, l) is entry l of DFT_n (conj(psi_j) * x), so

    A(v v^*)_{j,l}  = |(DFT_n (conj(psi_j) * v))_l|^2,
    A^*(w) v        = sum_j psi_j * DFT_n^* (w_j * DFT_n (conj(psi_j) * v)),

DFT_n unnormalised (numpy's fft) and DFT_n^* = n ifft.  The solver is the
trace-bounded SketchyCGAL (alg:sketchy-cgal with the set {tr X <= alpha} of
Appendix D.2; H = alpha v v^* when xi < 0, else 0) in complex arithmetic:
randomized Lanczos (alg:rand-lanczos) on the Hermitian D_t, the Nystrom sketch
(alg:nystrom-sketch-supp) with a complex test matrix, and the rounding of
Section 7.3.2 (chi = sqrt(lambda_1) u_1 from the top eigenpair of the
reconstruction) with the relative error of Section 7.3.3.

Readings (the library takes the same ones):
  P1  Scaling (eqn problem-scaling): C = I becomes I / sqrt(n); every A_i of
      waveform j is divided by ||a_i||^2 = ||psi_j||^2 (so all ||A_i||_F are
      equal) and then all by the norm N of the result, so ||A|| = 1; b is
      divided the same way and by alpha, alpha <- 1.  N has the closed form
      N^2 = n lambda_max(Q Q^T), Q_{j,m} = |psi_j(m)|^2 / ||psi_j||^2:
      <A_i, A_k> = |a_i^* a_k|^2 depends on l - l' only (circulant blocks),
      so the Gram matrix of the A_i splits by frequency and the zero
      frequency, whose entries bound all others, holds the top eigenvalue
      (pinned against the explicit Gram matrix in the tests).
  P2  alpha defaults to 3 n (Section 7.3.3).
  P3  The Lanczos start vector of iteration t and column c of Omega are
      complex with independent standard normal real and imaginary parts:
      complex element m is the Box-Muller pair (2m, 2m + 1) of the Philox
      stream (seed; t, instance, purpose 2) resp. (seed; c, instance,
      purpose 3).
  P4  Lanczos as in the MaxCut oracle (readings R1-R4): omega_i = Re(v^* D v),
      the tridiagonal matrix is real; no reorthogonalisation.
  P5  Nystrom reconstruction in complex arithmetic with the same shift rule
      (R9): B = Omega^* S_sigma made Hermitian, B = L L^*, M = S_sigma L^{-*},
      X_hat = U diag(max(0, s^2 - sigma)) U^*; trace correction to the tracked
      trace tau (R14, the set tr X <= alpha).
  P6  Rounding uses the top eigenpair of the (trace-corrected) reconstruction,
      in original units: chi = sqrt(alpha lambda_1) u_1.  The relative error
      min_phi ||e^{i phi} chi - chi_nat|| / ||chi_nat|| has the closed form
      sqrt(||chi||^2 + ||chi_nat||^2 - 2 |chi^* chi_nat|) / ||chi_nat||.
  P7  Logged per iteration (scaled units) as for MaxCut with trace_mode 1:
      q, k, xi, v^* C v, p, ||z - b||, gamma, gap; stopping quantities and
      the eigen-residual are not formed (NaN).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg as sla

from .philox import normal_stream
from .sketchycgal import EPS64, dual_step_size, lanczos_q, tridiag_min_eigpair

__all__ = ["PhaseParams", "PhaseResult", "complex_start_vector", "complex_test_matrix", "operator_norm",
           "scale_phase", "CDPOperator", "approx_min_evec_complex", "nystrom_reconstruct_complex",
           "sketchy_cgal_phase", "round_phase", "relative_error"]


@dataclasses.dataclass
class PhaseParams:
    R: int = 5
    T: int = 100
    beta0: float = 1.0
    K: float = math.inf
    alpha: float | None = None      # None: 3 n (P2)
    seed: int = 0
    q_mode: int = 0
    q_fixed: int = 0
    scale: bool = True
    trace_correct: bool = True
    instance: int = 0


def _complex_stream(n: int, seed: int, index: int, instance: int, purpose: int) -> np.ndarray:
    g = normal_stream(2 * n, seed, index, instance, purpose)
    return g[0::2] + 1j * g[1::2]


def complex_start_vector(n: int, seed: int, t: int, instance: int = 0) -> np.ndarray:
    """Start vector of alg:rand-lanczos for iteration t (P3)."""
    return _complex_stream(n, seed, t, instance, 2)


def complex_test_matrix(n: int, R: int, seed: int, instance: int = 0) -> np.ndarray:
    """Omega (n x R, complex) of NystromSketch.Init (P3)."""
    return np.stack([_complex_stream(n, seed, c, instance, 3) for c in range(R)], axis=1)


def operator_norm(psi: np.ndarray, weights: np.ndarray) -> float:
    """||A|| for A_{j,l} = weights_j a_{j,l} a_{j,l}^* (P1 closed form)."""
    n = psi.shape[1]
    Q = weights[:, None] * np.abs(psi) ** 2
    return math.sqrt(n * float(np.linalg.eigvalsh(Q @ Q.T)[-1]))


def scale_phase(psi: np.ndarray, b: np.ndarray, alpha: float, scale: bool = True):
    """Scaling of eqn problem-scaling for this problem (P1).
    Returns (s, b_s, alpha_s, c_F): the scaled operator is diag(s) A per waveform."""
    L, n = psi.shape
    if not scale:
        return np.ones(L), np.asarray(b, dtype=np.float64).copy(), float(alpha), 1.0
    s0 = 1.0 / np.sum(np.abs(psi) ** 2, axis=1)       # 1 / ||psi_j||^2 = 1 / ||A_i||_F
    s = s0 / operator_norm(psi, s0)
    return s, s[:, None] * b / alpha, 1.0, math.sqrt(n)


class CDPOperator:
    """A and A^* of the coded diffraction model, waveform j weighted by s_j."""

    def __init__(self, psi: np.ndarray, s: np.ndarray | None = None):
        self.psi = np.asarray(psi, dtype=np.complex128)
        self.L, self.n = self.psi.shape
        self.s = np.ones(self.L) if s is None else np.asarray(s, dtype=np.float64)

    def forward(self, v: np.ndarray) -> np.ndarray:
        """A(v v^*) as an L x n array: s_j |DFT_n (conj(psi_j) v)|^2."""
        f = np.fft.fft(np.conj(self.psi) * v[None, :], axis=1)
        return self.s[:, None] * (f.real ** 2 + f.imag ** 2)

    def adjoint_apply(self, w: np.ndarray, v: np.ndarray) -> np.ndarray:
        """A^*(w) v for w an L x n array."""
        f = np.fft.fft(np.conj(self.psi) * v[None, :], axis=1)
        g = self.n * np.fft.ifft((self.s[:, None] * w) * f, axis=1)
        return np.sum(self.psi * g, axis=0)


def approx_min_evec_complex(matvec, g: np.ndarray, q: int):
    """Randomized Lanczos (alg:rand-lanczos) for a Hermitian operator (P4)."""
    v = g / np.linalg.norm(g)
    basis = [v]
    omega, rho = [], []
    v_prev = np.zeros_like(v)
    rho_prev = 0.0
    broke = False
    for i in range(1, q + 1):
        u = matvec(v)
        om = float(np.vdot(v, u).real)
        u = u - om * v - rho_prev * v_prev
        r = float(np.linalg.norm(u))
        omega.append(om)
        if r <= 64.0 * EPS64 * (abs(om) + rho_prev):
            broke = True
            break
        if i == q:
            break
        rho.append(r)
        v_prev, v = v, u / r
        rho_prev = r
        basis.append(v)
    k = len(omega)
    xi, uu = tridiag_min_eigpair(np.array(omega), np.array(rho[: k - 1]))
    x = np.zeros_like(g)
    for j in range(k):
        x = x + uu[j] * basis[j]
    x = x / np.linalg.norm(x)
    return xi, x, {"k": k, "broke": broke, "omega": np.array(omega), "rho": np.array(rho[: k - 1])}


def nystrom_reconstruct_complex(S: np.ndarray, Omega: np.ndarray, tau: float, alpha: float | None = None):
    """NystromSketch.Reconstruct (alg:nystrom-sketch-supp) for a complex sketch (P5).
    Returns dict(U, lam_raw, lam, err, sigma) with X_hat = U diag(lam_raw) U^*."""
    S = np.asarray(S, dtype=np.complex128)
    Omega = np.asarray(Omega, dtype=np.complex128)
    n, R = S.shape
    sigma = math.sqrt(n) * float(np.spacing(np.float64(np.linalg.norm(S, 2))))
    for _ in range(4):
        S_sig = S + sigma * Omega
        B = Omega.conj().T @ S_sig
        B = 0.5 * (B + B.conj().T)
        try:
            Lc = np.linalg.cholesky(B)         # B = Lc Lc^*
            break
        except np.linalg.LinAlgError:
            sigma *= 10.0
    else:
        raise np.linalg.LinAlgError("Cholesky of Omega^* S_sigma failed after 3 shift increases")
    # M = S_sig Lc^{-*}:  M Lc^* = S_sig  <=>  Lc M^* = S_sig^*
    M = sla.solve_triangular(Lc, S_sig.conj().T, lower=True).conj().T
    U, sv, _ = np.linalg.svd(M, full_matrices=False)
    lam_raw = np.maximum(0.0, sv * sv - sigma)
    err = tau - np.cumsum(lam_raw)
    lam = lam_raw.copy()
    if alpha is not None:
        lam = lam + (alpha - lam.sum()) / R
    return {"U": U, "lam_raw": lam_raw, "lam": lam, "err": err, "sigma": sigma}


@dataclasses.dataclass
class PhaseResult:
    n: int
    L: int
    alpha: float          # original alpha
    s: np.ndarray         # per-waveform scaling of A
    c_F: float            # ||C||_F = sqrt(n) (1 unscaled)
    alpha_s: float
    b_s: np.ndarray       # L x n, scaled
    p: float
    z: np.ndarray         # L x n, scaled
    y: np.ndarray         # L x n, scaled
    S: np.ndarray         # n x R complex
    tau: float
    Omega: np.ndarray
    log: dict

    @property
    def objective(self) -> float:
        """tr X in the original units."""
        return self.c_F * self.alpha * self.p / self.alpha_s

    @property
    def infeasibility(self) -> float:
        """||A X - b|| in the original units."""
        return self.alpha / self.alpha_s * float(np.linalg.norm((self.z - self.b_s) / self.s[:, None]))


_LOG_KEYS = ("t", "q", "k", "xi", "cv", "p", "infeas", "gamma", "gap", "beta", "eta")


def sketchy_cgal_phase(psi: np.ndarray, b: np.ndarray, params: PhaseParams, Omega: np.ndarray | None = None,
                       state0: dict | None = None, t_stop: int | None = None,
                       start_vectors=None) -> PhaseResult:
    """SketchyCGAL (alg:sketchy-cgal, trace-bounded set of Appendix D.2) for the phase retrieval SDP.

    `b` is L x n (b[j, l] measurement l of waveform j, original units).
    `state0` = dict(t, z, y, p, S, tau) resumes from the state before iteration
    t (scaled units); iterations run up to `t_stop` (default T)."""
    psi = np.asarray(psi, dtype=np.complex128)
    L, n = psi.shape
    b = np.asarray(b, dtype=np.float64).reshape(L, n)
    alpha0 = 3.0 * n if params.alpha is None else float(params.alpha)
    s, bs, alpha, c_F = scale_phase(psi, b, alpha0, params.scale)
    op = CDPOperator(psi, s)
    c_scale = 1.0 / c_F                    # C_s = I / ||I||_F
    if Omega is None:
        Omega = complex_test_matrix(n, params.R, params.seed, params.instance)
    Omega = np.asarray(Omega, dtype=np.complex128)
    z = np.zeros((L, n))
    y = np.zeros((L, n))
    S = np.zeros((n, params.R), dtype=np.complex128)
    p = 0.0
    tau = 0.0
    t0 = 1
    if state0 is not None:
        t0 = int(state0["t"])
        z = np.array(state0["z"], dtype=np.float64).reshape(L, n)
        y = np.array(state0["y"], dtype=np.float64).reshape(L, n)
        p = float(state0["p"])
        S = np.array(state0["S"], dtype=np.complex128).reshape(n, params.R)
        tau = float(state0["tau"])
    beta0 = params.beta0
    log = {k: [] for k in _LOG_KEYS}
    for t in range(t0, (params.T if t_stop is None else t_stop) + 1):
        beta = beta0 * math.sqrt(t + 1.0)
        eta = 2.0 / (t + 1.0)
        w = y + beta * (z - bs)                    # D_t = C + A^*(w)
        q = lanczos_q(t, n, params.q_mode, params.q_fixed)
        g = start_vectors(t) if start_vectors is not None else complex_start_vector(n, params.seed, t,
                                                                                     params.instance)
        xi, v, info = approx_min_evec_complex(lambda x: c_scale * x + op.adjoint_apply(w, x), g, q)
        cv = c_scale * float(np.vdot(v, v).real)
        ha = alpha if xi < 0.0 else 0.0            # H = ha v v^*
        gap = p + float(np.sum(w * z)) - ha * xi
        p = (1.0 - eta) * p + eta * ha * cv
        z = (1.0 - eta) * z + eta * ha * op.forward(v)
        zb = z - bs
        r2 = float(np.sum(zb * zb))
        gamma = dual_step_size(r2, t, alpha, beta0)
        y_new = y + gamma * zb
        if np.linalg.norm(y_new) > params.K:
            gamma = 0.0
        else:
            y = y_new
        S = (1.0 - eta) * S + eta * ha * np.outer(v, v.conj() @ Omega)
        tau = (1.0 - eta) * tau + eta * ha * float(np.vdot(v, v).real)
        for key, val in zip(_LOG_KEYS, (t, q, info["k"], xi, cv, p, math.sqrt(r2), gamma, gap, beta, eta)):
            log[key].append(val)
    log = {k: np.array(v) for k, v in log.items()}
    return PhaseResult(n=n, L=L, alpha=alpha0, s=s, c_F=c_F, alpha_s=alpha, b_s=bs, p=p, z=z, y=y, S=S,
                       tau=tau, Omega=Omega, log=log)


def round_phase(U: np.ndarray, lam: np.ndarray, alpha_scale: float = 1.0) -> np.ndarray:
    """chi = sqrt(lambda_1) u_1 for the top eigenpair of U diag(lam) U^* times alpha_scale (P6)."""
    i = int(np.argmax(lam))
    return math.sqrt(max(0.0, float(lam[i])) * alpha_scale) * U[:, i]


def relative_error(chi: np.ndarray, chi_nat: np.ndarray) -> float:
    """min over phi of ||e^{i phi} chi - chi_nat|| / ||chi_nat|| (Section 7.3.3; closed form P6)."""
    a = float(np.vdot(chi, chi).real)
    c = float(np.vdot(chi_nat, chi_nat).real)
    m = abs(complex(np.vdot(chi, chi_nat)))
    return math.sqrt(max(0.0, a + c - 2.0 * m)) / math.sqrt(c)
