"""Plain FP64 SketchyCGAL for the MaxCut SDP (oracle; test infrastructure only).

Follows the paper step by step:
  * problem scaling                    Section 7.1.1, eqn problem-scaling
  * iteration                          Section 6.1, alg:sketchy-cgal
  * ApproxMinEvec (randomized Lanczos) Section 4.2, alg:rand-lanczos
  * dual step size                     eqn sketchy-cgal-dual-step
  * Nystrom sketch and reconstruction  Section 5 / Appendix B,
                                       alg:nystrom-sketch-supp, eqn sketch-err-supp
  * objective tracking, gap            Section 6.2 (p_t update, surrogate gap)
  * stopping quantities                Appendix E, eqn scgal-stopping-supp

Readings of points the paper leaves open (the library takes the same ones):
  R1  q_t = ceil(t^(1/4) ln n), at least 1, at most n - 1 (alg:rand-lanczos
      loop bound).  A fixed q is also supported.
  R2  rho_i is the norm of the new, unnormalised Lanczos vector (the listing
      writes the norm of v_i, which is a unit vector).
  R3  Breakdown: stop when rho_i <= 64 eps (|omega_i| + rho_{i-1}); T_k then
      uses omega_1..k and rho_1..k-1.  An exact zero test never fires.
  R4  The Ritz vector is renormalised to unit length.
  R5  The Lanczos basis is stored (Remark "time-storage tradeoff"); in exact
      arithmetic this equals regenerating it, which approx_min_evec_regenerated
      does (the storage-optimal form of Section 4.2).
  R6  gamma = beta0 when ||z - b|| = 0; ||A|| = 1 for A = diag.
  R7  Scaling: C <- C / ||C||_F, b <- b / alpha, alpha <- 1 (||A|| = 1 and
      ||A_i||_F = 1 already hold for A = diag).  Reported objective and
      infeasibility are converted back to the original units.
  R8  The objective tracker uses an explicit product C v; the same product
      gives the eigen-residual ||D v - xi v||.
  R9  sigma = sqrt(n) * eps(||S||_2) with eps the spacing of the storage
      precision of S; Omega^T S_sigma is symmetrised before Cholesky; on
      Cholesky failure sigma grows tenfold, at most three times.
  R10 Gap and stopping quantities at iteration t use the state before the
      update (p_t, z_t, y_t, beta_t) and xi_t in place of lambda_min(D_t), with
      the factor alpha on xi that the general trace bound alpha implies.
  R11 Reorthogonalisation is an option (approx_min_evec): reorth = 1 against the
      two most recent Lanczos vectors, reorth = 2 against all of them.
  R12 General template (Appendix D, alg:full-sketchy-cgal-supp) with A = diag and
      K a box {lo <= u <= hi}: the projection onto the box is the entrywise
      clamp (the inequality example of Appendix D.3 prints the negative part
      of w - b; the projection onto {u <= b} is b + (w - b)_- = min(w, b)).
      The scaling divides lo and hi by alpha like b.  The norm-constraint
      example of the same appendix is taken with the l2 norm, centred at b:
      proj(w) = b + (w - b) min(1, r / ||w - b||), r scaled like b.  The dual
      step rule of Appendix D.4 has the same bound as eqn sketchy-cgal-dual-step.
  R13 With H = 0 (trace-bounded set, xi >= 0) the sketch takes
      RankOneUpdate(0, eta), so it keeps following X_t+1 = (1 - eta) X_t.  The
      logged infeasibility is dist_K(z_t+1), the feasibility gap of Appendix E;
      the gap is <D_t, X_t - H_t>.
  R14 With tr X <= alpha the trace correction of the reconstruction targets the
      tracked trace tau = tr X_T instead of alpha.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .philox import normal_stream

EPS64 = np.finfo(np.float64).eps


@dataclasses.dataclass
class OracleParams:
    R: int = 10
    T: int = 100
    beta0: float = 1.0
    K: float = math.inf
    alpha: float | None = None      # None: sum(b) (MaxCut: n)
    seed: int = 0
    q_mode: int = 0                 # 0: ceil(t^(1/4) ln n); 1: fixed q_fixed
    q_fixed: int = 0
    scale: bool = True
    trace_correct: bool = True
    instance: int = 0
    reorth: int = 0                 # 0: none (paper); 1: local (last two vectors); 2: full
    trace_mode: int = 0             # 0: tr X = alpha (alpha Delta_n); 1: tr X <= alpha (Appendix D.2)


@dataclasses.dataclass
class OracleResult:
    n: int
    alpha: float          # original alpha
    c_F: float            # ||C||_F used for scaling (1 if unscaled)
    alpha_s: float        # alpha in scaled units
    b_s: np.ndarray       # b in scaled units
    p: float              # <C_s, X_T+1> in scaled units
    z: np.ndarray
    y: np.ndarray
    S: np.ndarray
    tau: float
    Omega: np.ndarray
    log: dict
    vs: list | None = None
    trace_mode: int = 0
    dist_K: float | None = None   # general template: dist_K(z_T+1), scaled units

    @property
    def objective(self) -> float:
        """<C, X> in the original units."""
        return self.c_F * self.alpha * self.p / self.alpha_s

    @property
    def infeasibility(self) -> float:
        """||diag(X) - b|| (general template: dist_K(diag X)) in the original units."""
        d = float(np.linalg.norm(self.z - self.b_s)) if self.dist_K is None else self.dist_K
        return self.alpha / self.alpha_s * d


def lanczos_q(t: int, n: int, q_mode: int = 0, q_fixed: int = 0) -> int:
    """Lanczos iteration count for CGAL iteration t (R1)."""
    if q_mode == 1:
        q = int(q_fixed)
    else:
        q = int(math.ceil(t ** 0.25 * math.log(n))) if n > 1 else 1
    return max(1, min(q, max(n - 1, 1)))


def start_vector(n: int, seed: int, t: int, instance: int = 0) -> np.ndarray:
    """randn(n, 1) of alg:rand-lanczos for CGAL iteration t."""
    return normal_stream(n, seed, t, instance, 0)


def gaussian_test_matrix(n: int, R: int, seed: int, instance: int = 0) -> np.ndarray:
    """Omega = randn(n, R) of NystromSketch.Init, as an n x R array."""
    return np.stack([normal_stream(n, seed, c, instance, 1) for c in range(R)], axis=1)


def scale_problem(C: sp.csr_matrix, b: np.ndarray, alpha: float, scale: bool = True):
    """Scaling of Section 7.1.1: returns (C_s, b_s, alpha_s, c_F)  (R7)."""
    if not scale:
        return C, b.astype(np.float64), float(alpha), 1.0
    c_F = float(np.sqrt(np.sum(C.data.astype(np.float64) ** 2)))
    if c_F == 0.0:
        c_F = 1.0
    return C / c_F, b / alpha, 1.0, c_F


def tridiag_min_eigpair(omega: np.ndarray, rho: np.ndarray):
    """Minimum eigenpair of tridiag(rho, omega, rho) (alg:rand-lanczos MinEvec)."""
    k = len(omega)
    if k == 1:
        return float(omega[0]), np.ones(1)
    w, u = sla.eigh_tridiagonal(np.asarray(omega, dtype=np.float64), np.asarray(rho, dtype=np.float64),
                                select="i", select_range=(0, 0))
    return float(w[0]), u[:, 0]


def approx_min_evec(matvec, g: np.ndarray, q: int, reorth: int = 0):
    """Randomized Lanczos ApproxMinEvec (alg:rand-lanczos) with a stored basis.

    `g` is the Gaussian start vector, `q` the iteration cap (already limited
    to n - 1).  Returns (xi, v, info) with v a unit vector.

    reorth = 2 adds one classical Gram-Schmidt pass of the new vector against
    every stored Lanczos vector after the three-term recurrence (full
    reorthogonalisation; not in the paper's listing, which has none);
    reorth = 1 makes the same pass against the two most recent ones only
    (local reorthogonalisation, O(n) per step).
    """
    v = g / np.linalg.norm(g)
    basis = [v]
    omega, rho = [], []
    v_prev = np.zeros_like(v)
    rho_prev = 0.0
    broke = False
    for i in range(1, q + 1):
        u = matvec(v)
        om = float(np.dot(v, u))
        u = u - om * v - rho_prev * v_prev
        if reorth in (1, 2):
            Vm = np.stack(basis if reorth == 2 else basis[-2:], axis=1)
            u = u - Vm @ (Vm.T @ u)
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


def approx_min_evec_regenerated(matvec, g: np.ndarray, q: int, reorth: int = 0):
    """Storage-optimal randomized Lanczos (alg:rand-lanczos as Section 4.2 states it).

    Only the two most recent Lanczos vectors are ever held.  The first sweep
    records the tridiagonal coefficients; the minimum eigenvector u of T_k is
    computed; the second sweep restarts the same recurrence from the same
    start vector and sums u_j v_j as the vectors come back.  Returns what
    approx_min_evec returns (reading R5: in exact arithmetic the two agree).
    reorth = 1 (local reorthogonalisation) needs only the vectors held here.
    """
    if reorth not in (0, 1):
        raise ValueError("the regenerated basis supports reorth 0 or 1")
    def sweep(coef):
        v = g / np.linalg.norm(g)
        v_prev = np.zeros_like(v)
        rho_prev = 0.0
        omega, rho = [], []
        x = np.zeros_like(g)
        broke = False
        for i in range(1, q + 1):
            if coef is not None:
                if i > len(coef):
                    break
                x = x + coef[i - 1] * v
            u = matvec(v)
            om = float(np.dot(v, u))
            u = u - om * v - rho_prev * v_prev
            if reorth == 1:
                Vm = np.stack([v] if i == 1 else [v_prev, v], axis=1)
                u = u - Vm @ (Vm.T @ u)
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
        return omega, rho, broke, x

    omega, rho, broke, _ = sweep(None)
    k = len(omega)
    xi, uu = tridiag_min_eigpair(np.array(omega), np.array(rho[: k - 1]))
    _, _, _, x = sweep(uu)
    x = x / np.linalg.norm(x)
    return xi, x, {"k": k, "broke": broke, "omega": np.array(omega), "rho": np.array(rho[: k - 1])}


def dual_step_size(r2: float, t: int, alpha: float, beta0: float, normA: float = 1.0) -> float:
    """Largest gamma with gamma*r2 <= 4 alpha^2 beta0 ||A||^2 / (t+1)^(3/2), 0 <= gamma <= beta0."""
    if r2 == 0.0:
        return beta0
    return min(beta0, 4.0 * alpha * alpha * beta0 * normA * normA / ((t + 1.0) ** 1.5 * r2))


class NystromSketch:
    """Nystrom sketch (S = X Omega, tau = tr X) of Section 5 / Appendix B."""

    def __init__(self, Omega: np.ndarray):
        self.Omega = np.asarray(Omega, dtype=np.float64)
        self.n, self.R = self.Omega.shape
        self.S = np.zeros((self.n, self.R))
        self.tau = 0.0

    def rank_one_update(self, v: np.ndarray, eta: float):
        """S <- (1-eta) S + eta v (v^T Omega);  tau <- (1-eta) tau + eta ||v||^2."""
        self.S = (1.0 - eta) * self.S + eta * np.outer(v, v @ self.Omega)
        self.tau = (1.0 - eta) * self.tau + eta * float(np.dot(v, v))

    def reconstruct(self, alpha: float | None = None, storage: str = "f64"):
        return nystrom_reconstruct(self.S, self.Omega, self.tau, alpha=alpha, storage=storage)


def _spacing(x: float, storage: str) -> float:
    if storage == "f32":
        return float(np.spacing(np.float32(x)))
    return float(np.spacing(np.float64(x)))


def nystrom_reconstruct(S: np.ndarray, Omega: np.ndarray, tau: float, alpha: float | None = None,
                        storage: str = "f64"):
    """NystromSketch.Reconstruct (alg:nystrom-sketch-supp) plus trace correction.

    Returns dict(U, lam_raw, lam, err, sigma): X_hat = U diag(lam_raw) U^T;
    `lam` is trace-corrected to `alpha` when alpha is given
    (alg:sketchy-cgal, eqn trace-correct-supp); err_r = tau - sum_{j<=r} lam_raw_j
    (eqn sketch-err-supp).
    """
    S = np.asarray(S, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    n, R = S.shape
    sigma = math.sqrt(n) * _spacing(float(np.linalg.norm(S, 2)), storage)
    for _ in range(4):
        S_sig = S + sigma * Omega
        B = Omega.T @ S_sig
        B = 0.5 * (B + B.T)
        try:
            Lc = np.linalg.cholesky(B)         # B = Lc Lc^T; MATLAB chol gives L = Lc^T
            break
        except np.linalg.LinAlgError:
            sigma *= 10.0
    else:
        raise np.linalg.LinAlgError("Cholesky of Omega^T S_sigma failed after 3 shift increases")
    # M = S_sig / L with L = Lc^T upper:  M Lc^T = S_sig  <=>  Lc M^T = S_sig^T
    M = sla.solve_triangular(Lc, S_sig.T, lower=True).T
    U, sv, _ = np.linalg.svd(M, full_matrices=False)
    lam_raw = np.maximum(0.0, sv * sv - sigma)
    err = tau - np.cumsum(lam_raw)
    lam = lam_raw.copy()
    if alpha is not None:
        lam = lam + (alpha - lam.sum()) / R
    return {"U": U, "lam_raw": lam_raw, "lam": lam, "err": err, "sigma": sigma}


def maxcut_dual_bound(C: np.ndarray, b: np.ndarray, y: np.ndarray, alpha: float) -> float:
    """Dual function phi(y) = alpha lambda_min(C + diag y) - <y, b>  (Appendix E,
    eqn model-dual-function-supp); phi(y) <= min <C, X> for every y (dense; small n)."""
    D = np.asarray(C, dtype=np.float64) + np.diag(y)
    lam = float(np.linalg.eigvalsh(D)[0])
    return alpha * lam - float(np.dot(y, b))


_LOG_KEYS = ("t", "q", "k", "xi", "cv", "p", "infeas", "gamma", "gap", "stop_obj", "stop_feas",
             "resid", "beta", "eta")


def sketchy_cgal(C: sp.csr_matrix, b: np.ndarray, params: OracleParams, Omega: np.ndarray | None = None,
                 record_v: bool = False, start_vectors=None, state0: dict | None = None,
                 t_stop: int | None = None, lo: np.ndarray | None = None,
                 hi: np.ndarray | None = None, radius: float | None = None) -> OracleResult:
    """SketchyCGAL (alg:sketchy-cgal) for min <C,X> s.t. diag X = b, X in alpha*Delta_n,
    and its general template (Appendix D, alg:full-sketchy-cgal-supp) with A = diag.

    General template: given `lo` and/or `hi` (original units; a missing side is
    unbounded), the constraint is diag X in K = {u : lo <= u <= hi} and every
    use of b in the iteration becomes a projection onto K (R12); b then only
    supplies the default alpha = sum(b).  Given `radius` instead, K is the
    ball {u : ||u - b|| <= radius} (the norm-constraint example of Appendix
    D.3, l2 norm), centred at b.  trace_mode = 1 replaces
    X in alpha*Delta_n by tr X <= alpha, whose linear minimisation returns
    H = alpha v v^T when xi < 0 and H = 0 otherwise (Appendix D.2).

    `start_vectors(t)` may override the Philox start vector of iteration t.
    `state0` = dict(t, z, y, p, S, tau) resumes from the state before
    iteration t (scaled units); iterations run up to `t_stop` (default T).
    Logged per iteration (scaled units): q, Lanczos steps k, xi, v^T C v, p_t,
    dist_K(z_t+1) (= ||z_t+1 - b|| for K = {b}), gamma, gap, the two stopping
    quantities (K = {b} with tr X = alpha only, else NaN), ||D v - xi v||.
    """
    C = sp.csr_matrix(C, dtype=np.float64)
    n = C.shape[0]
    b = np.asarray(b, dtype=np.float64)
    alpha0 = float(b.sum()) if params.alpha is None else float(params.alpha)
    Cs, bs, alpha, c_F = scale_problem(C, b, alpha0, params.scale)
    box = lo is not None or hi is not None
    ball = radius is not None
    if box and ball:
        raise ValueError("K is a box or a ball, not both")
    if ball:
        rad_s = float(radius) / (alpha0 if params.scale else 1.0)

        def proj(u):   # Euclidean projection onto the ball K (Appendix D.3): b + (u - b) min(1, r / ||u - b||)
            d = u - bs
            nd = float(np.linalg.norm(d))
            c = 1.0 if nd <= rad_s else rad_s / nd
            return bs + c * d
    elif box:
        sK = alpha0 if params.scale else 1.0    # the scaling divides the constraint values by alpha
        lo_s = np.full(n, -np.inf) if lo is None else np.asarray(lo, dtype=np.float64) / sK
        hi_s = np.full(n, np.inf) if hi is None else np.asarray(hi, dtype=np.float64) / sK

        def proj(u):   # Euclidean projection onto the box K (Appendix D.3)
            return np.minimum(np.maximum(u, lo_s), hi_s)
    else:
        def proj(u):   # K = {b}
            return bs
    if Omega is None:
        Omega = gaussian_test_matrix(n, params.R, params.seed, params.instance)
    sketch = NystromSketch(Omega)
    z = np.zeros(n)
    y = np.zeros(n)
    p = 0.0
    t0 = 1
    if state0 is not None:
        t0 = int(state0["t"])
        z = np.array(state0["z"], dtype=np.float64)
        y = np.array(state0["y"], dtype=np.float64)
        p = float(state0["p"])
        sketch.S = np.array(state0["S"], dtype=np.float64)
        sketch.tau = float(state0["tau"])
    beta0 = params.beta0
    log = {k: [] for k in _LOG_KEYS}
    vs = [] if record_v else None
    nb = float(np.linalg.norm(bs))
    for t in range(t0, (params.T if t_stop is None else t_stop) + 1):
        beta = beta0 * math.sqrt(t + 1.0)
        eta = 2.0 / (t + 1.0)
        wK = proj(z + y / beta)              # slack w_t = proj_K(z + y / beta)
        w = y + beta * (z - wK)              # D = C + diag(w)
        q = lanczos_q(t, n, params.q_mode, params.q_fixed)
        g = start_vectors(t) if start_vectors is not None else start_vector(n, params.seed, t, params.instance)
        xi, v, info = approx_min_evec(lambda x: Cs @ x + w * x, g, q, params.reorth)
        Cv = Cs @ v
        cv = float(np.dot(v, Cv))
        resid = float(np.linalg.norm(Cv + w * v - xi * v))
        # linear minimisation over the trace set: H = ha v v^T
        ha = alpha if (params.trace_mode == 0 or xi < 0.0) else 0.0
        # surrogate gap <D_t, X_t - H_t> with <D_t, X_t> = p_t + <w, z_t> and <D_t, H_t> = ha xi
        gap = p + float(np.dot(w, z)) - ha * xi
        if not (box or ball) and params.trace_mode == 0:
            zb = z - bs
            stop_obj = (p + float(np.dot(y, bs)) + 0.5 * beta * float(np.dot(zb, z + bs)) - alpha * xi) / (1.0 + abs(p))
            stop_feas = float(np.linalg.norm(zb)) / (1.0 + nb)
        else:
            stop_obj = stop_feas = math.nan
        # primal state, objective tracker and dual (alg:sketchy-cgal; Section 6.2)
        p = (1.0 - eta) * p + eta * ha * cv
        z = (1.0 - eta) * z + eta * ha * (v * v)
        zb = z - proj(z + y / (beta0 * math.sqrt(t + 2.0)))   # z - w_bar
        r2 = float(np.dot(zb, zb))
        infeas = math.sqrt(r2) if not (box or ball) else float(np.linalg.norm(z - proj(z)))
        gamma = dual_step_size(r2, t, alpha, beta0)
        y_new = y + gamma * zb
        if np.linalg.norm(y_new) > params.K:
            gamma = 0.0
        else:
            y = y_new
        # sketch: RankOneUpdate(sqrt(ha) v, eta), i.e. the sketch follows X <- (1-eta) X + eta H
        sketch.rank_one_update(math.sqrt(ha) * v, eta)
        for key, val in zip(_LOG_KEYS, (t, q, info["k"], xi, cv, p, infeas, gamma, gap, stop_obj,
                                        stop_feas, resid, beta, eta)):
            log[key].append(val)
        if record_v:
            vs.append(v.copy())
    log = {k: np.array(v) for k, v in log.items()}
    return OracleResult(n=n, alpha=alpha0, c_F=c_F, alpha_s=alpha, b_s=bs, p=p, z=z, y=y, S=sketch.S,
                        tau=sketch.tau, Omega=sketch.Omega, log=log, vs=vs, trace_mode=params.trace_mode,
                        dist_K=float(np.linalg.norm(z - proj(z))) if (box or ball) else None)


def state_of(res: OracleResult, t_next: int) -> dict:
    """State of a finished run, to resume at iteration t_next."""
    return {"t": t_next, "z": res.z.copy(), "y": res.y.copy(), "p": res.p, "S": res.S.copy(), "tau": res.tau}


def reconstruct_result(res: OracleResult, trace_correct: bool = True, storage: str = "f64"):
    """Reconstruct the final sketch of a run; U, Lambda in scaled units (X_hat = U diag(lam) U^T).
    The trace correction targets alpha, or the tracked trace tau of X_T when tr X <= alpha (R14)."""
    target = res.alpha_s if res.trace_mode == 0 else res.tau
    return nystrom_reconstruct(res.S, res.Omega, res.tau, alpha=target if trace_correct else None,
                               storage=storage)
