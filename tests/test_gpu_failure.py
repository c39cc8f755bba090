"""Failure paths of the C ABI on the GPU, with every kernel exiting normally.

* The shift retry of NystromSketch.Reconstruct (alg:nystrom-sketch-supp,
  reading R9: on a Cholesky failure sigma grows tenfold, at most three
  times).  A caller test matrix and an injected sketch make the Cholesky
  factor's first pivot exactly -kappa + sigma, so the first shift fails and
  the second succeeds; the result is compared with the oracle, which retries
  the same way.
* A test matrix with a zero column: every pivot of that column is exactly
  zero whatever the shift, so all four attempts fail and the call returns
  SCG_ENUMERIC (the oracle raises).
* A non-finite iteration state (set_state with a NaN in z): the next
  iteration sets the device's NaN/Inf flag, summary() returns SCG_ENUMERIC
  and reports the flag, step() itself never synchronises and returns SCG_OK.
"""
import math

import numpy as np
import pytest

import synth
from oracle.sketchycgal import nystrom_reconstruct

from gpu_util import need_gpu, make_solver, announce

pytestmark = pytest.mark.gpu

N = 16
R = 2


def _retry_case(fp32: bool):
    """Omega = [e_0, w], S = [-kappa e_0, w] with w_0 = 0, ||w|| = 1.5: B(sigma) = Omega^T (S + sigma Omega)
    = diag(sigma - kappa, (1 + sigma) ||w||^2) exactly.  sigma_0 = sqrt(n) eps(||S||_2) with eps the spacing at
    1.5 of the sketch's storage precision; kappa = 3 sigma_0, so sigma_0 fails and 10 sigma_0 succeeds."""
    w = np.zeros(N)
    w[1:] = 1.5 / math.sqrt(N - 1)
    sig0 = math.sqrt(N) * (2.0 ** -23 if fp32 else 2.0 ** -52)
    Omega = np.stack([np.eye(N)[0], w], axis=1)
    S = np.stack([-3.0 * sig0 * np.eye(N)[0], w], axis=1)
    if fp32:   # the FP32-stream form stores Omega and S in FP32
        Omega = Omega.astype(np.float32).astype(np.float64)
        S = S.astype(np.float32).astype(np.float64)
    return Omega, S, sig0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_reconstruct_shift_retry_matches_oracle(precision):
    need_gpu()
    fp32 = precision == "fp32"
    Omega, S, sig0 = _retry_case(fp32)
    ref = nystrom_reconstruct(S, Omega, 1.0, alpha=1.0, storage="f32" if fp32 else "f64")
    assert ref["sigma"] == 10.0 * sig0          # exactly one retry
    inst = synth.laplacian_instance(synth.cycle(N))
    announce(f"shift retry {precision}")
    s = make_solver(inst, omega=Omega.reshape(-1), R=R, T=5, seed=1, precision=precision)
    z = np.full(N, 1.0 / N)
    s.set_state(3, z, np.zeros(N), S, -0.1, 1.0)
    U, lam, err = s.reconstruct()
    U, lam, err = U.cpu().numpy(), lam.cpu().numpy(), err.cpu().numpy()
    assert np.abs(lam - ref["lam"]).max() < 1e-8
    assert np.abs(err - ref["err"]).max() < 1e-8
    assert np.abs(U.T @ U - np.eye(R)).max() < 1e-10
    Xg = U @ np.diag(lam) @ U.T
    Xo = ref["U"] @ np.diag(ref["lam"]) @ ref["U"].T
    assert np.abs(Xg - Xo).max() < 1e-8


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_reconstruct_zero_omega_column_reports_numeric_failure(precision):
    need_gpu()
    from paper_1912_02949_amd._lib import SCGError, SCG_ENUMERIC
    rng = np.random.default_rng(4)
    Omega = rng.standard_normal((N, R))
    Omega[:, 1] = 0.0
    S = rng.standard_normal((N, R))
    S[:, 1] = 0.0                                   # S = X Omega has a zero column too
    if precision == "fp32":
        Omega = Omega.astype(np.float32).astype(np.float64)
        S = S.astype(np.float32).astype(np.float64)
    with pytest.raises(np.linalg.LinAlgError):
        nystrom_reconstruct(S, Omega, 1.0, alpha=1.0, storage="f32" if precision == "fp32" else "f64")
    inst = synth.laplacian_instance(synth.cycle(N))
    announce(f"zero Omega column {precision}")
    s = make_solver(inst, omega=Omega.reshape(-1), R=R, T=5, seed=1, precision=precision)
    s.set_state(3, np.full(N, 1.0 / N), np.zeros(N), S, -0.1, 1.0)
    with pytest.raises(SCGError) as e:
        s.reconstruct()
    assert e.value.status == SCG_ENUMERIC
    # the context stays usable: the iteration itself is unaffected
    s.step(1)
    assert s.summary()["status_flags"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nonfinite_state_reports_numeric_failure(precision):
    need_gpu()
    from paper_1912_02949_amd._lib import SCGError, SCG_ENUMERIC
    inst = synth.laplacian_instance(synth.cycle(9))
    announce(f"non-finite state {precision}")
    s = make_solver(inst, R=R, T=5, seed=1, precision=precision)
    s.step(1)
    assert s.summary()["status_flags"] == 0
    g = s.get_state()
    z = g["z"].cpu().numpy()
    z[3] = np.nan
    s.set_state(2, z, g["y"], g["S"], g["p"], g["tau"])
    s.step(1)                                       # asynchronous: no status from the device yet
    with pytest.raises(SCGError) as e:
        s.summary()
    assert e.value.status == SCG_ENUMERIC
    assert s.summary(check_numeric=False)["status_flags"] == 1
    lg = s.log()
    # the NaN in z reaches the shift, so the Ritz value and ||z - b|| of that iteration are NaN
    assert not np.isfinite(lg["xi"][1]) and not np.isfinite(lg["infeas"][1])
