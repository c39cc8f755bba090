"""The C/OpenMP oracle (oracle/c/maxcut_oracle.c) against the Python oracle.

Both take the paper's steps in the same order with the same readings; the C
one uses another tridiagonal eigensolver (cyclic Jacobi) and its own Philox
and Box-Muller code, so its results agree with the Python oracle's to
rounding.  On trajectories that are reproducible to ~1e-11 under a 1-ulp
change (tests/test_oracle_floor.py) the two are held to 1e-9; its results do
not depend on the number of threads (fixed-block reductions).
"""
import numpy as np
import pytest

import synth
from oracle import OracleParams, sketchy_cgal
from oracle.c_oracle import MaxCutIterations


@pytest.fixture(scope="module")
def cfg1():
    return synth.config_instance(1)


def _rel(a, b):
    return np.max(np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(np.asarray(b)), 1e-300))


def test_c_oracle_matches_python_oracle_workload1(cfg1):
    prm = OracleParams(R=10, T=40, seed=synth.CONFIG_SEEDS[1], q_mode=1, q_fixed=8)
    ref = sketchy_cgal(cfg1.to_scipy(), cfg1.b, prm)
    c = MaxCutIterations(cfg1.to_scipy(), cfg1.b, prm)
    lg = c.run(40, threads=2)
    assert lg[:, 0].tolist() == ref.log["k"].tolist()
    assert _rel(lg[:, 1], ref.log["xi"]) < 1e-9
    assert _rel(lg[:, 3], ref.log["p"]) < 1e-9
    assert _rel(lg[:, 4], ref.log["infeas"]) < 1e-9
    assert _rel(lg[:, 5], ref.log["gamma"]) < 1e-9
    assert np.abs(c.z - ref.z).max() < 1e-9 * np.abs(ref.z).max()
    assert np.abs(c.y - ref.y).max() < 1e-9 * np.abs(ref.y).max()
    assert np.abs(c.S - ref.S).max() < 1e-7 * np.abs(ref.S).max()
    assert abs(c.tau.value - ref.tau) < 1e-12
    assert abs(c.objective - ref.objective) < 1e-9 * abs(ref.objective)


def test_c_oracle_paper_schedule_and_breakdown():
    # the paper's q_t on a 4096-vertex +-1 torus (first iterations), and an odd
    # cycle whose Krylov space (5 distinct eigenvalues) is exhausted before
    # q = 8 steps (breakdown at k = 5)
    for inst, T, kw, tol in ((synth.laplacian_instance(synth.torus_longrange(64, 5)), 3, {}, 1e-9),
                             (synth.laplacian_instance(synth.cycle(9)), 10, dict(q_mode=1, q_fixed=8), 1e-9)):
        prm = OracleParams(R=4, T=T, seed=7, **kw)
        ref = sketchy_cgal(inst.to_scipy(), inst.b, prm)
        c = MaxCutIterations(inst.to_scipy(), inst.b, prm)
        lg = c.run(T)
        assert lg[:, 0].tolist() == ref.log["k"].tolist()
        if kw:
            assert lg[0, 0] == 5
        assert _rel(lg[:, 3], ref.log["p"]) < tol
        assert _rel(lg[:, 4], ref.log["infeas"]) < tol


def test_c_oracle_is_independent_of_thread_count(cfg1):
    prm = OracleParams(R=10, T=10, seed=synth.CONFIG_SEEDS[1], q_mode=1, q_fixed=12)
    runs = []
    for th in (1, 3, 8):
        c = MaxCutIterations(cfg1.to_scipy(), cfg1.b, prm)
        runs.append((c.run(10, threads=th), c.z.copy(), c.S.copy()))
    for lg, z, S in runs[1:]:
        assert np.array_equal(lg, runs[0][0]) and np.array_equal(z, runs[0][1]) and np.array_equal(S, runs[0][2])
