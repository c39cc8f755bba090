"""Self-sensitivity ("parity floor") of the oracle on the n = 800 workload.

Two runs of the same arithmetic that differ only by a 1-ulp perturbation of
the Lanczos start vectors measure how far rounding differences alone move the
result.  This sets which GPU-versus-oracle comparisons can be held to 1e-9:

* paper Lanczos (no reorthogonalisation) with q = 8: trajectories stay within
  1e-11 for 40 iterations;
* full reorthogonalisation, q = 36: a single iteration from a common state is
  reproducible to 1e-13;
* paper Lanczos with q = 36 (the n = 800 workload as specified): the
  trajectory is chaotic (floating-point Lanczos loses orthogonality once Ritz
  values converge, and the minimum eigenspace of D_t clusters as CGAL
  converges), so whole-run results differ by far more than 1e-9 and are
  compared at this measured floor instead.
"""
import numpy as np
import pytest

import synth
from oracle import OracleParams, sketchy_cgal, start_vector
from oracle.sketchycgal import state_of

N = 800


@pytest.fixture(scope="module")
def inst():
    return synth.config_instance(1)


def _pert(seed, rng):
    def f(t):
        g = start_vector(N, seed, t)
        return g * (1 + np.where(rng.random(N) < 0.5, -1.0, 1.0) * 2.0 ** -52)
    return f


def _rel(a, b):
    return abs(a - b) / abs(a)


def test_small_q_trajectory_is_reproducible(inst):
    prm = OracleParams(R=10, T=40, seed=synth.CONFIG_SEEDS[1], q_mode=1, q_fixed=8)
    A = sketchy_cgal(inst.to_scipy(), inst.b, prm)
    B = sketchy_cgal(inst.to_scipy(), inst.b, prm, start_vectors=_pert(prm.seed, np.random.default_rng(1)))
    assert np.max(np.abs(A.log["p"] - B.log["p"]) / np.abs(A.log["p"])) < 1e-11
    assert np.max(np.abs(A.log["infeas"] - B.log["infeas"]) / A.log["infeas"]) < 1e-10


@pytest.mark.parametrize("t", [1, 100])
def test_full_reorth_single_iteration_is_reproducible(inst, t):
    prm = OracleParams(R=10, T=500, seed=synth.CONFIG_SEEDS[1], q_mode=1, q_fixed=36, reorth=2)
    C = inst.to_scipy()
    st = state_of(sketchy_cgal(C, inst.b, prm, t_stop=t - 1), t) if t > 1 else None
    A = sketchy_cgal(C, inst.b, prm, state0=st, t_stop=t)
    B = sketchy_cgal(C, inst.b, prm, state0=st, t_stop=t, start_vectors=_pert(prm.seed, np.random.default_rng(2)))
    assert _rel(A.p, B.p) < 1e-13
    assert _rel(A.log["infeas"][-1], B.log["infeas"][-1]) < 1e-12
    assert np.abs(A.z - B.z).max() < 1e-12 * np.abs(A.z).max()


def test_paper_lanczos_q36_trajectory_is_chaotic(inst):
    prm = OracleParams(R=10, T=60, seed=synth.CONFIG_SEEDS[1], q_mode=1, q_fixed=36)
    A = sketchy_cgal(inst.to_scipy(), inst.b, prm)
    B = sketchy_cgal(inst.to_scipy(), inst.b, prm, start_vectors=_pert(prm.seed, np.random.default_rng(3)))
    d = np.abs(A.log["infeas"] - B.log["infeas"]) / A.log["infeas"]
    assert d.max() > 1e-6


# The batched-engine test instances (uneven Erdos-Renyi graphs of average
# degree 8 plus a cycle and a star): the floors behind the batched tolerances.
def _batched_pert(n, seed, inst_id, rng, eps=2.0 ** -52):
    def f(t):
        g = start_vector(n, seed, t, inst_id)
        return g * (1 + np.where(rng.random(n) < 0.5, -1.0, 1.0) * eps)
    return f


def test_batched_instances_small_q_trajectory_floor():
    from batch_cases import SEED4, traj_batch, signed_batch, valued_traj_batch
    worst = np.zeros(3)
    for batch in (traj_batch(), signed_batch(), valued_traj_batch()):
        for i, g in enumerate(batch):
            prm = OracleParams(R=8, T=40, seed=SEED4, q_mode=1, q_fixed=8, instance=i)
            A = sketchy_cgal(g.to_scipy(), g.b, prm)
            B = sketchy_cgal(g.to_scipy(), g.b, prm,
                             start_vectors=_batched_pert(g.n, SEED4, i, np.random.default_rng(i)))
            d = [np.abs(A.log["p"] - B.log["p"]).max() / np.abs(A.log["p"]).max(),
                 np.max(np.abs(A.log["infeas"] - B.log["infeas"]) / A.log["infeas"]),
                 np.abs(A.z - B.z).max() / np.abs(A.z).max()]
            worst = np.maximum(worst, d)
    # p and ||z - b|| reach 1e-8 for one member (n = 1205, unconverged Lanczos at t = 2), z 4e-8:
    # the GPU is held to 1e-7 on p and ||z - b|| and 5e-7 on z
    assert worst[0] < 1e-8 and worst[1] < 1e-8 and worst[2] < 5e-8, worst


def test_batched_instances_full_reorth_single_iteration_floor():
    from batch_cases import SEED4, small_batch, valued_batch
    for batch in (small_batch(), valued_batch()):
        for i, g in enumerate(batch):
            prm = OracleParams(R=8, T=40, seed=SEED4, q_mode=1, q_fixed=36, reorth=2, instance=i)
            C = g.to_scipy()
            st = state_of(sketchy_cgal(C, g.b, prm, t_stop=1), 2)
            A = sketchy_cgal(C, g.b, prm, state0=st, t_stop=2)
            B = sketchy_cgal(C, g.b, prm, state0=st, t_stop=2,
                             start_vectors=_batched_pert(g.n, SEED4, i, np.random.default_rng(10 + i)))
            assert _rel(A.p, B.p) < 1e-13, i
            assert _rel(A.log["infeas"][-1], B.log["infeas"][-1]) < 1e-12, i


class _ReversedRows:
    """The same matrix with the products of each row summed in reverse order."""

    def __init__(self, A):
        self.A, self.shape = A, A.shape

    def __matmul__(self, x):
        A = self.A
        out = np.empty(A.shape[0])
        for r in range(A.shape[0]):
            lo, hi = A.indptr[r], A.indptr[r + 1]
            prod = A.data[lo:hi][::-1] * x[A.indices[lo:hi][::-1]]
            acc = 0.0
            for v in prod:
                acc += v
            out[r] = acc
        return out


def test_weighted_star_trajectory_is_rounding_sensitive(monkeypatch):
    """A hub row holding most nonzeros: its top eigenvector converges in two
    Lanczos steps, after which the q = 8 recurrence is driven by rounding, so
    merely summing each row in reverse order moves ||z - b|| by ~2e-5 within
    six iterations.  Such members are compared one iteration at a time."""
    import oracle.sketchycgal as osc
    from batch_cases import SEED4, valued_batch
    g = valued_batch()[0]
    prm = OracleParams(R=8, T=6, seed=SEED4, q_mode=1, q_fixed=8, instance=0)
    A = sketchy_cgal(g.to_scipy(), g.b, prm)
    orig = osc.scale_problem

    def reversed_scale(C, b, alpha, scale=True):
        Cs, bs, a, cF = orig(C, b, alpha, scale)
        return _ReversedRows(Cs), bs, a, cF

    monkeypatch.setattr(osc, "scale_problem", reversed_scale)
    B = sketchy_cgal(g.to_scipy(), g.b, prm)
    assert np.max(np.abs(A.log["infeas"] - B.log["infeas"]) / A.log["infeas"]) > 1e-6


def test_full_size_torus_second_iteration_floor():
    """The 2^20-vertex torus workload, iteration 2 (q_2 = 17) from the oracle's
    own state: the paper's recurrence loses orthogonality once a Ritz value
    of the large diagonal shift converges, so merely summing the dot products
    and norms in another order changes the coefficients from step 10 on and
    xi by more than 1e-7; with full reorthogonalisation the same change moves
    xi by less than 1e-12.  GPU-versus-oracle comparisons at this size are
    made for the first iteration and with full reorthogonalisation."""
    import math
    from oracle.sketchycgal import scale_problem, approx_min_evec, tridiag_min_eigpair
    big = synth.config_instance(2)
    seed = synth.CONFIG_SEEDS[2]
    a1 = sketchy_cgal(big.to_scipy(), big.b, OracleParams(R=10, T=1, seed=seed))
    Cs, bs, _, _ = scale_problem(big.to_scipy(), big.b, float(big.n))
    w = a1.y + math.sqrt(3.0) * (a1.z - bs)
    g = start_vector(big.n, seed, 2)

    def mv(x):
        return Cs @ x + w * x

    def rdot(a, b):   # the same sums taken in another order
        return float(np.sum((a * b)[::-1].reshape(-1, 1024), axis=1)[::-1].sum())

    def lanczos_reordered(q, full):
        v = g / math.sqrt(rdot(g, g))
        vp, rp, om, rh, B = np.zeros_like(v), 0.0, [], [], [v]
        for i in range(1, q + 1):
            u = mv(v)
            o = rdot(v, u)
            u = u - o * v - rp * vp
            if full:
                u = u - np.stack(B, 1) @ np.array([rdot(b, u) for b in B])
            r = math.sqrt(rdot(u, u))
            om.append(o)
            if i == q:
                break
            rh.append(r)
            vp, v = v, u / r
            rp = r
            B.append(v)
        return tridiag_min_eigpair(np.array(om), np.array(rh))[0]

    xi0, _, _ = approx_min_evec(mv, g, 17)
    assert _rel(xi0, lanczos_reordered(17, False)) > 1e-7
    xi2, _, _ = approx_min_evec(mv, g, 17, 2)
    assert _rel(xi2, lanczos_reordered(17, True)) < 1e-12


# ---------------------------------------------------------------------------
# Whole-run floors of the n = 800 workload as specified (paper's Lanczos,
# q = 36, T = 500) and the FP32-level floors.  "FP32 products" runs the oracle
# with C rounded to FP32, the multiplied vector rounded to FP32 and the
# product accumulated in FP32 (scipy's single-precision CSR kernel), every
# other step in FP64: the rounding an FP32-stream SpMV adds to each Lanczos
# step, and nothing else.

class _F32Products:
    def __init__(self, A):
        self.A, self.shape = A.astype(np.float32), A.shape

    def __matmul__(self, x):
        return (self.A @ np.asarray(x, dtype=np.float32)).astype(np.float64)


def _fp32_products(monkeypatch):
    import oracle.sketchycgal as osc
    orig = osc.scale_problem

    def f32_scale(C, b, alpha, scale=True):
        Cs, bs, a, cF = orig(C, b, alpha, scale)
        return _F32Products(Cs), bs, a, cF

    monkeypatch.setattr(osc, "scale_problem", f32_scale)


def _w1_params(**kw):
    return OracleParams(R=10, T=500, seed=synth.CONFIG_SEEDS[1], q_mode=1, q_fixed=36, **kw)


@pytest.fixture(scope="module")
def w1_reference(inst):
    return {r: sketchy_cgal(inst.to_scipy(), inst.b, _w1_params(reorth=r)) for r in (0, 1, 2)}


def test_workload1_as_specified_whole_run_floor(inst, w1_reference):
    """A 1-ulp change of the start vectors (three draws) moves the final
    objective by 3.5e-4 .. 7.3e-4 and ||z - b|| by up to 35%: the GPU result
    of this workload is held to 1e-2 on the objective and 3x on ||z - b||
    (tests/test_gpu_parity.py), at most 30x and about 2x those spreads.  Full
    reorthogonalisation (reorth = 2) still moves the objective by 1e-4, so no
    Lanczos variant makes 1e-9 attainable over 500 iterations here."""
    A = w1_reference[0]
    d_obj, ratio = [], []
    for s in range(3):
        B = sketchy_cgal(inst.to_scipy(), inst.b, _w1_params(), start_vectors=_pert(synth.CONFIG_SEEDS[1], np.random.default_rng(100 + s)))
        d_obj.append(_rel(A.objective, B.objective))
        ratio.append(B.infeasibility / A.infeasibility)
    print("objective spread", d_obj, "infeasibility ratios", ratio)
    assert 3e-4 < max(d_obj) < 1e-2 / 10
    assert max(max(ratio), 1 / min(ratio)) > 1.3
    A2 = w1_reference[2]
    B2 = sketchy_cgal(inst.to_scipy(), inst.b, _w1_params(reorth=2),
                      start_vectors=_pert(synth.CONFIG_SEEDS[1], np.random.default_rng(100)))
    print("full reorthogonalisation objective spread", _rel(A2.objective, B2.objective))
    assert _rel(A2.objective, B2.objective) > 5e-5


def test_fp32_products_single_iteration_floor(inst, monkeypatch):
    """One iteration from a common oracle state (q = 8) with FP32 products:
    at t = 100 the Ritz value moves by 1.9e-3, ||z - b|| by 8.8e-4 and z by
    8.9e-3, while the objective moves by 1.6e-5.  The GPU's FP32-stream
    one-iteration bars (xi 2e-2, ||z - b|| 1e-2) are about 10x these; the
    objective bar is the stated 1e-4, which the method itself meets."""
    prm = OracleParams(R=10, T=500, seed=synth.CONFIG_SEEDS[1], q_mode=1, q_fixed=8)
    C = inst.to_scipy()
    worst = np.zeros(4)
    refs = {}
    for t in (1, 20, 100, 300):
        st = state_of(sketchy_cgal(C, inst.b, prm, t_stop=t - 1), t) if t > 1 else None
        refs[t] = (st, sketchy_cgal(C, inst.b, prm, state0=st, t_stop=t))
    _fp32_products(monkeypatch)
    for t, (st, A) in refs.items():
        B = sketchy_cgal(C, inst.b, prm, state0=st, t_stop=t)
        d = [_rel(A.p, B.p), _rel(A.log["xi"][-1], B.log["xi"][-1]),
             _rel(A.log["infeas"][-1], B.log["infeas"][-1]), np.abs(A.z - B.z).max() / np.abs(A.z).max()]
        print(t, d)
        worst = np.maximum(worst, d)
    assert worst[0] < 1e-4
    assert 1e-3 < worst[1] < 2e-2
    assert 5e-4 < worst[2] < 1e-2
    assert worst[3] > 5e-3


def test_fp32_products_whole_run_floor(inst, w1_reference, monkeypatch):
    """FP32 products over 500 iterations of this workload move the final
    objective by 2.7e-3 (q = 36) with the paper's Lanczos; with local or full
    reorthogonalisation the final difference is smaller (2e-5, 1e-4) but
    reaches 7e-3 and 2e-2 on the way (9.5e-3 without).  So an end-of-run FP32-stream
    objective within 1e-4 of FP64 is not attainable for this method on this
    workload: the whole-run FP32 results are reported against this floor, and
    the 1e-4 bar applies per iteration from a common state."""
    _fp32_products(monkeypatch)
    out = {}
    for r in (0, 1, 2):
        A = w1_reference[r]
        B = sketchy_cgal(inst.to_scipy(), inst.b, _w1_params(reorth=r))
        out[r] = (_rel(A.objective, B.objective), float(np.max(np.abs(A.log["p"] - B.log["p"]) / np.abs(A.log["p"]))))
    print(out)
    assert out[0][0] > 1e-3
    assert all(out[r][1] > 1e-4 for r in (0, 1, 2))


def _spreads(A, B):
    return np.array([_rel(A.p, B.p), _rel(A.log["infeas"][-1], B.log["infeas"][-1]),
                     _rel(A.log["xi"][-1], B.log["xi"][-1]), np.abs(A.z - B.z).max() / np.abs(A.z).max(),
                     np.abs(A.S - B.S).max() / np.abs(A.S).max()])


def test_batched_local_reorth_single_iteration_floor():
    """Local reorthogonalisation (reorth = 1, q = 8), one iteration from the
    oracle's own state at t = 2 and t = 25, on the batched test problems: a
    1-ulp change of the start vector (three draws) moves p, ||z - b||, xi
    and z by up to ~1e-8 and S by ~1e-5 (the 2500-vertex star at t = 2, whose
    Ritz vector is unconverged).  The batched engine is held to 2e-7 on the
    former and 1e-4 on S (tests/test_gpu_batched.py)."""
    from batch_cases import SEED4, small_batch
    worst = np.zeros(5)
    for i, g in enumerate(small_batch()):
        prm = OracleParams(R=8, T=40, seed=SEED4, q_mode=1, q_fixed=8, reorth=1, instance=i)
        C = g.to_scipy()
        for t in (2, 25):
            st = state_of(sketchy_cgal(C, g.b, prm, t_stop=t - 1), t)
            A = sketchy_cgal(C, g.b, prm, state0=st, t_stop=t)
            for s in range(3):
                B = sketchy_cgal(C, g.b, prm, state0=st, t_stop=t,
                                 start_vectors=_batched_pert(g.n, SEED4, i, np.random.default_rng(50 + 3 * i + s)))
                worst = np.maximum(worst, _spreads(A, B))
    print("p, infeas, xi, z, S:", worst)
    assert 1e-8 < worst[:4].max() < 2e-7
    assert 1e-5 < worst[4] < 1e-4


def test_batched_per_instance_beta0_floor(monkeypatch):
    """Trajectories (40 iterations, q = 8) of the batched test problems, each
    with its own beta_0 in {0.5, 2, 1, 4}: a 1-ulp start-vector change and
    summing every row in reverse order move p by up to ~7e-9, ||z - b|| by
    ~2e-8 and z by ~3e-7.  The batched engine is held to 4e-7 on the log
    quantities and 6e-6 on z (tests/test_gpu_batched.py), 20x these."""
    import oracle.sketchycgal as osc
    from batch_cases import SEED4, traj_batch
    betas = [0.5, 2.0, 1.0, 4.0]
    orig = osc.scale_problem
    worst = np.zeros(3)
    for i, g in enumerate(traj_batch()):
        prm = OracleParams(R=8, T=40, seed=SEED4, q_mode=1, q_fixed=8, instance=i, beta0=betas[i % 4])
        A = sketchy_cgal(g.to_scipy(), g.b, prm)
        runs = [sketchy_cgal(g.to_scipy(), g.b, prm,
                             start_vectors=_batched_pert(g.n, SEED4, i, np.random.default_rng(70 + i)))]

        def reversed_scale(C, b, alpha, scale=True):
            Cs, bs, a, cF = orig(C, b, alpha, scale)
            return _ReversedRows(Cs), bs, a, cF

        monkeypatch.setattr(osc, "scale_problem", reversed_scale)
        runs.append(sketchy_cgal(g.to_scipy(), g.b, prm))
        monkeypatch.setattr(osc, "scale_problem", orig)
        for B in runs:
            worst = np.maximum(worst, [np.max(np.abs(A.log["p"] - B.log["p"]) / np.abs(A.log["p"])),
                                       np.max(np.abs(A.log["infeas"] - B.log["infeas"]) / A.log["infeas"]),
                                       np.abs(A.z - B.z).max() / np.abs(A.z).max()])
    print("p, infeas, z:", worst)
    assert 1e-9 < worst[0] < 4e-8
    assert 5e-9 < worst[1] < 4e-8
    assert 1e-7 < worst[2] < 6e-7


def test_entry_chunk_trajectory_instances_floor(monkeypatch):
    """The instances of the entry-chunk product's trajectory test (rows of
    mixed lengths 0..64; a 20 000-vertex random geometric graph), 40
    iterations at q = 8: summing every row of every product in reverse order
    moves the oracle's own p, ||z - b|| and z by less than 1e-11, so the GPU
    trajectories are held to 1e-9 there.  The weighted Erdos-Renyi instance
    with isolated vertices moves by ~1e-9 under the same change (its Ritz
    values lie closer), so that instance is checked through the operator only."""
    import oracle.sketchycgal as osc
    from test_gpu_entry_chunks import CASES
    orig = osc.scale_problem

    def reversed_scale(C, b, alpha, scale=True):
        Cs, bs, a, cF = orig(C, b, alpha, scale)
        return _ReversedRows(Cs), bs, a, cF

    spreads = {}
    for which in ("mixed", "geometric", "er_isolated"):
        g = CASES[which]()
        prm = OracleParams(R=10, T=40, seed=synth.CONFIG_SEEDS[1], q_mode=1, q_fixed=8)
        A = sketchy_cgal(g.to_scipy(), g.b, prm)
        monkeypatch.setattr(osc, "scale_problem", reversed_scale)
        B = sketchy_cgal(g.to_scipy(), g.b, prm)
        monkeypatch.setattr(osc, "scale_problem", orig)
        spreads[which] = max(np.max(np.abs(A.log["p"] - B.log["p"]) / np.abs(A.log["p"])),
                             np.max(np.abs(A.log["infeas"] - B.log["infeas"]) / A.log["infeas"]),
                             np.abs(A.z - B.z).max() / np.abs(A.z).max())
    print("spreads:", spreads)
    assert spreads["mixed"] < 1e-11 and spreads["geometric"] < 1e-11
    assert spreads["er_isolated"] > 1e-10


def test_sliced_chunk_instance_two_iteration_floor(monkeypatch):
    """The power-law instance with stored values of the sliced entry-chunk
    test (40 000 vertices, hub rows of ~900 entries), two iterations at
    q = 10: summing every row of every product in reverse order moves the
    oracle's own p, ||z - b||, v^T C v and z by at most ~3e-12, so the two GPU
    forms of the eight concurrent segments are held to 5e-11 there."""
    import oracle.sketchycgal as osc
    from test_gpu_sliced_chunks import CASES
    inst = CASES["powerlaw_values"]()
    prm = OracleParams(R=6, T=2, seed=7, q_mode=1, q_fixed=10)
    A = sketchy_cgal(inst.to_scipy(), inst.b, prm)
    orig = osc.scale_problem

    def reversed_scale(C, b, alpha, scale=True):
        Cs, bs, a, cF = orig(C, b, alpha, scale)
        return _ReversedRows(Cs), bs, a, cF

    monkeypatch.setattr(osc, "scale_problem", reversed_scale)
    B = sketchy_cgal(inst.to_scipy(), inst.b, prm)
    spread = max([np.max(np.abs(A.log[k] - B.log[k])) / np.max(np.abs(A.log[k])) for k in ("p", "infeas", "cv")]
                 + [np.abs(A.z - B.z).max() / np.abs(A.z).max()])
    print("spread:", spread)
    assert 1e-13 < spread < 5e-12
