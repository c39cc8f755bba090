"""GPU (HIP) path against the FP64 oracle, through the C ABI.

Tolerances follow the measured self-sensitivity of the method
(tests/test_oracle_floor.py):
  * FP64 within 1e-9 relative on the objective p and ||z - b|| wherever the
    oracle itself is reproducible to far better than that: one iteration from
    a common state with full reorthogonalisation, and whole trajectories with
    the paper's Lanczos at q = 8 (40 iterations);
  * the n = 800 workload exactly as specified (paper's Lanczos, q = 36,
    T = 500) is chaotic under rounding, so its end result is compared at the
    oracle's own measured spread (1e-2 objective), plus the invariants;
  * FP32-stream within 1e-4 relative on the objective for one iteration from
    a common state.
"""
import math

import numpy as np
import pytest

import synth
from oracle import sketchy_cgal, approx_min_evec, start_vector
from oracle.sketchycgal import scale_problem, nystrom_reconstruct

from gpu_util import need_gpu, make_solver, oracle_params, oracle_run, oracle_snapshots, rel, maxrel, announce

pytestmark = pytest.mark.gpu

SEED1 = synth.CONFIG_SEEDS[1]


@pytest.fixture(scope="module")
def cfg1():
    return synth.config_instance(1)


def _star_plus(n, seed):
    """Star (one row longer than an LDS block) + random edges + isolated vertices."""
    rng = np.random.default_rng(seed)
    hub = np.zeros(n - 11, dtype=np.int64)
    leaf = np.arange(1, n - 10, dtype=np.int64)
    er = synth.erdos_renyi(n - 10, 3 * n, seed)
    src = np.concatenate([hub, er.src])
    dst = np.concatenate([leaf, er.dst])
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    key = np.unique(lo * n + hi)
    w = rng.uniform(0.5, 1.5, key.size)
    return synth.laplacian_instance(synth.Graph(n, key // n, key % n, w))


@pytest.mark.parametrize("matrix_format", [0, 1])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
@pytest.mark.parametrize("which", ["cfg1", "star", "cycle", "pm1"])
def test_apply_matches_operator(which, precision, tol, matrix_format, cfg1):
    """D x against the oracle's operator; cfg1/cycle have unit weights (columns
    only), pm1 has +-1 weights (sign in the column word), star has general
    weights and a row longer than an LDS block, plus isolated vertices."""
    need_gpu()
    inst = {"cfg1": lambda: cfg1, "star": lambda: _star_plus(5000, 3),
            "cycle": lambda: synth.laplacian_instance(synth.cycle(7)),
            "pm1": lambda: synth.laplacian_instance(synth.torus_longrange(64, 5))}[which]()
    s = make_solver(inst, R=4, T=5, seed=1, precision=precision, matrix_format=matrix_format)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(inst.n)
    y = s.apply(x).cpu().numpy()
    Cs, bs, _, _ = scale_problem(inst.to_scipy(), inst.b, float(inst.n))
    w = math.sqrt(2.0) * (0 - bs)
    ref = Cs @ x + w * x
    assert maxrel(y, ref) < tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
@pytest.mark.parametrize("lanes,grid", [(2, 16), (4, 8), (8, 0), (32, 24), (1, 0), (1, 16)])
def test_apply_with_forced_spmv_shape(lanes, grid, precision, tol):
    """Fewer workgroups than row-block ranges (each wave walks several blocks)
    and every lane count give the same product."""
    need_gpu()
    inst = synth.laplacian_instance(synth.torus_longrange(256, 77))
    s = make_solver(inst, R=4, T=5, seed=3, precision=precision, spmv_lanes=lanes, spmv_grid=grid)
    summ = s.summary()
    assert summ["spmv_lanes"] == lanes
    if grid:
        assert 8 <= summ["spmv_grid"] <= grid
    rng = np.random.default_rng(5)
    x = rng.standard_normal(inst.n)
    y = s.apply(x).cpu().numpy()
    Cs, bs, _, _ = scale_problem(inst.to_scipy(), inst.b, float(inst.n))
    ref = Cs @ x + math.sqrt(2.0) * (0 - bs) * x
    assert maxrel(y, ref) < tol


def test_first_lanczos_run_matches(cfg1):
    need_gpu()
    s = make_solver(cfg1, R=10, T=3, seed=SEED1, q_mode=1, q_fixed=8)
    s.step(1)
    om, rh, xi = s.lanczos_coeffs()
    Cs, bs, _, _ = scale_problem(cfg1.to_scipy(), cfg1.b, 800.0)
    w = math.sqrt(2.0) * (0 - bs)
    g = start_vector(800, SEED1, 1)
    xi_o, _, info = approx_min_evec(lambda x: Cs @ x + w * x, g, 8)
    assert len(om) == info["k"] == 8
    assert maxrel(om, info["omega"]) < 1e-12
    assert maxrel(rh, info["rho"]) < 1e-12
    assert rel(xi, xi_o) < 1e-12


@pytest.mark.parametrize("reorth,q", [(2, 36), (0, 8), (1, 8)])
def test_single_iteration_from_oracle_state_fp64(cfg1, reorth, q):
    need_gpu()
    kw = dict(R=10, T=500, seed=SEED1, q_mode=1, q_fixed=q, reorth=reorth)
    ts = [1, 2, 5, 20, 100, 300, 500]
    snaps = oracle_snapshots(cfg1, ts, **kw)
    s = make_solver(cfg1, **kw)
    C = cfg1.to_scipy()
    op = oracle_params(**kw)
    for t in ts:
        st = snaps[t]
        announce(f"state-injected iteration t={t} reorth={reorth} q={q}")
        if st is None:
            s2 = make_solver(cfg1, **kw)
        else:
            s2 = s
            s2.set_state(t, st["z"], st["y"], st["S"], st["p"], st["tau"])
        s2.step(1)
        ref = sketchy_cgal(C, cfg1.b, op, state0=st, t_stop=t)
        g = s2.get_state()
        lg = s2.log()
        assert g["t"] == t + 1
        assert rel(g["p"], ref.p) < 1e-9, t
        assert rel(lg["infeas"][t - 1], ref.log["infeas"][-1]) < 1e-9, t
        assert rel(lg["xi"][t - 1], ref.log["xi"][-1]) < 1e-10, t
        assert maxrel(g["z"].cpu().numpy(), ref.z) < 1e-9, t
        assert maxrel(g["y"].cpu().numpy(), ref.y) < 1e-9, t
        # the sketch takes the full Ritz-vector direction error (z and p are
        # damped by eta): with the paper's Lanczos the oracle's own S moves by
        # up to 2e-9 under rounding-level noise in the products (t = 300)
        assert maxrel(g["S"].cpu().numpy(), ref.S) < (1e-9 if reorth == 2 else 1e-7), t
        assert rel(g["tau"], ref.tau) < 1e-12, t
        assert rel(lg["cv"][t - 1], ref.log["cv"][-1]) < 1e-9, t


@pytest.mark.parametrize("reorth", [0, 1])
def test_trajectory_small_q_fp64(cfg1, reorth):
    need_gpu()
    kw = dict(R=10, T=40, seed=SEED1, q_mode=1, q_fixed=8, reorth=reorth)
    s = make_solver(cfg1, **kw)
    s.run()
    lg = s.log()
    ref = oracle_run(cfg1, **kw)
    assert lg["k"].tolist() == ref.log["k"].tolist()
    assert maxrel(lg["p"], ref.log["p"]) < 1e-9
    assert np.max(np.abs(lg["infeas"] - ref.log["infeas"]) / ref.log["infeas"]) < 1e-9
    for key in ("xi", "gap", "stop_obj", "stop_feas", "gamma", "cv"):
        assert np.max(np.abs(lg[key] - ref.log[key]) / np.maximum(np.abs(ref.log[key]), 1e-12)) < 1e-8, key
    summ = s.summary()
    assert rel(summ["objective"], ref.objective) < 1e-9
    assert rel(summ["infeasibility"], ref.infeasibility) < 1e-9


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
@pytest.mark.parametrize("segments", [2, 4, 8])
@pytest.mark.parametrize("which", ["cfg1", "star", "pm1", "odd"])
def test_apply_with_column_segments(which, segments, precision, tol, cfg1):
    # 8 segments: all in one launch (segment s on XCD s) plus the combining pass;
    # "odd" has n = 4099, so the last segment and the last row quad are partial
    need_gpu()
    inst = {"cfg1": lambda: cfg1, "star": lambda: _star_plus(5000, 3),
            "pm1": lambda: synth.laplacian_instance(synth.torus_longrange(64, 5)),
            "odd": lambda: synth.laplacian_instance(synth.erdos_renyi(4099, 30000, 13))}[which]()
    rng = np.random.default_rng(0)
    x = rng.standard_normal(inst.n)
    Cs, bs, _, _ = scale_problem(inst.to_scipy(), inst.b, float(inst.n))
    ref = Cs @ x + math.sqrt(2.0) * (0 - bs) * x
    for grid in (0, 8, 64):
        s = make_solver(inst, R=4, T=5, seed=1, segments=segments, spmv_grid=grid, precision=precision)
        assert s.summary()["spmv_segments"] == segments
        y = s.apply(x).cpu().numpy()
        assert maxrel(y, ref) < tol, grid


@pytest.mark.parametrize("segments", [4, 8])
def test_trajectory_with_column_segments_fp64(cfg1, segments):
    need_gpu()
    kw = dict(R=10, T=40, seed=SEED1, q_mode=1, q_fixed=8)
    s = make_solver(cfg1, segments=segments, **kw)
    s.run()
    lg = s.log()
    ref = oracle_run(cfg1, **kw)
    assert maxrel(lg["p"], ref.log["p"]) < 1e-9
    assert np.max(np.abs(lg["infeas"] - ref.log["infeas"]) / ref.log["infeas"]) < 1e-9


def test_compressed_matrix_format_matches_values(cfg1):
    """Columns-only storage (unit weights) against stored values, FP64, q = 8."""
    need_gpu()
    kw = dict(R=10, T=40, seed=SEED1, q_mode=1, q_fixed=8)
    a = make_solver(cfg1, matrix_format=0, **kw)
    a.run()
    b = make_solver(cfg1, matrix_format=1, **kw)
    b.run()
    la, lb = a.log(), b.log()
    assert maxrel(la["p"], lb["p"]) < 1e-9
    assert np.max(np.abs(la["infeas"] - lb["infeas"]) / lb["infeas"]) < 1e-9


def test_workload1_as_specified_fp64(cfg1):
    """n = 800 ER, paper's Lanczos q = 36, T = 500, FP64: compared at the oracle's floor."""
    need_gpu()
    kw = dict(R=10, T=500, seed=SEED1, q_mode=1, q_fixed=36)
    s = make_solver(cfg1, **kw)
    s.run()
    summ = s.summary()
    g = s.get_state()
    ref = oracle_run(cfg1, **kw)
    assert rel(summ["objective"], ref.objective) < 1e-2
    assert summ["infeasibility"] < 3 * ref.infeasibility + 1e-3
    z = g["z"].cpu().numpy()
    assert abs(z.sum() - 1.0) < 1e-12 and z.min() >= 0
    assert abs(g["tau"] - 1.0) < 1e-12
    lg = s.log()
    assert lg["stop_feas"][-1] < 5 * ref.log["stop_feas"][-1]
    assert abs(lg["stop_obj"][-1]) < 0.05


def test_single_iteration_fp32_stream(cfg1):
    """FP32 streams against the FP64 oracle from a common state.

    The objective is held to 1e-4.  The Ritz vector itself is not: near
    convergence the minimum eigenspace of D_t clusters, and FP32-level noise
    in the products moves the oracle's own z by up to 5e-2 (measured), while
    the objective and the Ritz value stay put.
    """
    need_gpu()
    kw = dict(R=10, T=500, seed=SEED1, q_mode=1, q_fixed=8)
    ts = [1, 20, 300]
    snaps = oracle_snapshots(cfg1, ts, **kw)
    C = cfg1.to_scipy()
    op = oracle_params(**kw)
    s = make_solver(cfg1, precision="fp32", **kw)
    for t in ts:
        st = snaps[t]
        if st is not None:
            s.set_state(t, st["z"], st["y"], st["S"], st["p"], st["tau"])
        s.step(1)
        ref = sketchy_cgal(C, cfg1.b, op, state0=st, t_stop=t)
        g = s.get_state()
        lg = s.log()
        assert rel(g["p"], ref.p) < 1e-4, t
        # measured spread of xi under FP32-level noise: up to 1e-2 (t = 100)
        assert rel(lg["xi"][t - 1], ref.log["xi"][-1]) < 2e-2, t
        assert rel(lg["infeas"][t - 1], ref.log["infeas"][-1]) < 1e-2, t
        z = g["z"].cpu().numpy()
        assert abs(z.sum() - 1.0) < 1e-9 and z.min() >= 0, t


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("graph,ref", [(synth.cycle(9), 4.5 * (1 + math.cos(math.pi / 9))),
                                       (synth.complete(7), 12.25), (synth.complete_bipartite(3, 4), 12.0)])
def test_gpu_reaches_closed_form_sdp_value(graph, ref, precision):
    need_gpu()
    inst = synth.laplacian_instance(graph)
    s = make_solver(inst, R=4, T=2000, seed=1, precision=precision)
    s.run()
    cut = -s.summary()["objective"]
    assert abs(cut - ref) / ref < 2e-3


def test_reconstruct_matches_oracle_on_same_sketch(cfg1):
    need_gpu()
    for precision, tol in (("fp64", 1e-8), ("fp32", 1e-5)):
        kw = dict(R=10, T=60, seed=SEED1, q_mode=1, q_fixed=12, precision=precision)
        s = make_solver(cfg1, **kw)
        s.run()
        g = s.get_state()
        U, lam, err = s.reconstruct()
        U, lam, err = U.cpu().numpy(), lam.cpu().numpy(), err.cpu().numpy()
        Om = np.stack([synth_normal(800, SEED1, c) for c in range(10)], axis=1)
        if precision == "fp32":
            Om = Om.astype(np.float32).astype(np.float64)
        ref = nystrom_reconstruct(g["S"].cpu().numpy(), Om, g["tau"], alpha=1.0,
                                  storage="f32" if precision == "fp32" else "f64")
        assert np.abs(U.T @ U - np.eye(10)).max() < 1e-10
        assert maxrel(lam, ref["lam"]) < tol
        assert maxrel(err, ref["err"]) < tol
        Xg = (U * lam) @ U.T
        Xo = (ref["U"] * ref["lam"]) @ ref["U"].T
        assert maxrel(Xg, Xo) < 10 * tol
        assert abs(lam.sum() - 1.0) < 1e-12


def synth_normal(n, seed, c):
    from oracle.philox import normal_stream
    return normal_stream(n, seed, c, 0, 1)


def test_runs_are_bitwise_reproducible(cfg1):
    need_gpu()
    kw = dict(R=10, T=30, seed=SEED1, q_mode=1, q_fixed=20)
    a = make_solver(cfg1, **kw)
    a.run()
    b = make_solver(cfg1, **kw)
    b.run()
    la, lb = a.log(), b.log()
    for key in ("p", "infeas", "xi", "gamma"):
        assert np.array_equal(la[key], lb[key]), key
    assert np.array_equal(a.get_state()["S"].cpu().numpy(), b.get_state()["S"].cpu().numpy())


def test_checkpoint_resume_is_exact(cfg1):
    need_gpu()
    kw = dict(R=10, T=40, seed=SEED1, q_mode=1, q_fixed=10)
    a = make_solver(cfg1, **kw)
    a.run()
    b = make_solver(cfg1, **kw)
    b.step(17)
    st = b.get_state()
    c = make_solver(cfg1, **kw)
    c.set_state(st["t"], st["z"], st["y"], st["S"], st["p"], st["tau"])
    c.step(40 - 17)
    assert np.array_equal(a.get_state()["z"].cpu().numpy(), c.get_state()["z"].cpu().numpy())
    assert a.get_state()["p"] == c.get_state()["p"]


def test_validation_errors_on_device():
    need_gpu()
    from paper_1912_02949_amd._lib import SCGError, SCG_EINVAL, SCG_ESTATE
    inst = synth.laplacian_instance(synth.cycle(9))
    bad_col = inst.col.copy()
    bad_col[3] = 99
    from paper_1912_02949_amd import Params, SketchyCGAL
    with pytest.raises(SCGError) as e:
        SketchyCGAL(inst.row_ptr, bad_col, inst.val, inst.b, Params(R=3, T=5))
    assert e.value.status == SCG_EINVAL
    bad_val = inst.val.copy()
    bad_val[5] = np.nan
    with pytest.raises(SCGError):
        SketchyCGAL(inst.row_ptr, inst.col, bad_val, inst.b, Params(R=3, T=5))
    bad_rp = inst.row_ptr.copy()
    bad_rp[4] = bad_rp[5] + 1
    with pytest.raises(SCGError):
        SketchyCGAL(bad_rp, inst.col, inst.val, inst.b, Params(R=3, T=5))
    s = SketchyCGAL(inst.row_ptr, inst.col, inst.val, inst.b, Params(R=3, T=5))
    s.step(5)
    with pytest.raises(SCGError) as e:
        s.step(1)
    assert e.value.status == SCG_ESTATE


@pytest.mark.parametrize("segments", [0, 8])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
@pytest.mark.parametrize("which", ["cfg1", "star", "pm1"])
def test_rounding_matches_oracle_on_same_reconstruction(which, precision, tol, segments, cfg1):
    """MaxCut rounding (Section 7.2): the same U gives the same R cut weights,
    the same heaviest cut and bit-identical indicators (also with the matrix
    stored in eight column segments)."""
    need_gpu()
    from oracle import round_maxcut, cut_indicators
    inst = {"cfg1": lambda: cfg1, "star": lambda: _star_plus(5000, 3),
            "pm1": lambda: synth.laplacian_instance(synth.torus_longrange(64, 5))}[which]()
    s = make_solver(inst, R=6, T=60, seed=SEED1, q_mode=1, q_fixed=12, precision=precision, segments=segments)
    s.run()
    U, lam, err = s.reconstruct()
    w, best, chi = s.round_cut(U)
    w_ref, best_ref, chi_ref = round_maxcut(U.cpu().numpy(), inst.to_scipy())
    assert np.abs(w - w_ref).max() < tol * np.abs(w_ref).max()
    # integer cut weights can tie: the chosen cut must be a heaviest one, its indicator exact
    assert w_ref[best] >= w_ref[best_ref] - tol * abs(w_ref[best_ref])
    assert np.array_equal(chi.cpu().numpy(), cut_indicators(U.cpu().numpy())[:, best])


@pytest.mark.parametrize("graph,opt", [(synth.complete_bipartite(3, 4), 12.0), (synth.cycle(8), 8.0),
                                       (synth.cycle(7), 6.0)])
def test_gpu_solve_reconstruct_round_finds_the_max_cut(graph, opt):
    need_gpu()
    inst = synth.laplacian_instance(graph)
    s = make_solver(inst, R=4, T=2000, seed=1)
    s.run()
    U, _, _ = s.reconstruct()
    w, best, chi = s.round_cut(U)
    assert w[best] == pytest.approx(opt, abs=1e-9)
    x = chi.cpu().numpy().astype(np.float64)
    assert -(x @ (inst.to_scipy() @ x)) == pytest.approx(opt, abs=1e-9)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["paper_q", "fixed_q", "storage_optimal", "box_reorth"])
def test_graph_replays_match_eager_launches(case, precision, cfg1):
    """On a non-null stream every iteration is a replay of a captured graph (one
    per Lanczos step count, the iteration counter read on the device).  With
    eager host work and synchronisations between the calls, every replayed
    iteration's record, and the state after each call, equal the eager run's
    bit for bit."""
    need_gpu()
    import torch
    kw = dict(R=10, T=40, seed=SEED1, precision=precision)
    if case == "fixed_q":
        kw.update(q_mode=1, q_fixed=12)
    elif case == "storage_optimal":
        kw.update(basis_mode=1, omega_mode=1)
    elif case == "box_reorth":
        kw.update(constraint_set=1, reorth=1)
    eager = make_solver(cfg1, **kw)
    if case == "box_reorth":
        eager.set_constraints(lo=np.full(cfg1.n, 0.9), hi=np.full(cfg1.n, 1.1))
    eager.run()
    stream = torch.cuda.Stream()
    from paper_1912_02949_amd import Params, SketchyCGAL
    g = SketchyCGAL(cfg1.row_ptr, cfg1.col, cfg1.val, cfg1.b, Params(**kw), stream=stream)
    if case == "box_reorth":
        g.set_constraints(lo=np.full(cfg1.n, 0.9), hi=np.full(cfg1.n, 1.1))
    announce(f"graph replays {case} {precision}")
    for chunk in (7, 13, 20):
        g.step(chunk)
        st = g.get_state()                     # synchronises; eager copies between the replays
        assert st["t"] == 1 + sum((7, 13, 20)[:(7, 13, 20).index(chunk) + 1])
    le, lg = eager.log(), g.log()
    for key in le:
        assert np.array_equal(le[key], lg[key], equal_nan=True), key
    se, sg = eager.get_state(), g.get_state()
    for key in ("z", "y", "S"):
        assert torch.equal(se[key], sg[key]), key
    assert se["p"] == sg["p"] and se["tau"] == sg["tau"]
