"""Batched engine (every instance advanced by one launch per iteration)
against the FP64 oracle run on each instance alone, through the C ABI.

Tolerances follow the oracle's measured self-sensitivity on these very
instances (tests/test_oracle_floor.py, batched cases):
  * one iteration from a common oracle state with full reorthogonalisation
    (q = 36): reproducible to ~1e-15, held to 1e-9 on p, ||z - b|| and z;
  * whole trajectories with the paper's Lanczos at q = 8 (40 iterations):
    a 1-ulp change of a start vector moves p and ||z - b|| by up to 1e-8 and
    z by 4e-8 on these graphs (unconverged Lanczos at t = 2), so
    trajectories are held to 1e-7 (z to 5e-7).  Star graphs are
    rounding-sensitive beyond that (reversing the summation order of each
    row moves ||z - b|| by 2e-5) and take part only in the per-iteration
    comparisons;
  * FP32 streams: one iteration from a common state, objective within 1e-4.
"""
import math

import numpy as np
import pytest

import synth
from oracle import sketchy_cgal
from oracle.sketchycgal import gaussian_test_matrix, nystrom_reconstruct

from batch_cases import SEED4, small_batch, signed_batch, traj_batch, valued_batch, valued_traj_batch
from gpu_util import need_gpu, oracle_params, oracle_run, oracle_snapshots, rel, maxrel, announce

pytestmark = pytest.mark.gpu

TRAJ_TOL = 1e-7
Z_TOL = 5e-7


def make_batch(insts, **kw):
    from paper_1912_02949_amd import BatchedSketchyCGAL, Params
    prm = Params(**kw)
    announce(f"batch init sizes={[g.n for g in insts]} {prm}")
    return BatchedSketchyCGAL(insts, prm)


def _check_trajectory(lg, ref, tol, where):
    assert lg["k"].tolist() == ref.log["k"].tolist(), where
    assert maxrel(lg["p"], ref.log["p"]) < tol, where
    assert np.max(np.abs(lg["infeas"] - ref.log["infeas"]) / ref.log["infeas"]) < tol, where
    # derived quantities (stop_obj nearly cancels at some iterations): relative to the trajectory's scale
    for key in ("xi", "gap", "stop_obj", "stop_feas", "gamma", "cv"):
        assert maxrel(lg[key], ref.log[key]) < 10 * tol, (where, key)


@pytest.mark.parametrize("kind,fmt", [("pattern", 1), ("signed", 2), ("values", 0), ("forced_values", 0)])
def test_batched_trajectories_match_oracle_fp64(kind, fmt):
    need_gpu()
    insts = {"pattern": traj_batch, "signed": signed_batch, "values": valued_traj_batch,
             "forced_values": traj_batch}[kind]()
    extra = {"matrix_format": 1} if kind == "forced_values" else {}
    kw = dict(R=8, T=40, seed=SEED4, q_mode=1, q_fixed=8)
    bt = make_batch(insts, **kw, **extra)
    bt.run()
    for i, inst in enumerate(insts):
        ref = oracle_run(inst, instance=i, **kw)
        _check_trajectory(bt.log(i), ref, TRAJ_TOL, (kind, i))
        summ = bt.summary(i)
        assert summ["matrix_format"] == fmt
        assert summ["t_done"] == 40
        assert rel(summ["objective"], ref.objective) < TRAJ_TOL, i
        assert rel(summ["infeasibility"], ref.infeasibility) < TRAJ_TOL, i
        g = bt.get_state(i)
        assert maxrel(g["z"].cpu().numpy(), ref.z) < Z_TOL, i


def test_batched_per_instance_beta0_matches_oracle_fp64():
    # Each problem with its own beta_0 (0.5 .. 4) against the oracle run with it.
    # Oracle floors of these seven runs, measured by a 1-ulp start-vector change
    # and by summing every row in reverse order: p <= 3.4e-9, ||z - b|| <= 1.9e-8,
    # z <= 2.8e-7 (the n = 1205 member at beta_0 = 2); bars at 20x those.
    tol, ztol = 4e-7, 6e-6
    need_gpu()
    insts = traj_batch()
    betas = [0.5, 2.0, 1.0, 4.0]
    kw = dict(R=8, T=40, seed=SEED4, q_mode=1, q_fixed=8)
    bt = make_batch(insts, **kw)
    b0 = np.array([betas[i % len(betas)] for i in range(len(insts))])
    bt.set_beta0(b0)
    bt.run()
    for i, inst in enumerate(insts):
        ref = oracle_run(inst, instance=i, beta0=float(b0[i]), **kw)
        _check_trajectory(bt.log(i), ref, tol, ("beta0", i))
        assert maxrel(bt.get_state(i)["z"].cpu().numpy(), ref.z) < ztol, i
        assert np.allclose(bt.log(i)["beta"], b0[i] * np.sqrt(np.arange(2, 42))), i


def test_batched_set_beta0_errors():
    need_gpu()
    from paper_1912_02949_amd._lib import SCGError, SCG_EINVAL, SCG_ESTATE
    insts = traj_batch()[:3]
    bt = make_batch(insts, R=8, T=5, seed=SEED4, q_mode=1, q_fixed=6)
    for bad in ([1.0, 0.0, 1.0], [1.0, -2.0, 1.0], [1.0, np.nan, 1.0], [np.inf, 1.0, 1.0]):
        with pytest.raises(SCGError) as e:
            bt.set_beta0(bad)
        assert e.value.status == SCG_EINVAL
    bt.step(1)
    with pytest.raises(SCGError) as e:
        bt.set_beta0([1.0, 1.0, 1.0])
    assert e.value.status == SCG_ESTATE


@pytest.mark.parametrize("which,reorth,q", [("unit", 2, 36), ("weighted", 2, 36), ("unit", 1, 8)])
def test_batched_single_iteration_from_oracle_state_fp64(which, reorth, q):
    need_gpu()
    kw = dict(R=8, T=40, seed=SEED4, q_mode=1, q_fixed=q, reorth=reorth)
    insts = small_batch() if which == "unit" else valued_batch()
    bt = make_batch(insts, **kw)
    # full reorthogonalisation: the oracle reproduces itself to 1e-12 here, bar
    # 1e-9 (S 1e-8).  Local (reorth = 1, q = 8): at t = 2 the Ritz vector of the
    # 2500-vertex problem is unconverged, and a 1-ulp change of the start vector
    # (three draws) moves the oracle's own p by 2.2e-9, ||z - b|| by 1.0e-8, xi
    # by 9.2e-9, z by 2.1e-8 and S by 1.2e-5; bars at about 10x: 2e-7, S 1e-4.
    tol, tol_s = (1e-9, 1e-8) if reorth == 2 else (2e-7, 1e-4)
    for t in (2, 25):
        refs = []
        for i, inst in enumerate(insts):
            st = oracle_snapshots(inst, [t], instance=i, **kw)[t]
            bt.set_state(i, t, st["z"], st["y"], st["S"], st["p"], st["tau"])
            refs.append(sketchy_cgal(inst.to_scipy(), inst.b, oracle_params(instance=i, **kw), state0=st,
                                     t_stop=t))
        announce(f"batched one iteration at t={t}")
        bt.step(1)
        for i, ref in enumerate(refs):
            g = bt.get_state(i)
            lg = bt.log(i)
            assert g["t"] == t + 1
            assert lg["k"][t - 1] == ref.log["k"][-1], (t, i)
            assert rel(g["p"], ref.p) < tol, (t, i)
            assert rel(lg["infeas"][t - 1], ref.log["infeas"][-1]) < tol, (t, i)
            assert rel(lg["xi"][t - 1], ref.log["xi"][-1]) < tol, (t, i)
            assert maxrel(g["z"].cpu().numpy(), ref.z) < tol, (t, i)
            assert maxrel(g["y"].cpu().numpy(), ref.y) < tol, (t, i)
            assert maxrel(g["S"].cpu().numpy(), ref.S) < tol_s, (t, i)
            assert rel(g["tau"], ref.tau) < 1e-12, (t, i)


def test_batched_single_iteration_fp32_stream():
    need_gpu()
    kw = dict(R=8, T=40, seed=SEED4, q_mode=1, q_fixed=8)
    insts = small_batch()
    bt = make_batch(insts, precision="fp32", **kw)
    for t in (1, 20):
        refs = []
        for i, inst in enumerate(insts):
            st = oracle_snapshots(inst, [t], instance=i, **kw)[t]
            if st is not None:
                bt.set_state(i, t, st["z"], st["y"], st["S"], st["p"], st["tau"])
            refs.append(sketchy_cgal(inst.to_scipy(), inst.b, oracle_params(instance=i, **kw), state0=st,
                                     t_stop=t))
        announce(f"batched fp32 one iteration at t={t}")
        bt.step(1)
        for i, ref in enumerate(refs):
            g = bt.get_state(i)
            lg = bt.log(i)
            assert rel(g["p"], ref.p) < 1e-4, (t, i)
            assert rel(lg["xi"][t - 1], ref.log["xi"][-1]) < 2e-2, (t, i)
            assert rel(lg["infeas"][t - 1], ref.log["infeas"][-1]) < 1e-2, (t, i)
            z = g["z"].cpu().numpy()
            assert abs(z.sum() - 1.0) < 1e-9 and z.min() >= 0, (t, i)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_graph_replays_match_eager_launches(precision):
    """step(40) replays a captured 16-iteration graph twice, then launches 8
    iterations eagerly; stepping one iteration at a time never uses the
    graph.  Both must agree bit for bit on every instance."""
    need_gpu()
    kw = dict(R=8, T=40, seed=SEED4, q_mode=1, q_fixed=10, precision=precision)
    insts = small_batch()
    a = make_batch(insts, **kw)
    a.step(40)
    b = make_batch(insts, **kw)
    for _ in range(40):
        b.step(1)
    for i in range(len(insts)):
        la, lb = a.log(i), b.log(i)
        for key in ("p", "infeas", "xi", "gamma", "k"):
            assert np.array_equal(la[key], lb[key]), (i, key)
        sa, sb = a.get_state(i), b.get_state(i)
        assert np.array_equal(sa["S"].cpu().numpy(), sb["S"].cpu().numpy()), i
        assert np.array_equal(sa["y"].cpu().numpy(), sb["y"].cpu().numpy()), i


def test_batched_instance_matches_single_engine():
    need_gpu()
    from paper_1912_02949_amd import Params, SketchyCGAL
    kw = dict(R=8, T=40, seed=SEED4, q_mode=1, q_fixed=8)
    insts = traj_batch()
    bt = make_batch(insts, **kw)
    bt.run()
    for i in (0, 5, 6):
        inst = insts[i]
        s = SketchyCGAL(inst.row_ptr, inst.col, inst.val, inst.b, Params(instance=i, **kw))
        s.run()
        lb, ls = bt.log(i), s.log()
        assert lb["k"].tolist() == ls["k"].tolist(), i
        assert maxrel(lb["p"], ls["p"]) < TRAJ_TOL, i
        assert maxrel(lb["infeas"], ls["infeas"]) < TRAJ_TOL, i


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_wide_columns_and_global_gathers(precision):
    """An instance with n > 65536 forces 32-bit column words, and its vector
    no longer fits the LDS budget, so the SpMV gathers from global memory."""
    need_gpu()
    big = synth.laplacian_instance(synth.erdos_renyi(70_000, 280_000, SEED4 + 500))
    insts = [synth.laplacian_instance(synth.erdos_renyi(400, 1600, SEED4 + 501)), big]
    kw = dict(R=8, T=4, seed=SEED4, q_mode=1, q_fixed=8)
    bt = make_batch(insts, precision=precision, **kw)
    bt.run()
    for i, inst in enumerate(insts):
        ref = oracle_run(inst, instance=i, **kw)
        lg = bt.log(i)
        if precision == "fp64":
            _check_trajectory(lg, ref, TRAJ_TOL, i)
        else:
            assert rel(lg["p"][0], ref.log["p"][0]) < 1e-4, i
            assert maxrel(lg["infeas"], ref.log["infeas"]) < 1e-2, i


def test_batched_reconstruct_matches_oracle_on_same_sketch():
    need_gpu()
    insts = small_batch()
    for precision, tol in (("fp64", 1e-8), ("fp32", 1e-5)):
        kw = dict(R=8, T=60, seed=SEED4, q_mode=1, q_fixed=12, precision=precision)
        bt = make_batch(insts, **kw)
        bt.run()
        for i in (1, 5, 7):
            n = insts[i].n
            g = bt.get_state(i)
            U, lam, err = (x.cpu().numpy() for x in bt.reconstruct(i))
            Om = gaussian_test_matrix(n, 8, SEED4, i)
            if precision == "fp32":
                Om = Om.astype(np.float32).astype(np.float64)
            ref = nystrom_reconstruct(g["S"].cpu().numpy(), Om, g["tau"], alpha=1.0,
                                      storage="f32" if precision == "fp32" else "f64")
            assert np.abs(U.T @ U - np.eye(8)).max() < 1e-10, (precision, i)
            assert maxrel(lam, ref["lam"]) < tol, (precision, i)
            assert maxrel(err, ref["err"]) < tol, (precision, i)
            assert abs(lam.sum() - 1.0) < 1e-12, (precision, i)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_reaches_closed_form_sdp_values(precision):
    need_gpu()
    graphs = [(synth.cycle(9), 4.5 * (1 + math.cos(math.pi / 9))), (synth.complete(7), 12.25),
              (synth.complete_bipartite(3, 4), 12.0)]
    insts = [synth.laplacian_instance(g) for g, _ in graphs]
    bt = make_batch(insts, R=4, T=2000, seed=1, precision=precision)
    bt.run()
    for i, (_, ref) in enumerate(graphs):
        cut = -bt.summary(i)["objective"]
        assert abs(cut - ref) / ref < 2e-3, i


def test_batched_validation_errors():
    need_gpu()
    from paper_1912_02949_amd._lib import SCGError, SCG_EINVAL, SCG_ESTATE
    insts = small_batch()[:3]
    # a column of instance 0 that points into instance 1's block
    bad = synth.MaxCutInstance(**{**insts[0].__dict__})
    bad.col = insts[0].col.copy()
    bad.col[5] = insts[0].n + 3
    with pytest.raises(SCGError) as e:
        make_batch([bad] + insts[1:], R=8, T=10, seed=1)
    assert e.value.status == SCG_EINVAL
    with pytest.raises(SCGError):
        make_batch(insts, R=8, T=10, seed=1, reorth=3)
    with pytest.raises(SCGError):
        make_batch(insts + [synth.laplacian_instance(synth.cycle(5))], R=8, T=10, seed=1)
    bt = make_batch(insts, R=8, T=10, seed=1, q_mode=1, q_fixed=6)
    bt.step(7)
    with pytest.raises(SCGError) as e:
        bt.step(4)
    assert e.value.status == SCG_ESTATE
    n0 = insts[0].n
    z = np.zeros(n0)
    with pytest.raises(SCGError) as e:
        bt.set_state(0, 12, z, z, np.zeros((n0, 8)), 0.0, 0.0)
    assert e.value.status == SCG_EINVAL
    bt.step(3)
    assert bt.summary(2)["t_done"] == 10


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_batched_rounding_matches_oracle_on_same_reconstruction(precision, tol):
    need_gpu()
    from oracle import round_maxcut, cut_indicators
    insts = valued_batch() + small_batch()[:2]
    bt = make_batch(insts, R=8, T=60, seed=SEED4, q_mode=1, q_fixed=12, precision=precision)
    bt.run()
    for i in range(len(insts)):
        U, _, _ = bt.reconstruct(i)
        w, best, chi = bt.round_cut(i, U)
        w_ref, best_ref, chi_ref = round_maxcut(U.cpu().numpy(), insts[i].to_scipy())
        assert np.abs(w - w_ref).max() < tol * np.abs(w_ref).max(), i
        assert w_ref[best] >= w_ref[best_ref] - tol * abs(w_ref[best_ref]), i
        assert np.array_equal(chi.cpu().numpy(), cut_indicators(U.cpu().numpy())[:, best]), i


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("form", [1, 2, 3])
def test_batched_kernel_forms_trajectories(form, precision):
    """Each iteration kernel form forced (1: the vector in LDS, 2: two LDS column
    tiles, 3: gathers from global memory): FP64 trajectories against the oracle
    at the trajectory bar, FP32 first iteration at its one-iteration bars."""
    need_gpu()
    insts = traj_batch()
    T = 40 if precision == "fp64" else 1
    kw = dict(R=8, T=T, seed=SEED4, q_mode=1, q_fixed=8, precision=precision)
    bt = make_batch(insts, batch_kernel=form, **kw)
    assert bt.summary(0)["batch_kernel"] == form
    bt.run()
    for i, inst in enumerate(insts):
        ref = oracle_run(inst, instance=i, **kw)
        lg = bt.log(i)
        if precision == "fp64":
            _check_trajectory(lg, ref, TRAJ_TOL, (form, i))
            assert maxrel(bt.get_state(i)["z"].cpu().numpy(), ref.z) < Z_TOL, (form, i)
        else:   # (the 9-cycle's FP32 recurrence need not break down where the FP64 one does)
            assert rel(lg["p"][0], ref.log["p"][0]) < 1e-4, (form, i)
            assert rel(lg["xi"][0], ref.log["xi"][0]) < 2e-2, (form, i)


@pytest.mark.parametrize("form", [2, 3])
def test_batched_kernel_forms_single_iteration_with_hub_rows(form):
    """Forms 2 and 3 with a star (hub row summed by a whole wave, across both
    column tiles) and valued members: one iteration from the oracle's state
    with full reorthogonalisation, held to 1e-9 (S 1e-8)."""
    need_gpu()
    insts = valued_batch()
    kw = dict(R=8, T=40, seed=SEED4, q_mode=1, q_fixed=36, reorth=2)
    bt = make_batch(insts, batch_kernel=form, **kw)
    t = 2
    refs = []
    for i, inst in enumerate(insts):
        st = oracle_snapshots(inst, [t], instance=i, **kw)[t]
        bt.set_state(i, t, st["z"], st["y"], st["S"], st["p"], st["tau"])
        refs.append(sketchy_cgal(inst.to_scipy(), inst.b, oracle_params(instance=i, **kw), state0=st, t_stop=t))
    bt.step(1)
    for i, ref in enumerate(refs):
        g = bt.get_state(i)
        assert rel(g["p"], ref.p) < 1e-9, (form, i)
        assert rel(bt.log(i)["infeas"][t - 1], ref.log["infeas"][-1]) < 1e-9, (form, i)
        assert maxrel(g["z"].cpu().numpy(), ref.z) < 1e-9, (form, i)
        assert maxrel(g["S"].cpu().numpy(), ref.S) < 1e-8, (form, i)


def test_batched_kernel_forced_form_that_does_not_fit():
    """The whole-vector LDS form cannot hold an FP64 vector of 20 000 entries."""
    need_gpu()
    from paper_1912_02949_amd._lib import SCGError, SCG_EINVAL
    big = synth.laplacian_instance(synth.erdos_renyi(20000, 80000, 3))
    with pytest.raises(SCGError) as e:
        make_batch([big], R=8, T=2, seed=SEED4, precision="fp64", batch_kernel=1)
    assert e.value.status == SCG_EINVAL
