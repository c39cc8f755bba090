"""The eight concurrent column segments over entry chunks (spmv_lanes = 1 with
segments = 8) against the oracle's operator, within the forward-error bound of
the arithmetic, and against the row-block form of the same eight segments.

Each column slice holds the segments of every row packed into chunks of 256
entries; a segment with no entry, or with more than 64 (stored apart and summed
by a wave of its own), holds one padding entry.  Cases: a Chung-Lu power-law
graph whose hubs have long segments in every slice (unit weights: columns only),
the same with +-1 weights (sign bit) and with weights U[0.5, 1.5] (values
stored), an Erdos-Renyi graph with isolated vertices (empty segments), and a
graph of 1000 vertices, fewer rows than one slice's chunk holds.
"""
import numpy as np
import pytest

import synth
from gpu_util import need_gpu, make_solver, maxrel, announce
from test_gpu_fullsize import _check_operator

pytestmark = pytest.mark.gpu


def _reweight(g: synth.Graph, kind: str, seed: int) -> synth.Graph:
    rng = np.random.default_rng(seed)
    if kind == "pm1":
        w = np.where(rng.random(g.m) < 0.5, -1.0, 1.0)
    else:
        w = rng.uniform(0.5, 1.5, g.m)
    return synth.Graph(n=g.n, src=g.src, dst=g.dst, w=w)


def _isolated(g: synth.Graph, extra: int) -> synth.Graph:
    return synth.Graph(n=g.n + extra, src=g.src, dst=g.dst, w=g.w)


CASES = {
    "powerlaw_unit": lambda: synth.laplacian_instance(synth.chung_lu(40000, 400000, 2.5, 31)),
    "powerlaw_pm1": lambda: synth.laplacian_instance(_reweight(synth.chung_lu(40000, 400000, 2.5, 32), "pm1", 1)),
    "powerlaw_values": lambda: synth.laplacian_instance(
        _reweight(synth.chung_lu(40000, 400000, 2.5, 33), "uniform", 2)),
    "er_isolated": lambda: synth.laplacian_instance(_isolated(synth.erdos_renyi(20000, 80000, 34), 333)),
    "small": lambda: synth.laplacian_instance(synth.erdos_renyi(1000, 6000, 35)),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("which", list(CASES))
def test_sliced_chunk_product_within_rounding_bound(which, precision):
    need_gpu()
    inst = CASES[which]()
    deg = np.diff(inst.row_ptr)
    announce(f"sliced chunks {which} n={inst.n} max row {deg.max()} {precision}")
    for grid in (0, 64):
        s = make_solver(inst, R=4, T=5, seed=3, precision=precision, spmv_lanes=1, segments=8, autotune=0,
                        spmv_grid=grid)
        summ = s.summary()
        assert summ["spmv_lanes"] == 1 and summ["spmv_segments"] == 8
        _check_operator(inst, s, precision)
    # the row-block form of the same eight segments agrees to rounding
    x = np.random.default_rng(5).standard_normal(inst.n)
    a = make_solver(inst, R=4, T=5, seed=3, precision=precision, spmv_lanes=1, segments=8, autotune=0)
    b = make_solver(inst, R=4, T=5, seed=3, precision=precision, spmv_lanes=2, segments=8, autotune=0)
    tol = 1e-13 if precision == "fp64" else 1e-5
    assert maxrel(a.apply(x).cpu().numpy(), b.apply(x).cpu().numpy()) < tol


def test_sliced_chunk_first_iterations_match_row_block_form_fp64():
    # two whole iterations (every Lanczos and objective product through the
    # sliced chunks) against the same iterations through the row-block form of
    # the eight segments: the two sum each row in another order only.  Summing
    # every row in reverse order moves the oracle's own results by at most 5e-12
    # on this instance (tests/test_oracle_floor.py); the bar is 10x that
    need_gpu()
    inst = CASES["powerlaw_values"]()
    kw = dict(R=6, T=2, seed=7, q_mode=1, q_fixed=10, segments=8, autotune=0)
    a = make_solver(inst, spmv_lanes=1, **kw)
    b = make_solver(inst, spmv_lanes=2, **kw)
    a.run()
    b.run()
    la, lb = a.log(), b.log()
    assert la["k"].tolist() == lb["k"].tolist()
    for key in ("p", "xi", "infeas", "cv"):
        assert maxrel(la[key], lb[key]) < 5e-11, key
    assert maxrel(a.get_state()["z"].cpu().numpy(), b.get_state()["z"].cpu().numpy()) < 5e-11


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sliced_chunk_graph_replays_match_eager_launches(precision):
    # on a non-null stream every iteration replays a captured graph, here with
    # the slice pass, the long segments and the combining pass in each Lanczos
    # step: every record and the state equal the eager run's bit for bit
    need_gpu()
    import torch
    from paper_1912_02949_amd import Params, SketchyCGAL
    inst = CASES["powerlaw_unit"]()
    kw = dict(R=6, T=20, seed=9, precision=precision, spmv_lanes=1, segments=8, autotune=0)
    eager = make_solver(inst, **kw)
    eager.run()
    g = SketchyCGAL(inst.row_ptr, inst.col, inst.val, inst.b, Params(**kw), stream=torch.cuda.Stream())
    announce(f"sliced chunk graph replays {precision}")
    g.step(7)
    assert g.get_state()["t"] == 8
    g.step(13)
    le, lg = eager.log(), g.log()
    for key in le:
        assert np.array_equal(le[key], lg[key], equal_nan=True), key
    se, sg = eager.get_state(), g.get_state()
    for key in ("z", "y", "S"):
        assert torch.equal(se[key], sg[key]), key
