"""The quad-chunk product (spmv_lanes = 1) against the oracle's operator and
trajectories, and against the row-block product on the same matrix.

The layout pads each row's column words to whole 16-byte quads and packs
rows, whole, into chunks of 64 quads; one wave takes a chunk, finds each
lane's row from the row-start flags, and sums the rows by a scan across the
lanes.  It takes the compressed formats (one off-diagonal magnitude) and rows
of at most 128 off-diagonal entries (stored values take the entry-chunk
layout, tests/test_gpu_entry_chunks.py).  Cases: the pattern format (workload 1,
unit weights, rows of about 50 entries), the sign-bit format (a +-1 torus with
long-range edges), isolated vertices (empty rows: one padding quad each),
rows that straddle no chunk, breakdown of the recurrence, and the rejections.
"""
import math

import numpy as np
import pytest

import synth
from gpu_util import need_gpu, make_solver, oracle_run, rel, maxrel, announce
from oracle.sketchycgal import scale_problem

pytestmark = pytest.mark.gpu

SEED1 = synth.CONFIG_SEEDS[1]


def _with_isolated(g: synth.Graph, extra: int) -> synth.Graph:
    # the same edges on n + extra vertices: the last `extra` rows are empty
    return synth.Graph(n=g.n + extra, src=g.src, dst=g.dst, w=g.w)


def _circulant(n: int, half_degree: int) -> synth.Graph:
    # vertex i joined to i +- 1 .. i +- half_degree (mod n): every row holds 2 half_degree entries
    src = np.repeat(np.arange(n, dtype=np.int64), half_degree)
    dst = (src + np.tile(np.arange(1, half_degree + 1, dtype=np.int64), n)) % n
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    return synth.Graph(n=n, src=lo, dst=hi, w=np.ones(lo.size))


CASES = {
    "cfg1": lambda: synth.config_instance(1),
    "torus_pm1": lambda: synth.laplacian_instance(synth.torus_longrange(128, 91)),
    "isolated": lambda: synth.laplacian_instance(_with_isolated(synth.erdos_renyi(3000, 9000, 17), 77)),
    # rows of 17 quads: three rows per chunk, 13 quads of every chunk unused
    "circulant68": lambda: synth.laplacian_instance(_circulant(1000, 34)),
    # rows at the layout's limit of 128 entries: two rows fill a chunk
    "circulant128": lambda: synth.laplacian_instance(_circulant(700, 64)),
}


def _operator_ref(inst, x):
    Cs, bs, _, _ = scale_problem(inst.to_scipy(), inst.b, float(inst.n))
    return Cs @ x + math.sqrt(2.0) * (0 - bs) * x      # D_1 = C + diag(y + beta_1 (z - b)), z = y = 0


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
@pytest.mark.parametrize("which", list(CASES))
def test_quad_product_matches_operator(which, precision, tol):
    # rows of up to 128 entries summed in FP32: the bar for that precision is
    # the one every product test uses (2e-6 relative to the largest entry)
    need_gpu()
    inst = CASES[which]()
    announce(f"quad product {which} n={inst.n} {precision}")
    x = np.random.default_rng(7).standard_normal(inst.n)
    ref = _operator_ref(inst, x)
    for grid in (0, 8, 64):
        s = make_solver(inst, R=4, T=5, seed=3, precision=precision, spmv_lanes=1, spmv_grid=grid)
        assert s.summary()["spmv_lanes"] == 1
        y = s.apply(x).cpu().numpy()
        assert maxrel(y, ref) < tol, (which, grid)
    # the row-block product on the same matrix agrees to rounding
    s2 = make_solver(inst, R=4, T=5, seed=3, precision=precision, spmv_lanes=2)
    assert maxrel(s2.apply(x).cpu().numpy(), y) < tol


@pytest.mark.parametrize("which", ["cfg1", "isolated"])
def test_quad_trajectory_matches_oracle_fp64(which):
    # whole trajectories with the paper's Lanczos at q = 8 (on both instances a
    # 1-ulp change of the start vectors moves the oracle's own p, xi and
    # ||z - b|| by at most 4e-13, v^T C v and z by 5e-12); every Lanczos and
    # objective product of the run goes through the quad-chunk kernel
    need_gpu()
    inst = CASES[which]()
    kw = dict(R=10, T=40, seed=SEED1, q_mode=1, q_fixed=8)
    announce(f"quad trajectory {which}")
    s = make_solver(inst, spmv_lanes=1, **kw)
    s.run()
    lg = s.log()
    ref = oracle_run(inst, **kw)
    assert lg["k"].tolist() == ref.log["k"].tolist()
    assert maxrel(lg["p"], ref.log["p"]) < 1e-9
    assert np.max(np.abs(lg["infeas"] - ref.log["infeas"]) / ref.log["infeas"]) < 1e-9
    for key in ("xi", "cv", "gamma"):
        assert np.max(np.abs(lg[key] - ref.log[key]) / np.maximum(np.abs(ref.log[key]), 1e-12)) < 1e-8, key
    g = s.get_state()
    assert maxrel(g["z"].cpu().numpy(), ref.z) < 1e-9


def test_quad_breakdown_matches_row_block_product():
    # K_{3,4} at t = 1: the Krylov space has the dimension of the Laplacian's
    # distinct eigenvalues (4) and the recurrence stops there
    need_gpu()
    inst = synth.laplacian_instance(synth.complete_bipartite(3, 4))
    kw = dict(R=4, T=1, seed=1, q_mode=1, q_fixed=6)
    a = make_solver(inst, spmv_lanes=1, **kw)
    a.run()
    ref = oracle_run(inst, **kw)
    lg = a.log()
    assert lg["flags"][0] & 1 and lg["k"][0] == ref.log["k"][0] == 4
    assert rel(lg["xi"][0], ref.log["xi"][0]) < 1e-12
    assert rel(lg["p"][0], ref.log["p"][0]) < 1e-12


def test_quad_product_rejects_matrices_it_cannot_take():
    need_gpu()
    from paper_1912_02949_amd._lib import SCGError, SCG_EINVAL
    # a hub row of 200 off-diagonal entries
    star = synth.laplacian_instance(synth.Graph(n=201, src=np.zeros(200, dtype=np.int64),
                                                dst=np.arange(1, 201, dtype=np.int64), w=np.ones(200)))
    with pytest.raises(SCGError) as e:
        make_solver(star, R=4, T=5, seed=3, spmv_lanes=1)
    assert e.value.status == SCG_EINVAL
