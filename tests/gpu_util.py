"""Helpers shared by the GPU parity tests (not a test module)."""
from __future__ import annotations

import dataclasses
import sys

import numpy as np
import pytest

import synth
from oracle import OracleParams, sketchy_cgal
from oracle.sketchycgal import state_of


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_02949_amd import _lib
    _lib.load()   # fails loudly when the HIP library is missing


def announce(msg: str):
    print(f"[gpu case] {msg}", file=sys.stderr, flush=True)


def make_solver(inst: synth.MaxCutInstance, omega=None, **kw):
    from paper_1912_02949_amd import Params, SketchyCGAL
    prm = Params(**kw)
    announce(f"init n={inst.n} nnz={inst.nnz} {prm}")
    return SketchyCGAL(inst.row_ptr, inst.col, inst.val, inst.b, prm, omega=omega)


def oracle_params(**kw) -> OracleParams:
    kw = dict(kw)
    for key in ("precision", "matrix_format", "segments", "autotune", "spmv_lanes", "spmv_grid",
                "basis_mode", "omega_mode", "constraint_set", "batch_kernel"):
        kw.pop(key, None)
    alpha = kw.pop("alpha", 0.0)
    op = OracleParams(**{k: v for k, v in kw.items() if k in {f.name for f in dataclasses.fields(OracleParams)}})
    if alpha and alpha > 0:
        op.alpha = alpha
    op.scale = bool(kw.get("scale", 1))
    op.trace_correct = bool(kw.get("trace_correct", 1))
    return op


def oracle_run(inst, lo=None, hi=None, **kw):
    return sketchy_cgal(inst.to_scipy(), inst.b, oracle_params(**kw), lo=lo, hi=hi)


def oracle_snapshots(inst, ts, **kw):
    """Oracle states before iterations t in `ts` (sorted), from one run."""
    op = oracle_params(**kw)
    C = inst.to_scipy()
    snaps = {}
    st = None
    for t in ts:
        if t == 1:
            snaps[1] = None
            continue
        res = sketchy_cgal(C, inst.b, op, state0=st, t_stop=t - 1)
        st = state_of(res, t)
        snaps[t] = st
    return snaps


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def maxrel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
