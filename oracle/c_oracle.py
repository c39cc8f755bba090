"""ctypes front end of oracle/c/maxcut_oracle.c (test infrastructure only).

The C oracle runs the MaxCut loop body of alg:sketchy-cgal with OpenMP; this
module scales the problem exactly as oracle/sketchycgal.py does (Section
7.1.1) and passes the same Philox test matrix, so the two oracles can be
compared, and so that the benchmark's CPU baseline can use every host core.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import scipy.sparse as sp

from .sketchycgal import OracleParams, gaussian_test_matrix, scale_problem

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c", "maxcut_oracle.c")
LIB = os.path.join(HERE, "c", "libmaxcut_oracle.so")

_lib = None


def build(verbose: bool = False) -> str:
    import subprocess
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", SRC, "-o", LIB, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = C.CDLL(LIB)
        P = C.POINTER(C.c_double)
        lib.scgal_maxcut_iterate.argtypes = [
            C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int, C.c_void_p,
            C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
            C.c_void_p, P, P, C.c_void_p, C.c_int]
        lib.scgal_maxcut_iterate.restype = C.c_int
        _lib = lib
    return _lib


class MaxCutIterations:
    """State of the C oracle on one scaled MaxCut problem (model problem, K = +inf)."""

    def __init__(self, Cm: sp.csr_matrix, b: np.ndarray, params: OracleParams, Omega: np.ndarray | None = None):
        Cm = sp.csr_matrix(Cm, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        alpha0 = float(b.sum()) if params.alpha is None else float(params.alpha)
        Cs, bs, alpha, c_F = scale_problem(Cm, b, alpha0, params.scale)
        self.Cs = sp.csr_matrix(Cs)
        self.n = self.Cs.shape[0]
        self.rp = np.ascontiguousarray(self.Cs.indptr, dtype=np.int64)
        self.col = np.ascontiguousarray(self.Cs.indices, dtype=np.int32)
        self.val = np.ascontiguousarray(self.Cs.data, dtype=np.float64)
        self.b = np.ascontiguousarray(bs)
        self.alpha, self.alpha0, self.c_F = alpha, alpha0, c_F
        self.prm = params
        self.Omega = np.ascontiguousarray(gaussian_test_matrix(self.n, params.R, params.seed, params.instance)
                                          if Omega is None else Omega, dtype=np.float64)
        self.z = np.zeros(self.n)
        self.y = np.zeros(self.n)
        self.S = np.zeros((self.n, params.R))
        self.p = C.c_double(0.0)
        self.tau = C.c_double(0.0)
        self.t_next = 1
        self.log = []

    def run(self, iters: int, threads: int = 0):
        """Advance `iters` iterations on `threads` OpenMP threads (0: the runtime's default)."""
        lib = load()
        t0, t1 = self.t_next, self.t_next + iters - 1
        lg = np.zeros((iters, 6))
        ptr = lambda a: a.ctypes.data
        st = lib.scgal_maxcut_iterate(self.n, ptr(self.rp), ptr(self.col), ptr(self.val), ptr(self.b), self.alpha,
                                      self.prm.R, ptr(self.Omega), self.prm.seed, self.prm.instance, self.prm.q_mode,
                                      self.prm.q_fixed, self.prm.beta0, t0, t1, ptr(self.z), ptr(self.y),
                                      ptr(self.S), C.byref(self.p), C.byref(self.tau), ptr(lg), threads)
        if st != 0:
            raise MemoryError("C oracle: out of memory")
        self.t_next = t1 + 1
        self.log.append(lg)
        return lg

    @property
    def objective(self) -> float:
        return self.c_F * self.alpha0 * self.p.value / self.alpha

    @property
    def infeasibility(self) -> float:
        return self.alpha0 / self.alpha * float(np.linalg.norm(self.z - self.b))
