"""Python front end of the SketchyCGAL library (marshalling only).

Device buffers are torch CUDA tensors; every computation happens in the HIP
library through the C ABI of include/sketchycgal.h.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math

import numpy as np
import torch

from . import _lib
from ._lib import check


@dataclasses.dataclass
class Params:
    """Mirror of scg_params (defaults: the paper's, Section 7.1.2)."""
    R: int = 10
    T: int = 100
    beta0: float = 1.0
    K: float = math.inf
    alpha: float = 0.0            # <= 0: sum(b)
    seed: int = 0
    q_mode: int = 0               # 0: ceil(t^(1/4) ln n); 1: fixed q_fixed
    q_fixed: int = 0
    scale: int = 1
    trace_correct: int = 1
    reorth: int = 0               # 0: paper's Lanczos; 1: local; 2: full reorthogonalisation
    precision: str = "fp64"       # "fp64" or "fp32"
    instance: int = 0
    matrix_format: int = 0        # 0: compress equal-magnitude off-diagonal values; 1: keep values
    autotune: int = 1
    segments: int = 0             # SpMV column segments: 0 auto, or 1, 2, 4, 8 (8: one per XCD, one launch)
    spmv_lanes: int = 0           # SpMV lanes per row: 0 auto, or 2, 4, 8, 16, 32; 1 chunk products (quad or
                                  # entry chunks by storage format; with segments = 8 the column slices in entry chunks)
    spmv_grid: int = 0            # SpMV workgroups: 0 auto, or a cap
    basis_mode: int = 0           # 0: keep the Lanczos basis; 1: three vectors, basis regenerated
    omega_mode: int = 0           # 0: store the test matrix; 1: regenerate it from its counters
    trace_mode: int = 0           # 0: tr X = alpha; 1: tr X <= alpha
    constraint_set: int = 0       # 0: diag X = b; 1: lo <= diag X <= hi (set_constraints); 2: ball (set_ball)
    batch_kernel: int = 0         # batched engine: 0 chosen at init, 1 vector in LDS, 2 two LDS tiles, 3 global

    def to_c(self) -> _lib.scg_params:
        p = _lib.scg_params()
        p.R, p.T, p.beta0, p.K, p.alpha = self.R, self.T, self.beta0, self.K, self.alpha
        p.seed, p.q_mode, p.q_fixed, p.scale = self.seed, self.q_mode, self.q_fixed, self.scale
        p.trace_correct, p.reorth, p.instance = self.trace_correct, self.reorth, self.instance
        p.matrix_format, p.autotune, p.segments = self.matrix_format, self.autotune, self.segments
        p.spmv_lanes, p.spmv_grid = self.spmv_lanes, self.spmv_grid
        p.basis_mode, p.omega_mode = self.basis_mode, self.omega_mode
        p.trace_mode, p.constraint_set = self.trace_mode, self.constraint_set
        p.batch_kernel = self.batch_kernel
        p.precision = {"fp64": _lib.SCG_FP64, "fp32": _lib.SCG_FP32_STREAM}[self.precision]
        return p


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _dev(x, dtype, device):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=device, dtype=dtype).contiguous()


def workspace_bytes(params: Params, n: int, nnz: int) -> int:
    lib = _lib.load()
    out = C.c_size_t()
    check(lib.scg_workspace_size(C.byref(params.to_c()), n, nnz, C.byref(out)), "scg_workspace_size")
    return out.value


class SketchyCGAL:
    """One MaxCut SDP instance: C (CSR, symmetric, diagonal included), b.

    Inputs may be numpy arrays or torch tensors; they are copied to `device`.
    """

    def __init__(self, row_ptr, col, val, b, params: Params, omega=None, device="cuda:0", stream=None):
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.params = params
        rp = _dev(row_ptr, torch.int64, self.device)
        cl = _dev(col, torch.int32, self.device)
        vl = _dev(val, torch.float64, self.device)
        bb = _dev(b, torch.float64, self.device)
        om = None if omega is None else _dev(omega, torch.float64, self.device)
        self.n = int(bb.shape[0])
        self.nnz = int(cl.shape[0])
        if rp.shape[0] != self.n + 1 or vl.shape[0] != self.nnz:
            raise ValueError("CSR arrays have inconsistent sizes")
        if om is not None and om.numel() != self.n * params.R:
            raise ValueError("omega must have n*R entries")
        nbytes = workspace_bytes(params, self.n, self.nnz)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p()
        cp = params.to_c()
        st = self.lib.sketchycgal_init(C.byref(self.ctx), C.byref(cp), self.n, self.nnz, _ptr(rp), _ptr(cl),
                                       _ptr(vl), _ptr(bb), _ptr(om), base + off, nbytes, self.stream.cuda_stream)
        check(st, "sketchycgal_init")

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self.lib.sketchycgal_destroy(ctx)
            self.ctx = None

    def set_constraints(self, lo=None, hi=None):
        """Box constraint set lo <= diag X <= hi (original units; None = unbounded side)."""
        lo_t = None if lo is None else _dev(lo, torch.float64, self.device)
        hi_t = None if hi is None else _dev(hi, torch.float64, self.device)
        check(self.lib.sketchycgal_set_constraints(self.ctx, _ptr(lo_t), _ptr(hi_t)), "sketchycgal_set_constraints")

    def set_ball(self, radius: float):
        """Ball constraint set ||diag X - b|| <= radius (original units)."""
        check(self.lib.sketchycgal_set_ball(self.ctx, float(radius)), "sketchycgal_set_ball")

    def step(self, iters: int = 1):
        check(self.lib.sketchycgal_step(self.ctx, iters), "sketchycgal_step")

    def run(self, iters: int | None = None):
        self.step(self.params.T if iters is None else iters)

    def reconstruct(self):
        R = self.params.R
        U = torch.empty(R * self.n, dtype=torch.float64, device=self.device)
        lam = torch.empty(R, dtype=torch.float64, device=self.device)
        err = torch.empty(R, dtype=torch.float64, device=self.device)
        check(self.lib.sketchycgal_reconstruct(self.ctx, _ptr(U), _ptr(lam), _ptr(err)), "sketchycgal_reconstruct")
        return U.view(R, self.n).t(), lam, err

    def round_cut(self, U):
        """MaxCut rounding of a reconstruction U (n x R): every cut weight, the heaviest's index and indicator."""
        U = _dev(U.t().contiguous().reshape(-1) if isinstance(U, torch.Tensor) else np.asarray(U).T.reshape(-1),
                 torch.float64, self.device)
        chi = torch.empty(self.n, dtype=torch.int8, device=self.device)
        w = (C.c_double * self.params.R)()
        best = C.c_int32()
        check(self.lib.sketchycgal_round(self.ctx, _ptr(U), _ptr(chi), w, C.byref(best)), "sketchycgal_round")
        return np.array(w[:]), best.value, chi

    def log(self) -> dict:
        cap = self.params.T
        arr = (_lib.scg_iter_log * cap)()
        cnt = C.c_int32()
        check(self.lib.sketchycgal_log(self.ctx, arr, cap, C.byref(cnt)), "sketchycgal_log")
        out = {}
        for name, _ in _lib.scg_iter_log._fields_:
            out[name] = np.array([getattr(arr[i], name) for i in range(cnt.value)])
        return out

    def summary(self, check_numeric: bool = True) -> dict:
        s = _lib.scg_summary()
        st = self.lib.sketchycgal_summary(self.ctx, C.byref(s))
        if check_numeric:
            check(st, "sketchycgal_summary")
        return {name: getattr(s, name) for name, _ in _lib.scg_summary._fields_}

    def get_state(self):
        z = torch.empty(self.n, dtype=torch.float64, device=self.device)
        y = torch.empty_like(z)
        S = torch.empty(self.n * self.params.R, dtype=torch.float64, device=self.device)
        t = C.c_int32()
        p = C.c_double()
        tau = C.c_double()
        check(self.lib.sketchycgal_get_state(self.ctx, C.byref(t), _ptr(z), _ptr(y), _ptr(S), C.byref(p),
                                             C.byref(tau)), "sketchycgal_get_state")
        return {"t": t.value, "z": z, "y": y, "S": S.view(self.n, self.params.R), "p": p.value, "tau": tau.value}

    def set_state(self, t, z, y, S, p, tau):
        z = _dev(z, torch.float64, self.device)
        y = _dev(y, torch.float64, self.device)
        S = _dev(S, torch.float64, self.device).reshape(-1)
        check(self.lib.sketchycgal_set_state(self.ctx, int(t), _ptr(z), _ptr(y), _ptr(S), float(p), float(tau)),
              "sketchycgal_set_state")

    def lanczos_coeffs(self):
        cap = 512
        om = (C.c_double * cap)()
        rh = (C.c_double * cap)()
        k = C.c_int32()
        xi = C.c_double()
        check(self.lib.sketchycgal_lanczos_coeffs(self.ctx, om, rh, cap, C.byref(k), C.byref(xi)),
              "sketchycgal_lanczos_coeffs")
        kk = k.value
        return np.array(om[:kk]), np.array(rh[:max(kk - 1, 0)]), xi.value

    def apply(self, x):
        x = _dev(x, torch.float64, self.device)
        y = torch.empty_like(x)
        check(self.lib.sketchycgal_apply(self.ctx, _ptr(x), _ptr(y)), "sketchycgal_apply")
        return y

    def time_spmv(self, reps: int = 50) -> float:
        ms = C.c_double()
        check(self.lib.sketchycgal_time_spmv(self.ctx, reps, C.byref(ms)), "sketchycgal_time_spmv")
        return ms.value


def batch_workspace_bytes(params: Params, inst_n, nnz: int) -> int:
    lib = _lib.load()
    ns = np.ascontiguousarray(np.asarray(inst_n, dtype=np.int64))
    out = C.c_size_t()
    check(lib.scg_batch_workspace_size(C.byref(params.to_c()), len(ns), ns.ctypes.data, int(nnz), C.byref(out)),
          "scg_batch_workspace_size")
    return out.value


class BatchedSketchyCGAL:
    """Many independent instances advanced together, one launch per iteration.

    `instances` is a sequence of objects with row_ptr, col, val, b (numpy, CSR
    with instance-local column numbers); they are concatenated into one
    block-diagonal CSR here.  Instance i draws its random streams with Philox
    counter word params.instance + i.  A private non-default stream is used so
    that runs of iterations replay a captured HIP graph.
    """

    def __init__(self, instances, params: Params, device="cuda:0", stream=None):
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.params = params
        ns = np.array([int(len(g.b)) for g in instances], dtype=np.int64)
        offs = np.concatenate([[0], np.cumsum(ns)])
        nnzs = np.array([int(g.row_ptr[-1]) for g in instances], dtype=np.int64)
        eoffs = np.concatenate([[0], np.cumsum(nnzs)])
        rp = np.concatenate([np.asarray(g.row_ptr[:-1], dtype=np.int64) + eoffs[i] for i, g in enumerate(instances)]
                            + [np.array([eoffs[-1]], dtype=np.int64)])
        cl = np.concatenate([np.asarray(g.col, dtype=np.int64) + offs[i] for i, g in enumerate(instances)])
        vl = np.concatenate([np.asarray(g.val, dtype=np.float64) for g in instances])
        bb = np.concatenate([np.asarray(g.b, dtype=np.float64) for g in instances])
        self.inst_n = ns
        self.n_inst = len(ns)
        self.nnz = int(eoffs[-1])
        nbytes = batch_workspace_bytes(params, ns, self.nnz)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        d_rp = _dev(rp, torch.int64, self.device)
        d_cl = _dev(cl.astype(np.int32), torch.int32, self.device)
        d_vl = _dev(vl, torch.float64, self.device)
        d_b = _dev(bb, torch.float64, self.device)
        torch.cuda.current_stream(self.device).synchronize()
        self.ctx = C.c_void_p()
        cp = params.to_c()
        st = self.lib.sketchycgal_batch_init(C.byref(self.ctx), C.byref(cp), self.n_inst, ns.ctypes.data, self.nnz,
                                             _ptr(d_rp), _ptr(d_cl), _ptr(d_vl), _ptr(d_b), base + off, nbytes,
                                             self.stream.cuda_stream)
        check(st, "sketchycgal_batch_init")

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self.lib.sketchycgal_batch_destroy(ctx)
            self.ctx = None

    def set_beta0(self, beta0):
        """Per-problem initial penalty beta_0 (before the first step)."""
        arr = np.ascontiguousarray(np.asarray(beta0, dtype=np.float64))
        if arr.shape != (len(self.inst_n),):
            raise ValueError("one beta0 per problem")
        check(self.lib.sketchycgal_batch_set_beta0(self.ctx, arr.ctypes.data), "sketchycgal_batch_set_beta0")

    def step(self, iters: int = 1):
        check(self.lib.sketchycgal_batch_step(self.ctx, iters), "sketchycgal_batch_step")

    def run(self, iters: int | None = None):
        self.step(self.params.T if iters is None else iters)

    def synchronize(self):
        self.stream.synchronize()

    def log(self, inst: int) -> dict:
        cap = self.params.T
        arr = (_lib.scg_iter_log * cap)()
        cnt = C.c_int32()
        check(self.lib.sketchycgal_batch_log(self.ctx, inst, arr, cap, C.byref(cnt)), "sketchycgal_batch_log")
        return {name: np.array([getattr(arr[i], name) for i in range(cnt.value)])
                for name, _ in _lib.scg_iter_log._fields_}

    def summary(self, inst: int, check_numeric: bool = True) -> dict:
        s = _lib.scg_summary()
        st = self.lib.sketchycgal_batch_summary(self.ctx, inst, C.byref(s))
        if check_numeric:
            check(st, "sketchycgal_batch_summary")
        return {name: getattr(s, name) for name, _ in _lib.scg_summary._fields_}

    def get_state(self, inst: int):
        n = int(self.inst_n[inst])
        R = self.params.R
        z = torch.empty(n, dtype=torch.float64, device=self.device)
        y = torch.empty_like(z)
        S = torch.empty(n * R, dtype=torch.float64, device=self.device)
        t = C.c_int32()
        p = C.c_double()
        tau = C.c_double()
        check(self.lib.sketchycgal_batch_get_state(self.ctx, inst, C.byref(t), _ptr(z), _ptr(y), _ptr(S),
                                                   C.byref(p), C.byref(tau)), "sketchycgal_batch_get_state")
        return {"t": t.value, "z": z, "y": y, "S": S.view(n, R), "p": p.value, "tau": tau.value}

    def set_state(self, inst: int, t, z, y, S, p, tau):
        z = _dev(z, torch.float64, self.device)
        y = _dev(y, torch.float64, self.device)
        S = _dev(S, torch.float64, self.device).reshape(-1)
        torch.cuda.current_stream(self.device).synchronize()
        check(self.lib.sketchycgal_batch_set_state(self.ctx, inst, int(t), _ptr(z), _ptr(y), _ptr(S), float(p),
                                                   float(tau)), "sketchycgal_batch_set_state")

    def round_cut(self, inst: int, U):
        """MaxCut rounding of instance `inst` from its reconstruction U (n_i x R)."""
        n = int(self.inst_n[inst])
        U = _dev(U.t().contiguous().reshape(-1) if isinstance(U, torch.Tensor) else np.asarray(U).T.reshape(-1),
                 torch.float64, self.device)
        chi = torch.empty(n, dtype=torch.int8, device=self.device)
        w = (C.c_double * self.params.R)()
        best = C.c_int32()
        check(self.lib.sketchycgal_batch_round(self.ctx, inst, _ptr(U), _ptr(chi), w, C.byref(best)),
              "sketchycgal_batch_round")
        return np.array(w[:]), best.value, chi

    def reconstruct(self, inst: int):
        n = int(self.inst_n[inst])
        R = self.params.R
        U = torch.empty(R * n, dtype=torch.float64, device=self.device)
        lam = torch.empty(R, dtype=torch.float64, device=self.device)
        err = torch.empty(R, dtype=torch.float64, device=self.device)
        check(self.lib.sketchycgal_batch_reconstruct(self.ctx, inst, _ptr(U), _ptr(lam), _ptr(err)),
              "sketchycgal_batch_reconstruct")
        return U.view(R, n).t(), lam, err


@dataclasses.dataclass
class PhaseParams:
    """Mirror of scg_pr_params (phase retrieval; defaults R = 5, alpha = 3 n)."""
    R: int = 5
    T: int = 100
    beta0: float = 1.0
    K: float = math.inf
    alpha: float = 0.0            # 0: 3 n
    seed: int = 0
    q_mode: int = 0
    q_fixed: int = 0
    scale: int = 1
    trace_correct: int = 1
    instance: int = 0
    mask_groups: int = 0          # inverse column pass: waveform groups (0: chosen)
    tile_cols: int = 0            # column-pass tile width (0: chosen)
    mask_format: int = 0          # 0: dictionary codes when the waveforms take <= 256 values; 1: whole
    autotune: int = 1             # 1: time the waveform group counts at init when mask_groups = 0

    def to_c(self) -> _lib.scg_pr_params:
        p = _lib.scg_pr_params()
        for name, _ in _lib.scg_pr_params._fields_:
            setattr(p, name, getattr(self, name))
        return p


def _cplx(x, device):
    """Complex data as an interleaved float64 device tensor."""
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=torch.complex128).contiguous()
    else:
        t = torch.as_tensor(np.ascontiguousarray(np.asarray(x, dtype=np.complex128))).to(device).contiguous()
    return torch.view_as_real(t).contiguous()


class PhaseRetrieval:
    """Phase retrieval SDP on coded diffraction measurements (psi: L x n complex
    waveforms, b: L x n measurements), solved by the library's complex engine."""

    def __init__(self, psi, b, params: PhaseParams, omega=None, device="cuda:0", stream=None):
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.params = params
        ps = _cplx(psi, self.device)
        self.L, self.n = int(ps.shape[0]), int(ps.shape[1])
        bb = _dev(b, torch.float64, self.device).reshape(-1)
        if bb.numel() != self.L * self.n:
            raise ValueError("b must have L * n entries")
        om = None
        if omega is not None:   # n x R complex -> column-contiguous R x n
            o = omega.t() if isinstance(omega, torch.Tensor) else np.asarray(omega).T
            om = _cplx(o, self.device)
            if om.shape[0] != params.R or om.shape[1] != self.n:
                raise ValueError("omega must be n x R")
        out = C.c_size_t()
        cp = params.to_c()
        check(self.lib.scg_pr_workspace_size(C.byref(cp), self.n, self.L, C.byref(out)), "scg_pr_workspace_size")
        nbytes = out.value
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p()
        torch.cuda.current_stream(self.device).synchronize()
        check(self.lib.scg_pr_init(C.byref(self.ctx), C.byref(cp), self.n, self.L, _ptr(ps), _ptr(bb), _ptr(om),
                                   base + off, nbytes, self.stream.cuda_stream), "scg_pr_init")

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self.lib.scg_pr_destroy(ctx)
            self.ctx = None

    def step(self, iters: int = 1):
        check(self.lib.scg_pr_step(self.ctx, iters), "scg_pr_step")

    def run(self, iters: int | None = None):
        self.step(self.params.T if iters is None else iters)

    def synchronize(self):
        self.stream.synchronize()

    def apply(self, w, x) -> torch.Tensor:
        """(C + A^*(w)) x in scaled units; w is L x n (scaled dual weights), x complex n."""
        wt = _dev(w, torch.float64, self.device).reshape(-1)
        xt = _cplx(x, self.device)
        y = torch.empty(self.n, 2, dtype=torch.float64, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        check(self.lib.scg_pr_apply(self.ctx, _ptr(wt), _ptr(xt), _ptr(y)), "scg_pr_apply")
        return torch.view_as_complex(y)

    def measure(self, x) -> torch.Tensor:
        """A(x x^*) in scaled units, L x n."""
        xt = _cplx(x, self.device)
        m = torch.empty(self.L * self.n, dtype=torch.float64, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        check(self.lib.scg_pr_measure(self.ctx, _ptr(xt), _ptr(m)), "scg_pr_measure")
        return m.view(self.L, self.n)

    def log(self) -> dict:
        cap = self.params.T
        arr = (_lib.scg_iter_log * cap)()
        cnt = C.c_int32()
        check(self.lib.scg_pr_log(self.ctx, arr, cap, C.byref(cnt)), "scg_pr_log")
        return {name: np.array([getattr(arr[i], name) for i in range(cnt.value)])
                for name, _ in _lib.scg_iter_log._fields_}

    def summary(self, check_numeric: bool = True) -> dict:
        s = _lib.scg_pr_info()
        st = self.lib.scg_pr_summary(self.ctx, C.byref(s), 1 if check_numeric else 0)
        check(st, "scg_pr_summary")
        return {name: getattr(s, name) for name, _ in _lib.scg_pr_info._fields_}

    def get_state(self) -> dict:
        z = torch.empty(self.L * self.n, dtype=torch.float64, device=self.device)
        y = torch.empty_like(z)
        S = torch.empty(self.params.R, self.n, 2, dtype=torch.float64, device=self.device)
        t = C.c_int32()
        p = C.c_double()
        tau = C.c_double()
        check(self.lib.scg_pr_get_state(self.ctx, C.byref(t), _ptr(z), _ptr(y), _ptr(S), C.byref(p), C.byref(tau)),
              "scg_pr_get_state")
        return {"t": t.value, "z": z.view(self.L, self.n), "y": y.view(self.L, self.n),
                "S": torch.view_as_complex(S).t(), "p": p.value, "tau": tau.value}

    def set_state(self, t, z, y, S, p, tau):
        """S: n x R complex (scaled units), z, y: L x n."""
        zt = _dev(z, torch.float64, self.device).reshape(-1)
        yt = _dev(y, torch.float64, self.device).reshape(-1)
        St = _cplx(S.t() if isinstance(S, torch.Tensor) else np.asarray(S).T, self.device)
        torch.cuda.current_stream(self.device).synchronize()
        check(self.lib.scg_pr_set_state(self.ctx, int(t), _ptr(zt), _ptr(yt), _ptr(St), float(p), float(tau)),
              "scg_pr_set_state")

    def reconstruct(self):
        """(U n x R complex, lambda, err), scaled units."""
        R = self.params.R
        U = torch.empty(R, self.n, 2, dtype=torch.float64, device=self.device)
        lam = torch.empty(R, dtype=torch.float64, device=self.device)
        err = torch.empty(R, dtype=torch.float64, device=self.device)
        check(self.lib.scg_pr_reconstruct(self.ctx, _ptr(U), _ptr(lam), _ptr(err)), "scg_pr_reconstruct")
        return torch.view_as_complex(U).t(), lam, err

    def time_apply(self, reps: int = 20) -> dict:
        """Event-timed average ms of the three DFT passes of one product and of the whole product."""
        ms = (C.c_double * 4)()
        check(self.lib.scg_pr_time_apply(self.ctx, reps, ms), "scg_pr_time_apply")
        return {"colfwd": ms[0], "row": ms[1], "colinv": ms[2], "apply": ms[3]}

    def round(self, U, lam, chi_true=None):
        """chi = sqrt(alpha lambda_1) u_1 (original units) and, given chi_true, the relative error."""
        Ut = _cplx(U.t() if isinstance(U, torch.Tensor) else np.asarray(U).T, self.device)
        lt = _dev(lam, torch.float64, self.device)
        ct = None if chi_true is None else _cplx(chi_true, self.device)
        chi = torch.empty(self.n, 2, dtype=torch.float64, device=self.device)
        rel = C.c_double(float("nan"))
        torch.cuda.current_stream(self.device).synchronize()
        check(self.lib.scg_pr_round(self.ctx, _ptr(Ut), _ptr(lt), _ptr(ct), _ptr(chi),
                                    C.byref(rel) if ct is not None else None), "scg_pr_round")
        return torch.view_as_complex(chi), rel.value
