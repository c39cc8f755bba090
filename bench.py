"""Benchmark: SketchyCGAL MaxCut solves per second on one MI355X.

Headline workload: MaxCut SDP on a 1024 x 1024 torus (4-neighbour) plus 2n
random long-range edges, weights +-1 (n = 1,048,576), sketch size R = 10,
T = 2000 iterations, the paper's Lanczos schedule q_t = ceil(t^(1/4) ln n),
plain FP64 (the paper's precision).  One step = one whole solve on inputs
resident in HBM: initialisation (validation, scaling, diagonal split, Omega,
SpMV autotuning), T iterations, and the Nystrom reconstruction.  `value` is
CGAL iterations per second of that solve.

Also reported:
  result_fp64   the FP64 solve's result and Lanczos SpMV line, and how far the
                same solve with its products summed in another order ends up
                (whole runs of this method follow rounding)
  fp32_stream   the FP32-stream/FP64-critical form of the same workload: one
                solve, its difference from FP64, the speedup at equal final
                ||diag X - b||, MaxCut rounding of its reconstruction, its SpMV
  other_workloads  whole FP32-stream solves of the 2^23-vertex random geometric
                workload (T = 500) and the 2^22-vertex power-law workload
                (T = 1000), with their Lanczos SpMV lines
  workload_1    the 800-vertex G(n, m) workload as its text specifies it (FP64,
                q = 36, R = 10, T = 500): iterations/s of the single engine and
                of the batched engine running it as a one-instance batch
  batched       256 Erdos-Renyi instances (average degree 8, n uniform in
                [200, 20000]), R = 8, T = 1000, all advanced by one launch per
                iteration; FP32 and FP64
  roofline      the Lanczos SpMV of the geometric workload (its working set
                exceeds the 256 MB last-level cache): algorithmic bytes per
                product (values + int32 columns, row pointers, x, shift, u) over
                its average duration (HIP events on the solver's stream) against
                the MI355X HBM peak; `traffic` is the rocprofv3-measured HBM bytes
                per launch of the chosen shape from the committed counter summary
                when it matches the current kernel source, else null
  cpu_baseline  the FP64 oracle on this host, on a bounded sample of the
                headline workload, extrapolated over the whole Lanczos schedule
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# SpMV shapes whose HBM traffic the profile records: (lanes per row, workgroups cap, column segments);
# workgroups 0 = one row-block range per wave; lanes 1 = a chunk product (k_spmvq over padded column-word
# quads; k_spmve over unpadded entries with their values); 8 segments = the concurrent form (k_spmv slice
# sums + k_xcombine)
PROBE_SHAPES = {
    2: tuple((l, g, 1) for l in (2, 4) for g in (1024, 1536, 0)) + ((2, 1536, 2), (2, 0, 2), (1, 1536, 1), (1, 2048, 1)),
    3: ((2, 1024, 8), (2, 2048, 8), (4, 1536, 4), (4, 0, 1), (1, 1024, 8), (1, 2048, 8)),
    5: tuple((l, g, 1) for l in (2, 4) for g in (1024, 1536, 0)) + ((1, 1536, 1), (1, 1792, 1), (1, 2048, 1)),
}
TRAFFIC_FILES = {
    (2, "fp32"): os.path.join(ROOT, "profiles", "spmv_traffic_torus_1m_fp32.json"),
    (3, "fp32"): os.path.join(ROOT, "profiles", "spmv_traffic_powerlaw_4m_fp32.json"),
    (5, "fp32"): os.path.join(ROOT, "profiles", "spmv_traffic_geometric_8m_fp32.json"),
    (5, "fp64"): os.path.join(ROOT, "profiles", "spmv_traffic_geometric_8m_fp64.json"),
}


def measured_traffic(k: int, summ: dict, precision: str = "fp32"):
    """HBM bytes per SpMV launch of the shape in `summ`, from the committed counter summary of workload k
    in that precision."""
    path = TRAFFIC_FILES.get((k, precision))
    if path is None or not os.path.exists(path):
        return None
    with open(path) as f:
        tr = json.load(f)
    if tr.get("kernel_source_sha") != kernel_source_sha():
        return None
    for sh in tr.get("shapes", []):
        if (sh["lanes"], sh["workgroups"], sh["segments"]) == (summ["spmv_lanes"], summ["spmv_grid"],
                                                               summ["spmv_segments"]):
            return sh["hbm_bytes_per_launch"]
    return None
KERNEL_SOURCES = ["scg_kernels.hpp", "scg_device.hpp", "scg_internal.hpp"]


def spmv_kernel_name(summ: dict) -> str:
    """The product kernel the autotuner chose: lanes 1 is a chunk layout (quad chunks of column words, or
    entry chunks when values are stored); with 8 column segments the row-block kernel runs them in one launch
    and k_xcombine adds the segment sums."""
    if summ["spmv_lanes"] == 1 and summ["spmv_segments"] == 8:
        return "k_spmvx + k_xcombine"
    if summ["spmv_lanes"] == 1:
        return "k_spmve" if summ["matrix_format"] == 0 else "k_spmvq"
    return "k_spmv + k_xcombine" if summ["spmv_segments"] == 8 else "k_spmv"


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1912_02949_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def q_schedule(T: int, n: int):
    return [max(1, min(math.ceil(t ** 0.25 * math.log(n)), n - 1)) for t in range(1, T + 1)]


class Solve:
    """Preallocated device buffers for repeated whole solves through the C ABI."""

    def __init__(self, inst, params, torch):
        from paper_1912_02949_amd import _lib
        from paper_1912_02949_amd.api import workspace_bytes
        self.lib = _lib.load()
        self.torch = torch
        dev = torch.device("cuda:0")
        self.prm = params
        self.rp = torch.as_tensor(inst.row_ptr).to(dev)
        self.col = torch.as_tensor(inst.col).to(dev)
        self.val = torch.as_tensor(inst.val).to(dev)
        self.b = torch.as_tensor(inst.b).to(dev)
        self.n, self.nnz = inst.n, inst.nnz
        self.nbytes = workspace_bytes(params, self.n, self.nnz)
        self.ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=dev)
        self.base = self.ws.data_ptr() + ((-self.ws.data_ptr()) % 256)
        self.U = torch.empty(params.R * self.n, dtype=torch.float64, device=dev)
        self.lam = torch.empty(params.R, dtype=torch.float64, device=dev)
        self.err = torch.empty(params.R, dtype=torch.float64, device=dev)
        self.stream = torch.cuda.current_stream(dev).cuda_stream
        self.ctx = None

    def init(self):
        from paper_1912_02949_amd._lib import check
        ctx = C.c_void_p()
        cp = self.prm.to_c()
        check(self.lib.sketchycgal_init(C.byref(ctx), C.byref(cp), self.n, self.nnz, self.rp.data_ptr(),
                                        self.col.data_ptr(), self.val.data_ptr(), self.b.data_ptr(), None,
                                        self.base, self.nbytes, self.stream), "init")
        self.ctx = ctx

    def run(self, keep=False):
        from paper_1912_02949_amd._lib import check
        self.init()
        check(self.lib.sketchycgal_step(self.ctx, self.prm.T), "step")
        check(self.lib.sketchycgal_reconstruct(self.ctx, self.U.data_ptr(), self.lam.data_ptr(),
                                               self.err.data_ptr()), "reconstruct")
        if not keep:
            self.close()

    def round_cut(self):
        """MaxCut rounding of the last reconstruction: (heaviest cut weight, its index, seconds)."""
        from paper_1912_02949_amd._lib import check
        w = (C.c_double * self.prm.R)()
        best = C.c_int32()
        chi = self.torch.empty(self.n, dtype=self.torch.int8, device=self.U.device)
        self.torch.cuda.synchronize()
        t0 = time.perf_counter()
        check(self.lib.sketchycgal_round(self.ctx, self.U.data_ptr(), chi.data_ptr(), w, C.byref(best)), "round")
        dt = time.perf_counter() - t0
        return w[best.value], best.value, dt

    def close(self):
        if self.ctx is not None:
            self.lib.sketchycgal_destroy(self.ctx)
            self.ctx = None

    def summary(self):
        from paper_1912_02949_amd import _lib
        s = _lib.scg_summary()
        self.lib.sketchycgal_summary(self.ctx, C.byref(s))
        return {k: getattr(s, k) for k, _ in _lib.scg_summary._fields_}

    def record(self, which: int = -1):
        """One iteration's log record (scaled units) as a dict: the last by default, 0 for t = 1."""
        from paper_1912_02949_amd import _lib
        cap = self.prm.T
        arr = (_lib.scg_iter_log * cap)()
        cnt = C.c_int32()
        _lib.check(self.lib.sketchycgal_log(self.ctx, arr, cap, C.byref(cnt)), "log")
        rec = arr[which if which >= 0 else cnt.value + which]
        return {k: getattr(rec, k) for k, _ in _lib.scg_iter_log._fields_}

    def infeasibility_log(self):
        """||diag X_{t+1} - b|| per iteration, original units."""
        from paper_1912_02949_amd import _lib
        cap = self.prm.T
        arr = (_lib.scg_iter_log * cap)()
        cnt = C.c_int32()
        _lib.check(self.lib.sketchycgal_log(self.ctx, arr, cap, C.byref(cnt)), "log")
        s = self.summary()
        return [arr[i].infeas * s["alpha"] / s["alpha_scaled"] for i in range(cnt.value)]


def timed(solve: Solve, steps: int, warmup: int, torch):
    for _ in range(warmup):
        solve.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        solve.run(keep=(k == steps - 1))
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_baseline(inst, T: int, seconds: float = 15.0):
    """The FP64 oracle in its C/OpenMP form (oracle/c, checked against the Python oracle by the CPU tests) on a
    bounded prefix of the workload: first on every host core the process may use, then on one thread, about
    seconds / 2 each; each rate is extrapolated over the whole Lanczos schedule by operator applications."""
    import oracle
    from oracle.c_oracle import MaxCutIterations
    from oracle.sketchycgal import gaussian_test_matrix
    import synth

    qs = q_schedule(T, inst.n)
    Cm = inst.to_scipy()
    prm = oracle.OracleParams(R=10, T=T, seed=synth.CONFIG_SEEDS[2])
    Om = gaussian_test_matrix(inst.n, 10, prm.seed)      # drawn once, outside the timing
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    work_all = sum(q + 1 for q in qs)
    rates = {}
    for threads in (cores, 1):
        c = MaxCutIterations(Cm, inst.b, prm, Omega=Om)
        done, spent = 0, 0.0
        while spent < seconds / 2 and done < T:
            t0 = time.perf_counter()
            c.run(1, threads=threads)
            spent += time.perf_counter() - t0
            done += 1
        work_done = sum(q + 1 for q in qs[:done])
        rates[threads] = (T / (spent / work_done * work_all), done, spent, work_done)
    v, done, spent, wd = rates[cores]
    v1, done1, spent1, wd1 = rates[1]
    return {
        "value": v,
        "unit": "CGAL iters/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"first {done} of {T} iterations ({wd} operator applications incl. the objective product) in "
                   f"{spent:.1f} s on {cores} OpenMP threads, FP64, the C form of the oracle; extrapolated over the "
                   f"whole schedule ({work_all} applications)"),
        "single_thread_value": v1,
        "single_thread_sample": f"first {done1} iterations in {spent1:.1f} s on one thread, extrapolated the same way",
        "host_cpus": os.cpu_count(),
    }


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gather_reference(torch, n: int, count: int, reps: int = 20):
    """Reference rate of random 4-byte gathers on this GPU: torch.index_select of `count` uniform random int32
    indices from an n-entry FP32 vector (the size of the torus workload's x and its off-diagonal count), HIP
    events.  Every index is uniform here, while half of the torus's are local, so the SpMV can exceed it."""
    g = torch.Generator(device="cuda:0")
    g.manual_seed(0x5C6A)
    x = torch.rand(n, device="cuda:0", dtype=torch.float32, generator=g)
    idx = torch.randint(0, n, (count,), device="cuda:0", generator=g).to(torch.int32)
    torch.index_select(x, 0, idx)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.index_select(x, 0, idx)
    e1.record()
    torch.cuda.synchronize()
    return count * reps / (e0.elapsed_time(e1) * 1e-3)


def copy_ceiling(torch, nbytes: int = 1 << 30, reps: int = 10):
    """Device-to-device copy rate (read + write bytes per second) of a 1 GiB buffer, HIP events: the
    bandwidth a plain streaming kernel reaches on this GPU, beside the 8 TB/s vendor figure."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    rate = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return rate


def workload1_leg(torch) -> dict:
    """Workload 1 (n = 800, 19 176 unit edges, FP64, q = 36, R = 10, T = 500): T iterations timed
    after initialisation, once per engine, the first run of each untimed."""
    import synth
    from paper_1912_02949_amd import BatchedSketchyCGAL, Params, SketchyCGAL
    inst = synth.config_instance(1)
    prm = Params(R=10, T=500, seed=synth.CONFIG_SEEDS[1], q_mode=1, q_fixed=36, precision="fp64")
    out = {"workload": "G(n, m), n = 800, m = 19176, unit weights, R = 10, T = 500, q = 36, FP64"}
    st = torch.cuda.Stream()   # a non-null stream: every iteration a replay of one captured graph
    makers = {"single_engine": lambda: SketchyCGAL(inst.row_ptr, inst.col, inst.val, inst.b, prm),
              "single_engine_graph_replays": lambda: SketchyCGAL(inst.row_ptr, inst.col, inst.val, inst.b, prm,
                                                                 stream=st),
              "batched_engine_one_instance": lambda: BatchedSketchyCGAL([inst], prm, stream=st)}
    for name, make in makers.items():
        best, obj = None, None
        for rep in range(2):
            s = make()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.run()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            obj = s.summary()["objective"] if name.startswith("single") else s.summary(0)["objective"]
            if rep == 1:
                best = dt
            del s
        out[name] = {"iters_per_s": prm.T / best, "ms_per_iteration": 1e3 * best / prm.T,
                     "sdp_value": -obj}
    return out


def batched_bytes(n: int, m: int, k: int, es: int, cb: int, vb: int, R: int) -> int:
    """Bytes one batched iteration of a problem with n rows, m off-diagonal entries and k Lanczos steps
    streams through memory, each array counted once per pass as the kernel reads or writes it:
    prep (z, y, b, diag C read; shift and start vector written), the shift in slice order (permutation,
    shift gathered and written), k products (permutation, shift, product written; column words and
    values), k - 1 three-term updates (product and v_{i-1} read, v_{i+1} written), the Ritz combination
    (k basis vectors), the norm and v^T Omega (Omega), the objective product (permutation, shift,
    diagonal; column words and values) and the tail (z, y read and written, b twice, S read and written)."""
    per_row = (32 + 2 * es) + (4 + 2 * es) + k * (4 + 2 * es) + (k - 1) * 3 * es + k * es + R * es \
        + (12 + es) + (56 + 2 * es * R)
    return n * per_row + (k + 1) * (cb + vb) * m


def batched_leg(torch, T: int, with_fp64: bool):
    """Whole batched solves (init excluded from the rate, reported beside it)."""
    import synth
    from paper_1912_02949_amd import BatchedSketchyCGAL, Params
    insts = synth.batched_erdos_renyi(256, 200, 20000, 8)
    out = {"workload": "256 MaxCut SDPs, Erdos-Renyi average degree 8, n uniform in [200, 20000] "
                       "(sum n = %d), R=8, T=%d, q_t=ceil(t^(1/4) ln n_i)" % (sum(g.n for g in insts), T),
           "instances": len(insts)}
    for prec in (("fp32", "fp64") if with_fp64 else ("fp32",)):
        prm = Params(R=8, T=T, seed=synth.CONFIG_SEEDS[4], precision=prec)
        t0 = time.perf_counter()
        b = BatchedSketchyCGAL(insts, prm)
        b.synchronize()
        t1 = time.perf_counter()
        b.step(T)
        b.synchronize()
        t2 = time.perf_counter()
        infeas = [b.summary(i)["infeasibility"] / math.sqrt(insts[i].n) for i in range(len(insts))]
        # algorithmic bytes of the whole run from every problem's recorded Lanczos steps (each array
        # counted once per pass of the algorithm, whatever the kernel form re-reads)
        es = 4 if prec == "fp32" else 8
        fmt = b.summary(0)["matrix_format"]
        nmax = max(g.n for g in insts)
        cb = 2 if nmax <= (32767 if fmt == 2 else 65535) else 4
        total = sum(batched_bytes(g.n, g.nnz - g.n, int(kk), es, cb, 0 if fmt != 0 else es, 8)
                    for i, g in enumerate(insts) for kk in b.log(i)["k"])
        gbs = total / (t2 - t1) / 1e9
        out[prec] = {"kernel_form": {1: "vector in LDS", 2: "two LDS column tiles", 3: "global gathers"}.get(
                         b.summary(0)["batch_kernel"]),
                     "batch_iters_per_s": T / (t2 - t1), "instance_iters_per_s": len(insts) * T / (t2 - t1),
                     "ms_per_iteration": 1e3 * (t2 - t1) / T, "init_s": t1 - t0,
                     "max_rel_infeasibility": max(infeas),
                     "objective_sum": sum(b.summary(i)["objective"] for i in range(len(insts))),
                     "algorithmic_bytes_per_iteration": total / T,
                     "algorithmic_GBps": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
        del b
        progress(f"batched {prec}: {out[prec]['ms_per_iteration']:.3f} ms per iteration")
    if with_fp64:
        out["speedup_fp32_vs_fp64"] = out["fp32"]["batch_iters_per_s"] / out["fp64"]["batch_iters_per_s"]
    return out


def spmv_roofline(solve, inst, precision: str, reps: int, k: int) -> dict:
    """The Lanczos SpMV of a solver context: `reps` back-to-back products of Lanczos step 1 on the solver's
    stream, timed with HIP events; algorithmic bytes per product as the scope table counts them (values +
    int32 columns, row pointers, x, shift, u written) and, beside them, the bytes the chosen storage format
    needs (no value stream when the off-diagonal values share one magnitude)."""
    ms = C.c_double()
    from paper_1912_02949_amd._lib import check
    check(solve.lib.sketchycgal_time_spmv(solve.ctx, reps, C.byref(ms)), "time_spmv")
    summ = solve.summary()
    es = 4 if precision == "fp32" else 8
    n, nnz_off = inst.n, inst.nnz - inst.n
    by = (4 + es) * nnz_off + 4 * (n + 1) + 3 * es * n
    by_fmt = (4 + (es if summ["matrix_format"] == 0 else 0)) * nnz_off + 4 * (n + 1) + 3 * es * n
    us = ms.value * 1e3
    gbs = by / (us * 1e-6) / 1e9
    return {"kernel": spmv_kernel_name(summ), "lanes_per_row": summ["spmv_lanes"],
            "column_segments": summ["spmv_segments"], "workgroups": summ["spmv_grid"],
            "matrix_format": ["values", "columns only", "columns with sign bit"][summ["matrix_format"]],
            "avg_product_us": us, "launches_per_product": summ["spmv_segments"],
            "algorithmic_bytes_per_product": by, "achieved_GBps": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
            "format_bytes_per_product": by_fmt, "format_GBps": by_fmt / (us * 1e-6) / 1e9,
            "gathers_per_s": nnz_off / (us * 1e-6),
            "traffic": measured_traffic(k, summ, precision)}


def solve_leg(torch, k: int, inst, precision: str, T: int, spmv_reps: int = 100, warm_T: int = 20) -> dict:
    """Whole solve of workload k (init, T iterations, reconstruction) timed once after a short warm-up
    solve (T = warm_T) of the same problem; then its Lanczos SpMV line."""
    import synth
    from paper_1912_02949_amd import Params
    warm = Solve(inst, Params(R=10, T=warm_T, seed=synth.CONFIG_SEEDS[k], precision=precision), torch)
    warm.run()
    del warm
    sv = Solve(inst, Params(R=10, T=T, seed=synth.CONFIG_SEEDS[k], precision=precision), torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv.init()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    from paper_1912_02949_amd._lib import check
    check(sv.lib.sketchycgal_step(sv.ctx, T), "step")
    check(sv.lib.sketchycgal_reconstruct(sv.ctx, sv.U.data_ptr(), sv.lam.data_ptr(), sv.err.data_ptr()),
          "reconstruct")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    summ = sv.summary()
    last = sv.record()
    norm_b = math.sqrt(float((inst.b * inst.b).sum()))
    out = {"precision": precision, "T": T, "iters_per_s": T / (t2 - t0), "solve_ms": 1e3 * (t2 - t0),
           "init_ms": 1e3 * (t1 - t0), "iters_per_s_after_init": T / (t2 - t1),
           "lanczos_steps_total": sum(q_schedule(T, inst.n)),
           "objective": summ["objective"], "infeasibility_rel": summ["infeasibility"] / norm_b,
           "eigen_residual_scaled": last["resid"],
           "spmv": spmv_roofline(sv, inst, precision, spmv_reps, k)}
    sv.close()
    return out


def spmv_leg(torch, k: int, inst, precision: str, reps: int = 100) -> dict:
    """The Lanczos SpMV line of workload k in one precision, without a whole solve (init, autotuning,
    then `reps` timed products)."""
    import synth
    from paper_1912_02949_amd import Params
    sv = Solve(inst, Params(R=10, T=20, seed=synth.CONFIG_SEEDS[k], precision=precision), torch)
    sv.init()
    out = spmv_roofline(sv, inst, precision, reps, k)
    sv.close()
    return out


def phase_bytes(n: int, L: int, G: int, psi_bytes: int) -> dict:
    """Algorithmic bytes of the three passes of one phase retrieval product D v (complex FP64 = 16 B,
    real FP64 = 8 B, a waveform entry psi_bytes: 1 as a dictionary code, 16 whole), each array counted
    once per pass: column pass v, psi, Y; row pass Y in, c, Y out; inverse column pass Y, psi, v, the G
    group sums."""
    return {"colfwd": 16 * n + (16 + psi_bytes) * L * n, "row": 40 * L * n,
            "colinv": (16 + psi_bytes) * L * n + 16 * n * (1 + G)}


PHASE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "phase_traffic_cdp_1m_fp64.json")


def phase_traffic() -> dict:
    """Counted HBM bytes per launch of the three passes, when the profile matches the current source."""
    try:
        doc = json.load(open(PHASE_TRAFFIC_FILE))
    except (OSError, ValueError):
        return {}
    with open(os.path.join(ROOT, "paper_1912_02949_amd", "csrc", "scg_phase.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    if doc.get("phase_source_sha") != sha:
        return {}
    return {"colfwd": doc["passes"]["k_pr_colfwd"]["hbm_bytes_per_launch"],
            "row": doc["passes"]["k_pr_row<0>"]["hbm_bytes_per_launch"],
            "colinv": doc["passes"]["k_pr_colinv"]["hbm_bytes_per_launch"]}


def phase_accuracy(torch, sizes, T: int) -> list:
    """Relative error of the rounded signal (Section 7.3.3) against solve time, at checkpoints.
    The reconstruction and rounding at a checkpoint are not part of the solve time."""
    import synth.phase as sp
    from paper_1912_02949_amd.api import PhaseParams, PhaseRetrieval
    out = []
    for n in sizes:
        k = int(round(math.log10(n)))
        inst = sp.coded_diffraction(n, sp.PHASE_SEEDS.get(k, 0x5C6A5000 + k), L=12)
        st = torch.cuda.Stream()   # a non-null stream: iterations replay captured graphs
        s = PhaseRetrieval(inst.psi, inst.b, PhaseParams(R=5, T=T, seed=0x5C6A5000 + k), stream=st)
        pts, t_done, solve_s = [], 0, 0.0
        marks = sorted({c for c in (50, 100, 200, 300, 500, 700, 1000, 1500, 2000, 3000, 4000, 5000, 7000,
                                    10000, 15000, 20000) if c <= T} | {T})
        for cp in marks:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(cp - t_done)
            s.synchronize()
            solve_s += time.perf_counter() - t0
            t_done = cp
            if s.get_state()["tau"] == 0.0:
                rel = 1.0          # X = 0 so far (every H was 0): the rounded signal is 0
            else:
                U, lam, _ = s.reconstruct()
                _, rel = s.round(U, lam, inst.chi)
            pts.append({"t": cp, "rel_error": rel, "solve_s": solve_s})
            progress(f"phase accuracy n={n} t={cp}: relative error {rel:.3e}, {solve_s:.2f} s")
            if rel < 1e-3:
                break
        out.append({"n": n, "points": pts})
        del s
    return out


def phase_sweep(torch) -> list:
    """Per-pass times of the n = 10^6 product for several column-tile widths and waveform groups."""
    import synth.phase as sp
    from paper_1912_02949_amd.api import PhaseParams, PhaseRetrieval
    n, L = 10 ** 6, 12
    inst = sp.coded_diffraction(n, sp.PHASE_SEEDS[6], L=L)
    rows = []
    for tc, G in ((16, 4), (16, 1), (16, 2), (16, 3), (16, 6), (16, 12), (8, 4), (4, 4)):
        s = PhaseRetrieval(inst.psi, inst.b, PhaseParams(R=5, T=2, seed=1, tile_cols=tc, mask_groups=G))
        tm = s.time_apply(20)
        info = s.summary()
        rows.append({"tile_cols": info["tile_cols"], "mask_groups": info["mask_groups"],
                     **{k: round(v * 1e3, 1) for k, v in tm.items()}})
        progress(f"phase sweep {rows[-1]}")
        del s
    return rows


def phase_leg(torch, T: int, groups: int = 0) -> dict:
    """Phase retrieval at the paper's largest size (n = 10^6, 12 coded diffraction patterns, R = 5,
    alpha = 3n, FP64): T iterations timed as a whole, and the three passes of the D v product."""
    import synth.phase as sp
    from paper_1912_02949_amd.api import PhaseParams, PhaseRetrieval
    n, L = 10 ** 6, 12
    inst = sp.coded_diffraction(n, sp.PHASE_SEEDS[6], L=L)
    prm = PhaseParams(R=5, T=T, seed=sp.PHASE_SEEDS[6], mask_groups=groups)
    s = PhaseRetrieval(inst.psi, inst.b, prm, stream=torch.cuda.Stream())   # graph replays
    info = s.summary()
    tm = s.time_apply(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run()
    s.synchronize()
    dt = time.perf_counter() - t0
    lg = s.log()
    qs = [int(q) for q in lg["q"]]
    products = sum(q + 1 for q in qs)      # q Lanczos products and the measurement pass per iteration
    byt = phase_bytes(n, L, info["mask_groups"], 1 if info["mask_codes"] else 16)
    passes = {}
    counted = phase_traffic() if (info["n1"], info["n2"], info["mask_groups"]) == (250, 4000, 1) else {}
    for key in ("colfwd", "row", "colinv"):
        gbs = byt[key] / (tm[key] * 1e-3) / 1e9
        passes[key] = {"avg_us": tm[key] * 1e3, "algorithmic_bytes": byt[key], "achieved_GBps": gbs,
                       "frac_of_hbm_peak": gbs / HBM_PEAK_GBS, "traffic": counted.get(key)}
    tot = sum(byt.values())
    out = {"workload": "phase retrieval SDP, coded diffraction patterns, n = 10^6, L = 12 (d = 12n), R = 5, "
                       "alpha = 3n, FP64 complex, first %d iterations" % T,
           "n": n, "L": L, "split": [info["n1"], info["n2"]], "tile_cols": info["tile_cols"],
           "mask_groups": info["mask_groups"], "waveform_codes": bool(info["mask_codes"]), "iters_per_s": T / dt, "ms_per_iteration": 1e3 * dt / T,
           "lanczos_steps": int(sum(qs)), "products_per_s": products / dt,
           "product_us": tm["apply"] * 1e3, "passes": passes,
           "product_algorithmic_GBps": tot / (tm["apply"] * 1e-3) / 1e9,
           "infeasibility_rel": s.summary()["infeasibility"] / math.sqrt(float((inst.b * inst.b).sum()))}
    del s
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--T", type=int, default=2000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-other-workloads", action="store_true")
    ap.add_argument("--batched-T", type=int, default=1000)
    ap.add_argument("--no-storage-optimal", action="store_true")
    ap.add_argument("--phase-T", type=int, default=30, help="iterations of the phase retrieval leg (0: skip)")
    ap.add_argument("--phase-only", action="store_true", help="only the phase retrieval leg")
    ap.add_argument("--phase-groups", type=int, default=0,
                    help="waveform groups of the phase retrieval leg (0: tuned at init; the counter passes fix 1, "
                         "since timing under counter collection is not representative)")
    ap.add_argument("--phase-accuracy", type=str, default="",
                    help="only the relative error of the rounded signal against solve time, for these comma-separated n")
    ap.add_argument("--phase-accuracy-T", type=int, default=5000)
    ap.add_argument("--phase-sweep", action="store_true",
                    help="only per-pass times of the phase retrieval product over tile widths and waveform groups")
    ap.add_argument("--probe-workload", type=int, default=2, choices=(2, 3, 5),
                    help="workload of --traffic-probe")
    ap.add_argument("--probe-precision", default="fp32", choices=("fp32", "fp64"),
                    help="precision of --traffic-probe")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only the SpMV kernel, 20 launches in each shape the autotuner chooses from (lanes per "
                         "row x workgroups), for rocprofv3 --pmc, plus a 256 MiB device copy whose counters "
                         "calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU path is a design "
                                   "(row partition with halo exchange) and is not built"}), flush=True)
        sys.exit(2)

    import torch
    import synth
    from paper_1912_02949_amd import Params

    inst = synth.config_instance(2)
    T = args.T
    qs = q_schedule(T, inst.n)
    p32 = Params(R=10, T=T, seed=synth.CONFIG_SEEDS[2], precision="fp32")
    p64 = Params(R=10, T=T, seed=synth.CONFIG_SEEDS[2], precision="fp64")

    if args.traffic_probe:
        kp = args.probe_workload
        pinst = inst if kp == 2 else synth.config_instance(kp)
        pqs = qs if kp == 2 else q_schedule(100, pinst.n)
        shapes = []
        for lanes, grid, seg in PROBE_SHAPES[kp]:
            prm = Params(R=10, T=100 if kp != 2 else T, seed=synth.CONFIG_SEEDS[kp], precision=args.probe_precision,
                         autotune=0, segments=seg, spmv_lanes=lanes, spmv_grid=grid)
            sp = Solve(pinst, prm, torch)
            sp.init()
            sp.lib.sketchycgal_step(sp.ctx, 2)
            ms = C.c_double()
            sp.lib.sketchycgal_time_spmv(sp.ctx, 20, C.byref(ms))
            summ = sp.summary()
            sp.close()
            shapes.append({"lanes": lanes, "workgroups": summ["spmv_grid"], "segments": summ["spmv_segments"],
                           "spmv_avg_us": ms.value * 1e3,
                           # two iterations' Lanczos products, then the step-0 product time_spmv forms first
                           "lanczos_launches_before_timing": sum(pqs[:2]) + 1})
            progress(f"probe lanes={lanes} workgroups={summ['spmv_grid']} segments={seg}: {ms.value * 1e3:.1f} us")
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"workload": kp, "precision": args.probe_precision, "shapes": shapes, "copy_bytes": 4 * a.numel(),
                          "kernel_source_sha": kernel_source_sha()}), flush=True)
        return

    if args.phase_accuracy:
        sizes = [int(float(v)) for v in args.phase_accuracy.split(",")]
        print(json.dumps({"phase_accuracy": phase_accuracy(torch, sizes, args.phase_accuracy_T)}), flush=True)
        return
    if args.phase_sweep:
        print(json.dumps({"phase_sweep": phase_sweep(torch)}), flush=True)
        return
    if args.phase_only:
        ph = phase_leg(torch, args.phase_T, args.phase_groups)
        # a 256 MiB device copy: calibrates FETCH_SIZE / WRITE_SIZE when this runs under rocprofv3 --pmc
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"phase_retrieval": ph, "copy_bytes": 4 * a.numel()}), flush=True)
        return

    norm_b = math.sqrt(float((inst.b * inst.b).sum()))
    # headline: the plain-FP64 form (the paper's precision), whole solves of workload 2
    s64 = Solve(inst, p64, torch)
    dt64 = timed(s64, args.steps, args.warmup, torch)
    progress(f"fp64 solves: {1e3 * dt64 / args.steps:.1f} ms each")
    sum64 = s64.summary()
    last64 = s64.record()
    first64 = s64.record(0)
    spmv64 = spmv_roofline(s64, inst, "fp64", 100, 2)
    s64.close()
    del s64

    # FP32-stream form of the same workload: one warm-up and one timed solve
    s32 = Solve(inst, p32, torch)
    dt32 = timed(s32, 1, 1, torch)
    progress(f"fp32 solve: {1e3 * dt32:.1f} ms")
    sum32 = s32.summary()
    infeas32 = s32.infeasibility_log()
    last32 = s32.record()
    first32 = s32.record(0)
    cut_w, cut_j, cut_s = s32.round_cut()
    spmv32 = spmv_roofline(s32, inst, "fp32", 200, 2)
    ws32 = s32.nbytes
    s32.close()
    del s32
    # the same FP64 solve with its products summed in another order (another SpMV shape): how far rounding
    # alone moves the whole-run result, the yardstick for the FP32-versus-FP64 difference
    alt_lanes = 2 if spmv64["lanes_per_row"] != 2 else 4
    s64b = Solve(inst, Params(R=10, T=T, seed=synth.CONFIG_SEEDS[2], precision="fp64", autotune=0,
                              spmv_lanes=alt_lanes), torch)
    timed(s64b, 1, 0, torch)
    sum64b = s64b.summary()
    s64b.close()
    del s64b
    progress("fp64 solve with another summation order done")
    # speedup at equal final infeasibility: the FP32 solve stopped at the first iteration whose
    # ||diag X - b|| is at most the FP64 solve's final value, timed as a whole solve
    equal = None
    hit = next((i + 1 for i, v in enumerate(infeas32) if v <= sum64["infeasibility"]), None)
    if hit is not None:
        s_eq = Solve(inst, Params(R=10, T=hit, seed=synth.CONFIG_SEEDS[2], precision="fp32"), torch)
        dt_eq = timed(s_eq, 1, 0, torch)
        s_eq.close()
        del s_eq
        equal = {"fp32_iterations": hit, "fp32_ms": 1e3 * dt_eq, "fp64_iterations": T,
                 "fp64_ms": 1e3 * dt64 / args.steps, "speedup_fp32_vs_fp64": (dt64 / args.steps) / dt_eq}
        progress(f"fp32 reaches the fp64 final infeasibility at t = {hit}: {1e3 * dt_eq:.1f} ms")

    # storage-optimal mode: three Lanczos vectors (basis regenerated by a second sweep) and
    # Omega regenerated from its counters; same arithmetic, so the same iterates
    storage = None
    if not args.no_storage_optimal:
        pso = Params(R=10, T=T, seed=synth.CONFIG_SEEDS[2], precision="fp32", basis_mode=1, omega_mode=1,
                     autotune=0, segments=spmv32["column_segments"], spmv_lanes=spmv32["lanes_per_row"],
                     spmv_grid=spmv32["workgroups"] if spmv32["workgroups"] <= 2048 else 0)
        sso = Solve(inst, pso, torch)
        dtso = timed(sso, 1, 0, torch)
        sumso = sso.summary()
        sso.close()
        storage = {
            "value": T / dtso, "unit": "CGAL iters/s", "ms_per_step": 1e3 * dtso,
            "workspace_bytes": sso.nbytes, "workspace_bytes_stored_mode": ws32,
            "workspace_ratio": sso.nbytes / ws32,
            "objective_equals_stored_mode": sumso["objective"] == sum32["objective"],
        }
        del sso
        progress(f"storage-optimal fp32 solve: {1e3 * dtso:.1f} ms")
    gref = gather_reference(torch, inst.n, inst.nnz - inst.n)
    copy_gbs = copy_ceiling(torch)

    batched = None if args.no_batched else batched_leg(torch, args.batched_T, True)
    others, w1 = None, None
    if not args.no_other_workloads:
        others = {}
        for k, name, Tk in ((5, "random geometric, n=2^23, ~2.0e7 edges, weights U[0.5,1.5]", 500),
                            (3, "Chung-Lu power law (exponent 2.5), n=2^22, ~3.4e7 edges, unit weights", 1000)):
            ik = synth.config_instance(k)
            others[f"workload_{k}"] = {"graph": name, "n": ik.n, "nnz_offdiag": ik.nnz - ik.n,
                                       "fp32": solve_leg(torch, k, ik, "fp32", Tk)}
            if k == 5:   # the FP64 product of the HBM-bound workload, the headline's precision
                others["workload_5"]["fp64_spmv"] = spmv_leg(torch, k, ik, "fp64")
            del ik
            progress(f"workload {k}: {others[f'workload_{k}']['fp32']['iters_per_s']:.2f} CGAL iterations/s")
        w1 = workload1_leg(torch)
        progress("workload 1 done")
    phase = None
    if args.phase_T > 0:
        phase = phase_leg(torch, args.phase_T)
        progress(f"phase retrieval n=10^6: {phase['ms_per_iteration']:.1f} ms per iteration")
    cpu = None if args.no_cpu else cpu_baseline(inst, T, args.cpu_seconds)

    # the roofline object: the Lanczos SpMV of the largest workload (its working set far exceeds the
    # 256 MB last-level cache, so the bandwidth is HBM bandwidth), else the headline workload's FP32 kernel
    rl_src, rl_name = spmv32, "workload 2 (torus, n=2^20) Lanczos SpMV, FP32"
    if others is not None:
        rl_src, rl_name = others["workload_5"]["fp32"]["spmv"], "workload 5 (random geometric, n=2^23) Lanczos SpMV, FP32"
    roofline = {
        "bound": "hbm",
        "kernel": rl_src["kernel"] + " (" + rl_name + ")",
        "achieved": rl_src["achieved_GBps"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": rl_src["achieved_GBps"] / HBM_PEAK_GBS,
        "traffic": rl_src["traffic"],
        "algorithmic_bytes_per_launch": rl_src["algorithmic_bytes_per_product"],
        "avg_launch_us": rl_src["avg_product_us"],
        "copy_ceiling_GBps": copy_gbs,
        "frac_of_copy_ceiling": rl_src["achieved_GBps"] / copy_gbs,
    }
    if others is not None and "fp64_spmv" in others["workload_5"]:
        r64 = others["workload_5"]["fp64_spmv"]
        roofline["fp64"] = {"kernel": r64["kernel"] + " (workload 5 Lanczos SpMV, FP64)",
                            "achieved": r64["achieved_GBps"], "frac": r64["achieved_GBps"] / HBM_PEAK_GBS,
                            "traffic": r64["traffic"],
                            "algorithmic_bytes_per_launch": r64["algorithmic_bytes_per_product"],
                            "avg_launch_us": r64["avg_product_us"]}
    value = args.steps * T / dt64
    out = {
        "metric": "CGAL iters/sec + Lanczos SpMV HBM GB/s (% peak), FP32/batched vs FP64 plain",
        "value": value,
        "unit": "CGAL iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt64 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "MaxCut SDP plain FP64, 1024x1024 torus + 2n random long-range edges, weights +-1, "
                        "n=1048576, R=10, T=%d, q_t=ceil(t^(1/4) ln n)" % T,
            "n": inst.n, "nnz_offdiag": inst.nnz - inst.n, "R": 10, "T": T, "lanczos_steps_total": sum(qs),
        },
        "roofline": roofline,
        "result_fp64": {"objective": sum64["objective"], "infeasibility_rel": sum64["infeasibility"] / norm_b,
                        "eigen_residual_scaled": last64["resid"], "spmv": spmv64,
                        "objective_rel_diff_other_summation_order": abs(sum64b["objective"] - sum64["objective"]) /
                        abs(sum64["objective"]),
                        "other_summation_order_lanes": alt_lanes},
        "fp32_stream": {
            "value": T / dt32, "unit": "CGAL iters/s", "ms_per_step": 1e3 * dt32,
            "speedup_vs_fp64": (T / dt32) / value, "equal_infeasibility": equal,
            "objective": sum32["objective"], "infeasibility_rel": sum32["infeasibility"] / norm_b,
            "eigen_residual_scaled": last32["resid"], "xi_scaled": last32["xi"],
            # whole runs follow rounding: the FP64 solve with another summation order above is the yardstick
            "objective_rel_diff_vs_fp64": abs(sum32["objective"] - sum64["objective"]) / abs(sum64["objective"]),
            # from the same (zero) state: the per-iteration FP32-stream error
            "first_iteration_objective_rel_diff_vs_fp64": abs(first32["p"] - first64["p"]) / abs(first64["p"]),
            "rounded_cut_weight": cut_w, "rounded_cut_column": cut_j, "rounding_ms": 1e3 * cut_s,
            "cut_over_sdp_objective": cut_w / -sum32["objective"],
            "spmv": spmv32,
            "gathers_over_uniform_reference": spmv32["gathers_per_s"] / gref,
            "uniform_gather_reference_per_s": gref,
        },
        "storage_optimal_fp32": storage,
        "batched": batched,
        "other_workloads": others,
        "workload_1": w1,
        "phase_retrieval": phase,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
