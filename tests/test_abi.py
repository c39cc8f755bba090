"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/sketchycgal.h, and rejects bad parameters before any
device work."""
import ctypes as C
import math
import os
import re

import pytest

from paper_1912_02949_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "sketchycgal.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b((?:scg|sketchycgal)_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = _lib.load()
    names = _declared()
    assert "sketchycgal_init" in names and "sketchycgal_step" in names and "sketchycgal_reconstruct" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTS)


def test_default_params_are_the_papers():
    lib = _lib.load()
    p = _lib.scg_params()
    lib.scg_default_params(C.byref(p))
    assert p.beta0 == 1.0 and math.isinf(p.K) and p.scale == 1 and p.trace_correct == 1
    assert p.q_mode == 0 and p.reorth == 0 and p.precision == _lib.SCG_FP64


def _ws(**kw):
    lib = _lib.load()
    p = _lib.scg_params()
    lib.scg_default_params(C.byref(p))
    n = kw.pop("n", 100)
    nnz = kw.pop("nnz", 500)
    for k, v in kw.items():
        setattr(p, k, v)
    out = C.c_size_t()
    return lib.scg_workspace_size(C.byref(p), n, nnz, C.byref(out)), out.value


def test_workspace_size_and_validation():
    st, b = _ws()
    assert st == _lib.SCG_OK and b > 0
    st2, b2 = _ws(precision=_lib.SCG_FP32_STREAM)
    assert st2 == _lib.SCG_OK and b2 < b
    bad = [dict(R=0), dict(R=33), dict(n=5, R=6), dict(T=0), dict(beta0=0.0), dict(beta0=-1.0), dict(K=-1.0),
           dict(q_mode=2), dict(q_mode=1, q_fixed=0), dict(reorth=3), dict(reorth=-1), dict(precision=7), dict(n=0),
           dict(spmv_lanes=3), dict(spmv_lanes=64), dict(spmv_lanes=1, segments=2), dict(spmv_grid=-1), dict(spmv_grid=4096),
           dict(q_mode=1, q_fixed=600, n=10_000), dict(basis_mode=2), dict(basis_mode=-1), dict(omega_mode=2),
           dict(basis_mode=1, reorth=2), dict(trace_mode=2), dict(trace_mode=-1), dict(constraint_set=3), dict(constraint_set=-1),
               dict(batch_kernel=1)]
    for kw in bad:
        st, _ = _ws(**dict(kw))
        assert st == _lib.SCG_EINVAL, kw


def test_storage_optimal_modes_shrink_the_workspace():
    # Section 4.2: regenerating the Lanczos basis keeps three n-vectors (plus an
    # FP64 accumulator) instead of q + 1; a regenerated Omega drops the n x R array.
    n, R, T = 1_000_000, 10, 100
    q_max = max(math.ceil(t ** 0.25 * math.log(n)) for t in range(1, T + 1))
    st0, b0 = _ws(n=n, nnz=5 * n, R=R, T=T)
    st1, b1 = _ws(n=n, nnz=5 * n, R=R, T=T, basis_mode=1)
    st2, b2 = _ws(n=n, nnz=5 * n, R=R, T=T, omega_mode=1)
    st3, b3 = _ws(n=n, nnz=5 * n, R=R, T=T, basis_mode=1, omega_mode=1)
    assert st0 == st1 == st2 == st3 == _lib.SCG_OK
    slack = 16 * 256
    assert b0 - b1 >= 8 * n * (q_max + 1 - 3) - 8 * n - slack
    assert b0 - b2 >= 8 * n * R - slack
    assert b0 - b3 >= (b0 - b1) + (b0 - b2) - slack
    # with the regenerated basis a larger q costs O(q) words of partial sums, not q n-vectors
    st4, b4 = _ws(n=n, nnz=5 * n, R=R, T=T, basis_mode=1, omega_mode=1, q_mode=1, q_fixed=120)
    st5, b5 = _ws(n=n, nnz=5 * n, R=R, T=T, q_mode=1, q_fixed=120)
    assert st4 == st5 == _lib.SCG_OK
    assert b5 - b0 >= 8 * n * (120 - q_max)
    # ... and the same number of bytes at twice the size
    n2 = 2 * n
    _, c3 = _ws(n=n2, nnz=5 * n2, R=R, T=T, basis_mode=1, omega_mode=1, q_mode=1, q_fixed=44)
    _, c4 = _ws(n=n2, nnz=5 * n2, R=R, T=T, basis_mode=1, omega_mode=1, q_mode=1, q_fixed=120)
    _, d3 = _ws(n=n, nnz=5 * n, R=R, T=T, basis_mode=1, omega_mode=1, q_mode=1, q_fixed=44)
    assert abs((c4 - c3) - (b4 - d3)) <= slack


def test_chunk_layout_reservation():
    # the quad-chunk layout: column words for chunks of 64 quads, each row
    # padded to whole quads: at most nnz/4 + n quads, every chunk but the last
    # holding at least 33 of them; the entry-chunk layout (stored values):
    # chunks of 256 entries, a row taking max(1, d) <= 64 of them, every chunk
    # but the last holding at least 193: words for the larger count, values
    # (FP64 here) for the entry layout only, which stored values force; neither
    # when a row-block product is forced
    n, nnz = 1_000_000, 9_000_000
    st0, b_auto = _ws(n=n, nnz=nnz)
    st1, b_rows = _ws(n=n, nnz=nnz, spmv_lanes=2)
    st2, b_vals = _ws(n=n, nnz=nnz, matrix_format=1)
    st3, b_quad = _ws(n=n, nnz=nnz, spmv_lanes=1)
    assert st0 == st1 == st2 == st3 == _lib.SCG_OK
    chunks = (nnz // 4 + n + 1) // 33 + 2
    echunks = (nnz + n) // 193 + 2
    assert chunks > echunks
    # with the eight concurrent segments possible (autotuned, n >= 2^18): their entry-chunk
    # layout too, (nnz + 8 n) / 193 + 16 chunks of words and values, and the long segments
    # (descriptors for at most nnz / 65 + 8 of them, their words and values)
    xc = (nnz + 8 * n) // 193 + 16
    nlw = nnz + 4 * (nnz // 65 + 8)   # long entries, each segment padded to a 16-byte quad
    xbytes = 256 * 4 * xc + 8 * 256 * xc + 8 * xc + 16 * (nnz // 65 + 8) + 4 * nlw + 8 * nlw
    assert 0 <= (b_auto - b_rows) - (256 * 4 * chunks + 8 * 256 * echunks + 8 * chunks + xbytes) <= 9 * 256
    assert 0 <= (b_vals - b_rows) - (256 * 4 * echunks + 8 * 256 * echunks + 8 * echunks + xbytes) <= 9 * 256
    # the forced chunk products never split columns: no room for eight segments' row
    # pointers, row-block descriptors, concurrent partial sums and their chunks (FP64, ld = n here)
    seg = 7 * 4 * (n + 1) + 7 * 8 * (n + 2) + 8 * 8 * n
    assert abs((b_auto - b_quad) - seg - xbytes) <= 9 * 256   # each region is rounded up to 256 bytes


def test_box_constraint_set_adds_two_vectors():
    n = 100_000
    st0, b0 = _ws(n=n, nnz=6 * n)
    st1, b1 = _ws(n=n, nnz=6 * n, constraint_set=1, trace_mode=1)
    assert st0 == st1 == _lib.SCG_OK
    assert 16 * n <= b1 - b0 <= 16 * n + 2 * 256
    lib = _lib.load()
    assert lib.sketchycgal_set_constraints(None, None, None) == _lib.SCG_EINVAL
    assert lib.sketchycgal_set_ball(None, 1.0) == _lib.SCG_EINVAL


def test_init_rejects_null_and_misaligned_arguments():
    lib = _lib.load()
    p = _lib.scg_params()
    lib.scg_default_params(C.byref(p))
    ctx = C.c_void_p()
    # NULL arrays and a misaligned workspace are rejected before any HIP call
    assert lib.sketchycgal_init(C.byref(ctx), C.byref(p), 10, 20, None, None, None, None, None, None, 0,
                                None) == _lib.SCG_EINVAL
    assert lib.sketchycgal_init(C.byref(ctx), C.byref(p), 10, 20, 8, 8, 8, 8, None, 12345, 1 << 30,
                                None) == _lib.SCG_EINVAL
    assert ctx.value is None
    assert lib.sketchycgal_step(None, 1) == _lib.SCG_EINVAL
    assert lib.scg_status_string(_lib.SCG_ENOMEM) == b"workspace too small"


def _bws(sizes, nnz=1000, **kw):
    import numpy as np
    lib = _lib.load()
    p = _lib.scg_params()
    lib.scg_default_params(C.byref(p))
    p.R = 8
    for k, v in kw.items():
        setattr(p, k, v)
    ns = np.ascontiguousarray(np.asarray(sizes, dtype=np.int64))
    out = C.c_size_t()
    return lib.scg_batch_workspace_size(C.byref(p), len(ns), ns.ctypes.data, nnz, C.byref(out)), out.value


def test_batch_workspace_size_and_validation():
    st, b = _bws([200, 5000, 20000])
    assert st == _lib.SCG_OK and b > 0
    st2, b2 = _bws([200, 5000, 20000], precision=_lib.SCG_FP32_STREAM)
    assert st2 == _lib.SCG_OK and b2 < b
    st3, b3 = _bws([200, 5000, 20000, 300])
    assert st3 == _lib.SCG_OK and b3 > b
    for sizes, kw in [([200, 5], {}), ([], {}), ([100], dict(reorth=3)), ([100], dict(T=0)),
                      ([1000], dict(q_mode=1, q_fixed=129)), ([100], dict(precision=3)), ([100], dict(R=33)),
                      ([100], dict(basis_mode=1)), ([100], dict(omega_mode=1)), ([100], dict(trace_mode=1)),
                      ([100], dict(constraint_set=1)), ([100], dict(batch_kernel=4)), ([100], dict(batch_kernel=-1))]:
        st, _ = _bws(sizes, **kw)
        assert st == _lib.SCG_EINVAL, (sizes, kw)


def test_batch_init_rejects_null_and_misaligned_arguments():
    import numpy as np
    lib = _lib.load()
    p = _lib.scg_params()
    lib.scg_default_params(C.byref(p))
    p.R = 8
    ns = np.array([100, 200], dtype=np.int64)
    ctx = C.c_void_p()
    assert lib.sketchycgal_batch_init(C.byref(ctx), C.byref(p), 2, ns.ctypes.data, 900, None, None, None, None,
                                      None, 0, None) == _lib.SCG_EINVAL
    assert lib.sketchycgal_batch_init(C.byref(ctx), C.byref(p), 2, ns.ctypes.data, 900, 8, 8, 8, 8, 12345,
                                      1 << 30, None) == _lib.SCG_EINVAL
    assert ctx.value is None
    assert lib.sketchycgal_batch_step(None, 1) == _lib.SCG_EINVAL
    assert lib.sketchycgal_batch_set_beta0(None, None) == _lib.SCG_EINVAL
