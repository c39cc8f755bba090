"""scg_round_csr, the rounding entry point that allocates nothing, against
sketchycgal_round on the same reconstruction, through the C ABI.

Two calls in a row share the library's static scratch array: a larger
problem, then a smaller one (fewer rows, fewer columns of U), each compared
with the context-based rounding of an FP64 solve (weights within 1e-12
relative, the same heaviest column, the same indicator).  Malformed input is
rejected with SCG_EINVAL without the kernel reading outside the arrays.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from gpu_util import need_gpu, make_solver, announce

pytestmark = pytest.mark.gpu


def _round_csr(inst, U, R, lib, row_ptr=None, col=None):
    dev = torch.device("cuda:0")
    rp = torch.as_tensor(inst.row_ptr if row_ptr is None else row_ptr).to(dev)
    cl = torch.as_tensor(inst.col if col is None else col).to(dev)
    vl = torch.as_tensor(inst.val).to(dev)
    Ud = U.t().contiguous().reshape(-1).to(dev, torch.float64)
    chi = torch.empty(inst.n, dtype=torch.int8, device=dev)
    w = (C.c_double * R)()
    best = C.c_int32()
    st = lib.scg_round_csr(inst.n, inst.nnz, rp.data_ptr(), cl.data_ptr(), vl.data_ptr(), R, Ud.data_ptr(),
                           chi.data_ptr(), w, C.byref(best), torch.cuda.current_stream().cuda_stream)
    return st, np.array(w[:]), best.value, chi.cpu().numpy()


def _case(inst, R, seed):
    s = make_solver(inst, R=R, T=30, seed=seed, precision="fp64")
    s.run()
    U, lam, err = s.reconstruct()
    return s, U


def test_round_csr_matches_context_rounding_twice():
    need_gpu()
    from paper_1912_02949_amd import _lib
    lib = _lib.load()
    big = synth.laplacian_instance(synth.torus_longrange(96, 7))      # n = 9216, weights +-1
    small = synth.config_instance(1)                                    # n = 800, unit weights
    for inst, R, seed in ((big, 12, 5), (small, 6, 9)):
        announce(f"round_csr n={inst.n} R={R}")
        s, U = _case(inst, R, seed)
        w_ref, b_ref, chi_ref = s.round_cut(U)
        st, w, b, chi = _round_csr(inst, U, R, lib)
        assert st == _lib.SCG_OK
        assert np.abs(w - w_ref).max() <= 1e-12 * np.abs(w_ref).max()
        assert b == b_ref
        assert np.array_equal(chi, chi_ref.cpu().numpy())


def test_round_csr_rejects_malformed_input():
    need_gpu()
    from paper_1912_02949_amd import _lib
    lib = _lib.load()
    inst = synth.laplacian_instance(synth.cycle(9))
    U = torch.ones(9, 3, dtype=torch.float64)
    col = inst.col.copy()
    col[5] = 9                                   # column outside [0, n)
    st, _, _, _ = _round_csr(inst, U, 3, lib, col=col)
    assert st == _lib.SCG_EINVAL
    rp = inst.row_ptr.copy()
    rp[4] = rp[6]                                # row pointers not monotone
    st, _, _, _ = _round_csr(inst, U, 3, lib, row_ptr=rp)
    assert st == _lib.SCG_EINVAL
    for R in (0, 33):
        st = lib.scg_round_csr(9, inst.nnz, 0, 0, 0, R, 0, None, (C.c_double * 1)(), C.byref(C.c_int32()), None)
        assert st == _lib.SCG_EINVAL
    # a well-formed call after the rejected ones
    st, w, b, chi = _round_csr(inst, U, 3, lib)
    assert st == _lib.SCG_OK and np.all(w == w[0]) and b == 0
