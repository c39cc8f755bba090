"""The ABI from plain C: tests/c/abi_cycle.c (built by __graft_entry__.build())
allocates every device buffer itself, solves the 9-cycle MaxCut SDP through
sketchycgal_init / step / summary / reconstruct / round and checks the
closed-form value (9/2)(1 + cos(pi/9)), the reconstruction's trace and the
rounded cut; tests/c/abi_phase.c recovers a 64-dimensional signal from coded
diffraction measurements through scg_pr_* (adjoint identity between measure and
apply, relative error below 1e-2, tr X within 1% of the signal energy)."""
import os
import subprocess
import sys

import pytest

from gpu_util import need_gpu, announce

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "abi_cycle")


def test_plain_c_consumer_solves_the_nine_cycle():
    need_gpu()
    assert os.path.exists(EXE), f"{EXE} is missing: build it with __graft_entry__.build()"
    announce("plain C consumer of the ABI")
    out = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(out.stdout, out.stderr, file=sys.stderr, flush=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "abi_cycle: SDP value" in out.stdout


EXE_PHASE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "abi_phase")


def test_plain_c_consumer_recovers_a_phase_retrieval_signal():
    need_gpu()
    assert os.path.exists(EXE_PHASE), f"{EXE_PHASE} is missing: build it with __graft_entry__.build()"
    announce("plain C consumer of the phase retrieval ABI")
    out = subprocess.run([EXE_PHASE], capture_output=True, text=True, timeout=120)
    print(out.stdout, out.stderr, file=sys.stderr, flush=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "abi_phase: adjoint identity" in out.stdout
