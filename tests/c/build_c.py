"""Compile the plain-C consumers of the ABI (tests/c/abi_cycle.c, tests/c/abi_phase.c) against the built library."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
EXE = os.path.join(HERE, "abi_cycle")


EXE_PHASE = os.path.join(HERE, "abi_phase")


def build_c_example(verbose: bool = False) -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    pkg = os.path.join(ROOT, "paper_1912_02949_amd")
    for src, exe in (("abi_cycle.c", EXE), ("abi_phase.c", EXE_PHASE)):
        cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
               "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"),
               os.path.join(HERE, src), "-o", exe,
               "-L", pkg, "-lsketchycgal", "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm",
               "-Wl,-rpath,$ORIGIN/../../paper_1912_02949_amd", "-Wl,-rpath," + os.path.join(rocm, "lib")]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    return EXE


if __name__ == "__main__":
    print(build_c_example(verbose=True))
