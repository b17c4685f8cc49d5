"""Builds and runs the gfx950 instruction-rate and reciprocal-accuracy
benchmark (isa_rates.hip): the figures behind the issue-slot model of the
evaluation kernels.

    python -m paper_1606_06508_amd.isa_rates          # build (if needed) and run
"""
import os
import subprocess
import sys

from .build import ARCH, HIPCC

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "isa_rates.hip")
EXE = os.path.join(HERE, "_build", "isa_rates")
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(force=False):
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    if force or not os.path.exists(EXE) or os.path.getmtime(EXE) < os.path.getmtime(SRC):
        res = subprocess.run([HIPCC, *FLAGS, SRC, "-o", EXE], capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed for {SRC}:\n{res.stderr}")
    return EXE


def main():
    exe = build()
    return subprocess.run([exe]).returncode


if __name__ == "__main__":
    sys.exit(main())
