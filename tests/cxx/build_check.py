"""Builds tests/cxx/tfcp_check (host code only, with hipcc) against the
in-tree libtwofold_hip.so: the check program of the C++ convenience header
include/twofold.hpp.  Run by __graft_entry__.build() and by the tests when the
program is missing."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
EXE = os.path.join(HERE, "tfcp_check")


def build(verbose=False):
    pkg = os.path.join(ROOT, "paper_1502_05216_amd")
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    cmd = [hipcc, "-O2", "-std=c++17", os.path.join(HERE, "tfcp_check.cpp"), "-o", EXE,
           "-L" + pkg, "-ltwofold_hip", "-Wl,-rpath,$ORIGIN/../../paper_1502_05216_amd"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, capture_output=not verbose)
    return EXE


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
