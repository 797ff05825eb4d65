"""Builds tests/cxx/tfcp_check (host code only, with hipcc) against the
in-tree libtwofold_hip.so: the check program of the C++ convenience header
include/twofold.hpp; and tests/cxx/libtfcp_device.so (hipcc, gfx950), the check
library of the device value type of include/twofold_device.hpp.  Run by
__graft_entry__.build() and by the tests when they are missing."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
EXE = os.path.join(HERE, "tfcp_check")
DEVLIB = os.path.join(HERE, "libtfcp_device.so")


def build(verbose=False):
    pkg = os.path.join(ROOT, "paper_1502_05216_amd")
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    cmd = [hipcc, "-O2", "-std=c++17", os.path.join(HERE, "tfcp_check.cpp"), "-o", EXE,
           "-L" + pkg, "-ltwofold_hip", "-Wl,-rpath,$ORIGIN/../../paper_1502_05216_amd"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, capture_output=not verbose)
    build_device(verbose)
    return EXE


def build_device(verbose=False):
    """The device value type's check library, with the library's own flags."""
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    cmd = [hipcc, "--offload-arch=" + os.environ.get("TF_OFFLOAD_ARCH", "gfx950"), "-O3",
           "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-gpu-flush-denormals-to-zero",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "tfcp_device.hip"),
           "-o", DEVLIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(DEVLIB + ".tmp", DEVLIB)
    return DEVLIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
