"""The C++ convenience header include/twofold.hpp (the paper's C++ interface:
one function name for float and double, standard-like exp/expm1/log/log1p,
for twofold arrays), through the compiled check program tests/cxx/tfcp_check:

* without a GPU: every overload validates its arguments before any GPU work
  (n = 0 -> TF_OK; arrays of different lengths or NULL with n > 0 ->
  TF_EINVAL);
* on the GPU: every overload's outputs equal the C entry point's bit for bit,
  binary64 and binary32, on 100003-element device arrays.
"""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "cxx", "tfcp_check")


def _exe():
    if not os.path.exists(EXE):
        # built by __graft_entry__.build(); built here only on a host without one
        sys.path.insert(0, os.path.join(HERE, "cxx"))
        import build_check
        build_check.build()
    return EXE


def _run(mode):
    r = subprocess.run([_exe(), mode], capture_output=True, text=True, timeout=120)
    print(r.stdout[-3000:])
    assert r.returncode == 0 and "ALL OK" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]
    return r.stdout


def test_header_argument_handling():
    out = _run("cpu")
    assert out.count("ok  ") == 2 * (18 + 8 + 4)


@pytest.mark.gpu
def test_header_equals_c_abi_on_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    out = _run("gpu")
    assert out.count("ok  ") == 2 * (18 + 8 + 4)
