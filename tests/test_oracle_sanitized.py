"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/tfo.cpp and the binary128 etalon oracle/qref.c are built, host code
only (g++ and gcc, no GPU code), with
``-fsanitize=address,undefined,float-cast-overflow -fno-sanitize-recover=all``
together with the driver tests/cxx/oracle_san.cpp, which calls every function
they export (scalar, array on two OpenMP threads, operation counting) on bit
patterns of every class: NaN, infinities, signed zeros, subnormals, the
largest normals, and the arguments the functions are meant for.  A heap or
stack access out of bounds, a use after free, a signed overflow, an
out-of-range shift or a float-to-integer conversion out of range (C++
undefined behaviour, which argument reduction by rounding to an integer could
reach on huge or NaN arguments) aborts the program and fails the test.

A planted program checks first that the sanitizers of this toolchain do report
such mistakes, so that a clean run is not vacuous.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
       "-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all"]
# the oracle's own floating-point flags (oracle/__init__.py)
FP = ["-mfma", "-ffp-contract=off", "-fno-fast-math", "-frounding-math"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")

PLANTED = r"""
#include <cstdio>
#include <cstdlib>
#include <vector>
int main(int argc, char** argv) {
    volatile double huge = 1e300;
    std::vector<double> v(8, 1.0);
    if (argv[1][0] == 'a') std::printf("%g\n", v.data()[8 + argc - 2]);   // one past the end
    if (argv[1][0] == 'c') std::printf("%d\n", (int)(huge * argc));        // out of int's range
    return 0;
}
"""


def _tools():
    for t in ("g++", "gcc"):
        if shutil.which(t) is None:
            pytest.skip("%s not found" % t)


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, env=ENV, timeout=600, **kw)


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    _tools()
    d = tmp_path_factory.mktemp("oracle_san")
    src = d / "planted.cpp"
    src.write_text(PLANTED)
    r = _run(["g++", "-std=c++17"] + SAN + [str(src), "-o", str(d / "planted")])
    if r.returncode != 0:
        pytest.skip("the toolchain cannot build sanitized programs: " + r.stderr[-400:])
    qo = d / "qref.o"
    r = _run(["gcc"] + SAN + ["-c", os.path.join(ROOT, "oracle", "qref.c"), "-o", str(qo)])
    assert r.returncode == 0, r.stderr
    exe = d / "oracle_san"
    r = _run(["g++", "-std=c++17"] + SAN + FP +
             [os.path.join(HERE, "cxx", "oracle_san.cpp"), os.path.join(ROOT, "oracle", "tfo.cpp"),
              str(qo), "-lquadmath", "-o", str(exe)])
    assert r.returncode == 0, r.stderr
    return d


@pytest.mark.parametrize("case,report", [("a", "AddressSanitizer"),
                                         ("c", "runtime error")])
def test_planted_mistakes_are_reported(sanitized, case, report):
    r = _run([str(sanitized / "planted"), case])
    assert r.returncode != 0 and report in r.stderr, (r.returncode, r.stderr[-600:])


def test_oracle_clean_under_sanitizers(sanitized):
    r = _run([str(sanitized / "oracle_san")])
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.stdout.startswith("SANITIZED OK"), r.stdout
    assert int(r.stdout.split()[2]) > 1_000_000
