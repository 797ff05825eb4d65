"""Builds libtwofold_hip.so (HIP, gfx950) in-tree with hipcc."""
import hashlib
import re
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libtwofold_hip.so")
SOURCES = [os.path.join(PKG, "csrc", f) for f in ("tf_kernels.hip", "tf_iface.hip", "tf_arith.hip")]
ARCH = os.environ.get("TF_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    # every fused multiply-add is explicit: no contraction of a*b+c
    "-ffp-contract=off",
    # keep binary32 subnormals (the float twofolds reach them)
    "-fno-gpu-flush-denormals-to-zero",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd))
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l
                    and "is not a recognized feature for this target" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)


# Flagged build variants of the same sources: name -> extra defines.
#   horner2x: every Horner step of pexp0 and pexpm10 in twofold arithmetic
#             (the algorithm listings' scheme; the default library runs the
#             highest-degree steps in 1x, as the paper's cost discussion allows)
#   k6:       pexp0 with the finer decomposition K = 6 (|y| <= 2^-7, one
#             Taylor term fewer, a C table of twice the entries), the
#             rebalancing of table size against Horner length that the section
#             "Function pexp0()" closes with; validated against the binary128
#             etalon, not the oracle (whose parameters are the paper's)
#   accexp:   texp's second part with the product z0 t1 taken exactly for a
#             coupled x1 and its low part carried apart (pexp renormalises
#             it); validated against the binary128 etalon, not the oracle
VARIANTS = {
    "horner2x": ["-DTF_HORNER_1X_TAIL=0"],
    "k6": ["-DTF_PEXP0_K=6"],
    "accexp": ["-DTF_TEXP_ACC=1"],
}


def variant_path(name):
    """Path of the shared library of build variant `name`."""
    if name not in VARIANTS:
        raise ValueError("unknown variant %r" % (name,))
    return os.path.join(PKG, "libtwofold_hip_%s.so" % name)


def build(verbose=False, extra=(), out=None):
    """Compile the library (always recompiles: one object per source, in
    parallel, then the shared-library link) and return its path."""
    out = out or LIB
    tmpdir = tempfile.mkdtemp(prefix="tf_build_")
    try:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in SOURCES]
        cmds = [[hipcc()] + HIPCC_FLAGS + list(extra) + ["-c", src, "-o", obj]
                for src, obj in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = out + ".tmp"
        _run([hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp],
             verbose)
        os.replace(tmp, out)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return out


def build_variant(name, verbose=False):
    """Compile build variant `name` of the library; return its path."""
    return build(verbose=verbose, extra=VARIANTS[name], out=variant_path(name))


def build_all(verbose=False):
    """The library and every build variant, concurrently."""
    jobs = [lambda: build(verbose=verbose)] + [
        (lambda n=n: build_variant(n, verbose=verbose)) for n in VARIANTS]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        return [f.result() for f in [ex.submit(j) for j in jobs]]


def _code_only(text):
    """C/C++ source without comments and with whitespace runs collapsed (string
    literals in these sources contain no comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_hash():
    """Hash of the library's code (csrc/: the HIP sources with comments and
    whitespace removed, and the table generator): ties a measurement to the
    code it measured, and survives edits of comments."""
    h = hashlib.sha256()
    d = os.path.join(PKG, "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".inc", ".py")):
            with open(os.path.join(d, f), encoding="utf-8") as fh:
                text = fh.read()
            if not f.endswith(".py"):
                text = _code_only(text)
            h.update(f.encode() + b"\0" + text.encode())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    print(build_all(verbose=True))
