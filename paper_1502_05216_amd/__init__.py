"""MI355X-native twofold exp/log (E. Latkin, "Twofold exp and log", 2015).

Elementwise twofold functions over split arrays of twofolds x0 + x1 on the
GPU, in binary64 and binary32:

    z0, z1 = texp(x0, x1)      # z0 = exp(x0) bitwise, z0 + z1 ~ e^(x0 + x1)
    z0, z1 = texpm1(x0, x1)    # expm1
    z0, z1 = tlog(x0, x1)      # log
    z0, z1 = tlog1p(x0, x1)    # log1p
    z = exp1x(x), expm1_1x(x), log1x(x), log1p_1x(x)   # the 1x main parts
    z0, z1 = pexp0(x0), texp0(x0), pexpm10(x0), texpm10(x0),
             plog0(y0), tlog0(y0), plog1p0(y0), tlog1p0(y0)  # dotted argument
    z0, z1 = texpp(x0, x1), pexp(x0, x1), texpm1p(x0, x1), pexpm1(x0, x1),
             tlogp(y0, y1), plog(y0, y1), tlog1pp(y0, y1), plog1p(y0, y1)
                                                        # coupled argument
    z0, z1 = tadd(x0, x1, y0, y1), tsub(...), tmul(...), tdiv(...), tsqrt(x0, x1)
                                                        # twofold arithmetic
    gx0, gx1 = texp_bwd(z0, z1, g0, g1)                 # twofold adjoints
    autograd.TExp / TExpm1 / TLog / TLog1p              # torch.autograd.Function

Arguments are contiguous torch tensors on the GPU; work is enqueued on the
current stream.  The kernels live in libtwofold_hip.so (csrc/, C ABI in
include/twofold_hip.h); this package only marshals arguments.
"""
from ._lib import (ARITH, COUPLED, DOTTED, ONEX, TWOFOLD, TwofoldError, arith_call,
                   backward_call, chain_bwd_call, declared_functions, dotted_call, lib, onex_call,
                   twofold_call)


def texp(x0, x1, out=None):
    return twofold_call("texp", x0, x1, out)


def texpm1(x0, x1, out=None):
    return twofold_call("texpm1", x0, x1, out)


def tlog(x0, x1, out=None):
    return twofold_call("tlog", x0, x1, out)


def tlog1p(x0, x1, out=None):
    return twofold_call("tlog1p", x0, x1, out)


def exp1x(x, out=None):
    return onex_call("exp1x", x, out)


def expm1_1x(x, out=None):
    return onex_call("expm1_1x", x, out)


def log1x(x, out=None):
    return onex_call("log1x", x, out)


def log1p_1x(x, out=None):
    return onex_call("log1p_1x", x, out)


def texp_bwd(s0, s1, g0, g1, out=None):
    return backward_call("texp", s0, s1, g0, g1, out)


def texpm1_bwd(s0, s1, g0, g1, out=None):
    return backward_call("texpm1", s0, s1, g0, g1, out)


def tlog_bwd(s0, s1, g0, g1, out=None):
    return backward_call("tlog", s0, s1, g0, g1, out)


def tlog1p_bwd(s0, s1, g0, g1, out=None):
    return backward_call("tlog1p", s0, s1, g0, g1, out)


def chain_bwd(names, saved, g0, g1, out=None):
    """Gradient of the chain y = names[-1](... names[0](x)) from the saved
    forward values of its stages, in one pass (see chain_bwd_call)."""
    return chain_bwd_call(names, saved, g0, g1, out)


def _dotted(name):
    def f(x0, out=None):
        return dotted_call(name, x0, out)
    f.__name__ = name
    f.__doc__ = "z0, z1 = %s(x0) elementwise (dotted argument)" % name
    return f


def _coupled(name):
    def f(x0, x1, out=None):
        return twofold_call(name, x0, x1, out)
    f.__name__ = name
    f.__doc__ = "z0, z1 = %s(x0 + x1) elementwise (coupled argument)" % name
    return f


def _arith(name):
    def f(x0, x1, y0, y1, out=None):
        return arith_call(name, x0, x1, y0, y1, out)
    f.__name__ = name
    f.__doc__ = "z0, z1 = %s of the twofolds x0 + x1 and y0 + y1, elementwise" % name
    return f


def tsqrt(x0, x1, out=None):
    """z0, z1 = sqrt(x0 + x1) elementwise (twofold square root)."""
    return twofold_call("tsqrt", x0, x1, out)


def trenorm(x0, x1, out=None):
    """z0, z1: the renormalized twofold of exactly the value x0 + x1
    (z0 = RN(x0 + x1), z1 the remainder), elementwise."""
    return twofold_call("trenorm", x0, x1, out)


for _n in ARITH:
    globals()[_n] = _arith(_n)
for _n in DOTTED:
    globals()[_n] = _dotted(_n)
for _n in COUPLED:
    globals()[_n] = _coupled(_n)


def build(verbose=False):
    from . import _build
    return _build.build(verbose=verbose)


__all__ = ["texp", "texpm1", "tlog", "tlog1p", "exp1x", "expm1_1x", "log1x", "log1p_1x",
           "texp_bwd", "texpm1_bwd", "tlog_bwd", "tlog1p_bwd", "chain_bwd",
           "TwofoldError", "declared_functions", "lib", "build", "TWOFOLD", "ONEX",
           "DOTTED", "COUPLED", "ARITH", "tsqrt", "trenorm"] + list(DOTTED) + list(COUPLED) + list(ARITH)
