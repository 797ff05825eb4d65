"""torch.autograd.Function wrappers of the twofold functions.

A twofold pair (x0, x1) is one number x = x0 + x1, and so is its gradient:
the backward of f receives the twofold upstream gradient (g0, g1) and returns
the twofold gradient (gx0, gx1) ~ (g0 + g1) f'(x0 + x1), computed by the
library's backward kernels in twofold arithmetic (texp: g z, texpm1:
g (z + 1), tlog: g / y, tlog1p: g / (1 + y)).  Chaining these Functions
therefore propagates a twofold gradient through a composition such as
tlog1p(texpm1(texp(x))).

    y0, y1 = TExp.apply(x0, x1)
"""
import torch

from . import _lib


def _forward(name, keep_output, ctx, x0, x1):
    x0 = x0.contiguous()
    x1 = x1.contiguous()
    z0, z1 = _lib.twofold_call(name, x0, x1)
    # texp/texpm1 differentiate through their value z, tlog/tlog1p through y
    ctx.save_for_backward(*((z0, z1) if keep_output else (x0, x1)))
    return z0, z1


def _backward(name, ctx, g0, g1):
    s0, s1 = ctx.saved_tensors
    g0 = torch.zeros_like(s0) if g0 is None else g0.contiguous()
    g1 = torch.zeros_like(s0) if g1 is None else g1.contiguous()
    return _lib.backward_call(name, s0, s1, g0, g1)


class TExp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, x1):
        return _forward("texp", True, ctx, x0, x1)

    @staticmethod
    def backward(ctx, g0, g1):
        return _backward("texp", ctx, g0, g1)


class TExpm1(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, x1):
        return _forward("texpm1", True, ctx, x0, x1)

    @staticmethod
    def backward(ctx, g0, g1):
        return _backward("texpm1", ctx, g0, g1)


class TLog(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, x1):
        return _forward("tlog", False, ctx, x0, x1)

    @staticmethod
    def backward(ctx, g0, g1):
        return _backward("tlog", ctx, g0, g1)


class TLog1p(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, x1):
        return _forward("tlog1p", False, ctx, x0, x1)

    @staticmethod
    def backward(ctx, g0, g1):
        return _backward("tlog1p", ctx, g0, g1)


class TChain(torch.autograd.Function):
    """y = names[-1](... names[0](x)) as one autograd node: the forward runs
    the stage kernels in order and keeps each stage's saved value (texp and
    texpm1 their output, tlog and tlog1p their argument); the backward is one
    fused pass of the library (tf_chain_bwd), equal bit for bit to chaining
    the single-stage Functions but reading each saved array once and keeping
    the intermediate gradients in registers."""

    @staticmethod
    def forward(ctx, names, x0, x1):
        z = (x0.contiguous(), x1.contiguous())
        saved = []
        for name in names:
            y = _lib.twofold_call(name, *z)
            saved.append(y if name in ("texp", "texpm1") else z)
            z = y
        ctx.names = tuple(names)
        ctx.save_for_backward(*[t for pair in saved for t in pair])
        return z

    @staticmethod
    def backward(ctx, g0, g1):
        flat = ctx.saved_tensors
        saved = [(flat[2 * j], flat[2 * j + 1]) for j in range(len(ctx.names))]
        g0 = torch.zeros_like(flat[0]) if g0 is None else g0.contiguous()
        g1 = torch.zeros_like(flat[0]) if g1 is None else g1.contiguous()
        gx0, gx1 = _lib.chain_bwd_call(ctx.names, saved, g0, g1)
        return None, gx0, gx1


def chain(names, x0, x1):
    """y = names[-1](... names[0](x0 + x1)), differentiable with the fused
    chain backward; names from texp, texpm1, tlog, tlog1p."""
    return TChain.apply(tuple(names), x0, x1)


def chain_exp_expm1_log1p(x0, x1):
    """y = tlog1p(texpm1(texp(x))) (= e^x in closed form), differentiable."""
    return chain(("texp", "texpm1", "tlog1p"), x0, x1)
