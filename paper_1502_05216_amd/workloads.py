"""Seeded synthetic inputs for the twofold functions (numpy, PCG64).

This module holds only input recipes: no step of the twofold method.  Both the
GPU library's tests/benchmark and the CPU oracle's checks draw their inputs
here, so the two sides see identical arrays.

The paper measures on random samples (section "Accuracy"); these recipes give
each function the argument range it is meant for, with a second part
x1 = (x0 * u) * eps, u ~ U[-1, 1], eps = 2^-53 (double) or 2^-24 (float), so
that x0 + x1 is a coupled twofold as produced by twofold arithmetic upstream.

    twofold_inputs(fn, n, dtype, seed, edges=0.001) -> (x0, x1)
    batch_descriptors(count, seed, max_log2=20) -> list of (func, dtype, n)
    chain_inputs(n, seed) -> (x0, x1, g0, g1)
"""
import numpy as np

SEED = 1502052160
FUNCS = ("texp", "texpm1", "tlog", "tlog1p")


def _eps(dt):
    return np.float64(2.0 ** -53) if dt == np.float64 else np.float32(2.0 ** -24)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def edge_values(fn, dtype):
    """Edge arguments x0 for fn in the given dtype: signed zeros, subnormals,
    the overflow/underflow boundaries of exp and their neighbours, branch
    boundaries of the method (ln2, 1/2, 2, -1/2, 1), infinities and NaN."""
    dt = np.dtype(dtype).type
    fi = np.finfo(dt)
    tiny = dt(fi.smallest_subnormal)
    big = dt(fi.max)
    norm = dt(fi.tiny)
    inf = dt(np.inf)

    def nb(v):
        v = dt(v)
        return [np.nextafter(v, dt(-np.inf)), v, np.nextafter(v, dt(np.inf))]

    common = [dt(0.0), dt(-0.0), tiny, -tiny, norm, -norm, inf, -inf, dt(np.nan), big, -big]
    if dt == np.float64:
        xmax, xlo, xsub, ln2 = 709.782712893384, -745.1332191019411, -708.3964185322641, 0.6931471805599453
    else:
        xmax, xlo, xsub, ln2 = 88.72283, -103.97208, -87.33655, 0.6931472
    if fn == "texp":
        vals = common + nb(xmax) + nb(xlo) + nb(xsub) + nb(1.0) + nb(-1.0)
        # half-way points of the decomposition M = round(32 x)
        vals += [dt((k + 0.5) / 32.0) for k in (-3, -1, 0, 1, 2, 17)]
        # ends of the exponent table
        vals += [dt(-744.0), dt(708.0), dt(-700.0), dt(700.0)] if dt == np.float64 else \
                [dt(-102.0), dt(88.0), dt(-100.0), dt(80.0)]
    elif fn == "texpm1":
        vals = common + nb(xmax) + nb(ln2) + nb(-ln2) + [dt(-40.0), dt(-20.0), dt(2.0 ** -54),
                                                         dt(-2.0 ** -54), dt(2.0 ** -25)]
        vals += nb(2.0 ** -30) + nb(-(2.0 ** -30)) + [dt(89.5 / 128), dt(-89.5 / 128)]
    elif fn == "tlog":
        vals = common + nb(1.0) + nb(0.5) + nb(2.0) + [dt(-1.0), dt(-2.0), dt(4.0), dt(0.25)]
    elif fn == "tlog1p":
        vals = common + [dt(-1.0), np.nextafter(dt(-1.0), dt(0.0)), dt(-2.0)] + nb(-0.5) + \
            nb(1.0) + nb(2.0 ** -8) + [dt(-0.75), dt(3.0)]
    else:
        raise ValueError(fn)
    return np.array(vals, dtype=dt)


def _x0(fn, n, dt, rng):
    if fn == "texp":
        lo, hi = (-745.0, 709.7) if dt == np.float64 else (-103.9, 88.7)
        x = rng.uniform(lo, hi, n)
    elif fn == "tlog":
        lo, hi = (-1074.0, 1023.0) if dt == np.float64 else (-149.0, 127.0)
        x = np.exp2(rng.uniform(lo, hi, n))
    elif fn in ("texpm1", "tlog1p"):
        s = np.where(rng.uniform(-1.0, 1.0, n) < 0, -1.0, 1.0)
        x = s * np.exp2(rng.uniform(-60.0, 2.0, n))
        if fn == "tlog1p":
            bad = x <= -1.0
            while bad.any():
                m = int(bad.sum())
                x[bad] = -np.exp2(rng.uniform(-60.0, 2.0, m))
                bad = x <= -1.0
    else:
        raise ValueError(fn)
    return x.astype(dt)


# The other entry points of the paper's interface, by the argument recipe
# they share with one of the four twofold functions.
INTERFACE_BASE = {
    "pexp0": "texp", "texp0": "texp", "texpp": "texp", "pexp": "texp",
    "pexpm10": "texpm1", "texpm10": "texpm1", "texpm1p": "texpm1", "pexpm1": "texpm1",
    "plog0": "tlog", "tlog0": "tlog", "tlogp": "tlog", "plog": "tlog",
    "plog1p0": "tlog1p", "tlog1p0": "tlog1p", "tlog1pp": "tlog1p", "plog1p": "tlog1p",
}
DOTTED = ("pexp0", "texp0", "pexpm10", "texpm10", "plog0", "tlog0", "plog1p0", "tlog1p0")
COUPLED = ("texpp", "pexp", "texpm1p", "pexpm1", "tlogp", "plog", "tlog1pp", "plog1p")


def twofold_inputs(fn, n, dtype=np.float64, seed=SEED, edges=0.001, x0_range=None,
                   coupled=False):
    """Twofold arguments (x0, x1) for fn: n elements of dtype, seeded.

    texp: x0 ~ U[-745, 709.7] (float U[-103.9, 88.7]); tlog: x0 = 2^U[-1074, 1023]
    (float 2^U[-149, 127]); texpm1/tlog1p: |x0| = 2^U[-60, 2] with a random sign
    (tlog1p redraws x0 <= -1).  x1 = (x0 u) eps.  A fraction `edges` of the
    indices (chosen by the same generator) takes values from edge_values(fn)
    with x1 = 0, except every 8th of them, whose x1 cycles through
    +inf, -inf, NaN and the least subnormal.  x0_range=(lo, hi) replaces the
    x0 law by U[lo, hi].  coupled=True halves eps, so that x0 + x1 rounds to x0
    (the arguments of the paper's coupled-argument functions).  fn may also
    name one of the other interface functions (INTERFACE_BASE)."""
    fn = INTERFACE_BASE.get(fn, fn)
    dt = np.dtype(dtype).type
    rng = _rng(seed)
    if x0_range is None:
        x0 = _x0(fn, n, dt, rng)
    else:
        x0 = rng.uniform(x0_range[0], x0_range[1], n).astype(dt)
    u = rng.uniform(-1.0, 1.0, n).astype(dt)
    with np.errstate(over="ignore", invalid="ignore", under="ignore"):
        x1 = (x0 * u) * (_eps(dt) / dt(2) if coupled else _eps(dt))
        x1 = x1.astype(dt)
        if coupled:
            # near the subnormal range x1 rounds onto a coarse grid and can
            # reach half an ulp of x0: drop it there
            x1[(x0 + x1) != x0] = dt(0.0)
    ne = int(round(n * edges))
    if ne > 0:
        ev = edge_values(fn, dt)
        idx = rng.choice(n, size=ne, replace=False)
        x0[idx] = ev[rng.integers(0, ev.size, ne)]
        x1[idx] = dt(0.0)
        special = np.array([np.inf, -np.inf, np.nan, np.finfo(dt).smallest_subnormal], dtype=dt)
        sel = idx[::8]
        x1[sel] = special[np.arange(sel.size) % special.size]
    return np.ascontiguousarray(x0), np.ascontiguousarray(x1)


def cfg1_inputs(n=65536, seed=SEED):
    """texp over double twofolds: x0 ~ U[-700, 700], x1 = x0 u 2^-53, no edges."""
    return twofold_inputs("texp", n, np.float64, seed=seed, edges=0.0, x0_range=(-700.0, 700.0))


def batch_descriptors(count=4096, seed=SEED + 3, max_log2=20, p_double=0.75):
    """Ragged batch recipe: `count` arrays with length clip(floor(2^U[0, max_log2]),
    1, 2^max_log2), function uniform over FUNCS, dtype float64 with probability
    p_double else float32.  Returns a list of (func, dtype, n)."""
    rng = _rng(seed)
    lens = np.clip(np.floor(np.exp2(rng.uniform(0.0, max_log2, count))), 1, 2 ** max_log2)
    fids = rng.integers(0, 4, count)
    dbl = rng.uniform(0.0, 1.0, count) < p_double
    return [(FUNCS[int(f)], np.float64 if d else np.float32, int(m))
            for f, d, m in zip(fids, dbl, lens)]


def chain_inputs(n, seed=SEED + 4, dtype=np.float64):
    """Inputs of y = tlog1p(texpm1(texp(x))): x0 ~ U[-20, 20], x1 = x0 u 2^-53,
    upstream gradient g0 ~ U[-1, 1], g1 = g0 u' 2^-53."""
    dt = np.dtype(dtype).type
    rng = _rng(seed)
    x0 = rng.uniform(-20.0, 20.0, n).astype(dt)
    x1 = ((x0 * rng.uniform(-1.0, 1.0, n).astype(dt)) * _eps(dt)).astype(dt)
    g0 = rng.uniform(-1.0, 1.0, n).astype(dt)
    g1 = ((g0 * rng.uniform(-1.0, 1.0, n).astype(dt)) * _eps(dt)).astype(dt)
    return x0, x1, g0, g1


def batch_inputs(descs, seed=SEED + 5, edges=0.001, align=16):
    """Inputs for a ragged batch: for each (func, dtype) one pool drawn with
    twofold_inputs over the total length, cut into the batch's arrays in
    order, each array starting on an `align`-byte boundary of the pool.
    Returns a list of (func, dtype, x0, x1) numpy views (pool slices)."""
    out = [None] * len(descs)
    groups = {}
    for i, (fn, dt, n) in enumerate(descs):
        groups.setdefault((fn, np.dtype(dt).type), []).append(i)
    for k, ((fn, dt), idx) in enumerate(sorted(groups.items(), key=lambda t: (t[0][0], str(t[0][1])))):
        step = max(1, align // np.dtype(dt).itemsize)
        offs, pos = [], 0
        for i in idx:
            offs.append(pos)
            pos += -(-descs[i][2] // step) * step
        x0, x1 = twofold_inputs(fn, max(pos, 1), dt, seed=seed + 17 * k, edges=edges)
        for i, o in zip(idx, offs):
            n = descs[i][2]
            out[i] = (fn, dt, x0[o:o + n], x1[o:o + n])
    return out
