"""Pins of the oracle's float32 library functions: correctly rounded.

Reading: the float32 evaluation rounds the exact value of every function
once, to nearest even, as IEEE arithmetic does for +, -, *, / and sqrt (the
paper names the functions of Sec. III-D1 but no library).  These tests check
the oracle's float32 path against mpmath (60 significant digits, an
implementation independent of the C library the oracle calls), bit for bit:
  * random float32 inputs across every binade, both signs, and the special
    values;
  * the hardest inputs of a scan: those whose double-precision result lies
    closest to a float32 rounding boundary (where the oracle must consult
    its extended-precision fallback);
and that no rounding was left undecided.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import ATAN, ATAN2, CBRT, COS, EXP, LOG, SIN, TAN, TANH, VAR, node

FUNCS = {SIN: "sin", COS: "cos", TAN: "tan", LOG: "log", EXP: "exp", TANH: "tanh", ATAN: "atan", CBRT: "cbrt"}


def _mp(op, x, y=None):
    import mpmath
    m = mpmath.mpf(float(x))
    if op == LOG:
        return mpmath.log(abs(m)) if abs(float(x)) > 0.0010000000474974513 else mpmath.mpf(0)
    if op == CBRT:
        return mpmath.cbrt(m) if m >= 0 else -mpmath.cbrt(-m)
    if op == ATAN2:
        return mpmath.atan2(m, mpmath.mpf(float(y)))
    return getattr(mpmath, FUNCS[op])(m)


def cr32(exact):
    """The float32 nearest to an mpmath value (ties cannot occur here)."""
    import mpmath
    d = float(exact)
    with np.errstate(over="ignore"):
        f = np.float32(d)
    if np.isinf(f):
        top = mpmath.mpf(2) ** 128 - mpmath.mpf(2) ** 103      # FLT_MAX + half its spacing
        if abs(exact) < top:
            return np.float32(math.copysign(np.finfo(np.float32).max, d))
        return f
    cands = [f, np.nextafter(f, np.float32(np.inf)), np.nextafter(f, np.float32(-np.inf))]
    return min(cands, key=lambda c: abs(mpmath.mpf(float(c)) - exact))


def _inputs(op, rng, n):
    e = rng.integers(-149, 128, n)
    m = rng.integers(0, 1 << 23, n)
    bits = np.where(e < -126, m >> np.clip(-126 - e, 0, 31), ((np.clip(e, -126, 127) + 127) << 23) | m)
    x = bits.astype(np.uint32).view(np.float32) * np.where(rng.random(n) < 0.5, -1, 1).astype(np.float32)
    if op in (SIN, COS, TAN):   # also the ordinary range
        x = np.concatenate([x, rng.uniform(-20, 20, n // 2).astype(np.float32)])
    if op == EXP:
        x = np.concatenate([x, rng.uniform(-104, 89, n // 2).astype(np.float32)])
    if op == LOG:
        x = np.concatenate([x, rng.uniform(0.5, 2.0, n // 2).astype(np.float32)])
    special = np.array([0.0, -0.0, 1.0, -1.0, 0.5, 2.0, 1e-45, -1e-45, 3.4028235e38, -3.4028235e38,
                        np.float32(np.pi), 0.0010000000474974513, 0.0009999999310821295], np.float32)
    return np.concatenate([x, special]).astype(np.float32)


def _hardest(op, rng, n_scan, k):
    """The k inputs (of n_scan random ones) whose double result lies closest
    to a float32 rounding boundary, in units of the double's spacing."""
    f64 = {SIN: np.sin, COS: np.cos, TAN: np.tan, LOG: lambda a: np.log(np.abs(a)), EXP: np.exp,
           TANH: np.tanh, ATAN: np.arctan, CBRT: np.cbrt}[op]
    lo, hi = {EXP: (-100, 88), LOG: (0.002, 1e6), TANH: (-9, 9)}.get(op, (-1e4, 1e4))
    x = rng.uniform(lo, hi, n_scan).astype(np.float32)
    with np.errstate(all="ignore"):
        v = f64(x.astype(np.float64))
        f = v.astype(np.float32)
        up = np.nextafter(f, np.float32(np.inf)).astype(np.float64)
        dn = np.nextafter(f, np.float32(-np.inf)).astype(np.float64)
        d = np.minimum(v - (f.astype(np.float64) + dn) / 2, (f.astype(np.float64) + up) / 2 - v)
        d = d / np.spacing(np.abs(v))
    d[~np.isfinite(d)] = np.inf
    return x[np.argsort(d)[:k]], float(np.sort(d)[0])


def _oracle32(op, x, y=None):
    if op == ATAN2:
        pop = oracle.from_programs([([node(ATAN2), node(VAR, 0), node(VAR, 1)], [])])
        X = np.ascontiguousarray(np.stack([x, y]))
    else:
        pop = oracle.from_programs([([node(op), node(VAR, 0)], [])])
        X = np.ascontiguousarray(x[None, :])
    return oracle.evaluate_f32(pop, X, n_threads=1)[0]


def _check(op, x, got, y=None):
    import mpmath
    mpmath.mp.dps = 60
    for i in range(x.size):
        ex = _mp(op, x[i], None if y is None else y[i])
        want = cr32(ex)
        if ex == 0 and x[i] == 0 and op in (SIN, TAN, TANH, ATAN, CBRT):
            want = x[i]          # odd functions keep the sign of a zero (mpmath has no -0)
        g = got[i]
        ok = (g == want and np.signbit(g) == np.signbit(want)) or (np.isnan(g) and np.isnan(want))
        assert ok, (FUNCS.get(op, "atan2"), repr(x[i]), repr(g), repr(want))


@pytest.mark.parametrize("op", sorted(FUNCS))
def test_float32_functions_correctly_rounded(op):
    rng = np.random.default_rng(100 + op)
    x = _inputs(op, rng, 600)
    oracle.cr_reset()
    _check(op, x, _oracle32(op, x))
    assert oracle.cr_undecided() == 0


@pytest.mark.parametrize("op", sorted(FUNCS))
def test_float32_functions_hardest_roundings(op):
    """The inputs of a scan whose double result sits closest to a float32
    rounding boundary, where a double-then-float rounding could go wrong:
    with the default fallback margin, and with the margin widened to 2^26
    double ulps so that about a quarter of the inputs take the
    extended-precision path."""
    rng = np.random.default_rng(200 + op)
    x, closest = _hardest(op, rng, 400_000, 40)
    assert closest < 2 ** 14, closest     # within 2^-14 of the spacing between boundaries
    x = np.concatenate([x, _inputs(op, rng, 200)])
    try:
        for margin in (8.0, 2.0 ** 26):
            oracle.cr_set_margin(margin)
            oracle.cr_reset()
            _check(op, x, _oracle32(op, x))
            assert oracle.cr_undecided() == 0
    finally:
        oracle.cr_set_margin()


def test_atan2_correctly_rounded():
    rng = np.random.default_rng(7)
    a = rng.uniform(-50, 50, 500).astype(np.float32)
    b = rng.uniform(-50, 50, 500).astype(np.float32)
    oracle.cr_reset()
    _check(ATAN2, a, _oracle32(ATAN2, a, b), b)
    assert oracle.cr_undecided() == 0


def test_exact_functions_contribute_no_bound():
    """With sin, cos and log taken as correctly rounded on both sides, a
    program over the nine-function set of the benchmark (every other function
    in it is one IEEE operation) has a zero bound and no flagged predicate on
    every row: two correct evaluations agree bit for bit (a predicate the
    float64 path decides differently says nothing about two float32
    evaluations that agree on every operand).  With the 4-ulp allowance on
    those three functions instead, the same rows get positive bounds."""
    import synth
    pop = oracle.build_population(64, 2, "exact_len", min_len=1, max_len=200, seed=11)
    X, _ = synth.pagie(300, seed=4)
    prog = np.repeat(np.arange(64, dtype=np.int32), 300)
    row = np.tile(np.arange(300, dtype=np.int64), 64)
    exact = (1 << SIN) | (1 << COS) | (1 << LOG)
    ra = oracle.evaluate_pairs(pop, X, prog, row, exact=exact)
    assert (ra.bound == 0).all() and not ra.near.any()
    rb = oracle.evaluate_pairs(pop, X, prog, row)
    assert (rb.bound > 0).mean() > 0.5
    assert np.array_equal(ra.v32.view(np.uint32), rb.v32.view(np.uint32))
