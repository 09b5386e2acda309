"""Pins of the oracle's program evaluation against things other than itself:
hand-evaluated programs, the protected-operator special cases, the Pagie closed
form (Sec. IV-A, Eq. (pagie)), brute force against an independent recursive
tree evaluator, and a brute-force check of the validity scan against a
recursive-descent parser."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import ADD, SUB, MUL, DIV, NEG, LOG, SQRT, SIN, COS, TAN, VAR, CONST, node

import synth


def one(nodes, consts, X):
    pop = oracle.from_programs([(nodes, consts)])
    return oracle.evaluate_f32(pop, X)[0], oracle.evaluate_f64(pop, X)[0]


def cols(*vals):
    return np.array([[v] for v in vals], dtype=np.float32)


# ---- hand-evaluated programs (operand order: first pop = first argument) ----
@pytest.mark.parametrize("prog,consts,row,expect", [
    ([node(SUB), node(VAR, 0), node(VAR, 1)], [], (1, 2), -1.0),
    ([node(DIV), node(VAR, 0), node(VAR, 1)], [], (1, 4), 0.25),
    ([node(MUL), node(ADD), node(VAR, 0), node(CONST, 0), node(VAR, 1)], [0.5], (1, 2), 3.0),
    ([node(NEG), node(VAR, 0)], [], (3, 0), -3.0),
    ([node(SUB), node(CONST, 0), node(CONST, 1)], [5.0, 2.0], (0, 0), 3.0),
    ([node(DIV), node(SUB), node(VAR, 1), node(VAR, 0), node(CONST, 0)], [4.0], (1, 9), 2.0),
    ([node(SQRT), node(MUL), node(VAR, 0), node(VAR, 1)], [], (-2, 8), 4.0),
    ([node(VAR, 1)], [], (7, 8), 8.0),
    ([node(CONST, 0)], [0.25], (7, 8), 0.25),
])
def test_hand_evaluated(prog, consts, row, expect):
    o32, o64 = one(prog, consts, cols(*row))
    assert o32[0] == np.float32(expect)
    assert o64[0] == expect


# ---- protected operators ----
@pytest.mark.parametrize("prog,x0,x1,expect", [
    ([node(DIV), node(VAR, 0), node(VAR, 1)], 1.0, 0.0, 1.0),           # pdiv(1, 0) = 1
    ([node(DIV), node(VAR, 0), node(VAR, 1)], 1.0, 5e-4, 1.0),          # |b| <= 0.001
    ([node(DIV), node(VAR, 0), node(VAR, 1)], 1.0, -5e-4, 1.0),
    ([node(DIV), node(VAR, 0), node(VAR, 1)], 3.0, float("nan"), 1.0),  # NaN fails |b| > eps
    ([node(LOG), node(VAR, 0)], 0.0, 0.0, 0.0),                         # plog(0) = 0
    ([node(LOG), node(VAR, 0)], -1.0, 0.0, 0.0),
    ([node(LOG), node(VAR, 0)], float("nan"), 0.0, 0.0),
    ([node(SQRT), node(VAR, 0)], -4.0, 0.0, 2.0),                       # psqrt(-4) = 2
    ([node(SQRT), node(VAR, 0)], -0.0, 0.0, 0.0),
])
def test_protected_special_cases(prog, x0, x1, expect):
    o32, o64 = one(prog, [], cols(x0, x1))
    assert o32[0] == np.float32(expect)
    assert o64[0] == expect


def test_protected_threshold_is_float_0p001():
    eps = np.float32(0.001)
    above = np.nextafter(eps, np.float32(1))
    p = [node(DIV), node(VAR, 0), node(VAR, 1)]
    assert one(p, [], cols(2.0, eps))[0][0] == 1.0            # not strictly above
    assert one(p, [], cols(2.0, above))[0][0] == np.float32(2.0) / above
    pl = [node(LOG), node(VAR, 0)]
    assert one(pl, [], cols(eps, 0))[0][0] == 0.0
    e32 = float(np.float32(math.e))
    assert one(pl, [], cols(-e32, 0))[0][0] == np.float32(math.log(e32))


def test_ieee_specials_propagate():
    inf = float("inf")
    o32, _ = one([node(ADD), node(VAR, 0), node(VAR, 1)], [], cols(inf, 1.0))
    assert o32[0] == inf
    o32, _ = one([node(SIN), node(VAR, 0)], [], cols(inf, 0))
    assert np.isnan(o32[0])
    o32, _ = one([node(DIV), node(VAR, 0), node(VAR, 1)], [], cols(1.0, inf))
    assert o32[0] == 0.0
    o32, _ = one([node(LOG), node(VAR, 0)], [], cols(-inf, 0))
    assert o32[0] == inf


# ---- the Pagie closed form ----
def _x4(f):
    return [node(MUL), node(MUL), node(VAR, f), node(VAR, f), node(MUL), node(VAR, f), node(VAR, f)]


def pagie_program():
    half = lambda f: [node(DIV)] + _x4(f) + [node(ADD)] + _x4(f) + [node(CONST, f)]
    return [node(ADD)] + half(0) + half(1), [1.0, 1.0]


def test_pagie_closed_form_program_has_zero_error():
    prog, consts = pagie_program()
    assert len(prog) == 35
    X, y = synth.pagie(4096, seed=5)
    pop = oracle.from_programs([(prog, consts)])
    f32p, f64 = oracle.fitness(pop, X, y, metric="mse")
    assert f32p[0] < 1e-12
    assert f64[0] < 1e-13
    o64 = oracle.evaluate_f64(pop, X)[0]
    assert np.max(np.abs(o64 - y.astype(np.float64))) < 1e-7


def test_pagie_reciprocal_form_exposes_protected_division():
    # 1/(1 + 1/x^4): where |x^4| <= 0.001 the protected inner division returns
    # 1 instead of 1/x^4, so that half evaluates to 1/(1+1) = 0.5.
    def half(f):
        return ([node(DIV), node(CONST, 0), node(ADD), node(CONST, 0), node(DIV), node(CONST, 0)]
                + _x4(f))
    prog = half(0)
    X, _ = synth.pagie(20000, seed=6)
    X[0, :50] = np.linspace(-0.2, 0.2, 50, dtype=np.float32)
    o32, o64 = one(prog, [1.0], X)
    x = X[0]
    x4 = (x * x) * (x * x)
    small = np.abs(x4) <= np.float32(0.001)
    assert small.sum() > 10
    assert np.all(o32[small] == 0.5)
    xd = x.astype(np.float64)
    target = xd ** 4 / (1 + xd ** 4)
    assert np.max(np.abs(o64[~small] - target[~small])) < 1e-12


# ---- brute force against an independent recursive evaluator ----
def _tree_eval(nodes, consts, xs, pos=0):
    """Recursive-descent evaluation in numpy float32, left to right: a
    different algorithm from the oracle's right-to-left stack scan."""
    w = int(nodes[pos])
    op, arg = w & 0xFF, w >> 8
    f = np.float32
    if op == VAR:
        return f(xs[arg]), pos + 1
    if op == CONST:
        return f(consts[arg]), pos + 1
    a, pos = _tree_eval(nodes, consts, xs, pos + 1)
    if op in (NEG, LOG, SQRT, SIN, COS, TAN):
        if op == NEG:
            return f(-a), pos
        if op == SQRT:
            return f(np.sqrt(np.abs(a))), pos
        if op == LOG:
            return (f(math.log(abs(float(a)))) if abs(a) > f(0.001) else f(0.0)), pos
        fn = {SIN: math.sin, COS: math.cos, TAN: math.tan}[op]
        return f(fn(float(a))), pos
    b, pos = _tree_eval(nodes, consts, xs, pos)
    with np.errstate(all="ignore"):
        if op == ADD:
            return f(a + b), pos
        if op == SUB:
            return f(a - b), pos
        if op == MUL:
            return f(a * b), pos
        return (f(a / b) if abs(b) > f(0.001) else f(1.0)), pos


def _enumerate(n_max, terms, unary, binary):
    """All prefix lists of at most n_max nodes."""
    out = []

    def rec(prefix, need):
        if need == 0:
            out.append(list(prefix))
            return
        if len(prefix) + need > n_max:
            return
        for t in terms:
            rec(prefix + [t], need - 1)
        for u in unary:
            rec(prefix + [u], need)
        for b in binary:
            rec(prefix + [b], need + 1)

    rec([], 1)
    return out


def _rows():
    rng = np.random.default_rng(3)
    x = rng.uniform(-3, 3, size=(2, 61)).astype(np.float32)
    special = np.array([[0, 0.0005, -1, 2], [0, 1, 0.001, -2]], dtype=np.float32)
    return np.ascontiguousarray(np.concatenate([x, special], axis=1))


def test_bruteforce_arithmetic_bit_exact():
    terms = [node(VAR, 0), node(VAR, 1), node(CONST, 0)]
    progs = _enumerate(5, terms, [], [node(ADD), node(SUB), node(MUL), node(DIV)])
    assert len(progs) == 3 + 4 * 9 + 2 * 16 * 27
    X = _rows()
    pop = oracle.from_programs([(p, [0.5]) for p in progs])
    got = oracle.evaluate_f32(pop, X)
    for i, p in enumerate(progs):
        for r in range(X.shape[1]):
            ref, end = _tree_eval(p, [0.5], X[:, r])
            assert end == len(p)
            g = got[i, r]
            assert (np.isnan(ref) and np.isnan(g)) or g == ref, (p, r, g, ref)


def test_bruteforce_unary_within_one_ulp():
    terms = [node(VAR, 0), node(CONST, 0)]
    progs = _enumerate(4, terms, [node(NEG), node(LOG), node(SQRT), node(SIN), node(COS)],
                       [node(ADD), node(MUL), node(DIV)])
    X = _rows()
    pop = oracle.from_programs([(p, [0.5]) for p in progs])
    got = oracle.evaluate_f32(pop, X)
    for i, p in enumerate(progs):
        for r in range(X.shape[1]):
            ref, _ = _tree_eval(p, [0.5], X[:, r])
            g = got[i, r]
            if np.isnan(ref):
                assert np.isnan(g)
                continue
            # libm float functions vs correctly rounded double-then-round:
            # at most one ulp apart per transcendental, amplified by at most
            # this depth-4 program's conditioning.
            tol = 4 * np.spacing(np.float32(max(abs(ref), 1e-30)))
            assert abs(np.float64(g) - np.float64(ref)) <= max(tol, 1e-6 * max(1.0, abs(ref))), (p, r)


# ---- validity scan vs recursive-descent parse, every arity sequence <= 8 ----
def _parse_ok(ar):
    def rec(i):
        if i >= len(ar):
            return -1
        j = i + 1
        for _ in range(ar[i]):
            j = rec(j)
            if j < 0:
                return -1
        return j
    return rec(0) == len(ar)


def _depth(ar):
    def rec(i):
        d = 0
        j = i + 1
        for _ in range(ar[i]):
            sub, j = rec(j)
            d = max(d, sub + 1)
        return d, j
    return rec(0)[0]


def test_validity_scan_matches_parser_bruteforce():
    rep = {0: node(VAR, 0), 1: node(NEG), 2: node(ADD)}
    n_valid = 0
    for n in range(1, 9):
        for ar in itertools.product((0, 1, 2), repeat=n):
            nodes = [rep[a] for a in ar]
            rc, h = oracle.check_program(nodes, 1, 0)
            ok = _parse_ok(ar)
            assert (rc == 0) == ok, ar
            if ok:
                n_valid += 1
                assert h <= _depth(ar) + 1
                if all(a != 1 for a in ar):
                    # for binary-only trees, a stack of m holds depth m-1
                    assert h <= _depth(ar) + 1
    assert n_valid > 100


def test_validity_error_codes():
    assert oracle.check_program([node(VAR, 2)], 2, 0)[0] == 4
    assert oracle.check_program([node(CONST, 1)], 2, 1)[0] == 5
    assert oracle.check_program([node(13)], 2, 0)[0] == 1
    assert oracle.check_program([], 2, 0)[0] == 6
    # ADD^19 x^20 is a left comb: read right to left it pushes 20 terminals
    # before the first ADD, so it needs exactly the full stack of 20 ...
    rc, h = oracle.check_program([node(ADD)] * 19 + [node(VAR, 0)] * 20, 1, 0)
    assert (rc, h) == (0, 20)
    # ... and one more level overflows it
    assert oracle.check_program([node(ADD)] * 20 + [node(VAR, 0)] * 21, 1, 0)[0] == 3
    # the right comb (ADD x)^20 x is deep but needs a stack of only 2
    comb = [node(ADD), node(VAR, 0)] * 20 + [node(VAR, 0)]
    assert oracle.check_program(comb, 1, 0) == (0, 2)
