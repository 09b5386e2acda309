"""Pins of the oracle's program evaluation against things other than itself:
hand-evaluated programs, the protected-operator special cases, the Pagie closed
form (Sec. IV-A, Eq. (pagie)), brute force against an independent recursive
tree evaluator, and a brute-force check of the validity scan against a
recursive-descent parser."""
import ctypes
import ctypes.util
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
    assert oracle.check_program([node(23)], 2, 0)[0] == 1
    assert oracle.check_program([node(255)], 2, 0)[0] == 1
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


# ---- the wider function set (max, min, atan2, abs, exp, inv, sq, cube, tanh,
# atan, cbrt; Sec. III-D1 counts the functions without listing them, these
# follow the library the paper compares against) ----
from oracle import MAX, MIN, ATAN2, ABS, EXP, INV, SQ, CUBE, TANH, ATAN, CBRT  # noqa: E402

PI = math.pi


@pytest.mark.parametrize("prog,row,e32,e64", [
    ([node(MAX), node(VAR, 0), node(VAR, 1)], (1, 2), 2.0, 2.0),
    ([node(MAX), node(VAR, 0), node(VAR, 1)], (-1, -2), -1.0, -1.0),
    ([node(MIN), node(VAR, 0), node(VAR, 1)], (1, 2), 1.0, 1.0),
    ([node(MIN), node(VAR, 0), node(VAR, 1)], (-1, -2), -2.0, -2.0),
    ([node(ABS), node(VAR, 0)], (-3, 0), 3.0, 3.0),
    ([node(EXP), node(VAR, 0)], (0, 0), 1.0, 1.0),
    ([node(INV), node(VAR, 0)], (4, 0), 0.25, 0.25),
    ([node(INV), node(VAR, 0)], (-0.5, 0), -2.0, -2.0),
    ([node(SQ), node(VAR, 0)], (-3, 0), 9.0, 9.0),
    ([node(CUBE), node(VAR, 0)], (-2, 0), -8.0, -8.0),
    ([node(TANH), node(VAR, 0)], (0, 0), 0.0, 0.0),
    ([node(TANH), node(VAR, 0)], (30, 0), 1.0, 1.0),
    ([node(ATAN), node(VAR, 0)], (0, 0), 0.0, 0.0),
    ([node(CBRT), node(VAR, 0)], (-8, 0), -2.0, -2.0),
    ([node(CBRT), node(VAR, 0)], (27, 0), 3.0, 3.0),
    # atan2(first operand, second operand): the first popped value is y
    ([node(ATAN2), node(VAR, 0), node(VAR, 1)], (0, 1), 0.0, 0.0),
    ([node(ATAN2), node(VAR, 0), node(VAR, 1)], (1, 0), np.float32(PI / 2), PI / 2),
    ([node(ATAN2), node(VAR, 0), node(VAR, 1)], (-1, 0), np.float32(-PI / 2), -PI / 2),
    ([node(ATAN2), node(VAR, 0), node(VAR, 1)], (0, -1), np.float32(PI), PI),
    ([node(ATAN2), node(VAR, 0), node(VAR, 1)], (-0.0, -1), np.float32(-PI), -PI),
    ([node(ATAN2), node(VAR, 1), node(VAR, 0)], (0, 1), np.float32(PI / 2), PI / 2),
    # composite: (x0^2)^3 = x0^6 and cbrt(x0^3) = x0, both exact here
    ([node(CUBE), node(SQ), node(VAR, 0)], (2, 0), 64.0, 64.0),
    ([node(CBRT), node(CUBE), node(VAR, 0)], (-4, 0), -4.0, -4.0),
])
def test_wider_set_hand_evaluated(prog, row, e32, e64):
    o32, o64 = one(prog, [], cols(*row))
    # library functions (exp, tanh, atan, cbrt, atan2) are allowed one ulp
    # from the exact value; IEEE operations must be exact
    lib_fn = any(int(w) & 0xFF in (EXP, TANH, ATAN, CBRT, ATAN2) for w in prog)
    assert _ulps(o32[0], np.float32(e32)) <= (1 if lib_fn else 0), (o32[0], e32)
    assert abs(o64[0] - e64) <= (np.spacing(abs(e64)) if lib_fn else 0), (o64[0], e64)


@pytest.mark.parametrize("x,expect", [
    (0.0, 0.0), (5e-4, 0.0), (-5e-4, 0.0), (float("nan"), 0.0),   # |a| <= 0.001 -> 0
    (2.0, 0.5), (float("inf"), 0.0), (-float("inf"), -0.0),
])
def test_protected_inverse(x, expect):
    o32, o64 = one([node(INV), node(VAR, 0)], [], cols(x, 0))
    assert o32[0] == np.float32(expect) and o64[0] == expect
    eps = np.float32(0.001)
    above = np.nextafter(eps, np.float32(1))
    assert one([node(INV), node(VAR, 0)], [], cols(eps, 0))[0][0] == 0.0
    assert one([node(INV), node(VAR, 0)], [], cols(above, 0))[0][0] == np.float32(1) / above


def test_max_min_ignore_nan_and_order_signed_zeros():
    nan = float("nan")
    mx = [node(MAX), node(VAR, 0), node(VAR, 1)]
    mn = [node(MIN), node(VAR, 0), node(VAR, 1)]
    for prog, x0, x1, expect in [(mx, nan, 2.0, 2.0), (mx, 2.0, nan, 2.0),
                                 (mn, nan, -2.0, -2.0), (mn, -2.0, nan, -2.0)]:
        o32, o64 = one(prog, [], cols(x0, x1))
        assert o32[0] == expect and o64[0] == expect
    assert np.isnan(one(mx, [], cols(nan, nan))[0][0])
    # -0 orders below +0 in both operand orders; atan2 exposes the sign:
    # atan2(0, +0) = 0, atan2(0, -0) = pi
    for a, b in [(-0.0, 0.0), (0.0, -0.0)]:
        o32, o64 = one([node(ATAN2), node(CONST, 0), node(MAX), node(VAR, 0), node(VAR, 1)],
                       [0.0], cols(a, b))
        assert o32[0] == 0.0 and o64[0] == 0.0
        o32, o64 = one([node(ATAN2), node(CONST, 0), node(MIN), node(VAR, 0), node(VAR, 1)],
                       [0.0], cols(a, b))
        assert o32[0] == np.float32(PI) and o64[0] == PI
    o32, _ = one(mx, [], cols(-0.0, -0.0))
    assert o32[0] == 0.0 and np.signbit(o32[0])


def _ulps(g, ref):
    """Distance in float32 ulps of ref (same non-finite class required)."""
    g, ref = np.float32(g), np.float32(ref)
    if not np.isfinite(ref):
        return 0.0 if (g == ref or (np.isnan(g) and np.isnan(ref))) else np.inf
    return abs(float(g) - float(ref)) / float(np.spacing(np.abs(ref)) or np.float32(1e-45))


_UNARY64 = {ABS: abs, EXP: math.exp, SQ: lambda a: a * a, CUBE: lambda a: (a * a) * a,
            TANH: math.tanh, ATAN: math.atan,
            INV: lambda a: 1.0 / a if abs(a) > 0.0010000000474974513 else 0.0}


def _grid():
    g = np.concatenate([np.linspace(-12, 12, 241), np.geomspace(1e-6, 1e3, 60),
                        -np.geomspace(1e-6, 1e3, 60),
                        [0.0, -0.0, 88.5, 88.8, 100.0, -100.0, -103.0, 1e30, -1e30]])
    return g.astype(np.float32)


def _mp_exact(op, x):
    """The exact function value at float x, to 40 digits, by mpmath (an
    implementation independent of both C libraries)."""
    import mpmath
    mpmath.mp.dps = 40
    m = mpmath.mpf(x)
    if op == ABS:
        return abs(m)
    if op == EXP:
        return mpmath.exp(m)
    if op == INV:
        return 1 / m if abs(x) > 0.0010000000474974513 else mpmath.mpf(0)
    if op == SQ:
        return m * m
    if op == CUBE:
        return m * m * m
    if op == TANH:
        return mpmath.tanh(m)
    if op == ATAN:
        return mpmath.atan(m)
    return mpmath.cbrt(m) if x >= 0 else -mpmath.cbrt(-m)


def _err_ulps(got, exact, dtype):
    """|got - exact| in ulps of the correctly rounded result (dtype's ulp);
    infinite results must match exactly."""
    import mpmath
    with np.errstate(over="ignore"):
        r = dtype(float(exact))      # mpmath turns a value beyond float64 into inf
    if not np.isfinite(r):
        return 0.0 if got == r else np.inf
    if not np.isfinite(got):
        return np.inf
    sp = float(np.spacing(np.abs(r))) or float(np.finfo(dtype).smallest_subnormal)
    return float(abs(mpmath.mpf(float(got)) - exact) / sp)


# largest error allowed of the C library's double functions, in ulps of the
# exact value; the library documents errors of a few ulps, and these
# allowances sit just above the worst case seen on the grid below (cbrt 2.02,
# all others 1.14 or less)
_LIBM64_ULPS = {EXP: 1.0, TANH: 2.0, ATAN: 1.0, CBRT: 3.0}


@pytest.mark.parametrize("op", [ABS, EXP, INV, SQ, CUBE, TANH, ATAN, CBRT])
def test_wider_unary_within_library_error_of_exact(op):
    """Each function on a grid of float32 inputs against its exact value: the
    float32 path correctly rounded (half an ulp; every function rounds its
    exact value once), except cube, which rounds twice (1.5 ulp); the float64
    path within the C library's error."""
    x = _grid()
    X = np.ascontiguousarray(np.stack([x, np.zeros_like(x)]))
    o32, o64 = one([node(op), node(VAR, 0)], [], X)
    for i, xi in enumerate(x):
        ex = _mp_exact(op, float(xi))
        e32 = _err_ulps(o32[i], ex, np.float32)
        assert e32 <= (1.5 if op == CUBE else 0.5), (op, xi, o32[i], ex, e32)
        e64 = _err_ulps(o64[i], ex, np.float64)
        assert e64 <= _LIBM64_ULPS.get(op, 1.0), (op, xi, o64[i], ex, e64)


def test_wider_binary_against_exact_values():
    """max / min exactly (written out with comparisons here), atan2 correctly
    rounded in float32 and within one ulp in float64 of its exact value
    (mpmath), with the signs of zero results and the quadrant conventions at
    signed zeros and infinities."""
    import mpmath
    mpmath.mp.dps = 40
    v = np.array([0.0, -0.0, 1.0, -1.0, 0.5, -2.5, 3.0, 1e-6, -1e-6, 1e6, -7.25, float("inf"),
                  -float("inf")], dtype=np.float32)
    a, b = np.meshgrid(v, v, indexing="ij")
    X = np.ascontiguousarray(np.stack([a.ravel(), b.ravel()]))
    for op in (MAX, MIN, ATAN2):
        o32, o64 = one([node(op), node(VAR, 0), node(VAR, 1)], [], X)
        for i in range(X.shape[1]):
            x0, x1 = float(X[0, i]), float(X[1, i])
            if op == ATAN2:
                if math.isinf(x0) or math.isinf(x1) or x0 == 0.0:
                    # the conventions of C's atan2 at the axes and infinities
                    r64 = math.atan2(x0, x1)
                    assert o64[i] == r64 and np.signbit(o64[i]) == np.signbit(r64), (x0, x1)
                    assert np.float32(o64[i]) == o32[i], (x0, x1)
                    continue
                ex = mpmath.atan2(mpmath.mpf(x0), mpmath.mpf(x1))
                assert _err_ulps(o32[i], ex, np.float32) <= 0.5, (x0, x1, o32[i], ex)
                assert _err_ulps(o64[i], ex, np.float64) <= 1.0, (x0, x1, o64[i], ex)
                continue
            if x0 == x1:
                # equal operands: only the sign of zero can differ; -0 < +0
                neg0, neg1 = math.copysign(1, x0) < 0, math.copysign(1, x1) < 0
                r64 = (x1 if neg0 else x0) if op == MAX else (x0 if neg0 else x1)
            else:
                r64 = max(x0, x1) if op == MAX else min(x0, x1)
            assert o64[i] == r64 and np.signbit(o64[i]) == np.signbit(r64), (op, x0, x1, o64[i])
            assert o32[i] == np.float32(r64) and np.signbit(o32[i]) == np.signbit(r64), \
                (op, x0, x1, o32[i])


_LIBM = ctypes.CDLL(ctypes.util.find_library("m"))
_LIBM.cbrt.restype = ctypes.c_double
_LIBM.cbrt.argtypes = [ctypes.c_double]


def _tree_eval64(nodes, consts, xs, pos=0):
    """Recursive float64 evaluation, left to right, over the full function set."""
    w = int(nodes[pos])
    op, arg = w & 0xFF, w >> 8
    if op == VAR:
        return float(xs[arg]), pos + 1
    if op == CONST:
        return float(np.float32(consts[arg])), pos + 1
    a, pos = _tree_eval64(nodes, consts, xs, pos + 1)
    if oracle.ARITY[op] == 1:
        if op == CBRT:
            # the C library's cbrt, so that the comparison can be bit for bit:
            # this test pins the evaluation order, the grid test the function
            return _LIBM.cbrt(a), pos
        if op in _UNARY64:
            try:
                return _UNARY64[op](a), pos
            except OverflowError:
                return math.inf, pos
        if op == NEG:
            return -a, pos
        if op == SQRT:
            return math.sqrt(abs(a)), pos
        if op == LOG:
            return (math.log(abs(a)) if abs(a) > 0.0010000000474974513 else 0.0), pos
        return {SIN: math.sin, COS: math.cos, TAN: math.tan}[op](a), pos
    b, pos = _tree_eval64(nodes, consts, xs, pos)
    if op == ADD:
        return a + b, pos
    if op == SUB:
        return a - b, pos
    if op == MUL:
        return a * b, pos
    if op == DIV:
        return (a / b if abs(b) > 0.0010000000474974513 else 1.0), pos
    if op == ATAN2:
        return math.atan2(a, b), pos
    if math.isnan(a):
        return b, pos
    if math.isnan(b):
        return a, pos
    if a == b:
        neg_a = math.copysign(1, a) < 0
        return ((b if neg_a else a) if op == MAX else (a if neg_a else b)), pos
    return (max(a, b) if op == MAX else min(a, b)), pos


def test_bruteforce_wider_set_float64_bit_exact():
    """Every program of at most 4 nodes over the wider set, on 40 rows: the
    oracle's right-to-left stack scan equals a recursive left-to-right
    evaluation bit for bit in float64 (same libm, same operation order)."""
    terms = [node(VAR, 0), node(VAR, 1), node(CONST, 0)]
    progs = _enumerate(4, terms, [node(o) for o in (ABS, EXP, INV, SQ, CUBE, TANH, ATAN, CBRT)],
                       [node(o) for o in (MAX, MIN, ATAN2, SUB)])
    assert len(progs) > 2000
    rng = np.random.default_rng(8)
    X = rng.uniform(-4, 4, size=(2, 36)).astype(np.float32)
    X = np.ascontiguousarray(np.concatenate(
        [X, np.array([[0, -0.0, 5e-4, 0.5], [-0.0, 0, 1, 0.5]], np.float32)], axis=1))
    pop = oracle.from_programs([(p, [0.5]) for p in progs])
    got = oracle.evaluate_f64(pop, X)
    for i, p in enumerate(progs):
        for r in range(X.shape[1]):
            with np.errstate(all="ignore"):
                ref, end = _tree_eval64(p, [0.5], X[:, r])
            assert end == len(p)
            g = got[i, r]
            assert (np.isnan(ref) and np.isnan(g)) or (g == ref and np.signbit(g) == np.signbit(ref)), \
                (p, r, g, ref)
