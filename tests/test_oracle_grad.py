"""Pins of the oracle's float64 reverse-mode constant gradients: a closed
form, and central finite differences (an independent method) on random
programs for every metric."""
import numpy as np
import pytest

import oracle
from oracle import MUL, SIN, ADD, VAR, CONST, node

import synth


def test_closed_form_mul_c_x0():
    rng = np.random.default_rng(0)
    n = 4000
    x = rng.uniform(-3, 3, size=n).astype(np.float32)
    X = x[None, :]
    y = (2.0 * x).astype(np.float32)
    w = rng.uniform(0.5, 1.5, size=n).astype(np.float32)
    c = np.float32(0.7)
    pop = oracle.from_programs([([node(MUL), node(CONST, 0), node(VAR, 0)], [c])])
    g, f = oracle.grad_consts(pop, X, y, w, "mse")
    wd, xd = w.astype(np.float64), x.astype(np.float64)
    expect = 2.0 * (float(c) - 2.0) * np.sum(wd * xd * xd) / np.sum(wd)
    assert abs(g[0] - expect) <= 1e-12 * abs(expect)


def test_closed_form_sin_cx():
    # d/dc mean (sin(c x) - y)^2 = mean 2 (sin(c x) - y) cos(c x) x
    rng = np.random.default_rng(1)
    n = 3000
    x = rng.uniform(-2, 2, size=n).astype(np.float32)
    y = rng.normal(size=n).astype(np.float32)
    c = np.float32(1.3)
    pop = oracle.from_programs([([node(SIN), node(MUL), node(CONST, 0), node(VAR, 0)], [c])])
    g, _ = oracle.grad_consts(pop, x[None, :], y, None, "mse")
    xd, yd = x.astype(np.float64), y.astype(np.float64)
    cx = float(c) * xd
    expect = np.mean(2 * (np.sin(cx) - yd) * np.cos(cx) * xd)
    assert abs(g[0] - expect) <= 1e-12 * abs(expect)


def _fd1(pop, X, y, w, metric, h):
    """Central differences of the float64 fitness, one constant at a time."""
    out = np.zeros(pop.consts.shape[0])
    for p in range(pop.n_programs):
        for k in range(int(pop.const_off[p]), int(pop.const_off[p + 1])):
            c0 = pop.consts[k]
            cp, cm = np.float32(c0 + h), np.float32(c0 - h)
            pop.consts[k] = cp
            fp = oracle.fitness(pop, X, y, w, metric)[1][p]
            pop.consts[k] = cm
            fm = oracle.fitness(pop, X, y, w, metric)[1][p]
            pop.consts[k] = c0
            out[k] = (fp - fm) / (float(cp) - float(cm))
    return out


def _fd(pop, X, y, w, metric, h=1e-3):
    """Central differences at h and h/2 combined by Richardson extrapolation
    (truncation error O(h^4) instead of O(h^2))."""
    d1 = _fd1(pop, X, y, w, metric, h)
    d2 = _fd1(pop, X, y, w, metric, h / 2)
    return (4.0 * d2 - d1) / 3.0


SMOOTH = sum(1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL, oracle.NEG, oracle.SIN,
                              oracle.COS))


@pytest.mark.parametrize("metric", ["mse", "rmse", "logloss", "pearson", "mae"])
def test_reverse_mode_matches_central_differences(metric):
    n = 512
    X, y = synth.diff_target(n, seed=3)
    if metric == "logloss":
        y = (y > np.median(y)).astype(np.float32)
    w = synth.weights(n, seed=4)
    pop = oracle.build_population(24, 8, "exact_len", min_len=3, max_len=40, fmask=SMOOTH,
                                  max_consts=16, seed=5)
    g, f = oracle.grad_consts(pop, X, y, w, metric)
    fd = _fd(pop, X, y, w, metric)
    checked = 0
    for p in range(pop.n_programs):
        a, b = int(pop.const_off[p]), int(pop.const_off[p + 1])
        if a == b:
            continue
        scale = max(np.max(np.abs(g[a:b])), 1e-3 * max(abs(f[p]), 1e-6))
        err = np.max(np.abs(g[a:b] - fd[a:b])) / scale
        if metric == "mae":
            # |.| has kinks where a row's residual crosses 0; FD straddling one
            # differs by O(w/n): accept that size
            assert err < 2e-2, (p, err)
        else:
            assert err < 1e-5, (p, err)
        checked += 1
    assert checked >= 10


def test_gradient_scale_and_const_free_programs():
    X, y = synth.diff_target(256, seed=6)
    progs = [([node(ADD), node(VAR, 0), node(VAR, 1)], []),
             ([node(MUL), node(CONST, 0), node(VAR, 2)], [0.5])]
    pop = oracle.from_programs(progs)
    g1, _ = oracle.grad_consts(pop, X, y, None, "mse")
    g2, _ = oracle.grad_consts(pop, X, y, None, "mse", gscale=np.array([1.0, -3.0]))
    assert g1.shape == (1,)
    assert abs(g2[0] + 3.0 * g1[0]) <= 1e-12 * abs(g1[0])


def test_monte_carlo_spread_matches_first_order_sensitivity():
    """Monte Carlo arithmetic estimate of float32 conditioning.

    One row of x1 / cos(c0 / x3) with y = 0 under MSE: the derivative is
    G = 2 x1^2 sin(t) / (x3 cos(t)^3), t = c0 / x3.  A relative error d on
    t moves it by (cot t + 3 tan t) t d to first order, which near a zero
    of cos dominates the few-u moves the other operations add.  Each
    perturbed run must show that move (in size) and the signs must vary."""
    from oracle import DIV, COS
    u = 2.0 ** -22
    c0 = np.float32(0.5)
    x3 = np.float32(0.5 / (np.pi / 2 - 2e-3))   # cos(t) near 2e-3, above the 0.001 guard
    X = np.array([[0.0], [1.0], [0.0], [x3]], dtype=np.float32)
    y = np.zeros(1, np.float32)
    prog = [node(DIV), node(VAR, 1), node(COS), node(DIV), node(CONST, 0), node(VAR, 3)]
    pop = oracle.from_programs([(prog, [c0])])
    g0, _ = oracle.grad_consts(pop, X, y, None, "mse")
    t = float(c0) / float(x3)
    closed = 2.0 * np.sin(t) / (float(x3) * np.cos(t) ** 3)
    assert abs(g0[0] - closed) <= 1e-12 * abs(closed)
    main = abs((1.0 / np.tan(t) + 3.0 * np.tan(t)) * t) * u
    assert main > 1000 * u
    signs = set()
    for seed in range(16):
        g, _ = oracle.grad_consts(pop, X, y, None, "mse", mc_u=u, mc_seed=seed)
        rel = (g[0] - g0[0]) / g0[0]
        assert abs(abs(rel) - main) <= 10 * u + 0.01 * main, (seed, rel, main)
        signs.add(rel > 0)
    assert signs == {True, False}
    # u = 0 perturbs nothing
    gz, _ = oracle.grad_consts(pop, X, y, None, "mse", mc_u=0.0, mc_seed=7)
    assert gz[0] == g0[0]


def test_monte_carlo_spread_small_when_well_conditioned():
    """c x0 against y = 2 x0: every row's term moves by a few u at most."""
    rng = np.random.default_rng(3)
    x = rng.uniform(1, 2, size=500).astype(np.float32)
    y = (2.0 * x).astype(np.float32)
    pop = oracle.from_programs([([node(MUL), node(CONST, 0), node(VAR, 0)], [0.7])])
    g0, _ = oracle.grad_consts(pop, x[None, :], y, None, "mse")
    u = 2.0 ** -22
    for seed in range(4):
        g, _ = oracle.grad_consts(pop, x[None, :], y, None, "mse", mc_u=u, mc_seed=seed)
        assert 0 < abs(g[0] - g0[0]) <= 8 * u * abs(g0[0])


# the wider function set: smooth everywhere (exp, tanh, atan, sq, cube) and
# smooth away from a measure-zero set (atan2 off the origin and branch cut,
# cbrt off 0, inv off its threshold, max / min / abs off their kinks)
SMOOTH_WIDE = sum(1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL, oracle.EXP, oracle.TANH,
                                   oracle.ATAN, oracle.SQ, oracle.CUBE))
KINKED_WIDE = sum(1 << o for o in (oracle.ADD, oracle.MUL, oracle.SIN, oracle.ATAN2, oracle.CBRT,
                                   oracle.INV, oracle.MAX, oracle.MIN, oracle.ABS))


@pytest.mark.parametrize("fmask,seed", [(SMOOTH_WIDE, 7), (KINKED_WIDE, 8)])
def test_reverse_mode_matches_central_differences_wider_set(fmask, seed):
    """Every partial of the wider set against Richardson central differences
    of the float64 fitness (MSE).  Where a program's rows cross a kink inside
    the difference stencil, the two disagree by the size of that row's share;
    such programs are allowed, but must stay a small minority."""
    n = 384
    X, y = synth.diff_target(n, seed=seed)
    w = synth.weights(n, seed=seed + 1)
    pop = oracle.build_population(48, 8, "exact_len", min_len=3, max_len=24, fmask=fmask,
                                  max_consts=16, seed=seed + 2)
    g, f = oracle.grad_consts(pop, X, y, w, "mse")
    fd = _fd(pop, X, y, w, "mse")
    checked = agree = 0
    for p in range(pop.n_programs):
        a, b = int(pop.const_off[p]), int(pop.const_off[p + 1])
        if a == b or not np.isfinite(f[p]) or not np.all(np.isfinite(g[a:b])) \
                or not np.all(np.isfinite(fd[a:b])):
            continue
        scale = max(np.max(np.abs(g[a:b])), 1e-3 * max(abs(f[p]), 1e-6))
        err = np.max(np.abs(g[a:b] - fd[a:b])) / scale
        checked += 1
        if err < 1e-5:
            agree += 1
        elif fmask == SMOOTH_WIDE:
            raise AssertionError((p, err))
    assert checked >= 12
    print(f"checked {checked}, agree {agree}")
    assert agree >= 0.8 * checked, (agree, checked)


# ---- the float32-tape mode: derivatives taken at the float32 evaluation ----

def test_f32_tape_equals_float64_when_float32_is_exact():
    """Small-integer data and constants keep every float32 sum and product
    exact, so the float32 and float64 evaluations coincide and the two modes
    must give the same derivatives bit for bit."""
    rng = np.random.default_rng(7)
    n = 500
    X = rng.integers(-3, 4, size=(3, n)).astype(np.float32)
    y = rng.integers(-20, 21, size=n).astype(np.float32)
    progs = []
    for _ in range(60):
        # a random expression tree over add/sub/mul with <= 6 leaves
        def tree(d):
            if d == 0 or rng.random() < 0.3:
                if rng.random() < 0.5:
                    return [node(VAR, int(rng.integers(0, 3)))]
                return [node(CONST, -1)]
            op = [oracle.ADD, oracle.SUB, oracle.MUL][int(rng.integers(0, 3))]
            return [node(op)] + tree(d - 1) + tree(d - 1)
        nodes = tree(3)
        k = 0
        consts = []
        for i, w in enumerate(nodes):
            if (w & 0xFF) == CONST:
                nodes[i] = node(CONST, k)
                consts.append(float(rng.integers(-2, 3)))
                k += 1
        progs.append((nodes, consts))
    pop = oracle.from_programs(progs)
    for metric in ("mse", "mae", "pearson"):
        g64, f64 = oracle.grad_consts(pop, X, y, None, metric)
        g32, f32 = oracle.grad_consts(pop, X, y, None, metric, f32_tape=True)
        assert np.array_equal(g64, g32), metric
        assert np.array_equal(f64, f32), metric


def test_f32_tape_closed_form_with_rounding():
    """mul(c, x0) against y = 2 x0: the derivative at the float32 evaluation
    is 2 mean((fl32(c x0) - y) x0), with the rounded products."""
    rng = np.random.default_rng(8)
    n = 5000
    x = rng.uniform(-3, 3, size=n).astype(np.float32)
    y = (2.0 * x).astype(np.float32)
    c = np.float32(0.7)
    pop = oracle.from_programs([([node(MUL), node(CONST, 0), node(VAR, 0)], [c])])
    g, f = oracle.grad_consts(pop, x[None, :], y, None, "mse", f32_tape=True)
    yh = (c * x).astype(np.float64)          # float32 products
    d = yh - y.astype(np.float64)
    assert abs(f[0] - np.mean(d * d)) <= 1e-12 * np.mean(d * d)
    expect = np.mean(2.0 * d * x.astype(np.float64))
    assert abs(g[0] - expect) <= 1e-12 * abs(expect)


def test_f32_tape_follows_float32_protected_branch():
    """x0 / (x1 * c): rows where the float32 product rounds to |p| <= 0.001
    while the exact product exceeds it take the protected arm (value 1,
    derivative 0) in the float32 evaluation, the division in float64."""
    thr = np.float32(0.001)
    # c one float above 1: for x1 just below 0.001 the exact product x1 c
    # can exceed 0.001 while its float32 rounding does not
    c = np.nextafter(np.float32(1.0), np.float32(2.0))
    cand = np.nextafter(thr, np.float32(0.0)) - np.arange(0, 64, dtype=np.float32) * np.float32(1e-12)
    cand = cand.astype(np.float32)
    prod32 = (cand * c).astype(np.float32)
    prod64 = cand.astype(np.float64) * np.float64(c)
    hit = np.nonzero((np.abs(prod32) <= thr) & (np.abs(prod64) > np.float64(thr)))[0]
    assert hit.size > 0
    x1 = cand[hit[:1]]
    X = np.ascontiguousarray(np.stack([np.float32([2.0]), x1]))
    y = np.float32([0.0])
    pop = oracle.from_programs([([node(oracle.DIV), node(VAR, 0), node(MUL), node(VAR, 1), node(CONST, 0)],
                                 [c])])
    g32, f32 = oracle.grad_consts(pop, X, y, None, "mse", f32_tape=True)
    g64, f64 = oracle.grad_consts(pop, X, y, None, "mse")
    assert g32[0] == 0.0 and f32[0] == 1.0      # protected arm: value 1, no dependence on c
    assert g64[0] != 0.0                        # the float64 evaluation divides


def test_long_program_closed_form():
    """A program of 8,401 nodes (beyond any fixed buffer): c0 + (c1 + (... +
    (c4199 + x0))), whose MSE gradient is 2 mean(yhat - y) for every
    constant."""
    rng = np.random.default_rng(12)
    n_c = 4200
    c = rng.uniform(-1e-3, 1e-3, size=n_c).astype(np.float32)
    prog = []
    for k in range(n_c):
        prog += [node(ADD), node(CONST, k)]
    prog.append(node(VAR, 0))
    assert len(prog) == 8401
    pop = oracle.from_programs([(prog, c)])
    X = rng.normal(size=(1, 300)).astype(np.float32)
    y = rng.normal(size=300).astype(np.float32)
    g, f = oracle.grad_consts(pop, X, y, None, "mse")
    yh = oracle.evaluate_f64(pop, X)[0]
    want = 2.0 * np.mean(yh - y.astype(np.float64))
    assert np.all(np.isfinite(g)) and np.allclose(g, want, rtol=1e-12, atol=1e-15)
    assert np.isclose(f[0], np.mean((yh - y) ** 2), rtol=1e-12)
