"""Pin of the oracle's conditioning bound (the part of the tolerance policy
that decides which rows are ill-conditioned): the first-order bound on how far
a program's value moves when every sin / cos / tan / log result is scaled by
(1 +- u) is checked against an independent experiment that perturbs those
results in a recursive float64 evaluation."""
import math

import numpy as np
import pytest

import oracle
from oracle import ARITY, CONST, VAR, ADD, SUB, MUL, DIV, NEG, LOG, SQRT, SIN, COS, TAN

import synth

TRANS = (LOG, SIN, COS, TAN)


def perturbed_value(nodes, consts, xs, signs, u):
    """Recursive float64 evaluation with transcendental node i's result scaled
    by (1 + signs[i] * u)."""
    def rec(i):
        w = int(nodes[i])
        op, arg = w & 0xFF, w >> 8
        if op == VAR:
            return float(xs[arg]), i + 1
        if op == CONST:
            return float(consts[arg]), i + 1
        a, j = rec(i + 1)
        if ARITY[op] == 1:
            if op == NEG:
                v = -a
            elif op == SQRT:
                v = math.sqrt(abs(a))
            elif op == LOG:
                v = math.log(abs(a)) if abs(a) > 0.0010000000474974513 else 0.0
            elif op == SIN:
                v = math.sin(a)
            elif op == COS:
                v = math.cos(a)
            else:
                v = math.tan(a)
            if op in TRANS:
                v *= 1.0 + signs[i] * u
            return v, j
        b, j = rec(j)
        if op == ADD:
            return a + b, j
        if op == SUB:
            return a - b, j
        if op == MUL:
            return a * b, j
        return (a / b if abs(b) > 0.0010000000474974513 else 1.0), j

    return rec(0)[0]


def test_single_transcendental_bound_is_tight():
    # value = 3 * sin(x0) + x1: the bound is exactly u |3 sin x0|
    nodes = [oracle.node(ADD), oracle.node(MUL), oracle.node(CONST, 0), oracle.node(SIN),
             oracle.node(VAR, 0), oracle.node(VAR, 1)]
    pop = oracle.from_programs([(nodes, [3.0])])
    X, _ = synth.pagie(200, seed=1)
    u = 1e-9
    ra = oracle.evaluate_pairs(pop, X, np.zeros(200, np.int32), np.arange(200), u=u)
    expect = u * np.abs(3.0 * np.sin(X[0].astype(np.float64)))
    assert np.allclose(ra.bound, expect, rtol=1e-12, atol=0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bound_dominates_perturbation_experiment(seed):
    fmask = oracle.DEFAULT_FMASK | (1 << TAN)
    pop = oracle.build_population(40, 2, "exact_len", min_len=2, max_len=60, fmask=fmask,
                                  seed=100 + seed)
    X, _ = synth.pagie(30, seed=seed)
    u = 1e-10
    rng = np.random.default_rng(seed)
    tight = 0
    checked = 0
    for p in range(pop.n_programs):
        nodes, consts = pop.program(p)
        ra = oracle.evaluate_pairs(pop, X, np.full(30, p, np.int32), np.arange(30), u=u)
        for r in range(30):
            if ra.near[r] or ra.flip[r] or not np.isfinite(ra.bound[r]) or not np.isfinite(ra.v64[r]):
                continue
            # the regime the tolerance policy works in: at its own allowance
            # the bound stays well below 1e-3 relative (amplification of a
            # perturbation up to ~2000); beyond that second-order terms are
            # not small, and such rows are excluded by the policy anyway
            if ra.bound[r] / u * oracle.ULP_ALLOWANCE > 1e-3 * max(1.0, abs(ra.v64[r])):
                continue
            base = perturbed_value(nodes, consts, X[:, r], np.zeros(len(nodes)), 0.0)
            # the experiment's own libm calls may round differently from the
            # oracle's C build by an ulp; it only ever compares with itself
            worst = 0.0
            for _ in range(24):
                s = rng.choice([-1.0, 1.0], size=len(nodes))
                d = abs(perturbed_value(nodes, consts, X[:, r], s, u) - base)
                worst = max(worst, d)
            # first order: every pattern stays inside the bound (slack for
            # second-order terms, O(u * amplification), and for the float64
            # rounding of the experiment, amplified the same way)
            slack = 2e-4 * ra.bound[r] + 1e-13 * max(1.0, abs(base))
            assert worst <= ra.bound[r] + slack, (p, r, worst, ra.bound[r])
            checked += 1
            if ra.bound[r] > 0 and worst >= 0.25 * ra.bound[r]:
                tight += 1
    assert checked > 500
    assert tight > 0.2 * checked      # the bound is not vacuous


def test_near_threshold_flag():
    # pdiv(1, x0 - c) with x0 - c straddling 0.001 by less than the bound of
    # an upstream sin: flagged as near
    nodes = [oracle.node(DIV), oracle.node(CONST, 0), oracle.node(SUB), oracle.node(SIN),
             oracle.node(VAR, 0), oracle.node(CONST, 1)]
    x = np.float32(0.5)
    c1 = np.float32(np.sin(np.float64(x)) - 0.001)      # sin(x) - c1 ~ 0.001
    pop = oracle.from_programs([(nodes, [1.0, c1])])
    X = np.array([[x], [0.0]], dtype=np.float32)
    ra = oracle.evaluate_pairs(pop, X, [0], [0])
    assert ra.near[0]
    X2 = np.array([[0.1], [0.0]], dtype=np.float32)
    assert not oracle.evaluate_pairs(pop, X2, [0], [0]).near[0]


def _metric64(metric, v, y, w):
    W = np.sum(w)
    if metric == "mae":
        return np.sum(w * np.abs(v - y)) / W
    if metric in ("mse", "rmse"):
        m = np.sum(w * (v - y) ** 2) / W
        return np.sqrt(m) if metric == "rmse" else m
    if metric == "logloss":
        return np.sum(w * (np.maximum(v, 0) - y * v + np.log1p(np.exp(-np.abs(v))))) / W
    a = v - np.sum(w * v) / W
    b = y - np.sum(w * y) / W
    return abs(np.sum(w * a * b) / np.sqrt(np.sum(w * a * a) * np.sum(w * b * b)))


@pytest.mark.parametrize("metric", ["mae", "mse", "rmse", "logloss", "pearson"])
def test_fitness_bound_dominates_row_displacements(metric):
    """The fitness-level bound is the metric's propagation of the row bounds:
    moving every row's value anywhere within its (pinned) bound moves the
    fitness by at most the fitness bound, and the worst-case signs reach it."""
    N = 400
    X, y = synth.pagie(N, seed=3)
    if metric == "logloss":
        y = (y > np.median(y)).astype(np.float32)
    w = synth.weights(N, seed=4)
    fmask = oracle.DEFAULT_FMASK | (1 << TAN)
    pop = oracle.build_population(30, 2, "exact_len", min_len=3, max_len=40, fmask=fmask, seed=77)
    u = 1e-7
    f32p, f64, fb, fn = oracle.fitness(pop, X, y, w, metric, with_bound=True, u=u)
    rng = np.random.default_rng(5)
    yd, wd = y.astype(np.float64), w.astype(np.float64)
    checked = 0
    for p in range(pop.n_programs):
        ra = oracle.evaluate_pairs(pop, X, np.full(N, p, np.int32), np.arange(N), u=u)
        v, E = ra.v32.astype(np.float64), ra.bound
        if fn[p] or not (np.all(np.isfinite(v)) and np.all(np.isfinite(E))) or not np.isfinite(fb[p]):
            continue
        if fb[p] == 0.0 or fb[p] > 1e-3 * max(abs(f32p[p]), 1e-30):
            continue   # constant programs; or outside the first-order regime
        F0 = _metric64(metric, v, yd, wd)
        for _ in range(10):
            s = rng.choice([-1.0, 1.0], size=N)
            F1 = _metric64(metric, v + s * E, yd, wd)
            assert abs(F1 - F0) <= fb[p] * (1 + 1e-3) + 1e-12 * abs(F0), (metric, p)
        checked += 1
        if metric == "logloss":
            # bounded with the loss's Lipschitz constant 1 while its slope
            # |sigmoid(v) - y| may be far smaller: domination only
            continue
        # worst-case signs: along the derivative of the metric
        h = 1e-6 * np.maximum(np.abs(v), 1.0)
        g = np.array([(_metric64(metric, v + h * (np.arange(N) == r), yd, wd) - F0) for r in range(0, N, 1)])
        F2 = _metric64(metric, v + np.sign(g) * E, yd, wd)
        assert abs(F2 - F0) >= 0.5 * fb[p], (metric, p, abs(F2 - F0), fb[p])
    assert checked >= 5


def test_spearman_bound_dominates_rank_changes():
    """Displacing every row within its bound reorders only rows whose
    intervals chain-overlap; the change of Spearman's |rho| stays inside the
    bound (recomputed with scipy's average ranks and numpy)."""
    from scipy.stats import rankdata
    N = 300
    X, y = synth.pagie(N, seed=8)
    w = synth.weights(N, seed=9)
    fmask = oracle.DEFAULT_FMASK | (1 << TAN)
    pop = oracle.build_population(30, 2, "exact_len", min_len=3, max_len=30, fmask=fmask, seed=81)
    u = 1e-5        # large: many near ties
    f32p, f64, fb, fn = oracle.fitness(pop, X, y, w, "spearman", with_bound=True, u=u)
    rng = np.random.default_rng(2)
    wd = w.astype(np.float64)
    rb = rankdata(y.astype(np.float64))

    def rho(v):
        ra = rankdata(v)
        ma, mb = np.sum(wd * ra) / wd.sum(), np.sum(wd * rb) / wd.sum()
        va, vb = np.sum(wd * (ra - ma) ** 2), np.sum(wd * (rb - mb) ** 2)
        return 0.0 if va == 0 or vb == 0 else abs(np.sum(wd * (ra - ma) * (rb - mb)) / np.sqrt(va * vb))
    nonzero = 0
    for p in range(pop.n_programs):
        ra_ = oracle.evaluate_pairs(pop, X, np.full(N, p, np.int32), np.arange(N), u=u)
        v, E = ra_.v32.astype(np.float64), ra_.bound
        if fn[p] or not (np.all(np.isfinite(v)) and np.all(np.isfinite(E))):
            continue
        R0 = rho(v)
        assert abs(R0 - f32p[p]) <= 1e-12
        for _ in range(20):
            R1 = rho(v + rng.uniform(-1, 1, size=N) * E)
            assert abs(R1 - R0) <= fb[p] * 1.05 + 1e-12, (p, abs(R1 - R0), fb[p])
        nonzero += fb[p] > 0
        if np.all(E == 0):
            assert fb[p] == 0.0       # exact values: ranks cannot differ
    assert nonzero >= 5
