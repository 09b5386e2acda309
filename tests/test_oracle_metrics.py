"""Pins of the oracle's fitness metrics (Sec. III-C3) against closed forms,
special cases and library routines."""
import math

import numpy as np
import pytest

import oracle
from oracle import ADD, MUL, VAR, CONST, node


def const_prog(c):
    return ([node(CONST, 0)], [c])


def x0_prog():
    return ([node(VAR, 0)], [])


def fit(progs, X, y, w=None, metric="mse"):
    pop = oracle.from_programs(progs)
    return oracle.fitness(pop, X, y, w, metric)


@pytest.mark.parametrize("weighted", [False, True])
def test_constant_program_mse_is_variance_plus_bias(weighted):
    rng = np.random.default_rng(1)
    n = 5000
    X = rng.normal(size=(1, n)).astype(np.float32)
    y = rng.normal(2.0, 3.0, size=n).astype(np.float32)
    w = rng.uniform(0.5, 2.0, size=n).astype(np.float32) if weighted else None
    c = np.float32(0.75)
    f32p, f64 = fit([const_prog(c)], X, y, w, "mse")
    wd = np.ones(n) if w is None else w.astype(np.float64)
    yd = y.astype(np.float64)
    ybar = np.sum(wd * yd) / np.sum(wd)
    var = np.sum(wd * (yd - ybar) ** 2) / np.sum(wd)
    expect = var + (float(c) - ybar) ** 2
    assert abs(f32p[0] - expect) <= 1e-12 * expect
    assert abs(f64[0] - expect) <= 1e-12 * expect
    r32, _ = fit([const_prog(c)], X, y, w, "rmse")
    assert abs(r32[0] - math.sqrt(expect)) <= 1e-12 * math.sqrt(expect)


def test_shifted_target_mae_mse_exact():
    # y = x0 + d with d = +-0.5 exactly representable: MAE 0.5, MSE 0.25
    rng = np.random.default_rng(2)
    n = 4097
    x = (rng.integers(-64, 64, size=n) / 8.0).astype(np.float32)
    d = np.where(rng.random(n) < 0.5, 0.5, -0.5).astype(np.float32)
    y = x + d
    X = x[None, :]
    assert np.all(y.astype(np.float64) - x.astype(np.float64) == d)
    assert fit([x0_prog()], X, y, None, "mae")[0][0] == 0.5
    assert fit([x0_prog()], X, y, None, "mse")[0][0] == 0.25
    assert fit([x0_prog()], X, y, None, "rmse")[0][0] == 0.5


def test_zero_logit_log_loss_is_ln2():
    rng = np.random.default_rng(3)
    n = 1000
    X = rng.normal(size=(1, n)).astype(np.float32)
    y = (rng.random(n) < 0.3).astype(np.float32)
    f32p, f64 = fit([const_prog(0.0)], X, y, None, "logloss")
    assert abs(f32p[0] - math.log(2.0)) <= 1e-7       # float32 row loss, one rounding
    assert abs(f64[0] - math.log(2.0)) <= 1e-13       # 1000 float64 additions


def test_constant_logit_log_loss_closed_form_and_symmetry():
    rng = np.random.default_rng(4)
    n = 3000
    X = rng.normal(size=(1, n)).astype(np.float32)
    y = (rng.random(n) < 0.4).astype(np.float32)
    c = 1.25
    _, f64 = fit([const_prog(c)], X, y, None, "logloss")
    softplus = math.log1p(math.exp(c))
    expect = softplus - float(np.mean(y.astype(np.float64))) * c
    assert abs(f64[0] - expect) <= 1e-12
    # relabel y -> 1-y and negate the logit: same loss
    _, g64 = fit([const_prog(-c)], X, (1 - y).astype(np.float32), None, "logloss")
    assert abs(g64[0] - f64[0]) <= 1e-12


def test_pearson_special_cases():
    rng = np.random.default_rng(5)
    n = 2000
    x = rng.normal(size=n).astype(np.float32)
    X = x[None, :]
    y = (2 * x.astype(np.float64) + 1).astype(np.float32)
    f32p, f64 = fit([x0_prog(), const_prog(3.0)], X, y, None, "pearson")
    assert abs(f32p[0] - 1.0) < 1e-6
    assert f32p[1] == 0.0 and f64[1] == 0.0
    yn = (-3 * x.astype(np.float64)).astype(np.float32)
    assert abs(fit([x0_prog()], X, yn, None, "pearson")[0][0] - 1.0) < 1e-6


def test_pearson_matches_numpy_corrcoef():
    rng = np.random.default_rng(6)
    n = 3000
    X = rng.normal(size=(2, n)).astype(np.float32)
    y = rng.normal(size=n).astype(np.float32)
    prog = ([node(ADD), node(VAR, 0), node(MUL), node(VAR, 1), node(CONST, 0)], [0.5])
    f32p, _ = fit([prog], X, y, None, "pearson")
    yh = oracle.evaluate_f32(oracle.from_programs([prog]), X)[0]
    r = np.corrcoef(yh.astype(np.float64), y.astype(np.float64))[0, 1]
    assert abs(f32p[0] - abs(r)) < 1e-12


@pytest.mark.parametrize("metric", ["mae", "mse", "rmse", "logloss", "pearson"])
def test_integer_weights_equal_row_duplication(metric):
    rng = np.random.default_rng(7)
    n = 700
    X = rng.normal(size=(2, n)).astype(np.float32)
    if metric == "logloss":
        y = (rng.random(n) < 0.5).astype(np.float32)
    else:
        y = rng.normal(size=n).astype(np.float32)
    wi = rng.integers(1, 4, size=n)
    prog = ([node(MUL), node(VAR, 0), node(ADD), node(VAR, 1), node(CONST, 0)], [0.3])
    f_w, _ = fit([prog], X, y, wi.astype(np.float32), metric)
    Xd = np.ascontiguousarray(np.repeat(X, wi, axis=1))
    yd = np.repeat(y, wi)
    f_d, _ = fit([prog], Xd, yd, None, metric)
    assert abs(f_w[0] - f_d[0]) <= 1e-12 * max(1.0, abs(f_d[0]))


def test_nonfinite_propagates():
    X = np.array([[1.0, float("inf"), 2.0]], dtype=np.float32)
    y = np.zeros(3, np.float32)
    f32p, _ = fit([x0_prog()], X, y, None, "mse")
    assert np.isinf(f32p[0])
    X2 = np.array([[1.0, float("nan"), 2.0]], dtype=np.float32)
    assert np.isnan(fit([x0_prog()], X2, y, None, "mae")[0][0])
    # Pearson with a non-finite variance reads as 0 (no correlation)
    assert fit([x0_prog()], X2, np.array([1, 2, 3], np.float32), None, "pearson")[0][0] == 0.0


def test_pearson_constant_program_is_exactly_zero_with_weights():
    # a constant column has zero weighted variance in exact arithmetic, so
    # r = 0 exactly however the float64 mean rounds
    rng = np.random.default_rng(8)
    n = 20013
    X = rng.normal(size=(1, n)).astype(np.float32)
    y = rng.normal(size=n).astype(np.float32)
    w = rng.uniform(0.5, 1.5, size=n).astype(np.float32)
    for c in (0.1, 1.0 / 3.0, 123.456, -7.25e-3):
        f32p, f64 = fit([const_prog(c)], X, y, w, "pearson")
        assert f32p[0] == 0.0 and f64[0] == 0.0


# ---- Spearman: Pearson of the average-rank vectors (Sec. III-C3) ----

def _spearman_progs():
    from oracle import ADD, MUL, SIN, SQRT, NEG
    return [
        ([node(VAR, 0)], []),
        ([node(MUL), node(MUL), node(VAR, 0), node(VAR, 0), node(VAR, 0)], []),       # x0^3: monotone
        ([node(SIN), node(VAR, 1)], []),
        ([node(ADD), node(SQRT), node(VAR, 0), node(NEG), node(VAR, 1)], []),
        ([node(CONST, 0)], [0.5]),                                                       # constant
    ]


def test_spearman_matches_scipy_without_weights():
    from scipy.stats import spearmanr
    rng = np.random.default_rng(11)
    n = 3001
    X = rng.uniform(-2, 2, size=(2, n)).astype(np.float32)
    # y with ties (rounded to a coarse grid)
    y = np.round(rng.normal(size=n) * 4).astype(np.float32)
    pop = oracle.from_programs(_spearman_progs())
    f32p, f64 = oracle.fitness(pop, X, y, None, "spearman")
    for p in range(pop.n_programs - 1):
        v = oracle.evaluate_f64(pop, X)[p]
        expect = abs(spearmanr(v, y.astype(np.float64)).correlation)
        assert abs(f64[p] - expect) <= 1e-12, p
    assert f64[-1] == 0.0 and f32p[-1] == 0.0                                          # constant program


def test_spearman_invariant_under_monotone_maps_and_weight_scale():
    rng = np.random.default_rng(12)
    n = 2000
    X = rng.uniform(0.1, 3, size=(2, n)).astype(np.float32)
    y = rng.normal(size=n).astype(np.float32)
    pop = oracle.from_programs(_spearman_progs()[:2])                                 # x0 and x0^3
    _, f = oracle.fitness(pop, X, y, None, "spearman")
    assert f[0] == f[1]
    w = rng.uniform(0.5, 1.5, size=n).astype(np.float32)
    _, fa = oracle.fitness(pop, X, y, w, "spearman")
    _, fb = oracle.fitness(pop, X, y, (w * 4).astype(np.float32), "spearman")
    assert np.allclose(fa, fb, rtol=1e-12, atol=0)


def test_spearman_weighted_hand_example_with_ties():
    # values (1, 2, 2, 5) -> ranks (1, 2.5, 2.5, 4); y (10, 30, 20, 40) -> (1, 3, 2, 4)
    X = np.array([[1, 2, 2, 5]], dtype=np.float32)
    y = np.array([10, 30, 20, 40], dtype=np.float32)
    w = np.array([1, 2, 1, 2], dtype=np.float32)
    pop = oracle.from_programs([([node(VAR, 0)], [])])
    _, f = oracle.fitness(pop, X, y, w, "spearman")
    a = np.array([1, 2.5, 2.5, 4.0])
    b = np.array([1, 3, 2, 4.0])
    wd = w.astype(np.float64)
    ma, mb = np.sum(wd * a) / wd.sum(), np.sum(wd * b) / wd.sum()
    r = np.sum(wd * (a - ma) * (b - mb)) / np.sqrt(np.sum(wd * (a - ma) ** 2) * np.sum(wd * (b - mb) ** 2))
    assert abs(f[0] - abs(r)) <= 1e-15


def test_spearman_nan_is_nan():
    X = np.array([[1.0, np.nan, 3.0]], dtype=np.float32)
    y = np.array([1.0, 2.0, 3.0], dtype=np.float32)
    pop = oracle.from_programs([([node(VAR, 0)], [])])
    f32p, f64 = oracle.fitness(pop, X, y, None, "spearman")
    assert np.isnan(f32p[0]) and np.isnan(f64[0])


def test_spearman_nan_target_is_nan():
    # NaN has no rank: a NaN in the target makes every program's fitness NaN
    # (either sign of NaN, anywhere in the column), with a zero bound
    X = np.array([[1.0, 2.0, 3.0, 4.0]], dtype=np.float32)
    pop = oracle.from_programs([([node(VAR, 0)], []), ([node(CONST, 0)], [2.0])])
    for k in range(4):
        for nan in (np.float32(np.nan), -np.float32(np.nan)):
            y = np.array([1.0, 3.0, 2.0, 4.0], dtype=np.float32)
            y[k] = nan
            f32p, f64, fb, fn = oracle.fitness(pop, X, y, None, "spearman", with_bound=True)
            assert np.isnan(f32p).all() and np.isnan(f64).all(), (k, nan)
            assert (fb == 0.0).all()
    # without the NaN the same column is an ordinary rank correlation
    y = np.array([1.0, 3.0, 2.0, 4.0], dtype=np.float32)
    f32p, _ = oracle.fitness(pop, X, y, None, "spearman")
    assert abs(f32p[0] - 0.8) <= 1e-6 and f32p[1] == 0.0
