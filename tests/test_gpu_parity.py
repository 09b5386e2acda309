"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Shapes follow the paper's workloads: the Pagie polynomial on x, y ~ U[-5,5]
(Sec. IV-A), ramped-half-and-half and exact-length populations, a 28-feature
classification set (the Higgs column count, Sec. IV-B).  Sizes span several
tiles and chunks with ragged tails.

Every function of the benchmark set is correctly rounded on both sides (sin,
cos and log by gp_crmath.h on the device), so programs over it are checked
bit for bit on every row and their fitness within 1e-4 relative, with no row
or program excluded.  The wider set's tan, exp, tanh, atan, cbrt and atan2
are the device library's and are checked against the oracle's bound.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from _parity import CR_MASK, check_fitness, check_fitness_exact, check_rows, check_rows_exact, to_oracle

pytestmark = pytest.mark.gpu

NT = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def gp():
    import torch
    import paper_2110_11226_amd as gp
    torch.cuda.set_device(0)
    yield gp
    gp.set_launch_config(None)


def run_eval(gp, host, X, F, cfg=None):
    import torch
    gp.set_launch_config(cfg)
    try:
        pop = gp.DevicePopulation(host, n_features=F)
        data = gp.DeviceDataset(X)
        out = gp.evaluate(pop, data)
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        gp.set_launch_config(None)


def rows_exact(gp, host, X, F, cfg, label):
    got = run_eval(gp, host, X, F, cfg)
    ref = oracle.evaluate_f32(to_oracle(host), X, n_threads=NT)
    return check_rows_exact(got, ref, label)


def all_pairs(P, N):
    prog = np.repeat(np.arange(P, dtype=np.int32), N)
    row = np.tile(np.arange(N, dtype=np.int64), P)
    return prog, row


CONFIGS = [None, (1, 0, 1), (1, 2, 3), (2, 2, 2), (2, 8, 1), (4, 0, 5), (4, 2, 1), (4, 8, 2),
           (1, 2, 3, 1), (2, 0, 2, 2), (4, 8, 3, 1)]   # last: waves per block


@pytest.mark.parametrize("cfg", CONFIGS)
def test_evaluate_pagie_rhh_all_launch_configs(gp, cfg):
    N = 4096 + 77                                   # ragged tail
    X, _ = synth.pagie(N, seed=11227)
    host = gp.build_population(256, 2, "rhh", min_depth=2, max_depth=6, seed=2111)
    rows_exact(gp, host, X, 2, cfg, f"rhh cfg={cfg}")


@pytest.mark.parametrize("cfg", [None, (1, 2, 1), (4, 2, 3), (4, 0, 2)])
def test_evaluate_exact_length_up_to_200(gp, cfg):
    N = 3000
    X, _ = synth.pagie(N, seed=5)
    host = gp.build_population(96, 2, "exact_len", min_len=1, max_len=200, seed=2113)
    rows_exact(gp, host, X, 2, cfg, f"exact cfg={cfg}")


def test_evaluate_deep_stacks_bit_exact(gp):
    """Exact-length programs over 28 features fill the stack to its 20
    entries, so the slots held in LDS are read and written on most rows."""
    N = 1500
    X, _ = synth.higgs_like(N, seed=4)
    host = gp.build_population(64, 28, "exact_len", min_len=150, max_len=200, seed=91)
    for cfg in (None, (1, 0, 2), (2, 0, 1, 1)):
        rows_exact(gp, host, X, 28, cfg, f"deep cfg={cfg}")


def test_evaluate_correctly_rounded_ops_bit_exact(gp):
    # add, sub, mul, protected div, neg, protected sqrt are correctly rounded
    # on both sides: every row must be bit-identical, none excluded
    fmask = sum(1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL, oracle.DIV, oracle.NEG,
                                 oracle.SQRT))
    N = 5000
    X, _ = synth.diff_target(N, seed=9)
    host = gp.build_population(128, 8, "exact_len", min_len=1, max_len=200, function_mask=fmask,
                               seed=77)
    for cfg in (None, (1, 8, 2), (4, 0, 1), (2, 8, 7)):
        got = run_eval(gp, host, X, 8, cfg)
        ref = oracle.evaluate_f32(to_oracle(host), X, n_threads=NT)
        same = (got.view(np.uint32) == ref.view(np.uint32)) | (np.isnan(got) & np.isnan(ref))
        assert same.all(), (cfg, int((~same).sum()))


def test_evaluate_28_features(gp):
    N = 2500
    X, _ = synth.higgs_like(N, seed=3)
    host = gp.build_population(64, 28, "exact_len", min_len=1, max_len=200, seed=2114)
    rows_exact(gp, host, X, 28, None, "F=28")
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        run_eval(gp, host, X, 28, (4, 8, 1))    # 28 features do not fit 8 registers


def test_evaluate_edge_shapes(gp):
    N_list = [1, 2, 63, 64, 65, 255, 257, 1025]
    progs = [([oracle.node(oracle.VAR, 1)], []), ([oracle.node(oracle.CONST, 0)], [0.375]),
             ([oracle.node(oracle.ADD)] * 19 + [oracle.node(oracle.VAR, 0)] * 20, []),   # stack 20
             ([oracle.node(oracle.NEG), oracle.node(oracle.SIN), oracle.node(oracle.VAR, 0)], []),
             ([oracle.node(oracle.LOG), oracle.node(oracle.COS), oracle.node(oracle.VAR, 1)], [])]
    op = oracle.from_programs(progs)
    host = gp.HostPopulation(op.nodes, op.prog_off, op.consts, op.const_off, op.length)
    for N in N_list:
        X, _ = synth.pagie(N, seed=N)
        X[0, 0] = np.nan
        if N > 2:
            X[1, 1] = np.inf
        for cfg in (None, (1, 2, 1), (4, 0, 1)):
            rows_exact(gp, host, X, 2, cfg, f"N={N} cfg={cfg}")


def _fitness_case(gp, host, X, y, w, metric, F, cfg=None):
    import torch
    gp.set_launch_config(cfg)
    try:
        pop = gp.DevicePopulation(host, n_features=F)
        data = gp.DeviceDataset(X, y, w)
        fit = gp.fitness(pop, data, metric)
        torch.cuda.synchronize()
        got = fit.cpu().numpy()
    finally:
        gp.set_launch_config(None)
    ref = oracle.fitness(to_oracle(host), X, y, w, metric, n_threads=NT, with_bound=True, exact=CR_MASK)
    return (got,) + tuple(ref)


def _fitness_exact(gp, host, X, y, w, metric, F, cfg, label):
    import torch
    gp.set_launch_config(cfg)
    try:
        pop = gp.DevicePopulation(host, n_features=F)
        fit = gp.fitness(pop, gp.DeviceDataset(X, y, w), metric)
        torch.cuda.synchronize()
        got = fit.cpu().numpy()
    finally:
        gp.set_launch_config(None)
    f32p, f64 = oracle.fitness(to_oracle(host), X, y, w, metric, n_threads=NT)
    return check_fitness_exact(got, f32p, f64, label)


CR_FMASK = sum(1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL, oracle.DIV, oracle.NEG,
                                oracle.SQRT))


def _metric_data(metric, N, seed):
    if metric == "logloss":
        X, y = synth.higgs_like(N, seed=seed)
        return np.ascontiguousarray(X[:8]), y, 8
    X, y = synth.pagie(N, seed=seed)
    return X, y, 2


@pytest.mark.parametrize("metric", ["mae", "mse", "rmse", "logloss", "pearson"])
@pytest.mark.parametrize("weighted", [False, True])
def test_fitness_all_metrics_rhh(gp, metric, weighted):
    """Ramped half-and-half programs (depth 2-8) over the nine-function set:
    every program."""
    N = 20000 + 13
    X, y, F = _metric_data(metric, N, 11228)
    w = synth.weights(N) if weighted else None
    host = gp.build_population(300, F, "rhh", min_depth=2, max_depth=8, seed=31)
    for cfg in (None, (1, 8, 4), (4, 0, 3)):
        st = _fitness_exact(gp, host, X, y, w, metric, F, cfg, f"rhh {metric} w={weighted} cfg={cfg}")
        print(f"rhh {metric} weighted={weighted} cfg={cfg}: {st.checked} programs, "
              f"max rel err vs f64 {st.max_rel_err_f64:.2e}")


@pytest.mark.parametrize("metric", ["mae", "mse", "rmse", "logloss", "pearson"])
@pytest.mark.parametrize("weighted", [False, True])
def test_fitness_all_metrics_long_programs(gp, metric, weighted):
    """Programs of 1-200 nodes over the nine-function set: every program."""
    N = 20000 + 13
    X, y, F = _metric_data(metric, N, 11229)
    w = synth.weights(N) if weighted else None
    host = gp.build_population(200, F, "exact_len", min_len=1, max_len=200, seed=32)
    for cfg in (None, (2, 8, 4), (4, 0, 3)):
        _fitness_exact(gp, host, X, y, w, metric, F, cfg, f"long {metric} w={weighted} cfg={cfg}")


def test_fitness_rhh_pagie_small_config(gp):
    """The 4,096-row Pagie configuration: 256 programs, every row."""
    N = 4096
    X, y = synth.pagie(N, seed=11227)
    host = gp.build_population(256, 2, "rhh", min_depth=2, max_depth=6, seed=2111)
    rows_exact(gp, host, X, 2, None, "pagie-4K rows")
    _fitness_exact(gp, host, X, y, None, "mse", 2, None, "pagie-4K fitness")


def test_full_size_pagie_1m_rhh_all_programs(gp):
    """The 1,048,576-row Pagie configuration with 1,000 ramped half-and-half
    programs (depth 2-8) at the automatic launch configuration: every
    program's fitness over every row against the oracle."""
    N = 1_048_576
    X, y = synth.pagie(N, seed=11228)
    host = gp.build_population(1000, 2, "rhh", min_depth=2, max_depth=8, seed=2112)
    st = _fitness_exact(gp, host, X, y, None, "mse", 2, None, "pagie-1M fitness")
    print(f"pagie-1M: {st.checked} programs checked, none excluded, max rel err vs f64 "
          f"{st.max_rel_err_f64:.2e}")


def test_fitness_edge_cases(gp):
    # single row, single program, constant programs, zero weights on half
    progs = [([oracle.node(oracle.CONST, 0)], [0.5]), ([oracle.node(oracle.VAR, 0)], []),
             ([oracle.node(oracle.SUB), oracle.node(oracle.VAR, 0), oracle.node(oracle.VAR, 0)], [])]
    op = oracle.from_programs(progs)
    host = gp.HostPopulation(op.nodes, op.prog_off, op.consts, op.const_off, op.length)
    for N in (1, 3, 300):
        X, y = synth.pagie(N, seed=N + 100)
        w = synth.weights(N)
        w[::2] = 0.0
        if N == 1:
            w[0] = 1.0
        for metric in ("mse", "mae", "pearson", "rmse"):
            _fitness_exact(gp, host, X, y, w, metric, 2, None, f"edge N={N} {metric}")


def test_fitness_nonfinite_propagates(gp):
    N = 1000
    X, y = synth.pagie(N, seed=1)
    X[0, 10] = np.inf
    X[1, 20] = np.nan
    progs = [([oracle.node(oracle.VAR, 0)], []), ([oracle.node(oracle.VAR, 1)], []),
             ([oracle.node(oracle.SIN), oracle.node(oracle.VAR, 0)], [])]
    op = oracle.from_programs(progs)
    host = gp.HostPopulation(op.nodes, op.prog_off, op.consts, op.const_off, op.length)
    for metric in ("mse", "mae", "pearson"):
        _fitness_exact(gp, host, X, y, None, metric, 2, None, f"nonfinite {metric}")
    got, *_ = _fitness_case(gp, host, X, y, None, "mse", 2)
    assert np.isinf(got[0]) and np.isnan(got[1]) and np.isnan(got[2])


@pytest.mark.parametrize("metric,parsimony", [("mse", 0.0), ("mse", 1e-3), ("mse", 1e-2),
                                              ("pearson", 1e-2), ("logloss", 1e-3)])
def test_tournament_bit_exact(gp, metric, parsimony):
    import torch
    P = 1000
    rng = np.random.default_rng(3)
    fit = np.round(rng.normal(size=P), 2).astype(np.float32)     # many ties
    fit[rng.integers(0, P, 20)] = np.nan
    fit[rng.integers(0, P, 5)] = np.inf
    ln = rng.integers(1, 201, size=P).astype(np.int32)
    T = 1713
    for seed, gen in ((7, 0), (7, 1), (123456789012345, 19)):
        w = gp.tournament(torch.from_numpy(fit).cuda(), torch.from_numpy(ln).cuda(), metric,
                          parsimony, 20, T, seed, gen)
        ref = oracle.tournament(fit, ln, gp.larger_is_better(metric), parsimony, 20, T, seed, gen)
        assert np.array_equal(w.cpu().numpy(), ref)
    for k in (1, 2, 3, 4, 5, 64):
        w = gp.tournament(torch.from_numpy(fit).cuda(), torch.from_numpy(ln).cuda(), metric,
                          parsimony, k, 333, 5, 2)
        ref = oracle.tournament(fit, ln, gp.larger_is_better(metric), parsimony, k, 333, 5, 2)
        assert np.array_equal(w.cpu().numpy(), ref)


def test_tournament_on_gpu_fitness(gp):
    import torch
    N = 4096
    X, y = synth.pagie(N, seed=11227)
    host = gp.build_population(256, 2, "rhh", min_depth=2, max_depth=6, seed=2111)
    pop = gp.DevicePopulation(host, n_features=2)
    data = gp.DeviceDataset(X, y)
    fit = gp.fitness(pop, data, "mse")
    win = gp.tournament(fit, pop.length, "mse", 0.01, 20, 256, 99, 0)
    torch.cuda.synchronize()
    ref = oracle.tournament(fit.cpu().numpy(), host.length, False, 0.01, 20, 256, 99, 0)
    assert np.array_equal(win.cpu().numpy(), ref)


def random_sample(host, rng, k_random=24, k_long=8, long_min=150):
    """Programs drawn at random (no conditioning filter): k_random over the
    whole population and k_long more among those of long_min nodes or more."""
    P = host.n_programs
    pick = rng.choice(P, size=k_random, replace=False)
    longs = np.setdiff1d(np.nonzero(host.length >= long_min)[0], pick)
    pick = np.concatenate([pick, rng.choice(longs, size=min(k_long, len(longs)), replace=False)])
    return np.sort(pick)


def full_size_case(gp, X, y, host, F, metric, label, seed):
    """The full workload at the automatic launch configuration:
      1. every program's fitness over every row on the GPU; 32 programs
         drawn at random (8 of them with 150 nodes or more) against the
         oracle over every row;
      2. every program's fitness over the first 32,768 rows against the
         oracle;
      3. every program's outputs on 2,048 rows spread over the dataset, bit
         for bit."""
    import torch
    N = X.shape[1]
    pop = gp.DevicePopulation(host, n_features=F)
    data = gp.DeviceDataset(X, y)
    fit = gp.fitness(pop, data, metric)
    torch.cuda.synchronize()
    got = fit.cpu().numpy()
    assert got.shape == (host.n_programs,)
    rng = np.random.default_rng(seed)
    sample = random_sample(host, rng)
    sub = oracle.from_programs([(host.nodes[host.prog_off[p]:host.prog_off[p + 1]],
                                 host.consts[host.const_off[p]:host.const_off[p + 1]]) for p in sample])
    f32p, _ = oracle.fitness(sub, X, y, None, metric, n_threads=NT, with_f64=False)
    st = check_fitness_exact(got[sample], f32p, None, f"{label} full N, sampled programs")
    print(f"{label}: {st.checked} sampled programs over all {N} rows, lengths "
          f"{sorted(host.length[sample].tolist())}")
    # every program on the first 32,768 rows
    n2 = 32768
    X2, y2 = np.ascontiguousarray(X[:, :n2]), np.ascontiguousarray(y[:n2])
    fit2 = gp.fitness(pop, gp.DeviceDataset(X2, y2), metric)
    torch.cuda.synchronize()
    f32p, f64 = oracle.fitness(to_oracle(host), X2, y2, None, metric, n_threads=NT)
    st = check_fitness_exact(fit2.cpu().numpy(), f32p, f64, f"{label} all programs, {n2} rows")
    print(f"{label}: all {st.checked} programs over {n2} rows, max rel err vs f64 {st.max_rel_err_f64:.2e}")
    # every program's outputs on rows spread over the whole dataset
    rows = np.unique(np.concatenate([rng.integers(0, N, 2046), [0, N - 1]])).astype(np.int64)
    X3 = np.ascontiguousarray(X[:, rows])
    out = gp.evaluate(pop, gp.DeviceDataset(X3))
    torch.cuda.synchronize()
    ref = oracle.evaluate_f32(to_oracle(host), X3, n_threads=NT)
    st = check_rows_exact(out.cpu().numpy(), ref, f"{label} all programs, sampled rows")
    print(f"{label}: {st.checked} outputs (all programs x {len(rows)} rows) bit-exact")


def test_full_size_pagie_16m(gp):
    """The 16,777,216-row Pagie workload, 4096 exact-length programs of 1-200
    nodes, at the launch configuration the benchmark uses."""
    X, y = synth.pagie(16_777_216, seed=11229)
    host = gp.build_population(4096, 2, "exact_len", min_len=1, max_len=200, seed=2113)
    full_size_case(gp, X, y, host, 2, "mse", "pagie-16M", 0)


def test_full_size_higgs_like_logloss(gp):
    """The 11,000,000-row, 28-feature classification workload, 2000
    exact-length programs, log-loss."""
    X, y = synth.higgs_like(11_000_000, seed=11230)
    host = gp.build_population(2000, 28, "exact_len", min_len=1, max_len=200, seed=2114)
    full_size_case(gp, X, y, host, 28, "logloss", "higgs-11M", 1)


# ---- the wider function set (max, min, atan2, abs, exp, inv, sq, cube, tanh,
# atan, cbrt, next to the nine functions and tan) ----
WIDE_CR_FMASK = CR_MASK


@pytest.mark.parametrize("cfg", [None, (1, 0, 1), (2, 2, 2), (4, 2, 1), (4, 8, 3, 1), (2, 0, 2, 2)])
def test_evaluate_wider_set_rhh(gp, cfg):
    N = 4096 + 77
    X, _ = synth.pagie(N, seed=11227)
    host = gp.build_population(256, 2, "rhh", min_depth=2, max_depth=6,
                               function_mask=oracle.ALL_FMASK, seed=2117)
    got = run_eval(gp, host, X, 2, cfg)
    ra = oracle.evaluate_pairs(to_oracle(host), X, *all_pairs(256, N), n_threads=NT, exact=CR_MASK)
    st = check_rows(got, ra, f"wide cfg={cfg}")
    print(f"wide cfg={cfg}: {st.checked} rows checked ({st.tight} within the plain tolerance), "
          f"{st.escaped} with a predicate near its threshold")
    assert st.escaped < 0.01 * got.size


def test_evaluate_wider_correctly_rounded_bit_exact(gp):
    """max, min, abs, protected inverse, square and cube are IEEE operations
    (cube is two products in the same order on both sides): with the nine
    functions, every row is bit-identical."""
    N = 5000
    X, _ = synth.diff_target(N, seed=19)
    host = gp.build_population(128, 8, "exact_len", min_len=1, max_len=200,
                               function_mask=WIDE_CR_FMASK, seed=78)
    for cfg in (None, (1, 8, 2), (4, 0, 1), (2, 8, 7, 2)):
        got = run_eval(gp, host, X, 8, cfg)
        ref = oracle.evaluate_f32(to_oracle(host), X, n_threads=NT)
        same = (got.view(np.uint32) == ref.view(np.uint32)) | (np.isnan(got) & np.isnan(ref))
        assert same.all(), (cfg, int((~same).sum()))


def test_evaluate_wider_set_special_values(gp):
    """NaN operands of max / min, the sign of a zero max / min seen through
    atan2, the protected inverse at its threshold, exp overflow: bit for bit
    (each case is exact or a correctly rounded constant on both sides)."""
    n = oracle.node
    V0, V1, C0 = n(oracle.VAR, 0), n(oracle.VAR, 1), n(oracle.CONST, 0)
    progs = [([n(oracle.MAX), V0, V1], []), ([n(oracle.MIN), V0, V1], []),
             ([n(oracle.ATAN2), C0, n(oracle.MAX), V0, V1], [0.0]),
             ([n(oracle.ATAN2), C0, n(oracle.MIN), V0, V1], [0.0]),
             ([n(oracle.ATAN2), C0, n(oracle.MAX), V1, V0], [0.0]),
             ([n(oracle.ATAN2), C0, n(oracle.MIN), V1, V0], [0.0]),
             ([n(oracle.INV), V0], []), ([n(oracle.INV), V1], []), ([n(oracle.ABS), V0], []),
             ([n(oracle.CUBE), V0], []), ([n(oracle.SQ), V1], [])]
    op = oracle.from_programs(progs)
    host = gp.HostPopulation(op.nodes, op.prog_off, op.consts, op.const_off, op.length)
    eps = np.float32(0.001)
    vals = np.array([0.0, -0.0, np.nan, 1.0, -1.0, eps, -eps, np.nextafter(eps, np.float32(1)),
                     np.inf, -np.inf, 3e38], np.float32)
    a, b = np.meshgrid(vals, vals, indexing="ij")
    X = np.ascontiguousarray(np.stack([a.ravel(), b.ravel()]))
    got = run_eval(gp, host, X, 2, None)
    ref = oracle.evaluate_f32(op, X, n_threads=NT)
    same = (got.view(np.uint32) == ref.view(np.uint32)) | (np.isnan(got) & np.isnan(ref))
    bad = np.argwhere(~same)
    assert same.all(), [(int(p), float(X[0, r]), float(X[1, r]), float(got[p, r]), float(ref[p, r]))
                        for p, r in bad[:8]]
    # atan2 on the same grid: exact at zeros and infinities (C's conventions,
    # correctly rounded multiples of pi / 4), within 4 ulps elsewhere
    op = oracle.from_programs([([n(oracle.ATAN2), V0, V1], [])])
    host = gp.HostPopulation(op.nodes, op.prog_off, op.consts, op.const_off, op.length)
    got = run_eval(gp, host, X, 2, None)[0]
    ref = oracle.evaluate_f32(op, X, n_threads=NT)[0]
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    special = (X[0] == 0) | (X[1] == 0) | np.isinf(X[0]) | np.isinf(X[1])
    fin = ~np.isnan(ref)
    ex = special & fin
    assert np.array_equal(got[ex].view(np.uint32), ref[ex].view(np.uint32))
    gen = ~special & fin
    assert np.all(np.abs(got[gen] - ref[gen]) <= 4 * np.spacing(np.abs(ref[gen])))
    # exp overflows to +inf and underflows towards 0 like the oracle
    progs = [([n(oracle.EXP), V0], [])]
    op = oracle.from_programs(progs)
    host = gp.HostPopulation(op.nodes, op.prog_off, op.consts, op.const_off, op.length)
    X = np.ascontiguousarray(np.array([[100.0, 89.0, -100.0, -200.0, 0.0], [0.0] * 5], np.float32))
    got = run_eval(gp, host, X, 2, None)[0]
    assert np.isposinf(got[0]) and np.isposinf(got[1]) and got[4] == 1.0
    assert 0.0 <= got[2] < 1e-43 and got[3] == 0.0


@pytest.mark.parametrize("metric", ["mae", "mse", "logloss", "pearson"])
def test_fitness_wider_set_rhh(gp, metric):
    N = 20000 + 13
    X, y, F = _metric_data(metric, N, 5)
    host = gp.build_population(300, F, "rhh", min_depth=2, max_depth=7,
                               function_mask=oracle.ALL_FMASK, seed=2118)
    for cfg in (None, (1, 8, 4), (4, 0, 3, 2)):
        got, *ref = _fitness_case(gp, host, X, y, None, metric, F, cfg)
        st = check_fitness(got, *ref, f"wide {metric} cfg={cfg}")
        print(f"wide {metric} cfg={cfg}: {st.checked} checked ({st.tight} within the plain tolerance), "
              f"{st.escaped} escaped, max rel err vs f64 {st.max_rel_err_f64:.2e}")
        assert st.checked >= 0.8 * 300
