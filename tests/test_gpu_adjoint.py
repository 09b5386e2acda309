"""GPU parity of gp_fitness_backward (d fitness / d program constants; not in
the paper) against the oracle's float64 reverse mode, whose own pins are a
closed form and central finite differences (tests/test_oracle_grad.py).

The GPU runs forward values, tape and adjoints in float32, so near a
singularity of the program (a zero of cos under a division, say) its
derivative can differ from the float64 one by far more than the forward
value does.  The oracle estimates that float32 conditioning by Monte Carlo
arithmetic: the spread of its derivatives when every operation is perturbed
by a relative +-2^-22 (about the error of a float32 transcendental), over
three seeds.

Tolerance, per program, with scale = max_k |g_64[k]|:
  * well-conditioned programs (no protected predicate near its threshold,
    derivative spread at most 2.5e-5 * scale):
        max_k |g_gpu[k] - g_64[k]| <= 1e-4 * scale;
  * every program whose fitness is well-conditioned (no protected predicate
    near its threshold, fitness bound within the fitness tolerance):
        max_k |g_gpu[k] - g_64[k]| <= 1e-4 * scale + 10 * max_k spread[k].
"""
import os

import numpy as np
import pytest

import oracle
import synth
from _parity import to_oracle

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)
GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def gp():
    import torch
    import paper_2110_11226_amd as gp
    torch.cuda.set_device(0)
    return gp


def run_backward(gp, host, X, y, w, metric, F, gscale=None):
    import torch
    pop = gp.DevicePopulation(host, n_features=F)
    data = gp.DeviceDataset(X, y, w)
    fit = torch.empty(host.n_programs, dtype=torch.float32, device="cuda")
    gs = None if gscale is None else torch.from_numpy(np.asarray(gscale, np.float32)).cuda()
    g = gp.fitness_backward(pop, data, metric, grad_fitness=gs, fitness_out=fit)
    fwd = gp.fitness(pop, data, metric)
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64), fit.cpu().numpy(), fwd.cpu().numpy()


MC_U = 2.0 ** -22
MC_SEEDS = (1, 2, 3)
SPREAD_TOL = 2.5e-5


def well_conditioned(f32p, f64, fbound, fnear):
    with np.errstate(invalid="ignore", divide="ignore"):
        return ((np.asarray(fnear) == 0) & (np.abs(f32p - f64) <= 1e-6 * np.abs(f64))
                & (fbound <= 1e-5 * np.abs(f32p)))


def oracle_reference(opop, X, y, w, metric, gscale=None):
    """float64 derivatives, their Monte Carlo spread, and the fitness
    conditioning of every program."""
    ref, _ = oracle.grad_consts(opop, X, y, w, metric, gscale=gscale, n_threads=NT)
    spread = np.zeros_like(ref)
    with np.errstate(invalid="ignore"):
        for seed in MC_SEEDS:
            gm, _ = oracle.grad_consts(opop, X, y, w, metric, gscale=gscale, n_threads=NT,
                                       mc_u=MC_U, mc_seed=seed)
            spread = np.fmax(spread, np.abs(gm - ref))
    cond = oracle.fitness(opop, X, y, w, metric, n_threads=NT, with_bound=True)
    return ref, spread, cond


def check_grads(host, g, ref, spread, cond, label):
    f32p, _, fbound, fnear = cond
    # a fitness whose own conditioning bound exceeds the fitness tolerance is
    # chaotic in float32 (e.g. sin of a cube that reaches 1e10 on some rows):
    # a few Monte Carlo samples of such a heavy-tailed sum do not bound its
    # derivative, so only the tight bar's exclusion applies there
    with np.errstate(invalid="ignore"):
        fit_ok = (np.asarray(fnear) == 0) & ((np.asarray(fbound) <= 1e-4 * np.abs(f32p))
                                              | (np.asarray(fbound) == 0))
    checked = ill = 0
    for p in range(host.n_programs):
        a, b = int(host.const_off[p]), int(host.const_off[p + 1])
        if a == b:
            continue
        r, sp = ref[a:b], spread[a:b]
        # a fitness or derivative beyond the float32 range (nested cubes
        # reaching 1e49, say) has no float32 value to compare with
        big = np.finfo(np.float32).max
        if not (np.all(np.isfinite(r)) and np.all(np.isfinite(sp)) and abs(f32p[p]) <= big
                and np.all(np.abs(r) <= big)):
            ill += 1
            continue
        scale = np.max(np.abs(r))
        err = np.max(np.abs(g[a:b] - r))
        if fit_ok[p]:
            assert err <= GRAD_TOL * scale + 10.0 * np.max(sp), \
                (label, p, "beyond the conditioning estimate", err, np.max(sp), g[a:b], r)
        if not (fnear[p] == 0 and np.max(sp) <= SPREAD_TOL * scale):
            ill += 1
            continue
        if scale == 0.0:
            assert err == 0.0, (label, p)
        else:
            assert err <= GRAD_TOL * scale, (label, p, err / scale, g[a:b], r)
        checked += 1
    return checked, ill


def test_closed_form_mul_c_x0(gp):
    n = 100_000 + 17
    rng = np.random.default_rng(0)
    x = rng.uniform(-3, 3, size=n).astype(np.float32)
    X = np.ascontiguousarray(np.stack([x, x]))
    y = (2.0 * x).astype(np.float32)
    w = rng.uniform(0.5, 1.5, size=n).astype(np.float32)
    progs = [([oracle.node(oracle.MUL), oracle.node(oracle.CONST, 0), oracle.node(oracle.VAR, 0)], [c])
             for c in (0.7, -1.25, 2.0, 3.5)]
    op = oracle.from_programs(progs)
    host = gp.HostPopulation(op.nodes, op.prog_off, op.consts, op.const_off, op.length)
    g, _, _ = run_backward(gp, host, X, y, w, "mse", 2)
    wd, xd = w.astype(np.float64), x.astype(np.float64)
    m2 = np.sum(wd * xd * xd) / np.sum(wd)
    for i, c in enumerate((0.7, -1.25, 2.0, 3.5)):
        expect = 2.0 * (float(np.float32(c)) - 2.0) * m2
        assert abs(g[i] - expect) <= 1e-5 * max(abs(expect), 1e-3)


@pytest.mark.parametrize("metric", ["mse", "mae", "rmse", "logloss", "pearson"])
@pytest.mark.parametrize("weighted", [False, True])
def test_matches_float64_reverse_mode(gp, metric, weighted):
    """Ramped half-and-half programs (depth 2-6, up to 16 constants)."""
    N = 30_000 + 5
    X, y = synth.diff_target(N, seed=5)
    if metric == "logloss":
        y = (y > np.median(y)).astype(np.float32)
    w = synth.weights(N, seed=6) if weighted else None
    P = 384
    host = gp.build_population(P, 8, "rhh", min_depth=2, max_depth=6, max_consts=16, seed=2116)
    rng = np.random.default_rng(1)
    gscale = rng.uniform(0.5, 2.0, size=P)
    g, fit_out, fwd = run_backward(gp, host, X, y, w, metric, 8, gscale)
    ref, spread, cond = oracle_reference(to_oracle(host), X, y, w, metric, gscale)
    checked, ill = check_grads(host, g, ref, spread, cond, f"{metric} w={weighted}")
    print(f"{metric} weighted={weighted}: {checked} programs checked, {ill} ill-conditioned")
    # near-uncorrelated programs (|r| << 1) dominate the ill-conditioned Pearson set
    assert checked >= (15 if metric == "pearson" else 40)
    # fitness_out agrees with gp_fitness (different summation order only)
    fin = np.isfinite(fwd)
    assert np.array_equal(fin, np.isfinite(fit_out))
    assert np.allclose(fit_out[fin], fwd[fin], rtol=1e-6, atol=0)


@pytest.mark.parametrize("cfg", [(1, 0, 3), (2, 0, 2), (2, 8, 1), (4, 0, 5), (4, 2, 1)])
def test_forced_rows_per_lane(gp, cfg):
    """Each rows-per-lane variant of the adjoint (the automatic choice takes
    2 or 4 by occupancy), with features from memory and from registers, and
    row chunks that do not divide the rows evenly."""
    N = 20_000 + 3
    X, y = synth.diff_target(N, seed=15)
    F = 2 if cfg[1] == 2 else 8
    X = np.ascontiguousarray(X[:F])
    host = gp.build_population(192, F, "rhh", min_depth=2, max_depth=6, max_consts=16, seed=2117)
    gp.set_launch_config(cfg)
    try:
        g, fit_out, fwd = run_backward(gp, host, X, y, None, "mse", F)
    finally:
        gp.set_launch_config(None)
    ref, spread, cond = oracle_reference(to_oracle(host), X, y, None, "mse")
    checked, ill = check_grads(host, g, ref, spread, cond, f"forced {cfg}")
    assert checked >= 40
    fin = np.isfinite(fwd)
    assert np.allclose(fit_out[fin], fwd[fin], rtol=1e-6, atol=0)


def test_long_programs_float64_reverse_mode(gp):
    """Programs of 1-200 nodes over the nine-function set (the shape of the
    differentiation workload): many are chaotic in float32; the
    well-conditioned ones must meet the bar."""
    N = 30_000
    X, y = synth.diff_target(N, seed=12)
    host = gp.build_population(160, 8, "exact_len", min_len=1, max_len=200, max_consts=16, seed=2115)
    g, _, _ = run_backward(gp, host, X, y, None, "mse", 8)
    ref, spread, cond = oracle_reference(to_oracle(host), X, y, None, "mse")
    checked, ill = check_grads(host, g, ref, spread, cond, "long")
    print(f"long programs: {checked} checked, {ill} ill-conditioned")
    assert checked >= 20


def test_correctly_rounded_function_set_all_programs(gp):
    # no transcendental: every program is well-conditioned, all are checked
    fmask = sum(1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL, oracle.NEG))
    N = 20_000
    X, y = synth.diff_target(N, seed=7)
    host = gp.build_population(128, 8, "exact_len", min_len=1, max_len=120, max_consts=16,
                               function_mask=fmask, seed=8)
    g, _, _ = run_backward(gp, host, X, y, None, "mse", 8)
    ref, spread, (f32p, f64, fb, fn) = oracle_reference(to_oracle(host), X, y, None, "mse")
    checked, ill = check_grads(host, g, ref, spread, (f32p, f32p, fb, fn), "add/sub/mul/neg")
    assert ill == 0 and checked == sum(int(host.const_off[p + 1] > host.const_off[p]) for p in range(128))


@pytest.mark.parametrize("metric", ["mse", "pearson"])
def test_wider_function_set_float64_reverse_mode(gp, metric):
    """Ramped half-and-half programs over every function (the wider set's
    partials: max / min pass the derivative to the selected operand, atan2's
    two partials, abs, exp, protected inverse, square, cube, tanh, atan,
    cbrt)."""
    N = 30_000 + 5
    X, y = synth.diff_target(N, seed=15)
    P = 384
    host = gp.build_population(P, 8, "rhh", min_depth=2, max_depth=6, max_consts=16,
                               function_mask=oracle.ALL_FMASK, seed=2119)
    g, fit_out, fwd = run_backward(gp, host, X, y, None, metric, 8)
    ref, spread, cond = oracle_reference(to_oracle(host), X, y, None, metric)
    checked, ill = check_grads(host, g, ref, spread, cond, f"wide {metric}")
    print(f"wide {metric}: {checked} programs checked, {ill} ill-conditioned")
    assert checked >= (15 if metric == "pearson" else 40)
    fin = np.isfinite(fwd)
    assert np.array_equal(fin, np.isfinite(fit_out))
    assert np.allclose(fit_out[fin], fwd[fin], rtol=1e-6, atol=0)


def test_wider_correctly_rounded_set_all_programs(gp):
    # max, min, abs, square, cube with add / sub / mul / neg: no library
    # function, so every program is well-conditioned and all are checked
    fmask = sum(1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL, oracle.NEG, oracle.MAX,
                                 oracle.MIN, oracle.ABS, oracle.SQ, oracle.CUBE))
    N = 20_000
    X, y = synth.diff_target(N, seed=17)
    host = gp.build_population(128, 8, "exact_len", min_len=1, max_len=60, max_consts=16,
                               function_mask=fmask, seed=18)
    g, _, _ = run_backward(gp, host, X, y, None, "mse", 8)
    ref, spread, (f32p, f64, fb, fn) = oracle_reference(to_oracle(host), X, y, None, "mse")
    checked, ill = check_grads(host, g, ref, spread, (f32p, f32p, fb, fn), "wide correctly rounded")
    print(f"wide correctly rounded: {checked} checked, {ill} ill")
    n_const = sum(int(host.const_off[p + 1] > host.const_off[p]) for p in range(128))
    assert checked >= 0.9 * n_const


def test_more_than_sixteen_constants_and_edge_rows(gp):
    # 24 constants in one program (slots beyond 16 take the atomic path); row
    # counts that leave ragged tiles; a constant-free program
    terms = []
    for k in range(24):
        terms += [oracle.node(oracle.ADD), oracle.node(oracle.MUL), oracle.node(oracle.CONST, k),
                  oracle.node(oracle.VAR, k % 8)]
    prog = terms + [oracle.node(oracle.VAR, 0)]
    progs = [(prog, list(np.linspace(-1, 1, 24))),
             ([oracle.node(oracle.SIN), oracle.node(oracle.VAR, 1)], []),
             ([oracle.node(oracle.CONST, 0)], [0.25])]
    op = oracle.from_programs(progs)
    host = gp.HostPopulation(op.nodes, op.prog_off, op.consts, op.const_off, op.length)
    for N in (1, 63, 65, 4099):
        X, y = synth.diff_target(N, seed=N)
        g, _, _ = run_backward(gp, host, X, y, None, "mse", 8)
        ref, _ = oracle.grad_consts(op, X, y, None, "mse")
        scale = max(np.max(np.abs(ref)), 1e-30)
        assert np.max(np.abs(g - ref)) <= GRAD_TOL * scale, N


def test_autograd_function_and_refinement(gp):
    import torch
    N = 20_000
    X, y = synth.diff_target(N, seed=9)
    host = gp.build_population(64, 8, "exact_len", min_len=3, max_len=60, max_consts=16, seed=10)
    pop = gp.DevicePopulation(host, n_features=8)
    data = gp.DeviceDataset(X, y)
    c = pop.consts.clone().requires_grad_(True)
    fit = gp.GPFitness.apply(c, pop, data, "mse")
    wgt = torch.linspace(0.5, 1.5, 64, device="cuda")
    (fit * wgt).sum().backward()
    direct = gp.fitness_backward(pop, data, "mse", grad_fitness=wgt)
    torch.cuda.synchronize()
    assert torch.allclose(c.grad[:host.consts.shape[0]], direct, rtol=1e-6, atol=0)
    # the forward of the Function is gp_fitness
    assert torch.equal(fit.detach(), gp.fitness(pop, data, "mse"))
    # refinement never makes a program worse and improves some
    elite = torch.argsort(fit.detach())[:8].cpu().numpy()
    new_c, f0, f1 = gp.refine_constants(pop, data, "mse", elite, steps=5, lr=1e-2)
    torch.cuda.synchronize()
    f0, f1 = f0.cpu().numpy(), f1.cpu().numpy()
    ok = np.isfinite(f0)
    assert np.all(f1[ok] <= f0[ok])
    assert np.sum(f1[elite] < f0[elite]) >= 1
    # programs outside the elite keep their constants
    co = host.const_off
    keep = np.ones(host.consts.shape[0], bool)
    for p in elite:
        keep[co[p]:co[p + 1]] = False
    assert np.array_equal(new_c.cpu().numpy()[keep], host.consts[keep])


def test_full_size_differentiation_workload_sampled(gp):
    """1,048,576 rows x 8 features, 2048 programs with up to 16 constants:
    one backward launch for the whole population; sampled programs checked
    against float64 reverse mode over every row."""
    import torch
    N = 1_048_576
    X, y = synth.diff_target(N, seed=11231)
    host = gp.build_population(2048, 8, "exact_len", min_len=1, max_len=200, max_consts=16, seed=2115)
    pop = gp.DevicePopulation(host, n_features=8)
    data = gp.DeviceDataset(X, y)
    g = gp.fitness_backward(pop, data, "mse")
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(3)
    cand = rng.choice(np.nonzero(np.diff(host.const_off) > 0)[0], size=96, replace=False)
    sub = oracle.from_programs([(host.nodes[host.prog_off[p]:host.prog_off[p + 1]],
                                 host.consts[host.const_off[p]:host.const_off[p + 1]]) for p in cand])
    idx = np.linspace(0, N - 1, 16384).astype(np.int64)
    f32p, f64, fb, fn = oracle.fitness(sub, np.ascontiguousarray(X[:, idx]), y[idx], None, "mse",
                                       n_threads=NT, with_bound=True)
    ok = well_conditioned(f32p, f64, fb, fn) & (fb <= 1e-6 * np.abs(f32p))
    ref_s, spread_s, _ = oracle_reference(sub, np.ascontiguousarray(X[:, idx]), y[idx], None, "mse")
    for i in range(len(cand)):
        a, b = int(sub.const_off[i]), int(sub.const_off[i + 1])
        ok[i] &= bool(np.max(spread_s[a:b]) <= 0.1 * SPREAD_TOL * np.max(np.abs(ref_s[a:b])))
    good = list(np.nonzero(ok)[0][:6])
    assert len(good) >= 3
    pick = cand[good]
    sub = oracle.from_programs([(host.nodes[host.prog_off[p]:host.prog_off[p + 1]],
                                 host.consts[host.const_off[p]:host.const_off[p + 1]]) for p in pick])
    ref, _ = oracle.grad_consts(sub, X, y, None, "mse", n_threads=NT)
    k = 0
    for i, p in enumerate(pick):
        a, b = int(host.const_off[p]), int(host.const_off[p + 1])
        r = ref[k:k + (b - a)]
        k += b - a
        assert np.max(np.abs(g[a:b] - r)) <= GRAD_TOL * max(np.max(np.abs(r)), 1e-30), (p, g[a:b], r)
    print(f"differentiation workload: {len(pick)} sampled programs checked, lengths "
          f"{host.length[pick].tolist()}")
