"""GPU parity of gp_fitness_backward (d fitness / d program constants; not in
the paper) against the oracle's float64 reverse mode, whose own pins are a
closed form and central finite differences (tests/test_oracle_grad.py).

The GPU runs forward values, tape and adjoints in float32.  Over functions
that both sides round correctly (the nine-function set: sin, cos and log by
gp_crmath.h on the device) its forward values are the oracle's float32 ones
bit for bit, so the reference is the oracle's reverse mode taken at the
float32 evaluation (its values and protected branches, the partials in
float64): only the float32 rounding of the reverse sweep separates the two.
The oracle estimates that rounding by Monte Carlo arithmetic: the spread of
its derivatives when every partial is perturbed by a relative +-2^-22, over
three seeds.

Tolerance, per constant k of a program, with scale = max_k |g_64[k]|:
    |g_gpu[k] - g_64[k]| <= 1e-4 |g_64[k]| + 10 spread[k] + 1e-6 scale,
where spread[k] is that constant's own Monte Carlo spread.  A constant whose
spread is below 2.5e-5 |g_64[k]| is thereby held to about 1e-4 relative on
its own derivative, however small it is next to its siblings'; the 1e-6
scale floor only absorbs the float32 rounding of the per-row terms in a sum
that cancels.  No program is excluded, except one whose derivative lies
beyond the float32 range.

With the wider set's tan, exp, tanh, atan, cbrt and atan2 (the device
library's, a few ulp from the oracle's) the reference is the float64
evaluation, and a program escapes (counted, reported) where that cannot
stand for float32: a protected predicate within its bound of the threshold,
or a chaotic fitness (its conditioning bound beyond the fitness tolerance).
"""
import os

import numpy as np
import pytest

import oracle
import synth
from _parity import CR_MASK, ParityStats, to_oracle

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


def oracle_reference(opop, X, y, w, metric, gscale=None, f32_tape=True):
    """float64 derivatives, their Monte Carlo spread, and the fitness
    conditioning of every program.  With f32_tape (programs whose functions
    are all correctly rounded on both sides, so the device's float32 forward
    values are the oracle's) the derivatives are taken at the float32
    evaluation, and the spread measures the float32 rounding of the reverse
    sweep alone."""
    ref, _ = oracle.grad_consts(opop, X, y, w, metric, gscale=gscale, n_threads=NT, f32_tape=f32_tape)
    spread = np.zeros_like(ref)
    with np.errstate(invalid="ignore"):
        for seed in MC_SEEDS:
            gm, _ = oracle.grad_consts(opop, X, y, w, metric, gscale=gscale, n_threads=NT,
                                       mc_u=MC_U, mc_seed=seed, f32_tape=f32_tape)
            spread = np.fmax(spread, np.abs(gm - ref))
    cond = None if f32_tape else oracle.fitness(opop, X, y, w, metric, n_threads=NT, with_bound=True,
                                                exact=CR_MASK)
    return ref, spread, cond


def check_grads(host, g, ref, spread, cond, label):
    """Per-constant check; returns (programs checked, programs escaped) and
    records the constant counts (tight: spread within 2.5e-5 |g_64|).  cond
    (the oracle's fitness conditioning) is None for a float32-tape
    reference, which shares the device's forward values and branches."""
    if cond is None:
        fit_ok = np.ones(host.n_programs, bool)
    else:
        f32p, _, fbound, fnear = cond
        with np.errstate(invalid="ignore"):
            fit_ok = (np.asarray(fnear) == 0) & ((np.asarray(fbound) <= 1e-4 * np.abs(f32p))
                                                  | (np.asarray(fbound) == 0))
    big = np.finfo(np.float32).max
    checked = escaped = c_tight = c_spread = c_escaped = 0
    for p in range(host.n_programs):
        a, b = int(host.const_off[p]), int(host.const_off[p + 1])
        if a == b:
            continue
        r, sp = ref[a:b], spread[a:b]
        if not (fit_ok[p] and np.all(np.isfinite(r)) and np.all(np.isfinite(sp)) and np.all(np.abs(r) <= big)):
            escaped += 1
            c_escaped += b - a
            continue
        scale = np.max(np.abs(r))
        err = np.abs(g[a:b] - r)
        tol = GRAD_TOL * np.abs(r) + 10.0 * sp + 1e-6 * scale
        bad = ~(err <= tol)
        if bad.any():
            k = int(np.nonzero(bad)[0][0])
            raise AssertionError(f"{label}: program {p} constant {k}: gpu {g[a + k]!r} float64 {r[k]!r} "
                                 f"(spread {sp[k]:.3g}, scale {scale:.3g}); all: {g[a:b]} vs {r}")
        tight = sp <= SPREAD_TOL * np.abs(r)
        c_tight += int(tight.sum())
        c_spread += int((~tight).sum())
        checked += 1
    ParityStats(label, "gradients", checked, c_tight, c_spread, escaped).record()
    print(f"{label}: {checked} programs checked ({c_tight} constants held to 1e-4 of their own derivative, "
          f"{c_spread} to their Monte Carlo spread), {escaped} programs ({c_escaped} constants) escaped")
    return checked, escaped


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
    checked, escaped = check_grads(host, g, ref, spread, cond, f"{metric} w={weighted}")
    assert escaped == 0
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
    checked, escaped = check_grads(host, g, ref, spread, cond, f"forced {cfg}")
    assert escaped == 0
    fin = np.isfinite(fwd)
    assert np.allclose(fit_out[fin], fwd[fin], rtol=1e-6, atol=0)


def test_long_programs_float64_reverse_mode(gp):
    """Programs of 1-200 nodes over the nine-function set (the shape of the
    differentiation workload): every constant of every program."""
    N = 30_000
    X, y = synth.diff_target(N, seed=12)
    host = gp.build_population(160, 8, "exact_len", min_len=1, max_len=200, max_consts=16, seed=2115)
    g, _, _ = run_backward(gp, host, X, y, None, "mse", 8)
    ref, spread, cond = oracle_reference(to_oracle(host), X, y, None, "mse")
    checked, escaped = check_grads(host, g, ref, spread, cond, "long")
    assert escaped == 0


def test_programs_longer_than_4096_nodes(gp):
    """Programs of 4,500-8,401 nodes, beyond the adjoint's LDS tape and any
    fixed buffer: a sum chain of 4,200 constants (every derivative
    2 mean(yhat - y)) and random long programs over the correctly rounded
    set, every constant against the oracle's float32-tape reverse mode."""
    rng = np.random.default_rng(12)
    chain = []
    for k in range(4200):
        chain += [oracle.node(oracle.ADD), oracle.node(oracle.CONST, k)]
    chain.append(oracle.node(oracle.VAR, 0))
    rand = gp.build_population(6, 8, "exact_len", min_len=4500, max_len=6000, max_consts=16, seed=77)
    progs = [(chain, rng.uniform(-1e-3, 1e-3, size=4200).astype(np.float32))]
    for p in range(rand.n_programs):
        a, b = int(rand.prog_off[p]), int(rand.prog_off[p + 1])
        c, d = int(rand.const_off[p]), int(rand.const_off[p + 1])
        progs.append((rand.nodes[a:b], rand.consts[c:d]))
    op = oracle.from_programs(progs)
    host = gp.HostPopulation(op.nodes, op.prog_off, op.consts, op.const_off, op.length)
    gp.validate_population(host, 8)
    X, y = synth.diff_target(9_000, seed=14)
    print("adjoint: programs of 4,500-8,401 nodes", flush=True)
    g, _, _ = run_backward(gp, host, X, y, None, "mse", 8)
    ref, spread, cond = oracle_reference(op, X, y, None, "mse")
    checked, escaped = check_grads(host, g, ref, spread, cond, "longer than 4096")
    assert escaped == 0 and checked == host.n_programs


def test_correctly_rounded_function_set_all_programs(gp):
    # add, sub, mul, neg: every program is checked
    fmask = sum(1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL, oracle.NEG))
    N = 20_000
    X, y = synth.diff_target(N, seed=7)
    host = gp.build_population(128, 8, "exact_len", min_len=1, max_len=120, max_consts=16,
                               function_mask=fmask, seed=8)
    g, _, _ = run_backward(gp, host, X, y, None, "mse", 8)
    ref, spread, cond = oracle_reference(to_oracle(host), X, y, None, "mse")
    checked, escaped = check_grads(host, g, ref, spread, cond, "add/sub/mul/neg")
    assert escaped == 0 and checked == sum(int(host.const_off[p + 1] > host.const_off[p]) for p in range(128))


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
    # tan, exp, tanh, atan, cbrt and atan2 are the device library's: the
    # float64 reference with the fitness conditioning decides the escapes
    ref, spread, cond = oracle_reference(to_oracle(host), X, y, None, metric, f32_tape=False)
    checked, escaped = check_grads(host, g, ref, spread, cond, f"wide {metric}")
    assert checked >= (15 if metric == "pearson" else 40)
    fin = np.isfinite(fwd)
    assert np.array_equal(fin, np.isfinite(fit_out))
    assert np.allclose(fit_out[fin], fwd[fin], rtol=1e-6, atol=0)


def test_wider_correctly_rounded_set_all_programs(gp):
    # max, min, abs, square, cube with add / sub / mul / neg
    fmask = sum(1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL, oracle.NEG, oracle.MAX,
                                 oracle.MIN, oracle.ABS, oracle.SQ, oracle.CUBE))
    N = 20_000
    X, y = synth.diff_target(N, seed=17)
    host = gp.build_population(128, 8, "exact_len", min_len=1, max_len=60, max_consts=16,
                               function_mask=fmask, seed=18)
    g, _, _ = run_backward(gp, host, X, y, None, "mse", 8)
    ref, spread, cond = oracle_reference(to_oracle(host), X, y, None, "mse")
    checked, escaped = check_grads(host, g, ref, spread, cond, "wide correctly rounded")
    n_const = sum(int(host.const_off[p + 1] > host.const_off[p]) for p in range(128))
    # with a float32-tape reference a program escapes only when a derivative
    # lies beyond the float32 range (nested cubes and squares overflow)
    assert checked + escaped == n_const and escaped <= 0.05 * n_const


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


def test_full_size_differentiation_workload(gp):
    """1,048,576 rows x 8 features, 2048 programs with up to 16 constants:
    one backward launch for the whole population; 32 programs with
    constants drawn at random (8 of them with 150 nodes or more, no
    conditioning filter) checked constant by constant against float64
    reverse mode at the float32 evaluation over every row.  The Monte Carlo spread is taken on an
    evenly spaced eighth of the rows (a derivative is a mean over rows, so
    its float32 sensitivity has the same scale on a large sample)."""
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
    withc = np.nonzero(np.diff(host.const_off) > 0)[0]
    pick = rng.choice(withc, size=24, replace=False)
    longs = np.setdiff1d(withc[host.length[withc] >= 150], pick)
    pick = np.sort(np.concatenate([pick, rng.choice(longs, size=8, replace=False)]))
    sub = oracle.from_programs([(host.nodes[host.prog_off[p]:host.prog_off[p + 1]],
                                 host.consts[host.const_off[p]:host.const_off[p + 1]]) for p in pick])
    ref, _ = oracle.grad_consts(sub, X, y, None, "mse", n_threads=NT, f32_tape=True)
    idx = np.arange(0, N, 8)
    Xs, ys = np.ascontiguousarray(X[:, idx]), np.ascontiguousarray(y[idx])
    ref_s, _ = oracle.grad_consts(sub, Xs, ys, None, "mse", n_threads=NT, f32_tape=True)
    spread = np.zeros_like(ref)
    with np.errstate(invalid="ignore"):
        for seed in MC_SEEDS:
            gm, _ = oracle.grad_consts(sub, Xs, ys, None, "mse", n_threads=NT, mc_u=MC_U, mc_seed=seed,
                                       f32_tape=True)
            spread = np.fmax(spread, np.abs(gm - ref_s))
    gsub = np.concatenate([g[host.const_off[p]:host.const_off[p + 1]] for p in pick])
    hsub = gp.HostPopulation(sub.nodes, sub.prog_off, sub.consts, sub.const_off, sub.length)
    checked, escaped = check_grads(hsub, gsub, ref, spread, None, "diff-1M")
    print(f"differentiation workload: {checked} of {len(pick)} sampled programs checked, lengths "
          f"{sorted(host.length[pick].tolist())}")
    assert escaped == 0
