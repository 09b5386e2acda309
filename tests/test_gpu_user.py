"""User-defined functions and losses on the GPU (Sec. V: custom function sets
and loss functions during GP runs) against the oracle.

The evaluation stream expands every user function in place (its arguments'
entries copied for each use, its own values on the stack above them), and a
user loss wraps the program: the row's target below it, the loss function on
(output, target) after it.  Definitions here use the correctly rounded
functions only, so every row must match the oracle's float32 evaluation bit
for bit, and every fitness within the float64 summation tolerance."""
import numpy as np
import pytest

import oracle
import synth
from _parity import check_fitness_exact, check_rows_exact, to_oracle

pytestmark = pytest.mark.gpu

n = oracle.node
A, B = n(oracle.VAR, 0), n(oracle.VAR, 1)
U1, U2 = oracle.USER1, oracle.USER2
C = lambda k: n(oracle.CONST, k)  # noqa: E731
DEFS = {
    U1 + 0: ([n(oracle.MUL), A, A], []),                                                      # a^2
    U1 + 1: ([n(oracle.SIN), n(oracle.ADD), n(oracle.MUL), C(0), A, C(1)], [1.5, 0.25]),       # sin(1.5 a + .25)
    U1 + 2: ([n(oracle.LOG), n(oracle.ADD), C(0), n(oracle.MUL), A, A], [1.0]),               # log(1 + a^2)
    U2 + 0: ([n(oracle.SQRT), n(oracle.ADD), n(oracle.MUL), A, A, n(oracle.MUL), B, B], []),  # hypot
    U2 + 1: ([n(oracle.DIV), n(oracle.SUB), A, B, n(oracle.ADD), C(0), n(oracle.MUL), A, B], [1.0]),
    # a deep one: six values on its own stack
    U2 + 2: ([n(oracle.ADD), n(oracle.MUL), n(oracle.ADD), n(oracle.SUB), n(oracle.ADD), A, B, A, B, A, B], []),
    # pseudo-Huber loss sqrt(1 + (a - b)^2) - 1
    U2 + 3: ([n(oracle.SUB), n(oracle.SQRT), n(oracle.ADD), C(0), n(oracle.MUL), n(oracle.SUB), A, B,
              n(oracle.SUB), A, B, C(0)], [1.0]),
}
MASK = oracle.DEFAULT_FMASK | sum(1 << op for op in DEFS)


@pytest.fixture(scope="module")
def gp():
    import torch
    import paper_2110_11226_amd as gp
    torch.cuda.set_device(0)
    gp.set_launch_config(None)
    for op, (d, c) in DEFS.items():
        gp.register_function(op, d, c)
        oracle.set_user_function(op, d, c)
    yield gp
    for op in DEFS:
        gp.register_function(op)
        oracle.set_user_function(op)
    gp.set_launch_config(None)


def rows_exact(gp, host, X, label):
    import torch
    pop = gp.DevicePopulation(host, n_features=X.shape[0])
    out = gp.evaluate(pop, gp.DeviceDataset(X))
    torch.cuda.synchronize()
    ref = oracle.evaluate_f32(to_oracle(host), X, n_threads=8)
    return check_rows_exact(out.cpu().numpy(), ref, label)


@pytest.mark.parametrize("cfg", [None, (1, 0, 1, 1), (2, 2, 3, 2), (4, 8, 2, 4)])
def test_random_programs_with_user_functions_bit_exact(gp, cfg):
    X, _ = synth.pagie(20_000, seed=11240)
    host = gp.build_population(200, 2, "exact_len", min_len=1, max_len=150, max_consts=8, function_mask=MASK,
                               seed=31)
    ops = host.nodes & 0xFF
    assert all((ops == op).any() for op in DEFS)
    gp.set_launch_config(cfg)
    try:
        print(f"user functions: launch config {cfg}", flush=True)
        rows_exact(gp, host, X, f"user functions {cfg}")
    finally:
        gp.set_launch_config(None)


def test_user_function_at_the_deepest_stack(gp):
    """A program whose stack is 20 deep when it calls the six-deep user
    function: the expansion's values reach the last LDS slots."""
    X, _ = synth.pagie(5000, seed=11241)
    x0, x1 = n(oracle.VAR, 0), n(oracle.VAR, 1)
    prog = [n(oracle.ADD)] * 18 + [n(U2 + 2), x0, x1] + [x1] * 18
    assert oracle.check_program(prog, 2, 0) == (0, 20)
    progs = [(prog, []), ([n(U2 + 2), x0, x1], []), ([n(oracle.SUB)] * 18 + [n(U2 + 0), x1, x0] + [x0] * 18, [])]
    op = oracle.from_programs(progs)
    host = gp.HostPopulation(op.nodes, op.prog_off, op.consts, op.const_off, op.length)
    gp.validate_population(host, 2)
    for cfg in ((1, 0, 1, 1), (4, 2, 2, 4)):
        gp.set_launch_config(cfg)
        try:
            rows_exact(gp, host, X, f"deep user call {cfg}")
        finally:
            gp.set_launch_config(None)


@pytest.mark.parametrize("metric", ["user3", "user1"])
@pytest.mark.parametrize("weighted", [False, True])
def test_user_loss_fitness(gp, metric, weighted):
    import torch
    X, y = synth.pagie(300_000, seed=11242)
    w = np.random.default_rng(4).uniform(0, 2, size=y.shape[0]).astype(np.float32) if weighted else None
    host = gp.build_population(256, 2, "exact_len", min_len=1, max_len=120, function_mask=MASK, seed=41)
    pop = gp.DevicePopulation(host, n_features=2)
    fit = gp.fitness(pop, gp.DeviceDataset(X, y, w), metric)
    torch.cuda.synchronize()
    f32p, f64 = oracle.fitness(to_oracle(host), X, y, w, metric, n_threads=8)
    print(f"user loss {metric} weighted={weighted}", flush=True)
    check_fitness_exact(fit.cpu().numpy(), f32p, f64, label=f"user loss {metric} w={weighted}")


def test_generations_with_user_functions_and_loss(gp):
    """The graph-captured generational loop with user functions in the
    function set (generation and mutation draw them) and a user loss: the
    last population's fitness against the oracle."""
    X, y = synth.pagie(65_536, seed=11243)
    data = gp.DeviceDataset(X, y)
    init = dict(n_features=2, method="rhh", min_depth=2, max_depth=6, seed=2111, function_mask=MASK)
    ev = dict(p_crossover=0.7, p_subtree=0.1, p_hoist=0.05, p_point=0.1, p_point_replace=0.05, max_len=256)
    res = gp.run_generations(data, 3, 200, init, "user3", 20, 0.01, ev, seed=7, use_graph=True)
    pop = res.population
    ops = pop.nodes & 0xFF
    assert ((ops >= U1) & (ops < U2 + 4)).any()
    f32p, f64 = oracle.fitness(to_oracle(pop), X, y, None, "user3", n_threads=8)
    check_fitness_exact(res.fitness, f32p, f64, label="generations with user functions")


def test_backward_rejects_user_functions_and_losses(gp):
    import torch
    X, y = synth.pagie(4096, seed=11244)
    data = gp.DeviceDataset(X, y)
    host = gp.build_population(32, 2, "rhh", function_mask=MASK, seed=3)
    assert ((host.nodes & 0xFF) >= U1).any()
    pop = gp.DevicePopulation(host, n_features=2)
    with pytest.raises(gp.GPError, match="user functions"):
        gp.fitness_backward(pop, data, "mse")
    plain = gp.DevicePopulation(gp.build_population(32, 2, "rhh", seed=3), n_features=2)
    with pytest.raises(gp.GPError, match="user losses"):
        gp.fitness_backward(plain, data, "user3")
    grad = gp.fitness_backward(plain, data, "mse")   # still works without user functions in it
    torch.cuda.synchronize()
    assert np.isfinite(grad.cpu().numpy()).any()
