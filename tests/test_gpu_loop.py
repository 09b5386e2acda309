"""GPU tests of the generational loop (Alg. 1; Sec. III-C order): the
graph-captured loop against the loop of plain calls (bit-identical fitness
sequences and populations), and every generation against the oracle given
the GPU's fitness arrays (tournament winners and offspring bit-exact,
fitness within the parity tolerance)."""
import numpy as np
import pytest

import oracle
import synth
from _parity import to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    import torch
    import paper_2110_11226_amd as gp
    torch.cuda.set_device(0)
    gp.set_launch_config(None)
    return gp


def record(store):
    def cb(log, pop, fit):
        store.append((log, gp_copy(pop), fit.copy()))
    return cb


def gp_copy(pop):
    import paper_2110_11226_amd as gp
    return gp.HostPopulation(pop.nodes.copy(), pop.prog_off.copy(), pop.consts.copy(), pop.const_off.copy(),
                             pop.length.copy())


INIT = dict(n_features=2, method="rhh", min_depth=2, max_depth=6, seed=2111)
EVOLVE = dict(p_crossover=0.7, p_subtree=0.1, p_hoist=0.05, p_point=0.1, p_point_replace=0.05, max_len=256)


def test_graph_loop_equals_plain_loop(gp):
    X, y = synth.pagie(65_536, seed=11228)
    data = gp.DeviceDataset(X, y)
    a, b = [], []
    ra = gp.run_generations(data, 4, 200, INIT, "mse", 20, 0.01, EVOLVE, seed=7, use_graph=True, callback=record(a))
    rb = gp.run_generations(data, 4, 200, INIT, "mse", 20, 0.01, EVOLVE, seed=7, use_graph=False,
                            callback=record(b))
    assert len(a) == len(b) == 5
    for (la, pa, fa), (lb, pb, fb) in zip(a, b):
        assert np.array_equal(fa.view(np.uint32), fb.view(np.uint32)), la.generation
        assert np.array_equal(pa.nodes, pb.nodes) and np.array_equal(pa.consts.view(np.uint32),
                                                                      pb.consts.view(np.uint32))
    assert np.array_equal(ra.fitness.view(np.uint32), rb.fitness.view(np.uint32))


def test_loop_against_oracle_each_generation(gp):
    N, P, G = 4096, 64, 3
    X, y = synth.pagie(N, seed=11227)
    data = gp.DeviceDataset(X, y)
    steps = []
    seed = 11
    gp.run_generations(data, G, P, INIT, "mse", 20, 0.01, EVOLVE, seed=seed, callback=record(steps))
    init = dict(INIT)
    init.pop("seed")
    ev = oracle.EvolveParams(**EVOLVE, seed=seed)
    oi = oracle.InitParams(n_features=2, method="rhh", min_depth=2, max_depth=6)
    # generation 0 is the initial population
    o0 = oracle.build_population(P, 2, "rhh", min_depth=2, max_depth=6, seed=2111)
    assert np.array_equal(steps[0][1].nodes, o0.nodes)
    for g in range(G):
        _, pop, fit = steps[g]
        opop = to_oracle(pop)
        f32p, f64 = oracle.fitness(opop, X, y, None, "mse", n_threads=8)
        # every function is correctly rounded on both sides: every program
        ok = np.isfinite(f32p)
        assert np.allclose(fit[ok], f32p[ok], rtol=1e-4, atol=0), g
        assert np.array_equal(np.isfinite(fit), np.isfinite(f32p))
        ops, ft, T = oracle.plan_generation(ev, P, g)
        win = oracle.tournament(fit, pop.length, False, 0.01, 20, T, seed, g)
        kids = oracle.mutate(ev, oi, opop, ops, ft, win, g)
        nxt = steps[g + 1][1]
        assert np.array_equal(kids.nodes, nxt.nodes), g
        assert np.array_equal(kids.consts.view(np.uint32), nxt.consts.view(np.uint32)), g
        assert np.array_equal(kids.length, nxt.length), g


def test_pagie_one_million_rows_twenty_generations(gp):
    """The 1,048,576-row loop shape: population 1000, RHH depth 2-8, twenty
    generations of crossover / subtree / hoist / point mutation."""
    import time
    X, y = synth.pagie(1_048_576, seed=11228)
    data = gp.DeviceDataset(X, y)
    init = dict(n_features=2, method="rhh", min_depth=2, max_depth=8, seed=2112)
    t0 = time.time()
    res = gp.run_generations(data, 20, 1000, init, "mse", 20, 0.01, EVOLVE, seed=2112, time_kernel=True)
    wall = time.time() - t0
    assert len(res.history) == 21
    gp.validate_population(res.population, 2)
    assert np.isfinite(min(h.best for h in res.history))
    assert all(h.kernel_ms > 0 for h in res.history)
    print(f"1M-row loop: 20 generations in {wall:.2f} s; best MSE {res.history[0].best:.4g} -> "
          f"{min(h.best for h in res.history):.4g}; kernel ms/gen "
          f"{np.mean([h.kernel_ms for h in res.history]):.2f}")


@pytest.mark.parametrize("init,metric", [
    (INIT, "mse"),
    (dict(n_features=2, method="exact_len", min_len=1, max_len=60, max_consts=6, function_mask=oracle.ALL_FMASK,
          seed=33), "pearson"),
])
def test_device_loop_equals_host_loop(gp, init, metric):
    """Every generation on the device (Evolution) against the graph loop with
    host genetic operations: bit-identical fitness in every generation and
    the same final population."""
    X, y = synth.pagie(20_000 + 17, seed=11229)
    data = gp.DeviceDataset(X, y)
    host_steps = []
    ra = gp.run_generations(data, 8, 256, init, metric, 20, 0.01, EVOLVE, seed=5, callback=record(host_steps))
    dev_fit = []
    rb = gp.run_generations(data, 8, 256, init, metric, 20, 0.01, EVOLVE, seed=5, device_loop=True,
                            callback=lambda log, pop, fit: dev_fit.append(fit.copy()))
    assert len(dev_fit) == len(host_steps) == 9
    for g, ((_, _, fa), fb) in enumerate(zip(host_steps, dev_fit)):
        assert np.array_equal(fa.view(np.uint32), fb.view(np.uint32)), g
    for la, lb in zip(ra.history, rb.history):
        assert la.total_nodes == lb.total_nodes and la.best_program == lb.best_program
    pa, pb = ra.population, rb.population
    assert np.array_equal(pa.nodes, pb.nodes) and np.array_equal(pa.prog_off, pb.prog_off)
    assert np.array_equal(pa.consts.view(np.uint32), pb.consts.view(np.uint32))
    assert np.array_equal(pa.const_off, pb.const_off) and np.array_equal(pa.length, pb.length)
    assert rb.launch_config == ra.launch_config


def test_device_loop_pagie_one_million_rows(gp):
    """The 1,048,576-row shape with the loop on the device: twenty
    generations, the evolution improving, and its time next to the host loop."""
    import time
    X, y = synth.pagie(1_048_576, seed=11228)
    data = gp.DeviceDataset(X, y)
    init = dict(n_features=2, method="rhh", min_depth=2, max_depth=8, seed=2112)
    t0 = time.time()
    rd = gp.run_generations(data, 20, 1000, init, "mse", 20, 0.01, EVOLVE, seed=2112, device_loop=True,
                            time_kernel=True)
    t_dev = time.time() - t0
    t0 = time.time()
    rh = gp.run_generations(data, 20, 1000, init, "mse", 20, 0.01, EVOLVE, seed=2112)
    t_host = time.time() - t0
    assert [h.best for h in rd.history] == [h.best for h in rh.history]
    gp.validate_population(rd.population, 2)
    assert rd.history[-2].kernel_ms > 0
    print(f"1M-row loop, 20 generations: device loop {t_dev:.3f} s, host-mutation loop {t_host:.3f} s; "
          f"best MSE {rd.history[0].best:.4g} -> {min(h.best for h in rd.history):.4g}")


def test_device_loop_limits(gp):
    X, y = synth.pagie(2000, seed=3)
    data = gp.DeviceDataset(X, y)
    pop = gp.build_population(32, 2, "rhh", seed=1)
    evo = gp.Evolution(data, pop, dict(n_features=2), dict(EVOLVE, seed=1), max_generations=3)
    try:
        evo.run(3)
        with pytest.raises(gp.GPError, match="INVALID_ARG"):
            evo.run(1)
        evo.evaluate()
        fit, nodes = evo.history()
        assert fit.shape == (4, 32) and nodes.shape == (4,)
        assert evo.info()[2] == 3
    finally:
        evo.close()
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.Evolution(data, pop, dict(n_features=3), dict(EVOLVE, seed=1))     # init features != data's


def test_spearman_in_every_loop_form(gp):
    """Spearman fitness (Sec. III-C3) in the plain loop, the captured
    generation graph and the device-resident loop: bit-identical fitness in
    every generation and the same final population."""
    X, y = synth.pagie(8192 + 5, seed=11230)
    data = gp.DeviceDataset(X, y)
    runs = []
    for kw in (dict(use_graph=False), dict(use_graph=True), dict(device_loop=True)):
        fits = []
        r = gp.run_generations(data, 4, 128, INIT, "spearman", 20, 0.01, EVOLVE, seed=21,
                               callback=lambda log, pop, fit: fits.append(fit.copy()), **kw)
        runs.append((r, fits))
    (r0, f0) = runs[0]
    assert all(np.isfinite(f).any() for f in f0)
    for r, f in runs[1:]:
        for g, (a, b) in enumerate(zip(f0, f)):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), g
        assert np.array_equal(r.population.nodes, r0.population.nodes)
        assert np.array_equal(r.population.consts.view(np.uint32), r0.population.consts.view(np.uint32))
    assert max(h.best for h in r0.history) > r0.history[0].best - 1e-12


@pytest.mark.parametrize("device_loop", [False, True])
def test_resume_from_checkpoint_continues_exactly(gp, device_loop, tmp_path):
    """Six generations in one run equal three, a checkpoint, and three more
    resumed from it (counter-based draws: the population and its generation
    number are the whole state)."""
    X, y = synth.pagie(16_384 + 3, seed=11231)
    data = gp.DeviceDataset(X, y)
    full = gp.run_generations(data, 6, 200, INIT, "mse", 20, 0.01, EVOLVE, seed=9, device_loop=device_loop)
    part = gp.run_generations(data, 3, 200, INIT, "mse", 20, 0.01, EVOLVE, seed=9, device_loop=device_loop)
    assert part.generation == 3
    path = tmp_path / "gen3.npz"
    gp.save_checkpoint(path, part.population, part.generation)
    pop, g, _ = gp.load_checkpoint(path)
    rest = gp.run_generations(data, 3, 200, INIT, "mse", 20, 0.01, EVOLVE, seed=9, device_loop=device_loop,
                              population=pop, first_generation=g)
    assert rest.generation == 6 and [h.generation for h in rest.history] == [3, 4, 5, 6]
    assert [h.best for h in rest.history] == [h.best for h in full.history[3:]]
    assert np.array_equal(rest.population.nodes, full.population.nodes)
    assert np.array_equal(rest.population.consts.view(np.uint32), full.population.consts.view(np.uint32))
    assert np.array_equal(rest.fitness.view(np.uint32), full.fitness.view(np.uint32))
    rest.write_history(tmp_path / "h.jsonl")
    import json
    rows = [json.loads(l) for l in open(tmp_path / "h.jsonl")]
    assert [r["generation"] for r in rows] == [3, 4, 5, 6]


def test_loop_with_constant_refinement(gp):
    """The differentiation workload's loop (8 features, programs with up to
    16 constants), smaller: in every generation the best 10% take 5 Adam
    steps on their constants before selection.  At generation 0 (the same
    programs in both runs) refinement only ever lowers a program's MSE, it
    lowers some, and the fitness selection sees is that of the constants
    kept."""
    X, y = synth.diff_target(65_536, seed=12)
    data = gp.DeviceDataset(X, y)
    init = dict(n_features=8, method="exact_len", min_len=1, max_len=40, max_consts=16, seed=2115)
    ev = dict(EVOLVE, max_len=64)
    plain, refined = [], []
    gp.run_generations(data, 3, 256, init, "mse", 20, 0.0, ev, seed=4, use_graph=False, callback=record(plain))
    res = gp.run_generations(data, 3, 256, init, "mse", 20, 0.0, ev, seed=4,
                             refine=dict(top=0.1, steps=5, lr=1e-2), callback=record(refined))
    f_plain, f_ref = plain[0][2], refined[0][2]
    same_nan = np.isnan(f_plain) == np.isnan(f_ref)
    assert same_nan.all()
    ok = ~np.isnan(f_plain)
    assert np.all(f_ref[ok] <= f_plain[ok])
    assert int((f_ref[ok] < f_plain[ok]).sum()) >= 5
    pop0 = refined[0][1]
    again = gp.fitness(gp.DevicePopulation(pop0, n_features=8), data, "mse").cpu().numpy()
    assert np.array_equal(again.view(np.uint32), f_ref.view(np.uint32))
    with pytest.raises(ValueError):
        gp.run_generations(data, 1, 16, init, "mse", refine=dict(top=0.1), device_loop=True)
    gp.validate_population(res.population, 8)


def test_classification_11m_rows_ten_generations_device_loop(gp):
    """The classification shape at full size: 11,000,000 rows x 28 features
    (the Higgs column count), 2,000 programs of 1-200 nodes, log-loss
    fitness, tournament size 20, ten generations on the device."""
    import time
    X, y = synth.higgs_like(11_000_000, seed=11230)
    data = gp.DeviceDataset(X, y)
    init = dict(n_features=28, method="exact_len", min_len=1, max_len=200, seed=2114)
    t0 = time.time()
    res = gp.run_generations(data, 10, 2000, init, "logloss", 20, 0.0, EVOLVE, seed=2114, device_loop=True)
    wall = time.time() - t0
    assert len(res.history) == 11 and res.generation == 10
    gp.validate_population(res.population, 28)
    best = [h.best for h in res.history]
    assert np.isfinite(best).all() and min(best[1:]) <= best[0]
    print(f"11M x 28 log-loss, 2000 programs: 10 generations in {wall:.1f} s; best {best[0]:.4f} -> {min(best):.4f}")


def test_differentiation_workload_loop_with_refinement_full_size(gp):
    """The differentiation shape at full size: 1,048,576 rows x 8 features,
    2,048 programs with up to 16 constants, MSE, two generations with 5
    Adam steps of constant refinement on the best 10% in each."""
    import time
    X, y = synth.diff_target(1_048_576, seed=11231)
    data = gp.DeviceDataset(X, y)
    init = dict(n_features=8, method="exact_len", min_len=1, max_len=200, max_consts=16, seed=2115)
    t0 = time.time()
    seen = []
    res = gp.run_generations(data, 2, 2048, init, "mse", 20, 0.0, EVOLVE, seed=5,
                             refine=dict(top=0.1, steps=5, lr=1e-2), callback=record(seen))
    wall = time.time() - t0
    assert len(res.history) == 3
    gp.validate_population(res.population, 8)
    # every logged fitness is that of the constants the population holds
    pop1, fit1 = seen[1][1], seen[1][2]
    again = gp.fitness(gp.DevicePopulation(pop1, n_features=8), data, "mse").cpu().numpy()
    assert np.array_equal(again.view(np.uint32), fit1.view(np.uint32))
    print(f"diff-1M, 2048 programs, refinement: 2 generations in {wall:.1f} s; best MSE "
          f"{res.history[0].best:.4g} -> {min(h.best for h in res.history):.4g}")
