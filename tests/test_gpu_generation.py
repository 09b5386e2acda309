"""GPU tests of the batching layer: the autotuner (and its cache) and one
generation captured as a HIP graph (population upload, fitness, tournaments,
result download), replayed over generations whose populations differ.

A replay must give exactly what the plain entry points give on the same
population under the same launch configuration: gp_fitness (same kernels,
same summation order, so bit-identical) and gp_tournament with the same
seed and generation (bit-identical winners).  Eager library work runs
between replays, and every replay is checked."""
import os

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
    gp.autotune_clear()
    yield gp
    gp.set_launch_config(None)
    gp.autotune_clear()


def eager(gp, host, data, metric, parsimony, k, T, seed, generation, F):
    import torch
    pop = gp.DevicePopulation(host, n_features=F)
    fit = gp.fitness(pop, data, metric)
    win = gp.tournament(fit, pop.length, metric, parsimony, k, T, seed, generation)
    torch.cuda.synchronize()
    return fit.cpu().numpy(), win.cpu().numpy()


def populations(gp, P, F, n):
    """n populations of P programs with different total lengths."""
    out = []
    for g in range(n):
        if g % 2 == 0:
            out.append(gp.build_population(P, F, "rhh", min_depth=2, max_depth=3 + g, seed=100 + g))
        else:
            out.append(gp.build_population(P, F, "exact_len", min_len=1, max_len=40 * g, max_consts=8,
                                           seed=100 + g))
    return out


@pytest.mark.parametrize("metric", ["mse", "pearson", "logloss", "spearman"])
def test_graph_replays_match_plain_calls(gp, metric):
    P, N, F = 256, 70_001, 2
    X, y = synth.pagie(N, seed=11227)
    if metric == "logloss":
        y = (y > np.median(y)).astype(np.float32)
    w = synth.weights(N, seed=4) if metric in ("pearson", "spearman") else None
    data = gp.DeviceDataset(X, y, w)
    pops = populations(gp, P, F, 5)
    cap_nodes = max(int(p.nodes.shape[0]) for p in pops)
    cap_consts = max(int(p.consts.shape[0]) for p in pops)
    T, k, c, seed = 300, 20, 0.01, 77
    gen = gp.Generation(data, P, cap_nodes, cap_consts, metric, parsimony=c, tournament_size=k,
                        n_tournaments=T, seed=seed)
    try:
        for g, host in enumerate(pops):
            fit_g, win_g = gen.run(host, g)
            fit_e, win_e = eager(gp, host, data, metric, c, k, T, seed, g, F)
            assert np.array_equal(fit_g.view(np.uint32), fit_e.view(np.uint32)), (metric, g)
            assert np.array_equal(win_g, win_e), (metric, g)
            # and against the oracle's tournament on the same fitness array
            ow = oracle.tournament(fit_g, host.length, gp.larger_is_better(metric), c, k, T, seed, g)
            assert np.array_equal(win_g, ow), (metric, g)
        # a population replayed a second time gives the same results
        fit_a, win_a = gen.run(pops[1], 1)
        fit_b, win_b = gen.run(pops[1], 1)
        assert np.array_equal(fit_a.view(np.uint32), fit_b.view(np.uint32))
        assert np.array_equal(win_a, win_b)
    finally:
        gen.close()


def test_graph_spearman_in_several_batches(gp):
    """Spearman fitness captured with a working-set limit that splits the
    programs into six batches (the last one short): every replay equals the
    plain call under the same limit, bit for bit."""
    P, N, F = 256, 20_001, 2
    X, y = synth.pagie(N, seed=11227)
    data = gp.DeviceDataset(X, y)
    pops = populations(gp, P, F, 3)
    cap_nodes = max(int(p.nodes.shape[0]) for p in pops)
    cap_consts = max(int(p.consts.shape[0]) for p in pops)
    gp.set_spearman_workset(16 * N * 50)          # 50 programs a batch
    try:
        gen = gp.Generation(data, P, cap_nodes, cap_consts, "spearman", parsimony=0.0, tournament_size=7,
                            n_tournaments=P, seed=5)
        try:
            for g, host in enumerate(pops):
                fit_g, win_g = gen.run(host, g)
                fit_e, win_e = eager(gp, host, data, "spearman", 0.0, 7, P, 5, g, F)
                assert np.array_equal(fit_g.view(np.uint32), fit_e.view(np.uint32)), g
                assert np.array_equal(win_g, win_e), g
        finally:
            gen.close()
    finally:
        gp.set_spearman_workset(0)
    # and the batched result is the one-batch result
    fit_one, _ = eager(gp, pops[2], data, "spearman", 0.0, 7, P, 5, 2, F)
    assert np.array_equal(fit_g.view(np.uint32), fit_one.view(np.uint32))


def test_graph_fitness_matches_oracle(gp):
    P, N, F = 128, 20_000, 2
    X, y = synth.pagie(N, seed=11227)
    data = gp.DeviceDataset(X, y)
    host = gp.build_population(P, F, "rhh", min_depth=2, max_depth=6, function_mask=sum(
        1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL, oracle.DIV, oracle.SQRT, oracle.NEG)), seed=5)
    gen = gp.Generation(data, P, host.nodes.shape[0], host.consts.shape[0], "mse", tournament_size=5)
    try:
        fit, _ = gen.run(host, 0)
    finally:
        gen.close()
    f32p, f64 = oracle.fitness(to_oracle(host), X, y, None, "mse", n_threads=8)
    ok = np.isfinite(f32p)
    assert np.array_equal(np.isfinite(fit), ok)
    assert np.allclose(fit[ok], f32p[ok], rtol=1e-4, atol=0)


def test_graph_rejects_what_it_cannot_run(gp):
    P, N, F = 64, 5000, 2
    X, y = synth.pagie(N, seed=1)
    data = gp.DeviceDataset(X, y)
    small = gp.build_population(P, F, "rhh", min_depth=1, max_depth=2, seed=1)
    big = gp.build_population(P, F, "rhh", min_depth=5, max_depth=6, seed=2)
    gen = gp.Generation(data, P, small.nodes.shape[0], small.consts.shape[0], "mse")
    try:
        gen.run(small, 0)
        with pytest.raises(gp.GPError, match="BUFFER_TOO_SMALL"):
            gen.run(big, 1)
        # a function as a program's last node leaves it without operands
        bad = gp.HostPopulation(small.nodes.copy(), small.prog_off, small.consts, small.const_off, small.length)
        bad.nodes[int(small.prog_off[1]) - 1] = oracle.node(oracle.ADD)
        with pytest.raises(gp.GPError, match="INVALID_PROGRAM"):
            gen.run(bad, 1)
        # feature 7 of a 2-feature dataset
        bad = gp.HostPopulation(small.nodes.copy(), small.prog_off, small.consts, small.const_off, small.length)
        bad.nodes[int(small.prog_off[1]) - 1] = oracle.node(oracle.VAR, 7)
        with pytest.raises(gp.GPError, match="INVALID_PROGRAM"):
            gen.run(bad, 1)
        with pytest.raises(gp.GPError, match="INVALID_ARG"):
            gen.run(small, 2 ** 32)
        # still usable after the refusals
        f1, w1 = gen.run(small, 3)
        f2, w2 = eager(gp, small, data, "mse", 0.0, 20, P, 0, 3, F)
        assert np.array_equal(f1.view(np.uint32), f2.view(np.uint32)) and np.array_equal(w1, w2)
    finally:
        gen.close()
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.Generation(data, 0, 10, 0, "mse")
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.Generation(data, 4, 10, 0, 99)                  # no such metric


def test_autotune_cache_and_tuned_graph(gp, tmp_path):
    P, N, F = 512, 300_000, 2
    X, y = synth.pagie(N, seed=11228)
    data = gp.DeviceDataset(X, y)
    host = gp.build_population(P, F, "exact_len", min_len=1, max_len=100, seed=9)
    pop = gp.DevicePopulation(host, n_features=F)
    gp.autotune_clear()
    heur = gp.get_launch_config(F, N, P, "mse")
    best, ms = gp.autotune(pop, data, "mse", repeats=1)
    assert ms > 0
    assert gp.get_launch_config(F, N, P, "mse") == best
    # the metric's kernel is part of the key
    assert gp.get_launch_config(F, N, P, "logloss") == heur
    path = os.path.join(str(tmp_path), "tune.jsonl")
    gp.autotune_save(path)
    gp.autotune_clear()
    assert gp.get_launch_config(F, N, P, "mse") == heur
    gp.autotune_load(path)
    assert gp.get_launch_config(F, N, P, "mse") == best
    with open(path, "a") as f:
        f.write('{"arch": "gfx950", "n_cu": 1}\n')
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.autotune_load(path)
    # results under the tuned configuration agree with the heuristic's
    f_tuned = gp.fitness(pop, data, "mse").cpu().numpy()
    gp.set_launch_config(heur)
    try:
        f_heur = gp.fitness(pop, data, "mse").cpu().numpy()
    finally:
        gp.set_launch_config(None)
    ok = np.isfinite(f_heur)
    assert np.array_equal(np.isfinite(f_tuned), ok)
    assert np.allclose(f_tuned[ok], f_heur[ok], rtol=1e-6, atol=0)
    # a graph built with autotune and kernel timing
    gp.autotune_clear()
    gen = gp.Generation(data, P, host.nodes.shape[0], host.consts.shape[0], "mse", autotune=True,
                        time_kernel=True, seed=3)
    try:
        fit_g, win_g = gen.run(host, 0)
        cfg, kernel_ms, tuned_ms = gen.info()
        assert kernel_ms > 0 and tuned_ms > 0
        gp.set_launch_config(cfg)
        try:
            fit_e, win_e = eager(gp, host, data, "mse", 0.0, 20, P, 3, 0, F)
        finally:
            gp.set_launch_config(None)
        assert np.array_equal(fit_g.view(np.uint32), fit_e.view(np.uint32))
        assert np.array_equal(win_g, win_e)
        fit_g2, _ = gen.run(host, 1)
        assert np.array_equal(fit_g.view(np.uint32), fit_g2.view(np.uint32))
        t = gen.timing()
        print(f"tuned graph: {t}")
        assert t["kernel_ms"] > 0 and t["clock_ms"] > 0
        # events and clock stamps bracket the same kernel
        assert abs(t["kernel_ms"] - t["clock_ms"]) <= 0.2 * t["clock_ms"] + 0.05
    finally:
        gen.close()
        gp.autotune_clear()
