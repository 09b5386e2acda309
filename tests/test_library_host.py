"""CPU tests of the library's host side: the C ABI loads and exports every
symbol include/gp.h declares, population generation is bit-exact with the
oracle's, validation agrees with the oracle's scan, and host-checked argument
errors are reported before anything reaches the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gp():
    import paper_2110_11226_amd as gp
    return gp


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(gp_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol(gp):
    lib = ctypes.CDLL(gp.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert gp.version().startswith("gp-mi355x")


CASES = [
    dict(method="rhh", min_depth=2, max_depth=6),
    dict(method="rhh", min_depth=0, max_depth=3),
    dict(method="full", min_depth=1, max_depth=8),
    dict(method="grow", min_depth=2, max_depth=10),
    dict(method="exact_len", min_len=1, max_len=200),
    dict(method="exact_len", min_len=1, max_len=200, max_consts=16),
    dict(method="exact_len", min_len=5, max_len=60,
         fmask=sum(1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL))),
    dict(method="rhh", min_depth=2, max_depth=5, const_lo=1.0, const_hi=0.0),
    dict(method="exact_len", min_len=30, max_len=30,
         fmask=sum(1 << o for o in (oracle.ADD, oracle.MUL, oracle.SIN, oracle.TAN))),
    # every function, and the wider set on its own
    dict(method="rhh", min_depth=2, max_depth=7, fmask=oracle.ALL_FMASK),
    dict(method="exact_len", min_len=1, max_len=150, max_consts=8, fmask=oracle.ALL_FMASK),
    dict(method="grow", min_depth=1, max_depth=9,
         fmask=sum(1 << o for o in (oracle.MAX, oracle.MIN, oracle.ATAN2, oracle.ABS, oracle.EXP,
                                    oracle.INV, oracle.SQ, oracle.CUBE, oracle.TANH, oracle.ATAN,
                                    oracle.CBRT))),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("n_features", [1, 2, 28])
def test_build_population_bit_exact_with_oracle(gp, case, n_features):
    kw = dict(case)
    fmask = kw.pop("fmask", oracle.DEFAULT_FMASK)
    a = gp.build_population(300, n_features, function_mask=fmask, seed=2024, **kw)
    b = oracle.build_population(300, n_features, fmask=fmask, seed=2024, **kw)
    assert np.array_equal(a.nodes, b.nodes)
    assert np.array_equal(a.consts.view(np.uint32), b.consts.view(np.uint32))
    assert np.array_equal(a.prog_off, b.prog_off)
    assert np.array_equal(a.const_off, b.const_off)
    assert np.array_equal(a.length, b.length)


def test_build_population_errors(gp):
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.build_population(10, 2, "rhh", min_depth=3, max_depth=2)
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.build_population(10, 2, "exact_len", min_len=0)
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.build_population(10, 0, "rhh")
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.build_population(10, 2, "rhh", function_mask=1 << 23)


def test_validate_matches_oracle_on_mutated_programs(gp):
    rng = np.random.default_rng(0)
    base = gp.build_population(400, 3, "exact_len", min_len=1, max_len=60, max_consts=4, seed=5)
    nodes = base.nodes.copy()
    # corrupt one node in about half the programs
    for p in range(base.n_programs):
        if rng.random() < 0.5:
            i = int(base.prog_off[p] + rng.integers(0, base.length[p]))
            op = int(rng.integers(0, 24))
            arg = int(rng.integers(0, 6))
            nodes[i] = op | (arg << 8)
    expected_codes = {1: -2, 2: -2, 3: -3, 4: -2, 5: -2, 6: -2}
    for p in range(base.n_programs):
        a, b = int(base.prog_off[p]), int(base.prog_off[p + 1])
        one = gp.HostPopulation(nodes[a:b], np.array([0, b - a], np.int64),
                                base.consts[base.const_off[p]:base.const_off[p + 1]],
                                np.array([0, base.const_off[p + 1] - base.const_off[p]], np.int64),
                                np.array([b - a], np.int32))
        rc, h = oracle.check_program(nodes[a:b], 3, int(base.const_off[p + 1] - base.const_off[p]))
        if rc == 0:
            assert gp.validate_population(one, 3)[0] == h
        else:
            with pytest.raises(gp.GPError) as ei:
                gp.validate_population(one, 3)
            assert ei.value.status == expected_codes[rc]


def test_validate_stack_limit(gp):
    def prog(nodes):
        n = len(nodes)
        return gp.HostPopulation(np.array(nodes, np.uint32), np.array([0, n], np.int64),
                                 np.zeros(0, np.float32), np.array([0, 0], np.int64),
                                 np.array([n], np.int32))
    ok = [oracle.node(oracle.ADD)] * 19 + [oracle.node(oracle.VAR, 0)] * 20
    assert gp.validate_population(prog(ok), 1)[0] == 20
    over = [oracle.node(oracle.ADD)] * 20 + [oracle.node(oracle.VAR, 0)] * 21
    with pytest.raises(gp.GPError, match="STACK_OVERFLOW"):
        gp.validate_population(prog(over), 1)


def test_device_entry_points_reject_bad_arguments_before_launch(gp):
    from paper_2110_11226_amd import _binding as B
    # NULL population / dataset / outputs are rejected on the host
    assert B._fitness(None, None, 1, None, None) == -1
    assert B._evaluate(None, None, None, None) == -1
    pv = B.PopulationDev(None, None, None, None, None, 3, 10, 5, 0)
    dv = B.DatasetDev(None, 0, 2, 0, None, None)
    assert B._fitness(ctypes.byref(pv), ctypes.byref(dv), 1, None, None) == -1
    # tournament argument checks
    assert B._tournament(None, None, 0, 1, 0.0, 20, 10, 0, 0, None, None) == -1
    assert B._tournament(None, None, 10, 1, 0.0, 0, 10, 0, 0, None, None) == -1
    assert B._tournament(None, None, 10, 9, 0.0, 2, 10, 0, 0, None, None) == -1
    assert B._tournament(None, None, 10, 1, 0.0, 2, 10, 0, 2 ** 33, None, None) == -1
    # unsupported metric
    assert B._fitness(ctypes.byref(pv), ctypes.byref(dv), 5, None, None) == -1
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.set_launch_config((3, 0, 1))
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.set_launch_config((4, 5, 1))
    gp.set_launch_config(None)
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.set_spearman_workset(-1)
    gp.set_spearman_workset(0)
    # the adjoint: programs beyond its reverse-walk links, and Spearman (no
    # derivative), are refused before any device work (the pointers are
    # placeholders, never read)
    fake = ctypes.c_void_p(256)
    pv = B.PopulationDev(fake, fake, None, fake, fake, 4, 40, (1 << 25) + 1, 0)
    dv = B.DatasetDev(fake, 100, 2, 100, fake, None)
    assert B._backward(ctypes.byref(pv), ctypes.byref(dv), 1, None, None, None, None) == -1
    assert "2^25" in B._last_error().decode()
    pv.max_len = 50
    assert B._backward(ctypes.byref(pv), ctypes.byref(dv), 5, None, None, None, None) == -6
    assert "Spearman" in B._last_error().decode()


def test_metric_direction(gp):
    assert [gp.larger_is_better(m) for m in ("mae", "mse", "rmse", "logloss", "pearson", "spearman")] == \
        [False, False, False, False, True, True]


MUT_CASES = [
    dict(F=1, method="rhh", max_consts=0, p_point_replace=0.05, max_len=4096),
    dict(F=2, method="exact_len", max_consts=4, p_point_replace=0.5, max_len=40),
    dict(F=8, method="grow", max_consts=16, p_point_replace=1.0, max_len=8),
    dict(F=3, method="full", max_consts=0, p_point_replace=0.2, max_len=64),
    dict(F=4, method="rhh", max_consts=6, p_point_replace=0.3, max_len=120, fmask=oracle.ALL_FMASK),
]


@pytest.mark.parametrize("case", MUT_CASES)
@pytest.mark.parametrize("generation", [0, 7])
def test_genetic_operations_bit_exact_with_oracle(gp, case, generation):
    F, meth = case["F"], case["method"]
    fmask = case.get("fmask", oracle.DEFAULT_FMASK)
    init = dict(n_features=F, method=meth, min_depth=1, max_depth=7, min_len=1, max_len=80,
                max_consts=case["max_consts"])
    if "fmask" in case:
        init["fmask"] = fmask
    parents = gp.build_population(96, F, meth, min_depth=1, max_depth=7, min_len=1, max_len=80,
                                  max_consts=case["max_consts"], function_mask=fmask,
                                  seed=generation + 11)
    ev = dict(p_crossover=0.4, p_subtree=0.2, p_hoist=0.15, p_point=0.15,
              p_point_replace=case["p_point_replace"], max_len=case["max_len"], seed=4242)
    ops, ft, T = gp.plan_generation(96, generation, **ev)
    o_ops, o_ft, o_T = oracle.plan_generation(oracle.EvolveParams(**ev), 96, generation)
    assert np.array_equal(ops, o_ops) and np.array_equal(ft, o_ft) and T == o_T
    win = np.random.default_rng(generation).integers(0, 96, size=T).astype(np.int32)
    ginit = dict(init)
    if "fmask" in ginit:
        ginit["function_mask"] = ginit.pop("fmask")
    a = gp.mutate(parents, ops, ft, win, generation, ginit, **ev)
    b = oracle.mutate(oracle.EvolveParams(**ev), oracle.InitParams(**init),
                      oracle.Population(parents.nodes, parents.prog_off, parents.consts, parents.const_off,
                                        parents.length), ops, ft, win, generation)
    assert np.array_equal(a.nodes, b.nodes)
    assert np.array_equal(a.consts.view(np.uint32), b.consts.view(np.uint32))
    assert np.array_equal(a.prog_off, b.prog_off) and np.array_equal(a.const_off, b.const_off)
    assert np.array_equal(a.length, b.length)
    gp.validate_population(a, F)


def test_genetic_operation_errors(gp):
    parents = gp.build_population(10, 2, "rhh", seed=1)
    init = dict(n_features=2)
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.plan_generation(10, 0, p_crossover=0.8, p_subtree=0.3)     # sums above 1
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.plan_generation(10, 0, p_hoist=-0.1)
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.plan_generation(10, 0, max_len=0)
    ops, ft, T = gp.plan_generation(10, 0)
    win = np.zeros(T, np.int32)
    bad = win.copy()
    bad[-1] = 10                                                        # not a parent index
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.mutate(parents, ops, ft, bad, 0, init)
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.mutate(parents, ops, ft, win[:-1], 0, init)                  # too few winners
    broken = gp.HostPopulation(parents.nodes.copy(), parents.prog_off, parents.consts, parents.const_off,
                               parents.length)
    broken.nodes[int(parents.prog_off[1]) - 1] = oracle.node(oracle.ADD)
    with pytest.raises(gp.GPError, match="INVALID_PROGRAM"):
        gp.mutate(broken, ops, ft, win, 0, init)


def test_checkpoint_round_trip(gp, tmp_path):
    """The loop's state (flat population + generation number + settings)
    saves to .npz without pickles and loads back bit for bit."""
    pop = gp.build_population(50, 3, "exact_len", min_len=1, max_len=40, max_consts=4,
                              function_mask=oracle.ALL_FMASK, seed=9)
    path = tmp_path / "state.npz"
    gp.save_checkpoint(path, pop, 17, seed=5, metric="mse")
    back, g, meta = gp.load_checkpoint(path)
    assert g == 17 and meta == {"seed": 5, "metric": "mse"}
    assert np.array_equal(back.nodes, pop.nodes) and np.array_equal(back.prog_off, pop.prog_off)
    assert np.array_equal(back.consts.view(np.uint32), pop.consts.view(np.uint32))
    assert np.array_equal(back.const_off, pop.const_off) and np.array_equal(back.length, pop.length)
    gp.validate_population(back, 3)
