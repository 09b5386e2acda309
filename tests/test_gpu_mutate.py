"""GPU parity of the device genetic operations (gp_plan_generation_device,
gp_mutate_device) against the oracle's operations (Sec. II-A mutation list,
Sec. III-C pre-draw of operation types, Sec. III-C2 hoisted crossover): the
plans, the offspring's node words, constant bits and offsets must be
identical, over every initialisation method, constant settings, the wider
function set, hoisting-heavy length bounds and several chained generations.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    import torch
    import paper_2110_11226_amd as gp
    torch.cuda.set_device(0)
    return gp


EV = dict(p_crossover=0.4, p_subtree=0.2, p_hoist=0.15, p_point=0.15)

CASES = [
    dict(F=1, method="rhh", max_consts=0, p_point_replace=0.05, max_len=4096),
    dict(F=2, method="exact_len", max_consts=4, p_point_replace=0.5, max_len=40),
    dict(F=8, method="grow", max_consts=16, p_point_replace=1.0, max_len=8),
    dict(F=3, method="full", max_consts=0, p_point_replace=0.2, max_len=64),
    dict(F=4, method="rhh", max_consts=6, p_point_replace=0.3, max_len=120, fmask=oracle.ALL_FMASK),
    # no unary functions: the exact-length generator's parity rule
    dict(F=2, method="exact_len", max_consts=3, p_point_replace=0.4, max_len=30,
         fmask=sum(1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL, oracle.ATAN2))),
]


def _init(case):
    init = dict(n_features=case["F"], method=case["method"], min_depth=1, max_depth=7, min_len=1,
                max_len=80, max_consts=case["max_consts"])
    if "fmask" in case:
        init["fmask"] = case["fmask"]
    return init


def _lib_init(init):
    g = dict(init)
    if "fmask" in g:
        g["function_mask"] = g.pop("fmask")
    return g


def _same(a, b, label):
    assert np.array_equal(a.prog_off, b.prog_off), label
    assert np.array_equal(a.const_off, b.const_off), label
    assert np.array_equal(a.length, b.length), label
    assert np.array_equal(np.asarray(a.nodes, np.uint32), np.asarray(b.nodes, np.uint32)), label
    assert np.array_equal(np.asarray(a.consts, np.float32).view(np.uint32),
                          np.asarray(b.consts, np.float32).view(np.uint32)), label


def _oracle_pop(h):
    return oracle.Population(h.nodes, h.prog_off, h.consts, h.const_off, h.length)


@pytest.mark.parametrize("n_off,generation", [(0, 0), (1, 0), (1000, 3), (5000, 12345), (70000, 2)])
def test_plan_matches_oracle(gp, n_off, generation):
    ev = dict(EV, seed=99)
    ops, ft, nt = gp.plan_generation_device(n_off, generation, **ev)
    o_ops, o_ft, o_T = oracle.plan_generation(oracle.EvolveParams(**ev), n_off, generation)
    assert np.array_equal(ops.cpu().numpy(), o_ops)
    assert np.array_equal(ft.cpu().numpy(), o_ft)
    assert int(nt.cpu()[0]) == o_T


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("generation", [0, 7])
def test_mutate_bit_exact_with_oracle(gp, case, generation):
    F = case["F"]
    init = _init(case)
    parents = gp.build_population(300, F, init["method"], min_depth=1, max_depth=7, min_len=1, max_len=80,
                                  max_consts=case["max_consts"],
                                  function_mask=init.get("fmask", oracle.DEFAULT_FMASK), seed=generation + 11)
    ev = dict(EV, p_point_replace=case["p_point_replace"], max_len=case["max_len"], seed=4242)
    ops, ft, nt = gp.plan_generation_device(300, generation, **ev)
    T = int(nt.cpu()[0])
    win = np.random.default_rng(generation).integers(0, 300, size=T).astype(np.int32)
    dpar = gp.DevicePopulation(parents, n_features=F)
    off = gp.mutate_device(dpar, ops, ft, win, generation, _lib_init(init), **ev)
    got = off.to_host()
    o_ops, o_ft, _ = oracle.plan_generation(oracle.EvolveParams(**ev), 300, generation)
    ref = oracle.mutate(oracle.EvolveParams(**ev), oracle.InitParams(**init), _oracle_pop(parents), o_ops, o_ft,
                        win, generation)
    _same(got, ref, f"{case} gen {generation}")
    gp.validate_population(got, F)
    counts = np.bincount(ops.cpu().numpy(), minlength=5)
    assert (counts[:4] > 0).all(), counts      # every operation took part


def test_chained_generations_stay_on_device(gp):
    """Six generations in which each offspring population is the next one's
    parents without leaving the device, against the oracle's chain."""
    F = 3
    init = dict(n_features=F, method="rhh", min_depth=2, max_depth=5, max_consts=5, fmask=oracle.ALL_FMASK)
    host = gp.build_population(512, F, "rhh", min_depth=2, max_depth=5, max_consts=5,
                               function_mask=oracle.ALL_FMASK, seed=5)
    ev = dict(EV, p_point_replace=0.1, max_len=60, seed=777)
    dev = gp.DevicePopulation(host, n_features=F)
    ref = _oracle_pop(host)
    rng = np.random.default_rng(9)
    for g in range(6):
        ops, ft, nt = gp.plan_generation_device(512, g, **ev)
        T = int(nt.cpu()[0])
        win = rng.integers(0, 512, size=T).astype(np.int32)
        off = gp.mutate_device(dev, ops, ft, win, g, _lib_init(init), **ev)
        o_ops, o_ft, _ = oracle.plan_generation(oracle.EvolveParams(**ev), 512, g)
        ref = oracle.mutate(oracle.EvolveParams(**ev), oracle.InitParams(**init), ref, o_ops, o_ft, win, g)
        got = off.to_host()
        _same(got, ref, f"generation {g}")
        assert got.length.max() <= 60 or got.length.max() <= host.length.max()
        dev = off.as_parents()


def test_status_and_argument_errors(gp):
    import torch
    host = gp.build_population(64, 2, "rhh", min_depth=2, max_depth=4, max_consts=2, seed=1)
    dpar = gp.DevicePopulation(host, n_features=2)
    init = dict(n_features=2, method="rhh", min_depth=2, max_depth=4, max_consts=2)
    ev = dict(EV, p_point_replace=0.2, max_len=50, seed=3)
    ops, ft, nt = gp.plan_generation_device(64, 0, **ev)
    T = int(nt.cpu()[0])
    win = np.zeros(T, np.int32)
    win[0] = 64                                   # not a parent index
    off = gp.mutate_device(dpar, ops, ft, win, 0, init, **ev)
    tn, tc, st = off.status()
    assert st == 2
    h = off.nodes[:tn].cpu().numpy().view(np.uint32)
    first_prog = h[int(off.prog_off[0]):int(off.prog_off[1])]
    assert first_prog.tolist() == [oracle.node(oracle.VAR, 0)]
    # a short capacity writes nothing and says so
    good = np.zeros(T, np.int32)
    off = gp.mutate_device(dpar, ops, ft, good, 0, init, node_capacity=10, **ev)
    assert off.status()[2] == 1
    with pytest.raises(gp.GPError):
        off.to_host()
    # no offspring
    off = gp.mutate_device(dpar, torch.empty(0, dtype=torch.int32, device="cuda"),
                           torch.empty(0, dtype=torch.int32, device="cuda"), good, 0, init, **ev)
    assert off.status() == (0, 0, 0)
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.plan_generation_device(10, 0, p_crossover=0.8, p_subtree=0.3)
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.mutate_device(dpar, ops, ft, good, 0, dict(init, max_depth=19), **ev)   # donor bound
    with pytest.raises(gp.GPError, match="INVALID_ARG"):
        gp.mutate_device(dpar, ops, ft, good, 0, dict(init, function_mask=1 << 23), **ev)
