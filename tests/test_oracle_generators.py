"""Pins of the oracle's program generators (Sec. II-A: Full, Grow, ramped
half-and-half; plus the exact-length generator): validity, shape invariants
and the distributions the readings fix."""
import numpy as np
import pytest

import oracle
from oracle import ARITY, CONST, VAR


def leaf_depths(nodes):
    """Depth of every leaf, by recursive descent over the prefix list."""
    out = []

    def rec(i, d):
        op = int(nodes[i]) & 0xFF
        a = ARITY[op]
        j = i + 1
        if a == 0:
            out.append(d)
        for _ in range(a):
            j = rec(j, d + 1)
        return j

    assert rec(0, 0) == len(nodes)
    return out


def check_valid(pop, n_features, max_consts=0, lo=-1.0, hi=1.0):
    for p in range(pop.n_programs):
        nodes, consts = pop.program(p)
        rc, h = oracle.check_program(nodes, n_features, len(consts))
        assert rc == 0, (p, rc)
        assert h <= 20
        slots = [int(w) >> 8 for w in nodes if (int(w) & 0xFF) == CONST]
        assert slots == list(range(len(consts)))           # prefix-order numbering
        if max_consts:
            assert len(consts) <= max_consts
        if len(consts):
            assert consts.min() >= lo and consts.max() <= hi
        assert pop.length[p] == len(nodes)


def test_full_every_leaf_at_drawn_depth():
    pop = oracle.build_population(400, 2, "full", min_depth=2, max_depth=6, seed=1)
    check_valid(pop, 2)
    seen = set()
    for p in range(pop.n_programs):
        d = leaf_depths(pop.program(p)[0])
        assert len(set(d)) == 1
        seen.add(d[0])
    assert seen == {2, 3, 4, 5, 6}


def test_grow_depth_bounded():
    pop = oracle.build_population(400, 3, "grow", min_depth=1, max_depth=5, seed=2)
    check_valid(pop, 3)
    depths = [max(leaf_depths(pop.program(p)[0])) for p in range(pop.n_programs)]
    assert max(depths) <= 5 and min(depths) >= 1
    # grow trees are not all full: some leaves sit above the maximum depth
    assert any(len(set(leaf_depths(pop.program(p)[0]))) > 1 for p in range(pop.n_programs))


def test_rhh_half_full_and_depth_ramp():
    P = 4000
    pop = oracle.build_population(P, 2, "rhh", min_depth=2, max_depth=6, seed=3)
    check_valid(pop, 2)
    full = 0
    depth_counts = np.zeros(7, int)
    for p in range(P):
        d = leaf_depths(pop.program(p)[0])
        if len(set(d)) == 1 and d[0] == max(d):
            full += 1
        depth_counts[max(d)] += 1
    # every Full tree is uniform-depth; a Grow tree can be by chance, so the
    # count is at least the Full half: 0.5 P minus noise
    assert full >= 0.5 * P - 4 * np.sqrt(P * 0.25)
    # the root is a function (drawn depth >= 2), Grow may stop early, and
    # every depth of the ramp is reached
    assert depth_counts[0] == 0
    assert np.all(depth_counts[2:] > 0)


def test_rhh_root_is_function_when_depth_positive():
    pop = oracle.build_population(500, 2, "rhh", min_depth=1, max_depth=4, seed=4)
    for p in range(pop.n_programs):
        op = int(pop.program(p)[0][0]) & 0xFF
        assert ARITY[op] > 0


@pytest.mark.parametrize("max_consts", [0, 16])
def test_exact_len_lengths_uniform_and_valid(max_consts):
    P = 6000
    pop = oracle.build_population(P, 8, "exact_len", min_len=1, max_len=200,
                                  max_consts=max_consts, seed=5)
    check_valid(pop, 8, max_consts=max_consts)
    counts = np.bincount(pop.length, minlength=201)[1:]
    expect = P / 200
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    assert chi2 < 300          # 199 dof: mean 199, sd 20
    assert pop.length.min() >= 1 and pop.length.max() <= 200


def test_exact_len_without_unary_needs_odd_lengths():
    fmask = sum(1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL))
    pop = oracle.build_population(500, 2, "exact_len", min_len=1, max_len=60, fmask=fmask, seed=6)
    check_valid(pop, 2)
    assert np.all(pop.length % 2 == 1)


def test_no_constants_when_range_empty():
    pop = oracle.build_population(300, 2, "rhh", const_lo=1.0, const_hi=0.0, seed=7)
    assert pop.consts.shape[0] == 0
    for p in range(pop.n_programs):
        assert all((int(w) & 0xFF) != CONST for w in pop.program(p)[0])


def test_deterministic_and_seed_sensitive():
    a = oracle.build_population(100, 2, "rhh", seed=8)
    b = oracle.build_population(100, 2, "rhh", seed=8)
    c = oracle.build_population(100, 2, "rhh", seed=9)
    assert np.array_equal(a.nodes, b.nodes) and np.array_equal(a.consts, b.consts)
    assert not np.array_equal(a.nodes[:50], c.nodes[:50])


def test_variables_cover_features():
    pop = oracle.build_population(500, 28, "exact_len", min_len=1, max_len=200, seed=10)
    feats = {int(w) >> 8 for w in pop.nodes if (int(w) & 0xFF) == VAR}
    assert feats == set(range(28))


def test_bad_arguments_rejected():
    with pytest.raises(ValueError):
        oracle.build_population(10, 2, "rhh", min_depth=3, max_depth=2)
    with pytest.raises(ValueError):
        oracle.build_population(10, 2, "rhh", max_depth=20)
    with pytest.raises(ValueError):
        oracle.build_population(10, 2, "exact_len", min_len=0)
    with pytest.raises(ValueError):
        oracle.build_population(10, 2, "rhh", fmask=0)


@pytest.mark.parametrize("method", ["rhh", "exact_len"])
def test_every_enabled_function_is_drawn_uniformly(method):
    """With every function enabled the generators draw each of the 21 about
    equally often among function nodes (the draw is uniform over the enabled
    set), and never one that is not enabled."""
    pop = oracle.build_population(2000, 3, method, min_depth=2, max_depth=6, min_len=1,
                                  max_len=60, fmask=oracle.ALL_FMASK, max_consts=4, seed=77)
    check_valid(pop, 3, max_consts=4)
    ops = pop.nodes & 0xFF
    funcs = [o for o, a in ARITY.items() if a > 0]
    assert len(funcs) == 21
    counts = np.array([(ops == o).sum() for o in funcs], np.float64)
    assert counts.min() > 0
    # exact_len chooses unary vs binary by the length budget, so compare
    # within each arity class
    for ar in (1, 2):
        c = np.array([counts[i] for i, o in enumerate(funcs) if ARITY[o] == ar])
        assert c.max() / c.min() < 1.15, (ar, c)
    only = sum(1 << o for o in (oracle.ATAN2, oracle.CBRT))
    pop2 = oracle.build_population(300, 2, method, min_depth=2, max_depth=5, min_len=1, max_len=40,
                                   fmask=only, seed=78)
    ops2 = set(np.unique(pop2.nodes & 0xFF).tolist())
    assert ops2 <= {VAR, CONST, oracle.ATAN2, oracle.CBRT} and {oracle.ATAN2, oracle.CBRT} <= ops2
