"""Pins of the oracle's genetic operations (Sec. II-A mutation list, Sec.
III-C pre-draw, Sec. III-C2 hoisted crossover), independent of how they are
computed: each child must be the splice its operation defines for SOME
choice of subtrees (found by brute force over all choices), the length and
stack bounds must hold, point mutation must keep the arity pattern, and the
pre-draw must hit each operation with its probability."""
import numpy as np
import pytest

import oracle
from oracle import ADD, MUL, SIN, NEG, VAR, CONST, node


def decode(pop, p):
    """Program p as a tuple of (opcode, feature) / ('c', value bits)."""
    a, b = int(pop.prog_off[p]), int(pop.prog_off[p + 1])
    c0 = int(pop.const_off[p])
    out = []
    for w in pop.nodes[a:b]:
        op, arg = int(w) & 0xff, int(w) >> 8
        out.append(("c", int(np.float32(pop.consts[c0 + arg]).view(np.uint32))) if op == CONST else (op, arg))
    return tuple(out)


def arity(t):
    op = t[0]
    if op == "c" or op in (oracle.VAR,):
        return 0
    return 2 if op in (oracle.ADD, oracle.SUB, oracle.MUL, oracle.DIV) else 1


def subtree_ends(prog):
    """end of the subtree at every start, by brute-force stack counting."""
    ends = []
    for s in range(len(prog)):
        need, i = 1, s
        while need:
            need += arity(prog[i]) - 1
            i += 1
        ends.append(i)
    return ends


def height(prog):
    h = m = 0
    for t in reversed(prog):
        h += 1 - arity(t)
        m = max(m, h)
    return m


def slots_in_prefix_order(pop, p):
    a, b = int(pop.prog_off[p]), int(pop.prog_off[p + 1])
    k = [int(w) >> 8 for w in pop.nodes[a:b] if int(w) & 0xff == CONST]
    return k == list(range(len(k))) and len(k) == int(pop.const_off[p + 1] - pop.const_off[p])


def valid_all(pop, F):
    for p in range(pop.n_programs):
        nodes, consts = pop.program(p)
        rc, h = oracle.check_program(nodes, F, len(consts))
        assert rc == 0 and h <= 20, p
        assert slots_in_prefix_order(pop, p), p


def setup(F=3, P=60, seed=0, method="rhh", max_depth=6):
    par = oracle.build_population(P, F, method, min_depth=1, max_depth=max_depth, max_len=50, seed=seed)
    init = oracle.InitParams(n_features=F, method=method, min_depth=1, max_depth=max_depth, max_len=50)
    return par, init


def offspring(par, init, op, n=60, gen=3, **kw):
    ev = oracle.EvolveParams(**{**dict(p_crossover=0, p_subtree=0, p_hoist=0, p_point=0), **kw})
    ops = np.full(n, op, np.int32)
    per = 2 if op == 0 else 1
    ft = (np.arange(n) * per).astype(np.int32)
    win = np.random.default_rng(gen).integers(0, par.n_programs, size=n * per).astype(np.int32)
    return oracle.mutate(ev, init, par, ops, ft, win, gen), ft, win


def test_plan_frequencies_and_tournament_count():
    n = 200_000
    ev = oracle.EvolveParams(p_crossover=0.7, p_subtree=0.1, p_hoist=0.05, p_point=0.1, seed=5)
    ops, ft, T = oracle.plan_generation(ev, n, 2)
    for k, p in enumerate([0.7, 0.1, 0.05, 0.1, 0.05]):
        f = np.mean(ops == k)
        assert abs(f - p) <= 5 * np.sqrt(p * (1 - p) / n), (k, f)
    assert T == n + int(np.sum(ops == 0))
    per = np.where(ops == 0, 2, 1)
    assert np.array_equal(ft, np.concatenate([[0], np.cumsum(per)[:-1]]))
    # all-crossover and all-reproduction limits
    assert np.all(oracle.plan_generation(oracle.EvolveParams(1, 0, 0, 0), 100, 0)[0] == 0)
    assert np.all(oracle.plan_generation(oracle.EvolveParams(0, 0, 0, 0), 100, 0)[0] == 4)


def test_reproduction_copies_the_winner():
    par, init = setup()
    kids, ft, win = offspring(par, init, 4)
    for i in range(kids.n_programs):
        assert decode(kids, i) == decode(par, win[ft[i]])


def test_point_mutation_keeps_arities_and_replaces_at_its_rate():
    par, init = setup(F=4)
    kids, ft, win = offspring(par, init, 3, n=400, p_point_replace=1.0)
    changed = total = 0
    n_var = n_term = 0
    for i in range(kids.n_programs):
        c, p = decode(kids, i), decode(par, win[ft[i]])
        assert len(c) == len(p)
        assert [arity(t) for t in c] == [arity(t) for t in p]
        changed += sum(x != y for x, y in zip(c, p))
        total += len(c)
        for t in c:
            if arity(t) == 0:
                n_term += 1
                n_var += t[0] == VAR
                if t[0] == "c":
                    v = np.uint32(t[1]).view(np.float32)
                    assert -1.0 <= v < 1.0
    assert changed > 0.5 * total
    # terminals: 4 features and 1 constant choice, uniformly
    assert abs(n_var / n_term - 0.8) < 0.05
    kids0, ft0, win0 = offspring(par, init, 3, p_point_replace=0.0)
    for i in range(kids0.n_programs):
        assert decode(kids0, i) == decode(par, win0[ft0[i]])


def test_hoist_is_a_subtree_of_a_subtree():
    par, init = setup(seed=2)
    kids, ft, win = offspring(par, init, 2, n=80)
    for i in range(kids.n_programs):
        c, p = decode(kids, i), decode(par, win[ft[i]])
        assert len(c) <= len(p)
        ends = subtree_ends(p)
        found = any(p[:s] + p[s2:ends[s2]] + p[ends[s]:] == c
                    for s in range(len(p)) for s2 in range(s, ends[s]))
        assert found, i
    valid_all(kids, 3)


def test_crossover_is_a_splice_of_parent_and_donor():
    par, init = setup(seed=3)
    kids, ft, win = offspring(par, init, 0, n=80)
    for i in range(kids.n_programs):
        c, p, d = decode(kids, i), decode(par, win[ft[i]]), decode(par, win[ft[i] + 1])
        pe, de = subtree_ends(p), subtree_ends(d)
        found = any(len(c) == s + (de[ds] - ds) + len(p) - pe[s] and
                    p[:s] + d[ds:de[ds]] + p[pe[s]:] == c
                    for s in range(len(p)) for ds in range(len(d)))
        assert found, i
    valid_all(kids, 3)


def test_hoisted_crossover_respects_the_stack_and_the_length_bound():
    # parents of stack height 19-20 and donors as deep: a plain crossover
    # would often need more than 20 slots
    F = 2
    par = oracle.build_population(80, F, "full", min_depth=10, max_depth=12,
                                  fmask=sum(1 << o for o in (ADD, MUL, SIN, NEG)), seed=9)
    heights = [height(decode(par, p)) for p in range(par.n_programs)]
    assert max(heights) <= 20
    init = oracle.InitParams(n_features=F, method="full", min_depth=10, max_depth=12,
                             fmask=sum(1 << o for o in (ADD, MUL, SIN, NEG)))
    kids, ft, win = offspring(par, init, 0, n=200, max_len=100000)
    for i in range(kids.n_programs):
        assert height(decode(kids, i)) <= 20
    valid_all(kids, F)
    # length bound: met whenever the parent meets it
    kids, ft, win = offspring(par, init, 0, n=200, max_len=3000)
    for i in range(kids.n_programs):
        if par.length[win[ft[i]]] <= 3000:
            assert kids.length[i] <= 3000
    # subtree mutation obeys the same bounds
    kids, ft, win = offspring(par, init, 1, n=100, max_len=2500)
    for i in range(kids.n_programs):
        assert height(decode(kids, i)) <= 20
        if par.length[win[ft[i]]] <= 2500:
            assert kids.length[i] <= 2500
    valid_all(kids, F)


def test_subtree_mutation_replaces_one_subtree_by_a_new_program_part():
    par, init = setup(seed=4)
    kids, ft, win = offspring(par, init, 1, n=60)
    for i in range(kids.n_programs):
        c, p = decode(kids, i), decode(par, win[ft[i]])
        pe = subtree_ends(p)
        ok = False
        for s in range(len(p)):
            tail = p[pe[s]:]
            mid_len = len(c) - s - len(tail)
            if mid_len >= 1 and c[:s] == p[:s] and c[len(c) - len(tail):] == tail:
                mid = c[s:s + mid_len]
                if subtree_ends(mid)[0] == len(mid):
                    ok = True
                    break
        assert ok, i
    valid_all(kids, 3)


def test_constants_keep_their_values():
    par = oracle.build_population(40, 2, "exact_len", min_len=5, max_len=40, max_consts=6, seed=8)
    init = oracle.InitParams(n_features=2, method="exact_len", min_len=5, max_len=40, max_consts=6)
    for op in (0, 2, 4):
        kids, ft, win = offspring(par, init, op, n=60)
        pool = set(np.float32(par.consts).view(np.uint32).tolist())
        assert set(np.float32(kids.consts).view(np.uint32).tolist()) <= pool
        valid_all(kids, 2)
    # point mutation adds constants only while fewer than max_consts remain
    kids, ft, win = offspring(par, init, 3, n=200, p_point_replace=1.0)
    assert np.max(np.diff(kids.const_off)) <= 6
    assert np.sum(np.diff(kids.const_off)) > 0
