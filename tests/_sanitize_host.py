"""Driver of the sanitizer test (not a test module): exercises the library's
host C ABI (generators, validation, the generation pre-draw, genetic
operations), built with AddressSanitizer and UndefinedBehaviorSanitizer and
loaded from the path in argv[1], against the oracle (itself loaded from the
sanitizer build GP_ORACLE_LIB names).  Any memory or undefined-behaviour
error aborts the process; results must equal the oracle's bit for bit."""
import ctypes
import sys

import numpy as np

import oracle

lib = ctypes.CDLL(sys.argv[1])
vp, i32, i64, u32, u64, f32 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64,
                               ctypes.c_float)


class Init(ctypes.Structure):
    _fields_ = [("n_programs", i32), ("n_features", i32), ("method", i32), ("min_depth", i32),
                ("max_depth", i32), ("min_len", i32), ("max_len", i32), ("function_mask", u32),
                ("const_lo", f32), ("const_hi", f32), ("max_consts", i32), ("seed", u64)]


class Evolve(ctypes.Structure):
    _fields_ = [("p_crossover", f32), ("p_subtree", f32), ("p_hoist", f32), ("p_point", f32),
                ("p_point_replace", f32), ("max_len", i32), ("seed", u64)]


lib.gp_build_population.argtypes = [ctypes.POINTER(Init)] + [vp] * 9
lib.gp_build_population.argtypes = [ctypes.POINTER(Init), vp, i64, vp, vp, i64, vp, vp, vp, vp]
lib.gp_validate_population.argtypes = [vp, vp, vp, i32, i32, vp, vp]
lib.gp_plan_generation.argtypes = [ctypes.POINTER(Evolve), i32, u64, vp, vp, vp]
lib.gp_mutate.argtypes = [ctypes.POINTER(Evolve), ctypes.POINTER(Init), vp, vp, vp, vp, i32, vp, vp, vp, i32, i32,
                          u64, vp, i64, vp, vp, i64, vp, vp, vp, vp]


def P(a):
    return None if a is None else a.ctypes.data_as(vp)


def build(init):
    tn, tc = np.zeros(1, np.int64), np.zeros(1, np.int64)
    assert lib.gp_build_population(ctypes.byref(init), None, 0, None, None, 0, None, None, P(tn), P(tc)) == 0
    n = init.n_programs
    nodes, consts = np.zeros(max(int(tn[0]), 1), np.uint32), np.zeros(max(int(tc[0]), 1), np.float32)
    po, co, ln = np.zeros(n + 1, np.int64), np.zeros(n + 1, np.int64), np.zeros(max(n, 1), np.int32)
    assert lib.gp_build_population(ctypes.byref(init), P(nodes), nodes.shape[0], P(po), P(consts), consts.shape[0],
                                   P(co), P(ln), P(tn), P(tc)) == 0
    return oracle.Population(nodes[:int(tn[0])], po, consts[:int(tc[0])], co, ln[:n])


rng = np.random.default_rng(12)
checked = 0
for trial in range(40):
    method = int(rng.integers(0, 4))
    F = int(rng.integers(1, 30))
    mask = int(rng.choice([oracle.DEFAULT_FMASK, oracle.ALL_FMASK, (1 << oracle.ADD) | (1 << oracle.MUL)]))
    lo_d = int(rng.integers(0, 5))
    lo_l = int(rng.integers(1, 60))
    init = Init(int(rng.integers(0, 60)), F, method, lo_d, lo_d + int(rng.integers(0, 4)), lo_l,
                lo_l + int(rng.integers(0, 140)), mask, -1.0, 1.0, int(rng.integers(0, 17)), int(rng.integers(1, 1 << 40)))
    pop = build(init)
    ref = oracle.build_population(init.n_programs, F, method, init.min_depth, init.max_depth, init.min_len,
                                  init.max_len, mask, -1.0, 1.0, init.max_consts, init.seed)
    assert np.array_equal(pop.nodes, ref.nodes) and np.array_equal(pop.consts.view(np.uint32),
                                                                   ref.consts.view(np.uint32))
    n = init.n_programs
    mh = np.zeros(max(n, 1), np.int32)
    bad = np.zeros(1, np.int32)
    assert lib.gp_validate_population(P(pop.nodes), P(pop.prog_off), P(pop.const_off), n, F, P(mh), P(bad)) == 0
    # corrupted copies: any status, no fault
    for _ in range(4):
        cor = pop.nodes.copy()
        if cor.size:
            k = int(rng.integers(0, cor.size))
            cor[k] ^= np.uint32(1 << int(rng.integers(0, 32)))
        lib.gp_validate_population(P(cor), P(pop.prog_off), P(pop.const_off), n, F, P(mh), P(bad))
    if n == 0:
        continue
    ev = Evolve(0.5, 0.15, 0.1, 0.15, 0.1, int(rng.integers(8, 300)), int(rng.integers(1, 1 << 40)))
    ops, ft, nt = np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(1, np.int32)
    assert lib.gp_plan_generation(ctypes.byref(ev), n, trial, P(ops), P(ft), P(nt)) == 0
    winners = rng.integers(0, n, size=max(int(nt[0]), 1)).astype(np.int32)
    cap = max(n * max(ev.max_len, int(pop.length.max(initial=1))), 1)
    out = [np.zeros(cap, np.uint32), np.zeros(n + 1, np.int64), np.zeros(cap, np.float32), np.zeros(n + 1, np.int64),
           np.zeros(n, np.int32), np.zeros(1, np.int64), np.zeros(1, np.int64)]
    pc = pop.consts if pop.consts.size else np.zeros(1, np.float32)
    rc = lib.gp_mutate(ctypes.byref(ev), ctypes.byref(init), P(pop.nodes), P(pop.prog_off), P(pc), P(pop.const_off),
                       n, P(ops), P(ft), P(winners), winners.shape[0], n, trial, P(out[0]), cap, P(out[1]),
                       P(out[2]), cap, P(out[3]), P(out[4]), P(out[5]), P(out[6]))
    assert rc == 0, rc
    e = oracle.EvolveParams(ev.p_crossover, ev.p_subtree, ev.p_hoist, ev.p_point, ev.p_point_replace, ev.max_len,
                            ev.seed)
    ip = oracle.InitParams(F, ["rhh", "full", "grow", "exact_len"][method], init.min_depth, init.max_depth,
                           init.min_len, init.max_len, mask, -1.0, 1.0, init.max_consts)
    kids = oracle.mutate(e, ip, pop, ops, ft, winners, trial)
    assert np.array_equal(out[0][:int(out[5][0])], kids.nodes)
    # out-of-range winners and a too-small buffer: an error status, no fault
    bad_w = winners.copy()
    bad_w[0] = n + 5
    lib.gp_mutate(ctypes.byref(ev), ctypes.byref(init), P(pop.nodes), P(pop.prog_off), P(pc), P(pop.const_off),
                  n, P(ops), P(ft), P(bad_w), bad_w.shape[0], n, trial, P(out[0]), 1, P(out[1]), P(out[2]), 1,
                  P(out[3]), P(out[4]), P(out[5]), P(out[6]))
    checked += 1
print(f"sanitized host driver: {checked} populations built, validated and mutated bit-exactly")
