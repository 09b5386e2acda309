"""CPU oracle for GP population evaluation, fitness, tournament selection,
program generation and constant gradients (arXiv 2110.11226).

TEST INFRASTRUCTURE ONLY: the product library never imports this package.
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use it.  The arithmetic lives in ``gp_oracle.c`` (plain C built
with gcc, no contraction, no fast-math); this module marshals numpy arrays.

Every function here wraps one function of ``gp_oracle.c``; the citations of
the paper are in that file next to each function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# (tests/test_sanitizers.py points this at an AddressSanitizer build)
_LIB = os.environ.get("GP_ORACLE_LIB", _LIB)

# opcodes as the oracle reads them (op in bits 0-7, argument in bits 8-31)
VAR, CONST, ADD, SUB, MUL, DIV, NEG, LOG, SQRT, SIN, COS, TAN = range(12)
MAX, MIN, ATAN2 = 12, 13, 14
ABS, EXP, INV, SQ, CUBE, TANH, ATAN, CBRT = range(15, 23)
ARITY = {VAR: 0, CONST: 0, ADD: 2, SUB: 2, MUL: 2, DIV: 2,
         NEG: 1, LOG: 1, SQRT: 1, SIN: 1, COS: 1, TAN: 1,
         MAX: 2, MIN: 2, ATAN2: 2,
         ABS: 1, EXP: 1, INV: 1, SQ: 1, CUBE: 1, TANH: 1, ATAN: 1, CBRT: 1}
# every function: the nine of the benchmark configurations, tan, and the wider set
ALL_FMASK = sum(1 << op for op, a in ARITY.items() if a > 0)
METRICS = {"mae": 0, "mse": 1, "rmse": 2, "logloss": 3, "pearson": 4, "spearman": 5,
           "user0": 6, "user1": 7, "user2": 8, "user3": 9}
LARGER_IS_BETTER = {0: 0, 1: 0, 2: 0, 3: 0, 4: 1, 5: 1, 6: 0, 7: 0, 8: 0, 9: 0}
# user-defined functions (Sec. V): 24..27 of one argument, 28..31 of two
USER1, USER2 = 24, 28
INIT = {"rhh": 0, "full": 1, "grow": 2, "exact_len": 3}
# the nine-function set used by the Pagie / classification workloads
DEFAULT_FMASK = sum(1 << op for op in (ADD, SUB, MUL, DIV, NEG, LOG, SQRT, SIN, COS))
# relative allowance for a library-function result in the conditioning bound:
# 4 float32 ulps (an ulp of v is at most 2^-23 |v|)
ULP_ALLOWANCE = 4.0 * 2.0 ** -23
# the spacing of float32 relative to |v| (at most): a correctly rounded
# operation whose operands differ between two evaluations may round to
# neighbouring floats, one spacing apart
ROUND_FLIP = 2.0 ** -23


def build(force: bool = True) -> str:
    """Compile gp_oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_SRC) > os.path.getmtime(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u32, u64, f32 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_float)
        L.orc_set_user_function.argtypes = [ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int]
        L.orc_set_user_function.restype = ctypes.c_int
        L.orc_check_program.argtypes = [P, i64, i32, i64, P]
        L.orc_check_program.restype = ctypes.c_int
        L.orc_evaluate_f32.argtypes = [P, P, P, P, i32, P, i64, i64, P, ctypes.c_int]
        L.orc_evaluate_f64.argtypes = [P, P, P, P, i32, P, i64, i64, P, ctypes.c_int]
        L.orc_evaluate_pairs.argtypes = [P, P, P, P, P, i64, P, P, i64, ctypes.c_double, ctypes.c_double,
                                         u32, P, P, P, P, ctypes.c_int]
        L.orc_fitness.argtypes = [P, P, P, P, i32, P, i64, i64, P, P, i32, P, P, ctypes.c_double,
                                  ctypes.c_double, u32, P, P, ctypes.c_int]
        L.orc_cr_undecided.restype = ctypes.c_longlong
        L.orc_cr_undecided.argtypes = []
        L.orc_cr_reset.argtypes = []
        L.orc_cr_set_margin.argtypes = [ctypes.c_double]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_philox_words.argtypes = [u64, u32, u32, u32, u32, u32, P]
        L.orc_tournament.argtypes = [P, P, i32, i32, f32, i32, i32, u64, u64, P]
        L.orc_tournament_draws.argtypes = [i32, i32, i32, u64, u64, P]
        L.orc_build_population.argtypes = [i32, i32, i32, i32, i32, i32, i32, u32, f32, f32,
                                           i32, u64, P, i64, P, P, i64, P, P, P, P]
        L.orc_build_population.restype = ctypes.c_int
        L.orc_grad_consts.argtypes = [P, P, P, P, i32, P, i64, i64, P, P, i32, P, P, P,
                                      ctypes.c_double, u64, ctypes.c_int, ctypes.c_int]
        L.orc_plan_generation.argtypes = [f32, f32, f32, f32, u64, i32, u64, P, P, P]
        L.orc_plan_generation.restype = ctypes.c_int
        L.orc_mutate.argtypes = [f32, f32, f32, f32, f32, i32, u64,
                                 i32, i32, i32, i32, i32, i32, u32, f32, f32, i32,
                                 P, P, P, P, P, P, P, i32, u64,
                                 P, i64, P, P, i64, P, P, P, P]
        L.orc_mutate.restype = ctypes.c_int
        _lib = L
    return _lib


def cr_undecided() -> int:
    """Library-function roundings the float32 path could not decide since the
    last cr_reset() (its result is then the x87 extended value's rounding)."""
    return int(lib().orc_cr_undecided())


def cr_reset():
    lib().orc_cr_reset()


def cr_set_margin(ulps=8.0):
    """Distance (in double ulps) from a float32 rounding boundary below which
    the float32 path consults the extended-precision result (tests widen it
    to exercise that path; the default is 8)."""
    lib().orc_cr_set_margin(float(ulps))


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _threads(n):
    return int(n) if n else 1


@dataclass
class Population:
    """Flat prefix-list population (the layout the library also takes)."""
    nodes: np.ndarray      # uint32 [total_nodes]
    prog_off: np.ndarray   # int64 [P+1]
    consts: np.ndarray     # float32 [total_consts]
    const_off: np.ndarray  # int64 [P+1]
    length: np.ndarray     # int32 [P]

    @property
    def n_programs(self) -> int:
        return int(self.length.shape[0])

    def program(self, p):
        a, b = int(self.prog_off[p]), int(self.prog_off[p + 1])
        c, d = int(self.const_off[p]), int(self.const_off[p + 1])
        return self.nodes[a:b], self.consts[c:d]


def from_programs(programs) -> Population:
    """Pack a list of (nodes, consts) pairs into the flat layout."""
    nodes, consts, po, co, ln = [], [], [0], [0], []
    for pn, pc in programs:
        pn = np.asarray(pn, dtype=np.uint32)
        pc = np.asarray(pc, dtype=np.float32)
        nodes.append(pn)
        consts.append(pc)
        po.append(po[-1] + len(pn))
        co.append(co[-1] + len(pc))
        ln.append(len(pn))
    return Population(
        nodes=np.concatenate(nodes).astype(np.uint32) if nodes else np.zeros(0, np.uint32),
        prog_off=np.asarray(po, dtype=np.int64),
        consts=(np.concatenate(consts).astype(np.float32) if consts
                else np.zeros(0, np.float32)),
        const_off=np.asarray(co, dtype=np.int64),
        length=np.asarray(ln, dtype=np.int32))


def node(op, arg=0):
    return (int(op) & 0xFF) | (int(arg) << 8)


def set_user_function(op, nodes=None, consts=()):
    """Define user function `op` (USER1..USER1+3: one argument, USER2..USER2+3:
    two) as the prefix list `nodes` over the built-in functions, VAR k being
    argument k and CONST k consts[k]; no nodes removes it."""
    nd = np.ascontiguousarray(np.asarray(nodes if nodes else [0], np.uint32))
    cs = np.ascontiguousarray(np.asarray(consts if len(consts) else [0.0], np.float32))
    rc = lib().orc_set_user_function(int(op), _p(nd), len(nodes) if nodes else 0, _p(cs), len(consts))
    if rc != 0:
        raise ValueError("orc_set_user_function: bad arguments")


def check_program(nodes, n_features, n_consts):
    nodes = np.ascontiguousarray(nodes, dtype=np.uint32)
    h = np.zeros(1, np.int32)
    rc = lib().orc_check_program(_p(nodes), len(nodes), int(n_features), int(n_consts), _p(h))
    return int(rc), int(h[0])


def _ds(X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    assert X.ndim == 2
    return X, X.shape[1]


def evaluate_f32(pop: Population, X, n_threads=None):
    """out[p, r] = float32 stack value of program p on row r.  X is [F, N]."""
    X, N = _ds(X)
    out = np.empty((pop.n_programs, N), np.float32)
    lib().orc_evaluate_f32(_p(pop.nodes), _p(pop.prog_off), _p(pop.consts), _p(pop.const_off),
                           pop.n_programs, _p(X), N, N, _p(out), _threads(n_threads))
    return out


def evaluate_f64(pop: Population, X, n_threads=None):
    X, N = _ds(X)
    out = np.empty((pop.n_programs, N), np.float64)
    lib().orc_evaluate_f64(_p(pop.nodes), _p(pop.prog_off), _p(pop.consts), _p(pop.const_off),
                           pop.n_programs, _p(X), N, N, _p(out), _threads(n_threads))
    return out


@dataclass
class RowAnalysis:
    v32: np.ndarray      # float32 stack value
    v64: np.ndarray      # float64 stack value
    bound: np.ndarray    # first-order bound on the float32 value's sensitivity
    flip: np.ndarray     # a protected predicate differs between float32 and float64
    near: np.ndarray     # a protected predicate lies within its bound of the threshold


def evaluate_pairs(pop: Population, X, prog, row, n_threads=None, u=ULP_ALLOWANCE,
                   rf=ROUND_FLIP, exact=0) -> RowAnalysis:
    """Float32 and float64 values and the conditioning analysis of each
    (prog[i], row[i]) pair (see row_analysis in gp_oracle.c).  `exact` is a
    mask (bit per opcode) of the library functions the comparison takes as
    correctly rounded on both sides: they get no allowance u of their own."""
    X, N = _ds(X)
    prog = np.ascontiguousarray(prog, dtype=np.int32)
    row = np.ascontiguousarray(row, dtype=np.int64)
    n = prog.shape[0]
    o32 = np.empty(n, np.float32)
    o64 = np.empty(n, np.float64)
    eb = np.empty(n, np.float64)
    fl = np.empty(n, np.uint8)
    lib().orc_evaluate_pairs(_p(pop.nodes), _p(pop.prog_off), _p(pop.consts),
                             _p(pop.const_off), _p(X), N, _p(prog), _p(row), n, float(u), float(rf),
                             int(exact), _p(o32), _p(o64), _p(eb), _p(fl), _threads(n_threads))
    return RowAnalysis(o32, o64, eb, (fl & 1).astype(bool), (fl & 2).astype(bool))


def fitness(pop: Population, X, y, w=None, metric="mse", n_threads=None, with_f64=True,
            with_bound=False, u=ULP_ALLOWANCE, rf=ROUND_FLIP, exact=0):
    """(fitness from the float32 program values, fitness with every step in
    float64), as float64 arrays; the float32 result the library must match is
    the first one rounded to float32.  With with_bound=True also returns the
    first-order bound on the float32-path fitness's sensitivity and, per
    program, the number of rows with a protected predicate near its
    threshold.  `exact` as in evaluate_pairs."""
    X, N = _ds(X)
    y = np.ascontiguousarray(y, dtype=np.float32)
    w = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
    m = METRICS[metric] if isinstance(metric, str) else int(metric)
    f32p = np.empty(pop.n_programs, np.float64)
    f64 = np.empty(pop.n_programs, np.float64) if (with_f64 or with_bound) else None
    fb = np.empty(pop.n_programs, np.float64) if with_bound else None
    fn = np.empty(pop.n_programs, np.int32) if with_bound else None
    lib().orc_fitness(_p(pop.nodes), _p(pop.prog_off), _p(pop.consts), _p(pop.const_off),
                      pop.n_programs, _p(X), N, N, _p(y), _p(w), m, _p(f32p), _p(f64), float(u),
                      float(rf), int(exact), _p(fb), _p(fn), _threads(n_threads))
    if with_bound:
        return f32p, f64, fb, fn
    return f32p, f64


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def philox_words(seed, item, gen, tag, d0, n):
    out = np.empty(n, np.uint32)
    lib().orc_philox_words(seed, item, gen, tag, d0, n, _p(out))
    return out


def tournament(fit, length, larger_is_better, parsimony, k, n_tournaments, seed, generation):
    fit = np.ascontiguousarray(fit, dtype=np.float32)
    length = np.ascontiguousarray(length, dtype=np.int32)
    win = np.empty(n_tournaments, np.int32)
    lib().orc_tournament(_p(fit), _p(length), fit.shape[0], int(bool(larger_is_better)),
                         float(parsimony), int(k), int(n_tournaments), int(seed),
                         int(generation), _p(win))
    return win


def tournament_draws(n_programs, k, t, seed, generation):
    out = np.empty(k, np.int32)
    lib().orc_tournament_draws(n_programs, k, t, seed, generation, _p(out))
    return out


def build_population(n_programs, n_features, method="rhh", min_depth=2, max_depth=6,
                     min_len=1, max_len=200, fmask=DEFAULT_FMASK, const_lo=-1.0,
                     const_hi=1.0, max_consts=0, seed=0) -> Population:
    m = INIT[method] if isinstance(method, str) else int(method)
    L = lib()
    tn = np.zeros(1, np.int64)
    tc = np.zeros(1, np.int64)
    args = (n_programs, n_features, m, min_depth, max_depth, min_len, max_len, fmask,
            const_lo, const_hi, max_consts, seed)
    rc = L.orc_build_population(*args, None, 0, None, None, 0, None, None, _p(tn), _p(tc))
    if rc != 0:
        raise ValueError(f"orc_build_population: bad arguments (rc={rc})")
    nodes = np.zeros(max(int(tn[0]), 1), np.uint32)
    consts = np.zeros(max(int(tc[0]), 1), np.float32)
    po = np.zeros(n_programs + 1, np.int64)
    co = np.zeros(n_programs + 1, np.int64)
    ln = np.zeros(n_programs, np.int32)
    rc = L.orc_build_population(*args, _p(nodes), nodes.shape[0], _p(po), _p(consts),
                                consts.shape[0], _p(co), _p(ln), _p(tn), _p(tc))
    if rc != 0:
        raise ValueError(f"orc_build_population failed (rc={rc})")
    return Population(nodes=nodes[:int(tn[0])], prog_off=po, consts=consts[:int(tc[0])],
                      const_off=co, length=ln)


def grad_consts(pop: Population, X, y, w=None, metric="mse", gscale=None, n_threads=None,
                mc_u=0.0, mc_seed=0, f32_tape=False):
    """(d fitness / d consts for every constant, fitness) in float64.

    mc_u > 0 perturbs every operation's result by a relative +-mc_u (Monte
    Carlo arithmetic, signs from SplitMix64 keyed by mc_seed): the spread of
    the results over a few seeds estimates their float32 conditioning.
    f32_tape=True takes the derivative at the float32 evaluation (its
    values and protected branches), the partials still in float64; with
    mc_u > 0 only the reverse sweep is then perturbed."""
    X, N = _ds(X)
    y = np.ascontiguousarray(y, dtype=np.float32)
    w = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
    m = METRICS[metric] if isinstance(metric, str) else int(metric)
    gs = None if gscale is None else np.ascontiguousarray(gscale, dtype=np.float64)
    g = np.zeros(max(pop.consts.shape[0], 1), np.float64)
    fit = np.zeros(pop.n_programs, np.float64)
    lib().orc_grad_consts(_p(pop.nodes), _p(pop.prog_off), _p(pop.consts), _p(pop.const_off),
                          pop.n_programs, _p(X), N, N, _p(y), _p(w), m, _p(gs), _p(g), _p(fit),
                          float(mc_u), int(mc_seed), 1 if f32_tape else 0, _threads(n_threads))
    return g[:pop.consts.shape[0]], fit


@dataclass
class EvolveParams:
    """Genetic-operation probabilities (reproduction takes the rest), the
    per-node point replacement probability, the crossover length bound and
    the seed of the mutation streams."""
    p_crossover: float = 0.7
    p_subtree: float = 0.1
    p_hoist: float = 0.05
    p_point: float = 0.1
    p_point_replace: float = 0.05
    max_len: int = 4096
    seed: int = 0


@dataclass
class InitParams:
    """The initialisation settings donors of subtree mutation follow."""
    n_features: int
    method: str = "rhh"
    min_depth: int = 2
    max_depth: int = 6
    min_len: int = 1
    max_len: int = 200
    fmask: int = DEFAULT_FMASK
    const_lo: float = -1.0
    const_hi: float = 1.0
    max_consts: int = 0


def plan_generation(ev: EvolveParams, n_offspring, generation):
    """(ops, first_tournament, n_tournaments) of the pre-draw."""
    ops = np.zeros(max(n_offspring, 1), np.int32)
    ft = np.zeros(max(n_offspring, 1), np.int32)
    nt = np.zeros(1, np.int32)
    lib().orc_plan_generation(ev.p_crossover, ev.p_subtree, ev.p_hoist, ev.p_point, int(ev.seed),
                              int(n_offspring), int(generation), _p(ops), _p(ft), _p(nt))
    return ops[:n_offspring], ft[:n_offspring], int(nt[0])


def mutate(ev: EvolveParams, init: InitParams, parents: Population, ops, first_t, winners, generation):
    """The offspring population (one per entry of ops)."""
    n_off = int(len(ops))
    ops = np.ascontiguousarray(ops, np.int32)
    first_t = np.ascontiguousarray(first_t, np.int32)
    winners = np.ascontiguousarray(winners, np.int32)
    cap = max(n_off * max(int(ev.max_len), int(parents.length.max(initial=1)), 256) * 2, 1)
    nodes = np.zeros(cap, np.uint32)
    consts = np.zeros(cap, np.float32)
    po = np.zeros(n_off + 1, np.int64)
    co = np.zeros(n_off + 1, np.int64)
    ln = np.zeros(max(n_off, 1), np.int32)
    tn = np.zeros(1, np.int64)
    tc = np.zeros(1, np.int64)
    pc = parents.consts if parents.consts.shape[0] else np.zeros(1, np.float32)
    rc = lib().orc_mutate(ev.p_crossover, ev.p_subtree, ev.p_hoist, ev.p_point, ev.p_point_replace,
                          int(ev.max_len), int(ev.seed), INIT[init.method], init.n_features, init.min_depth,
                          init.max_depth, init.min_len, init.max_len, init.fmask, init.const_lo,
                          init.const_hi, init.max_consts, _p(parents.nodes), _p(parents.prog_off), _p(pc),
                          _p(parents.const_off), _p(ops), _p(first_t), _p(winners), n_off, int(generation),
                          _p(nodes), cap, _p(po), _p(consts), cap, _p(co), _p(ln), _p(tn), _p(tc))
    if rc != 0:
        raise RuntimeError(f"orc_mutate failed ({rc})")
    return Population(nodes[:int(tn[0])].copy(), po, consts[:int(tc[0])].copy(), co, ln[:n_off].copy())

