"""GPU parity of Spearman fitness (Sec. III-C3: the rank correlation whose
ranks come from a sort) against the oracle's Spearman.

The two sides rank their own float32 outputs, which may differ by a few
ulps wherever a transcendental sits in the program; rows whose values are
that close may then be ordered (or tied) differently.  The oracle bounds the
effect (the components of rows whose value intervals overlap); a program's
fitness must agree within 1e-6 relative plus that bound.  Programs of
correctly rounded operations have a zero bound and must agree to float32
rounding of the same float64 result."""
import os

import numpy as np
import pytest

import oracle
import synth
from _parity import CR_MASK, to_oracle

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def gp():
    import torch
    import paper_2110_11226_amd as gp
    torch.cuda.set_device(0)
    return gp


def gpu_spearman(gp, host, X, y, w, F):
    import torch
    pop = gp.DevicePopulation(host, n_features=F)
    data = gp.DeviceDataset(X, y, w)
    f = gp.fitness(pop, data, "spearman")
    torch.cuda.synchronize()
    return f.cpu().numpy().astype(np.float64)


def check(got, f32p, fb, fn, label):
    tight = 0
    for p in range(len(got)):
        if fn[p]:
            continue            # a protected predicate near its threshold
        if np.isnan(f32p[p]):
            assert np.isnan(got[p]), (label, p)
            continue
        tol = 1e-6 * abs(f32p[p]) + 1e-7 + fb[p]
        assert abs(got[p] - f32p[p]) <= tol, (label, p, got[p], f32p[p], fb[p])
        tight += fb[p] == 0.0
    return tight


@pytest.mark.parametrize("weighted", [False, True])
def test_spearman_rhh_population(gp, weighted):
    N = 4096 + 77
    X, y = synth.pagie(N, seed=11227)
    w = synth.weights(N, seed=3) if weighted else None
    host = gp.build_population(256, 2, "rhh", min_depth=2, max_depth=6, seed=2111)
    got = gpu_spearman(gp, host, X, y, w, 2)
    f32p, f64, fb, fn = oracle.fitness(to_oracle(host), X, y, w, "spearman", n_threads=NT, with_bound=True,
                                    exact=CR_MASK)
    tight = check(got, f32p, fb, fn, f"rhh w={weighted}")
    # every function of the set is correctly rounded on both sides: every
    # program's outputs are the oracle's, so every bound is zero
    assert tight == 256


@pytest.mark.parametrize("N", [3000, 70_000])
def test_spearman_ties_everywhere(gp, N):
    """Integer features and a coarse target: most values tie on both sides,
    and at 70,000 rows tied runs reach across many blocks of positions of the
    correlation kernel (a constant program is one run of all rows)."""
    rng = np.random.default_rng(5)
    X = rng.integers(-4, 5, size=(2, N)).astype(np.float32)
    y = np.round(rng.normal(size=N) * 2).astype(np.float32)
    fmask = sum(1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL, oracle.NEG))
    host = gp.build_population(200, 2, "exact_len", min_len=1, max_len=40, function_mask=fmask, seed=9)
    got = gpu_spearman(gp, host, X, y, None, 2)
    f32p, f64, fb, fn = oracle.fitness(to_oracle(host), X, y, None, "spearman", n_threads=NT, with_bound=True,
                                    exact=CR_MASK)
    # exact arithmetic on small integers: identical values, ranks and ties on both sides
    assert np.all(fb == 0.0)
    assert np.allclose(got, f32p, rtol=1e-6, atol=1e-7)
    assert np.sum(f32p == 0.0) >= 1            # constant programs exist


def test_spearman_nan_and_constant_programs(gp):
    N = 1000
    X, y = synth.pagie(N, seed=4)
    X = X.copy()
    X[0, 17] = np.nan
    progs = [([oracle.node(oracle.VAR, 0)], []), ([oracle.node(oracle.VAR, 1)], []),
             ([oracle.node(oracle.CONST, 0)], [2.0]),
             ([oracle.node(oracle.MUL), oracle.node(oracle.VAR, 1), oracle.node(oracle.VAR, 1)], [])]
    op = oracle.from_programs(progs)
    host = gp.HostPopulation(op.nodes, op.prog_off, op.consts, op.const_off, op.length)
    got = gpu_spearman(gp, host, X, y, None, 2)
    f32p, _ = oracle.fitness(op, X, y, None, "spearman")
    assert np.isnan(got[0]) and np.isnan(f32p[0])
    assert got[2] == 0.0 and f32p[2] == 0.0
    assert np.allclose(got[[1, 3]], f32p[[1, 3]], rtol=1e-6)


def test_spearman_nan_target_is_nan_for_every_program(gp):
    """A NaN in the target (either sign, first, last or inside a tile) makes
    every program's Spearman fitness NaN, in every batch, as in the oracle."""
    N = 9000
    X, y0 = synth.pagie(N, seed=8)
    host = gp.build_population(40, 2, "rhh", min_depth=1, max_depth=4, seed=3)
    for k in (0, N - 1, 4500):
        for nan in (np.float32(np.nan), -np.float32(np.nan)):
            y = y0.copy()
            y[k] = nan
            gp.set_spearman_workset(16 * N * 7)          # batches of 7 programs
            try:
                got = gpu_spearman(gp, host, X, y, None, 2)
            finally:
                gp.set_spearman_workset(0)
            f32p, _ = oracle.fitness(to_oracle(host), X, y, None, "spearman")
            assert np.isnan(got).all() and np.isnan(f32p).all(), (k, nan)
    # and the next call, without the NaN, is ordinary again
    got = gpu_spearman(gp, host, X, y0, None, 2)
    f32p, f64, fb, fn = oracle.fitness(to_oracle(host), X, y0, None, "spearman", n_threads=NT, with_bound=True,
                                    exact=CR_MASK)
    check(got, f32p, fb, fn, "after NaN target")


@pytest.mark.parametrize("N,workset", [(1, 0), (2, 0), (63, 0), (4097, 0), (1_500_000, 0),
                                       (1_500_000, 700 << 20)])
def test_spearman_sizes_and_batches(gp, N, workset):
    """Ragged tiles, tiny inputs, 1.5M rows in one batch and, with the working
    set limited to 700 MiB (16 bytes per row per program: 30 programs a
    batch), in six batches, the last one short."""
    X, y = synth.pagie(N, seed=N)
    fmask = sum(1 << o for o in (oracle.ADD, oracle.SUB, oracle.MUL, oracle.DIV, oracle.NEG, oracle.SQRT))
    P = 160 if N > 100_000 else 48
    host = gp.build_population(P, 2, "rhh", min_depth=1, max_depth=5, function_mask=fmask, seed=7)
    gp.set_spearman_workset(workset)
    try:
        got = gpu_spearman(gp, host, X, y, None, 2)
    finally:
        gp.set_spearman_workset(0)
    f32p, f64, fb, fn = oracle.fitness(to_oracle(host), X, y, None, "spearman", n_threads=NT, with_bound=True,
                                    exact=CR_MASK)
    check(got, f32p, fb, fn, f"N={N}")
