"""Pins of the oracle's tournament selection (Sec. III-C1, Eqs. (parsimony),
(fitness)): special cases with known winners, a brute-force recheck of the
winner over the drawn entrants, and the closed-form probability that the best
program wins a tournament."""
import numpy as np
import pytest

import oracle


def test_k1_returns_the_draw():
    rng = np.random.default_rng(0)
    P = 97
    fit = rng.normal(size=P).astype(np.float32)
    ln = rng.integers(1, 200, size=P).astype(np.int32)
    win = oracle.tournament(fit, ln, False, 0.01, 1, 500, 42, 3)
    for t in range(500):
        assert win[t] == oracle.tournament_draws(P, 1, t, 42, 3)[0]


def test_all_equal_fitness_returns_first_draw():
    P = 50
    fit = np.full(P, 2.5, np.float32)
    ln = np.full(P, 10, np.int32)
    win = oracle.tournament(fit, ln, False, 0.01, 7, 300, 9, 0)
    for t in range(300):
        assert win[t] == oracle.tournament_draws(P, 7, t, 9, 0)[0]


def test_huge_parsimony_picks_shortest_drawn():
    rng = np.random.default_rng(1)
    P = 64
    fit = rng.normal(size=P).astype(np.float32)
    ln = rng.permutation(np.arange(1, P + 1)).astype(np.int32)   # distinct lengths
    win = oracle.tournament(fit, ln, False, 1e6, 5, 400, 11, 2)
    for t in range(400):
        d = oracle.tournament_draws(P, 5, t, 11, 2)
        assert win[t] == d[np.argmin(ln[d])]
    win = oracle.tournament(fit, ln, True, 1e6, 5, 400, 11, 2)      # larger is better
    for t in range(400):
        d = oracle.tournament_draws(P, 5, t, 11, 2)
        assert win[t] == d[np.argmin(ln[d])]


@pytest.mark.parametrize("larger", [False, True])
@pytest.mark.parametrize("c", [0.0, 1e-3, 1e-2])
def test_winner_is_best_drawn_and_earliest_on_ties(larger, c):
    rng = np.random.default_rng(2)
    P = 40
    fit = np.round(rng.normal(size=P), 1).astype(np.float32)    # many ties
    ln = rng.integers(1, 5, size=P).astype(np.int32)
    fit[3] = np.nan
    k, T = 20, 300
    win = oracle.tournament(fit, ln, larger, c, k, T, 5, 1)
    c32 = np.float32(c)
    for t in range(T):
        d = oracle.tournament_draws(P, k, t, 5, 1)
        pen = (c32 * ln[d].astype(np.float32)).astype(np.float32)
        adj = (fit[d] - pen) if larger else (fit[d] + pen)
        ok = ~np.isnan(adj)
        if not ok.any():
            assert win[t] == d[0]
            continue
        best = np.max(adj[ok]) if larger else np.min(adj[ok])
        first = int(np.nonzero(ok & (adj == best))[0][0])
        assert win[t] == d[first]


def test_best_program_win_rate_closed_form():
    # with distinct fitness and no parsimony the best program wins exactly the
    # tournaments that draw it at least once: P(win) = 1 - (1 - 1/P)^k
    P, k, T = 50, 4, 200000
    fit = np.arange(P, dtype=np.float32)
    ln = np.ones(P, np.int32)
    win = oracle.tournament(fit, ln, False, 0.0, k, T, 77, 0)
    p = 1 - (1 - 1 / P) ** k
    got = np.mean(win == 0)
    sigma = np.sqrt(p * (1 - p) / T)
    assert abs(got - p) < 5 * sigma
