"""Shared helpers of the GPU parity tests (not a test module).

Tolerance policy (the acceptance bar for float work):
  * per-row program outputs: |gpu - oracle_f32| <= 1e-5 * max(1, |oracle_f32|),
    and the same non-finite class (NaN / +inf / -inf) where the oracle's value
    is not finite, on every row that is not ill-conditioned;
  * add, sub, mul, protected div, neg and protected sqrt are correctly
    rounded on both sides, so differences can only start at sin / cos / tan /
    log, where the device library and libm are each within a few ulp of the
    exact result but not bit-identical.  A row is ill-conditioned -- excluded
    from the check, counted and reported -- iff the oracle's first-order bound
    on how far a 4-ulp change of every such result can move the float32 output
    exceeds the tolerance, or a protected predicate's operand lies within its
    own bound of the 0.001 threshold, or a protected predicate differs between
    float32 and float64 (the bound follows the float64 arm);
  * fitness: |gpu - oracle| <= 1e-4 * |oracle| (oracle rounded to float32),
    same non-finite class; a program is ill-conditioned -- reported, not
    checked -- iff the bound propagated from its rows to its fitness exceeds
    that tolerance or one of its rows has a predicate near the threshold
    (within the bound, a result outside the tolerance can only be a defect).
"""
from __future__ import annotations

import numpy as np

import oracle

ROW_TOL = 1e-5
FIT_TOL = 1e-4


def to_oracle(host) -> oracle.Population:
    return oracle.Population(np.ascontiguousarray(host.nodes, np.uint32),
                             np.ascontiguousarray(host.prog_off, np.int64),
                             np.ascontiguousarray(host.consts, np.float32),
                             np.ascontiguousarray(host.const_off, np.int64),
                             np.ascontiguousarray(host.length, np.int32))


def nonfinite_class(v):
    v = np.asarray(v, np.float64)
    return np.where(np.isnan(v), 3, np.where(np.isposinf(v), 1, np.where(np.isneginf(v), 2, 0)))


def check_rows(got, ra, label=""):
    """Element-wise row parity against an oracle.RowAnalysis; returns
    (n_checked, n_ill).  Raises on a violation with the first offending index."""
    got = np.asarray(got, np.float32).ravel()
    g = got.astype(np.float64)
    r = np.asarray(ra.v32, np.float32).ravel().astype(np.float64)
    o64 = np.asarray(ra.v64, np.float64).ravel()
    bound = np.asarray(ra.bound, np.float64).ravel()
    with np.errstate(invalid="ignore"):
        tol = ROW_TOL * np.maximum(1.0, np.abs(r))
        ill = ra.near.ravel() | ra.flip.ravel() | ~(bound <= tol)
    ok = ~ill
    fin = np.isfinite(r)
    nf = ok & ~fin
    bad_nf = nf & (nonfinite_class(g) != nonfinite_class(r))
    if bad_nf.any():
        i = int(np.nonzero(bad_nf)[0][0])
        raise AssertionError(f"{label}: non-finite class differs at {i}: gpu {g[i]} oracle {r[i]}")
    fm = ok & fin
    with np.errstate(invalid="ignore"):
        bad = fm & ~(np.abs(g - r) <= tol)
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(f"{label}: {int(bad.sum())} rows out of tolerance; first at {i}: "
                             f"gpu {g[i]!r} oracle32 {r[i]!r} oracle64 {o64[i]!r} bound {bound[i]!r}")
    return int(ok.sum()), int(ill.sum())


def check_fitness(got, f32p, f64, fbound, fnear, label=""):
    """Fitness parity; returns (n_checked, n_ill, max_rel_err_vs_f64)."""
    got = np.asarray(got, np.float32).astype(np.float64)
    ref = np.asarray(f32p, np.float64).astype(np.float32).astype(np.float64)
    f64 = np.asarray(f64, np.float64)
    fbound = np.asarray(fbound, np.float64)
    with np.errstate(invalid="ignore"):
        ill = (np.asarray(fnear) > 0) | ~(fbound <= FIT_TOL * np.abs(ref))
    ill &= ~((fbound == 0) & (np.asarray(fnear) == 0))
    ok = ~ill
    fin = np.isfinite(ref)
    nf = ok & ~fin
    bad_nf = nf & (nonfinite_class(got) != nonfinite_class(ref))
    if bad_nf.any():
        i = int(np.nonzero(bad_nf)[0][0])
        raise AssertionError(f"{label}: non-finite fitness class differs at program {i}: "
                             f"{got[i]} vs {ref[i]}")
    fm = ok & fin
    with np.errstate(invalid="ignore", divide="ignore"):
        bad = fm & ~(np.abs(got - ref) <= FIT_TOL * np.abs(ref))
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(f"{label}: {int(bad.sum())} programs out of tolerance; first {i}: "
                             f"gpu {got[i]!r} oracle {ref[i]!r} (f64 {f64[i]!r}, bound {fbound[i]!r})")
    with np.errstate(invalid="ignore", divide="ignore"):
        e64 = np.abs(got - f64) / np.abs(f64)
    m = np.isfinite(e64) & fm
    return int(fm.sum()), int(ill.sum()), float(e64[m].max()) if m.any() else 0.0
