"""Shared helpers of the GPU parity tests (not a test module).

Tolerance policy (the acceptance bar for float work):
  * per-row program outputs: |gpu - oracle_f32| <= 1e-5 * max(1, |oracle_f32|)
    + bound, and the same non-finite class where the oracle's value is not
    finite.  `bound` is the oracle's rigorous bound on how far the float32
    output can move when every library-function result (sin, cos, tan, log
    and the wider set) moves by 4 ulp: add, sub, mul, protected div, neg and
    protected sqrt are correctly rounded on both sides, and the device library
    and the oracle's correctly rounded functions differ by a few ulp at most.
    Rows whose bound is 0 are held to the plain tolerance.  A row escapes the
    check -- counted and reported, never silently -- only where no bound
    exists: a protected predicate's operand lies within its own bound of the
    0.001 threshold (or float32 and float64 take different protected
    branches), or the bound is not finite;
  * fitness: |gpu - oracle| <= 1e-4 * |oracle| + fitness bound (oracle rounded
    to float32), the same non-finite class; a program escapes only if one of
    its rows has a predicate near its threshold or its bound is not finite.

Each check returns a ParityStats (iterable as (checked, escaped[, max rel
error against float64])) and, when GP_PARITY_LOG names a file, appends one
JSON line with its counts there.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass

import numpy as np

import oracle

ROW_TOL = 1e-5
FIT_TOL = 1e-4


@dataclass
class ParityStats:
    label: str
    kind: str           # "rows" or "fitness"
    checked: int        # compared: tight + bounded
    tight: int          # compared against the plain tolerance (bound within it)
    bounded: int        # compared against tolerance + bound (bound above the tolerance)
    escaped: int        # no bound: predicate near its threshold, or infinite bound
    max_rel_err_f64: float = 0.0

    def __iter__(self):
        yield self.checked
        yield self.escaped
        if self.kind == "fitness":
            yield self.max_rel_err_f64

    def record(self):
        path = os.environ.get("GP_PARITY_LOG")
        if path:
            with open(path, "a") as f:
                f.write(json.dumps(self.__dict__) + "\n")
        return self


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
    """Element-wise row parity against an oracle.RowAnalysis.  Raises on a
    violation, naming the first offending index."""
    got = np.asarray(got, np.float32).ravel()
    g = got.astype(np.float64)
    r = np.asarray(ra.v32, np.float32).ravel().astype(np.float64)
    o64 = np.asarray(ra.v64, np.float64).ravel()
    bound = np.asarray(ra.bound, np.float64).ravel()
    with np.errstate(invalid="ignore"):
        tol = ROW_TOL * np.maximum(1.0, np.abs(r))
        esc = ra.near.ravel() | ra.flip.ravel() | ~np.isfinite(bound)
    ok = ~esc
    fin = np.isfinite(r)
    nf = ok & ~fin
    bad_nf = nf & (nonfinite_class(g) != nonfinite_class(r))
    if bad_nf.any():
        i = int(np.nonzero(bad_nf)[0][0])
        raise AssertionError(f"{label}: non-finite class differs at {i}: gpu {g[i]} oracle {r[i]}")
    fm = ok & fin
    with np.errstate(invalid="ignore"):
        bad = fm & ~(np.abs(g - r) <= tol + bound)
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(f"{label}: {int(bad.sum())} rows out of tolerance; first at {i}: "
                             f"gpu {g[i]!r} oracle32 {r[i]!r} oracle64 {o64[i]!r} bound {bound[i]!r}")
    with np.errstate(invalid="ignore"):
        tight = ok & (bound <= tol)
    return ParityStats(label, "rows", int(ok.sum()), int(tight.sum()), int((ok & ~tight).sum()),
                       int(esc.sum())).record()


def check_fitness(got, f32p, f64, fbound, fnear, label=""):
    """Fitness parity of every program."""
    got = np.asarray(got, np.float32).astype(np.float64)
    ref = np.asarray(f32p, np.float64).astype(np.float32).astype(np.float64)
    f64 = np.asarray(f64, np.float64)
    fbound = np.asarray(fbound, np.float64)
    fnear = np.asarray(fnear)
    esc = (fnear > 0) | ~np.isfinite(fbound)
    ok = ~esc
    fin = np.isfinite(ref)
    nf = ok & ~fin
    bad_nf = nf & (nonfinite_class(got) != nonfinite_class(ref))
    if bad_nf.any():
        i = int(np.nonzero(bad_nf)[0][0])
        raise AssertionError(f"{label}: non-finite fitness class differs at program {i}: "
                             f"{got[i]} vs {ref[i]}")
    fm = ok & fin
    with np.errstate(invalid="ignore", divide="ignore"):
        tol = FIT_TOL * np.abs(ref)
        bad = fm & ~(np.abs(got - ref) <= tol + fbound)
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(f"{label}: {int(bad.sum())} programs out of tolerance; first {i}: "
                             f"gpu {got[i]!r} oracle {ref[i]!r} (f64 {f64[i]!r}, bound {fbound[i]!r})")
    with np.errstate(invalid="ignore", divide="ignore"):
        e64 = np.abs(got - f64) / np.abs(f64)
        tight = ok & (fbound <= tol)
    m = np.isfinite(e64) & fm
    return ParityStats(label, "fitness", int(ok.sum()), int(tight.sum()), int((ok & ~tight).sum()),
                       int(esc.sum()), float(e64[m].max()) if m.any() else 0.0).record()


# Functions both sides round correctly: the arithmetic ones, protected div and
# sqrt, and (on the device, gp_crmath.h; in the oracle, its float32 path)
# sin, cos and log.  A program over these has one float32 value per row.
CR_OPS = (oracle.ADD, oracle.SUB, oracle.MUL, oracle.DIV, oracle.NEG, oracle.SQRT, oracle.LOG,
          oracle.SIN, oracle.COS, oracle.MAX, oracle.MIN, oracle.ABS, oracle.INV, oracle.SQ, oracle.CUBE)
CR_MASK = sum(1 << o for o in CR_OPS)


def check_rows_exact(got, ref32, label=""):
    """Bit-for-bit row parity (NaN matches NaN) for programs whose functions
    are all correctly rounded on both sides."""
    got = np.asarray(got, np.float32).ravel()
    ref = np.asarray(ref32, np.float32).ravel()
    same = (got.view(np.uint32) == ref.view(np.uint32)) | (np.isnan(got) & np.isnan(ref))
    if not same.all():
        i = int(np.nonzero(~same)[0][0])
        raise AssertionError(f"{label}: {int((~same).sum())} of {got.size} rows differ; first at {i}: "
                             f"gpu {got[i]!r} ({got.view(np.uint32)[i]:#010x}) oracle {ref[i]!r} "
                             f"({ref.view(np.uint32)[i]:#010x})")
    return ParityStats(label, "rows", got.size, got.size, 0, 0).record()


def check_fitness_exact(got, f32p, f64=None, label=""):
    """Fitness of programs whose rows are bit-exact: every program within the
    tolerance (the two sides differ only in the order of the float64 sums),
    the same non-finite class, nothing excluded."""
    got = np.asarray(got, np.float32).astype(np.float64)
    ref = np.asarray(f32p, np.float64).astype(np.float32).astype(np.float64)
    fin = np.isfinite(ref)
    bad_nf = ~fin & (nonfinite_class(got) != nonfinite_class(ref))
    if bad_nf.any():
        i = int(np.nonzero(bad_nf)[0][0])
        raise AssertionError(f"{label}: non-finite fitness class differs at program {i}: {got[i]} vs {ref[i]}")
    with np.errstate(invalid="ignore"):
        bad = fin & ~(np.abs(got - ref) <= FIT_TOL * np.abs(ref))
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(f"{label}: {int(bad.sum())} programs out of tolerance; first {i}: "
                             f"gpu {got[i]!r} oracle {ref[i]!r}")
    e64 = 0.0
    if f64 is not None:
        f64 = np.asarray(f64, np.float64)
        with np.errstate(invalid="ignore", divide="ignore"):
            e = np.abs(got - f64) / np.abs(f64)
        m = np.isfinite(e) & fin
        e64 = float(e[m].max()) if m.any() else 0.0
    return ParityStats(label, "fitness", got.size, got.size, 0, 0, e64).record()
