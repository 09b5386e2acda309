"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds input recipes only -- datasets, targets and weights -- and
none of the method's arithmetic (no program evaluation, no metric, no
selection).  Both the test-suite and the benchmark draw their inputs here, so
the GPU library and the CPU oracle see identical bytes.

Datasets are feature-major, ``X[f, r]`` (the column-major layout of Sec. III),
float32, C-contiguous.

Recipes:
  * ``pagie``: x, y ~ U[-5, 5] (float32), target the Pagie polynomial
    (Sec. IV-A, Eq. (pagie)) 1/(1+x^-4) + 1/(1+y^-4), written as
    x^4/(1+x^4) + y^4/(1+y^4) so that it is finite at 0, computed in float64
    and rounded to float32.  The paper subsamples grids of 64^2 .. 4096^2
    points of the same square; uniform sampling stands in for the grid.
  * ``higgs_like``: 28 standard-normal features (the Higgs column count of
    Sec. IV-B), labels Bernoulli(sigmoid(g(x))) for a fixed 30-node
    expression g (below).  Stands in for the Higgs dataset, which is not
    available here.
  * ``diff_target``: 8 features ~ U[-3, 3], target a fixed 40-node expression
    plus Gaussian noise of variance 0.01 (sigma 0.1).
"""
from __future__ import annotations

import numpy as np


def pagie(n_rows: int, seed: int = 11227):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-5.0, 5.0, size=(2, n_rows)).astype(np.float32)
    x = X[0].astype(np.float64)
    z = X[1].astype(np.float64)
    x4 = x ** 4
    z4 = z ** 4
    y = (x4 / (1.0 + x4) + z4 / (1.0 + z4)).astype(np.float32)
    return np.ascontiguousarray(X), y


def _g30(X):
    """Fixed 30-node expression over features 0..27, in prefix form
    ADD(MUL(SUB(x0, MUL(x1, 0.5)), SIN(NEG(x3))),
        SUB(MUL(NEG(x5), x7),
            ADD(COS(x11), MUL(x13, SUB(x2, MUL(x19, ADD(x21, MUL(x24, COS(x26)))))))))
    evaluated directly in float64 (it is a fixed formula, not a program)."""
    x = [X[i].astype(np.float64) for i in range(X.shape[0])]
    return ((x[0] - x[1] * 0.5) * np.sin(-x[3])
            + ((-x[5]) * x[7]
               - (np.cos(x[11]) + x[13] * (x[2] - x[19] * (x[21] + x[24] * np.cos(x[26]))))))


def higgs_like(n_rows: int, seed: int = 11230, n_features: int = 28):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal(size=(n_features, n_rows), dtype=np.float32)
    logit = _g30(X)
    p = 1.0 / (1.0 + np.exp(-logit))
    y = (rng.random(n_rows) < p).astype(np.float32)
    return np.ascontiguousarray(X), y


def _t40(X):
    """Fixed 40-node expression over features 0..7, in prefix form
    ADD(ADD(ADD(SIN(MUL(x0, x1)), MUL(x2, COS(SUB(x3, 0.7)))),
            SUB(MUL(ADD(x4, 1.3), SUB(x5, MUL(x6, 0.4))),
                MUL(x7, SIN(ADD(x0, MUL(x3, x5)))))),
        MUL(COS(x1), SUB(x6, MUL(x2, NEG(x4)))))
    evaluated directly in float64."""
    x = [X[i].astype(np.float64) for i in range(X.shape[0])]
    return ((np.sin(x[0] * x[1]) + x[2] * np.cos(x[3] - 0.7))
            + ((x[4] + 1.3) * (x[5] - x[6] * 0.4) - x[7] * np.sin(x[0] + x[3] * x[5]))
            + np.cos(x[1]) * (x[6] - x[2] * (-x[4])))


def diff_target(n_rows: int, seed: int = 11231, n_features: int = 8):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-3.0, 3.0, size=(n_features, n_rows)).astype(np.float32)
    y = (_t40(X) + rng.normal(0.0, 0.1, size=n_rows)).astype(np.float32)
    return np.ascontiguousarray(X), y


def weights(n_rows: int, seed: int = 7):
    """Positive sample weights ~ U[0.5, 1.5] (float32)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.5, 1.5, size=n_rows).astype(np.float32)
