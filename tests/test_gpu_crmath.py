"""The device's correctly rounded sin, cos, log (gp_crmath.h) and protected
square root against the oracle's float32 functions, on every float.

The function set of Sec. III-D1 names its functions but no library; both
sides round each function's exact value once, to nearest, so the two must
agree bit for bit on all 2^32 inputs.  The values go through the evaluation
kernel itself: programs [SIN x0], [COS x0], [LOG x0] (the protected log
of |x0|, 0 where |x0| <= 0.001 or x0 is NaN) and [SQRT x0] (sqrt|x0|, IEEE
correctly rounded on the oracle's side) over a dataset whose rows are every
float bit pattern, 2^28 rows at a time.
"""
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

NT = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def gp():
    import torch
    import paper_2110_11226_amd as gp
    torch.cuda.set_device(0)
    yield gp


def programs(gp):
    n = oracle.node
    op = oracle.from_programs([([n(oracle.SIN), n(oracle.VAR, 0)], []), ([n(oracle.COS), n(oracle.VAR, 0)], []),
                               ([n(oracle.LOG), n(oracle.VAR, 0)], []), ([n(oracle.SQRT), n(oracle.VAR, 0)], [])])
    return op, gp.HostPopulation(op.nodes, op.prog_off, op.consts, op.const_off, op.length)


def compare(gp, op, pop, bits):
    import torch
    x = bits.view(np.float32)
    X = np.ascontiguousarray(x[None, :])
    out = gp.evaluate(pop, gp.DeviceDataset(X))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = oracle.evaluate_f32(op, X, n_threads=NT)
    same = (got.view(np.uint32) == ref.view(np.uint32)) | (np.isnan(got) & np.isnan(ref))
    if not same.all():
        p, i = np.argwhere(~same)[0]
        raise AssertionError(f"{int((~same).sum())} results differ; first: function {['sin', 'cos', 'log', 'sqrt'][p]} "
                             f"x = {x[i]!r} ({bits[i]:#010x}): gpu {got[p, i]!r} oracle {ref[p, i]!r}")
    return got.size


def test_sin_cos_log_sqrt_every_float(gp):
    op, host = programs(gp)
    pop = gp.DevicePopulation(host, n_features=1)
    oracle.cr_reset()
    chunk = 1 << 28
    n = 0
    for c in range(1 << 32 >> 28):
        bits = np.arange(c * chunk, (c + 1) * chunk, dtype=np.uint64).astype(np.uint32)
        n += compare(gp, op, pop, bits)
    # the oracle decided every rounding it made (no case left to its
    # extended-precision fallback without a margin)
    assert oracle.cr_undecided() == 0
    print(f"{n} function values bit-identical")


def test_special_and_boundary_inputs(gp):
    """Zeros, infinities, NaN, the protected-log threshold, the switch to
    Payne-Hanek reduction at 2^20 and the small-argument cut at 2^-12, in
    both signs."""
    op, host = programs(gp)
    pop = gp.DevicePopulation(host, n_features=1)
    f = np.float32
    base = [0.0, 1.0, 0.001, 2.0 ** 20, 2.0 ** -12, np.pi / 2, np.pi, 3.4e38, 1e-45]
    vals = []
    for v in base:
        v = f(v)
        vals += [v, np.nextafter(v, f(np.inf)), np.nextafter(v, f(0))]
    vals += [np.inf, np.nan]
    vals = np.array(vals + [-v for v in vals], np.float32)
    compare(gp, op, pop, vals.view(np.uint32))
