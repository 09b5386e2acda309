"""gp_fitness_noalloc (the entry point that allocates nothing) against
gp_fitness: the same kernels and launch configuration on the library's static
device scratch, so every program's fitness must be bit-identical; and both
within the parity tolerance of the oracle (programs over the correctly
rounded function set are bit-exact per row, fitness differs only in the order
of the float64 sums).

Two calls in a row on the same device array, the second on a smaller
population and dataset, then a call whose scratch would exceed the array:
rejected before anything is launched, the output left untouched."""
import numpy as np
import pytest

import oracle
import synth
from _parity import check_fitness_exact, to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    import torch
    import paper_2110_11226_amd as gp
    torch.cuda.set_device(0)
    gp.set_launch_config(None)
    yield gp
    gp.set_launch_config(None)


def case(gp, P, N, seed, metric):
    import torch
    X, y = synth.higgs_like(N, seed=seed) if metric == "logloss" else synth.pagie(N, seed=seed)
    F = X.shape[0]
    host = gp.build_population(P, F, method="exact_len", min_len=1, max_len=120, seed=seed)
    pop = gp.DevicePopulation(host, n_features=F)
    data = gp.DeviceDataset(X, y)
    want = gp.fitness(pop, data, metric)
    got = torch.full((P,), 12345.0, dtype=torch.float32, device="cuda")
    gp.fitness_noalloc(pop, data, metric, out=got)
    torch.cuda.synchronize()
    w, g = want.cpu().numpy(), got.cpu().numpy()
    same = (g.view(np.uint32) == w.view(np.uint32)) | (np.isnan(g) & np.isnan(w))
    assert same.all(), f"{metric} P={P} N={N}: {int((~same).sum())} programs differ from gp_fitness"
    f32p, f64 = oracle.fitness(to_oracle(host), X, y, None, metric, n_threads=8)
    check_fitness_exact(g, f32p, f64, label=f"noalloc {metric} P={P} N={N}")
    return g


@pytest.mark.parametrize("metric", ["mse", "pearson", "logloss"])
def test_two_calls_second_smaller(gp, metric):
    print(f"noalloc {metric}: P=300 N=200000, then P=100 N=50000", flush=True)
    case(gp, 300, 200_000, 11231, metric)
    case(gp, 100, 50_000, 11232, metric)


def test_oversize_rejected_untouched(gp):
    import torch
    # 64-row chunks: 16384 chunks x 600 programs x 8 bytes of partial sums
    # exceed the 64 MiB array
    N, P = 1 << 20, 600
    X, y = synth.pagie(N, seed=11233)
    host = gp.build_population(P, 2, method="rhh", min_depth=2, max_depth=4, seed=5)
    pop = gp.DevicePopulation(host, n_features=2)
    data = gp.DeviceDataset(X, y)
    gp.set_launch_config((1, 2, 1, 4))
    try:
        out = torch.full((P,), 7.0, dtype=torch.float32, device="cuda")
        with pytest.raises(gp.GPError, match="above the limit"):
            gp.fitness_noalloc(pop, data, "mse", out=out)
        torch.cuda.synchronize()
        assert bool((out == 7.0).all())
    finally:
        gp.set_launch_config(None)
    # the array still serves a call that fits
    case(gp, 64, 4096, 11234, "mse")
