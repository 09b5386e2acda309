"""The generational loop (Alg. 1 of the paper, with the Sec. III-C order:
pre-draw the genetic operations, select by tournament on the device,
mutate on the host, evaluate on the device).

Each generation is one replay of a captured graph (population upload,
fitness, tournaments, result download: ``Generation``), then the host pre-draw
(``plan_generation``) and genetic operations (``mutate``).  The graph always
runs the largest number of tournaments a generation can need (two per
offspring); a generation uses the first ones, which are the same as if only
those had been run (the draws are counter-based).  With ``use_graph=False``
the same steps run as plain calls (fitness, tournament), which gives the same
results bit for bit.
"""
from __future__ import annotations

import json
from dataclasses import asdict, dataclass, field

import numpy as np

from . import _binding as B


@dataclass
class GenerationLog:
    generation: int
    best: float
    best_program: int
    mean: float
    median: float
    total_nodes: int
    kernel_ms: float


@dataclass
class RunResult:
    population: B.HostPopulation     # the last generation's programs
    fitness: np.ndarray              # their fitness
    history: list = field(default_factory=list)
    launch_config: tuple | None = None
    generation: int = 0              # the generation number of `population`

    def write_history(self, path):
        """One JSON object per generation (generation, best, best_program,
        mean, median, total_nodes, kernel_ms)."""
        with open(path, "w") as f:
            for h in self.history:
                f.write(json.dumps(asdict(h)) + "\n")


def save_checkpoint(path, population: B.HostPopulation, generation: int, **meta):
    """The loop's whole state: the flat population and its generation
    number (the draws are counter-based, so no generator state is needed),
    with any JSON-serialisable settings in `meta`.  numpy .npz, no pickles."""
    np.savez(path, nodes=np.asarray(population.nodes, np.uint32), prog_off=np.asarray(population.prog_off, np.int64),
             consts=np.asarray(population.consts, np.float32), const_off=np.asarray(population.const_off, np.int64),
             length=np.asarray(population.length, np.int32), generation=np.int64(generation),
             meta=np.array(json.dumps(meta)))


def load_checkpoint(path):
    """(population, generation, meta) written by save_checkpoint."""
    with np.load(path, allow_pickle=False) as z:
        pop = B.HostPopulation(z["nodes"].copy(), z["prog_off"].copy(), z["consts"].copy(), z["const_off"].copy(),
                               z["length"].copy())
        return pop, int(z["generation"]), json.loads(str(z["meta"]))


def _log(g, fit, total_nodes, larger, kernel_ms):
    finite = np.where(np.isfinite(fit), fit, -np.inf if larger else np.inf)
    best = int(np.argmax(finite) if larger else np.argmin(finite))
    ok = fit[np.isfinite(fit)]
    return GenerationLog(g, float(fit[best]), best, float(ok.mean()) if ok.size else float("nan"),
                         float(np.median(ok)) if ok.size else float("nan"), int(total_nodes), kernel_ms)


def run_generations(data: B.DeviceDataset, n_generations: int, n_programs: int, init: dict,
                    metric="mse", tournament_size=20, parsimony=0.0, evolve: dict | None = None,
                    seed=0, use_graph=True, autotune=False, time_kernel=False, callback=None,
                    device_loop=False, population: B.HostPopulation | None = None,
                    first_generation: int = 0, refine: dict | None = None) -> RunResult:
    """Evolves `n_programs` programs for `n_generations` generations.

    init: initialisation settings (n_features, method, min_depth, max_depth,
    min_len, max_len, function_mask, const_lo, const_hi, max_consts, seed).
    evolve: genetic-operation settings (p_crossover, p_subtree, p_hoist,
    p_point, p_point_replace, max_len, seed); defaults are those of the
    paper's large-scale runs (crossover 0.7, subtree 0.1, hoist 0.05, point
    0.1, reproduction 0.05).

    device_loop=True keeps every generation on the device (``Evolution``):
    the same results bit for bit at the same launch configuration, with the
    history read back once at the end (the callback then runs afterwards,
    with no population, and kernel_ms is known for the last generation
    only).

    population / first_generation resume a run: the population of
    generation `first_generation` (e.g. from load_checkpoint) replaces the
    initial one, and generations are numbered from there, so the run
    continues exactly as if it had not stopped.

    refine = dict(top=0.1, steps=5, lr=1e-2) refines elite constants by
    gradient (not in the paper): in every generation, after fitness and
    before selection, the best `top` fraction of the programs that hold
    constants take `steps` Adam steps on them through gp_fitness_backward;
    a program keeps its new constants only if its fitness improved, and
    selection sees the refined fitness.  It runs as plain calls (the
    refinement sits between fitness and tournament), not in a graph or the
    device loop."""
    evolve = dict(evolve or {})
    evolve.setdefault("max_len", 1024)
    evolve.setdefault("seed", seed)
    init = dict(init)
    init_seed = init.pop("seed", seed)
    larger = B.larger_is_better(metric)
    gen_kw = {k: init[k] for k in ("min_depth", "max_depth", "min_len", "max_len", "function_mask", "const_lo",
                                   "const_hi", "max_consts") if k in init}
    if population is not None:
        if population.n_programs != n_programs:
            raise ValueError("the population's size differs from n_programs")
        pop = population
    else:
        pop = B.build_population(n_programs, init["n_features"], init.get("method", "rhh"), seed=init_seed,
                                 **gen_kw)
    g0 = int(first_generation)
    longest = int(pop.length.max(initial=1))
    cap = n_programs * max(int(evolve["max_len"]), longest)
    T_max = 2 * n_programs
    if refine is not None and device_loop:
        raise ValueError("constant refinement runs with the host loop (device_loop=False)")
    if device_loop:
        return _run_device(data, n_generations, pop, init, evolve, metric, tournament_size, parsimony, seed,
                           autotune, time_kernel, callback, larger, g0)
    graph = None
    if use_graph and refine is None:
        graph = B.Generation(data, n_programs, cap, cap, metric, parsimony, tournament_size, T_max, seed,
                             autotune=autotune, time_kernel=time_kernel)
    history = []
    try:
        for g in range(g0, g0 + n_generations + 1):
            if graph is not None:
                fit, win = graph.run(pop, g)
                kernel_ms = graph.info()[1]
            else:
                dpop = B.DevicePopulation(pop, validate=True, n_features=init["n_features"])
                fit_d = B.fitness(dpop, data, metric)
                if refine is not None:
                    pop, fit_d = _refine(pop, dpop, data, metric, fit_d, larger, **refine)
                    dpop = B.DevicePopulation(pop, validate=False)
                win_d = B.tournament(fit_d, dpop.length, metric, parsimony, tournament_size, T_max, seed, g)
                fit, win = fit_d.cpu().numpy(), win_d.cpu().numpy()
                kernel_ms = -1.0
            history.append(_log(g, fit, pop.nodes.shape[0], larger, kernel_ms))
            if callback is not None:
                callback(history[-1], pop, fit)
            if g == g0 + n_generations:
                break
            ops, ft, T = B.plan_generation(n_programs, g, **evolve)
            pop = B.mutate(pop, ops, ft, win[:T], g, init, **evolve)
        cfg = graph.info()[0] if graph is not None else None
        return RunResult(pop, fit, history, cfg, g0 + n_generations)
    finally:
        if graph is not None:
            graph.close()


def _run_device(data, n_generations, pop, init, evolve, metric, tournament_size, parsimony, seed, autotune,
                time_kernel, callback, larger, g0) -> RunResult:
    evo = B.Evolution(data, pop, init, evolve, metric=metric, parsimony=parsimony, tournament_size=tournament_size,
                      tournament_seed=seed, max_generations=max(n_generations, 1), autotune=autotune,
                      time_kernel=time_kernel, first_generation=g0)
    try:
        evo.run(n_generations)
        evo.evaluate()
        fit, nodes = evo.history()
        cfg, kernel_ms, _, _ = evo.info()
        history = [_log(g0 + k, fit[k], nodes[k], larger, kernel_ms if k == n_generations - 1 else -1.0)
                   for k in range(n_generations + 1)]
        if callback is not None:
            for k in range(n_generations + 1):
                callback(history[k], None, fit[k])
        return RunResult(evo.population(), fit[n_generations].copy(), history, cfg, g0 + n_generations)
    finally:
        evo.close()


def _refine(pop, dpop, data, metric, fit_d, larger, top=0.1, steps=5, lr=1e-2):
    """The elite's constants refined by gradient (see run_generations):
    (population with the kept constants, fitness after refinement)."""
    from .autograd import refine_constants
    fit = fit_d.cpu().numpy()
    n_const = np.diff(pop.const_off)
    key = np.where(np.isfinite(fit), fit, -np.inf if larger else np.inf)
    order = np.argsort(-key if larger else key, kind="stable")
    k = max(1, int(round(top * pop.n_programs)))
    elite = [int(p) for p in order[:k] if n_const[p] > 0]
    if not elite:
        return pop, fit_d
    new_c, _, f_after = refine_constants(dpop, data, metric, elite, steps=steps, lr=lr)
    consts = new_c.detach().cpu().numpy().astype(np.float32)
    return B.HostPopulation(pop.nodes, pop.prog_off, consts, pop.const_off, pop.length), f_after.contiguous()
