"""Throughput of the GP hot path on one MI355X.

One step = one generation of the 16,777,216-row Pagie workload (4096
programs of 1-200 nodes), replayed from a captured HIP graph: the host
validates and stages the population in pinned memory, and the graph uploads
it in one copy, runs the instruction pre-pass, the fused MSE fitness (one
persistent launch of the evaluation kernel over every (row chunk, program)
work item, launch configuration from the autotuner), the tournaments, and
downloads fitness and winners.  The dataset is resident in HBM before
timing starts.

Prints one JSON line: GPops/s = sum(len) * rows / time per step; the
evaluation kernel's roofline (its duration from HIP event nodes recorded
around it inside the graph); the same rows with an add/sub/mul-only
population (every node one vector operation); the adjoint/forward time
ratio on the
differentiation workload (1,048,576 rows x 8 features, 2048 programs with
up to 16 constants); and the CPU oracle on a row sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VALU = 157.3e12     # MI355X dense FP32 vector, FLOP/s (packed FMA = 4 flops/lane/clk)
ISSUE_RATE = 39.3e12          # VALU lane-instruction slots per second: 256 CUs x 64 lanes x 2.4 GHz
# Op-mix ceiling: a fixed cost per node-row in VALU lane-instruction slots,
# fixed before it was compared with any measurement.  Terminals are free
# (folded into operand fetch); a packed two-row FP32 operation counts 0.5; a
# quarter-rate transcendental instruction (rcp, sqrt, log, exp, sin, cos)
# counts 4, plus 1 for its argument scaling or predicate; IEEE division and
# square root take their shortest correctly rounded sequences.  Opcodes:
# VAR CONST ADD SUB MUL DIV NEG LOG SQRT SIN COS TAN MAX MIN ATAN2 ABS EXP INV
# SQ CUBE TANH ATAN CBRT.
OP_COST = (0.0, 0.0, 0.5, 0.5, 0.5, 10.0, 0.5, 5.0, 8.0, 5.0, 5.0, 14.0, 1.0, 1.0, 20.0, 0.5, 5.0, 10.0,
           0.5, 1.0, 10.0, 12.0, 10.0)
# The same table measured on this kernel (`--op-costs` under rocprofv3
# SQ_INSTS_VALU): VALU lane-instructions per row for each function itself,
# without dispatch.  A unary function's cost is its chain population's VALU
# per node-row less the negation chain's plus 1 (one instruction for neg); a
# binary function's is twice its fold population's excess over add's plus 1
# (a fold instruction covers two nodes).  add, sub and mul are one
# instruction per row (no packed FP32); sin, cos and log carry the double
# evaluation of their correctly rounded form.
OP_COST_MEASURED = (0.0, 0.0, 1.0, 1.0, 1.0, 12.9, 1.0, 27.0, 10.9, 23.0, 21.0, 28.7, 6.0, 6.0, 38.6, 1.4,
                    13.3, 13.3, 1.4, 2.4, 10.0, 16.3, 15.3)
# what the evaluation kernel is built from: its source, the headers it
# includes and the build flags
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2110_11226_amd", *f) for f in
                  (("csrc", "gp_device.hip"), ("csrc", "gp_crmath.h"), ("csrc", "gp_crmath_tables.h"),
                   ("csrc", "gp_internal.h"), ("build.py",))] + [os.path.join(ROOT, "include", "gp.h")]
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_eval_pagie-16M_traffic.md")

WORKLOADS = {
    "pagie-16M": dict(rows=16_777_216, programs=4096, features=2, metric="mse", data_seed=11229,
                      pop=dict(method="exact_len", min_len=1, max_len=200, seed=2113)),
    "pagie-4K": dict(rows=4096, programs=256, features=2, metric="mse", data_seed=11227,
                     pop=dict(method="rhh", min_depth=2, max_depth=6, seed=2111)),
    "higgs-11M": dict(rows=11_000_000, programs=2000, features=28, metric="logloss", data_seed=11230,
                      pop=dict(method="exact_len", min_len=1, max_len=200, seed=2114)),
}
DIFF = dict(rows=1_048_576, programs=2048, features=8, data_seed=11231,
            pop=dict(method="exact_len", min_len=1, max_len=200, max_consts=16, seed=2115))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_data(wl):
    import synth
    if wl["features"] == 28:
        return synth.higgs_like(wl["rows"], seed=wl["data_seed"])
    return synth.pagie(wl["rows"], seed=wl["data_seed"])


def source_sha():
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def committed_traffic():
    """HBM bytes per launch of the evaluation kernel from the committed PMC
    summary, if it was taken from the kernel source as it is now."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    text = open(TRAFFIC_SUMMARY).read()
    sha = re.search(r"kernel source sha256:\s*([0-9a-f]{64})", text)
    val = re.search(r"traffic bytes per launch:\s*([0-9.eE+]+)", text)
    if not sha or not val or sha.group(1) != source_sha():
        return None
    return float(val.group(1))


def host_threads():
    """(threads the oracle runs on, the host's core count as nproc reports
    it): every core this process may use, unless OMP_NUM_THREADS caps it."""
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cap = os.environ.get("OMP_NUM_THREADS")
    threads = min(nproc, int(cap)) if cap and cap.isdigit() and int(cap) > 0 else nproc
    return threads, nproc


def cpu_baseline(host, X, y, metric, budget_rows, single_rows=2048):
    """The oracle as it stands, timed on this host's cores over every program
    and an evenly spaced row subsample; and on one core over a smaller one."""
    import oracle
    N = X.shape[1]
    opop = oracle.Population(host.nodes, host.prog_off, host.consts, host.const_off, host.length)
    sum_len = float(host.length.astype(np.int64).sum())
    threads, nproc = host_threads()

    def timed(rows, n_threads):
        stride = max(1, N // rows)
        idx = np.arange(0, N, stride)[:rows]
        Xs, ys = np.ascontiguousarray(X[:, idx]), np.ascontiguousarray(y[idx])
        t0 = time.perf_counter()
        oracle.fitness(opop, Xs, ys, None, metric, n_threads=n_threads, with_f64=False)
        dt = time.perf_counter() - t0
        return sum_len * len(idx) / dt, len(idx), stride, dt

    gops, n, stride, dt = timed(budget_rows, threads)
    g1, n1, s1, dt1 = timed(single_rows, 1)
    return {"value": gops, "unit": "GPops/s", "cores": threads, "nproc": nproc, "kind": "oracle",
            "sample": f"all {host.n_programs} programs x {n} rows (every {stride}th row), float32 path, "
                      f"{dt:.1f} s on {threads} threads (nproc {nproc})",
            "single_core": {"value": g1, "unit": "GPops/s", "cores": 1,
                            "sample": f"all {host.n_programs} programs x {n1} rows (every {s1}th row), "
                                      f"{dt1:.1f} s"}}


def parity_sample(gp, torch, host, X, y, metric, rows=4096):
    """The step's population on an evenly spaced row sample of its dataset:
    every program's outputs against the oracle's float32 evaluation (bit for
    bit), and every program's fitness on those rows against the oracle's
    float32-path and float64 fitness."""
    import oracle
    N = X.shape[1]
    idx = np.linspace(0, N - 1, rows).astype(np.int64)
    Xs, ys = np.ascontiguousarray(X[:, idx]), np.ascontiguousarray(y[idx])
    pop = gp.DevicePopulation(host, n_features=X.shape[0])
    data = gp.DeviceDataset(Xs, ys)
    out = gp.evaluate(pop, data)
    fit = gp.fitness(pop, data, metric)
    torch.cuda.synchronize()
    got, gfit = out.cpu().numpy(), fit.cpu().numpy().astype(np.float64)
    threads, _ = host_threads()
    opop = oracle.Population(host.nodes, host.prog_off, host.consts, host.const_off, host.length)
    ref = oracle.evaluate_f32(opop, Xs, n_threads=threads)
    same = (got.view(np.uint32) == ref.view(np.uint32)) | (np.isnan(got) & np.isnan(ref))
    f32p, f64 = oracle.fitness(opop, Xs, ys, None, metric, n_threads=threads)
    ref32 = f32p.astype(np.float32).astype(np.float64)
    fin = np.isfinite(ref32)
    with np.errstate(invalid="ignore", divide="ignore"):
        e32 = np.abs(gfit - ref32) / np.abs(ref32)
        e64 = np.abs(gfit - f64) / np.abs(f64)
    m32, m64 = fin & np.isfinite(e32), fin & np.isfinite(e64)
    return {"rows": int(rows), "programs": int(host.n_programs), "outputs_checked": int(got.size),
            "outputs_bit_exact": int(same.sum()), "outputs_excluded": 0,
            "fitness_checked": int(fin.sum()), "fitness_excluded": 0,
            "fitness_nonfinite_class_match": bool(np.array_equal(np.isfinite(gfit), fin)),
            "max_rel_err_vs_oracle_f32": float(e32[m32].max()) if m32.any() else 0.0,
            "max_rel_err_vs_f64": float(e64[m64].max()) if m64.any() else 0.0,
            "median_rel_err_vs_f64": float(np.median(e64[m64])) if m64.any() else 0.0,
            "programs_within_1e-4_of_f64": int((e64[m64] <= 1e-4).sum()),
            "tolerance": "outputs bit-exact; fitness 1e-4 relative"}


def op_mix(host, gops):
    """The population's op-mix ceiling (ISSUE_RATE / mean cost per node-row)
    and the fraction of it that `gops` reaches, from the measured cost table
    (OP_COST_MEASURED); the frozen table's figures (OP_COST) beside them."""
    ops = np.asarray(host.nodes, np.uint32) & 0xFF
    hist = np.bincount(ops, minlength=len(OP_COST))

    def ceil(table):
        per = float((hist[:len(table)] * np.asarray(table)).sum() / hist.sum())
        return per, ISSUE_RATE / per

    per, ceiling = ceil(OP_COST_MEASURED)
    per0, ceiling0 = ceil(OP_COST)
    return {"lane_slots_per_node_row": per, "ceiling": ceiling, "unit": "GPops/s", "frac": gops / ceiling,
            "table": "measured (VALU per row of each function, no dispatch)",
            "frozen": {"lane_slots_per_node_row": per0, "ceiling": ceiling0, "frac": gops / ceiling0}}


CONFIGS = [
    dict(name="C1 pagie-4K", rows=4096, programs=256, features=2, metric="mse", data="pagie", data_seed=11227,
         pop=dict(method="rhh", min_depth=2, max_depth=6, seed=2111), runs=20),
    dict(name="C2 pagie-1M", rows=1_048_576, programs=1000, features=2, metric="mse", data="pagie",
         data_seed=11228, pop=dict(method="rhh", min_depth=2, max_depth=8, seed=2112), runs=20),
    dict(name="C3 pagie-16M", rows=16_777_216, programs=4096, features=2, metric="mse", data="pagie",
         data_seed=11229, pop=dict(method="exact_len", min_len=1, max_len=200, seed=2113), runs=5),
    dict(name="C4 higgs-11M", rows=11_000_000, programs=2000, features=28, metric="logloss", data="higgs",
         data_seed=11230, pop=dict(method="exact_len", min_len=1, max_len=200, seed=2114), runs=5),
    dict(name="C5 diff-1M", rows=1_048_576, programs=2048, features=8, metric="mse", data="diff",
         data_seed=11231, pop=dict(method="exact_len", min_len=1, max_len=200, max_consts=16, seed=2115),
         runs=20),
]


def config_table(gp, torch, oracle_rows=16_384):
    """gp_fitness throughput on each workload configuration: autotuned, 3
    warm-up calls, then the median of `runs` event-timed calls; the literal
    and op-mix fractions; the oracle on every program over an evenly spaced
    row sample (all rows when there are fewer)."""
    import synth
    out = []
    for c in CONFIGS:
        gen = {"pagie": synth.pagie, "higgs": synth.higgs_like, "diff": synth.diff_target}[c["data"]]
        X, y = gen(c["rows"], seed=c["data_seed"])
        host = gp.build_population(c["programs"], c["features"], **c["pop"])
        sum_len = int(host.length.astype(np.int64).sum())
        pop = gp.DevicePopulation(host, n_features=c["features"])
        data = gp.DeviceDataset(X, y)
        fit = torch.empty(host.n_programs, dtype=torch.float32, device="cuda")
        cfg, _ = gp.autotune(pop, data, c["metric"], repeats=2)
        s = torch.cuda.current_stream()
        ms = []
        for i in range(3 + c["runs"]):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            gp.fitness(pop, data, c["metric"], out=fit)
            b.record(s)
            b.synchronize()
            if i >= 3:
                ms.append(a.elapsed_time(b))
        t = float(np.median(ms))
        gops = sum_len * c["rows"] / (t / 1e3)
        row = {"config": c["name"], "rows": c["rows"], "programs": c["programs"], "features": c["features"],
               "metric": c["metric"], "population": c["pop"], "sum_len": sum_len, "launch": list(cfg),
               "fitness_ms_median": t, "runs": c["runs"], "gpops": gops, "frac_157T": gops / PEAK_FP32_VALU,
               "op_mix": op_mix(host, gops)}
        if c["data"] == "diff":
            row["adjoint"] = adjoint_ratio(gp, torch)
        log(f"[bench] {c['name']}: {t:.3f} ms, {gops:.3g} GPops/s ({100 * gops / PEAK_FP32_VALU:.2f}% of 157.3 T, "
            f"{100 * row['op_mix']['frac']:.1f}% of the op-mix ceiling)")
        row["oracle"] = cpu_baseline(host, X, y, c["metric"], min(oracle_rows, c["rows"]),
                                     single_rows=min(1024, c["rows"]))
        log(f"[bench] {c['name']} oracle: {row['oracle']['value']:.3g} GPops/s on {row['oracle']['cores']} threads")
        row["parity"] = parity_sample(gp, torch, host, X, y, c["metric"], rows=min(4096, c["rows"]))
        log(f"[bench] {c['name']} parity: {row['parity']['outputs_bit_exact']} of "
            f"{row['parity']['outputs_checked']} outputs bit-exact, max fitness rel err vs f64 "
            f"{row['parity']['max_rel_err_vs_f64']:.2e}")
        out.append(row)
        del pop, data, fit, X, y
    return out


def arith_only(gp, data, wl, steps):
    """The same rows with a population over add, sub and mul only (lengths
    1-200, same seed): the function set where every node is one vector
    operation, timed like the main step."""
    mask = sum(1 << op for op in (2, 3, 4))
    host = gp.build_population(wl["programs"], wl["features"], function_mask=mask, **wl["pop"])
    sum_len = int(host.length.astype(np.int64).sum())
    gen = gp.Generation(data, host.n_programs, host.nodes.shape[0], max(host.consts.shape[0], 1), wl["metric"],
                        tournament_size=20, seed=2025, autotune=True, time_kernel=True)
    try:
        gen.run(host, 0)
        ms = []
        for i in range(steps):
            gen.run(host, 1 + i)
            ms.append(gen.timing()["kernel_ms"])
        launch = gen.timing()["launch"]
    finally:
        gen.close()
    k = float(np.mean(ms))
    gops = sum_len * wl["rows"] / (k / 1e3)
    return {"population": "exact_len 1-200 over {add, sub, mul}, seed 2113", "sum_len": sum_len,
            "kernel_avg_ms": k, "value": gops, "unit": "GPops/s", "frac": gops / PEAK_FP32_VALU,
            "op_mix": op_mix(host, gops), "launch": list(launch)}


OPCOST_UNARY = ("neg", "log", "sqrt", "sin", "cos", "tan", "exp", "tanh", "atan", "cbrt", "abs", "inv", "sq", "cube")
OPCOST_BINARY = ("add", "sub", "mul", "div", "max", "min", "atan2")
OPCODE = {"add": 2, "sub": 3, "mul": 4, "div": 5, "neg": 6, "log": 7, "sqrt": 8, "sin": 9, "cos": 10, "tan": 11,
          "max": 12, "min": 13, "atan2": 14, "abs": 15, "exp": 16, "inv": 17, "sq": 18, "cube": 19, "tanh": 20,
          "atan": 21, "cbrt": 22}


def op_cost_populations():
    """Single-function populations for the per-function cost breakdown:
    'unary_f': x0 under a chain of 100 f (8 chained per instruction);
    'fold_f': f(x0, f(x1, f(x0, ... x1))), every terminal fused with its
    binary function (one instruction per two nodes); 'bin_f': f(f(x0, x1),
    f(f(x0, x1), ...)), the outer f of each level reading its second
    operand from the stack.  256 copies of one program each."""
    V0, V1 = 0, 1 << 8   # GP_NODE(VAR, 0), GP_NODE(VAR, 1)
    out = []
    for f in OPCOST_UNARY:
        out.append(("unary_" + f, [OPCODE[f]] * 100 + [V0]))
    for f in OPCOST_BINARY:
        fold = []
        for i in range(50):
            fold += [OPCODE[f], V0 if i % 2 == 0 else V1]
        out.append(("fold_" + f, fold + [V1]))
        out.append(("bin_" + f, [OPCODE[f], OPCODE[f], V0, V1] * 25 + [V0]))
    return out


def op_costs(gp, torch, rows=1 << 20):
    """One MSE fitness dispatch per single-function population on Pagie
    rows (launch configuration 4 rows per lane, 2 feature registers, 16
    tiles, 4 waves), in the order of op_cost_populations: the kernel time
    and node-rows of each (run under rocprofv3 --pmc to read the
    instruction counters of each dispatch)."""
    import synth
    X, y = synth.pagie(rows, seed=11229)
    data = gp.DeviceDataset(X, y)
    gp.set_launch_config((4, 2, 16, 4))
    gp.profile_enable(True)
    res = []
    try:
        for name, prog in op_cost_populations():
            L, P = len(prog), 256
            nodes = np.tile(np.asarray(prog, np.uint32), P)
            host = gp.HostPopulation(nodes, np.arange(P + 1, dtype=np.int64) * L, np.zeros(1, np.float32),
                                     np.zeros(P + 1, np.int64), np.full(P, L, np.int32))
            pop = gp.DevicePopulation(host, n_features=2)
            _, ms0, _ = gp.profile_read()
            gp.fitness(pop, data, "mse")
            torch.cuda.synchronize()
            _, ms1, _ = gp.profile_read()
            res.append({"case": name, "nodes": L, "kernel_ms": ms1 - ms0, "node_rows": P * L * rows})
            log(f"[bench] {name}: {ms1 - ms0:.3f} ms")
    finally:
        gp.set_launch_config(None)
        gp.profile_enable(False)
    return res


def loop_generation_time(gp, torch, n_gen=10):
    """Wall time per generation of the whole loop (fitness, tournaments,
    pre-draw, genetic operations) with the genetic operations on the host
    (captured generation graph + gp_mutate) and on the device (gp_evolution),
    on 65,536 Pagie rows x 4,096 ramped half-and-half programs: a small-N
    shape where the mutation step is visible next to the fitness."""
    import synth
    X, y = synth.pagie(65_536, seed=11229)
    data = gp.DeviceDataset(X, y)
    init = dict(n_features=2, method="rhh", min_depth=2, max_depth=6, seed=2111)
    ev = dict(p_crossover=0.7, p_subtree=0.1, p_hoist=0.05, p_point=0.1, p_point_replace=0.05, max_len=256)
    out = {"workload": "pagie, 65536 rows x 4096 programs (RHH depth 2-6), MSE", "generations": n_gen}
    for key, kw in (("host_mutation_ms_per_generation", {}), ("device_loop_ms_per_generation",
                                                           {"device_loop": True})):
        gp.run_generations(data, 1, 4096, init, "mse", 20, 0.01, ev, seed=3, **kw)     # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gp.run_generations(data, n_gen, 4096, init, "mse", 20, 0.01, ev, seed=3, **kw)
        torch.cuda.synchronize()
        out[key] = (time.perf_counter() - t0) * 1e3 / n_gen
    return out


def spearman_time(gp, torch, reps=3):
    """Spearman fitness (evaluate, segmented radix sort of every program's
    outputs, ranks, rank correlation) on 1,048,576 Pagie rows x 4,096
    exact-length programs: event-timed median of `reps` calls, with the MSE
    fitness of the same population beside it."""
    import synth
    X, y = synth.pagie(1_048_576, seed=11232)
    host = gp.build_population(4096, 2, "exact_len", min_len=1, max_len=200, seed=2113)
    pop = gp.DevicePopulation(host, n_features=2)
    data = gp.DeviceDataset(X, y)
    fit = torch.empty(4096, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream()

    def timed(metric):
        out = []
        for _ in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            gp.fitness(pop, data, metric, out=fit)
            b.record(s)
            b.synchronize()
            out.append(a.elapsed_time(b))
        return float(np.median(out[1:]))

    ms_sp, ms_mse = timed("spearman"), timed("mse")
    node_rows = float(host.length.astype(np.int64).sum()) * 1_048_576
    return {"workload": "pagie, 1048576 rows x 4096 programs (exact length 1-200)", "spearman_ms": ms_sp,
            "mse_ms": ms_mse, "spearman_gpops": node_rows / (ms_sp / 1e3),
            "sorted_keys_per_s": 4096 * 1_048_576 / (ms_sp / 1e3)}


def adjoint_ratio(gp, torch, reps=5):
    """gp_fitness_backward time / gp_fitness time on the differentiation
    workload (medians of `reps` event-timed calls each), the forward under
    the autotuner's launch configuration for this shape."""
    import synth
    X, y = synth.diff_target(DIFF["rows"], seed=DIFF["data_seed"])
    host = gp.build_population(DIFF["programs"], DIFF["features"], **DIFF["pop"])
    pop = gp.DevicePopulation(host, n_features=DIFF["features"])
    data = gp.DeviceDataset(X, y)
    fit = torch.empty(host.n_programs, dtype=torch.float32, device="cuda")
    grad = torch.empty(max(pop.n_consts, 1), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(fn):
        out = []
        for _ in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            out.append(a.elapsed_time(b))
        return float(np.median(out[1:]))

    cfg, _ = gp.autotune(pop, data, "mse", repeats=2)
    fwd = timed(lambda: gp.fitness(pop, data, "mse", out=fit))
    bwd = timed(lambda: gp.fitness_backward(pop, data, "mse", grad_out=grad))
    return {"workload": f"diff-1M: {DIFF['rows']} rows x {DIFF['features']} features, {DIFF['programs']} "
                        f"programs of 1-200 nodes with <= 16 constants, MSE",
            "forward_ms": fwd, "forward_launch": list(cfg), "backward_ms": bwd, "ratio": bwd / fwd,
            "target": 3.0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="pagie-16M", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true", help="skip the oracle parity sample")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-arith", action="store_true", help="skip the add/sub/mul-only population")
    ap.add_argument("--no-loop", action="store_true", help="skip the generation-loop timing")
    ap.add_argument("--no-spearman", action="store_true", help="skip the Spearman fitness timing")
    ap.add_argument("--only-spearman", action="store_true",
                    help="time only the Spearman fitness (for a kernel trace of it)")
    ap.add_argument("--only-loop", action="store_true",
                    help="only the generation-loop timing (host vs device genetic operations; for profiling)")
    ap.add_argument("--only-adjoint", action="store_true",
                    help="only the adjoint / forward ratio on the differentiation workload (for profiling)")
    ap.add_argument("--op-costs", action="store_true",
                    help="only the single-function populations of the per-function cost breakdown")
    ap.add_argument("--configs", action="store_true",
                    help="instead of the step, measure gp_fitness on every workload configuration")
    ap.add_argument("--cpu-rows", type=int, default=32_768)
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache (JSON lines): loaded if present, written after tuning")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard by programs or rows; one GPU's share is what runs here)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2110_11226_amd as gp

    wl = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.copy_calibration_mib} MiB done")
        del src, dst
    if args.configs:
        print(json.dumps({"configs": config_table(gp, torch)}), flush=True)
        return 0
    if args.op_costs:
        print(json.dumps({"op_costs": op_costs(gp, torch)}), flush=True)
        return 0
    if args.only_loop:
        loop = loop_generation_time(gp, torch)
        log(f"[bench] loop ms/generation: host mutation {loop['host_mutation_ms_per_generation']:.2f}, "
            f"device loop {loop['device_loop_ms_per_generation']:.2f}")
        print(json.dumps({"generation_loop": loop}), flush=True)
        return 0
    if args.only_adjoint:
        adj = adjoint_ratio(gp, torch)
        log(f"[bench] forward {adj['forward_ms']:.2f} ms, backward {adj['backward_ms']:.2f} ms, "
            f"ratio {adj['ratio']:.2f}")
        print(json.dumps({"adjoint": adj}), flush=True)
        return 0
    if args.only_spearman:
        spear = spearman_time(gp, torch)
        log(f"[bench] Spearman {spear['spearman_ms']:.1f} ms vs MSE {spear['mse_ms']:.1f} ms")
        print(json.dumps({"spearman": spear}))
        return 0
    log(f"[bench] building {args.workload}: {wl['rows']} rows x {wl['programs']} programs")
    X, y = make_data(wl)
    host = gp.build_population(wl["programs"], wl["features"], **wl["pop"])
    sum_len = int(host.length.astype(np.int64).sum())
    data = gp.DeviceDataset(X, y)
    metric = wl["metric"]
    T = host.n_programs
    loaded = bool(args.tune_cache and os.path.exists(args.tune_cache))
    if loaded:
        gp.autotune_load(args.tune_cache)
        log(f"[bench] autotuner cache loaded from {args.tune_cache}")
    gen = gp.Generation(data, host.n_programs, host.nodes.shape[0], max(host.consts.shape[0], 1), metric,
                        parsimony=0.0, tournament_size=20, n_tournaments=T, seed=2025,
                        autotune=not args.no_autotune and not loaded,
                        time_kernel=True)
    try:
        for i in range(args.warmup):
            gen.run(host, i)
            log(f"[bench] warmup {i + 1}/{args.warmup} done (graph captured; launch {gen.timing()['launch']})")
        kernel_ms = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            gen.run(host, args.warmup + i)
            kernel_ms.append(gen.timing()["kernel_ms"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tm = gen.timing()
        if args.tune_cache and tm["tuned_ms"] > 0:
            gp.autotune_save(args.tune_cache)
    finally:
        gen.close()
    ms_step = wall * 1e3 / args.steps
    gops = sum_len * wl["rows"] / (ms_step / 1e3)
    kern_avg_ms = float(np.mean(kernel_ms))
    ops_launch = float(sum_len) * wl["rows"]
    achieved = ops_launch / (kern_avg_ms / 1e3)
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step, evaluation kernel {kern_avg_ms:.3f} ms avg "
        f"({tm['timed_by']}; device clock {tm['clock_ms']:.3f} ms)")

    arith = None
    if not args.no_arith and args.workload == "pagie-16M":
        log("[bench] add/sub/mul-only population on the same rows")
        arith = arith_only(gp, data, wl, 3)
        log(f"[bench] add/sub/mul only: {arith['kernel_avg_ms']:.1f} ms, {arith['value']:.3g} GPops/s "
            f"({100 * arith['frac']:.2f}% of peak)")

    spear = None
    if not args.no_spearman and args.workload == "pagie-16M":
        log("[bench] Spearman fitness")
        spear = spearman_time(gp, torch)
        log(f"[bench] Spearman {spear['spearman_ms']:.1f} ms vs MSE {spear['mse_ms']:.1f} ms on "
            f"1M rows x 4096 programs ({spear['sorted_keys_per_s']:.3g} ranked outputs/s)")

    loop = None
    if not args.no_loop and args.workload == "pagie-16M":
        log("[bench] generation loop: host vs device genetic operations")
        loop = loop_generation_time(gp, torch)
        log(f"[bench] loop ms/generation: host mutation {loop['host_mutation_ms_per_generation']:.2f}, "
            f"device loop {loop['device_loop_ms_per_generation']:.2f}")

    adj = None
    if not args.no_adjoint:
        log("[bench] adjoint / forward ratio on the differentiation workload")
        adj = adjoint_ratio(gp, torch)
        log(f"[bench] forward {adj['forward_ms']:.2f} ms, backward {adj['backward_ms']:.2f} ms, "
            f"ratio {adj['ratio']:.2f}")

    base = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a row subsample")
        base = cpu_baseline(host, X, y, metric, args.cpu_rows)
        log(f"[bench] oracle {base['value']:.3g} GPops/s on {base['cores']} threads, "
            f"{base['single_core']['value']:.3g} on one")

    par = None
    if not args.no_parity:
        log("[bench] parity on a row sample")
        par = parity_sample(gp, torch, host, X, y, metric)
        log(f"[bench] parity: {par['outputs_bit_exact']} of {par['outputs_checked']} outputs bit-exact, "
            f"max fitness rel err {par['max_rel_err_vs_oracle_f32']:.2e} (oracle f32), "
            f"{par['max_rel_err_vs_f64']:.2e} (f64)")

    traffic = committed_traffic() if args.workload == "pagie-16M" else None
    line = {
        "metric": "GPops/s (program-node evals/sec) for population fitness",
        "value": gops,
        "unit": "GPops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_rows": wl["rows"], "n_programs": wl["programs"],
                   "n_features": wl["features"], "population": wl["pop"], "sum_len": sum_len,
                   "metric": metric, "tournament_size": 20, "n_tournaments": T,
                   "step": "validate+stage (host), one HIP graph: population upload, instruction pre-pass, "
                           "fused fitness, tournaments, result download",
                   "launch": {"rows_per_lane": tm["launch"][0], "feature_regs": tm["launch"][1],
                              "tiles_per_chunk": tm["launch"][2], "waves_per_block": tm["launch"][3],
                              "source": ("autotuner" if tm["tuned_ms"] > 0 else
                                         "autotuner cache" if loaded else "heuristic"),
                              "tuned_ms_row_prefix": tm["tuned_ms"]}},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU,
                     "traffic": traffic,
                     "kernel": "k_eval (persistent fused evaluation + MSE row loss + wave reduction)",
                     "kernel_avg_ms": kern_avg_ms, "kernel_timed_by": tm["timed_by"],
                     "ops_per_launch": ops_launch, "op": "one program node evaluated on one row",
                     "kernel_source_sha256": source_sha()},
        "op_mix": op_mix(host, achieved),
        "arith_only": arith,
        "generation_loop": loop,
        "spearman": spear,
        "adjoint": adj,
        "cpu_baseline": base,
        "parity": par,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
