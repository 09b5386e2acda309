"""Throughput of the GP hot path on one MI355X.

One step = one generation's pass over the hot path on the 16,777,216-row
Pagie workload: upload the population (one async copy per array from pinned
host memory), evaluate every program on every row with the fused MSE fitness
(gp_fitness), and run the tournament selection (gp_tournament).  The dataset
is resident in HBM before timing starts.

Prints one JSON line (metric GPops/s = sum(len) * rows / time per step).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VALU = 157.3e12     # MI355X dense FP32 vector, FLOP/s (packed FMA = 4 flops/lane/clk)

WORKLOADS = {
    # name: (rows, programs, init kwargs, metric, features)
    "pagie-16M": dict(rows=16_777_216, programs=4096, features=2, metric="mse", data_seed=11229,
                      pop=dict(method="exact_len", min_len=1, max_len=200, seed=2113)),
    "pagie-4K": dict(rows=4096, programs=256, features=2, metric="mse", data_seed=11227,
                     pop=dict(method="rhh", min_depth=2, max_depth=6, seed=2111)),
    "higgs-11M": dict(rows=11_000_000, programs=2000, features=28, metric="logloss", data_seed=11230,
                      pop=dict(method="exact_len", min_len=1, max_len=200, seed=2114)),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_data(wl):
    import synth
    if wl["features"] == 28:
        return synth.higgs_like(wl["rows"], seed=wl["data_seed"])
    return synth.pagie(wl["rows"], seed=wl["data_seed"])


def cpu_baseline(host, X, y, metric, budget_rows):
    """The oracle as it stands, timed on this host's cores over every program
    and an evenly spaced row subsample."""
    import oracle
    N = X.shape[1]
    stride = max(1, N // budget_rows)
    idx = np.arange(0, N, stride)[:budget_rows]
    Xs = np.ascontiguousarray(X[:, idx])
    ys = np.ascontiguousarray(y[idx])
    opop = oracle.Population(host.nodes, host.prog_off, host.consts, host.const_off, host.length)
    cores = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    oracle.fitness(opop, Xs, ys, None, metric, n_threads=cores, with_f64=False)
    dt = time.perf_counter() - t0
    gops = float(host.length.astype(np.int64).sum()) * len(idx) / dt
    return {"value": gops, "unit": "GPops/s", "cores": cores, "kind": "oracle",
            "sample": f"all {host.n_programs} programs x {len(idx)} rows (every {stride}th row), "
                      f"float32 path, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="pagie-16M", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=65536)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by programs or rows, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2110_11226_amd as gp

    wl = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    log(f"[bench] building {args.workload}: {wl['rows']} rows x {wl['programs']} programs")
    X, y = make_data(wl)
    host = gp.build_population(wl["programs"], wl["features"], **wl["pop"])
    gp.validate_population(host, wl["features"])
    sum_len = int(host.length.astype(np.int64).sum())
    data = gp.DeviceDataset(X, y)
    pop = gp.DevicePopulation(host, n_features=wl["features"], validate=False)
    # pinned staging copies of the population: the per-generation upload
    pinned = {k: torch.from_numpy(np.ascontiguousarray(v)).pin_memory()
              for k, v in (("nodes", host.nodes.view(np.int32)), ("prog_off", host.prog_off),
                           ("consts", host.consts if host.consts.size else np.zeros(1, np.float32)),
                           ("const_off", host.const_off), ("length", host.length))}
    dev = {"nodes": pop.nodes, "prog_off": pop.prog_off, "consts": pop.consts,
           "const_off": pop.const_off, "length": pop.length}
    fit = torch.empty(host.n_programs, dtype=torch.float32, device="cuda")
    T = host.n_programs
    win = torch.empty(T, dtype=torch.int32, device="cuda")
    metric = wl["metric"]
    stream = torch.cuda.current_stream()

    def step(g):
        for k in dev:
            dev[k].copy_(pinned[k], non_blocking=True)
        gp.fitness(pop, data, metric, out=fit)
        gp.tournament(fit, pop.length, metric, 0.0, 20, T, seed=2025, generation=g, out=win)

    for i in range(args.warmup):
        step(i)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")

    gp.profile_enable(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        step(args.warmup + i)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, kern_ms, node_rows = gp.profile_read()
    gp.profile_enable(False)
    ms_step = ev0.elapsed_time(ev1) / args.steps
    gops = sum_len * wl["rows"] / (ms_step / 1e3)
    kern_avg_ms = kern_ms / max(launches, 1)
    achieved = (node_rows / max(launches, 1)) / (kern_avg_ms / 1e3)
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step (wall {wall:.2f} s), eval kernel "
        f"{kern_avg_ms:.3f} ms avg over {launches} launches")

    base = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a row subsample")
        base = cpu_baseline(host, X, y, metric, args.cpu_rows)

    cfg = gp.get_launch_config(wl["features"], wl["rows"], wl["programs"])
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
                   "metric": metric, "tournament_size": 20,
                   "step": "H2D population + fused fitness + tournament",
                   "launch": {"rows_per_lane": cfg[0], "feature_regs": cfg[1], "tiles_per_chunk": cfg[2]}},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU, "traffic": None,
                     "kernel": "k_eval (fused evaluation + MSE row loss + wave reduction)",
                     "kernel_avg_ms": kern_avg_ms, "ops_per_launch": node_rows / max(launches, 1),
                     "op": "one program node evaluated on one row"},
        "cpu_baseline": base,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
