"""Benchmark of the Synchronised Louvain Method hot path on one MI355X.

One step = one full run of Algorithm 1 (every level: ASSIGN, COMPONENTS,
POSITIVE, MAXIMAL sweeps and resolutions, modularity, AGGREGATE) on the
R-MAT scale-20 graph (edge factor 16, a=0.57 b=0.19 c=0.19 d=0.05,
symmetrised, duplicates summed, self-loops dropped), resident in HBM before
the timed region.  The headline value is the throughput of the synchronous
move sweep measured live with HIP events on the library's stream: CSR
entries swept per second over every sweep of the timed steps (GTEPS).

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str):
    import graphgen as gg
    if name == "rmat20":
        return gg.config_graph("rmat20"), dict(
            workload="rmat20", kind="R-MAT", scale=20, edge_factor=16,
            abcd=[0.57, 0.19, 0.19, 0.05], seed=gg.CONFIG_SEEDS["rmat20"])
    if name == "sbm4096":
        return gg.config_graph("sbm4096"), dict(
            workload="sbm4096", kind="planted partition", nodes=4096, blocks=32,
            p_in=0.1, p_out=0.002, seed=gg.CONFIG_SEEDS["sbm4096"])
    if name == "lfr4m":
        return gg.config_graph("lfr4m"), dict(
            workload="lfr4m", kind="LFR-style", nodes=4_000_000, mean_degree=20,
            max_degree=2000, mixing=0.3, seed=gg.CONFIG_SEEDS["lfr4m"])
    raise SystemExit("unknown workload " + name)


def cpu_baseline(rp, col, w, budget_s: float):
    """The oracle's sweep (the plain sequential CPU implementation) on the
    same graph, with the labelling of its own ASSIGN, repeated for about
    budget_s seconds on one core."""
    import oracle
    g = oracle.Graph(rp, col, w)
    a = oracle.assign(g)
    lab, nc, _ = oracle.components(a)
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.sweep(g, lab, nc)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    entries = int(rp[-1]) * reps
    return dict(value=entries / el / 1e9, unit="GTEPS", cores=1, kind="oracle",
                sample="%d oracle sweeps of the full graph (labels from its ASSIGN), %.1f s"
                       % (reps, el))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="rmat20")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch
    import paper_1702_04645_amd as slm

    t = time.time()
    (rp, col, w), cfg = workload(args.workload)
    n, nnz = rp.size - 1, col.size
    log("workload %s: %d nodes, %d entries, generated in %.1fs" % (args.workload, n, nnz,
                                                                    time.time() - t))
    params = slm.params(seed=args.seed)
    g = slm.Graph(rp, col, w)
    info = g.level_info()
    for i in range(args.warmup):
        log("warmup %d" % i)
        g.run(params)
    torch.cuda.synchronize()
    g.timing(True)
    g.timing_read()  # clear
    log("timed steps: %d" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for i in range(args.steps):
        last = g.run(params)
        log("step %d done: %d levels" % (i, len(last)))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tm = g.timing_read()
    g.close()
    sweep_s = tm["sweep_ms"] / 1e3
    gteps = tm["entries"] / sweep_s / 1e9 if sweep_s > 0 else 0.0
    achieved = tm["bytes"] / sweep_s / 1e9 if sweep_s > 0 else 0.0
    out = {
        "metric": "GTEPS of sync move sweep",
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el * 1e3 / max(args.steps, 1), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": dict(cfg, nodes=n, entries=nnz, m2=info["m2"], seed_run=args.seed,
                       accept_p="1/2", max_rounds=64),
        "sweeps_timed": tm["sweeps"],
        "sweep_ms_mean": round(tm["sweep_ms"] / max(tm["sweeps"], 1), 4),
        "levels": len(last) if last else 0,
        "final_q": last[-1].q if last else None,
        "final_communities": last[-1].n_c if last else None,
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
        },
    }
    if rank == 0 and not args.no_cpu:
        log("cpu baseline (oracle sweep, about %.0f s)" % args.cpu_seconds)
        out["cpu_baseline"] = cpu_baseline(rp, col, w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
