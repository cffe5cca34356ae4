"""Benchmark of the Synchronised Louvain Method hot path on one MI355X.

One step = one full run of Algorithm 1 (every level: ASSIGN, COMPONENTS,
POSITIVE, MAXIMAL sweeps and resolutions, modularity, AGGREGATE) on the
LFR-style graph of 4,000,000 nodes (power-law degrees, exponent 2.5, mean
20, max 2000; power-law community sizes, exponent 1.5, 20-5000; mixing 0.3;
weights uniform 1-16), resident in HBM before the timed region.  The
headline value is the throughput of the synchronous move sweep measured
live with HIP events on the library's stream: CSR entries swept per second
over every sweep of the timed steps (GTEPS).  After the timed steps the same
line reports, each measured outside the timed region:
  - null_models: the same graph under the resolution (gamma = 1/2) and
    Erdos-Renyi (p = 1/4000) null models of Sec. 2.2-2.3;
  - louvain: the classical sequential Louvain method (exact sequential
    result) against the Synchronised Louvain Method on the same graph;
  - directed: a directed weighted LFR-shaped graph of the paper's experiments
    (Table 1: 10^6 nodes, mean degree 50, max 100, mixing 0.5 / 0.4) under
    the directed modularity of Sec. 2.4, with the oracle's sweep beside it;
  - batch: the 2048-graph planted-partition family batched against the plain
    per-graph path (graphs/s);
  - serve: a served Poisson mix with R-MAT scale-20 requests (p50/p99).

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
[--workload lfr4m|rmat20|sbm4096|batch2048|serve] [--no-extras]
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


def sweep_source_hash():
    """First 16 hex digits of the sha256 of the sweep's sources (kernels and
    the constants they share with the host)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("k_sweep.hip", "slm_impl.h"):
        with open(os.path.join(ROOT, "paper_1702_04645_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per sweep from the committed rocprofv3 counter summary, when
    it was taken on this workload with the current sweep sources; else None."""
    path = os.path.join(ROOT, "profiles", "%s_sweep_hbm_traffic.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("sweep_source_sha256_16") != sweep_source_hash():
        return None
    return round(rec["sweep_traffic_bytes"] / 1e9, 4)


def tuned_options(row_ptr, arch=None):
    """(options, file) that the autotuner kept for this GPU architecture and
    this graph's degree profile, or (None, None): then the library defaults
    stand.  arch: the current GPU's when not given.  A cache that cannot be
    read never stops the bench."""
    from paper_1702_04645_amd import autotune
    try:
        if arch is None:
            arch = autotune.device_arch()
        return autotune.find(row_ptr, arch)
    except Exception as e:  # noqa: BLE001
        log("tuned launch options not read (%s): library defaults" % e)
        return None, None


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


def singleton_sweep(g, nnz: int, n: int, reps: int = 10):
    """The sweep with every node in a community of its own (labels 0..n-1,
    the most distinct communities per row), timed like first_sweep."""
    import torch
    lab = torch.arange(n, dtype=torch.int32, device="cuda")
    g.sweep(lab, n)
    torch.cuda.synchronize()
    g.timing(True)
    g.timing_read()
    for _ in range(reps):
        g.sweep(lab, n)
    tm = g.timing_read()
    g.timing(False)
    ms = tm["sweep_ms"] / max(tm["sweeps"], 1)
    gbs = tm["bytes"] / max(tm["sweeps"], 1) / (ms * 1e-3) / 1e9
    return {"ms": round(ms, 4), "gteps": round(nnz / (ms * 1e-3) / 1e9, 3),
            "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "repetitions": reps}


def copy_gbs(reps: int = 10) -> float:
    """Bandwidth of a plain device-to-device copy of 1 GiB (bytes read plus
    bytes written per second): what a streaming kernel reaches on this GPU."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3
    out = 2.0 * a.numel() * 4 * reps / s / 1e9
    del a, b
    torch.cuda.empty_cache()
    return round(out, 1)


def first_sweep(g, nnz: int, n: int, reps: int = 20):
    """The sweep on the labels of the level's first MAXIMAL round (ASSIGN,
    POSITIVE, COMPONENTS), timed like the run's sweeps (HIP events on the
    library's stream) over `reps` repetitions, outside the timed step; the
    handle is reset afterwards."""
    import torch
    a = g.assign()
    a, _ = g.positive(a)
    lab, nc, _ = g.components(a)
    g.sweep(lab, nc)
    torch.cuda.synchronize()
    g.timing(True)
    g.timing_read()
    for _ in range(reps):
        g.sweep(lab, nc)
    tm = g.timing_read()
    g.timing(False)
    g.reset()
    ms = tm["sweep_ms"] / max(tm["sweeps"], 1)
    gbs = tm["bytes"] / max(tm["sweeps"], 1) / (ms * 1e-3) / 1e9
    return {"ms": round(ms, 4), "gteps": round(nnz / (ms * 1e-3) / 1e9, 3),
            "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "communities": int(nc), "repetitions": reps}


def cpu_model() -> str:
    """The host CPU's model name as the kernel reports it (lscpu reads the
    same), with its family / model / stepping numbers, which identify the
    part where a virtual machine shortens the name."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ":" not in ln:
                    if info:
                        break
                    continue
                k, v = ln.split(":", 1)
                info.setdefault(k.strip(), v.strip())
    except OSError:
        pass
    name = info.get("model name", "unknown")
    ids = [(k, info[k]) for k in ("cpu family", "model", "stepping") if k in info]
    if ids:
        name += " (%s)" % ", ".join("%s %s" % kv for kv in ids)
    return name


def cpu_baseline(rp, col, w, budget_s: float):
    """The oracle's sweep (the plain sequential CPU implementation) on the
    same graph and the same labels as the GPU's first level-0 sweep (the
    oracle's own ASSIGN, POSITIVE and COMPONENTS), repeated for about
    budget_s seconds on one core."""
    import oracle
    g = oracle.Graph(rp, col, w)
    t = time.perf_counter()
    a = oracle.assign(g)
    a, _ = oracle.positive(g, a)
    lab, nc, _ = oracle.components(a)
    t_setup = time.perf_counter() - t
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
                cpu=cpu_model(), host_threads=os.cpu_count(),
                sample="%d oracle sweeps of the full graph on the labels after its ASSIGN, "
                       "POSITIVE and COMPONENTS (%.1f s of set-up, not timed), %.1f s"
                       % (reps, t_setup, el))


def _gen_member(args):
    import graphgen as gg
    seed, i, count = args
    return gg.sbm_batch(count, 64, 65536, seed, indices=[i])[0]


def batch_members(count: int, seed: int, procs: int):
    """The batch family: planted-partition graphs with log-uniform node counts
    in [64, 65536], block sizes 16..256, p_in 0.2, mean external degree 2.
    Generated in a process pool (before the GPU is touched)."""
    import multiprocessing as mp
    work = [(seed, i, count) for i in range(count)]
    if procs <= 1:
        return [_gen_member(a) for a in work]
    with mp.get_context("fork").Pool(procs) as pool:
        return pool.map(_gen_member, work, chunksize=4)


def _oracle_member(args):
    import oracle
    rp, col, w, seed = args
    t = time.perf_counter()
    oracle.run(rp, col, w, seed=seed)
    return time.perf_counter() - t


def batch_inputs(args):
    """The batch members, their seeds, the plain-path sample and the oracle's
    graphs/s on a sample (one process per host core).  CPU only: runs before
    the GPU is touched."""
    import graphgen as gg
    count = args.batch_count
    seed = gg.CONFIG_SEEDS["batch2048"]
    procs = max(1, min(16, os.cpu_count() or 1))
    t = time.time()
    members = batch_members(count, seed, procs)
    seeds = [gg.batch_member_seed(args.seed, i) for i in range(count)]
    n_tot = sum(m[0].size - 1 for m in members)
    nnz_tot = sum(m[1].size for m in members)
    log("batch: %d graphs, %d nodes, %d entries, generated in %.1fs"
        % (count, n_tot, nnz_tot, time.time() - t))
    # the sample of the plain path and of the oracle (--plain-sample 0 skips
    # the plain path; the oracle still takes every 16-th member)
    stride = max(1, count // (args.plain_sample if args.plain_sample > 0 else 128))
    sample = list(range(0, count, stride))
    cpu = None
    if not args.no_cpu:
        import multiprocessing as mp
        osample = sample[: max(1, min(len(sample), 4 * procs))]
        t = time.perf_counter()
        with mp.get_context("fork").Pool(procs) as pool:
            times = pool.map(_oracle_member, [(*members[i], seeds[i]) for i in osample])
        el = time.perf_counter() - t
        cpu = dict(value=len(osample) / el, unit="graphs/s", cores=procs, kind="oracle",
                   cpu=cpu_model(),
                   sample="%d members (every %d-th), one oracle process per core, %.1f s"
                          % (len(osample), stride, el),
                   oracle_seconds_per_graph=sum(times) / len(times))
        log("oracle: %.2f graphs/s on %d cores" % (cpu["value"], procs))
    return dict(count=count, seed=seed, members=members, seeds=seeds, n_tot=n_tot,
                nnz_tot=nnz_tot, stride=stride, sample=sample, cpu=cpu)


def batch_gpu(args, inp):
    """Batched run of all members (warm-up, then timed), the plain path (one
    handle and one run per graph) on the sample, and the sample batched."""
    import torch
    import paper_1702_04645_amd as slm
    members, seeds, sample = inp["members"], inp["seeds"], inp["sample"]
    count = inp["count"]
    p = slm.params()
    t = time.perf_counter()
    b = slm.Batch(members, validate=False)
    t_create = time.perf_counter() - t
    for i in range(args.batch_warmup):
        b.run(p, seeds=seeds)
    b.timing(True)
    b.timing_read()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(args.batch_steps):
        res = b.run(p, seeds=seeds)
        log("batched step %d done" % i)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t) / max(args.batch_steps, 1)
    tm = b.timing_read()
    b.close()
    del b
    levels = sum(len(r) for r in res)
    sweep_s = tm["sweep_ms"] / 1e3
    achieved = tm["bytes"] / sweep_s / 1e9 if sweep_s > 0 else 0.0
    out = dict(
        graphs_per_s=round(count / t_batch, 2),
        ms_per_batched_run=round(t_batch * 1e3, 3),
        plain_graphs_per_s=None,
        sample_batched_graphs_per_s=None,
        plain_sample=None,
        create_s=round(t_create, 3),
        sweep_gteps=round(tm["entries"] / sweep_s / 1e9, 3) if sweep_s > 0 else 0.0,
        sweeps_timed=tm["sweeps"],
        sweep_frac_of_hbm_peak=round(achieved / HBM_PEAK_GBS, 4),
        emitted_levels=levels,
        config=dict(workload="batch2048", graphs=count, nodes=inp["n_tot"],
                    entries=inp["nnz_tot"], n_range=[64, 65536], block=[16, 256], p_in=0.2,
                    mean_ext_deg=2, seed=inp["seed"]),
    )
    if inp["cpu"]:
        out["cpu_baseline"] = inp["cpu"]
    if args.plain_sample <= 0:
        return out, achieved
    # plain path on the sample: one handle per graph, created outside the timing
    handles = [slm.Graph(*members[i], validate=False) for i in sample]
    for h, i in zip(handles, sample):
        h.run(slm.params(seed=seeds[i]))  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    for h, i in zip(handles, sample):
        h.run(slm.params(seed=seeds[i]))
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    for h in handles:
        h.close()
    # the same sample as one batch
    sb = slm.Batch([members[i] for i in sample], validate=False)
    sb.run(p, seeds=[seeds[i] for i in sample])
    torch.cuda.synchronize()
    t = time.perf_counter()
    sb.run(p, seeds=[seeds[i] for i in sample])
    torch.cuda.synchronize()
    t_sample_batch = time.perf_counter() - t
    sb.close()
    out.update(plain_graphs_per_s=round(len(sample) / t_plain, 2),
               sample_batched_graphs_per_s=round(len(sample) / t_sample_batch, 2),
               plain_sample="%d members (every %d-th)" % (len(sample), inp["stride"]))
    return out, achieved


def batch_bench(args):
    """Graphs per second of the batch family: all members in one batched run,
    against the plain path (one handle and one run per graph) on a sample,
    and the oracle (one process per host core) on a sample."""
    inp = batch_inputs(args)
    b, achieved = batch_gpu(args, inp)
    out = {
        "metric": "graphs/s batched vs plain",
        "value": b["graphs_per_s"],
        "unit": "graphs/s",
        "n_gpus": 1,
        "steps": args.batch_steps,
        "warmup": args.batch_warmup,
        "ms_per_step": b["ms_per_batched_run"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": dict(b["config"], emitted_levels=b["emitted_levels"]),
        "plain_graphs_per_s": b["plain_graphs_per_s"],
        "sample_batched_graphs_per_s": b["sample_batched_graphs_per_s"],
        "plain_sample": b["plain_sample"],
        "create_s": b["create_s"],
        "sweep_gteps": b["sweep_gteps"],
        "launch_options": "library defaults",
        "sweeps_timed": b["sweeps_timed"],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None},
    }
    if "cpu_baseline" in b:
        out["cpu_baseline"] = b["cpu_baseline"]
    print(json.dumps(out), flush=True)


def _gen_rmat(seed):
    import graphgen as gg
    return gg.rmat(20, 16, 0.57, 0.19, 0.19, seed)


def serve_inputs(args):
    """The served requests: Poisson arrivals at a fixed rate of graphs from
    the batch family plus, one request in 200, an R-MAT scale-20 graph (four
    distinct seeds, cycled).  CPU only: runs before the GPU is touched."""
    import multiprocessing as mp
    import graphgen as gg
    count, rate = args.serve_count, args.serve_rate
    seed = gg.CONFIG_SEEDS["serve"]
    rg = np.random.default_rng(seed)
    is_rmat = rg.random(count) < 1.0 / 200.0
    arrive = np.cumsum(rg.exponential(1.0 / rate, count))
    procs = max(1, min(16, os.cpu_count() or 1))
    t = time.time()
    small_idx = [i for i in range(count) if not is_rmat[i]]
    rmat_seeds = [gg.batch_member_seed(seed, 100000 + j) for j in range(min(4, int(is_rmat.sum())))]
    with mp.get_context("fork").Pool(procs) as pool:
        small = pool.map(_gen_member, [(seed, i, count) for i in small_idx], chunksize=8)
        rmats = pool.map(_gen_rmat, rmat_seeds) if rmat_seeds else []
    graphs = [None] * count
    for i, gph in zip(small_idx, small):
        graphs[i] = gph
    j = 0
    for i in range(count):
        if is_rmat[i]:
            graphs[i] = rmats[j % len(rmats)]
            j += 1
    seeds = [gg.batch_member_seed(args.seed, i) for i in range(count)]
    log("serve: %d requests (%d R-MAT) at %.0f/s, generated in %.1fs"
        % (count, int(is_rmat.sum()), rate, time.time() - t))
    return dict(count=count, rate=rate, seed=seed, is_rmat=is_rmat, arrive=arrive,
                graphs=graphs, seeds=seeds)


def serve_gpu(args, inp):
    """Submits the requests at their arrival times to a server of
    args.serve_lanes lanes (one for R-MAT-sized graphs); latency is measured
    by the library from submission to the end of the request's last level."""
    import paper_1702_04645_amd as slm
    count, is_rmat, arrive = inp["count"], inp["is_rmat"], inp["arrive"]
    graphs, seeds = inp["graphs"], inp["seeds"]
    sv = slm.Server(lanes=args.serve_lanes, large_lanes=1, large_nodes=200_000,
                    node_capacity=1 << 23, entry_capacity=1 << 28, max_members=4096,
                    validate=False)
    tickets = [None] * count
    t0 = time.perf_counter()
    for i in range(count):
        dt = arrive[i] - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets[i] = sv.submit(*graphs[i], seed=seeds[i])
    t_sub = time.perf_counter() - t0
    log("submitted in %.1fs" % t_sub)
    lat = np.zeros(count)
    levels = 0
    for i in range(count):
        res, lat[i] = sv.wait_timed(tickets[i])
        levels += len(res)
        if is_rmat[i] or i % 500 == 499:
            log("request %d done (%s): %.1f ms" % (i, "R-MAT" if is_rmat[i] else "small",
                                                  lat[i] * 1e3))
    t_all = time.perf_counter() - t0
    st = sv.stats()
    sv.close()

    def pct(x, q):
        return round(float(np.percentile(x, q)) * 1e3, 3) if x.size else None
    small_l, rmat_l = lat[~is_rmat], lat[is_rmat]
    return dict(
        graphs_per_s=round(count / t_all, 2),
        span_s=round(t_all, 3),
        p50_ms=pct(lat, 50),
        p99_ms=pct(lat, 99),
        small_p50_ms=pct(small_l, 50),
        small_p99_ms=pct(small_l, 99),
        rmat_p50_ms=pct(rmat_l, 50),
        rmat_max_ms=round(float(rmat_l.max()) * 1e3, 3) if rmat_l.size else None,
        submit_span_s=round(t_sub, 3),
        reserved_hbm_gb=round(st["reserved_bytes"] / 1e9, 2),
        config=dict(workload="serve", requests=count, rate_per_s=inp["rate"],
                    rmat_share="1/200", rmat_requests=int(is_rmat.sum()),
                    small="batch family, n in [64, 65536]", lanes=args.serve_lanes,
                    large_lanes=1,
                    lane_capacity=dict(nodes=1 << 23, entries=1 << 28, members=4096),
                    seed=inp["seed"], emitted_levels=levels),
    )


def serve_bench(args):
    """Serving: served graphs/s and p50/p99 latency of the Poisson mix."""
    inp = serve_inputs(args)
    sv = serve_gpu(args, inp)
    out = {
        "metric": "served graphs/s; p50/p99 latency",
        "value": sv["graphs_per_s"],
        "unit": "graphs/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": round(sv["span_s"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": sv["config"],
    }
    for k in ("p50_ms", "p99_ms", "small_p50_ms", "small_p99_ms", "rmat_p50_ms", "rmat_max_ms",
              "submit_span_s", "reserved_hbm_gb"):
        out[k] = sv[k]
    print(json.dumps(out), flush=True)


def _run_timed(g, p, runs: int, louvain: bool = False):
    """Full runs on a handle: one warm-up, then `runs` timed by the host
    clock around synchronised runs, the sweeps timed by the library's HIP
    events.  Returns (ms per run, sweep stats, last result)."""
    import torch
    run = g.louvain_run if louvain else g.run
    run(p)
    torch.cuda.synchronize()
    g.timing(True)
    g.timing_read()
    t = time.perf_counter()
    for _ in range(runs):
        res = run(p)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / runs
    tm = g.timing_read()
    g.timing(False)
    return ms, tm, res


def _sweep_stats(tm):
    sweep_s = tm["sweep_ms"] / 1e3
    if sweep_s <= 0:
        return dict(sweeps=tm["sweeps"], gteps=None, achieved_gbs=None, frac=None)
    gbs = tm["bytes"] / sweep_s / 1e9
    return dict(sweeps=tm["sweeps"], gteps=round(tm["entries"] / sweep_s / 1e9, 3),
                achieved_gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))


def models_gpu(args, rp, col, w, cfg):
    """The LFR-style 4M graph under the resolution and Erdos-Renyi null
    models (Sec. 2.2-2.3): full-run time, sweep rate, levels and Q."""
    import paper_1702_04645_amd as slm
    out = {}
    for name, kind, num, den in (("config_gamma_1_2", slm.MODEL_CONFIG, 1, 2),
                                 ("er_p_1_4000", slm.MODEL_ER, 1, 4000)):
        with slm.Graph(rp, col, w, validate=False, model=slm.model(kind, num, den)) as g:
            ms, tm, res = _run_timed(g, slm.params(seed=args.seed), args.extra_runs)
        out[name] = dict(model=dict(kind="config" if kind == slm.MODEL_CONFIG else "er",
                                    num=num, den=den),
                         ms_per_run=round(ms, 3), levels=len(res),
                         final_q=res[-1].q if res else None,
                         final_communities=res[-1].n_c if res else None,
                         sweep=_sweep_stats(tm))
        log("model %s: %.1f ms per run" % (name, ms))
    out["workload"] = cfg["workload"]
    return out


def louvain_gpu(args, rp, col, w, cfg):
    """Classical Louvain (the sequential comparison method, exact sequential
    result) against the Synchronised Louvain Method on the same graph."""
    import paper_1702_04645_amd as slm
    p = slm.params(seed=args.seed)
    with slm.Graph(rp, col, w, validate=False) as g:
        ms_l, _, res_l = _run_timed(g, p, 1, louvain=True)
        ms_s, _, res_s = _run_timed(g, p, args.extra_runs)
    log("louvain: %.1f ms per run, slm %.1f ms" % (ms_l, ms_s))
    return dict(workload=cfg["workload"], louvain_ms_per_run=round(ms_l, 3),
                louvain_levels=len(res_l), louvain_passes=[r.rounds for r in res_l],
                louvain_final_q=res_l[-1].q if res_l else None,
                louvain_final_communities=res_l[-1].n_c if res_l else None,
                slm_ms_per_run=round(ms_s, 3), slm_levels=len(res_s),
                slm_final_q=res_s[-1].q if res_s else None,
                slm_final_communities=res_s[-1].n_c if res_s else None)


def _gen_directed(seed):
    import graphgen as gg
    return gg.config_graph("lfr1m_dir")


def directed_cpu(rp, col, w, budget_s: float):
    """The oracle's sweep under the directed model on the labels after its
    own ASSIGN and POSITIVE, repeated for about budget_s seconds."""
    import oracle
    g = oracle.NullGraph(rp, col, w, oracle.DIRECTED, 1, 1)
    a = oracle.assign_nm(g)
    a, _ = oracle.positive_nm(g, a)
    lab, nc, _ = oracle.components(a)
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.sweep_nm(g, lab, nc)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return dict(value=int(g.rp[-1]) * reps / el / 1e9, unit="GTEPS", cores=1, kind="oracle",
                cpu=cpu_model(), sample="%d oracle sweeps of S = W + W^T (%d entries), %.1f s"
                % (reps, int(g.rp[-1]), el))


def directed_gpu(args, rp, col, w, cpu):
    """The directed weighted LFR-shaped graph of the paper's experiments
    (Table 1: N = 10^6, mean degree 50, max 100, mixing 0.5 / 0.4) under the
    directed modularity of Sec. 2.4."""
    import paper_1702_04645_amd as slm
    with slm.Graph(rp, col, w, validate=False,
                   model=slm.model(slm.MODEL_DIRECTED, 1, 1)) as g:
        info = g.level_info()
        ms, tm, res = _run_timed(g, slm.params(seed=args.seed), args.extra_runs)
    log("directed: %.1f ms per run" % ms)
    out = dict(workload="lfr1m_dir", kind="LFR-style directed, weighted", nodes=rp.size - 1,
               arcs=int(col.size), entries_of_s=info["nnz"], mean_degree=50, max_degree=100,
               mixing=[0.5, 0.4], ms_per_run=round(ms, 3), levels=len(res),
               final_q=res[-1].q if res else None,
               final_communities=res[-1].n_c if res else None, sweep=_sweep_stats(tm))
    if cpu:
        out["cpu_baseline"] = cpu
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="lfr4m")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-count", type=int, default=2048)
    ap.add_argument("--plain-sample", type=int, default=128,
                    help="members run on the plain path (0: skip it)")
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=400.0)
    ap.add_argument("--serve-lanes", type=int, default=4)
    ap.add_argument("--batch-steps", type=int, default=1)
    ap.add_argument("--extra-runs", type=int, default=2,
                    help="timed runs of each null-model, directed and Louvain measurement")
    ap.add_argument("--batch-warmup", type=int, default=1)
    ap.add_argument("--no-extras", action="store_true",
                    help="only the sweep line: no batched and served measurements")
    ap.add_argument("--no-tune", action="store_true",
                    help="library default launch options (no autotuned values for this "
                         "device and degree profile)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    if args.workload == "batch2048":
        return batch_bench(args)
    if args.workload == "serve":
        return serve_bench(args)

    t = time.time()
    (rp, col, w), cfg = workload(args.workload)
    n, nnz = rp.size - 1, col.size
    log("workload %s: %d nodes, %d entries, generated in %.1fs" % (args.workload, n, nnz,
                                                                    time.time() - t))
    # everything that runs on host cores (generators, oracle pools) comes
    # before the GPU is touched
    extras = not args.no_extras
    cpu = None
    if rank == 0 and not args.no_cpu:
        log("cpu baseline (oracle sweep, about %.0f s)" % args.cpu_seconds)
        cpu = cpu_baseline(rp, col, w, args.cpu_seconds)
    dpool = dres = None
    if extras:
        import multiprocessing as mp
        dpool = mp.get_context("fork").Pool(1)
        dres = dpool.apply_async(_gen_directed, (0,))
    binp = batch_inputs(args) if extras else None
    sinp = serve_inputs(args) if extras else None
    dgraph = dcpu = None
    if extras:
        dgraph = dres.get()
        dpool.close()
        dpool.join()
        log("directed graph: %d nodes, %d arcs" % (dgraph[0].size - 1, dgraph[1].size))
        if rank == 0 and not args.no_cpu:
            dcpu = directed_cpu(*dgraph, 5.0)

    import torch
    import paper_1702_04645_amd as slm
    params = slm.params(seed=args.seed)
    g = slm.Graph(rp, col, w)
    info = g.level_info()
    tuned, tuned_file = tuned_options(rp) if not args.no_tune else (None, None)
    if tuned:
        from paper_1702_04645_amd import autotune
        autotune.apply(g, tuned)
        log("launch options from %s" % os.path.relpath(tuned_file, ROOT))
    first = first_sweep(g, nnz, n)
    log("first level-0 sweep: %.4f ms" % first["ms"])
    single = singleton_sweep(g, nnz, n)
    log("singleton-label sweep: %.4f ms" % single["ms"])
    copy = copy_gbs()
    log("device copy: %.1f GB/s" % copy)
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
        log("step %d done: %d levels, %.1f ms into the timed steps"
            % (i, len(last), 1e3 * (time.perf_counter() - t0)))
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
        "launch_options": tuned or "library defaults",
        "level0_first_sweep": first,
        "singleton_label_sweep": single,
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
            "traffic": measured_traffic(args.workload),
            "traffic_unit": "GB per sweep (HBM read + write, counters scaled by a copy)",
            "algorithmic_gb_per_sweep": round(tm["bytes"] / max(tm["sweeps"], 1) / 1e9, 4),
            "copy_gbs": copy,
            "frac_of_copy": round(achieved / copy, 4) if copy > 0 else None,
        },
    }
    if cpu:
        out["cpu_baseline"] = cpu
    if extras:
        log("null models")
        out["null_models"] = models_gpu(args, rp, col, w, cfg)
        log("classical Louvain")
        out["louvain"] = louvain_gpu(args, rp, col, w, cfg)
        del rp, col, w
        log("directed")
        out["directed"] = directed_gpu(args, *dgraph, dcpu)
        del dgraph
        log("batched run of the 2048-graph family")
        out["batch"], _ = batch_gpu(args, binp)
        del binp
        log("served mix")
        out["serve"] = serve_gpu(args, sinp)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
