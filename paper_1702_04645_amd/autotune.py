"""Launch autotuner of the MAXIMAL sweep (Sec. 3.4).

The degree bins of the sweep (their limits and LDS table shapes) are fixed
when the library is compiled; what is left to the device at run time is set
through `slm_set_option`: the workgroup count of each bin's persistent
kernel, the partition table and pass size of hub rows, and the level size
from which the bins run on side streams.  `tune` times sweeps of one graph
with HIP events and walks those options one at a time (coordinate descent),
keeping a value only when it is faster by more than `min_gain`; the labels
the sweep returns are compared after every change, since no option may
alter a result.  `save` / `load` / `apply` keep the chosen values as JSON.

The tuned values are kept per device and degree profile: `save_keyed` files
them under a key made of the GPU architecture, the entry count (log2,
rounded) and each degree bin's share of the entries (in twentieths), and
`find` returns the values kept for a graph with the same key on the same
architecture, or None (then the library defaults stand).  The cache is the
folder `tuned/` beside this file, or the folder the environment variable
SLM_TUNE_CACHE names.

Usage (on a GPU):

    import graphgen as gg, paper_1702_04645_amd as slm
    from paper_1702_04645_amd import autotune
    rp, col, w = gg.config_graph("rmat20")
    with slm.Graph(rp, col, w, validate=False) as g:
        best = autotune.tune(g)
    autotune.save_keyed(rp, autotune.device_arch(), best, workload="rmat20")
"""
import hashlib
import json
import os

import numpy as np

# candidate values per option; 0 for a grid is the library's default
BIN_DEGREES = (64, 128, 256, 512, 1024, 2048, 4096)
CANDIDATES = {
    **{"grid_%d" % d: (0, 256, 512, 768, 1024, 2048, 4096) for d in BIN_DEGREES},
    "hub_table_bits": (9, 10, 11),
    "hub_pass_pairs": (384, 768, 1536),
    "fanout_min_entries": (0, 1 << 20, 1 << 22, 1 << 40),
}
DEFAULTS = {
    **{"grid_%d" % d: 0 for d in BIN_DEGREES},
    "hub_table_bits": 11,
    "hub_pass_pairs": 1536,
    "fanout_min_entries": 1 << 22,
}


# the sweep's degree bins by their largest row: isolated nodes, rows of up to
# 8, 32, 64, ..., 4096 entries, and hub rows above
BIN_LIMITS = (0, 8, 32, 64, 128, 256, 512, 1024, 2048, 4096)
PROFILE_STEPS = 20  # a bin's share of the entries is kept in twentieths


def degree_profile(row_ptr):
    """What the launch options depend on: log2 of the entry count (rounded)
    and each degree bin's share of the entries (rounded to twentieths)."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    deg = np.diff(rp)
    nnz = int(deg.sum())
    b = np.searchsorted(np.array(BIN_LIMITS, dtype=np.int64), deg, side="left")
    ent = np.bincount(b, weights=deg.astype(np.float64), minlength=len(BIN_LIMITS) + 1)
    shares = [int(round(x * PROFILE_STEPS / nnz)) if nnz else 0 for x in ent]
    return {"entries_log2": int(round(np.log2(nnz))) if nnz else 0, "bin_shares": shares}


def profile_key(row_ptr, arch: str) -> str:
    p = degree_profile(row_ptr)
    return "%s|e%d|%s" % (arch, p["entries_log2"], ",".join(str(x) for x in p["bin_shares"]))


def cache_dir() -> str:
    return os.environ.get("SLM_TUNE_CACHE") or os.path.join(os.path.dirname(__file__), "tuned")


def cache_path(key: str, directory=None) -> str:
    arch = key.split("|", 1)[0]
    h = hashlib.sha1(key.encode()).hexdigest()[:16]
    return os.path.join(directory or cache_dir(), "%s-%s.json" % (arch, h))


def device_arch() -> str:
    """The current GPU's architecture name (for example gfx950)."""
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return props.gcnArchName.split(":")[0]


def save_keyed(row_ptr, arch: str, result, directory=None, workload=None) -> str:
    """Files a `tune` result under the key of this graph and architecture;
    returns the file's path."""
    key = profile_key(row_ptr, arch)
    rec = dict(result)
    rec.update(key=key, arch=arch, profile=degree_profile(row_ptr))
    if workload:
        rec["workload"] = workload
    path = cache_path(key, directory)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    save(path, rec)
    return path


def find(row_ptr, arch: str, directory=None):
    """(options, path) kept for a graph of this key on this architecture, or
    (None, None)."""
    key = profile_key(row_ptr, arch)
    path = cache_path(key, directory)
    if not os.path.exists(path):
        return None, None
    rec = load(path)
    if rec.get("key") != key:
        return None, None
    return rec["options"], path


def _sweep_us(g, lab, nc, reps, blocks):
    """Best over `blocks` of the mean sweep time of `reps` sweeps (us)."""
    import torch
    g.sweep(lab, nc)
    torch.cuda.synchronize()
    g.timing(True)
    g.timing_read()
    best = float("inf")
    for _ in range(blocks):
        for _ in range(reps):
            g.sweep(lab, nc)
        t = g.timing_read()
        best = min(best, t["sweep_ms"] / max(t["sweeps"], 1) * 1e3)
    g.timing(False)
    return best


def level0_labels(g):
    """Labels of the first MAXIMAL sweep of a run: ASSIGN, POSITIVE, COMPONENTS."""
    a = g.assign()
    a, _ = g.positive(a)
    lab, nc, _ = g.components(a)
    return lab, nc


def tune(g, lab=None, nc=None, reps=8, blocks=3, passes=2, min_gain=0.01, log=None):
    """Coordinate descent over CANDIDATES on graph handle g (a Graph or Batch).

    lab / nc: the labels to sweep (default: those of the first sweep of a run).
    Returns {"options": {...}, "us": best time, "us_default": default time}."""
    if lab is None:
        lab, nc = level0_labels(g)
    for k, v in DEFAULTS.items():
        g.set_option(k, v)
    ref = [t.cpu().numpy() for t in g.sweep(lab, nc)]
    cur = dict(DEFAULTS)
    t_def = t_cur = _sweep_us(g, lab, nc, reps, blocks)
    if log:
        log("default %.1f us" % t_def)
    for _ in range(passes):
        changed = False
        for k, cands in CANDIDATES.items():
            for v in cands:
                if v == cur[k]:
                    continue
                g.set_option(k, v)
                out = [t.cpu().numpy() for t in g.sweep(lab, nc)]
                if not all(np.array_equal(a, b) for a, b in zip(out, ref)):
                    raise AssertionError("option %s=%d changed the sweep" % (k, v))
                t = _sweep_us(g, lab, nc, reps, blocks)
                if t < t_cur * (1.0 - min_gain):
                    cur[k], t_cur, changed = v, t, True
                    if log:
                        log("%s=%d %.1f us" % (k, v, t))
                g.set_option(k, cur[k])
        if not changed:
            break
    return {"options": cur, "us": t_cur, "us_default": t_def}


def apply(g, options):
    for k, v in options.items():
        g.set_option(k, int(v))


def save(path, result):
    with open(path, "w") as f:
        json.dump(result, f, indent=1, sort_keys=True)


def load(path):
    with open(path) as f:
        return json.load(f)
