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

Usage (on a GPU):

    import graphgen as gg, paper_1702_04645_amd as slm
    from paper_1702_04645_amd import autotune
    with slm.Graph(*gg.config_graph("rmat20"), validate=False) as g:
        best = autotune.tune(g)
    autotune.save("tuned.json", best)
"""
import json

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
