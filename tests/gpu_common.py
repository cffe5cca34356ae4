"""Shared helpers of the GPU parity tests: graph fixtures and oracle states.

Every expected value comes from the CPU oracle (oracle/), never from the GPU
path; the GPU path runs through the C ABI via paper_1702_04645_amd.
"""
from __future__ import annotations

import sys

import numpy as np

import graphgen as gg
import oracle


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


_configs = {}


def config_graph(name):
    """graphgen.config_graph(name), generated once per test session."""
    if name not in _configs:
        say("generating", name)
        _configs[name] = gg.config_graph(name)
    return _configs[name]


def small_graphs():
    """Named small graphs covering every degree bin, hubs, loops, isolated
    nodes and ragged sizes."""
    out = {}
    for s in range(6):
        rg = np.random.default_rng(31 + s)
        n = int(rg.integers(5, 300))
        out["random%d" % s] = gg.random_sparse(n, int(rg.integers(n, 6 * n)), 7, 31 + s,
                                               loops=(s % 2 == 0))
    out["sbm1000"] = gg.sbm(1000, 50, 0.3, 0.01, 5)
    out["rmat12"] = gg.rmat(12, 16, 0.57, 0.19, 0.19, 77)
    out["star5000"] = gg.star(5000)            # one hub row (> 4096 entries)
    out["star600"] = gg.star(600)              # one 4096-bin row
    out["cliques"] = gg.cliques([3, 5, 8, 13], isolated=3)
    out["path200"] = gg.path(200)              # deep assignment trees
    rp, col, w = gg.random_sparse(9000, 30000, 3, 99)
    # add a hub with ragged chunk tail: node 0 linked to 4500 random nodes
    hub_v = np.unique(np.random.default_rng(3).integers(1, 9000, 6000))[:4500]
    extra = gg.csr_from_pairs(9000, np.zeros(hub_v.size, np.int64), hub_v)
    u = np.repeat(np.arange(9000), np.diff(rp))
    u2 = np.repeat(np.arange(9000), np.diff(extra[0]))
    out["mixed_hub"] = gg.csr_from_pairs(9000, np.concatenate([u, u2]),
                                         np.concatenate([col, extra[1]]),
                                         np.concatenate([w, extra[2]]), symmetrise=False)
    return out


def oracle_states(rp, col, w, seed=1):
    """Level-0 states of the oracle: ASSIGN output, POSITIVE output, its
    canonical labels, and the state after one MAXIMAL round."""
    g = oracle.Graph(rp, col, w)
    a0 = oracle.assign(g)
    a1, splits = oracle.positive(g, a0)
    lab1, nc1, _ = oracle.components(a1)
    return g, a0, a1, lab1, nc1


def neighbour_assignment(rp, col, seed, frac=0.8):
    """Random assignment of every node to one of its neighbours (or itself),
    giving cycles of any length."""
    rg = np.random.default_rng(seed)
    n = rp.size - 1
    a = np.arange(n, dtype=np.int32)
    for i in range(n):
        nb = col[rp[i]:rp[i + 1]]
        nb = nb[nb != i]
        if nb.size and rg.random() < frac:
            a[i] = nb[int(rg.integers(0, nb.size))]
    return a
