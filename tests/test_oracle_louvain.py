"""Pins of the oracle's classical Louvain (the sequential method the SLM
builds on, the comparison named in Sec. 6): full runs against a brute force
that decides every move on N_Q recomputed from scratch, the strict increase
of N_Q with every move, exact recovery of disjoint cliques, and the pass
cap."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import bruteforce as bf
from test_oracle import tiny_graphs


def test_louvain_runs_match_bruteforce():
    for idx, (rp, col, w) in enumerate(tiny_graphs(40, seed0=1500)):
        A = bf.dense(rp, col, w)
        res = oracle.louvain_run(rp, col, w)
        ref = bf.louvain_run(A)
        assert len(res) == len(ref), idx
        for r1, r2 in zip(res, ref):
            assert np.array_equal(r1["labels"], r2["labels"]), idx
            assert r1["n_c"] == r2["n_c"] and r1["nq"] == r2["nq"]
            assert r1["rounds"] == r2["rounds"] and r1["converged"] == r2["converged"]


@pytest.mark.parametrize("passes,levels", [(1, 0), (2, 1), (1, 1)])
def test_louvain_caps_match_bruteforce(passes, levels):
    for idx, (rp, col, w) in enumerate(tiny_graphs(25, seed0=1600)):
        A = bf.dense(rp, col, w)
        res = oracle.louvain_run(rp, col, w, max_passes=passes, max_levels=levels)
        ref = bf.louvain_run(A, max_passes=passes, max_levels=levels)
        assert len(res) == len(ref)
        for r1, r2 in zip(res, ref):
            assert np.array_equal(r1["labels"], r2["labels"])
            assert r1["rounds"] == r2["rounds"] and r1["converged"] == r2["converged"]


@pytest.mark.parametrize("sizes", [[3], [4, 4], [3, 5, 7], [2, 2, 2, 6]])
def test_louvain_recovers_disjoint_cliques(sizes):
    rp, col, w = gg.cliques(sizes)
    res = oracle.louvain_run(rp, col, w)
    truth = np.repeat(np.arange(len(sizes)), sizes)
    assert len(res) >= 1
    assert np.array_equal(res[-1]["labels"], truth)


def test_louvain_levels_increase_modularity():
    for s in range(6):
        rp, col, w = gg.sbm(400, 40, 0.25, 0.01, 70 + s)
        res = oracle.louvain_run(rp, col, w)
        g = oracle.Graph(rp, col, w)
        prev = oracle.modularity_num(g, np.arange(g.n, dtype=np.int32), g.n)
        for r in res:
            assert r["nq"] > prev
            assert r["nq"] == oracle.modularity_num(g, r["labels"], r["n_c"])
            prev = r["nq"]
        # a level ends with no improving move: every node stays where it is
        lab, nc, p, conv, mv = oracle.louvain_level(g)
        assert conv
