"""Pins of the oracle's null models (Sec. 2.2-2.4): the configuration model
with a resolution, the Erdos-Renyi null model (p_ij = p) and the directed
weighted modularity with out- and in-strengths.

The brute force (tests/bruteforce.py) takes every decision on the quality
of a partition computed from its definition on the directed (or undirected)
matrix itself, with no gain formula and no symmetrised matrix or strength
vectors; the oracle runs on S = W + W^T with the strengths x, y and the
scale A.  Their quality values differ by a known positive factor (num for
the undirected models, 4 num for the directed one).  Closed forms and
library routines (connected components) pin the extremes.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import graphgen as gg
import oracle
import bruteforce as bf


def tiny_undirected(count, seed0):
    out = []
    for s in range(count):
        rg = np.random.default_rng(seed0 + s)
        n = int(rg.integers(2, 11))
        m = int(rg.integers(1, 3 * n))
        out.append(gg.random_sparse(n, m, int(rg.integers(1, 6)), seed0 + s, loops=(s % 3 == 0)))
    out.append(gg.cliques([3, 4], isolated=1))
    out.append(gg.path(8))
    return out


def tiny_directed(count, seed0):
    out = []
    for s in range(count):
        rg = np.random.default_rng(seed0 + s)
        n = int(rg.integers(2, 11))
        m = int(rg.integers(1, 4 * n))
        out.append(gg.random_directed(n, m, int(rg.integers(1, 6)), seed0 + s,
                                      loops=(s % 3 == 0)))
    # a directed ring with one heavy chord, and a one-way star
    n = 7
    u = np.arange(n)
    out.append(gg.csr_from_pairs(n, np.r_[u, 0], np.r_[(u + 1) % n, 3], np.r_[np.ones(n), 5],
                                 symmetrise=False))
    out.append(gg.csr_from_pairs(6, np.zeros(5), np.arange(1, 6), symmetrise=False))
    return out


def _compare(res, ref, factor):
    assert len(res) == len(ref)
    for r1, r2 in zip(res, ref):
        assert np.array_equal(r1["labels"], r2["labels"])
        assert r1["n_c"] == r2["n_c"]
        assert r1["rounds"] == r2["rounds"]
        assert r1["converged"] == r2["converged"]
        assert r1["nq"] == factor * r2["nq"]


@pytest.mark.parametrize("num,den", [(1, 2), (3, 2), (2, 1), (5, 4)])
def test_config_resolution_runs_match_bruteforce(num, den):
    for idx, (rp, col, w) in enumerate(tiny_undirected(20, 1200 + 31 * num + den)):
        A = bf.dense(rp, col, w)
        res = oracle.run_null(rp, col, w, oracle.CONFIG, num, den, seed=idx)
        ref = bf.run_null(A, bf.CONFIG, num, den, idx, oracle.draw)
        _compare(res, ref, num)


@pytest.mark.parametrize("num,den", [(1, 8), (1, 30), (2, 7)])
def test_erdos_renyi_runs_match_bruteforce(num, den):
    for idx, (rp, col, w) in enumerate(tiny_undirected(20, 2300 + num * 10 + den)):
        A = bf.dense(rp, col, w)
        res = oracle.run_null(rp, col, w, oracle.ER, num, den, seed=idx)
        ref = bf.run_null(A, bf.ER, num, den, idx, oracle.draw)
        _compare(res, ref, num)


@pytest.mark.parametrize("num,den", [(1, 1), (1, 2), (3, 2)])
def test_directed_runs_match_bruteforce(num, den):
    for idx, (rp, col, w) in enumerate(tiny_directed(24, 3400 + num * 10 + den)):
        W = bf.dense(rp, col, w)
        res = oracle.run_null(rp, col, w, oracle.DIRECTED, num, den, seed=idx)
        ref = bf.run_null(W, bf.DIRECTED, num, den, idx, oracle.draw)
        _compare(res, ref, 4 * num)


def test_directed_round_caps_match_bruteforce():
    for idx, (rp, col, w) in enumerate(tiny_directed(16, 5100)):
        W = bf.dense(rp, col, w)
        for mr, ml in ((1, 0), (2, 1)):
            res = oracle.run_null(rp, col, w, oracle.DIRECTED, 1, 1, seed=idx, max_rounds=mr,
                                  max_levels=ml)
            ref = bf.run_null(W, bf.DIRECTED, 1, 1, idx, oracle.draw, max_rounds=mr,
                              max_levels=ml)
            _compare(res, ref, 4)


def test_directed_steps_match_bruteforce():
    """Per step on random labellings: local gains have the sign of the
    brute-force loss of leaving, and the sweep's best community is the
    brute-force argmax of the quality gain (ties to the lowest label)."""
    for idx, (rp, col, w) in enumerate(tiny_directed(30, 6100)):
        W = bf.dense(rp, col, w)
        S = W + W.T
        n = W.shape[0]
        g = oracle.NullGraph(rp, col, w, oracle.DIRECTED, 1, 1)
        qual = lambda lab: bf.quality(W, lab, bf.DIRECTED, 1, 1, None)
        rg = np.random.default_rng(idx)
        lab = bf.canonical(rg.integers(0, max(1, n // 2), n))
        nc = int(lab.max()) + 1
        gl = oracle.local_gain_nm(g, lab, nc)
        base = qual(lab)
        loss = []
        for u in range(n):
            l2 = lab.copy()
            l2[u] = nc  # u alone
            loss.append(base - qual(l2))
        assert np.array_equal(gl, 2 * np.array(loss))  # g = 2 num times the loss
        best, delta, _ = oracle.sweep_nm(g, lab, nc)
        for i in range(n):
            cands = sorted({int(lab[j]) for j in range(n) if S[i, j] > 0 and j != i} - {lab[i]})
            stay_loss = None
            bestc, bestg = int(lab[i]), None
            for c in cands:
                l2 = lab.copy()
                l2[i] = c
                gain = qual(l2) - base
                if bestg is None or gain > bestg:
                    bestg, bestc = gain, c
            if bestg is None or bestg <= 0:
                bestc = int(lab[i])
            assert best[i] == bestc, (idx, i)
            assert (delta[i] > 0) == (bestc != lab[i])


def test_directed_on_a_symmetric_graph_is_the_undirected_run():
    """A symmetric W as a directed graph: S = 2A, x = 2k, y = 0, A = 2 M2, so
    every gain is 4 times the undirected one: the same run, N_Q times 4, the
    same Q."""
    graphs = [gg.sbm(600, 40, 0.2, 0.01, 4), gg.rmat(9, 8, 0.57, 0.19, 0.19, 5),
              gg.random_sparse(300, 900, 5, 6, loops=True)]
    for idx, (rp, col, w) in enumerate(graphs):
        a = oracle.run(rp, col, w, seed=idx)
        b = oracle.run_null(rp, col, w, oracle.DIRECTED, 1, 1, seed=idx)
        _compare(b, a, 4)
        for x, y in zip(a, b):
            assert x["q"] == y["q"]


def test_default_model_is_the_plain_run():
    for idx, (rp, col, w) in enumerate([gg.sbm(500, 25, 0.3, 0.01, 8),
                                        gg.random_sparse(200, 700, 4, 9)]):
        a = oracle.run(rp, col, w, seed=idx)
        b = oracle.run_null(rp, col, w, oracle.CONFIG, 1, 1, seed=idx)
        _compare(b, a, 1)
        for x, y in zip(a, b):
            assert x["q"] == y["q"]


def test_tiny_erdos_renyi_p_finds_the_connected_components():
    """With p far below 1 / n^2 every edge between two communities is worth
    merging, and communities only grow along edges: the last level is the
    set of connected components (scipy)."""
    for s in range(8):
        rp, col, w = gg.random_sparse(120, 90 + 10 * s, 5, 700 + s)
        n = rp.size - 1
        res = oracle.run_null(rp, col, w, oracle.ER, 1, 10**7, seed=s)
        M = sp.csr_matrix((w, col, rp), shape=(n, n))
        ncc, cc = csg.connected_components(M, directed=False)
        isolated = int((np.diff(rp) == 0).sum())
        assert len(res) >= 1
        last = res[-1]["labels"]
        assert np.array_equal(bf.canonical(cc), bf.canonical(last))
        assert res[-1]["n_c"] == ncc


def test_large_resolution_leaves_the_identity():
    """When gamma k_i k_j >= M2 A_ij on every edge no pair gain is positive:
    ASSIGN self-assigns every node and no level is emitted."""
    for s in range(6):
        rp, col, w = gg.random_sparse(60, 200, 3, 800 + s)
        g = oracle.Graph(rp, col, w)
        u = np.repeat(np.arange(g.n), np.diff(rp))
        off = u != col
        need = (g.m2 * w[off]) / (g.k[u[off]] * g.k[col[off]])
        num = int(np.ceil(need.max())) if need.size else 1
        assert oracle.run_null(rp, col, w, oracle.CONFIG, num, 1, seed=s) == []
        # just below the threshold some pair is positive again
        if need.size and num > 1:
            assert len(oracle.run_null(rp, col, w, oracle.CONFIG, 2 * num - 1, 2, seed=s)) >= 1 \
                or need.max() <= num - 0.5


def test_symmetrize_is_w_plus_w_transpose():
    for s in range(10):
        rp, col, w = gg.random_directed(30, 120, 7, 900 + s, loops=True)
        W = bf.dense(rp, col, w)
        rp2, col2, w2 = oracle.symmetrize(rp, col, w)
        assert np.array_equal(bf.dense(rp2, col2, w2), W + W.T)
        for i in range(30):
            assert np.all(np.diff(col2[rp2[i]:rp2[i + 1]]) > 0)


def test_null_model_arguments_and_bounds():
    rp, col, w = gg.random_sparse(40, 100, 3, 1)
    with pytest.raises(ValueError):
        oracle.run_null(rp, col, w, oracle.CONFIG, 0, 1)
    with pytest.raises(ValueError):
        oracle.run_null(rp, col, w, 7, 1, 1)
    with pytest.raises(OverflowError):
        oracle.run_null(rp, col, w, oracle.ER, 1 << 31, 1)
    with pytest.raises(OverflowError):
        oracle.run_null(rp, col, w, oracle.CONFIG, 1 << 20, 1 << 40)


def directed_assignments(count, seed0):
    """Directed graphs with an assignment along S = W + W^T: a ring over the
    first L nodes and the other nodes hung below random neighbours, so both
    branch and cycle cuts of POSITIVE are exercised."""
    out = []
    for s in range(count):
        rg = np.random.default_rng(seed0 + s)
        n = int(rg.integers(4, 12))
        L = int(rg.integers(2, min(n, 6) + 1))
        u = np.arange(L)
        extra = int(rg.integers(n, 4 * n))
        cu, cv = rg.integers(0, n, extra), rg.integers(0, n, extra)
        uu = np.r_[u, cu]
        vv = np.r_[(u + 1) % L, cv]
        wt = np.r_[rg.integers(1, 4, L), rg.integers(1, 9, extra)]
        keep = uu != vv
        rp, col, w = gg.csr_from_pairs(n, uu[keep], vv[keep], wt[keep], symmetrise=False)
        S = bf.dense(rp, col, w)
        S = S + S.T
        a0 = np.arange(n, dtype=np.int32)
        a0[:L] = (u + 1) % L
        for i in range(L, n):
            nb = [j for j in range(n) if S[i, j] > 0 and j != i and (j < i)]
            if nb:
                a0[i] = nb[int(rg.integers(0, len(nb)))]
        out.append((rp, col, w, a0))
    return out


def test_directed_positive_matches_bruteforce():
    """POSITIVE on given assignments, directed quality: the same splits and
    the same final assignment as the brute force."""
    for idx, (rp, col, w, a0) in enumerate(directed_assignments(150, 8800)):
        W = bf.dense(rp, col, w)
        g = oracle.NullGraph(rp, col, w, oracle.DIRECTED, 1, 1)
        qual = lambda lab: bf.quality(W, lab, bf.DIRECTED, 1, 1, None)
        a1, s1 = oracle.positive_nm(g, a0)
        a2, s2 = bf.positive(W + W.T, list(a0), qual)
        assert s1 == s2, idx
        assert np.array_equal(a1, np.array(a2)), idx
