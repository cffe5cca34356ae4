"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these checks re-types the oracle's formulas: they compare it with
the modularity numerator recomputed from scratch (tests/bruteforce.py), with
closed forms, with networkx, with exhaustive enumeration, with published
SplitMix64 outputs, and with structural invariants.
"""
import functools
import itertools
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_graphs(count=40, seed0=100):
    """Random tiny weighted graphs, some with self-loops, plus fixtures."""
    out = []
    for s in range(count):
        rg = np.random.default_rng(seed0 + s)
        n = int(rg.integers(2, 11))
        m = int(rg.integers(1, 3 * n))
        out.append(gg.random_sparse(n, m, int(rg.integers(1, 6)), seed0 + s, loops=(s % 3 == 0)))
    out.append(gg.path(9))
    out.append(gg.star(7))
    out.append(gg.cliques([3, 4], isolated=1))
    return out


# ------------------------------------------------------------------ draws

def test_splitmix64_known_answers():
    """SplitMix64 (Steele, Lea & Flood 2014) outputs of the stream seeded with
    0, as published with the reference implementation."""
    with open(os.path.join(GOLDEN, "splitmix64_seed0.json")) as f:
        kat = json.load(f)
    gamma = 0x9E3779B97F4A7C15
    for idx, val in enumerate(kat["outputs"], start=1):
        assert oracle.mix64((idx * gamma) % 2**64) == int(val, 16)
    # the draw is the high half of the (ctr+1)-th output with ctr = 0
    assert oracle.draw(0, 0, 0, 0) == int(kat["outputs"][0], 16) >> 32
    assert oracle.draw(0, 0, 0, 1) == int(kat["outputs"][1], 16) >> 32


def test_draw_counter_layout_and_uniformity():
    # level/round/node occupy disjoint counter fields: all distinct
    vals = {oracle.draw(7, l, r, i) for l in range(3) for r in range(3) for i in range(50)}
    assert len(vals) == 450
    xs = np.array([oracle.draw(12345, 0, 0, i) for i in range(20000)], dtype=np.float64)
    assert abs(xs.mean() / 2**32 - 0.5) < 0.01
    assert abs((xs < 2**31).mean() - 0.5) < 0.01


# ----------------------------------------------------------- closed forms

@pytest.mark.parametrize("sizes", [[3], [4, 4], [3, 5, 7], [2, 2, 2, 6]])
def test_cliques_recovered_exactly(sizes):
    rp, col, w = gg.cliques(sizes, isolated=2)
    res = oracle.run(rp, col, w, seed=3)
    assert len(res) == 1
    lab = res[0]["labels"]
    base = 0
    for c, s in enumerate(sizes):
        assert np.all(lab[base:base + s] == c)
        base += s
    assert res[0]["n_c"] == len(sizes) + 2
    m2 = sum(s * (s - 1) for s in sizes)
    q = 1.0 - sum((s * (s - 1)) ** 2 for s in sizes) / m2**2
    assert abs(res[0]["q"] - q) < 1e-12
    assert res[0]["nq"] == m2 * m2 - sum((s * (s - 1)) ** 2 for s in sizes)


def test_modularity_closed_forms():
    for rp, col, w in tiny_graphs(15):
        g = oracle.Graph(rp, col, w)
        if g.m2 == 0:
            continue
        A = bf.dense(rp, col, w)
        k = A.sum(1)
        # one community: Q = 0
        assert oracle.modularity_num(g, np.zeros(g.n, np.int32), 1) == 0
        # all singletons: N_Q = M2 * sum A_ii - sum k_i^2
        single = np.arange(g.n, dtype=np.int32)
        assert oracle.modularity_num(g, single, g.n) == g.m2 * int(np.trace(A)) - int((k * k).sum())
    # K_n: the single community is also the best; Q = 0
    rp, col, w = gg.cliques([6])
    assert oracle.run(rp, col, w)[0]["nq"] == 0


def test_modularity_matches_from_scratch_and_networkx():
    nx = pytest.importorskip("networkx")
    for idx, (rp, col, w) in enumerate(tiny_graphs(20)):
        g = oracle.Graph(rp, col, w)
        if g.m2 == 0:
            continue
        A = bf.dense(rp, col, w)
        rg = np.random.default_rng(idx)
        lab = bf.canonical(rg.integers(0, 3, g.n)).astype(np.int32)
        nc = int(lab.max()) + 1
        v = oracle.modularity_num(g, lab, nc)
        assert v == bf.nq(A, lab)
        q = oracle.modularity(v, g.m2)
        if np.trace(A) == 0:  # networkx counts a self-loop twice in the degree
            G = nx.Graph()
            G.add_nodes_from(range(g.n))
            for i in range(g.n):
                for j in range(i + 1, g.n):
                    if A[i, j]:
                        G.add_edge(i, j, weight=int(A[i, j]))
            comms = [set(np.flatnonzero(lab == c).tolist()) for c in range(nc)]
            assert abs(q - nx.community.modularity(G, comms, weight="weight")) < 1e-12


# ----------------------------------------------------- step-by-step pins

def test_assign_matches_bruteforce_and_structure():
    for rp, col, w in tiny_graphs(40):
        g = oracle.Graph(rp, col, w)
        A = bf.dense(rp, col, w)
        a = oracle.assign(g)
        assert list(a) == bf.assign(A)
        # cycles of the assignment graph have length 1 or 2 (pair is symmetric
        # and ties go to the lowest id), and a self-assigned node has no
        # incoming assignment
        for i in range(g.n):
            cyc = bf.cycle_nodes(list(a), i)
            assert len(cyc) in (1, 2)
            if a[i] == i:
                assert not np.any((a == i) & (np.arange(g.n) != i))


def test_components_match_bruteforce():
    rg = np.random.default_rng(5)
    for t in range(60):
        n = int(rg.integers(1, 30))
        a = rg.integers(0, n, n).astype(np.int32)
        lab, nc, cyc = oracle.components(a)
        ref = bf.wcc(list(a))
        assert np.array_equal(lab, ref)
        assert nc == int(ref.max()) + 1
        # every component holds exactly one cycle
        for c in range(nc):
            members = np.flatnonzero(lab == c)
            cn = bf.cycle_nodes(list(a), int(members[0]))
            assert set(np.flatnonzero(cyc & (lab == c)).tolist()) == set(cn)


def test_local_gain_is_half_the_nq_loss_of_leaving():
    for rp, col, w in tiny_graphs(20):
        g = oracle.Graph(rp, col, w)
        A = bf.dense(rp, col, w)
        a = oracle.assign(g)
        lab, nc, _ = oracle.components(a)
        assert list(oracle.local_gain(g, lab, nc)) == bf.local_gains(A, lab)


def test_positive_matches_bruteforce_and_leaves_no_negative_gain():
    for idx, (rp, col, w) in enumerate(tiny_graphs(40)):
        g = oracle.Graph(rp, col, w)
        A = bf.dense(rp, col, w)
        rg = np.random.default_rng(idx)
        # both ASSIGN outputs and arbitrary neighbour assignments (longer cycles)
        starts = [oracle.assign(g)]
        a_rand = np.arange(g.n, dtype=np.int32)
        for i in range(g.n):
            nb = [int(c) for c in col[rp[i]:rp[i + 1]] if c != i]
            if nb and rg.random() < 0.8:
                a_rand[i] = nb[int(rg.integers(0, len(nb)))]
        starts.append(a_rand)
        for a0 in starts:
            a1, s1 = oracle.positive(g, a0)
            a2, s2 = bf.positive(A, list(a0))
            assert list(a1) == a2
            assert s1 == s2
            lab, nc, _ = oracle.components(a1)
            assert np.all(oracle.local_gain(g, lab, nc) >= 0)


def test_sweep_delta_is_half_the_nq_gain():
    for idx, (rp, col, w) in enumerate(tiny_graphs(30)):
        g = oracle.Graph(rp, col, w)
        A = bf.dense(rp, col, w)
        rg = np.random.default_rng(idx)
        for lab in (np.arange(g.n), bf.canonical(rg.integers(0, 3, g.n))):
            lab = lab.astype(np.int32)
            nc = int(lab.max()) + 1
            best, delta, wown = oracle.sweep(g, lab, nc)
            base = bf.nq(A, lab)
            for i in range(g.n):
                gains = {}
                for j in range(g.n):
                    if j != i and A[i, j] and lab[j] != lab[i]:
                        l2 = lab.copy()
                        l2[i] = lab[j]
                        gains[int(lab[j])] = bf.nq(A, l2) - base
                top = max(gains.values()) if gains else None
                if top is not None and top > 0:
                    assert best[i] == min(c for c, v in gains.items() if v == top)
                    assert 2 * delta[i] == top
                else:
                    assert best[i] == lab[i] and delta[i] == 0
                assert wown[i] == sum(A[i, j] for j in range(g.n) if j != i and lab[j] == lab[i])


def test_maximal_round_matches_bruteforce():
    for idx, (rp, col, w) in enumerate(tiny_graphs(40, seed0=900)):
        g = oracle.Graph(rp, col, w)
        A = bf.dense(rp, col, w)
        a = oracle.assign(g)
        a, _ = oracle.positive(g, a)
        for rnd in range(3):
            for p in (1 << 31, 1 << 32):
                a1, v1, st = oracle.maximal_round(g, a, 77 + idx, 1, rnd, p)
                a2, v2 = bf.maximal_round(A, list(a), lambda i: oracle.draw(77 + idx, 1, rnd, i), p)
                assert v1 == v2
                assert list(a1) == a2
            a = a1


def test_contraction_is_st_a_s_and_conserves():
    for idx, (rp, col, w) in enumerate(tiny_graphs(25)):
        g = oracle.Graph(rp, col, w)
        A = bf.dense(rp, col, w)
        rg = np.random.default_rng(idx)
        lab = bf.canonical(rg.integers(0, 4, g.n)).astype(np.int32)
        nc = int(lab.max()) + 1
        rp2, col2, w2 = oracle.contract(g, lab, nc)
        A2 = bf.dense(rp2, col2, w2)
        assert np.array_equal(A2, bf.contract(A, lab))
        assert np.array_equal(A2, A2.T)
        assert int(w2.sum()) == g.m2
        for r in range(nc):  # rows sorted by column
            assert np.all(np.diff(col2[rp2[r]:rp2[r + 1]]) > 0)
        g2 = oracle.Graph(rp2, col2, w2)
        sig = np.bincount(lab, weights=g.k, minlength=nc).astype(np.int64)
        assert np.array_equal(g2.k, sig)
        ident = np.arange(nc, dtype=np.int32)
        assert oracle.modularity_num(g2, ident, nc) == oracle.modularity_num(g, lab, nc)


# ----------------------------------------------------------- whole runs

def test_full_run_matches_bruteforce():
    for idx, (rp, col, w) in enumerate(tiny_graphs(30, seed0=500)):
        A = bf.dense(rp, col, w)
        res = oracle.run(rp, col, w, seed=idx)
        ref = bf.run(A, idx, oracle.draw)
        assert len(res) == len(ref)
        for r1, r2 in zip(res, ref):
            assert np.array_equal(r1["labels"], r2["labels"])
            assert r1["n_c"] == r2["n_c"]
            assert r1["nq"] == r2["nq"]
            assert r1["rounds"] == r2["rounds"]
            assert r1["converged"] == r2["converged"]


@functools.lru_cache(maxsize=1)
def _cap_cases():
    """Graphs whose levels need several MAXIMAL rounds, so that small round
    caps cut them (the tiny graphs and the ring graphs; each is run with a
    low and the default acceptance threshold), plus unit-weight random graphs
    of 20-60 nodes whose dense from-scratch run emits at least three levels,
    so that a cap of two levels cuts a run."""
    out = [(rp, col, w, i) for i, (rp, col, w) in enumerate(tiny_graphs(30, seed0=900))]
    out += [(rp, col, w, 100 + i) for i, (rp, col, w, _) in enumerate(ring_graphs(30, seed0=9100))]
    deep = 0
    for s in range(400):
        rg = np.random.default_rng(6000 + s)
        n = int(rg.integers(20, 60))
        g = gg.random_sparse(n, int(rg.integers(n, 3 * n)), 1, 6000 + s)
        if len(bf.run(bf.dense(*g), s, oracle.draw)) >= 3:
            out.append((*g, s))
            deep += 1
            if deep == 3:
                break
    assert deep == 3
    return tuple(out)


@pytest.mark.parametrize("max_rounds,max_levels", [(0, 0), (1, 0), (2, 0), (3, 0), (1, 1),
                                                   (2, 1), (3, 2), (64, 1), (64, 2)])
def test_round_and_level_caps_match_bruteforce(max_rounds, max_levels):
    """The inner loop of Algorithm 1 runs MAXIMAL rounds while some move is
    valid; with a cap on rounds the level ends after that many rounds with
    converged = False, and the run stops after max_levels emitted levels.
    Compared with the dense from-scratch run level by level."""
    cut = short = 0
    for rp, col, w, idx in _cap_cases():
        A = bf.dense(rp, col, w)
        for accept in (1 << 28, 1 << 31):
            res = oracle.run(rp, col, w, seed=idx, accept_p=accept, max_rounds=max_rounds,
                             max_levels=max_levels)
            ref = bf.run(A, idx, oracle.draw, p_threshold=accept, max_rounds=max_rounds,
                         max_levels=max_levels)
            full = bf.run(A, idx, oracle.draw, p_threshold=accept, max_rounds=max_rounds)
            assert len(res) == len(ref)
            for r1, r2 in zip(res, ref):
                assert np.array_equal(r1["labels"], r2["labels"])
                assert r1["n_c"] == r2["n_c"] and r1["nq"] == r2["nq"]
                assert r1["rounds"] == r2["rounds"] and r1["converged"] == r2["converged"]
                assert r1["rounds"] <= max_rounds
                cut += int(not r1["converged"])
            if max_levels > 0:
                assert len(res) == min(max_levels, len(full))
                short += int(len(full) > max_levels)
    # the fixture really reaches the caps
    if max_rounds < 64:
        assert cut > 5
    if max_levels > 0 and max_rounds > 0:
        assert short > 0


def test_q_non_decreasing_and_below_optimum():
    for idx, (rp, col, w) in enumerate(tiny_graphs(25, seed0=300)):
        A = bf.dense(rp, col, w)
        n = A.shape[0]
        res = oracle.run(rp, col, w, seed=idx)
        if not res:
            continue
        g = oracle.Graph(rp, col, w)
        q_single = oracle.modularity(oracle.modularity_num(g, np.arange(n, dtype=np.int32), n),
                                     g.m2)
        qs = [q_single] + [r["q"] for r in res]
        assert all(b >= a for a, b in zip(qs, qs[1:]))
        if n <= 9:
            best = max(bf.nq(A, p) for p in bf.set_partitions(n))
            assert all(r["nq"] <= best for r in res)


def test_sbm_recovers_planted_blocks_mostly():
    rp, col, w = gg.sbm(1024, 64, 0.3, 0.002, 11)
    res = oracle.run(rp, col, w, seed=1)
    lab = res[-1]["labels"]
    blocks = np.arange(1024) // 64
    # most nodes share the label of the majority of their block
    agree = 0
    for b in range(16):
        vals, cnt = np.unique(lab[blocks == b], return_counts=True)
        agree += cnt.max()
    assert agree > 0.9 * 1024
    assert res[-1]["q"] > 0.8


def test_determinism_and_seed_dependence():
    rp, col, w = gg.sbm(600, 40, 0.2, 0.01, 3)
    r1 = oracle.run(rp, col, w, seed=9)
    r2 = oracle.run(rp, col, w, seed=9)
    assert len(r1) == len(r2)
    for x, y in zip(r1, r2):
        assert np.array_equal(x["labels"], y["labels"]) and x["nq"] == y["nq"]


def test_degenerate_inputs():
    # no nodes, no edges, a lone self-loop: nothing to emit
    empty = (np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert oracle.run(*empty) == []
    rp = np.zeros(6, np.int64)
    assert oracle.run(rp, np.zeros(0, np.int32), np.zeros(0, np.int32)) == []
    rp, col, w = gg.csr_from_pairs(3, np.array([1]), np.array([1]), np.array([5]))
    assert oracle.run(rp, col, w) == []
    # one edge: the pair merges; Q = 0 for the single community
    rp, col, w = gg.csr_from_pairs(2, np.array([0]), np.array([1]))
    res = oracle.run(rp, col, w)
    assert len(res) == 1 and res[0]["n_c"] == 1 and res[0]["nq"] == 0


def ring_graphs(count=60, seed0=4000):
    """A ring over the first L nodes plus heavier random edges to the other
    nodes; the assignment a(i) = i+1 on the ring gives one cycle of length L
    (the other nodes are self-assigned), so cycle cuts of many lengths and
    branch cuts get exercised."""
    out = []
    for s in range(count):
        rg = np.random.default_rng(seed0 + s)
        n = int(rg.integers(4, 12))
        L = int(rg.integers(3, n + 1))
        u = np.arange(L)
        v = (u + 1) % L
        extra = int(rg.integers(1, 2 * n))
        cu = rg.integers(0, n, extra)
        cv = rg.integers(0, n, extra)
        uu = np.concatenate([u, cu])
        vv = np.concatenate([v, cv])
        wt = np.concatenate([rg.integers(1, 4, L), rg.integers(1, 12, extra)])
        keep = uu != vv
        rp, col, w = gg.csr_from_pairs(n, uu[keep], vv[keep], wt[keep])
        a0 = np.arange(n, dtype=np.int32)
        a0[:L] = (u + 1) % L
        # hang a few non-ring nodes below ring nodes through existing edges
        for i in range(L, n):
            nb = [int(c) for c in col[rp[i]:rp[i + 1]] if c != i]
            if nb and rg.random() < 0.5:
                a0[i] = nb[0]
        out.append((rp, col, w, a0))
    return out


def test_positive_cycle_cuts_match_bruteforce():
    splits = cyc_cuts = 0
    for rp, col, w, a0 in ring_graphs(150):
        g = oracle.Graph(rp, col, w)
        A = bf.dense(rp, col, w)
        a1, s1 = oracle.positive(g, a0)
        a2, s2 = bf.positive(A, list(a0))
        assert list(a1) == a2 and s1 == s2
        splits += s1
        cyc_cuts += int(s1 > 0)
    assert splits > 40 and cyc_cuts > 30  # the fixture really exercises splits


def test_maximal_rounds_on_rings_match_bruteforce():
    valid = 0
    for idx, (rp, col, w, a0) in enumerate(ring_graphs(40, seed0=7000)):
        g = oracle.Graph(rp, col, w)
        A = bf.dense(rp, col, w)
        # start from single-node communities and pairs to get many candidates
        a = np.arange(g.n, dtype=np.int32)
        a[::3] = a0[::3]
        for rnd in range(4):
            a1, v1, _ = oracle.maximal_round(g, a, idx, 0, rnd, 1 << 31)
            a2, v2 = bf.maximal_round(A, list(a), lambda i: oracle.draw(idx, 0, rnd, i), 1 << 31)
            assert v1 == v2 and list(a1) == a2
            valid += v1
            a = a1
    assert valid > 40


def test_unit_weight_ties_match_bruteforce():
    """Unit weights make exact ties and zero gains common: the strict tests
    (pair > 0, join > stay, move > 0, g < 0) and the tie rules get checked."""
    valid = 0
    for s in range(150):
        rg = np.random.default_rng(20000 + s)
        n = int(rg.integers(3, 10))
        rp, col, w = gg.random_sparse(n, int(rg.integers(n, 3 * n)), 1, 20000 + s)
        g = oracle.Graph(rp, col, w)
        A = bf.dense(rp, col, w)
        a = np.arange(n, dtype=np.int32)
        for rnd in range(3):
            a1, v1, _ = oracle.maximal_round(g, a, s, 2, rnd, 1 << 32)
            a2, v2 = bf.maximal_round(A, list(a), lambda i: oracle.draw(s, 2, rnd, i), 1 << 32)
            assert v1 == v2 and list(a1) == a2
            valid += v1
            a = a1
    assert valid > 100
