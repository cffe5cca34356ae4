"""Parity of the GPU path under the directed model (Sec. 2.4 with out- and
in-strengths, resolution num/den) with the oracle's directed run: the GPU
takes the directed CSR W, builds S = W + W^T and the strengths itself, and
every level's labels, n_c, N_Q, rounds and convergence flag equal the
oracle's; the steps (ASSIGN, POSITIVE, sweep, modularity, rounds) match
element by element; a symmetric W gives the undirected run with N_Q x4."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_common import say, small_graphs

pytestmark = pytest.mark.gpu


def directed_graphs():
    out = {}
    for name, (rp, col, w) in small_graphs().items():
        out["dir_" + name] = gg.orient(rp, col, w, 17 + len(name), both=0.3,
                                       w_max=0 if name.startswith("star") else 6)
    for s in range(4):
        rg = np.random.default_rng(900 + s)
        n = int(rg.integers(5, 400))
        out["rand%d" % s] = gg.random_directed(n, int(rg.integers(n, 5 * n)), 9, 900 + s,
                                               loops=(s % 2 == 0))
    # a node with 6000 arcs out and 3000 in: a hub row of S
    n = 9000
    hv = np.arange(1, 6001)
    iv = np.arange(3001, 6001)
    out["hub_out_in"] = gg.csr_from_pairs(
        n, np.r_[np.zeros(hv.size, np.int64), iv, np.arange(1, n - 1)],
        np.r_[hv, np.zeros(iv.size, np.int64), np.arange(2, n)],
        np.r_[np.ones(hv.size), 2 * np.ones(iv.size), np.ones(n - 2)], symmetrise=False)
    return out


GRAPHS = directed_graphs()
NAMES = sorted(GRAPHS)


@pytest.fixture(scope="module")
def slm():
    import torch
    assert torch.cuda.is_available()
    import paper_1702_04645_amd as slm
    slm.lib()
    return slm


def _t(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("numden", [(1, 1), (1, 2), (3, 2)], ids=["g1", "g1-2", "g3-2"])
@pytest.mark.parametrize("name", NAMES)
def test_directed_run(slm, name, numden):
    num, den = numden
    rp, col, w = GRAPHS[name]
    say("directed run", name, numden)
    ref = oracle.run_null(rp, col, w, oracle.DIRECTED, num, den, seed=4)
    with slm.Graph(rp, col, w, model=slm.model(slm.MODEL_DIRECTED, num, den)) as g:
        res = g.run(slm.params(seed=4))
    assert len(res) == len(ref)
    for a, b in zip(res, ref):
        assert a.n_c == b["n_c"] and a.nq == b["nq"] and a.q == b["q"]
        assert a.rounds == b["rounds"] and a.converged == b["converged"]
        assert np.array_equal(a.labels, b["labels"])


@pytest.mark.parametrize("name", ["dir_rmat12", "dir_mixed_hub", "dir_sbm1000", "hub_out_in",
                                  "rand1", "dir_path200"])
def test_directed_steps(slm, name):
    rp, col, w = GRAPHS[name]
    say("directed steps", name)
    go = oracle.NullGraph(rp, col, w, oracle.DIRECTED, 1, 1)
    with slm.Graph(rp, col, w, model=slm.model(slm.MODEL_DIRECTED, 1, 1)) as g:
        info = g.level_info()
        assert info["m2"] == go.m2 and info["nnz"] == go.col.size
        rp_s, col_s, w_s = g.export_level()
        assert np.array_equal(rp_s, go.rp) and np.array_equal(col_s, go.col)
        assert np.array_equal(w_s, go.w)
        a_o = oracle.assign_nm(go)
        assert np.array_equal(_np(g.assign()), a_o)
        a1_o, s_o = oracle.positive_nm(go, a_o)
        a1_g, s_g = g.positive(_t(a_o))
        assert s_g == s_o and np.array_equal(_np(a1_g), a1_o)
        lab, nc, _ = oracle.components(a1_o)
        b_o, d_o, w_o = oracle.sweep_nm(go, lab, nc)
        b, d, wo = g.sweep(_t(lab), nc)
        assert np.array_equal(_np(b), b_o) and np.array_equal(_np(d), d_o)
        assert np.array_equal(_np(wo), w_o)
        nq, _ = g.modularity(_t(lab), nc)
        assert nq == oracle.modularity_num_nm(go, lab, nc)
        a_cur = a1_o
        for rnd in range(4):
            a_o2, v_o, st_o = oracle.maximal_round_nm(go, a_cur, 9, 0, rnd)
            a_g2, st_g = g.round(_t(a_cur), slm.params(seed=9), 0, rnd)
            assert st_g["valid"] == v_o and st_g["accepted"] == st_o["accepted"]
            assert st_g["splits"] == st_o["splits"]
            assert np.array_equal(_np(a_g2), a_o2)
            a_cur = a_o2


def _ring_assignments(count, seed0):
    """Directed graphs with a given assignment: a ring over L nodes and the
    others hung below random neighbours (POSITIVE's branch and cycle cuts)."""
    out = []
    for s in range(count):
        rg = np.random.default_rng(seed0 + s)
        n = int(rg.integers(6, 60))
        L = int(rg.integers(2, min(n, 12) + 1))
        u = np.arange(L)
        extra = int(rg.integers(n, 4 * n))
        cu, cv = rg.integers(0, n, extra), rg.integers(0, n, extra)
        uu = np.r_[u, cu]
        vv = np.r_[(u + 1) % L, cv]
        wt = np.r_[rg.integers(1, 4, L), rg.integers(1, 9, extra)]
        keep = uu != vv
        rp, col, w = gg.csr_from_pairs(n, uu[keep], vv[keep], wt[keep], symmetrise=False)
        S = np.zeros((n, n), np.int64)
        for i in range(n):
            S[i, col[rp[i]:rp[i + 1]]] = 1
        S = S + S.T
        a0 = np.arange(n, dtype=np.int32)
        a0[:L] = (u + 1) % L
        for i in range(L, n):
            nb = [j for j in range(i) if S[i, j] > 0]
            if nb:
                a0[i] = nb[int(rg.integers(0, len(nb)))]
        out.append((rp, col, w, a0))
    return out


def test_directed_positive_on_given_assignments(slm):
    for idx, (rp, col, w, a0) in enumerate(_ring_assignments(60, 4400)):
        go = oracle.NullGraph(rp, col, w, oracle.DIRECTED, 1, 1)
        a_o, s_o = oracle.positive_nm(go, a0)
        with slm.Graph(rp, col, w, model=slm.model(slm.MODEL_DIRECTED, 1, 1)) as g:
            a_g, s_g = g.positive(_t(a0))
        assert s_g == s_o, idx
        assert np.array_equal(_np(a_g), a_o), idx


def test_symmetric_input_is_the_undirected_run(slm):
    rp, col, w = small_graphs()["sbm1000"]
    with slm.Graph(rp, col, w) as g:
        ref = g.run(slm.params(seed=2))
    with slm.Graph(rp, col, w, model=slm.model(slm.MODEL_DIRECTED, 1, 1)) as g:
        res = g.run(slm.params(seed=2))
    assert len(res) == len(ref)
    for a, b in zip(res, ref):
        assert a.n_c == b.n_c and a.nq == 4 * b.nq and a.q == b.q
        assert np.array_equal(a.labels, b.labels)
