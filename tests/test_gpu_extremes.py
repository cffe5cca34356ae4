"""Graphs at the edge of the integer bound: M2 = 2^31 - 1 exactly, strengths
near 2^30, so every key M2*A - k_i*k_j (and the split and move keys) is a
product difference near 2^61.  Whole runs and the sweep on singleton labels
must still equal the oracle bit for bit."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_common import say

pytestmark = pytest.mark.gpu

BOUND = 2**31 - 1


@pytest.fixture(scope="module")
def slm():
    import torch
    assert torch.cuda.is_available()
    import paper_1702_04645_amd as slm
    slm.lib()
    return slm


def _fill_to_bound(n, u, v, wt):
    """Adds weight to the pair (u[0], v[0]) and a loop so that M2 is BOUND."""
    base = 2 * int(wt[u != v].sum()) + int(wt[u == v].sum())
    extra = BOUND - base
    assert extra >= 2
    wt = wt.copy()
    wt[0] += extra // 2  # off-diagonal: counts twice
    u2, v2, w2 = u, v, wt
    if extra % 2:
        u2 = np.append(u, n - 1)
        v2 = np.append(v, n - 1)
        w2 = np.append(wt, 1)
    rp, col, w = gg.csr_from_pairs(n, u2, v2, w2)
    assert int(w.astype(np.int64).sum()) == BOUND
    return rp, col, w


def graphs():
    out = {}
    rg = np.random.default_rng(11)
    # one heavy edge carrying almost all the weight
    n, m = 2000, 8000
    u = rg.integers(0, n, m)
    v = rg.integers(0, n, m)
    keep = u != v
    u, v = u[keep], v[keep]
    u[0], v[0] = 0, 1
    out["heavy_edge"] = _fill_to_bound(n, u, v, rg.integers(1, 50, u.size))
    # every weight large
    n, m = 300, 1500
    u = rg.integers(0, n, m)
    v = rg.integers(0, n, m)
    keep = u != v
    u, v = u[keep], v[keep]
    cap = BOUND // (2 * u.size) - 64
    out["heavy_all"] = _fill_to_bound(n, u, v, rg.integers(cap // 2, cap, u.size))
    # a hub row (> 4096 entries) whose strength is about 2^30
    n = 5001
    u = np.zeros(n - 1, np.int64)
    v = np.arange(1, n)
    cap = BOUND // (2 * (n - 1)) - 64
    out["heavy_hub"] = _fill_to_bound(n, u, v, rg.integers(cap // 2, cap, n - 1))
    return out


GRAPHS = graphs()


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("seed", [1, 5])
def test_run_at_the_bound(slm, name, seed):
    rp, col, w = GRAPHS[name]
    say("extreme run", name, seed)
    res_o = oracle.run(rp, col, w, seed=seed)
    with slm.Graph(rp, col, w) as g:
        assert g.level_info()["m2"] == BOUND
        res = g.run(slm.params(seed=seed))
    assert len(res) == len(res_o)
    for a, b in zip(res, res_o):
        assert (a.n_c, a.nq, a.q, a.rounds, a.converged) == \
            (b["n_c"], b["nq"], b["q"], b["rounds"], b["converged"])
        assert np.array_equal(a.labels, b["labels"])


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_steps_at_the_bound(slm, name):
    import torch
    rp, col, w = GRAPHS[name]
    say("extreme steps", name)
    g_or = oracle.Graph(rp, col, w)
    n = rp.size - 1
    a0 = oracle.assign(g_or)
    a1, s1 = oracle.positive(g_or, a0)
    lab0 = np.arange(n, dtype=np.int32)
    b_o, d_o, w_o = oracle.sweep(g_or, lab0, n)
    with slm.Graph(rp, col, w) as g:
        assert np.array_equal(g.assign().cpu().numpy(), a0)
        a1g, s1g = g.positive(torch.from_numpy(a0).cuda())
        assert s1g == s1 and np.array_equal(a1g.cpu().numpy(), a1)
        b, d, o = g.sweep(torch.from_numpy(lab0).cuda(), n)
        assert np.array_equal(b.cpu().numpy(), b_o)
        assert np.array_equal(d.cpu().numpy(), d_o)
        assert np.array_equal(o.cpu().numpy(), w_o)
        nq, q = g.modularity(torch.from_numpy(lab0).cuda(), n)
        assert nq == oracle.modularity_num(g_or, lab0, n)
