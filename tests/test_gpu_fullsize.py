"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times.

R-MAT scale 20 and the LFR-style 4M-node graph: ASSIGN, POSITIVE, the
sweep, the modularity numerator and the contraction are compared with the
oracle element by element on the whole graph.  Whole runs are checked by
properties that hold at any size (N_Q of every emitted level equals the
oracle's modularity of the GPU labels on the original graph, canonical
labels, Q non-decreasing, no negative local gain after the first level).
The 2048-graph batch runs whole on the GPU; every member's levels are
compared with the stored oracle runs of each member alone, and a spread
sample with oracle runs made in the test."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_common import config_graph, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slm():
    import torch
    assert torch.cuda.is_available()
    import paper_1702_04645_amd as slm
    slm.lib()
    return slm


def graph(name):
    return config_graph(name)


def _canonical(lab):
    """Labels numbered in order of first occurrence (smallest member)."""
    _, first = np.unique(lab, return_index=True)
    return np.array_equal(np.sort(first), first) and (lab.size == 0 or lab.min() == 0)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["rmat20", "lfr4m"])
def test_fullsize_steps(slm, name):
    import torch
    rp, col, w = graph(name)
    say(name, "oracle steps", col.size)
    g = oracle.Graph(rp, col, w)
    a0 = oracle.assign(g)
    lab0, nc0, _ = oracle.components(a0)
    best, delta, wown = oracle.sweep(g, lab0, nc0)
    nq0 = oracle.modularity_num(g, lab0, nc0)
    crp, ccol, cw = oracle.contract(g, lab0, nc0)
    say(name, "gpu steps")
    with slm.Graph(rp, col, w, validate=False) as G:
        assert G.level_info()["m2"] == g.m2
        a = G.assign()
        assert np.array_equal(a.cpu().numpy(), a0)
        lab, nc, cyc = G.components(a)
        assert nc == nc0 and np.array_equal(lab.cpu().numpy(), lab0)
        labd = torch.from_numpy(lab0).cuda()
        b, d, o = G.sweep(labd, nc0)
        assert np.array_equal(b.cpu().numpy(), best)
        assert np.array_equal(d.cpu().numpy(), delta)
        assert np.array_equal(o.cpu().numpy(), wown)
        nq, q = G.modularity(labd, nc0)
        assert nq == nq0 and q == oracle.modularity(nq0, g.m2)
        G.contract(labd, nc0)
        xrp, xcol, xw = G.export_level()
        assert np.array_equal(xrp, crp)
        assert np.array_equal(xcol, ccol)
        assert np.array_equal(xw, cw)
        G.reset()
        say(name, "oracle positive")
        a1, s1 = oracle.positive(g, a0)
        a1g, s1g = G.positive(torch.from_numpy(a0).cuda())
        assert s1g == s1
        assert np.array_equal(a1g.cpu().numpy(), a1)


def _check_run_properties(rp, col, w, res):
    """Properties of a whole run that hold at any size."""
    g = oracle.Graph(rp, col, w)
    prev_q, prev_nc = None, rp.size - 1
    for lv, r in enumerate(res):
        assert _canonical(r.labels), lv
        assert r.labels.max() + 1 == r.n_c, lv
        assert r.n_c < prev_nc, lv
        # contraction preserves N_Q: the level's N_Q is the modularity of its
        # labels on the original graph
        assert oracle.modularity_num(g, r.labels, r.n_c) == r.nq, lv
        assert r.q == oracle.modularity(r.nq, g.m2), lv
        if prev_q is not None:
            assert r.q >= prev_q, lv
        prev_q, prev_nc = r.q, r.n_c
    if res:
        # POSITIVE ends every level: no node of the first level has a
        # negative local gain
        gain = oracle.local_gain(g, res[0].labels, res[0].n_c)
        assert gain.min() >= 0


@pytest.mark.timeout(600)
def test_fullsize_lfr4m_run(slm):
    rp, col, w = graph("lfr4m")
    say("lfr4m run")
    with slm.Graph(rp, col, w, validate=False) as G:
        res = G.run(slm.params(seed=1))
        res2 = G.run(slm.params(seed=1))
    assert len(res) >= 1
    for a, b in zip(res, res2):
        assert np.array_equal(a.labels, b.labels) and a.nq == b.nq
    say("lfr4m levels", [(r.n_c, r.rounds, r.q) for r in res])
    _check_run_properties(rp, col, w, res)


def _gen_member(args):
    seed, i, count = args
    return gg.sbm_batch(count, 64, 65536, seed, indices=[i])[0]


def batch2048_golden():
    """Per member, the list of its emitted levels (n_c, N_Q, rounds,
    converged, sha256 of the composed labels) from the stored oracle runs
    (tests/golden/make_batch2048_golden.py)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "batch2048_levels.txt")
    out = {}
    for ln in open(path):
        if ln.startswith("#") or not ln.strip():
            continue
        f = ln.split()
        m, lv = int(f[0]), int(f[1])
        out.setdefault(m, [])
        assert len(out[m]) == lv
        out[m].append((int(f[2]), int(f[3]), int(f[4]), bool(int(f[5])), f[6]))
    return out


@pytest.mark.timeout(900)
def test_fullsize_batch2048(slm):
    """The 2048-member planted-partition batch in one batched run: every
    member's every level (n_c, N_Q, Q, rounds, converged, composed labels)
    equals the stored oracle run of that member alone; a spread sample and
    the largest member are also run through the oracle here."""
    import hashlib
    import multiprocessing as mp
    count, seed = 2048, gg.CONFIG_SEEDS["batch2048"]
    say("batch2048 generating")
    with mp.get_context("fork").Pool(8) as pool:
        members = pool.map(_gen_member, [(seed, i, count) for i in range(count)], chunksize=8)
    seeds = [gg.batch_member_seed(1, i) for i in range(count)]
    say("batch2048 gpu run", sum(m[1].size for m in members))
    with slm.Batch(members, validate=False) as b:
        res = b.run(slm.params(), seeds=seeds)
    gold = batch2048_golden()
    say("batch2048 against the stored oracle runs of all members")
    for i in range(count):
        rg, go = res[i], gold[i]
        assert len(rg) == len(go), i
        m2 = int(members[i][2].sum())
        for lv, (x, (nc, nq, rounds, conv, h)) in enumerate(zip(rg, go)):
            assert (x.n_c, x.nq, x.rounds, bool(x.converged)) == (nc, nq, rounds, conv), (i, lv)
            assert x.q == nq / m2 / m2, (i, lv)
            lab = np.ascontiguousarray(x.labels, dtype=np.int32)
            assert hashlib.sha256(lab.tobytes()).hexdigest() == h, (i, lv)
    sizes = np.array([m[0].size - 1 for m in members])
    pick = sorted(set(list(range(0, count, 97)) + [int(np.argmax(sizes))]))
    say("batch2048 oracle on", len(pick), "members")
    for i in pick:
        rp, col, w = members[i]
        ro = oracle.run(rp, col, w, seed=seeds[i])
        rg = res[i]
        assert len(rg) == len(ro), i
        for lv, (x, y) in enumerate(zip(rg, ro)):
            assert (x.n_c, x.nq, x.q, x.rounds, x.converged) == \
                (y["n_c"], y["nq"], y["q"], y["rounds"], y["converged"]), (i, lv)
            assert np.array_equal(x.labels, y["labels"]), (i, lv)
