"""Batched execution against the oracle: every graph of a batch, run
together with the others in one disjoint union, gives exactly the levels
the oracle gives for that graph alone (labels, n_c, N_Q, Q, rounds,
converged), and the single steps on the level-0 union equal the oracle's
steps on each member, offset to union numbering."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_common import say, small_graphs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slm():
    import torch
    assert torch.cuda.is_available()
    import paper_1702_04645_amd as slm
    slm.lib()
    return slm


def _compare(res_g, res_o, tag):
    assert len(res_g) == len(res_o), tag
    for lv, (a, b) in enumerate(zip(res_g, res_o)):
        t = (tag, lv)
        assert a.n_c == b["n_c"], t
        assert a.nq == b["nq"], t
        assert a.q == b["q"], t
        assert a.rounds == b["rounds"], t
        assert a.converged == b["converged"], t
        assert np.array_equal(a.labels, b["labels"]), t


def _mixed_members():
    """Small graphs of every shape, plus degenerate members: an empty graph,
    a graph without edges, a single node, and one with a self-loop only."""
    g = small_graphs()
    out = [g[k] for k in sorted(g)]
    out.insert(3, (np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32)))
    out.insert(5, (np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32)))
    out.append(gg.path(2))
    out.append((np.array([0, 1], np.int64), np.array([0], np.int32), np.array([3], np.int32)))
    out.append(gg.cliques([4, 4, 6]))
    return out


def test_batch_mixed_members(slm):
    members = _mixed_members()
    seeds = [11 + 7 * i for i in range(len(members))]
    say("batch mixed", len(members))
    with slm.Batch(members) as b:
        res = b.run(slm.params(), seeds=seeds)
        for i, (rp, col, w) in enumerate(members):
            _compare(res[i], oracle.run(rp, col, w, seed=seeds[i]), i)
        # a second run on the same handle is identical
        res2 = b.run(slm.params(), seeds=seeds)
        for i in range(len(members)):
            _compare(res2[i], oracle.run(*members[i], seed=seeds[i]), ("again", i))


@pytest.mark.parametrize("rounds,levels", [(64, 0), (5, 0), (64, 2)])
def test_batch_union_shrinks(slm, rounds, levels):
    """With no size floor the union shrinks to its members that still move
    after every round that lets it (several times at level 0, once per later
    level): each member still equals its oracle run alone."""
    members = _mixed_members() + gg.sbm_batch(24, 64, 4096, 77)
    seeds = [3 + 5 * i for i in range(len(members))]
    p = slm.params(max_rounds=rounds, max_levels=levels)
    say("batch shrink", len(members), rounds, levels)
    with slm.Batch(members) as b:
        b.set_option("union_shrink_min_nodes", 0)
        for rep in range(2):
            res = b.run(p, seeds=seeds)
            for i, (rp, col, w) in enumerate(members):
                _compare(res[i], oracle.run(rp, col, w, seed=seeds[i], max_rounds=rounds,
                                            max_levels=levels), (rep, i))


def test_union_shrink_option(slm):
    rp, col, w = gg.sbm(200, 10, 0.3, 0.02, 3)
    with slm.Graph(rp, col, w) as g:
        with pytest.raises(slm.SlmError) as e:
            g.set_option("union_shrink_min_nodes", 0)
        assert e.value.status == slm.SLM_E_INVALID
    with slm.Batch([(rp, col, w)] * 3) as b:
        b.set_option("union_shrink_min_nodes", -1)
        res = b.run(slm.params(seed=2))
    for i in range(3):
        _compare(res[i], oracle.run(rp, col, w, seed=2), i)


@pytest.mark.parametrize("acc,rounds,levels", [(1 << 32, 64, 0), (1 << 31, 2, 0),
                                               (1 << 31, 64, 1), (1 << 30, 3, 2)])
def test_batch_parameters(slm, acc, rounds, levels):
    members = gg.sbm_batch(12, 40, 3000, 321)
    say("batch params", acc, rounds, levels)
    with slm.Batch(members) as b:
        res = b.run(slm.params(seed=5, accept_p=acc, max_rounds=rounds, max_levels=levels))
    for i, (rp, col, w) in enumerate(members):
        _compare(res[i], oracle.run(rp, col, w, seed=5, accept_p=acc, max_rounds=rounds,
                                    max_levels=levels), i)


def test_batch_sbm_distribution(slm):
    """48 members of the planted-partition batch family (log-uniform node
    counts 64..8192, blocks 16..256, p_in 0.2, mean external degree 2)."""
    members = gg.sbm_batch(48, 64, 8192, gg.CONFIG_SEEDS["batch2048"])
    seeds = [gg.batch_member_seed(99, i) for i in range(len(members))]
    say("batch sbm", sum(m[1].size for m in members))
    with slm.Batch(members, validate=False) as b:
        res = b.run(slm.params(), seeds=seeds)
    for i, (rp, col, w) in enumerate(members):
        _compare(res[i], oracle.run(rp, col, w, seed=seeds[i]), i)


def _union_offsets(members):
    base = np.concatenate([[0], np.cumsum([m[0].size - 1 for m in members])])
    return base


def test_batch_steps_on_union(slm):
    """ASSIGN, COMPONENTS and the sweep on the level-0 union equal the
    oracle's on each member (nodes and labels offset into the union)."""
    import torch
    members = [m for m in _mixed_members() if m[0].size > 1]
    base = _union_offsets(members)
    say("batch steps", len(members))
    with slm.Batch(members) as b:
        a = b.assign().cpu().numpy()
        exp_a, exp_lab, exp_best, exp_delta, exp_wown = [], [], [], [], []
        cb = 0
        for i, (rp, col, w) in enumerate(members):
            g = oracle.Graph(rp, col, w)
            ai = oracle.assign(g)
            exp_a.append(ai + base[i])
            a1, _ = oracle.positive(g, ai)
            lab, nc, _ = oracle.components(a1)
            best, delta, wown = oracle.sweep(g, lab, nc)
            exp_lab.append(lab + cb)
            exp_best.append(best + cb)
            exp_delta.append(delta)
            exp_wown.append(wown)
            cb += nc
        assert np.array_equal(a, np.concatenate(exp_a))
        lab_u = np.concatenate(exp_lab).astype(np.int32)
        # components of the union assignment: labels offset per member
        lab_g, nc_g, _ = b.components(torch.from_numpy(np.concatenate(exp_a).astype(np.int32)).cuda())
        exp_lab0 = []
        cb0 = 0
        for i, (rp, col, w) in enumerate(members):
            l0, n0c, _ = oracle.components(exp_a[i] - base[i])
            exp_lab0.append(l0 + cb0)
            cb0 += n0c
        assert nc_g == cb0
        assert np.array_equal(lab_g.cpu().numpy(), np.concatenate(exp_lab0))
        best, delta, wown = b.sweep(torch.from_numpy(lab_u).cuda(), cb)
        assert np.array_equal(best.cpu().numpy(), np.concatenate(exp_best))
        assert np.array_equal(delta.cpu().numpy(), np.concatenate(exp_delta))
        assert np.array_equal(wown.cpu().numpy(), np.concatenate(exp_wown))


def test_batch_rejects_plain_calls(slm):
    members = [gg.path(5), gg.path(7)]
    with slm.Batch(members) as b:
        with pytest.raises(slm.SlmError):
            b.contract(__import__("torch").zeros(12, dtype=__import__("torch").int32).cuda(), 1)
        with pytest.raises(slm.SlmError):
            slm.Graph.run(b)
