"""The serving loop against the oracle: requests submitted while others run
are admitted at level boundaries as capacity frees up, share every launch
with the graphs resident at that time, and still give exactly the levels the
oracle gives for each graph alone with its seed."""
import time

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
        assert (a.n_c, a.nq, a.q, a.rounds, a.converged) == \
            (b["n_c"], b["nq"], b["q"], b["rounds"], b["converged"]), t
        assert np.array_equal(a.labels, b["labels"]), t


def _mix():
    g = small_graphs()
    out = [g[k] for k in sorted(g)]
    out += gg.sbm_batch(24, 40, 4000, 777)
    out.insert(4, (np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32)))
    out.insert(9, (np.zeros(4, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32)))
    return out


@pytest.mark.parametrize("lanes,large", [(1, 0), (2, 1), (4, 1)])
def test_serve_mix_matches_alone(slm, lanes, large):
    graphs = _mix()
    seeds = [1000 + 17 * i for i in range(len(graphs))]
    rg = np.random.default_rng(5)
    say("serve mix", len(graphs), "lanes", lanes, large)
    with slm.Server(lanes=lanes, large_lanes=large, large_nodes=3000, node_capacity=1 << 16,
                    entry_capacity=1 << 20, max_members=64) as sv:
        tickets = []
        for i, (rp, col, w) in enumerate(graphs):
            tickets.append(sv.submit(rp, col, w, seed=seeds[i]))
            time.sleep(float(rg.uniform(0, 0.004)))  # arrivals overlap running levels
        res = [sv.wait(t) for t in tickets]
        st = sv.stats()
    assert st["submitted"] == st["completed"] == len(graphs)
    for i, (rp, col, w) in enumerate(graphs):
        _compare(res[i], oracle.run(rp, col, w, seed=seeds[i]), i)


def test_serve_capacity_admission(slm):
    """A lane smaller than the queue: requests wait for capacity, results are
    unchanged, a graph that can never fit is refused at submission."""
    graphs = gg.sbm_batch(10, 200, 2500, 31)
    seeds = [7 * i + 3 for i in range(len(graphs))]
    cap = max(rp.size - 1 for rp, _, _ in graphs) + 10
    say("serve capacity", cap)
    with slm.Server(node_capacity=cap, entry_capacity=1 << 22, max_members=3) as sv:
        tickets = [sv.submit(*g, seed=seeds[i]) for i, g in enumerate(graphs)]
        big = gg.path(cap + 5)
        with pytest.raises(slm.SlmError):
            sv.submit(*big, seed=1)
        # poll until every result is in; each ticket is delivered once
        res = {}
        deadline = time.time() + 60
        while len(res) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t not in res:
                    r = sv.poll(t)
                    if r is not None:
                        res[t] = r
            time.sleep(0.002)
        assert len(res) == len(tickets)
        with pytest.raises(slm.SlmError):
            sv.poll(tickets[0])
    for i, g in enumerate(graphs):
        _compare(res[tickets[i]], oracle.run(*g, seed=seeds[i]), i)


def test_serve_parameters(slm):
    graphs = gg.sbm_batch(6, 100, 1500, 41)
    p = slm.params(accept_p=1 << 30, max_rounds=3, max_levels=2)
    with slm.Server(p=p) as sv:
        tickets = [sv.submit(*g, seed=i + 1) for i, g in enumerate(graphs)]
        res = [sv.wait(t) for t in tickets]
    for i, g in enumerate(graphs):
        _compare(res[i], oracle.run(*g, seed=i + 1, accept_p=1 << 30, max_rounds=3,
                                    max_levels=2), i)


@pytest.mark.timeout(600)
def test_serve_mix_with_rmat20(slm):
    """Four lanes, one of them for large graphs: the R-MAT scale-20 graph
    (seed 1) served among small graphs arriving before, during and after it.
    The R-MAT result equals the stored oracle run (every level's n_c, N_Q,
    rounds, convergence and the SHA-256 of the composed labels); every small
    result equals its oracle run alone."""
    import hashlib
    from test_gpu_rmat20_rounds import golden_levels
    lv = golden_levels()
    from gpu_common import config_graph
    rmat = config_graph("rmat20")
    small = _mix() + gg.sbm_batch(40, 64, 20000, 778)
    seeds = [3000 + 11 * i for i in range(len(small))]
    rg = np.random.default_rng(9)
    say("serve mix with R-MAT-20:", len(small), "small graphs")
    with slm.Server(lanes=4, large_lanes=1, large_nodes=200_000, node_capacity=1 << 21,
                    entry_capacity=1 << 26, max_members=256, validate=False) as sv:
        tickets = []
        for i in range(len(small) // 3):
            tickets.append(sv.submit(*small[i], seed=seeds[i]))
        t_rmat = sv.submit(*rmat, seed=1)
        for i in range(len(small) // 3, len(small)):
            tickets.append(sv.submit(*small[i], seed=seeds[i]))
            time.sleep(float(rg.uniform(0, 0.05)))  # arrivals during the R-MAT levels
        res = [sv.wait(t) for t in tickets]
        say("small graphs done")
        r_rmat = sv.wait(t_rmat)
        say("R-MAT done")
    assert len(r_rmat) == len(lv)
    for i, (r, (nc, nq, q, rounds, conv, h)) in enumerate(zip(r_rmat, lv)):
        assert (r.n_c, r.nq, r.rounds, bool(r.converged)) == (nc, nq, rounds, conv), i
        assert abs(r.q - q) <= 1e-12
        lab = np.ascontiguousarray(r.labels, dtype=np.int32)
        assert hashlib.sha256(lab.tobytes()).hexdigest() == h, "level %d labels differ" % i
    for i, g in enumerate(small):
        _compare(res[i], oracle.run(*g, seed=seeds[i]), i)
