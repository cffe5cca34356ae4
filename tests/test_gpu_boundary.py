"""The C-ABI boundary on the GPU: device memory from the caller's allocator
(and allocation failures), the one-shot batched run, and the server's
cancellation, queue cap and failed-lane paths.  Every result that is
returned is compared with the oracle run of the same graph alone."""
import threading
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


class Counting:
    """An allocator over torch's caching allocator that counts live buffers
    and refuses every allocation once `fail_after` have been made, or while
    `refuse` is set."""

    def __init__(self, slm, fail_after=None):
        import torch
        self.torch = torch
        self.live = {}
        self.calls = 0
        self.fail_after = fail_after
        self.refuse = False
        self.lock = threading.Lock()
        self.a = slm.Allocator(self._alloc, self._free)

    def _alloc(self, nbytes, stream):
        with self.lock:
            if self.refuse or (self.fail_after is not None and self.calls >= self.fail_after):
                return 0
            self.calls += 1
        p = self.torch.cuda.caching_allocator_alloc(nbytes, None, stream)
        with self.lock:
            self.live[p] = nbytes
        return p

    def _free(self, p, stream):
        with self.lock:
            assert p in self.live, "free of an address the allocator never gave"
            del self.live[p]
        self.torch.cuda.caching_allocator_delete(p)


def test_allocator_serves_every_buffer(slm):
    """With the caller's allocator every device buffer comes from it and
    goes back to it; the results equal the oracle's and hipMalloc's."""
    graphs = small_graphs()
    for name in ("star5000", "sbm1000", "mixed_hub"):
        rp, col, w = graphs[name]
        say("allocator", name)
        ca = Counting(slm)
        with slm.Graph(rp, col, w, allocator=ca.a) as g:
            assert ca.calls > 10 and ca.live
            res = g.run(slm.params(seed=3))
        assert not ca.live, "buffers left after destroy"
        with slm.Graph(rp, col, w, allocator=None) as g:
            res2 = g.run(slm.params(seed=3))
        ref = oracle.run(rp, col, w, seed=3)
        _compare(res, ref, name)
        _compare(res2, ref, name)


@pytest.mark.parametrize("fail_after", [0, 1, 7, 30, 60, 90])
def test_allocation_failure_gives_nomem_and_frees(slm, fail_after):
    """An allocator that returns NULL makes creation fail with SLM_E_NOMEM
    and nothing stays allocated; a handle that did get created runs on."""
    rp, col, w = small_graphs()["star5000"]
    ca = Counting(slm, fail_after=fail_after)
    say("allocation failure after", fail_after)
    try:
        with slm.Graph(rp, col, w, allocator=ca.a) as g:
            created = True
            try:
                res = g.run(slm.params(seed=2))
                _compare(res, oracle.run(rp, col, w, seed=2), fail_after)
            except slm.SlmError as e:
                assert e.status == slm.SLM_E_NOMEM
    except slm.SlmError as e:
        created = False
        assert e.status == slm.SLM_E_NOMEM and "allocation" in str(e)
    assert not ca.live, "buffers left after a failed creation"
    if fail_after <= 7:
        assert not created


def test_batch_solve_matches_alone(slm):
    graphs = gg.sbm_batch(12, 50, 3000, 91)
    graphs.insert(3, (np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32)))
    seeds = [5 * i + 1 for i in range(len(graphs))]
    ca = Counting(slm)
    res = slm.batch_solve(graphs, slm.params(), seeds=seeds, allocator=ca.a)
    assert not ca.live
    for i, g in enumerate(graphs):
        _compare(res[i], oracle.run(*g, seed=seeds[i]), i)


def _long_graph():
    """A graph of 60,000 nodes in planted blocks of 200 (about 30 internal
    and 1.2 external neighbours per node): its level 0 lasts tens of
    milliseconds on the GPU, and its run converges in a few levels."""
    return gg.sbm(60000, 200, 0.15, 0.00002, 17)


def test_cancel_queued_and_resident(slm):
    """A queued request is dropped at once, a resident one leaves at the end
    of its level; both report SLM_E_CANCELLED once; the requests around
    them still give the oracle's results."""
    big = _long_graph()
    small = gg.sbm_batch(4, 100, 800, 55)
    with slm.Server(lanes=1, max_members=1, node_capacity=1 << 17,
                    entry_capacity=1 << 23) as sv:
        say("cancel: submitting")
        t_res = sv.submit(*big, seed=1)       # admitted at once, then resident
        t_q = sv.submit(*small[0], seed=2)    # waits: one member per lane
        t_ok = [sv.submit(*g, seed=10 + i) for i, g in enumerate(small[1:])]
        time.sleep(0.005)
        sv.cancel(t_q)
        sv.cancel(t_res)
        with pytest.raises(slm.SlmError) as e:
            sv.wait(t_q)
        assert e.value.status == slm.SLM_E_CANCELLED
        with pytest.raises(slm.SlmError) as e:
            sv.wait(t_res)
        assert e.value.status == slm.SLM_E_CANCELLED
        # delivered once: the ticket is now unknown
        with pytest.raises(slm.SlmError) as e:
            sv.poll(t_res)
        assert e.value.status == slm.SLM_E_INVALID
        say("cancel: both cancelled")
        res = [sv.wait(t) for t in t_ok]
        # a finished, undelivered result can be cancelled too
        t_done = sv.submit(*small[1], seed=99)
        while sv.stats()["completed"] < 4:
            time.sleep(0.002)
        sv.cancel(t_done)
        with pytest.raises(slm.SlmError) as e:
            sv.wait(t_done)
        assert e.value.status == slm.SLM_E_CANCELLED
    for i, g in enumerate(small[1:]):
        _compare(res[i], oracle.run(*g, seed=10 + i), i)


def test_queue_cap_gives_busy(slm):
    big = _long_graph()
    small = gg.sbm_batch(6, 100, 800, 56)
    with slm.Server(lanes=1, max_members=1, node_capacity=1 << 17, entry_capacity=1 << 23,
                    queue_cap=2) as sv:
        accepted, busy = [], 0
        accepted.append((sv.submit(*big, seed=1), big, 1))
        for i, g in enumerate(small):
            try:
                accepted.append((sv.submit(*g, seed=20 + i), g, 20 + i))
            except slm.SlmError as e:
                assert e.status == slm.SLM_E_BUSY
                busy += 1
        say("queue cap:", len(accepted), "accepted,", busy, "busy")
        assert busy >= 3  # at most two wait behind the resident graph
        res = []
        for t, g, sd in accepted:
            res.append((sv.wait(t), g, sd))
            say("queue cap: request with seed", sd, "done")
        # once the queue drains, submissions are accepted again
        t = sv.submit(*small[-1], seed=77)
        last = sv.wait(t)
    for r, g, s in res:
        _compare(r, oracle.run(*g, seed=s), s)
    _compare(last, oracle.run(*small[-1], seed=77), 77)


@pytest.mark.timeout(120)
def test_failed_lane_fails_later_submissions(slm):
    """When the only lane of a class fails (here its allocator refuses the
    hub buffers of a star graph), its tickets report SLM_E_DEVICE and later
    submissions to that class fail at once instead of waiting forever."""
    ca = Counting(slm)
    star = gg.star(5000)
    sv = slm.Server(lanes=1, node_capacity=1 << 14, entry_capacity=1 << 16, max_members=8,
                    allocator=ca.a)
    try:
        ca.refuse = True
        t = sv.submit(*star, seed=1)
        with pytest.raises(slm.SlmError) as e:
            sv.wait(t)
        assert e.value.status == slm.SLM_E_DEVICE
        with pytest.raises(slm.SlmError) as e:
            sv.submit(*gg.path(10), seed=2)
        assert e.value.status == slm.SLM_E_DEVICE
    finally:
        ca.refuse = False
        sv.close()
    assert not ca.live
