"""Parity of the GPU classical Louvain (the sequential comparison method of
Sec. 6) with the oracle's: the speculative chunks must reproduce the
sequential result exactly -- every level's labels, n_c, N_Q, passes and
convergence -- on the small fixtures (every degree bin, hubs, loops, deep
paths), on the 2048-member batch family's members, and at full size on
R-MAT scale 16 and the LFR-style 4M graph's first level."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_common import config_graph, say, small_graphs

pytestmark = pytest.mark.gpu

GRAPHS = small_graphs()
NAMES = sorted(GRAPHS)


@pytest.fixture(scope="module")
def slm():
    import torch
    assert torch.cuda.is_available()
    import paper_1702_04645_amd as slm
    slm.lib()
    return slm


def _compare(res, ref):
    assert len(res) == len(ref)
    for a, b in zip(res, ref):
        assert a.n_c == b["n_c"] and a.nq == b["nq"] and a.q == b["q"]
        assert a.rounds == b["rounds"] and a.converged == b["converged"]
        assert np.array_equal(a.labels, b["labels"])


@pytest.mark.parametrize("name", NAMES)
def test_louvain_run_small(slm, name):
    rp, col, w = GRAPHS[name]
    say("louvain", name)
    ref = oracle.louvain_run(rp, col, w)
    with slm.Graph(rp, col, w) as g:
        res = g.louvain_run()
    _compare(res, ref)


def test_louvain_caps(slm):
    rp, col, w = GRAPHS["rmat12"]
    for passes, levels in ((1, 0), (2, 1), (3, 2)):
        ref = oracle.louvain_run(rp, col, w, max_passes=passes, max_levels=levels)
        with slm.Graph(rp, col, w) as g:
            res = g.louvain_run(slm.params(max_rounds=passes, max_levels=levels))
        _compare(res, ref)


def test_louvain_batch_family_members(slm):
    members = gg.sbm_batch(2048, 64, 65536, gg.CONFIG_SEEDS["batch2048"],
                           indices=[0, 3, 700, 1500, 2047])
    for rp, col, w in members:
        say("louvain member", rp.size - 1)
        ref = oracle.louvain_run(rp, col, w)
        with slm.Graph(rp, col, w, validate=False) as g:
            res = g.louvain_run()
        _compare(res, ref)


@pytest.mark.timeout(600)
def test_louvain_fullsize_rmat16(slm):
    rp, col, w = gg.rmat(16, 16, 0.57, 0.19, 0.19, 5)
    ref = oracle.louvain_run(rp, col, w)
    say("rmat16 levels", len(ref))
    with slm.Graph(rp, col, w, validate=False) as g:
        res = g.louvain_run()
    _compare(res, ref)


@pytest.mark.timeout(900)
def test_louvain_fullsize_lfr4m_first_level(slm):
    rp, col, w = config_graph("lfr4m")
    g_or = oracle.Graph(rp, col, w)
    lab_o, nc_o, ps_o, cv_o, mv_o = oracle.louvain_level(g_or)
    say("lfr4m louvain level 0: n_c", nc_o, "passes", ps_o, "moves", mv_o)
    with slm.Graph(rp, col, w, validate=False) as g:
        lab, nc, ps, cv = g.louvain_level()
    assert nc == nc_o and ps == ps_o and cv == cv_o
    assert np.array_equal(lab.cpu().numpy(), lab_o)
