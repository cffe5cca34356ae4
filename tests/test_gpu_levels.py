"""Parity of every step on the real states of every level: the oracle walks
Algorithm 1 (contracted graphs with self-loops included) and each GPU step
is fed the oracle's state and compared with the oracle's result."""
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


def _t(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def _np(t):
    return t.cpu().numpy()


def walk(slm, rp, col, w, seed, tag):
    level = 0
    while True:
        g_or = oracle.Graph(rp, col, w)
        if g_or.m2 == 0:
            return
        with slm.Graph(rp, col, w) as g:
            a0 = oracle.assign(g_or)
            say(tag, "level", level, "assign")
            assert np.array_equal(_np(g.assign()), a0)
            a1, s1 = oracle.positive(g_or, a0)
            ga, gs = g.positive(_t(a0))
            assert np.array_equal(_np(ga), a1) and gs == s1, (tag, level, "positive")
            a = a1
            for r in range(64):
                a_next, valid, st, rep = oracle.maximal_round(g_or, a, seed, level, r,
                                                             with_repointed=True)
                say(tag, "level", level, "round", r, st)
                if valid:
                    exp, sp = oracle.positive(g_or, rep)
                    got, gsp = g.positive(_t(rep))
                    assert np.array_equal(_np(got), exp) and gsp == sp, (tag, level, r, "positive")
                got, gst = g.round(_t(a), slm.params(seed=seed), level, r)
                assert gst["valid"] == valid and gst["accepted"] == st["accepted"]
                assert np.array_equal(_np(got), a_next), (tag, level, r, "round")
                a = a_next
                if valid == 0:
                    break
            lab, nc, _ = oracle.components(a)
            if nc == g_or.n:
                return
            rp, col, w = oracle.contract(g_or, lab, nc)
            level += 1


@pytest.mark.parametrize("name", sorted(small_graphs()))
@pytest.mark.parametrize("seed", [1, 2])
def test_levels(slm, name, seed):
    rp, col, w = small_graphs()[name]
    walk(slm, rp, col, w, seed, name)


@pytest.mark.parametrize("seed", [3, 4])
def test_levels_sbm4096(slm, seed):
    walk(slm, *gg.config_graph("sbm4096"), seed, "sbm4096")
