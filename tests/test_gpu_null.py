"""Parity of the GPU path under the null models of Sec. 2.2-2.3 with the
oracle (oracle.run_null and its step functions): the configuration model
with a resolution num/den and the Erdos-Renyi null model p = num/den, on
the small fixtures (every degree bin, hubs, loops) and at full size on the
LFR-style 4M graph (ASSIGN, the first sweep, and one round, element by
element).  Integer results are bit-exact; Q (host double from the exact
N_Q) is bit-identical."""
import numpy as np
import pytest

import oracle
from gpu_common import config_graph, say, small_graphs

pytestmark = pytest.mark.gpu

GRAPHS = small_graphs()
NAMES = sorted(GRAPHS)
MODELS = [("config", oracle.CONFIG, 1, 2), ("config", oracle.CONFIG, 3, 2),
          ("config", oracle.CONFIG, 2, 1), ("er", oracle.ER, 1, 64), ("er", oracle.ER, 1, 1000),
          ("er", oracle.ER, 3, 20)]
MODEL_IDS = ["%s-%d-%d" % (m[0], m[2], m[3]) for m in MODELS]


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


def _model(slm, kind, num, den):
    return slm.model(slm.MODEL_ER if kind == oracle.ER else slm.MODEL_CONFIG, num, den)


@pytest.mark.parametrize("mdl", MODELS, ids=MODEL_IDS)
@pytest.mark.parametrize("name", NAMES)
def test_run_under_model(slm, name, mdl):
    _, kind, num, den = mdl
    rp, col, w = GRAPHS[name]
    say("run", name, mdl)
    ref = oracle.run_null(rp, col, w, kind, num, den, seed=3)
    with slm.Graph(rp, col, w, model=_model(slm, kind, num, den)) as g:
        res = g.run(slm.params(seed=3))
    assert len(res) == len(ref)
    for a, b in zip(res, ref):
        assert a.n_c == b["n_c"] and a.nq == b["nq"] and a.q == b["q"]
        assert a.rounds == b["rounds"] and a.converged == b["converged"]
        assert np.array_equal(a.labels, b["labels"])


@pytest.mark.parametrize("mdl", MODELS, ids=MODEL_IDS)
@pytest.mark.parametrize("name", ["rmat12", "mixed_hub", "sbm1000", "star5000"])
def test_steps_under_model(slm, name, mdl):
    _, kind, num, den = mdl
    rp, col, w = GRAPHS[name]
    say("steps", name, mdl)
    go = oracle.NullGraph(rp, col, w, kind, num, den)
    with slm.Graph(rp, col, w, model=_model(slm, kind, num, den)) as g:
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
        for rnd in range(3):
            p = slm.params(seed=9)
            a_o2, v_o, st_o = oracle.maximal_round_nm(go, a_cur, 9, 0, rnd)
            a_g2, st_g = g.round(_t(a_cur), p, 0, rnd)
            assert st_g["valid"] == v_o and st_g["accepted"] == st_o["accepted"]
            assert st_g["splits"] == st_o["splits"]
            assert np.array_equal(_np(a_g2), a_o2)
            a_cur = a_o2


def test_model_arguments(slm):
    rp, col, w = GRAPHS["sbm1000"]
    for bad in (slm.model(slm.MODEL_CONFIG, 0, 1), slm.model(slm.MODEL_ER, 1, 0),
                slm.Model(9, 0, 1, 1)):
        with pytest.raises(slm.SlmError) as e:
            slm.Graph(rp, col, w, model=bad)
        assert e.value.status == slm.SLM_E_INVALID
    with pytest.raises(slm.SlmError) as e:
        slm.Graph(rp, col, w, model=slm.model(slm.MODEL_ER, 1 << 31, 1))
    assert e.value.status == slm.SLM_E_OVERFLOW
    with pytest.raises(slm.SlmError) as e:
        slm.Graph(rp, col, w, model=slm.model(slm.MODEL_CONFIG, 1 << 20, 1 << 40))
    assert e.value.status == slm.SLM_E_OVERFLOW


@pytest.mark.timeout(600)
@pytest.mark.parametrize("mdl", [("config", oracle.CONFIG, 1, 2), ("er", oracle.ER, 1, 4000)],
                         ids=["config-1-2", "er-1-4000"])
def test_fullsize_lfr4m_steps_under_model(slm, mdl):
    """At the LFR-style 4M size: ASSIGN, POSITIVE, the first sweep and the
    first MAXIMAL round, element by element against the oracle."""
    _, kind, num, den = mdl
    rp, col, w = config_graph("lfr4m")
    say("lfr4m steps", mdl)
    go = oracle.NullGraph(rp, col, w, kind, num, den)
    a_o = oracle.assign_nm(go)
    a1_o, s_o = oracle.positive_nm(go, a_o)
    lab, nc, _ = oracle.components(a1_o)
    b_o, d_o, w_o = oracle.sweep_nm(go, lab, nc)
    a2_o, v_o, st_o = oracle.maximal_round_nm(go, a1_o, 1, 0, 0)
    say("  oracle done: splits", s_o, "valid", v_o)
    with slm.Graph(rp, col, w, validate=False, model=_model(slm, kind, num, den)) as g:
        assert np.array_equal(_np(g.assign()), a_o)
        a1_g, s_g = g.positive(_t(a_o))
        assert s_g == s_o and np.array_equal(_np(a1_g), a1_o)
        b, d, wo = g.sweep(_t(lab), nc)
        assert np.array_equal(_np(b), b_o) and np.array_equal(_np(d), d_o)
        assert np.array_equal(_np(wo), w_o)
        a2_g, st_g = g.round(_t(a1_o), slm.params(seed=1), 0, 0)
        assert st_g["valid"] == v_o and st_g["splits"] == st_o["splits"]
        assert np.array_equal(_np(a2_g), a2_o)
