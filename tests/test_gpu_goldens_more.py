"""Whole runs at full size against stored oracle runs (tests/golden, written
by the oracle alone): the directed LFR-shaped graph of 10^6 nodes under the
directed model (Sec. 2.4), and the LFR-style 4M graph under the resolution
and Erdos-Renyi models (Sec. 2.2-2.3) and with the classical Louvain method.
Every emitted level's n_c, N_Q, Q, rounds (passes), convergence and the
SHA-256 of the composed labels of all original nodes must be equal."""
import hashlib
import os

import numpy as np
import pytest

from gpu_common import config_graph, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def read_levels(path, named=False):
    out = {}
    for ln in open(path):
        if ln.startswith("#") or not ln.strip():
            continue
        f = ln.split()
        name = f.pop(0) if named else ""
        out.setdefault(name, []).append((int(f[0]), int(f[1]), float(f[2]), int(f[3]),
                                         bool(int(f[4])), f[5]))
    return out


def _check(res, gold):
    assert len(res) == len(gold)
    for r, (nc, nq, q, rounds, conv, h) in zip(res, gold):
        assert (r.n_c, r.nq, r.rounds, r.converged) == (nc, nq, rounds, conv)
        assert r.q == q
        lab = np.ascontiguousarray(r.labels, dtype=np.int32)
        assert hashlib.sha256(lab.tobytes()).hexdigest() == h


@pytest.fixture(scope="module")
def slm():
    import torch
    assert torch.cuda.is_available()
    import paper_1702_04645_amd as slm
    slm.lib()
    return slm


@pytest.mark.timeout(600)
def test_directed_lfr1m_run_is_the_oracle_run(slm):
    gold = read_levels(os.path.join(HERE, "golden", "lfr1m_dir_seed1_levels.txt"))[""]
    rp, col, w = config_graph("lfr1m_dir")
    say("lfr1m_dir run")
    with slm.Graph(rp, col, w, validate=False,
                   model=slm.model(slm.MODEL_DIRECTED, 1, 1)) as g:
        res = g.run(slm.params(seed=1))
    _check(res, gold)


@pytest.mark.timeout(900)
def test_lfr4m_models_and_louvain_are_the_oracle_runs(slm):
    gold = read_levels(os.path.join(HERE, "golden", "lfr4m_models_levels.txt"), named=True)
    rp, col, w = config_graph("lfr4m")
    for name, kind, num, den in (("config_1_2", slm.MODEL_CONFIG, 1, 2),
                                 ("er_1_4000", slm.MODEL_ER, 1, 4000)):
        say("lfr4m", name)
        with slm.Graph(rp, col, w, validate=False, model=slm.model(kind, num, den)) as g:
            _check(g.run(slm.params(seed=1)), gold[name])
    say("lfr4m louvain")
    with slm.Graph(rp, col, w, validate=False) as g:
        _check(g.louvain_run(), gold["louvain"])
