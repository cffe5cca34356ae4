"""Full-size parity of Algorithm 1 on the LFR-style graph of 4,000,000
nodes (75 M entries), seed 1, against one oracle run stored in tests/golden
(written by the oracle alone, see make_lfr4m_golden.py there):

- level 0, round by round: after ASSIGN and POSITIVE, every MAXIMAL round's
  counters (candidates, valid moves, accepted moves, POSITIVE splits, Sec.
  3.4) equal the oracle's;
- the whole run: every emitted level's n_c, N_Q, rounds and convergence
  equal the oracle's, Q within 1e-12, and the composed labels of all
  4,000,000 nodes are identical (SHA-256 of their int32 bytes)."""
import hashlib
import os

import numpy as np
import pytest

from gpu_common import config_graph, say

HERE = os.path.dirname(os.path.abspath(__file__))
ROUNDS = os.path.join(HERE, "golden", "lfr4m_level0_rounds.txt")
LEVELS = os.path.join(HERE, "golden", "lfr4m_seed1_levels.txt")


def golden_rounds():
    rows = np.loadtxt(ROUNDS, dtype=np.int64, comments="#", ndmin=2)
    assert rows.shape[1] == 5 and np.array_equal(rows[:, 0], np.arange(rows.shape[0]))
    return rows


def golden_levels():
    out = []
    for ln in open(LEVELS):
        if ln.startswith("#") or not ln.strip():
            continue
        f = ln.split()
        out.append((int(f[0]), int(f[1]), float(f[2]), int(f[3]), bool(int(f[4])), f[5]))
    return out


def lfr4m():
    return config_graph("lfr4m")


@pytest.mark.gpu
@pytest.mark.timeout(600)
def test_lfr4m_level0_rounds_match_the_oracle():
    import torch
    assert torch.cuda.is_available()
    import paper_1702_04645_amd as slm
    rows = golden_rounds()
    rp, col, w = lfr4m()
    say("lfr4m level-0 rounds:", rows.shape[0])
    p = slm.params(seed=1)
    with slm.Graph(rp, col, w, validate=False) as g:
        a = g.assign()
        a, _ = g.positive(a)
        for r in range(rows.shape[0]):
            a, st = g.round(a, p, 0, r)
            got = (st["candidates"], st["valid"], st["accepted"], st["splits"])
            assert got == tuple(int(x) for x in rows[r, 1:]), "round %d: %s vs oracle %s" % (
                r, got, tuple(rows[r, 1:]))
            if r % 10 == 0:
                say("round", r, got)
        # the level converged: one more round finds no valid move
        _, st = g.round(a, p, 0, rows.shape[0])
        assert st["valid"] == 0


@pytest.mark.gpu
@pytest.mark.timeout(600)
def test_lfr4m_full_run_matches_the_oracle():
    import torch
    assert torch.cuda.is_available()
    import paper_1702_04645_amd as slm
    lv = golden_levels()
    rp, col, w = lfr4m()
    say("lfr4m full run, seed 1:", len(lv), "levels")
    with slm.Graph(rp, col, w, validate=False) as g:
        res = g.run(slm.params(seed=1))
    assert len(res) == len(lv)
    for i, (r, (nc, nq, q, rounds, conv, h)) in enumerate(zip(res, lv)):
        lab = np.ascontiguousarray(r.labels, dtype=np.int32)
        assert lab.size == rp.size - 1
        got = (r.n_c, r.nq, r.rounds, bool(r.converged))
        assert got == (nc, nq, rounds, conv), "level %d: %s vs oracle %s" % (i, got, (nc, nq, rounds, conv))
        assert abs(r.q - q) <= 1e-12
        assert hashlib.sha256(lab.tobytes()).hexdigest() == h, "level %d labels differ" % i
        say("level", i, got)
