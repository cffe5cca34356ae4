"""Full-size parity of Algorithm 1 on R-MAT scale 20 (1,048,576 nodes,
31.4 M entries), seed 1, against one oracle run stored in tests/golden
(written by the oracle alone, see make_rmat20_golden.py there):

- level 0, round by round: after ASSIGN and POSITIVE, every MAXIMAL round's
  counters (candidates, valid moves, accepted moves, POSITIVE splits, Sec.
  3.4) equal the oracle's, so a difference in the state shows up in the
  round where it happens;
- the whole run: every emitted level's n_c, N_Q, rounds and convergence
  equal the oracle's, Q within 1e-12, and the composed labels of all
  1,048,576 nodes are identical (SHA-256 of their int32 bytes)."""
import hashlib
import os

import numpy as np
import pytest

import graphgen as gg
from gpu_common import config_graph, say

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "rmat20_level0_rounds.txt")
LEVELS = os.path.join(HERE, "golden", "rmat20_seed1_levels.txt")


def golden_rounds():
    rows = np.loadtxt(GOLDEN, dtype=np.int64, comments="#", ndmin=2)
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


def test_golden_file_is_well_formed():
    rows = golden_rounds()
    assert rows.shape[0] == 64  # level 0 runs to the 64-round cap
    lv = golden_levels()
    assert len(lv) == 4 and lv[0][3] == 64 and not lv[0][4]
    # valid moves never exceed candidates, accepted never exceed valid
    assert np.all(rows[:, 2] <= rows[:, 1]) and np.all(rows[:, 3] <= rows[:, 2])


@pytest.mark.gpu
def test_rmat20_level0_rounds_match_the_oracle():
    import torch
    assert torch.cuda.is_available()
    import paper_1702_04645_amd as slm
    rows = golden_rounds()
    rp, col, w = config_graph("rmat20")
    say("rmat20 level-0 rounds:", rows.shape[0])
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


@pytest.mark.gpu
def test_rmat20_full_run_matches_the_oracle():
    import torch
    assert torch.cuda.is_available()
    import paper_1702_04645_amd as slm
    lv = golden_levels()
    rp, col, w = config_graph("rmat20")
    say("rmat20 full run, seed 1:", len(lv), "levels")
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
