"""Full-size parity of the level loop (Algorithm 1, Sec. 3.4) on R-MAT scale
20 (1,048,576 nodes, 31.4 M entries), seed 1: after ASSIGN and POSITIVE, every
MAXIMAL round's counters (candidates, valid moves, accepted moves, POSITIVE
splits) must equal the oracle's, round by round, for every round stored in
tests/golden/rmat20_level0_rounds.txt (written by the oracle alone, see
make_rmat20_level0_rounds.py there).  The counters depend on every move,
draw and split of the round, so a single difference in the state shows up
in the round where it happens or soon after."""
import os

import numpy as np
import pytest

import graphgen as gg
from gpu_common import say

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "rmat20_level0_rounds.txt")


def golden_rounds():
    rows = np.loadtxt(GOLDEN, dtype=np.int64, comments="#", ndmin=2)
    assert rows.shape[1] == 5 and np.array_equal(rows[:, 0], np.arange(rows.shape[0]))
    return rows


def test_golden_file_is_well_formed():
    rows = golden_rounds()
    assert rows.shape[0] >= 60
    # valid moves never exceed candidates, accepted never exceed valid
    assert np.all(rows[:, 2] <= rows[:, 1]) and np.all(rows[:, 3] <= rows[:, 2])


@pytest.mark.gpu
def test_rmat20_level0_rounds_match_the_oracle():
    import torch
    assert torch.cuda.is_available()
    import paper_1702_04645_amd as slm
    rows = golden_rounds()
    rp, col, w = gg.config_graph("rmat20")
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
