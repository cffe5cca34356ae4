"""The stored oracle runs under tests/golden are well formed and are what
the committed oracle computes (checked on a sample of the batch members,
which the oracle runs in seconds)."""
import hashlib
import os

import numpy as np

import graphgen as gg
import oracle
from test_gpu_fullsize import batch2048_golden


def test_batch2048_golden_is_well_formed():
    gold = batch2048_golden()
    assert sorted(gold) == list(range(2048))
    for m, levels in gold.items():
        assert levels, m  # every member has edges, so it emits a level
        ncs = [x[0] for x in levels]
        assert all(b < a for a, b in zip(ncs, ncs[1:])), m
        assert all(x[2] <= 64 for x in levels), m


def test_batch2048_golden_is_the_oracle_run():
    gold = batch2048_golden()
    seed = gg.CONFIG_SEEDS["batch2048"]
    for i in (0, 1, 2, 333, 1024, 2047):
        rp, col, w = gg.sbm_batch(2048, 64, 65536, seed, indices=[i])[0]
        res = oracle.run(rp, col, w, seed=gg.batch_member_seed(1, i))
        assert len(res) == len(gold[i]), i
        for r, (nc, nq, rounds, conv, h) in zip(res, gold[i]):
            assert (r["n_c"], r["nq"], r["rounds"], r["converged"]) == (nc, nq, rounds, conv)
            lab = np.ascontiguousarray(r["labels"], dtype=np.int32)
            assert hashlib.sha256(lab.tobytes()).hexdigest() == h


def test_lfr4m_golden_is_well_formed():
    from test_gpu_lfr4m_golden import golden_levels, golden_rounds
    lv = golden_levels()
    rows = golden_rounds()
    assert len(lv) >= 2
    assert lv[0][3] == rows.shape[0]  # level 0's rounds are the rows
    assert all(x[3] <= 64 for x in lv)
    # Q never decreases across levels and communities only merge
    assert all(b[2] >= a[2] for a, b in zip(lv, lv[1:]))
    assert all(b[0] < a[0] for a, b in zip(lv, lv[1:]))
    assert np.all(rows[:, 2] <= rows[:, 1]) and np.all(rows[:, 3] <= rows[:, 2])


def test_more_full_size_goldens_are_well_formed():
    """The stored directed LFR-1M run and the LFR-4M runs under the resolution
    and Erdos-Renyi models and with classical Louvain: per run, communities
    only merge, Q never decreases, at most 64 rounds, and one hash a level."""
    from test_gpu_goldens_more import read_levels
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    runs = read_levels(os.path.join(here, "lfr1m_dir_seed1_levels.txt"))
    runs.update(read_levels(os.path.join(here, "lfr4m_models_levels.txt"), named=True))
    assert sorted(runs) == ["", "config_1_2", "er_1_4000", "louvain"]
    for name, lv in runs.items():
        assert len(lv) >= 2, name
        assert all(b[0] < a[0] for a, b in zip(lv, lv[1:])), name
        assert all(b[2] >= a[2] and b[1] >= a[1] for a, b in zip(lv, lv[1:])), name
        assert all(0 <= x[3] <= 64 and 0 < x[2] < 1 for x in lv), name
        assert all(len(x[5]) == 64 and int(x[5], 16) >= 0 for x in lv), name
        assert lv[-1][4], name  # the last level converged
