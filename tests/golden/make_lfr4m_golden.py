"""Writes lfr4m_seed1_levels.txt from one oracle run of Algorithm 1 on
graphgen.config_graph("lfr4m") (the LFR-style graph of 4,000,000 nodes) with
seed 1, acceptance p = 1/2 and at most 64 MAXIMAL rounds per level.  Per
emitted level: n_c, N_Q, Q, rounds, converged, and the SHA-256 of the
composed labels of the original nodes as int32 bytes.  The level-0 MAXIMAL
round counters (candidates, valid, accepted, splits) go to
lfr4m_level0_rounds.txt.

Only the oracle runs here.

    python tests/golden/make_lfr4m_golden.py
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, HERE)

from make_rmat20_golden import parse_rounds  # noqa: E402

CODE = r"""
import hashlib
import numpy as np
import graphgen as gg, oracle
rp, col, w = gg.config_graph('lfr4m')
for l in oracle.run(rp, col, w, seed=1):
    h = hashlib.sha256(np.ascontiguousarray(l['labels'], dtype=np.int32).tobytes()).hexdigest()
    print('LEVEL', l['n_c'], l['nq'], repr(l['q']), l['rounds'], int(l['converged']), h, flush=True)
"""


def main():
    env = dict(os.environ, SLM_ORACLE_VERBOSE="1")
    r = subprocess.run([sys.executable, "-c", CODE], env=env, cwd=ROOT, capture_output=True,
                       text=True, check=True)
    rows = parse_rounds(r.stderr.splitlines())
    with open(os.path.join(HERE, "lfr4m_level0_rounds.txt"), "w") as f:
        f.write("# Oracle MAXIMAL rounds at level 0: LFR-style 4M (config graph lfr4m),\n")
        f.write("# seed 1, accept_p = 2^31, ASSIGN then POSITIVE before round 0.\n")
        f.write("# Written by make_lfr4m_golden.py from the oracle's level loop.\n")
        f.write("# round candidates valid accepted splits\n")
        for row in rows:
            f.write("%d %d %d %d %d\n" % row)
    levels = [ln.split()[1:] for ln in r.stdout.splitlines() if ln.startswith("LEVEL")]
    with open(os.path.join(HERE, "lfr4m_seed1_levels.txt"), "w") as f:
        f.write("# Oracle run of Algorithm 1: LFR-style 4M (config graph lfr4m), seed 1,\n")
        f.write("# accept_p = 2^31, at most 64 rounds per level.  Written by\n")
        f.write("# make_lfr4m_golden.py.  Per emitted level:\n")
        f.write("# n_c N_Q Q rounds converged sha256(composed labels as int32)\n")
        for lv in levels:
            f.write(" ".join(lv) + "\n")


if __name__ == "__main__":
    main()
