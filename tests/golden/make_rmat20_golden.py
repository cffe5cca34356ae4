"""Writes the R-MAT scale-20 golden files from one oracle run of Algorithm 1
on graphgen.config_graph("rmat20") with seed 1, acceptance p = 1/2 and at
most 64 MAXIMAL rounds per level (about ten hours on one core):

  rmat20_level0_rounds.txt  the counters of every MAXIMAL round (Sec. 3.4)
                            at level 0: candidates, valid moves, accepted
                            moves, POSITIVE splits after the round (printed
                            by the oracle's level loop when
                            SLM_ORACLE_VERBOSE is set);
  rmat20_seed1_levels.txt   every emitted level: n_c, N_Q, Q, rounds,
                            converged, and the SHA-256 of the composed
                            labels of the original nodes as int32 bytes.

Only the oracle runs here.

    python tests/golden/make_rmat20_golden.py
"""
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))

CODE = r"""
import hashlib
import numpy as np
import graphgen as gg, oracle
rp, col, w = gg.config_graph('rmat20')
for l in oracle.run(rp, col, w, seed=1):
    h = hashlib.sha256(np.ascontiguousarray(l['labels'], dtype=np.int32).tobytes()).hexdigest()
    print('LEVEL', l['n_c'], l['nq'], repr(l['q']), l['rounds'], int(l['converged']), h, flush=True)
"""


def parse_rounds(lines):
    out = []
    for ln in lines:
        if not ln.startswith("oracle level 0 round"):
            continue
        f = ln.replace(":", "").split()
        out.append((int(f[4]), int(f[6]), int(f[8]), int(f[10]), int(f[12])))
    return out


def write_rounds(rows, path):
    with open(path, "w") as f:
        f.write("# Oracle MAXIMAL rounds at level 0: R-MAT scale 20 (config graph rmat20),\n")
        f.write("# seed 1, accept_p = 2^31, ASSIGN then POSITIVE before round 0.\n")
        f.write("# Written by make_rmat20_golden.py from the oracle's level loop.\n")
        f.write("# round candidates valid accepted splits\n")
        for r in rows:
            f.write("%d %d %d %d %d\n" % r)


def write_levels(levels, path):
    with open(path, "w") as f:
        f.write("# Oracle run of Algorithm 1: R-MAT scale 20 (config graph rmat20), seed 1,\n")
        f.write("# accept_p = 2^31, at most 64 rounds per level.  Written by\n")
        f.write("# make_rmat20_golden.py.  Per emitted level:\n")
        f.write("# n_c N_Q Q rounds converged sha256(composed labels as int32)\n")
        for lv in levels:
            f.write(" ".join(str(x) for x in lv) + "\n")


if __name__ == "__main__":
    env = dict(os.environ, SLM_ORACLE_VERBOSE="1")
    r = subprocess.run([sys.executable, "-c", CODE], env=env, cwd=ROOT, capture_output=True,
                       text=True, check=True)
    write_rounds(parse_rounds(r.stderr.splitlines()), os.path.join(HERE, "rmat20_level0_rounds.txt"))
    levels = [ln.split()[1:] for ln in r.stdout.splitlines() if ln.startswith("LEVEL")]
    write_levels(levels, os.path.join(HERE, "rmat20_seed1_levels.txt"))
