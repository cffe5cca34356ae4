"""Writes rmat20_level0_rounds.txt: the oracle's counters of every MAXIMAL
round (Sec. 3.4) at level 0 of Algorithm 1 on the R-MAT scale-20 graph
(graphgen.config_graph("rmat20")) with seed 1, acceptance p = 1/2 and at most
64 rounds: candidates, valid moves, accepted moves and POSITIVE splits after
the round.  It runs the oracle alone (its level loop prints one line per
round when SLM_ORACLE_VERBOSE is set) and takes about ten hours on one core.

    python tests/golden/make_rmat20_level0_rounds.py [max_rounds_to_keep]
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))

CODE = ("import graphgen as gg, oracle\n"
        "rp, col, w = gg.config_graph('rmat20')\n"
        "oracle.level(oracle.Graph(rp, col, w), 1, 0)\n")


def parse(lines):
    out = []
    for ln in lines:
        if not ln.startswith("oracle level 0 round"):
            continue
        f = ln.replace(":", "").split()
        out.append((int(f[4]), int(f[6]), int(f[8]), int(f[10]), int(f[12])))
    return out


def write(rows, path):
    with open(path, "w") as f:
        f.write("# Oracle MAXIMAL rounds at level 0: R-MAT scale 20 (config graph rmat20),\n")
        f.write("# seed 1, accept_p = 2^31, ASSIGN then POSITIVE before round 0.\n")
        f.write("# Written by make_rmat20_level0_rounds.py from the oracle's level loop.\n")
        f.write("# round candidates valid accepted splits\n")
        for r in rows:
            f.write("%d %d %d %d %d\n" % r)


if __name__ == "__main__":
    env = dict(os.environ, SLM_ORACLE_VERBOSE="1")
    r = subprocess.run([sys.executable, "-c", CODE], env=env, cwd=ROOT, capture_output=True,
                       text=True, check=True)
    rows = parse(r.stderr.splitlines())
    if len(sys.argv) > 1:
        rows = rows[: int(sys.argv[1])]
    write(rows, os.path.join(HERE, "rmat20_level0_rounds.txt"))
