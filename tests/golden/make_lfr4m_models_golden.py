"""Writes lfr4m_models_levels.txt from oracle runs on graphgen.config_graph
("lfr4m") (the LFR-style graph of 4,000,000 nodes): Algorithm 1 with seed 1,
acceptance p = 1/2, at most 64 rounds per level, under the configuration
model with resolution 1/2 and the Erdos-Renyi model with p = 1/4000 (Sec.
2.2-2.3), and the classical Louvain run (at most 64 passes per level).  One
line per emitted level: the run's name, n_c, N_Q, Q, rounds (passes),
converged, and the SHA-256 of the composed labels as int32 bytes.

Only the oracle runs here.

    python tests/golden/make_lfr4m_models_golden.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402


def main():
    rp, col, w = gg.config_graph("lfr4m")
    runs = [("config_1_2", lambda: oracle.run_null(rp, col, w, oracle.CONFIG, 1, 2, seed=1)),
            ("er_1_4000", lambda: oracle.run_null(rp, col, w, oracle.ER, 1, 4000, seed=1)),
            ("louvain", lambda: oracle.louvain_run(rp, col, w))]
    with open(os.path.join(HERE, "lfr4m_models_levels.txt"), "w") as f:
        f.write("# Oracle runs on the LFR-style 4M graph (config graph lfr4m): Algorithm 1\n")
        f.write("# with seed 1, acceptance 1/2 (2^31 of 2^32), at most 64 rounds per level, under the\n")
        f.write("# resolution-1/2 and Erdos-Renyi p = 1/4000 models, and the classical\n")
        f.write("# Louvain run.  Written by make_lfr4m_models_golden.py.  Per emitted level:\n")
        f.write("# run n_c N_Q Q rounds converged sha256(composed labels as int32)\n")
        for name, fn in runs:
            for l in fn():
                h = hashlib.sha256(np.ascontiguousarray(l["labels"], dtype=np.int32).tobytes())
                f.write("%s %d %d %r %d %d %s\n" % (name, l["n_c"], l["nq"], l["q"], l["rounds"],
                                                    int(l["converged"]), h.hexdigest()))
                f.flush()


if __name__ == "__main__":
    main()
