"""Writes lfr1m_dir_seed1_levels.txt from one oracle run of Algorithm 1
under the directed model (Sec. 2.4, resolution 1) on
graphgen.config_graph("lfr1m_dir") (the directed LFR-shaped graph of
1,000,000 nodes) with seed 1, acceptance p = 1/2 and at most 64 MAXIMAL
rounds per level.  Per emitted level: n_c, N_Q, Q, rounds, converged, and
the SHA-256 of the composed labels of the original nodes as int32 bytes.

Only the oracle runs here.

    python tests/golden/make_lfr1m_dir_golden.py
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
    rp, col, w = gg.config_graph("lfr1m_dir")
    res = oracle.run_null(rp, col, w, oracle.DIRECTED, 1, 1, seed=1)
    with open(os.path.join(HERE, "lfr1m_dir_seed1_levels.txt"), "w") as f:
        f.write("# Oracle run of Algorithm 1 under the directed model: directed LFR-shaped\n")
        f.write("# graph of 10^6 nodes (config graph lfr1m_dir), seed 1, acceptance 1/2 (2^31 of 2^32),\n")
        f.write("# at most 64 rounds per level.  Written by make_lfr1m_dir_golden.py.\n")
        f.write("# Per emitted level: n_c N_Q Q rounds converged sha256(composed labels as int32)\n")
        for l in res:
            h = hashlib.sha256(np.ascontiguousarray(l["labels"], dtype=np.int32).tobytes())
            f.write("%d %d %r %d %d %s\n" % (l["n_c"], l["nq"], l["q"], l["rounds"],
                                             int(l["converged"]), h.hexdigest()))


if __name__ == "__main__":
    main()
