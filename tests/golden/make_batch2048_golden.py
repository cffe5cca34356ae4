"""Writes batch2048_levels.txt: the oracle run of Algorithm 1 on every member
of the 2048-graph planted-partition batch (graphgen.sbm_batch with the
batch2048 seed; member i drawn with seed graphgen.batch_member_seed(1, i),
acceptance p = 1/2, at most 64 MAXIMAL rounds per level), one line per
emitted level: member, level, n_c, N_Q, rounds, converged, and the SHA-256
of the member's composed labels as int32 bytes.

Only the oracle runs here (one process per core).

    python tests/golden/make_batch2048_golden.py [processes]
"""
import hashlib
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402

COUNT = 2048


def member_levels(i):
    import oracle
    seed = gg.CONFIG_SEEDS["batch2048"]
    rp, col, w = gg.sbm_batch(COUNT, 64, 65536, seed, indices=[i])[0]
    out = []
    for lv, r in enumerate(oracle.run(rp, col, w, seed=gg.batch_member_seed(1, i))):
        h = hashlib.sha256(np.ascontiguousarray(r["labels"], dtype=np.int32).tobytes()).hexdigest()
        out.append((i, lv, r["n_c"], r["nq"], r["rounds"], int(r["converged"]), h))
    return out


def main():
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else max(1, (os.cpu_count() or 2) - 1)
    with mp.get_context("fork").Pool(procs) as pool:
        rows = pool.map(member_levels, range(COUNT), chunksize=4)
    with open(os.path.join(HERE, "batch2048_levels.txt"), "w") as f:
        f.write("# Oracle runs of Algorithm 1 on the 2048 members of the planted-partition\n")
        f.write("# batch (config batch2048), member i with seed batch_member_seed(1, i),\n")
        f.write("# accept_p = 2^31, at most 64 rounds per level.  Written by\n")
        f.write("# make_batch2048_golden.py.  Per emitted level of each member:\n")
        f.write("# member level n_c N_Q rounds converged sha256(composed labels as int32)\n")
        for member in rows:
            for r in member:
                f.write(" ".join(str(x) for x in r) + "\n")


if __name__ == "__main__":
    main()
