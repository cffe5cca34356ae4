"""The oracle's C source built with AddressSanitizer and UndefinedBehavior-
Sanitizer (gcc, host code only) and run on the small fixtures: whole runs of
Algorithm 1 under the configuration model (resolution 1 and 1/2), the
Erdos-Renyi null model and the directed model (Sec. 2.2-2.4), classical
Louvain, and the single steps (ASSIGN, POSITIVE, COMPONENTS, the sweep, a
MAXIMAL round, AGGREGATE).  An out-of-bounds access, a use after free, a
signed overflow or any other undefined behaviour stops the run; the results
must equal those of the ordinary build, run here in-process."""
import hashlib
import json
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "slm_oracle.c")


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or _runtime("libasan.so") is None,
                                reason="needs gcc with the AddressSanitizer runtime")

# the digest of every case, computed by the same code in both builds
DRIVER = r'''
import hashlib, json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
sys.path.insert(0, sys.argv[1] + "/tests")
import oracle
if len(sys.argv) > 2:
    oracle._LIB = sys.argv[2]  # the sanitized build, newer than the source
import graphgen as gg
from gpu_common import small_graphs


def h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def levels(res):
    return [[r["n_c"], r["nq"], repr(r["q"]), r["rounds"], r["converged"], h(r["labels"])]
            for r in res]


out = {}
for name, (rp, col, w) in small_graphs().items():
    out["run/" + name] = levels(oracle.run(rp, col, w, seed=1))
    out["run_cap/" + name] = levels(oracle.run(rp, col, w, seed=2, max_rounds=2, max_levels=2))
    out["louvain/" + name] = levels(oracle.louvain_run(rp, col, w))
    if name != "mixed_hub":
        out["gamma/" + name] = levels(oracle.run_null(rp, col, w, oracle.CONFIG, 1, 2, seed=1))
        out["er/" + name] = levels(oracle.run_null(rp, col, w, oracle.ER, 1, 64, seed=1))
        d = gg.orient(rp, col, w, 17 + len(name), both=0.3,
                      w_max=0 if name.startswith("star") else 6)
        out["directed/" + name] = levels(oracle.run_null(*d, oracle.DIRECTED, 1, 1, seed=4))
    g = oracle.Graph(rp, col, w)
    a0 = oracle.assign(g)
    a1, s1 = oracle.positive(g, a0)
    lab, nc, cyc = oracle.components(a1)
    b, dl, wo = oracle.sweep(g, lab, nc)
    a2, v, st = oracle.maximal_round(g, a1, 3, 0, 0)
    crp, ccol, cw = oracle.contract(g, lab, nc)
    out["steps/" + name] = [h(a0), h(a1), s1, h(lab), nc, h(cyc), h(b), h(dl), h(wo), h(a2), v,
                            st, oracle.modularity_num(g, lab, nc), h(crp), h(ccol), h(cw)]
print(json.dumps(out, sort_keys=True))
'''


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-o", lib, SRC])
    drv = tmp_path / "drive.py"
    drv.write_text(DRIVER)
    env = dict(os.environ)
    env["LD_PRELOAD"] = _runtime("libasan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=86"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=87"
    san = subprocess.run([sys.executable, str(drv), ROOT, lib], capture_output=True, text=True,
                         env=env, timeout=900)
    assert san.returncode == 0, "sanitized oracle stopped (%d):\n%s" % (san.returncode,
                                                                       san.stderr[-6000:])
    plain = subprocess.run([sys.executable, str(drv), ROOT], capture_output=True, text=True,
                           timeout=900)
    assert plain.returncode == 0, plain.stderr[-3000:]
    got, ref = json.loads(san.stdout), json.loads(plain.stdout)
    assert sorted(got) == sorted(ref) and len(ref) > 50
    for k in ref:
        assert got[k] == ref[k], k
