"""The POSITIVE kernel (Sec. 3.3), compiled for the host by g++ with the
emulation header in tests/emu (one thread per lane, real barriers and
wavefront exchanges), against the oracle's POSITIVE on every POSITIVE input
of oracle runs: the assignment after ASSIGN and after each MAXIMAL round's
re-pointing, at every level.  Community and member orders are shuffled (on
the device they come from atomics), workgroups are shrunk so that every
loop runs over several blocks and the candidate set overflows, and lanes
other than 0 are held back after every barrier (or all lanes by random
amounts), so that a read of shared state that a single thread changes
before the next barrier shows up as a stuck barrier or a different result.
Needs no GPU."""
import os
import re
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import oracle  # noqa: E402
from gpu_common import small_graphs  # noqa: E402

CSRC = os.path.join(ROOT, "paper_1702_04645_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "emu")
# (workgroup lanes, candidate-set size, lane bests kept by a scan)
WORKGROUPS = {"wg512": (512, 4096, 4), "wg64": (64, 16, 1)}

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _kernel_source():
    s = open(os.path.join(CSRC, "k_positive.hip")).read()
    for name in ("PW_BS", "PW_CAND", "PW_TOP"):
        s, k = re.subn(r"^#define %s (\d+)(.*)$" % name,
                       r"#ifndef %s\n#define %s \1\2\n#endif" % (name, name), s, flags=re.M)
        assert k == 1, name
    s, k = re.subn(r"k_positive_wg<<<.*>>>\(A\);", "(void)A; (void)s;", s)
    assert k == 1
    return s


@pytest.fixture(scope="module")
def emulators(tmp_path_factory):
    d = tmp_path_factory.mktemp("positive_emu")
    (d / "k_positive_emu.inc").write_text(_kernel_source())
    out = {}
    for name, (bs, cand, top) in WORKGROUPS.items():
        exe = str(d / ("emu_" + name))
        cmd = ["g++", "-std=c++20", "-O1", "-pthread", "-I", EMU, "-I", CSRC, "-I", str(d),
               "-DPW_BS=%d" % bs, "-DPW_CAND=%d" % cand, "-DPW_TOP=%d" % top,
               os.path.join(EMU, "positive_emu.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-3000:]
        out[name] = exe
    return out


def positive_inputs(rp, col, w, seed, max_levels=6, max_rounds=64):
    """Every assignment an oracle run hands to POSITIVE, with its level graph."""
    out = []
    for lvl in range(max_levels):
        g = oracle.Graph(rp, col, w)
        if g.n == 0 or g.m2 == 0:
            break
        a = oracle.assign(g)
        out.append((g, a.copy()))
        a, _ = oracle.positive(g, a)
        for r in range(max_rounds):
            a2, valid, _, rep = oracle.maximal_round(g, a, seed, lvl, r, with_repointed=True)
            if valid == 0:
                break
            out.append((g, rep.copy()))
            a = a2
        lab, nc, _ = oracle.components(a)
        if nc == g.n:
            break
        rp, col, w = oracle.contract(g, lab, nc)
    return out


def run_emulator(exe, cases, orders, skew_us, tmp):
    fin, fout = str(tmp / "cases.bin"), str(tmp / "out.bin")
    with open(fin, "wb") as f:
        for g, a in cases:
            for s in orders:
                np.array([g.n, g.col.size, g.m2, s, 1], np.int64).tofile(f)
                g.rp.astype(np.int64).tofile(f)
                g.col.astype(np.int32).tofile(f)
                g.w.astype(np.int32).tofile(f)
                a.astype(np.int32).tofile(f)
    r = subprocess.run([exe, fin, fout, str(skew_us)], capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0, "emulated kernel stopped (%d):\n%s" % (r.returncode,
                                                                    r.stderr[-6000:])
    res = []
    with open(fout, "rb") as f:
        for g, a in cases:
            for s in orders:
                hdr = np.fromfile(f, np.int64, 3)
                res.append((hdr, np.fromfile(f, np.int32, g.n)))
    return res


GRAPHS = ["random0", "random1", "random2", "random3", "random4", "random5", "path200",
          "cliques", "sbm1000"]


# skew > 0: lanes other than 0 wait that many microseconds after every
# barrier (a single writer runs ahead of the readers); skew < 0: every lane
# waits a random 0..-skew microseconds (seeded per lane and case)
@pytest.mark.parametrize("config,skew", [("wg512", 20), ("wg64", 20), ("wg64", -30)])
def test_emulated_positive_matches_oracle(emulators, config, skew, tmp_path):
    graphs = small_graphs()
    cases = []
    for name in GRAPHS:
        rp, col, w = graphs[name]
        cases += positive_inputs(rp, col, w, seed=1)
    orders = [11 + WORKGROUPS[config][0] + abs(skew)]  # one member order per case
    res = run_emulator(emulators[config], cases, orders, skew_us=skew, tmp=tmp_path)
    splits = flagged = 0
    i = 0
    for g, a in cases:
        a_exp, s_exp = oracle.positive(g, a)
        for s in orders:
            hdr, a_got = res[i]
            i += 1
            assert hdr[1] == 0, "loop bound tripped (code %d)" % hdr[1]
            assert hdr[0] == s_exp
            assert np.array_equal(a_got, a_exp)
            splits += int(hdr[0])
            flagged += int(hdr[2])
    # the cases exercise the kernel: many communities split, many splits
    assert flagged > 30 * len(orders) and splits > 60 * len(orders), (flagged, splits)
